// Device code of the learned per-axis closure.
//
// A coarse grid (half the points of a fine grid on every axis, same box)
// replaces the right-hand side B f / h of the compact scheme of Sec. III B
// along each grid axis a by (B + S_a) f / h, with S_a skew-symmetric on the
// first kClosBands off-diagonals: S[i][i+k] = -S[i+k][i] = s (k = 1, 2).  The
// entries s come from a small network evaluated once per problem:
//   s = tanh(phi W1 + b1) W2 + b2,  phi: 16 features of (axis, entry, model),
// 32 hidden units, BF16 weights and activations in the products, FP32
// accumulation (MFMA 16x16x16 BF16 tiles), FP32 master weights and Adam.
//
// Training data come from fine-grid states of the solver itself: for each
// axis, the restricted fine derivative T = R(D_fine h) is the target of the
// coarse derivative of x = R h (R: 2:1 cell averages on every axis).  With
// r = T - D_coarse x, the loss of one (draw, axis) group is
//   sum_lines || r - A^{-1} S x / h ||^2 / sum_lines ||T||^2,
// a quadratic in the entries s whose coefficients follow from the line
// moments sum x x^T and sum x r^T (k_line_moments, k_gram).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.h"

namespace chfpe {

// Off-diagonals of the skew correction.  The stencil kernels take up to
// three; a third fits the training derivatives better but gave larger
// spectrum errors on held-out draws.
constexpr int kClosBands = 2;
constexpr int kClosFeat = 16;
constexpr int kClosHid = 32;
// parameters: W1 [16][32], b1 [32], W2 [32], b2
constexpr int kClosParams = kClosFeat * kClosHid + kClosHid + kClosHid + 1;

// ---------------------------------------------------------------------------
// grid operations on FP64 states [element][axis_0]...[axis_{2M-1}]
// ---------------------------------------------------------------------------
// Lines along one axis: length N, stride `inner` (elements), `outer` blocks
// of inner * N values per element, ne elements of E values.
struct AxisLines {
  int N;
  long long inner, outer, E, nlines;
};

__device__ __forceinline__ long long line_base(const AxisLines &al, const long long l) {
  const long long lo = l % al.inner;
  const long long t = l / al.inner;
  const long long hi = t % al.outer;
  const long long e = t / al.outer;
  return e * al.E + hi * al.inner * al.N + lo;
}

// Y = Yadd + alpha D X along the axis (plain compact derivative; Yadd may
// alias Y or be null).  One line per thread.
template <int NMAX>
__global__ void __launch_bounds__(256)
k_axis_deriv(const double *__restrict__ X, double *Y, const double *Yadd, const double alpha,
             const AxisLines al, const double ca, const double cb) {
  const long long l = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= al.nlines) return;
  const long long b = line_base(al, l);
  double f[NMAX];
#pragma unroll
  for (int i = 0; i < NMAX; ++i) f[i] = i < al.N ? X[b + i * al.inner] : 0.0;
  compact_line<double, NMAX>(f, al.N, ca, cb);
#pragma unroll
  for (int i = 0; i < NMAX; ++i)
    if (i < al.N) {
      const long long k = b + i * al.inner;
      Y[k] = (Yadd ? Yadd[k] : 0.0) + alpha * f[i];
    }
}

// Coarse dims and strides of the restriction (the fine grid has twice the
// points on every axis).
struct Restrict {
  int nd;             // grid axes (2M)
  int dc[6];          // coarse lengths
  long long sc[6];    // coarse strides within an element
  long long sf[6];    // fine strides within an element
  long long Ec, Ef;   // points per element
  long long total;    // ne * Ec
};

// Xc = R Xf: the mean of the 2^nd fine values of every coarse cell.
__global__ void __launch_bounds__(256)
k_restrict(const double *__restrict__ Xf, double *__restrict__ Xc, const Restrict rs) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= rs.total) return;
  const long long e = t / rs.Ec;
  long long rem = t - e * rs.Ec;
  long long fb = e * rs.Ef;
  for (int d = 0; d < rs.nd; ++d) {
    const long long i = rem / rs.sc[d];
    rem -= i * rs.sc[d];
    fb += 2 * i * rs.sf[d];
  }
  double acc = 0.0;
  const int ncorner = 1 << rs.nd;
  for (int cbits = 0; cbits < ncorner; ++cbits) {
    long long off = 0;
    for (int d = 0; d < rs.nd; ++d)
      if (cbits & (1 << d)) off += rs.sf[d];
    acc += Xf[fb + off];
  }
  Xc[t] = acc / ncorner;
}

// Per-workgroup partial moments over a range of lines along one axis:
// out[blk][0 .. N^2) = sum x_j x_k, [N^2 .. 2N^2) = sum x_j r_k,
// then sum r.r and sum T.T.  Lines are staged through LDS 32 at a time; each
// thread owns fixed entries, so the sums have a fixed order.  N <= 32.
constexpr int kMomLines = 32;
__global__ void __launch_bounds__(256)
k_line_moments(const double *__restrict__ x, const double *__restrict__ r, const double *__restrict__ T,
               const AxisLines al, const long long lines_per_block, double *__restrict__ out) {
  __shared__ double sx[kMomLines * kMaxAxis], sr[kMomLines * kMaxAxis], st[kMomLines * kMaxAxis];
  __shared__ double red[2][256];
  const int N = al.N;
  const int nent = 2 * N * N;
  const long long l0 = (long long)blockIdx.x * lines_per_block;
  const long long l1 = min(l0 + lines_per_block, al.nlines);
  double acc[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) acc[q] = 0.0;
  double cr = 0.0, ct = 0.0;
  for (long long lb = l0; lb < l1; lb += kMomLines) {
    const int nl = (int)min((long long)kMomLines, l1 - lb);
    for (int v = threadIdx.x; v < nl * N; v += blockDim.x) {
      const int li = v / N, i = v - li * N;
      const long long k = line_base(al, lb + li) + i * al.inner;
      sx[li * N + i] = x[k];
      sr[li * N + i] = r[k];
      st[li * N + i] = T[k];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int ent = threadIdx.x + q * 256;
      if (ent < nent) {
        const int half = ent / (N * N);
        const int jk = ent - half * N * N;
        const int j = jk / N, kk = jk - j * N;
        const double *other = half ? sr : sx;
        double s = acc[q];
        for (int li = 0; li < nl; ++li) s += sx[li * N + j] * other[li * N + kk];
        acc[q] = s;
      }
    }
    for (int v = threadIdx.x; v < nl * N; v += blockDim.x) {
      cr += sr[v] * sr[v];
      ct += st[v] * st[v];
    }
    __syncthreads();
  }
  double *o = out + (long long)blockIdx.x * (nent + 2);
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int ent = threadIdx.x + q * 256;
    if (ent < nent) o[ent] = acc[q];
  }
  red[0][threadIdx.x] = cr;
  red[1][threadIdx.x] = ct;
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0, b = 0.0;
    for (int i = 0; i < (int)blockDim.x; ++i) {
      a += red[0][i];
      b += red[1][i];
    }
    o[nent] = a;
    o[nent + 1] = b;
  }
}

// mom[v] = sum over blocks of part[blk][v] (fixed order), v < n.
__global__ void __launch_bounds__(256)
k_sum_blocks(const double *__restrict__ part, const int nblk, const int n, double *__restrict__ mom) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  double s = 0.0;
  for (int b = 0; b < nblk; ++b) s += part[(long long)b * n + v];
  mom[v] = s;
}

// Skew entry e of a line of N: S[i][i+k] for the off-diagonals
// k = 1 .. kClosBands in turn (N - k entries each).
__host__ __device__ __forceinline__ int skew_entries(const int N) {
  return kClosBands * N - kClosBands * (kClosBands + 1) / 2;
}
__device__ __forceinline__ void skew_entry(const int N, int e, int &i, int &k) {
  k = 1;
  while (e >= N - k) {
    e -= N - k;
    ++k;
  }
  i = e;
}

// G[e][f] and b[e] of the quadratic loss from the moments (mom: Mx, Cxr as
// written by k_line_moments) and Ai = A^{-1}, K = A^{-T} A^{-1} (N x N):
//   v_e = (x_{i+k} Ai[:, i] - x_i Ai[:, i+k]) / h,
//   G_ef = sum v_e.v_f,  b_e = sum v_e.r.
__global__ void __launch_bounds__(256)
k_gram(const double *__restrict__ mom, const double *__restrict__ Ai, const double *__restrict__ K,
       const int N, const double h, double *__restrict__ G, double *__restrict__ b) {
  const int P = skew_entries(N);
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const double *Mx = mom;
  const double *Cxr = mom + N * N;
  if (t < P * P) {
    const int e = t / P, f = t - e * P;
    int i, k, j, l;
    skew_entry(N, e, i, k);
    skew_entry(N, f, j, l);
    const double v = Mx[(i + k) * N + (j + l)] * K[i * N + j] - Mx[(i + k) * N + j] * K[i * N + (j + l)] -
                     Mx[i * N + (j + l)] * K[(i + k) * N + j] + Mx[i * N + j] * K[(i + k) * N + (j + l)];
    G[t] = v / (h * h);
  } else if (t < P * P + P) {
    const int e = t - P * P;
    int i, k;
    skew_entry(N, e, i, k);
    double v = 0.0;
    for (int n = 0; n < N; ++n) v += Cxr[(i + k) * N + n] * Ai[n * N + i] - Cxr[i * N + n] * Ai[n * N + (i + k)];
    b[e] = v / h;
  }
}

// ---------------------------------------------------------------------------
// network: MFMA 16x16x16 BF16 tiles of 16 rows
// ---------------------------------------------------------------------------
typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// Round to the nearest BF16 (ties to even); returns the raw 16 bits.
__device__ __forceinline__ short to_bf16(const float v) {
  const uint32_t u = __float_as_uint(v);
  const uint32_t r = (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
  return (short)(uint16_t)r;
}
__device__ __forceinline__ float from_bf16(const short b) {
  return __uint_as_float(((uint32_t)(uint16_t)b) << 16);
}

__global__ void __launch_bounds__(256)
k_to_bf16(const float *__restrict__ in, short *__restrict__ out, const int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = to_bf16(in[i]);
}

// The network state a workgroup keeps in LDS: BF16 copies of W1 ([feat][hid])
// and W2, FP32 biases.
struct ClosNet {
  short W1[kClosFeat * kClosHid];
  short W2[kClosHid];
  float b1[kClosHid];
  float b2;
};

// One tile of 16 rows (r0 ..), one wave.  Lane l: row r0 + l % 16 in the
// B operand and the results.  Forward:
//   H^T (hidden x rows) = W1^T (A: 16 hidden x 16 features) . phi^T (B)
// for hidden 0-15 and 16-31, then A1 = tanh(H + b1); lane l holds
// A1[row l%16][16 hh + 4 (l/16) + j] in a1[hh][j] (the MFMA result layout);
//   s^T = W2^T (A: row 0 only) . A1^T (B: exactly the layout above)
// leaves s[row l%16] in lanes 0-15.  feat: BF16 features, rows x 16.
__device__ __forceinline__ void clos_tile_forward(const ClosNet &net, const short *__restrict__ feat,
                                                  const int r0, const int rows, float (&a1)[2][4], float &s) {
  const int lane = threadIdx.x & 63;
  const int row = r0 + (lane & 15);
  const int kq = 4 * (lane >> 4);  // first k of this lane's four
  bf16x4 phiT;
#pragma unroll
  for (int j = 0; j < 4; ++j) phiT[j] = row < rows ? feat[(long long)row * kClosFeat + kq + j] : (short)0;
  f32x4 h[2];
#pragma unroll
  for (int hh = 0; hh < 2; ++hh) {
    bf16x4 w1T;
#pragma unroll
    for (int j = 0; j < 4; ++j) w1T[j] = net.W1[(kq + j) * kClosHid + 16 * hh + (lane & 15)];
    h[hh] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(w1T, phiT, f32x4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
  }
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int hh = 0; hh < 2; ++hh) {
    bf16x4 aT, w2T;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int hid = 16 * hh + kq + j;
      a1[hh][j] = tanhf(h[hh][j] + net.b1[hid]);
      aT[j] = to_bf16(a1[hh][j]);
      w2T[j] = (lane & 15) == 0 ? net.W2[hid] : (short)0;
    }
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(w2T, aT, acc, 0, 0, 0);
  }
  s = acc[0] + net.b2;  // meaningful in lanes 0-15
}

// Backward of one tile for dL/ds = gs (per row, broadcast to every lane of
// the row): accumulates
//   gW1 (features x hidden) += phi^T (A: 16 features x 16 rows) . gH (B),
// per hidden half, in the MFMA layout (lane l: feature 4 (l/16) + j,
// hidden 16 hh + l % 16), and, on VALU, per-lane partial sums of
// gW2[hid] = sum_rows A1 gs and gb1[hid] = sum_rows gH for the lane's
// hidden units (reduced over lanes by the caller).  gH goes through the
// wave's LDS scratch (16 rows x 32 hidden, BF16) to change layout.
__device__ __forceinline__ void clos_tile_backward(const ClosNet &net, const short *__restrict__ feat,
                                                   const int r0, const int rows, const float (&a1)[2][4],
                                                   const float gs, short *__restrict__ scratch,
                                                   f32x4 (&gW1)[2], float (&gW2p)[2][4], float (&gb1p)[2][4]) {
  const int lane = threadIdx.x & 63;
  const int kq = 4 * (lane >> 4);
  const int rl = lane & 15;
  const float gsr = (r0 + rl) < rows ? gs : 0.f;
  const float gsb = from_bf16(to_bf16(gsr));
#pragma unroll
  for (int hh = 0; hh < 2; ++hh)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int hid = 16 * hh + kq + j;
      const float gh = gsr * from_bf16(net.W2[hid]) * (1.f - a1[hh][j] * a1[hh][j]);
      scratch[rl * kClosHid + hid] = to_bf16(gh);
      gW2p[hh][j] += from_bf16(to_bf16(a1[hh][j])) * gsb;
      gb1p[hh][j] += gh;
    }
  // order this wave's LDS writes before its reads of other lanes' values
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  bf16x4 phiT;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int row = r0 + kq + j;
    phiT[j] = row < rows ? feat[(long long)row * kClosFeat + rl] : (short)0;
  }
#pragma unroll
  for (int hh = 0; hh < 2; ++hh) {
    bf16x4 g;
#pragma unroll
    for (int j = 0; j < 4; ++j) g[j] = scratch[(kq + j) * kClosHid + 16 * hh + rl];
    gW1[hh] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(phiT, g, gW1[hh], 0, 0, 0);
  }
  // and the reads before the next tile's writes
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
}

// Parameter layout (FP32): W1 [16][32] (feature-major), b1 [32], W2 [32], b2.
constexpr int kOffB1 = kClosFeat * kClosHid;
constexpr int kOffW2 = kOffB1 + kClosHid;
constexpr int kOffB2 = kOffW2 + kClosHid;

__device__ __forceinline__ void clos_load_net(ClosNet &net, const float *__restrict__ prm) {
  for (int v = threadIdx.x; v < kClosFeat * kClosHid; v += blockDim.x) net.W1[v] = to_bf16(prm[v]);
  for (int v = threadIdx.x; v < kClosHid; v += blockDim.x) {
    net.b1[v] = prm[kOffB1 + v];
    net.W2[v] = to_bf16(prm[kOffW2 + v]);
  }
  if (threadIdx.x == 0) net.b2 = prm[kOffB2];
}

// Workgroup scratch of the backward pass: per-wave partials and one 16 x 32
// BF16 layout-change tile per wave.
struct ClosBack {
  float gW1[4][kClosFeat * kClosHid];
  float gW2[4][kClosHid];
  float gb1[4][kClosHid];
  float gb2[4];
  short tile[4][16 * kClosHid];
};

// Forward and backward over every row (tiles of 16, wave w takes tiles
// w, w + 4, ...) for dL/ds = gs[row]; leaves d(sum gs s)/d(parameters) in
// grad[kClosParams] (LDS), summed over waves in a fixed order.  Requires
// blockDim.x == 256.
__device__ __forceinline__ void clos_backward_all(const ClosNet &net, const short *__restrict__ feat,
                                                  const int rows, const float *__restrict__ gs, ClosBack &cb,
                                                  float *grad) {
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int kq = 4 * (lane >> 4);
  const int rl = lane & 15;
  f32x4 gW1[2] = {{0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}};
  float gW2p[2][4] = {{0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}};
  float gb1p[2][4] = {{0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}};
  float gb2p = 0.f;
  const int ntiles = (rows + 15) / 16;
  for (int t = wave; t < ntiles; t += 4) {
    const int r0 = 16 * t;
    float a1[2][4], s;
    clos_tile_forward(net, feat, r0, rows, a1, s);
    const float g = (r0 + rl) < rows ? gs[r0 + rl] : 0.f;
    clos_tile_backward(net, feat, r0, rows, a1, g, cb.tile[wave], gW1, gW2p, gb1p);
    if (kq == 0) gb2p += g;
  }
  // sum the per-row partials over the 16 rows of each lane group
#pragma unroll
  for (int hh = 0; hh < 2; ++hh)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int o = 1; o < 16; o <<= 1) {
        gW2p[hh][j] += __shfl_xor(gW2p[hh][j], o);
        gb1p[hh][j] += __shfl_xor(gb1p[hh][j], o);
      }
#pragma unroll
  for (int o = 1; o < 16; o <<= 1) gb2p += __shfl_xor(gb2p, o);
  if (rl == 0) {
#pragma unroll
    for (int hh = 0; hh < 2; ++hh)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        cb.gW2[wave][16 * hh + kq + j] = gW2p[hh][j];
        cb.gb1[wave][16 * hh + kq + j] = gb1p[hh][j];
      }
  }
  if (lane == 0) cb.gb2[wave] = gb2p;
  // gW1 in the MFMA layout: lane l holds [feature kq + j][hidden 16 hh + l % 16]
#pragma unroll
  for (int hh = 0; hh < 2; ++hh)
#pragma unroll
    for (int j = 0; j < 4; ++j) cb.gW1[wave][(kq + j) * kClosHid + 16 * hh + rl] = gW1[hh][j];
  __syncthreads();
  for (int v = threadIdx.x; v < kClosParams; v += blockDim.x) {
    float a;
    if (v < kOffB1)
      a = ((cb.gW1[0][v] + cb.gW1[1][v]) + cb.gW1[2][v]) + cb.gW1[3][v];
    else if (v < kOffW2)
      a = ((cb.gb1[0][v - kOffB1] + cb.gb1[1][v - kOffB1]) + cb.gb1[2][v - kOffB1]) + cb.gb1[3][v - kOffB1];
    else if (v < kOffB2)
      a = ((cb.gW2[0][v - kOffW2] + cb.gW2[1][v - kOffW2]) + cb.gW2[2][v - kOffW2]) + cb.gW2[3][v - kOffW2];
    else
      a = ((cb.gb2[0] + cb.gb2[1]) + cb.gb2[2]) + cb.gb2[3];
    grad[v] = a;
  }
  __syncthreads();
}

// s[row] for every row; one wave per tile, any number of workgroups.
__global__ void __launch_bounds__(256)
k_clos_eval(const float *__restrict__ prm, const short *__restrict__ feat, const int rows, float *__restrict__ s) {
  __shared__ ClosNet net;
  clos_load_net(net, prm);
  __syncthreads();
  const int ntiles = (rows + 15) / 16;
  const int wave = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const int nw = gridDim.x * (blockDim.x >> 6);
  const int lane = threadIdx.x & 63;
  for (int t = wave; t < ntiles; t += nw) {
    float a1[2][4], sv;
    clos_tile_forward(net, feat, 16 * t, rows, a1, sv);
    if (lane < 16 && 16 * t + lane < rows) s[16 * t + lane] = sv;
  }
}

// grad = d(sum gs s)/d(parameters) at prm (one workgroup of 256 threads).
__global__ void __launch_bounds__(256)
k_clos_grad(const float *__restrict__ prm, const short *__restrict__ feat, const int rows,
            const float *__restrict__ gs, float *__restrict__ grad) {
  __shared__ ClosNet net;
  __shared__ ClosBack cb;
  __shared__ float g[kClosParams];
  clos_load_net(net, prm);
  __syncthreads();
  clos_backward_all(net, feat, rows, gs, cb, g);
  for (int v = threadIdx.x; v < kClosParams; v += blockDim.x) grad[v] = g[v];
}

// Training problem: rows grouped by (draw, axis); group q owns rows
// [gstart[q], gstart[q+1]) and the quadratic (G_q, b_q, c_q, t_q) of its
// P_q = gstart[q+1] - gstart[q] entries (G_q at goff[q], P_q x P_q; b_q at
// boff[q]; c_q, t_q at ct[2q], ct[2q + 1]).
struct ClosGroups {
  const int *gstart;
  const int *group_of_row;
  const long long *goff;
  const int *boff;
  const double *G;
  const double *b;
  const double *ct;
  int ngroups;
};

// n_steps Adam steps (beta1 0.9, beta2 0.999, eps 1e-8) of the mean group
// loss, one workgroup of 256 threads.  prm (FP32 master weights) and the
// moment estimates m, v are read at the start and written back at the end;
// loss[step] receives the loss at the weights the step starts from.
// s and gs are scratch arrays of rows floats.
__global__ void __launch_bounds__(256)
k_clos_train(float *__restrict__ prm, float *__restrict__ mom1, float *__restrict__ mom2, const int t0,
             const short *__restrict__ feat, const int rows, const ClosGroups gr, const int n_steps,
             const float lr, float *__restrict__ s, float *__restrict__ gs, float *__restrict__ loss) {
  __shared__ ClosNet net;
  __shared__ ClosBack cb;
  __shared__ float w[kClosParams], m1[kClosParams], m2[kClosParams], g[kClosParams];
  __shared__ double lred[256];
  for (int v = threadIdx.x; v < kClosParams; v += blockDim.x) {
    w[v] = prm[v];
    m1[v] = mom1[v];
    m2[v] = mom2[v];
  }
  __syncthreads();
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int ntiles = (rows + 15) / 16;
  const double inv_ng = 1.0 / gr.ngroups;
  for (int step = 0; step < n_steps; ++step) {
    clos_load_net(net, w);
    __syncthreads();
    // forward
    for (int t = wave; t < ntiles; t += 4) {
      float a1[2][4], sv;
      clos_tile_forward(net, feat, 16 * t, rows, a1, sv);
      if (lane < 16 && 16 * t + lane < rows) s[16 * t + lane] = sv;
    }
    __threadfence_block();
    __syncthreads();
    // loss and dL/ds
    double lp = 0.0;
    for (int row = threadIdx.x; row < rows; row += blockDim.x) {
      const int q = gr.group_of_row[row];
      const int i0 = gr.gstart[q];
      const int P = gr.gstart[q + 1] - i0;
      const int e = row - i0;
      const double *Gq = gr.G + gr.goff[q] + (long long)e * P;
      double Gs = 0.0;
      for (int f = 0; f < P; ++f) Gs += Gq[f] * (double)s[i0 + f];
      const double be = gr.b[gr.boff[q] + e];
      const double tq = gr.ct[2 * q + 1];
      const double se = s[row];
      gs[row] = (float)(2.0 * (Gs - be) / tq * inv_ng);
      lp += (se * Gs - 2.0 * be * se) / tq * inv_ng;
      if (e == 0) lp += gr.ct[2 * q] / tq * inv_ng;
    }
    lred[threadIdx.x] = lp;
    __threadfence_block();
    __syncthreads();
    if (threadIdx.x == 0) {
      double a = 0.0;
      for (int i = 0; i < 256; ++i) a += lred[i];
      loss[step] = (float)a;
    }
    // backward and Adam
    clos_backward_all(net, feat, rows, gs, cb, g);
    const int tt = t0 + step + 1;
    const float c1 = 1.f / (1.f - powf(0.9f, (float)tt));
    const float c2 = 1.f / (1.f - powf(0.999f, (float)tt));
    for (int v = threadIdx.x; v < kClosParams; v += blockDim.x) {
      m1[v] = 0.9f * m1[v] + 0.1f * g[v];
      m2[v] = 0.999f * m2[v] + 0.001f * g[v] * g[v];
      w[v] -= lr * (m1[v] * c1) / (sqrtf(m2[v] * c2) + 1e-8f);
    }
    __syncthreads();
  }
  for (int v = threadIdx.x; v < kClosParams; v += blockDim.x) {
    prm[v] = w[v];
    mom1[v] = m1[v];
    mom2[v] = m2[v];
  }
}

}  // namespace chfpe
