// Device code of the gfx950 CHFPE solver.
//
// Every state buffer holds the smooth factor h_n of W_n = exp(-beta H/2) h_n
// (the factorization of Sec. III A).  In h the hierarchy, Eq. (eq:HEOM), reads
//   dh_n/dt = L h_n - sum_s n_s gamma_s h_n
//           + sum_s V_s' (d/dp_s - beta p_s/2m_s) h_{n+e_s}
//           + sum_s n_s (m_s zeta_s gamma_s/beta) V_s' (d/dp_s + beta p_s/2m_s) h_{n-e_s},
// L h = sum_s F_s dh/dp_s - (p_s/m_s) dh/dq_s.
// The right-hand side is split by axis family so that every compact
// derivative (Sec. III B) sees whole lines:
//
//   k_pblock  -- for every element n, blocks of the innermost p axes (p_M,
//                and p_{M-1} for two or three modes; contiguous in memory)
//                are staged through LDS.  It forms the field the p_s
//                derivative acts on,
//                  G_{n,s} = F_s W_n + V_s' W_{n+e_s} + n_s zeta_s gamma_s (m_s/beta) V_s' W_{n-e_s},
//                solves those p_s lines (Thomas from both ends, two lanes per
//                line, streamed through LDS) and adds the pointwise terms
//                  sum_s V_s' p_s [ (n_s zeta_s gamma_s/2) h_{n-e_s} - (beta/2m_s) h_{n+e_s} ]
//                  - sum_s n_s gamma_s h_n.
//                D_p(F W) = F D_p W and D_p(V' W) = V' D_p W because F_s and
//                V_s' do not depend on p_s, so one solve per (n, s) covers the
//                Liouvillian, Phi and the derivative part of Theta.  For
//                three modes the p_1 derivative of G_{n,1} is taken by a
//                k_qpass over (q_1, p_1), which forms that field itself.
//   k_qpass   -- the -(p_s/m_s) D_{q_s} W_n terms.  A tile is one or two
//                q axes at full length times a chunk of consecutive p-block
//                positions; each thread holds one q_a line in registers, a
//                second q_b axis goes through LDS.  The last q pass of a
//                stage also applies the classical RK4 stage update.
//
// All state arithmetic is in the template type T (double, or float for FP32
// branch states); tables and reductions are FP64.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <type_traits>

namespace chfpe {

constexpr int kMaxAxis = 48;      // longest supported axis
constexpr int kTab = 48;          // per-mode stride of 1-D tables

// ---------------------------------------------------------------------------
// Thomas factors of the constant tridiagonal matrix tridiag(1/3, 1, 1/3).
// The forward factors do not depend on the line length (the first row is
// [1, 1/3] for every N), so one table serves every axis.
// ---------------------------------------------------------------------------
struct ThomasTable {
  double cp[kMaxAxis];   // super-diagonal after elimination
  double inv[kMaxAxis];  // 1 / pivot
};

constexpr ThomasTable make_thomas() {
  ThomasTable t{};
  const double alpha = 1.0 / 3.0;
  t.cp[0] = alpha;
  t.inv[0] = 1.0;
  for (int i = 1; i < kMaxAxis; ++i) {
    const double piv = 1.0 - alpha * t.cp[i - 1];
    t.inv[i] = 1.0 / piv;
    t.cp[i] = alpha / piv;
  }
  return t;
}

constexpr ThomasTable kThomas = make_thomas();

// Fused multiply-add in the arithmetic type (the double builtin would
// widen a float operation).
template <typename T>
__device__ __forceinline__ T fma_t(const T a, const T b, const T c) {
  if constexpr (sizeof(T) == 4)
    return __builtin_fmaf(a, b, c);
  else
    return __builtin_fma(a, b, c);
}

// Right-hand side of the compact scheme at position i of a line,
//   (1/3) f'_{i-1} + f'_i + (1/3) f'_{i+1}
//       = ca (f_{i+1} - f_{i-1}) + cb (f_{i+2} - f_{i-2}),  ca = 7/(9h), cb = 1/(36h),
// or, with a closure (CLOS), with the per-position weights of a table ct:
//   sum_{k=1..3} pk[i] f_{i+k} + mk[i] f_{i-k},
// rows p1, m1, p2, m2, p3, m3 of kTab entries each.  A closure adds a
// skew-symmetric band S to the scheme's right-hand side (A y = (B + S) f / h),
// so the plain weights are p1 = -m1 = ca, p2 = -m2 = cb, p3 = m3 = 0.
constexpr int kClosRows = 6;  // table rows per orientation
template <typename T, bool CLOS>
__device__ __forceinline__ T stencil_rhs(const int i, const T fm3, const T fm2, const T fm1, const T fp1,
                                         const T fp2, const T fp3, const T ca, const T cb, const double *ct) {
  if constexpr (CLOS)
    return T(ct[i]) * fp1 + T(ct[kTab + i]) * fm1 + T(ct[2 * kTab + i]) * fp2 + T(ct[3 * kTab + i]) * fm2 +
           T(ct[4 * kTab + i]) * fp3 + T(ct[5 * kTab + i]) * fm3;
  else
    return ca * (fp1 - fm1) + cb * (fp2 - fm2);
}

// Compact sixth-order first derivative of one line held in registers.
// On entry f[0..N) holds the line and f[N..NMAX) must be zero (values beyond
// the box are zero); on exit f[0..N) holds the derivative.
template <typename T, int NMAX, bool CLOS = false>
__device__ __forceinline__ void compact_deriv(T (&f)[NMAX], const int N, const T ca, const T cb,
                                              const double *ct = nullptr) {
  constexpr T third = T(1.0 / 3.0);
  T d[NMAX];
#pragma unroll
  for (int i = 0; i < NMAX; ++i) {
    if (i < N) {
      const T fm1 = (i >= 1) ? f[i >= 1 ? i - 1 : 0] : T(0);
      const T fm2 = (i >= 2) ? f[i >= 2 ? i - 2 : 0] : T(0);
      const T fm3 = (i >= 3) ? f[i >= 3 ? i - 3 : 0] : T(0);
      const T fp1 = (i + 1 < NMAX) ? f[i + 1 < NMAX ? i + 1 : NMAX - 1] : T(0);
      const T fp2 = (i + 2 < NMAX) ? f[i + 2 < NMAX ? i + 2 : NMAX - 1] : T(0);
      const T fp3 = (i + 3 < NMAX) ? f[i + 3 < NMAX ? i + 3 : NMAX - 1] : T(0);
      const T r = stencil_rhs<T, CLOS>(i, fm3, fm2, fm1, fp1, fp2, fp3, ca, cb, ct);
      if (i == 0)
        d[0] = r;
      else
        d[i] = (r - third * d[i >= 1 ? i - 1 : 0]) * T(kThomas.inv[i]);
    }
  }
#pragma unroll
  for (int i = NMAX - 1; i >= 0; --i) {
    if (i < N) {
      if (i == N - 1)
        f[i] = d[i];
      else
        f[i] = d[i] - T(kThomas.cp[i]) * f[i + 1 < NMAX ? i + 1 : NMAX - 1];
    }
  }
}

// Same, for a line of exactly N values (no guards; N known at compile time).
template <typename T, int N, bool CLOS = false>
__device__ __forceinline__ void compact_deriv_exact(T (&f)[N], const T ca, const T cb,
                                                    const double *ct = nullptr) {
  constexpr T third = T(1.0 / 3.0);
  T d[N];
#pragma unroll
  for (int i = 0; i < N; ++i) {
    const T fm1 = i >= 1 ? f[i >= 1 ? i - 1 : 0] : T(0);
    const T fm2 = i >= 2 ? f[i >= 2 ? i - 2 : 0] : T(0);
    const T fm3 = i >= 3 ? f[i >= 3 ? i - 3 : 0] : T(0);
    const T fp1 = i + 1 < N ? f[i + 1 < N ? i + 1 : 0] : T(0);
    const T fp2 = i + 2 < N ? f[i + 2 < N ? i + 2 : 0] : T(0);
    const T fp3 = i + 3 < N ? f[i + 3 < N ? i + 3 : 0] : T(0);
    const T r = stencil_rhs<T, CLOS>(i, fm3, fm2, fm1, fp1, fp2, fp3, ca, cb, ct);
    d[i] = i == 0 ? r : (r - third * d[i >= 1 ? i - 1 : 0]) * T(kThomas.inv[i]);
  }
  f[N - 1] = d[N - 1];
#pragma unroll
  for (int i = N - 2; i >= 0; --i) f[i] = d[i] - T(kThomas.cp[i]) * f[i + 1];
}

// Line of N <= NMAX values; takes the unguarded path when N == NMAX.
template <typename T, int NMAX, bool CLOS = false>
__device__ __forceinline__ void compact_line(T (&f)[NMAX], const int N, const T ca, const T cb,
                                             const double *ct = nullptr) {
  if (N == NMAX)
    compact_deriv_exact<T, NMAX, CLOS>(f, ca, cb, ct);
  else
    compact_deriv<T, NMAX, CLOS>(f, N, ca, cb, ct);
}

// Same derivative of a line in registers, overwritten in place with O(1)
// extra registers: the forward sweep stores d_i over f_i once the stencil no
// longer needs f_i as a right neighbour (a window of the three values
// behind it is kept), and back substitution overwrites d_i with the result.
// f[N..NMAX) must be zero on entry.
template <typename T, int NMAX, bool CLOS = false>
__device__ __forceinline__ void compact_inplace(T (&f)[NMAX], const int N, const T ca, const T cb,
                                                const double *ct = nullptr) {
  constexpr T third = T(1.0 / 3.0);
  T fm3 = T(0), fm2 = T(0), fm1 = T(0), dprev = T(0);
#pragma unroll
  for (int i = 0; i < NMAX; ++i) {
    if (i < N) {
      const T f0 = f[i];
      const T fp1 = (i + 1 < NMAX) ? f[i + 1 < NMAX ? i + 1 : 0] : T(0);
      const T fp2 = (i + 2 < NMAX) ? f[i + 2 < NMAX ? i + 2 : 0] : T(0);
      const T fp3 = (CLOS && i + 3 < NMAX) ? f[i + 3 < NMAX ? i + 3 : 0] : T(0);
      const T r = stencil_rhs<T, CLOS>(i, fm3, fm2, fm1, fp1, fp2, fp3, ca, cb, ct);
      const T d = i == 0 ? r : (r - third * dprev) * T(kThomas.inv[i]);
      fm3 = fm2;
      fm2 = fm1;
      fm1 = f0;
      f[i] = d;
      dprev = d;
    }
  }
#pragma unroll
  for (int i = NMAX - 2; i >= 0; --i)
    if (i < N - 1) f[i] = f[i] - T(kThomas.cp[i]) * f[i + 1];
}

// Same derivative for a line of N values held in LDS at base + i * stride,
// in place, with O(1) registers: a seven-value window of the input moves
// ahead of the forward sweep, which stores d_i over f_i once f_i is in the
// window; the backward sweep then overwrites d_i with the result.
template <typename T, bool CLOS = false>
__device__ __forceinline__ void compact_lds(T *G, const int base, const int stride, const int N, const T ca,
                                            const T cb, const double *ct = nullptr) {
  constexpr T third = T(1.0 / 3.0);
  T fm3 = T(0), fm2 = T(0), fm1 = T(0), f0 = G[base], fp1 = N > 1 ? G[base + stride] : T(0);
  T fp2 = N > 2 ? G[base + 2 * stride] : T(0);
  T fp3 = N > 3 ? G[base + 3 * stride] : T(0);
  T dprev = T(0);
  for (int i = 0; i < N; ++i) {
    const T r = stencil_rhs<T, CLOS>(i, fm3, fm2, fm1, fp1, fp2, fp3, ca, cb, ct);
    const T d = i == 0 ? r : (r - third * dprev) * T(kThomas.inv[i]);
    G[base + i * stride] = d;
    dprev = d;
    fm3 = fm2;
    fm2 = fm1;
    fm1 = f0;
    f0 = fp1;
    fp1 = fp2;
    fp2 = fp3;
    fp3 = (i + 4 < N) ? G[base + (i + 4) * stride] : T(0);
  }
  T y = dprev;
  for (int i = N - 2; i >= 0; --i) {
    y = G[base + i * stride] - T(kThomas.cp[i]) * y;
    G[base + i * stride] = y;
  }
}

// Same derivative for a line of exactly N values in LDS, solved by two
// neighbouring lanes (lane bit 0 = half): each eliminates N/2 equations from
// its own end of the line, the pair couples its last two unknowns through one
// exchange, and each back-substitutes its half.  tridiag(1/3, 1, 1/3) is
// persymmetric, so the far half is the same sweep on the mirrored line: the
// mirror reverses the load order and flips the sign of the stencil (ca, cb;
// a closure table carries its own mirrored rows at ct + kClosRows kTab), and the
// coupling of the two last equations
//   x_{H-1} + c x_H = d_own,  x_H + c x_{H-1} = d_partner  (c = cp_{H-1})
// gives x_own = (d_own - c d_partner) / (1 - c^2) in either lane.
// Both lanes of a pair must call this together.
template <typename T, int N, bool CLOS = false>
__device__ __forceinline__ void compact_split(T *G, const int base, const int stride, const int half,
                                              T ca, T cb, const double *ct = nullptr) {
  static_assert(N % 2 == 0 && N >= 6, "split solve needs an even line of at least 6");
  constexpr int H = N / 2;
  constexpr int R = CLOS ? 3 : 2;  // stencil reach
  constexpr int NL = H + R;        // values this lane reads: its half and R past the middle
  constexpr int PF = 2;            // LDS reads issued this many positions ahead of use
  constexpr double cm = kThomas.cp[H - 1];
  constexpr double inv1mc2 = 1.0 / (1.0 - cm * cm);
  const int step = half ? -stride : stride;
  const int start = base + (half ? (N - 1) * stride : 0);
  if (half) {
    ca = -ca;
    cb = -cb;
  }
  const double *cto = CLOS ? ct + (half ? kClosRows * kTab : 0) : ct;
  // Streamed through LDS so that few values are live at once: the forward
  // sweep stores d_i over f_i (already read), the back substitution stores
  // x_i over d_i.  The partner lane (same wave) overwrites its half from its
  // own end inward, so the R values past the middle are read before any
  // store; own values are read PF + R positions ahead of the sweep.  f and
  // dv are indexed by compile-time constants only (registers, not memory).
  T f[NL];
#pragma unroll
  for (int j = H; j < NL; ++j) f[j] = G[start + j * step];
#pragma unroll
  for (int j = 0; j < H && j < R + PF; ++j) f[j] = G[start + j * step];
  T dprev = T(0);
#pragma unroll
  for (int i = 0; i < H; ++i) {
    if (i + R + PF < H) f[i + R + PF < H ? i + R + PF : 0] = G[start + (i + R + PF) * step];
    const T fm1 = i >= 1 ? f[i >= 1 ? i - 1 : 0] : T(0);
    const T fm2 = i >= 2 ? f[i >= 2 ? i - 2 : 0] : T(0);
    const T fm3 = (CLOS && i >= 3) ? f[i >= 3 ? i - 3 : 0] : T(0);
    const T fp3 = CLOS ? f[i + 3 < NL ? i + 3 : NL - 1] : T(0);
    const T r = stencil_rhs<T, CLOS>(i, fm3, fm2, fm1, f[i + 1], f[i + 2], fp3, ca, cb, cto);
    // d_i = (r_i - d_{i-1}/3) / pivot_i, one dependent FMA
    const T d = i == 0 ? r : fma_t(T(-kThomas.inv[i] / 3.0), dprev, r * T(kThomas.inv[i]));
    G[start + i * step] = d;
    dprev = d;
  }
  const T other = __shfl_xor(dprev, 1);
  T x = (dprev - T(cm) * other) * T(inv1mc2);
  G[start + (H - 1) * step] = x;
  T dv[H];
#pragma unroll
  for (int j = H - 2; j >= 0 && j >= H - 2 - PF; --j) dv[j] = G[start + j * step];
#pragma unroll
  for (int i = H - 2; i >= 0; --i) {
    if (i - PF - 1 >= 0 && i - PF - 1 < H - 2 - PF) dv[i - PF - 1 >= 0 ? i - PF - 1 : 0] = G[start + (i - PF - 1) * step];
    x = dv[i] - T(kThomas.cp[i]) * x;
    G[start + i * step] = x;
  }
}

// Same solve as compact_split with the half-line in registers: each lane
// reads its N/2 values and the R values past the middle from LDS first (all
// reads independent of each other), eliminates and back-substitutes in
// registers, and writes its half at the end, so no LDS access sits in the
// elimination chain.  The partner lane reads before either lane writes (the
// writes depend on the exchanged value).  Both lanes of a pair must call this
// together.
template <typename T, int N, bool CLOS = false>
__device__ __forceinline__ void compact_split_regs(T *G, const int base, const int stride, const int half, T ca,
                                                   T cb, const double *ct = nullptr) {
  static_assert(N % 2 == 0 && N >= 6, "split solve needs an even line of at least 6");
  constexpr int H = N / 2;
  constexpr int R = CLOS ? 3 : 2;  // stencil reach
  constexpr int NL = H + R;
  constexpr double cm = kThomas.cp[H - 1];
  constexpr double inv1mc2 = 1.0 / (1.0 - cm * cm);
  const int step = half ? -stride : stride;
  const int start = base + (half ? (N - 1) * stride : 0);
  if (half) {
    ca = -ca;
    cb = -cb;
  }
  const double *cto = CLOS ? ct + (half ? kClosRows * kTab : 0) : ct;
  T f[NL];
#pragma unroll
  for (int j = 0; j < NL; ++j) f[j] = G[start + j * step];
  T d[H];
#pragma unroll
  for (int i = 0; i < H; ++i) {
    const T fm1 = i >= 1 ? f[i >= 1 ? i - 1 : 0] : T(0);
    const T fm2 = i >= 2 ? f[i >= 2 ? i - 2 : 0] : T(0);
    const T fm3 = (CLOS && i >= 3) ? f[i >= 3 ? i - 3 : 0] : T(0);
    const T fp3 = CLOS ? f[i + 3 < NL ? i + 3 : NL - 1] : T(0);
    const T r = stencil_rhs<T, CLOS>(i, fm3, fm2, fm1, f[i + 1], f[i + 2], fp3, ca, cb, cto);
    d[i] = i == 0 ? r : fma_t(T(-kThomas.inv[i] / 3.0), d[i >= 1 ? i - 1 : 0], r * T(kThomas.inv[i]));
  }
  const T other = __shfl_xor(d[H - 1], 1);
  T x = (d[H - 1] - T(cm) * other) * T(inv1mc2);
  d[H - 1] = x;
#pragma unroll
  for (int i = H - 2; i >= 0; --i) {
    x = d[i] - T(kThomas.cp[i]) * x;
    d[i] = x;
  }
#pragma unroll
  for (int i = 0; i < H; ++i) G[start + i * step] = d[i];
}

// Element idx of a workgroup-uniform base pointer.  The byte offset is formed
// in 32 bits, so the access takes the scalar-base form (one 32-bit offset
// register shared by every array indexed alike); callers keep idx * sizeof(T)
// below 2^32.
template <typename T>
__device__ __forceinline__ const T &at_u32(const T *__restrict__ base, const uint32_t idx) {
  return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) + idx * (uint32_t)sizeof(T));
}
template <typename T>
__device__ __forceinline__ T &at_u32(T *__restrict__ base, const uint32_t idx) {
  return *reinterpret_cast<T *>(reinterpret_cast<char *>(base) + idx * (uint32_t)sizeof(T));
}

// ---------------------------------------------------------------------------
// Geometry and tables passed by value to every kernel.
// ---------------------------------------------------------------------------
struct Geom {
  int M;         // modes
  int ne;        // hierarchy elements
  int nbatch;    // independent states (t1 branches) stored back to back
  int Nq[3], Np[3];
  int Q;         // prod Nq
  int P;         // prod Np (one p-block)
  int QS[3];     // stride of q_s in the q-linear index
  int PS[3];     // stride of p_s inside a p-block
  int PSp[3];    // same stride in the LDS layout (one pad value per p_M row)
  long long E;   // points per element = Q * P
  double dq_ca[3], dq_cb[3];  // 7/(9 h), 1/(36 h) for q_s
  double dp_ca[3], dp_cb[3];  // same for p_s
  double bm[3];               // beta / (2 m_s)
  // Hermite basis in p (a_s = sqrt(2 m_s / beta)): a_s / (sqrt(2) m_s),
  // 1 / (sqrt(2) a_s) and sqrt(2) / a_s
  double ha[3], hf[3], hl[3];
};

struct Tabs {
  const double *F;      // [s][qlin]  dU/dq_s
  const double *VpQ;    // [s][qlin]  V_s'(q_s) on the q grid
  const double *Vp;     // [s][j]     V_s'(q_s,j)          (stride kTab)
  const double *pm;     // [s][j]     p_s,j / m_s          (stride kTab)
  const double *pg;     // [s][j]     p_s,j                (stride kTab)
  const int *up;        // [e][s]     index of n + e_s or -1
  const int *dn;        // [e][s]     index of n - e_s or -1
  const double *cc;     // [e][s]     n_s zeta_s gamma_s m_s / beta
  const double *tc;     // [e][s]     n_s zeta_s gamma_s
  const double *damp;   // [e]        sum_s n_s gamma_s
  const double *clos;   // [axis][orientation][6][kTab] closure stencil weights (axis ids
                        // 0..M-1 q_s, M..2M-1 p_s; orientation 1 = mirrored line)
};

// Consecutive workgroup ids are dispatched round-robin over the 8 XCDs.
// Give each XCD a contiguous range of tasks so that tasks touching the same
// data (all elements of one q run) share that XCD's L2.  nblk is a multiple
// of 8 chosen by the host.
__device__ __forceinline__ int xcd_task(const int bid, const int nblk) {
  const int per = nblk >> 3;
  return (bid & 7) * per + (bid >> 3);
}

// Chunked form: workgroups go to the XCDs in turn (bid & 7), and each XCD
// takes every eighth chunk of G consecutive tasks, so the eight XCDs walk
// one task order side by side (the shared last-level cache then sees one
// front) while neighbouring tasks of a chunk share an L2.  Needs nblk to
// be a multiple of 8 G.
__device__ __forceinline__ int xcd_chunk_task(const int bid, const int G) {
  const int j = bid >> 3;
  return (((j / G) << 3) + (bid & 7)) * G + j % G;
}

// ---------------------------------------------------------------------------
// Tile descriptions passed by value.
// ---------------------------------------------------------------------------
// k_pblock: the innermost NB p axes (NB = 1 for one mode, else 2) form a
// contiguous block of rows x cols values (cols = Np_M; rows = Np_{M-1}, or 1
// for one mode); a task is one element and a run of nb consecutive blocks.
// Thread t owns column t % cols of every RG-th row of the run, so global
// accesses are row-contiguous and coordinates need no division per point.
// LDS holds the fields of the row axis (p_M) and column axis (p_{M-1}) with
// one pad value per row.
struct PBlock {
  int NB;            // p axes inside a block (1 or 2)
  int rows, cols;    // block shape
  int B;             // rows * cols
  int nb;            // blocks per task
  int nblocks;       // blocks per element
  int bpq;           // blocks per q point (P / B)
  int RG;            // row groups; threads = cols * RG
  int tileP;         // padded values of one LDS field = nb * rows * (cols + 1)
  int split;         // 1: two lanes per line (compact_split) where the line length allows
  int run;           // task order: `run` consecutive block groups of one state, then the
                     // next (branch, element); tasks past the last block exit
  int ntasks, nblk;
};

// Field of a strided-axis line pass.
enum Field : int {
  FQ = 0,  // W_n along q_s, coefficient -p_s/m_s
  FP = 1,  // G_{n,s} = F_s W_n + V_s'(W_{n+e_s} + cc W_{n-e_s}) along p_s, coefficient 1
  FX = 2   // dX/dq_s W_n along p_s (optical excitation), coefficient 1
};

// k_qpass: a tile is one element, full lines along axis a (one per thread,
// in registers) and optionally axis b (through LDS), times pc consecutive
// positions of the innermost contiguous run (length `run`), with all other
// indices fixed.  Axis ids: 0..M-1 are q_1..q_M, M..2M-1 are p_1..p_M.
struct QPass {
  int a, b;                 // axis ids; b < 0 for a single-axis pass
  int sa_mode, sb_mode;     // mode index s of axes a and b
  int Na, Nb;
  int sa, sb;               // strides within an element
  int run;                  // length of the contiguous run the chunks tile
  int nrest;                // combinations of the remaining outer indices
  int rN[3];                // their lengths (outer first)
  int rS[3];                // their strides within an element
  int pc;                   // run positions per tile
  int nchunk;               // tiles per run
  int ntasks, nblk;
  double ca_a, cb_a, ca_b, cb_b;
};

// ---------------------------------------------------------------------------
// k_pblock
// ---------------------------------------------------------------------------
// RHS mode: out = pointwise terms (all s) + sum_{s in block} D_{p_s} G_{n,s},
//   G_{n,s} = F_s h_n + V_s' (h_{n+e_s} + n_s (m_s zeta_s gamma_s/beta) h_{n-e_s}),
//   pointwise = sum_s V_s' p_s [ (n_s zeta_s gamma_s/2) h_{n-e_s} - (beta/2m_s) h_{n+e_s} ]
//               - sum_s n_s gamma_s h_n.
// PERTURB: out = -sum_s dX/dq_s (beta p_s/2m_s) h_n + sum_{s in block} D_{p_s}(dX/dq_s h_n)
//   (grad[s][qlin] = dX/dq_s): X^x W = sum_s dX/dq_s dW/dp_s written for h, Eq. (Opticalexc).
// Three phases: (1) one pass over the run loads h_n and its neighbours once,
// keeps the pointwise terms in registers and writes both derivative fields to
// LDS; (2) row and column lines are solved together; (3) one pass writes out.
// T: type of X and of the arithmetic; TO: type of out.  A batch of nbatch
// states is laid out [branch][n][q][p]; tasks cover every (branch, n).
template <typename T, typename TO, int NMAX, int RPT, int MM, bool PERTURB, bool CLOS = false>
__global__ void __launch_bounds__(256, (NMAX == 32 && MM == 2) ? 6 : NMAX <= 24 ? 5 : NMAX <= 32 ? 4 : 3)
k_pblock(const Geom g, const Tabs tb, const PBlock pb, const T *__restrict__ X, TO *__restrict__ out,
         const double *__restrict__ grad) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T *Ga = reinterpret_cast<T *>(smem_raw);  // row axis p_M
  T *Gb = Ga + pb.tileP;                    // column axis p_{M-1} (two or three modes)
  const int task = xcd_task(blockIdx.x, pb.nblk);
  if (task >= pb.ntasks) return;
  constexpr int NB = MM == 1 ? 1 : 2;
  constexpr int sa = MM - 1;  // row axis
  constexpr int sb = MM - 2;  // column axis (NB == 2)
  const int ne_all = g.ne * g.nbatch;
  const int jr = task % pb.run;
  const int t2 = task / pb.run;
  const int ea = t2 % ne_all;  // (branch, element)
  const int br = ea / g.ne;
  const int e = ea - br * g.ne;
  const int b0 = ((t2 / ne_all) * pb.run + jr) * pb.nb;
  if (b0 >= pb.nblocks) return;  // padding of the last run (whole workgroup)
  const int nbt = min(pb.nb, pb.nblocks - b0);
  const int rows = pb.rows, cols = pb.cols, cp = pb.cols + 1;
  const int nrows = nbt * rows;
  const int tid = threadIdx.x;
  const int col = tid % cols;
  const int rg = min(tid / cols, pb.RG - 1);  // surplus threads duplicate the last group's work
  const bool owner = tid < pb.RG * cols;
  const int Q = g.Q;

  // base pointers of the run in this element and its neighbours; a missing
  // neighbour points at the element itself and gets a zero factor, so every
  // load below is unconditional
  const long long run0 = (long long)b0 * pb.B;
  const T *Xe = X + (long long)ea * g.E + run0;
  TO *Oe = out + (long long)ea * g.E + run0;
  const T *Xb = X + (long long)br * g.ne * g.E;  // this branch's element 0
  const T *Xu[MM];
  const T *Xd[MM];
  double fu[MM], cc[MM], tcv[MM];
#pragma unroll
  for (int s = 0; s < MM; ++s) {
    const int up = PERTURB ? -1 : tb.up[e * 3 + s];
    const int dn = PERTURB ? -1 : tb.dn[e * 3 + s];
    Xu[s] = up >= 0 ? Xb + (long long)up * g.E + run0 : Xe;
    Xd[s] = dn >= 0 ? Xb + (long long)dn * g.E + run0 : Xe;
    fu[s] = up >= 0 ? 1.0 : 0.0;
    cc[s] = PERTURB ? 0.0 : tb.cc[e * 3 + s];        // zero when n_s = 0
    tcv[s] = PERTURB ? 0.0 : 0.5 * tb.tc[e * 3 + s];  // zero when n_s = 0
  }
  const double dmp = PERTURB ? 0.0 : tb.damp[e];
  const double p_col = tb.pg[sa * kTab + col];

  // ---- phase 1: rows R_k = k RG + rg of the run --------------------------------
  // Two or three modes: the host picks RG | rows, so the RG rows of batch k lie
  // in one block, (k RG) / rows, and all but the row index is uniform over the
  // workgroup (table values of the q point come through scalar loads).  Rows
  // past the run re-read block 0 and are not stored.  One mode: a block is one
  // row and row R is block R.
  int off[RPT], qlk[RPT], rk[RPT], jok[RPT];
  bool vk[RPT];
#pragma unroll
  for (int k = 0; k < RPT; ++k) {
    if constexpr (NB == 2) {
      const int R0 = k * pb.RG;
      const int bl = R0 / rows;
      vk[k] = bl < nbt;
      const int ob = b0 + (vk[k] ? bl : 0);
      qlk[k] = ob / pb.bpq;
      jok[k] = ob - qlk[k] * pb.bpq;
      rk[k] = (vk[k] ? R0 - bl * rows : 0) + rg;
      off[k] = (vk[k] ? R0 * cols : 0) + rg * cols + col;
    } else {
      const int R = k * pb.RG + rg;
      vk[k] = R < nrows;
      const int ob = b0 + (vk[k] ? R : 0);
      qlk[k] = ob / pb.bpq;
      jok[k] = 0;
      rk[k] = 0;
      off[k] = (vk[k] ? R : 0) * cols + col;
    }
  }
  T hv[RPT];
#pragma unroll
  for (int k = 0; k < RPT; ++k) hv[k] = at_u32(Xe, off[k]);
  T pw[RPT];
  if (PERTURB) {
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
      const int ql = qlk[k];
      double ps[MM];
      ps[sa] = p_col;
      if (NB == 2) ps[sb] = tb.pg[sb * kTab + rk[k]];
      if (MM == 3) ps[0] = tb.pg[0 * kTab + jok[k]];
      double c = 0.0;
#pragma unroll
      for (int s = 0; s < MM; ++s) c += grad[s * Q + ql] * g.bm[s] * ps[s];
      const T h = hv[k];
      pw[k] = -T(c) * h;
      const int li = (rg + k * pb.RG) * cp + col;
      Ga[li] = T(grad[sa * Q + ql]) * h;
      if (NB == 2) Gb[li] = T(grad[sb * Q + ql]) * h;
    }
  } else {
    T hu[MM][RPT], hd[MM][RPT];
#pragma unroll
    for (int s = 0; s < MM; ++s)
#pragma unroll
      for (int k = 0; k < RPT; ++k) {
        hu[s][k] = at_u32(Xu[s], off[k]);
        hd[s][k] = at_u32(Xd[s], off[k]);
      }
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
      const int ql = qlk[k];
      double ps[MM];
      ps[sa] = p_col;
      if (NB == 2) ps[sb] = tb.pg[sb * kTab + rk[k]];
      if (MM == 3) ps[0] = tb.pg[0 * kTab + jok[k]];
      const T h = hv[k];
      T acc = -T(dmp) * h;
      const int li = (rg + k * pb.RG) * cp + col;
#pragma unroll
      for (int s = 0; s < MM; ++s) {
        const double vp = tb.VpQ[s * Q + ql];
        const T u = T(fu[s]) * hu[s][k];
        acc += T(vp * ps[s] * tcv[s]) * hd[s][k] - T(vp * ps[s] * g.bm[s]) * u;
        if (s == sa || (NB == 2 && s == sb)) {
          const T G = T(tb.F[s * Q + ql]) * h + T(vp) * (u + T(cc[s]) * hd[s][k]);
          if (s == sa)
            Ga[li] = G;
          else
            Gb[li] = G;
        }
      }
      pw[k] = acc;
    }
  }
  // keep the pointwise terms computed here: sunk past the barriers, their
  // inputs would stay live (in registers) through the line solves
#pragma unroll
  for (int k = 0; k < RPT; ++k) asm volatile("" : "+v"(pw[k]));
  __syncthreads();

  // ---- phase 2: rows of Ga and columns of Gb ------------------------------------
  const int nla = nrows;
  const int nlb = NB == 2 ? nbt * cols : 0;
  if (pb.split && cols == NMAX && (NB == 1 || rows == NMAX)) {
    // two lanes per line; the pair (2l, 2l+1) is in one wave
    const T ca_a = T(g.dp_ca[sa]), cb_a = T(g.dp_cb[sa]);
    const T ca_b = T(g.dp_ca[NB == 2 ? sb : sa]), cb_b = T(g.dp_cb[NB == 2 ? sb : sa]);
    for (int hl = tid; hl < 2 * (nla + nlb); hl += blockDim.x) {
      const int l = hl >> 1;
      const bool is_row = l < nla;
      const int lb = l - nla;
      const int blk = lb / NMAX;
      const int base = is_row ? l * cp : blk * NMAX * cp + (lb - blk * NMAX);
      const double *ct = CLOS ? tb.clos + (MM + (is_row ? sa : (NB == 2 ? sb : sa))) * 2 * kClosRows * kTab : nullptr;
      compact_split<T, NMAX, CLOS>(is_row ? Ga : Gb, base, is_row ? 1 : cp, hl & 1, is_row ? ca_a : ca_b,
                                   is_row ? cb_a : cb_b, ct);
    }
  } else {
    for (int l = tid; l < nla + nlb; l += blockDim.x) {
      T *G;
      int base, stride, N;
      T ca, cb;
      const double *ct = nullptr;
      if (l < nla) {
        G = Ga;
        base = l * cp;
        stride = 1;
        N = cols;
        ca = T(g.dp_ca[sa]);
        cb = T(g.dp_cb[sa]);
        if (CLOS) ct = tb.clos + (MM + sa) * 2 * kClosRows * kTab;
      } else {
        const int lb = l - nla;
        const int blk = lb / cols;
        const int c = lb - blk * cols;
        G = Gb;
        base = blk * rows * cp + c;
        stride = cp;
        N = rows;
        ca = T(g.dp_ca[NB == 2 ? sb : sa]);
        cb = T(g.dp_cb[NB == 2 ? sb : sa]);
        if (CLOS) ct = tb.clos + (MM + (NB == 2 ? sb : sa)) * 2 * kClosRows * kTab;
      }
      compact_lds<T, CLOS>(G, base, stride, N, ca, cb, ct);
    }
  }
  __syncthreads();

  // ---- phase 3 ----------------------------------------------------------------
#pragma unroll
  for (int k = 0; k < RPT; ++k) {
    const int li = (rg + k * pb.RG) * cp + col;
    T v = pw[k] + Ga[li];
    if (NB == 2) v += Gb[li];
    if (owner && vk[k]) at_u32(Oe, off[k]) = TO(v);
  }
}

// ---------------------------------------------------------------------------
// k_pcube (three modes)
// ---------------------------------------------------------------------------
// A task is one (branch, element n, q point).  Its p block, N1 x N2 x N3
// values with p_1 outermost, is contiguous and holds every p line of the
// element at that q.  F_s(q), V_s'(q) and dX/dq_s(q) are constants of the
// task, so the three p-derivative fields
//   G_{n,s} = F_s h_n + V_s' (h_{n+e_s} + n_s (m_s zeta_s gamma_s/beta) h_{n-e_s})
// and the pointwise terms (as in k_pblock) are formed as the values arrive,
// and one launch covers D_{p_1}, D_{p_2} and D_{p_3} of every element: the
// q passes that follow read only h_n itself.
// Thread (j2, j3) of the (p_2, p_3) plane owns the p_1 line through it.
//   Phase A streams h_n and its two p_1 neighbours over every plane with no
//   barrier: the p_1 field and the p_1 and damping terms go to registers
//   (acc, g1), h_n to an LDS copy of the block; the p_1 lines are then
//   solved in registers and added to acc.
//   Phase B takes the planes in rounds of PL: h_n from the thread's own LDS
//   copy and the p_2, p_3 neighbours from memory (loads of round r + 1 are
//   issued before round r's LDS work) give the p_2, p_3 terms and fields;
//   the fields are solved along p_2 and p_3 in LDS planes (two lanes per
//   line when SPLIT: all three axes have NB1 points) and added to acc.
// Every neighbour read is skipped for a neighbour the task's element lacks.
// PERTURB: out = X^x h as in k_pblock, with fields dX/dq_s h_n.
struct PCube {
  int N1, N2, N3;  // p-axis lengths
  int plane;       // N2 * N3: threads that own a p_1 line
  int rs;          // LDS row stride of a plane field: N3 plus a pad
  int ntasks, nblk;
  int chunk;       // k_hcube: tasks per XCD chunk (0: one contiguous range per XCD)
  int ktile;       // k_hcube, three modes: width of the k_2 tiles of the task order
};

// Largest workgroup of k_pcube for a p_1 bucket: acc and g1 take
// 2 NB1 values per thread in phase A, acc and two rounds of loads in
// phase B, and every wave of the workgroup must fit the register file
// together (512 VGPRs per SIMD lane).
template <typename T, int NB1>
constexpr int pcube_max_threads() {
  return NB1 > 32 ? 256 : sizeof(T) == 8 ? (NB1 == 24 ? 768 : 512) : (NB1 >= 32 ? 768 : 1024);
}

// (p_2, p_3) planes per LDS round of k_pcube (the block copy takes the
// rest of the LDS).  Two modes use the same kernel with a unit third axis:
// the "planes" are p_2 rows and the p_3 fields vanish (zero tables).
constexpr int pcube_planes(const int nb1) { return nb1 >= 32 ? 2 : nb1 == 24 ? 4 : nb1 / 4; }

template <typename T, typename TO, int NB1, bool SPLIT, bool PERTURB, bool CLOS = false>
__global__ void __launch_bounds__((pcube_max_threads<T, NB1>()))
k_pcube(const Geom g, const Tabs tb, const PCube pc, const T *__restrict__ X, TO *__restrict__ out,
        const double *__restrict__ grad) {
  constexpr int PL = pcube_planes(NB1);     // planes per round
  constexpr int NR = (NB1 + PL - 1) / PL;  // rounds
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int task = xcd_task(blockIdx.x, pc.nblk);
  if (task >= pc.ntasks) return;
  // Cubic blocks solved by lane pairs (N1 = N2 = N3 = NB1) schedule their
  // loads explicitly: no load sits under a branch inside a loop (a load
  // under a branch is waited for at the branch's join, which serialised the
  // planes' loads).  Phase A and the final stores have one loop per
  // combination of p_1 neighbours the element has; phase B reads every
  // p_2, p_3 neighbour slot (an absent neighbour points at h_n itself and
  // enters with zero factors).
  constexpr bool FULL = SPLIT;
  const int N1 = pc.N1, N2 = pc.N2, N3 = pc.N3;
  const int plane = pc.plane;
  const int rs = pc.rs;                       // LDS row stride (p_3 row plus a pad)
  T *H = reinterpret_cast<T *>(smem_raw);     // [N1][plane] copy of h_n
  T *G2 = H + N1 * plane;                     // [PL][N2][rs]
  T *G3 = G2 + PL * N2 * rs;
  const int ne_all = g.ne * g.nbatch;
  const int ea = task % ne_all;  // (branch, element): elements of one q point are adjacent tasks
  const int ql = task / ne_all;
  const int br = ea / g.ne;
  const int e = ea - br * g.ne;
  const int tid = threadIdx.x;
  const bool own = tid < plane;
  const int j2 = own ? tid / N3 : 0;
  const int j3 = own ? tid - j2 * N3 : 0;
  const int Q = g.Q;

  const long long blk = (long long)ql * g.P;
  const T *Xe = X + (long long)ea * g.E + blk;
  TO *Oe = out + (long long)ea * g.E + blk;
  const T *Xb = X + (long long)br * g.ne * g.E;
  const T *Xu[3];
  const T *Xd[3];
  bool hu_[3], hd_[3];  // the element has n + e_s, n - e_s (uniform)
  T Fv[3], vu[3], vd[3], pwu[3], pwd[3];
  const double p2 = tb.pg[1 * kTab + j2], p3 = tb.pg[2 * kTab + j3];
#pragma unroll
  for (int s = 0; s < 3; ++s) {
    const int up = PERTURB ? -1 : tb.up[e * 3 + s];
    const int dn = PERTURB ? -1 : tb.dn[e * 3 + s];
    hu_[s] = up >= 0;
    hd_[s] = dn >= 0;
    Xu[s] = up >= 0 ? Xb + (long long)up * g.E + blk : Xe;
    Xd[s] = dn >= 0 ? Xb + (long long)dn * g.E + blk : Xe;
    if (PERTURB) {
      Fv[s] = T(grad[s * Q + ql]);
      vu[s] = vd[s] = pwu[s] = pwd[s] = T(0);
    } else {
      const double vp = tb.VpQ[s * Q + ql];
      Fv[s] = T(tb.F[s * Q + ql]);
      vu[s] = up >= 0 ? T(vp) : T(0);
      vd[s] = T(vp * tb.cc[e * 3 + s]);         // zero when n_s = 0
      pwd[s] = T(vp * 0.5 * tb.tc[e * 3 + s]);  // times p_s
      pwu[s] = up >= 0 ? T(vp * g.bm[s]) : T(0);
    }
  }
  // pointwise coefficient of h_n: -sum_s n_s gamma_s, or for PERTURB
  // -sum_s dX/dq_s beta p_s / 2 m_s (the p_1 part is added per plane)
  const T dmp = PERTURB ? T(0) : T(tb.damp[e]);
  const T c23 = PERTURB ? T(double(Fv[1]) * g.bm[1] * p2 + double(Fv[2]) * g.bm[2] * p3) : T(0);
  const T c1 = PERTURB ? T(double(Fv[0]) * g.bm[0]) : T(0);
  const T q2u = T(p2) * pwu[1], q2d = T(p2) * pwd[1], q3u = T(p3) * pwu[2], q3d = T(p3) * pwd[2];
  const uint32_t own_off = (uint32_t)(own ? tid : 0);

  // ---- phase A: h_n and its p_1 neighbours over every plane
  T acc[NB1], g1[NB1];
  // pointwise terms of h_n that involve p_1:
  // n_1 zeta_1 gamma_1 V_1' p_1/2 h_{n-e_1} - V_1' beta p_1/(2 m_1) h_{n+e_1} - sum n gamma h_n
  // (for PERTURB: -sum_s dX/dq_s beta p_s / 2 m_s h_n)
  auto point_a = [&](const T h, const T hu, const T hd, const T p1) {
    return PERTURB ? -(c23 + c1 * p1) * h : -dmp * h + p1 * (pwd[0] * hd - pwu[0] * hu);
  };
  auto plane_a = [&](const int i, const T h, const T hu, const T hd, const T p1) {
    if (!FULL) acc[i] = point_a(h, hu, hd, p1);
    g1[i] = PERTURB ? Fv[0] * h : Fv[0] * h + vu[0] * hu + vd[0] * hd;
    if (own) H[i * plane + tid] = h;
  };
  // FULL: p_1 values from an LDS copy of their table (a vector load of a
  // table value issued after the next group's loads would wait for all of
  // them), and load groups of GA planes whose offsets pass through an empty
  // asm statement: that keeps each group's loads after the previous
  // group's LDS stores (loads of read-only memory could otherwise all be
  // hoisted to the top, which exhausts the registers)
  T *P1t = G3 + PL * N2 * rs;
  constexpr int GA = 4;
  // RU, RD (std::bool_constant): read the p_1 neighbour above / below
  auto load_g = [&](const int i0, T (&h)[GA], T (&u)[GA], T (&d)[GA], T (&pp)[GA], const bool with_h, auto RU,
                    auto RD) {
    uint32_t b = own_off;
    asm volatile("" : "+v"(b));
#pragma unroll
    for (int k = 0; k < GA; ++k) {
      const uint32_t o = (uint32_t)((i0 + k) * plane) + b;
      pp[k] = P1t[i0 + k];
      h[k] = with_h ? at_u32(Xe, o) : H[(i0 + k) * plane + tid];
      u[k] = (PERTURB || !decltype(RU)::value) ? T(0) : at_u32(Xu[0], o);
      d[k] = (PERTURB || !decltype(RD)::value) ? T(0) : at_u32(Xd[0], o);
    }
  };
  const std::true_type yes{};
  const std::false_type no{};
  if constexpr (FULL) {
    // only the p_1 field is kept through phase A (the pointwise terms are
    // added at the end, from the LDS copy of h_n and a second read of the
    // p_1 neighbours), so two groups of loads fit in flight
    if (tid < N1) P1t[tid] = T(tb.pg[0 * kTab + tid]);
    __syncthreads();
    // one loop per combination of p_1 neighbours the element has (one
    // uniform branch around the loop), so that only those are read
    auto sweep_a = [&](auto RU, auto RD) {
      T ch[GA], cu[GA], cd[GA], cp[GA];
      load_g(0, ch, cu, cd, cp, true, RU, RD);
#pragma unroll
      for (int i0 = 0; i0 < NB1; i0 += GA) {
        T nh[GA], nu[GA], nd[GA], np[GA];
        if (i0 + GA < NB1) load_g(i0 + GA, nh, nu, nd, np, true, RU, RD);
#pragma unroll
        for (int k = 0; k < GA; ++k) plane_a(i0 + k, ch[k], cu[k], cd[k], cp[k]);
        if (i0 + GA < NB1) {
#pragma unroll
          for (int k = 0; k < GA; ++k) {
            ch[k] = nh[k];
            cu[k] = nu[k];
            cd[k] = nd[k];
            cp[k] = np[k];
          }
        }
      }
    };
    if (PERTURB || (!hu_[0] && !hd_[0]))
      sweep_a(no, no);
    else if (!hd_[0])
      sweep_a(yes, no);
    else if (!hu_[0])
      sweep_a(no, yes);
    else
      sweep_a(yes, yes);
  } else {
#pragma unroll
    for (int i = 0; i < NB1; ++i) {
      acc[i] = T(0);
      g1[i] = T(0);
      if (i < N1) {
        const uint32_t o = (uint32_t)(i * plane) + own_off;
        const T h = at_u32(Xe, o);
        const T hu = (!PERTURB && hu_[0]) ? at_u32(Xu[0], o) : T(0);
        const T hd = (!PERTURB && hd_[0]) ? at_u32(Xd[0], o) : T(0);
        plane_a(i, h, hu, hd, T(tb.pg[0 * kTab + i]));
      }
    }
  }
  compact_inplace<T, NB1, CLOS>(g1, N1, T(g.dp_ca[0]), T(g.dp_cb[0]),
                                CLOS ? tb.clos + g.M * 2 * kClosRows * kTab : nullptr);
#pragma unroll
  for (int i = 0; i < NB1; ++i) acc[i] = FULL ? g1[i] : acc[i] + g1[i];

  // ---- phase B: the p_2 and p_3 terms in rounds of PL planes
  const double *ct2 = CLOS ? tb.clos + (g.M + 1) * 2 * kClosRows * kTab : nullptr;
  const double *ct3 = CLOS ? tb.clos + (g.M + 2) * 2 * kClosRows * kTab : nullptr;
  // round loads: the p_2 and p_3 neighbours of PL planes (planes past the
  // block re-read its last plane: in bounds, unused)
  // FULL: UP, D2, D3 (std::bool_constant) say which neighbours are read;
  // the others are zero, as are their factors (a missing neighbour read
  // anyway is the element itself, with zero factors).  Otherwise the
  // element's own flags decide, at run time.
  auto load_round = [&](const int r, T (&u2)[PL], T (&d2)[PL], T (&u3)[PL], T (&d3)[PL], auto UP, auto D2,
                        auto D3) {
    constexpr bool up = decltype(UP)::value, dn2 = decltype(D2)::value, dn3 = decltype(D3)::value;
    uint32_t b = own_off;
    if constexpr (FULL) asm volatile("" : "+v"(b));  // these loads stay in their round
#pragma unroll
    for (int k = 0; k < PL; ++k) {
      const uint32_t o = (uint32_t)(min(r * PL + k, N1 - 1) * plane) + b;
      u2[k] = (!PERTURB && (FULL ? up : hu_[1])) ? at_u32(Xu[1], o) : T(0);
      d2[k] = (!PERTURB && (FULL ? dn2 : hd_[1])) ? at_u32(Xd[1], o) : T(0);
      u3[k] = (!PERTURB && (FULL ? up : hu_[2])) ? at_u32(Xu[2], o) : T(0);
      d3[k] = (!PERTURB && (FULL ? dn3 : hd_[2])) ? at_u32(Xd[2], o) : T(0);
    }
  };
  auto phase_b = [&](auto UP, auto D2, auto D3) {
    T cu2[PL], cd2[PL], cu3[PL], cd3[PL];
    load_round(0, cu2, cd2, cu3, cd3, UP, D2, D3);
  #pragma unroll
    for (int r = 0; r < NR; ++r) {
      const int i0 = r * PL;
      if (i0 >= N1) break;  // uniform
      T xu2[PL], xd2[PL], xu3[PL], xd3[PL];  // next round, in flight during this one
      if (r + 1 < NR) load_round(r + 1, xu2, xd2, xu3, xd3, UP, D2, D3);
  #pragma unroll
      for (int k = 0; k < PL; ++k) {
        const int i = i0 + k;
        if (i < N1 && own) {
          const T h = H[i * plane + tid];
          acc[i] += q2d * cd2[k] - q2u * cu2[k] + q3d * cd3[k] - q3u * cu3[k];
          const int li = (k * N2 + j2) * rs + j3;
          G2[li] = Fv[1] * h + vu[1] * cu2[k] + vd[1] * cd2[k];
          G3[li] = Fv[2] * h + vu[2] * cu3[k] + vd[2] * cd3[k];
        }
      }
      __syncthreads();
      // p_2 lines of G2 (fixed k, j3) and p_3 lines of G3 (fixed k, j2)
      const int npl = min(PL, N1 - i0);
      const int nl2 = npl * N3, nl = nl2 + npl * N2;
      if (SPLIT) {
        for (int hl = tid; hl < 2 * nl; hl += blockDim.x) {
          const int l = hl >> 1;
          if (l < nl2) {
            const int k = l / N3, c = l - k * N3;
            compact_split_regs<T, NB1, CLOS>(G2, k * N2 * rs + c, rs, hl & 1, T(g.dp_ca[1]), T(g.dp_cb[1]), ct2);
          } else {
            const int l3 = l - nl2;
            compact_split_regs<T, NB1, CLOS>(G3, l3 * rs, 1, hl & 1, T(g.dp_ca[2]), T(g.dp_cb[2]), ct3);
          }
        }
      } else {
        for (int l = tid; l < nl; l += blockDim.x) {
          if (l < nl2) {
            const int k = l / N3, c = l - k * N3;
            compact_lds<T, CLOS>(G2, k * N2 * rs + c, rs, N2, T(g.dp_ca[1]), T(g.dp_cb[1]), ct2);
          } else {
            compact_lds<T, CLOS>(G3, (l - nl2) * rs, 1, N3, T(g.dp_ca[2]), T(g.dp_cb[2]), ct3);
          }
        }
      }
      __syncthreads();
  #pragma unroll
      for (int k = 0; k < PL; ++k) {
        const int i = i0 + k;
        if (i < N1 && own) {
          const int li = (k * N2 + j2) * rs + j3;
          acc[i] += G2[li] + G3[li];
        }
      }
      __syncthreads();  // the next round overwrites the planes
      if (r + 1 < NR) {
  #pragma unroll
        for (int k = 0; k < PL; ++k) {
          cu2[k] = xu2[k];
          cd2[k] = xd2[k];
          cu3[k] = xu3[k];
          cd3[k] = xd3[k];
        }
      }
    }
  };
  // FULL: every neighbour is read (copies of phase B per combination of
  // neighbours, as phase A has, spill registers and were slower)
  phase_b(yes, yes, yes);
  if (!own) return;
  if constexpr (FULL) {
    // the pointwise terms of phase A, then the stores, in load groups; the
    // second read covers only the neighbours the element has (one uniform
    // branch around the whole loop, none inside it)
    auto finish = [&](auto RU, auto RD) {
      T ch[GA], cu[GA], cd[GA], cp[GA];
      load_g(0, ch, cu, cd, cp, false, RU, RD);
#pragma unroll
      for (int i0 = 0; i0 < NB1; i0 += GA) {
        T nh[GA], nu[GA], nd[GA], np[GA];
        if (i0 + GA < NB1) load_g(i0 + GA, nh, nu, nd, np, false, RU, RD);
#pragma unroll
        for (int k = 0; k < GA; ++k)
          at_u32(Oe, (uint32_t)((i0 + k) * plane + tid)) = TO(acc[i0 + k] + point_a(ch[k], cu[k], cd[k], cp[k]));
        if (i0 + GA < NB1) {
#pragma unroll
          for (int k = 0; k < GA; ++k) {
            ch[k] = nh[k];
            cu[k] = nu[k];
            cd[k] = nd[k];
            cp[k] = np[k];
          }
        }
      }
    };
    if (PERTURB || (!hu_[0] && !hd_[0]))
      finish(no, no);
    else if (!hd_[0])
      finish(yes, no);
    else if (!hu_[0])
      finish(no, yes);
    else
      finish(yes, yes);
  } else {
#pragma unroll
    for (int i = 0; i < NB1; ++i)
      if (i < N1) at_u32(Oe, (uint32_t)(i * plane + tid)) = TO(acc[i]);
  }
}

// ---------------------------------------------------------------------------
// k_pcube_s: k_pcube in one streamed sweep over the planes
// ---------------------------------------------------------------------------
// Same task, thread map and result as k_pcube.  Along a p_1 line, with s_i
// the pointwise, p_2 and p_3 terms of plane i and G_1 the p_1 field, the
// right-hand side is
//   t = s + A^{-1} B G_1 = A^{-1} (A s + B G_1),
// A = tridiag(1/3, 1, 1/3), B the explicit stencil.  Plane i, once its p_2
// and p_3 lines are solved, adds s_i and G_{1,i} to the rows r_{i-R}..r_{i+R}
// of A t = r that they touch (R = stencil reach), and row i - R, now
// complete, takes its forward Thomas step.  Every value is read once (no copy
// of the block), so the LDS holds only a round's two planes and the first ND
// forward results d_j of every line (the rest stay in registers); the back
// substitution then writes t.  At 24^3 in FP64 that is 78 KB of LDS and
// 96 VGPRs: two workgroups per CU, where k_pcube's block copy allows one.
// Plain stencils only (a closure keeps k_pcube).

// Task constants of k_pcube_s in LDS: slots of the groups below (three
// modes each) and the damping, then the p_2 and p_3 grids.
constexpr int kCfF = 0, kCfVu = 3, kCfVd = 6, kCfPu = 9, kCfPd = 12, kCfBm = 15, kCfDamp = 18;
constexpr int kCfP2 = 20, kCfP3 = kCfP2 + kTab;
constexpr int kPCubeCF = kCfP3 + kTab;
constexpr int pcube_s_planes(const int nb1) { return nb1 >= 24 ? 2 : nb1 / 4; }
constexpr int pcube_s_dlds(const int tsize, const int nb1) { return tsize == 8 && nb1 >= 24 ? nb1 / 2 + 1 : 0; }
// Waves per SIMD the register budget aims at: five for the cubic FP64 24^3
// block (two workgroups of nine waves per CU).
template <typename T, int NB1, bool SPLIT>
constexpr int pcube_s_waves() {
  return sizeof(T) == 8 && NB1 == 24 && SPLIT ? 5 : 4;
}

template <typename T, typename TO, int NB1, bool SPLIT, bool PERTURB>
__global__ void __launch_bounds__((pcube_max_threads<T, NB1>()), (pcube_s_waves<T, NB1, SPLIT>()))
k_pcube_s(const Geom g, const Tabs tb, const PCube pc, const T *__restrict__ X, TO *__restrict__ out,
          const double *__restrict__ grad) {
  constexpr int PL = pcube_s_planes(NB1);          // planes per round
  constexpr int NR = (NB1 + PL - 1) / PL;          // rounds
  constexpr int ND = pcube_s_dlds(sizeof(T), NB1);  // forward results kept in LDS
  constexpr int RC = 2;                            // stencil reach along p_1
  constexpr T third = T(1.0 / 3.0);
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int task = xcd_task(blockIdx.x, pc.nblk);
  if (task >= pc.ntasks) return;
  // SPLIT blocks are cubes of NB1 points: their loops have fixed trip counts
  const int N1 = SPLIT ? NB1 : pc.N1, N2 = SPLIT ? NB1 : pc.N2, N3 = SPLIT ? NB1 : pc.N3;
  const int plane = SPLIT ? NB1 * NB1 : pc.plane;
  const int rs = SPLIT ? NB1 + 1 : pc.rs;  // LDS row stride (p_3 row plus a pad)
  T *CF = reinterpret_cast<T *>(smem_raw);  // task constants, kPCubeCF values
  T *G2 = CF + kPCubeCF;                    // [PL][N2][rs]
  T *G3 = G2 + PL * N2 * rs;
  T *Dl = G3 + PL * N2 * rs;                // [ND][plane]
  const int ne_all = g.ne * g.nbatch;
  const int ea = task % ne_all;  // (branch, element): elements of one q point are adjacent tasks
  const int ql = task / ne_all;
  const int br = ea / g.ne;
  const int e = ea - br * g.ne;
  const int tid = threadIdx.x;
  const bool own = tid < plane;
  const int j2 = own ? tid / N3 : 0;
  const int j3 = own ? tid - j2 * N3 : 0;
  const int Q = g.Q;

  const long long blk = (long long)ql * g.P;
  const T *Xe = X + (long long)ea * g.E + blk;
  TO *Oe = out + (long long)ea * g.E + blk;
  const T *Xb = X + (long long)br * g.ne * g.E;
  // A missing neighbour points at the element itself and has zero factors,
  // so the neighbour loads are unconditional (no per-neighbour branch or
  // mask; the repeated address is served by the cache).
  const T *Xu[3];
  const T *Xd[3];
#pragma unroll
  for (int s = 0; s < 3; ++s) {
    const int up = PERTURB ? -1 : tb.up[e * 3 + s];
    const int dn = PERTURB ? -1 : tb.dn[e * 3 + s];
    Xu[s] = up >= 0 ? Xb + (long long)up * g.E + blk : Xe;
    Xd[s] = dn >= 0 ? Xb + (long long)dn * g.E + blk : Xe;
  }
  // The task's constants go to LDS once and are read where they are used
  // in every round, so that neither scalar nor vector registers hold them
  // through the line solves: per mode s (slot s of each group of three)
  // F_s (or dX/dq_s), V_s' for n + e_s and n - e_s, and the p_s-weighted
  // pointwise factors; then the damping and, for PERTURB, beta/2m_s dX/dq_s.
  if (tid < 3) {
    const int s = tid;
    const int up = PERTURB ? -1 : tb.up[e * 3 + s];
    if (PERTURB) {
      const double gr = grad[s * Q + ql];
      CF[kCfF + s] = T(gr);
      CF[kCfVu + s] = CF[kCfVd + s] = CF[kCfPu + s] = CF[kCfPd + s] = T(0);
      CF[kCfBm + s] = T(gr * g.bm[s]);
    } else {
      const double vp = tb.VpQ[s * Q + ql];
      CF[kCfF + s] = T(tb.F[s * Q + ql]);
      CF[kCfVu + s] = up >= 0 ? T(vp) : T(0);
      CF[kCfVd + s] = T(vp * tb.cc[e * 3 + s]);         // zero when n_s = 0
      CF[kCfPd + s] = T(vp * 0.5 * tb.tc[e * 3 + s]);  // times p_s
      CF[kCfPu + s] = up >= 0 ? T(vp * g.bm[s]) : T(0);
      CF[kCfBm + s] = T(0);
    }
    if (s == 0) CF[kCfDamp] = PERTURB ? T(0) : T(tb.damp[e]);
  }
  if (tid < N2) CF[kCfP2 + tid] = T(tb.pg[1 * kTab + tid]);
  if (tid < N3) CF[kCfP3 + tid] = T(tb.pg[2 * kTab + tid]);
  __syncthreads();
  const T ca1 = T(g.dp_ca[0]), cb1 = T(g.dp_cb[0]);
  const uint32_t own_off = (uint32_t)(own ? tid : 0);

  // ln[j]: row j of A t = r while it collects its terms, then its forward
  // result d_j (rows j < ND move to Dl once eliminated)
  T ln[NB1];
#pragma unroll
  for (int j = 0; j < NB1; ++j) ln[j] = T(0);
  T dprev = T(0);
  auto elim = [&](const int j) {
    const T d = j == 0 ? ln[j] : fma_t(T(-kThomas.inv[j] / 3.0), dprev, ln[j] * T(kThomas.inv[j]));
    dprev = d;
    if (j < ND) {
      if (own) Dl[j * plane + tid] = d;
    } else {
      ln[j] = d;
    }
  };

#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const int i0 = r * PL;
    if (i0 >= N1) break;  // uniform
    // h_n and its six neighbours on PL planes: pointwise terms and G_1 stay
    // in registers, G_2 and G_3 go to the LDS planes.  The thread's p_2, p_3
    // factors are formed again in every round from the LDS copies.
    const T p2 = CF[kCfP2 + j2], p3 = CF[kCfP3 + j3];
    T Fv[3], vu[3], vd[3];
#pragma unroll
    for (int s = 0; s < 3; ++s) {
      Fv[s] = CF[kCfF + s];
      vu[s] = CF[kCfVu + s];
      vd[s] = CF[kCfVd + s];
    }
    const T dmp = CF[kCfDamp], pwu1 = CF[kCfPu], pwd1 = CF[kCfPd];
    const T c1 = CF[kCfBm], c23 = CF[kCfBm + 1] * T(p2) + CF[kCfBm + 2] * T(p3);
    const T q2u = T(p2) * CF[kCfPu + 1], q2d = T(p2) * CF[kCfPd + 1];
    const T q3u = T(p3) * CF[kCfPu + 2], q3d = T(p3) * CF[kCfPd + 2];
    T sv[PL], gv[PL];
#pragma unroll
    for (int k = 0; k < PL; ++k) {
      const int i = i0 + k;
      sv[k] = gv[k] = T(0);
      if (i < N1) {
        // the offset is hidden from the optimiser so that every load takes
        // the scalar-base form (one 32-bit offset register) rather than a
        // 64-bit address per neighbour held through the kernel
        uint32_t o = (uint32_t)(i * plane) + own_off;
        asm volatile("" : "+v"(o));
        const T h = at_u32(Xe, o);
        const T p1 = T(tb.pg[0 * kTab + i]);
        T f2 = Fv[1] * h, f3 = Fv[2] * h;
        if (PERTURB) {
          sv[k] = -(c23 + c1 * p1) * h;
          gv[k] = Fv[0] * h;
        } else {
          const T u1 = at_u32(Xu[0], o), d1 = at_u32(Xd[0], o);
          const T u2 = at_u32(Xu[1], o), d2 = at_u32(Xd[1], o);
          const T u3 = at_u32(Xu[2], o), d3 = at_u32(Xd[2], o);
          sv[k] = -dmp * h + p1 * (pwd1 * d1 - pwu1 * u1) + q2d * d2 - q2u * u2 + q3d * d3 - q3u * u3;
          gv[k] = Fv[0] * h + vu[0] * u1 + vd[0] * d1;
          f2 += vu[1] * u2 + vd[1] * d2;
          f3 += vu[2] * u3 + vd[2] * d3;
        }
        if (own) {
          const int li = (k * N2 + j2) * rs + j3;
          G2[li] = f2;
          G3[li] = f3;
        }
      }
      // keep sv, gv computed here: sunk past the barrier, their seven
      // inputs per plane would stay live (in registers) through the solves
      asm volatile("" : "+v"(sv[k]), "+v"(gv[k]));
    }
    __syncthreads();
    // p_2 lines of G2 (fixed k, j3) and p_3 lines of G3 (fixed k, j2)
    const int npl = min(PL, N1 - i0);
    const int nl2 = npl * N3, nl = nl2 + npl * N2;
    if (SPLIT) {
#pragma unroll 1
      for (int hl = tid; hl < 2 * nl; hl += blockDim.x) {
        const int l = hl >> 1;
        if (l < nl2) {
          const int k = l / N3, c = l - k * N3;
          compact_split<T, NB1>(G2, k * N2 * rs + c, rs, hl & 1, T(g.dp_ca[1]), T(g.dp_cb[1]));
        } else {
          compact_split<T, NB1>(G3, (l - nl2) * rs, 1, hl & 1, T(g.dp_ca[2]), T(g.dp_cb[2]));
        }
      }
    } else {
#pragma unroll 1
      for (int l = tid; l < nl; l += blockDim.x) {
        if (l < nl2) {
          const int k = l / N3, c = l - k * N3;
          compact_lds<T>(G2, k * N2 * rs + c, rs, N2, T(g.dp_ca[1]), T(g.dp_cb[1]));
        } else {
          compact_lds<T>(G3, (l - nl2) * rs, 1, N3, T(g.dp_ca[2]), T(g.dp_cb[2]));
        }
      }
    }
    __syncthreads();
    // fold each plane into the p_1 rows it touches, oldest plane first
#pragma unroll
    for (int k = 0; k < PL; ++k) {
      const int i = i0 + k;
      if (i < N1) {
        const int li = (k * N2 + j2) * rs + j3;
        const T s = sv[k] + G2[li] + G3[li];
        const T gg = gv[k];
        ln[i] += s;  // A s
        if (i >= 1) ln[i >= 1 ? i - 1 : 0] += third * s;
        if (i + 1 < NB1) ln[i + 1 < NB1 ? i + 1 : 0] += third * s;
        // B G_1: row j takes ca (G_{j+1} - G_{j-1}) + cb (G_{j+2} - G_{j-2})
        if (i >= 1) ln[i >= 1 ? i - 1 : 0] += ca1 * gg;
        if (i >= 2) ln[i >= 2 ? i - 2 : 0] += cb1 * gg;
        if (i + 1 < NB1) ln[i + 1 < NB1 ? i + 1 : 0] -= ca1 * gg;
        if (i + 2 < NB1) ln[i + 2 < NB1 ? i + 2 : 0] -= cb1 * gg;
        if (i >= RC) elim(i >= RC ? i - RC : 0);  // row i - R has all its terms
        if (i == N1 - 1) {                        // last plane: the remaining rows
#pragma unroll
          for (int kk = RC - 1; kk >= 0; --kk)
            if (i - kk >= 0) elim(i - kk >= 0 ? i - kk : 0);
        }
      }
    }
    __syncthreads();  // the next round overwrites the planes
  }
  if (!own) return;
  // back substitution from the far end of the line, writing t
  T x = T(0);
#pragma unroll
  for (int j = NB1 - 1; j >= 0; --j) {
    if (j < N1) {
      const T d = j < ND ? Dl[j * plane + tid] : ln[j];
      x = d - T(kThomas.cp[j]) * x;
      uint32_t o = (uint32_t)(j * plane + tid);
      asm volatile("" : "+v"(o));
      at_u32(Oe, o) = TO(x);
    }
  }
}

// ---------------------------------------------------------------------------
// k_qpass
// ---------------------------------------------------------------------------
// Stage epilogues.  Eq. (eq:HEOM) is linear with a time-independent
// generator L, so one classical RK4 step is the degree-4 Taylor polynomial
//   y <- (1 + dt L + (dt L)^2/2 + (dt L)^3/6 + (dt L)^4/24) y,
// evaluated here in nested (Horner) form with four right-hand sides:
//   z1 = y + dt/4 L y,  z2 = y + dt/3 L z1,  z3 = y + dt/2 L z2,  y <- y + dt L z3.
// Each stage reads its input z and y and writes one state; no running sum
// of the stage slopes is kept.  c is the stage coefficient (dt/4 .. dt).
enum Epi : int {
  EPI_ACC = 0,  // Tacc += contribution
  EPI_OUT = 1,  // xo = Tacc + contribution               (one RHS evaluation)
  EPI_H1 = 2,   // xo = X + c k                           (first stage: X is y)
  EPI_H2 = 3,   // xo = y + c k                           (middle stages)
  EPI_H4 = 4    // xo = xo + c k                          (last stage: xo is y, in place)
};

// q-linear index and p index of a state position (within one element)
__device__ __forceinline__ void split_pos(const Geom &g, const int rel, int &ql, int &pix) {
  ql = rel / g.P;
  pix = rel - ql * g.P;
}

// value of the field of mode s at relative position rel of element e
// Xb: element 0 of the branch; e: element within the branch
template <typename T, int FIELD>
__device__ __forceinline__ T field_at(const Geom &g, const Tabs &tb, const T *__restrict__ Xb,
                                      const double *__restrict__ grad, const int e, const int s,
                                      const int rel, const T w) {
  if (FIELD == FQ) return w;
  int ql, pix;
  split_pos(g, rel, ql, pix);
  if (FIELD == FX) return T(grad[(long long)s * g.Q + ql]) * w;
  const int up = tb.up[e * 3 + s];
  const int dn = tb.dn[e * 3 + s];
  const double vp = tb.Vp[s * kTab + (ql / g.QS[s]) % g.Nq[s]];
  T Gv = T(tb.F[(long long)s * g.Q + ql]) * w;
  if (up >= 0) Gv += T(vp) * at_u32(Xb + (long long)up * g.E, rel);
  if (dn >= 0) Gv += T(vp * tb.cc[e * 3 + s]) * at_u32(Xb + (long long)dn * g.E, rel);
  return Gv;
}

// T: type of X and of the arithmetic; TO: type of Tacc, y, xo.
template <typename T, typename TO, int NMAX, bool TWO, int EPI, int FA, int FB, bool CLOS = false>
__global__ void __launch_bounds__(512)
k_qpass(const Geom g, const Tabs tb, const QPass qp, const T *__restrict__ X, TO *__restrict__ Tacc,
        const TO *__restrict__ y, TO *__restrict__ xo, const double *__restrict__ grad, const double cst) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T *lds = reinterpret_cast<T *>(smem_raw);
  const int task = xcd_task(blockIdx.x, qp.nblk);
  if (task >= qp.ntasks) return;
  // Task order.  A pass with a p-axis field (which reads hierarchy
  // neighbours) varies the element fastest: the tiles of all elements at one
  // position run close together on one XCD, so the neighbour reads hit its
  // L2.  Other passes walk each element's memory in order (DRAM locality).
  const int ne_all = g.ne * g.nbatch;
  int ea, chunk, rest;  // ea: (branch, element)
  if constexpr (FA == FP || FB == FP) {
    ea = task % ne_all;
    const int t2 = task / ne_all;
    chunk = t2 % qp.nchunk;
    rest = t2 / qp.nchunk;
  } else {
    chunk = task % qp.nchunk;
    const int t2 = task / qp.nchunk;
    rest = t2 % qp.nrest;
    ea = t2 / qp.nrest;
  }
  const int br = ea / g.ne;
  const int e = ea - br * g.ne;
  const int p0 = chunk * qp.pc;
  const int pcn = min(qp.pc, qp.run - p0);
  int rel = p0;
  {
    int r = rest;
    const int r2 = r % qp.rN[2];
    r /= qp.rN[2];
    const int r1 = r % qp.rN[1];
    const int r0 = r / qp.rN[1];
    rel += r0 * qp.rS[0] + r1 * qp.rS[1] + r2 * qp.rS[2];
  }
  const int tid = threadIdx.x;
  const int c = tid % qp.pc;
  const int jb = tid / qp.pc;
  const int Na = qp.Na;
  const bool active = (c < pcn) && (jb < (TWO ? qp.Nb : 1));
  const int lrel = rel + (TWO ? jb * qp.sb : 0) + c;  // line start within the element
  const long long ebase = (long long)ea * g.E;
  const T *Xb = X + (long long)br * g.ne * g.E;

  // element i of this thread's a-line: uniform pointer (element base plus
  // i strides) with the thread's 32-bit offset lrel
  T f[NMAX];
#pragma unroll
  for (int i = 0; i < NMAX; ++i)
    f[i] = (active && i < Na) ? at_u32(X + ebase + (long long)i * qp.sa, lrel) : T(0);

  // LDS tile [ja][jb][c] with row stride (Nb + 1) * pc: the pad keeps the
  // b-line reads of different ja in different banks
  const int rs = (qp.Nb + 1) * qp.pc;
  if (TWO) {
    const int Nb = qp.Nb, pc = qp.pc;
    if (active) {
#pragma unroll
      for (int i = 0; i < NMAX; ++i)
        if (i < Na) {
          lds[i * rs + jb * pc + c] =
              field_at<T, FB>(g, tb, Xb, grad, e, qp.sb_mode, lrel + i * qp.sa, f[i]);
        }
    }
    __syncthreads();
    const int ja = tid / pc;
    if (c < pcn && ja < Na) {
      T h[NMAX];
#pragma unroll
      for (int i = 0; i < NMAX; ++i) h[i] = (i < Nb) ? lds[ja * rs + i * pc + c] : T(0);
      compact_line<T, NMAX, CLOS>(h, Nb, T(qp.ca_b), T(qp.cb_b), CLOS ? tb.clos + qp.b * 2 * kClosRows * kTab : nullptr);
#pragma unroll
      for (int i = 0; i < NMAX; ++i)
        if (i < Nb) lds[ja * rs + i * pc + c] = h[i];
    }
    __syncthreads();
  }
  if (!active) return;  // no barrier below this point

  // field along a (a q axis: W itself; p axis: built from W and neighbours)
  T d[NMAX];
#pragma unroll
  for (int i = 0; i < NMAX; ++i) {
    if (FA == FQ)
      d[i] = f[i];
    else
      d[i] = (i < Na) ? field_at<T, FA>(g, tb, Xb, grad, e, qp.sa_mode, lrel + i * qp.sa, f[i]) : T(0);
  }
  compact_line<T, NMAX, CLOS>(d, Na, T(qp.ca_a), T(qp.cb_a), CLOS ? tb.clos + qp.a * 2 * kClosRows * kTab : nullptr);

  // coefficients: -p_s/m_s for q-type axes (p_s is fixed along the line)
  int ql0, pix0;
  split_pos(g, lrel, ql0, pix0);
  T ka = T(1), kb = T(1);
  if (FA == FQ) {
    const int s = qp.sa_mode;
    ka = T(-tb.pm[s * kTab + (pix0 / g.PS[s]) % g.Np[s]]);
  }
  if (TWO && FB == FQ) {
    const int s = qp.sb_mode;
    kb = T(-tb.pm[s * kTab + (pix0 / g.PS[s]) % g.Np[s]]);
  }
  const T cs = T(cst);
  if ((EPI == EPI_ACC || EPI == EPI_H1) && Na == NMAX) {
    // Full lines (one uniform branch): the epilogue's loads go in groups of
    // four points, issued one group ahead.  In the per-point form below each
    // point's load sits under an "i < Na" branch and is waited for before
    // the next point's load is issued.  Each group's offset passes through
    // an empty asm statement, which keeps its loads after the previous
    // group's stores.  (The stage-final passes that read y or xo as well run
    // at the device's streaming rate either way; grouped, they measured 1%
    // slower.)
    constexpr int GE = 4;  // NMAX is a multiple of 4
    T ct[GE], cy[GE];
    auto load_e = [&](const int i0, T (&tv)[GE], T (&yv)[GE]) {
      uint32_t b = (uint32_t)lrel;
      asm volatile("" : "+v"(b));
#pragma unroll
      for (int k = 0; k < GE; ++k) {
        const long long ui = ebase + (long long)(i0 + k) * qp.sa;
        tv[k] = T(at_u32(Tacc + ui, b));
        yv[k] = EPI == EPI_H2 ? T(at_u32(y + ui, b)) : EPI == EPI_H4 ? T(at_u32(xo + ui, b)) : T(0);
      }
    };
    load_e(0, ct, cy);
#pragma unroll
    for (int i0 = 0; i0 < NMAX; i0 += GE) {
      T nt[GE], ny[GE];
      if (i0 + GE < NMAX) load_e(i0 + GE, nt, ny);
#pragma unroll
      for (int k = 0; k < GE; ++k) {
        const int i = i0 + k;
        T kv = ka * d[i];
        if (TWO) kv += kb * lds[i * rs + jb * qp.pc + c];
        const long long ui = ebase + (long long)i * qp.sa;
        if (EPI == EPI_ACC) {
          at_u32(Tacc + ui, lrel) = TO(ct[k] + kv);
        } else {
          kv += ct[k];
          TO &xov = at_u32(xo + ui, lrel);
          if (EPI == EPI_OUT)
            xov = TO(kv);
          else if (EPI == EPI_H1)
            xov = TO(f[i] + cs * kv);
          else  // EPI_H2 (y) and EPI_H4 (xo itself)
            xov = TO(cy[k] + cs * kv);
        }
      }
      if (i0 + GE < NMAX) {
#pragma unroll
        for (int k = 0; k < GE; ++k) {
          ct[k] = nt[k];
          cy[k] = ny[k];
        }
      }
    }
    return;
  }
#pragma unroll
  for (int i = 0; i < NMAX; ++i) {
    if (i < Na) {
      T kv = ka * d[i];
      if (TWO) kv += kb * lds[i * rs + jb * qp.pc + c];
      const long long ui = ebase + (long long)i * qp.sa;  // uniform part of the index
      TO &tacc = at_u32(Tacc + ui, lrel);
      if (EPI == EPI_ACC) {
        tacc = TO(T(tacc) + kv);
      } else {
        kv += T(tacc);
        TO &xov = at_u32(xo + ui, lrel);
        if (EPI == EPI_OUT)
          xov = TO(kv);
        else if (EPI == EPI_H1)
          xov = TO(f[i] + cs * kv);
        else if (EPI == EPI_H2)
          xov = TO(T(at_u32(y + ui, lrel)) + cs * kv);
        else  // EPI_H4
          xov = TO(T(xov) + cs * kv);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// reductions and small kernels (FP64)
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// partial[branch][block] = sum over this block's share of element 0 of
// Cw[qlin] * wp[pidx] * W[qlin * P + pidx]   (fixed order for a fixed grid);
// blockIdx.y selects the branch, whose state starts at W + branch * bstride.
template <typename T>
__global__ void __launch_bounds__(256)
k_reduce_w0(const T *__restrict__ W, const double *__restrict__ Cw, const double *__restrict__ wp,
            const int Q, const int P, double *__restrict__ partial, const long long bstride) {
  __shared__ double sh[4];
  W += (long long)blockIdx.y * bstride;
  partial += (long long)blockIdx.y * gridDim.x;
  double s = 0.0;
  const int n = Q * P;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
    const int ql = i / P;
    const int pi = i - ql * P;
    s += Cw[ql] * wp[pi] * double(W[i]);
  }
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) partial[blockIdx.x] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

// out[b * ostride] = scale * sum(partial[b][0..n)), fixed order, one block per branch b.
__global__ void __launch_bounds__(256)
k_reduce_final(const double *__restrict__ partial, const int n, const double scale,
               double *__restrict__ out, const int ostride) {
  __shared__ double sh[4];
  partial += (long long)blockIdx.x * n;
  out += (long long)blockIdx.x * ostride;
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) s += partial[i];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) out[0] = scale * ((sh[0] + sh[1]) + (sh[2] + sh[3]));
}

// element 0: h_0 = exp(-beta H / 2) = sq[qlin] * sp[pidx] (unnormalised); other elements: 0
template <typename T>
__global__ void __launch_bounds__(256)
k_boltzmann(T *__restrict__ W, const double *__restrict__ sq, const double *__restrict__ sp,
            const int Q, const int P, const long long total) {
  const int n0 = Q * P;
  for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < total;
       i += (long long)gridDim.x * 256) {
    if (i < n0) {
      const int ii = (int)i;
      const int ql = ii / P;
      const int pi = ii - ql * P;
      W[i] = T(sq[ql] * sp[pi]);
    } else {
      W[i] = T(0);
    }
  }
}

// W <- W * sq[qlin] * sp[pidx] (mul != 0) or W / (sq * sp) (mul == 0), every element
template <typename T>
__global__ void __launch_bounds__(256)
k_sym_scale(T *__restrict__ W, const double *__restrict__ sq, const double *__restrict__ sp,
            const int Q, const int P, const long long total, const int mul) {
  const long long E = (long long)Q * P;
  for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < total;
       i += (long long)gridDim.x * 256) {
    const int ii = (int)(i % E);
    const int ql = ii / P;
    const int pi = ii - ql * P;
    const double f = sq[ql] * sp[pi];
    W[i] = mul ? T(double(W[i]) * f) : T(double(W[i]) / f);
  }
}

// W[0 .. n0) *= 1 / (dV * sum), sum read from device memory
template <typename T>
__global__ void __launch_bounds__(256)
k_normalise(T *__restrict__ W, const double *__restrict__ sum, const double dV, const int n0) {
  const double inv = 1.0 / (dV * sum[0]);
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n0; i += gridDim.x * 256)
    W[i] = T(double(W[i]) * inv);
}

// flag[0] = 1 if any value is not finite
template <typename T>
__global__ void __launch_bounds__(256)
k_check_finite(const T *__restrict__ W, const long long n, int *__restrict__ flag) {
  int bad = 0;
  for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n;
       i += (long long)gridDim.x * 256) {
    const double v = double(W[i]);
    bad |= !(v - v == 0.0);
  }
  if (bad) flag[0] = 1;  // benign race: every writer stores 1
}

// Discrete Fourier sums of the spectra, Eqs. (1DIR_Raman) and (2DThz_Raman),
// rectangle rule with weight 1 at t = 0.  Twiddles exp(sign 2 pi i k j / n)
// use the exact reduction (k j mod n) / n before sincospi.
//   out[row][k] = sum_j exp(sign 2 pi i k j / n) in[row][j]   (complex in/out)
__global__ void __launch_bounds__(256)
k_dft_rows(const double2 *__restrict__ in, double2 *__restrict__ out, const int rows, const int n,
           const int in_stride, const int in_step, const int out_stride, const int out_step,
           const double sign) {
  const long long id = (long long)blockIdx.x * 256 + threadIdx.x;
  if (id >= (long long)rows * n) return;
  const int row = (int)(id / n);
  const int k = (int)(id - (long long)row * n);
  double re = 0.0, im = 0.0;
  for (int j = 0; j < n; ++j) {
    const long long kj = ((long long)k * j) % n;
    double sv, cv;
    sincospi(2.0 * (double)kj / (double)n, &sv, &cv);
    sv *= sign;
    const double2 v = in[(long long)row * in_stride + (long long)j * in_step];
    re += v.x * cv - v.y * sv;
    im += v.x * sv + v.y * cv;
  }
  out[(long long)row * out_stride + (long long)k * out_step] = make_double2(re, im);
}

// real input -> complex (imaginary part 0)
__global__ void __launch_bounds__(256)
k_to_complex(const double *__restrict__ in, double2 *__restrict__ out, const long long n) {
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i < n) out[i] = make_double2(in[i], 0.0);
}

// I = scale * omega_k * Im(z)  (omega == nullptr: omega_k = 1)
__global__ void __launch_bounds__(256)
k_spectrum_out(const double2 *__restrict__ z, const long long n, const int n_fast, const double scale,
               const double dw, const int with_omega, double *__restrict__ I) {
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const double w = with_omega ? dw * (double)(i % n_fast) : 1.0;
  I[i] = scale * w * z[i].y;
}

// R[j2 * n_t1 + j0 + b] = Rw[j2 * B + b] for b < nb
__global__ void __launch_bounds__(256)
k_scatter_r(const double *__restrict__ Rw, double *__restrict__ R, const int n_t2, const int B, const int nb,
            const int n_t1, const int j0) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n_t2 * nb) return;
  const int j2 = i / nb;
  const int b = i - j2 * nb;
  R[(long long)j2 * n_t1 + j0 + b] = Rw[(long long)j2 * B + b];
}

// Bandwidth references.  k_stream_copy: dst = src in 16-byte vectors;
// k_stream_mix<NS>: dst = the sum of NS sources (pairs of doubles; NS = 0
// writes zeros), the read/write mixes of the streaming passes.  Each thread
// keeps eight vectors per source in flight before it stores, in a
// grid-stride loop over many workgroups per CU.
constexpr int kStreamU = 8;
__global__ void __launch_bounds__(256)
k_stream_copy(uint4 *__restrict__ dst, const uint4 *__restrict__ src, const long long n16) {
  const long long st = (long long)gridDim.x * 256;
  long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  for (; i + (kStreamU - 1) * st < n16; i += kStreamU * st) {
    uint4 v[kStreamU];
#pragma unroll
    for (int u = 0; u < kStreamU; ++u) v[u] = src[i + u * st];
#pragma unroll
    for (int u = 0; u < kStreamU; ++u) dst[i + u * st] = v[u];
  }
  for (; i < n16; i += st) dst[i] = src[i];
}

template <int NS>
__global__ void __launch_bounds__(256)
k_stream_mix(double2 *__restrict__ dst, const double2 *__restrict__ a, const double2 *__restrict__ b,
             const double2 *__restrict__ c, const long long n16) {
  const long long st = (long long)gridDim.x * 256;
  long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  auto sum = [&](const long long j) {
    double2 v = NS >= 1 ? a[j] : double2{0.0, 0.0};
    if (NS >= 2) {
      const double2 w = b[j];
      v.x += w.x;
      v.y += w.y;
    }
    if (NS >= 3) {
      const double2 w = c[j];
      v.x += w.x;
      v.y += w.y;
    }
    return v;
  };
  for (; i + (kStreamU - 1) * st < n16; i += kStreamU * st) {
    double2 v[kStreamU];
#pragma unroll
    for (int u = 0; u < kStreamU; ++u) v[u] = sum(i + u * st);
#pragma unroll
    for (int u = 0; u < kStreamU; ++u) dst[i + u * st] = v[u];
  }
  for (; i < n16; i += st) dst[i] = sum(i);
}


// ---------------------------------------------------------------------------
// Hermite basis in p: k_hcube, k_hperturb
// ---------------------------------------------------------------------------
// The paper's own discretisation (Sec. III A; Appendix A, Eq. (HEOM2FP-H))
// expands each element in Hermite functions of the momenta,
//   W_n = e^{-beta U/2} prod_s psi_0(p_s) sum_k c_{n,k}(q) prod_s psi_{k_s}(p_s),
// so a state is c[branch][n][k_1..k_M][q_1..q_M] on the q grid alone (k_s <
// Nh_s, held in Np[s]).  With a_s = sqrt(2 m_s / beta) the equation reads
//   dc_{n,k}/dt = - sum_s n_s gamma_s c_{n,k}
//     + sum_s F_s(q) / (sqrt2 a_s) (sqrt(k_s+1) c_{n,k+e_s} - sqrt(k_s) c_{n,k-e_s})
//     + sum_s D_{q_s} [ -a_s / (sqrt2 m_s) (sqrt(k_s+1) c_{n,k+e_s} + sqrt(k_s) c_{n,k-e_s}) ]
//     - sum_s sqrt2 / a_s sqrt(k_s) V_s'(q_s) c_{n+e_s,k-e_s}
//     + sum_s n_s zeta_s gamma_s (m_s/beta) sqrt2 / a_s sqrt(k_s+1) V_s'(q_s) c_{n-e_s,k+e_s}
// (the appendix's D^{+-}, Theta and Phi written out), and the only
// derivatives left are the compact ones along q.  That is the structure of
// k_pcube_s with p and q exchanged: a task is one (branch, element, Hermite
// index k) and its block is the whole q cube, contiguous; the fields of the
// q_2 and q_3 derivatives mix the Hermite neighbours k +- e_s of the same
// element, and the q_1 derivative is folded into one sweep over the q_1
// planes (t = A^{-1} (A s + B G_1), as in k_pcube_s).  Because one task sees
// every derivative of its block, the RK4 stage update is fused in: a whole
// stage is one launch (EPI_OUT writes the right-hand side itself).
// Missing neighbours (k_s at either end of the truncation, n +- e_s outside
// the hierarchy) point at the task's own block with zero factors.

// Largest workgroup for a q_1 bucket (the q_1 line and a round's loads in
// registers).
template <typename T, int NB1>
constexpr int hcube_max_threads() {
  return NB1 >= 48 ? 256 : NB1 >= 32 ? 512 : NB1 >= 24 ? 768 : 1024;
}
// Task constants of k_hcube in LDS: per mode s (slot s of each group of
// three) the factors of c_{k+e_s} and c_{k-e_s} in the q-derivative field
// (GU, GD) and in the force term (FU, FD), of c_{n+e_s,k-e_s} (PH) and
// c_{n-e_s,k+e_s} (TH); then the damping and V_2', V_3' on their grids.
constexpr int kHcGU = 0, kHcGD = 3, kHcFU = 6, kHcFD = 9, kHcPH = 12, kHcTH = 15, kHcDamp = 18;
constexpr int kHcV2 = 20, kHcV3 = kHcV2 + kTab;
constexpr int kHCubeCF = kHcV3 + kTab;
constexpr int kHCubePL = 2;  // q_1 planes per round

// Task order of k_hcube: branch slowest, then the Hermite multi-index kb,
// the element fastest.  For three modes kb walks k_2 in tiles of width T
// (k_3 fastest, then k_2 within the tile, then k_1), so the k_1 neighbours
// of a task are N_3 T multi-indices away rather than N_2 N_3; kb -> kl (the
// storage index, k_3 fastest) is a bijection for any 1 <= T.
__device__ __forceinline__ int hcube_kl(const Geom &g, const int T, const int kb) {
  if (g.M < 3 || T >= g.Np[1]) return kb;
  const int N1 = g.Np[0], N2 = g.Np[1], N3 = g.Np[2];
  const int per_tile = N1 * T * N3;
  const int tt = kb / per_tile;
  const int w = min(T, N2 - tt * T);  // the last tile may be narrower
  int r = kb - tt * per_tile;
  const int k3 = r % N3;
  r /= N3;
  const int k1 = r / w;
  const int k2 = tt * T + (r - k1 * w);
  return (k1 * N2 + k2) * N3 + k3;
}

template <typename T, int NB1, bool SPLIT, int EPI>
__global__ void __launch_bounds__((hcube_max_threads<T, NB1>()))
k_hcube(const Geom g, const Tabs tb, const PCube pc, const T *__restrict__ X, const T *__restrict__ y,
        T *__restrict__ out, const double cst) {
  constexpr int PL = kHCubePL;
  constexpr int NR = (NB1 + PL - 1) / PL;
  constexpr int RC = 2;  // stencil reach along q_1
  constexpr T third = T(1.0 / 3.0);
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int task = pc.chunk > 0 ? xcd_chunk_task(blockIdx.x, pc.chunk) : xcd_task(blockIdx.x, pc.nblk);
  if (task >= pc.ntasks) return;
  const int N1 = SPLIT ? NB1 : pc.N1, N2 = SPLIT ? NB1 : pc.N2, N3 = SPLIT ? NB1 : pc.N3;
  const int plane = SPLIT ? NB1 * NB1 : pc.plane;
  const int rs = SPLIT ? NB1 + 1 : pc.rs;
  T *CF = reinterpret_cast<T *>(smem_raw);
  T *G2 = CF + kHCubeCF;  // [PL][N2][rs]
  T *G3 = G2 + PL * N2 * rs;
  const int per_br = g.ne * g.P;
  const int br = task / per_br;
  const int kb = (task - br * per_br) / g.ne;
  const int e = task - br * per_br - kb * g.ne;  // the elements of one k are adjacent tasks
  const int ea = br * g.ne + e;
  const int kl = hcube_kl(g, pc.ktile, kb);  // Hermite multi-index, k_M fastest in storage
  const int tid = threadIdx.x;
  const bool own = tid < plane;
  const int j2 = own ? tid / N3 : 0;
  const int j3 = own ? tid - j2 * N3 : 0;
  const long long Q = g.Q;
  const long long slice = ((long long)ea * g.P + kl) * Q;  // this task's q cube
  const T *Xe = X + slice;
  T *Oe = out + slice;
  const T *Ye = EPI == EPI_H2 ? y + slice : nullptr;
  const T *Xb = X + (long long)br * g.ne * g.E;  // this branch's element 0
  int kk[3];
  {
    int rem = kl;
    for (int s = 2; s >= 0; --s) {
      kk[s] = s < g.M ? rem % g.Np[s] : 0;
      rem = s < g.M ? rem / g.Np[s] : rem;
    }
  }
  const T *Xu[3], *Xd[3], *Hu[3], *Hd[3];  // c_{k+e}, c_{k-e}, c_{n+e,k-e}, c_{n-e,k+e}
#pragma unroll
  for (int s = 0; s < 3; ++s) {
    const bool on = s < g.M;
    const bool kup = on && kk[s] + 1 < g.Np[s];
    const bool kdn = on && kk[s] > 0;
    const int up = on ? tb.up[e * 3 + s] : -1;
    const int dn = on ? tb.dn[e * 3 + s] : -1;
    const long long ks = on ? (long long)g.PS[s] * Q : 0;
    Xu[s] = kup ? Xe + ks : Xe;
    Xd[s] = kdn ? Xe - ks : Xe;
    Hu[s] = (kdn && up >= 0) ? Xb + ((long long)up * g.P + kl) * Q - ks : Xe;
    Hd[s] = (kup && dn >= 0) ? Xb + ((long long)dn * g.P + kl) * Q + ks : Xe;
  }
  if (tid < 3) {
    const int s = tid;
    const bool on = s < g.M;
    const bool kup = on && kk[s] + 1 < g.Np[s];
    const bool kdn = on && kk[s] > 0;
    const double sp = kup ? sqrt((double)(kk[s] + 1)) : 0.0;  // zero past the truncation
    const double sm = kdn ? sqrt((double)kk[s]) : 0.0;
    const int up = on ? tb.up[e * 3 + s] : -1;
    CF[kHcGU + s] = T(-g.ha[s] * sp);
    CF[kHcGD + s] = T(-g.ha[s] * sm);
    CF[kHcFU + s] = T(g.hf[s] * sp);
    CF[kHcFD + s] = T(-g.hf[s] * sm);
    CF[kHcPH + s] = T(up >= 0 ? -g.hl[s] * sm : 0.0);
    CF[kHcTH + s] = T(on ? tb.cc[e * 3 + s] * g.hl[s] * sp : 0.0);  // cc is zero when n_s = 0
    if (s == 0) CF[kHcDamp] = T(tb.damp[e]);
  }
  if (tid < N2) CF[kHcV2 + tid] = T(g.M > 1 ? tb.Vp[1 * kTab + tid] : 0.0);
  if (tid < N3) CF[kHcV3 + tid] = T(g.M > 2 ? tb.Vp[2 * kTab + tid] : 0.0);
  __syncthreads();
  const T ca1 = T(g.dq_ca[0]), cb1 = T(g.dq_cb[0]);
  const uint32_t own_off = (uint32_t)(own ? tid : 0);
  const double *F2 = tb.F + 1 * Q, *F3 = tb.F + 2 * Q;

  T ln[NB1];  // row j of A t = r while it collects its terms, then its forward result d_j
#pragma unroll
  for (int j = 0; j < NB1; ++j) ln[j] = T(0);
  T dprev = T(0);
  auto elim = [&](const int j) {
    const T d = j == 0 ? ln[j] : fma_t(T(-kThomas.inv[j] / 3.0), dprev, ln[j] * T(kThomas.inv[j]));
    dprev = d;
    ln[j] = d;
  };

#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const int i0 = r * PL;
    if (i0 >= N1) break;  // uniform
    T sv[PL], gv[PL];
#pragma unroll
    for (int k = 0; k < PL; ++k) {
      const int i = i0 + k;
      sv[k] = gv[k] = T(0);
      if (i < N1) {
        uint32_t o = (uint32_t)(i * plane) + own_off;
        asm volatile("" : "+v"(o));
        const T c0 = at_u32(Xe, o);
        const T u1 = at_u32(Xu[0], o), d1 = at_u32(Xd[0], o);
        const T u2 = at_u32(Xu[1], o), d2 = at_u32(Xd[1], o);
        const T u3 = at_u32(Xu[2], o), d3 = at_u32(Xd[2], o);
        const T a1 = at_u32(Hu[0], o), b1 = at_u32(Hd[0], o);
        const T a2 = at_u32(Hu[1], o), b2 = at_u32(Hd[1], o);
        const T a3 = at_u32(Hu[2], o), b3 = at_u32(Hd[2], o);
        const T f1 = T(at_u32(tb.F, o)), f2 = T(at_u32(F2, o)), f3 = T(at_u32(F3, o));
        const T v1 = T(tb.Vp[0 * kTab + i]), v2 = CF[kHcV2 + j2], v3 = CF[kHcV3 + j3];
        sv[k] = -CF[kHcDamp] * c0 + f1 * (CF[kHcFU] * u1 + CF[kHcFD] * d1) +
                f2 * (CF[kHcFU + 1] * u2 + CF[kHcFD + 1] * d2) + f3 * (CF[kHcFU + 2] * u3 + CF[kHcFD + 2] * d3) +
                v1 * (CF[kHcPH] * a1 + CF[kHcTH] * b1) + v2 * (CF[kHcPH + 1] * a2 + CF[kHcTH + 1] * b2) +
                v3 * (CF[kHcPH + 2] * a3 + CF[kHcTH + 2] * b3);
        gv[k] = CF[kHcGU] * u1 + CF[kHcGD] * d1;
        if (own) {
          const int li = (k * N2 + j2) * rs + j3;
          G2[li] = CF[kHcGU + 1] * u2 + CF[kHcGD + 1] * d2;
          G3[li] = CF[kHcGU + 2] * u3 + CF[kHcGD + 2] * d3;
        }
      }
      asm volatile("" : "+v"(sv[k]), "+v"(gv[k]));
    }
    __syncthreads();
    // q_2 lines of G2 (fixed k, j3) and q_3 lines of G3 (fixed k, j2)
    const int npl = min(PL, N1 - i0);
    const int nl2 = npl * N3, nl = nl2 + npl * N2;
    if (SPLIT) {
#pragma unroll 1
      for (int hl = tid; hl < 2 * nl; hl += blockDim.x) {
        const int l = hl >> 1;
        if (l < nl2) {
          const int k = l / N3, c = l - k * N3;
          compact_split<T, NB1>(G2, k * N2 * rs + c, rs, hl & 1, T(g.dq_ca[1]), T(g.dq_cb[1]));
        } else {
          compact_split<T, NB1>(G3, (l - nl2) * rs, 1, hl & 1, T(g.dq_ca[2]), T(g.dq_cb[2]));
        }
      }
    } else {
#pragma unroll 1
      for (int l = tid; l < nl; l += blockDim.x) {
        if (l < nl2) {
          const int k = l / N3, c = l - k * N3;
          compact_lds<T>(G2, k * N2 * rs + c, rs, N2, T(g.dq_ca[1]), T(g.dq_cb[1]));
        } else {
          compact_lds<T>(G3, (l - nl2) * rs, 1, N3, T(g.dq_ca[2]), T(g.dq_cb[2]));
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < PL; ++k) {
      const int i = i0 + k;
      if (i < N1) {
        const int li = (k * N2 + j2) * rs + j3;
        const T s = sv[k] + G2[li] + G3[li];
        const T gg = gv[k];
        ln[i] += s;  // A s
        if (i >= 1) ln[i >= 1 ? i - 1 : 0] += third * s;
        if (i + 1 < NB1) ln[i + 1 < NB1 ? i + 1 : 0] += third * s;
        // B G_1: row j takes ca (G_{j+1} - G_{j-1}) + cb (G_{j+2} - G_{j-2})
        if (i >= 1) ln[i >= 1 ? i - 1 : 0] += ca1 * gg;
        if (i >= 2) ln[i >= 2 ? i - 2 : 0] += cb1 * gg;
        if (i + 1 < NB1) ln[i + 1 < NB1 ? i + 1 : 0] -= ca1 * gg;
        if (i + 2 < NB1) ln[i + 2 < NB1 ? i + 2 : 0] -= cb1 * gg;
        if (i >= RC) elim(i >= RC ? i - RC : 0);
        if (i == N1 - 1) {
#pragma unroll
          for (int q = RC - 1; q >= 0; --q)
            if (i - q >= 0) elim(i - q >= 0 ? i - q : 0);
        }
      }
    }
    __syncthreads();  // the next round overwrites the planes
  }
  if (!own) return;
  // back substitution from the far end of the q_1 line, with the stage update
  T x = T(0);
#pragma unroll
  for (int j = NB1 - 1; j >= 0; --j) {
    if (j < N1) {
      x = ln[j] - T(kThomas.cp[j]) * x;
      uint32_t o = (uint32_t)(j * plane + tid);
      asm volatile("" : "+v"(o));
      if (EPI == EPI_OUT)
        at_u32(Oe, o) = x;
      else if (EPI == EPI_H1)
        at_u32(Oe, o) = at_u32(Xe, o) + T(cst) * x;
      else if (EPI == EPI_H2)
        at_u32(Oe, o) = at_u32(Ye, o) + T(cst) * x;
      else
        at_u32(Oe, o) = at_u32(Oe, o) + T(cst) * x;
    }
  }
}

// Excitation in the Hermite basis, Eq. (Opticalexc): dX/dq_s d/dp_s acts on
// W = e^{-beta H/2} h as dX/dq_s (d/dp_s - p_s / a_s^2) on h, which raises
// the Hermite index: (X^x c)_{n,k} = - sum_s dX/dq_s(q) sqrt2 / a_s sqrt(k_s)
// c_{n,k-e_s}, for every element n (grad[s][q] = dX/dq_s; one state).
template <typename TO>
__global__ void __launch_bounds__(256)
k_hperturb(const Geom g, const double *__restrict__ W, TO *__restrict__ out, const double *__restrict__ grad) {
  const long long Q = g.Q, S = (long long)g.ne * g.E;
  for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < S; i += (long long)gridDim.x * 256) {
    const long long sl = i / Q;  // (element, Hermite index)
    const int ql = (int)(i - sl * Q);
    const int kl = (int)(sl % g.P);
    double v = 0.0;
    for (int s = 0; s < g.M; ++s) {
      const int ks = (kl / g.PS[s]) % g.Np[s];
      if (ks > 0) v -= grad[s * Q + ql] * g.hl[s] * sqrt((double)ks) * W[i - (long long)g.PS[s] * Q];
    }
    out[i] = TO(v);
  }
}

}  // namespace chfpe
