// Host side of the gfx950 CHFPE solver: the C ABI declared in include/chfpe.h.
//
// Device buffers hold h_n with W_n = exp(-beta H/2) h_n (Sec. III A); the
// ABI exchanges W, converting with the separable factor
// exp(-beta U(q)/2) exp(-sum_s beta p_s^2/4m_s).
// A context owns (inside one device workspace) the coefficient tables of the
// right-hand side of Eq. (eq:HEOM), the equilibrium W_eq, the t1-branch state
// U of the double loop of Sec. IV C, and the buffers of RK4: y (the
// propagated state), xa/xb (stage states, alternating) and t (partial
// right-hand side).  One RK4 step is the degree-4 Taylor polynomial of the
// generator, which classical RK4 equals for a linear time-independent
// system, in nested form (four stages, see Epi in kernels.h).  A stage is one
// p-axis launch (k_pblock, or k_pcube for three modes) followed by one or two
// k_qpass launches, the last of which applies the stage update.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include <type_traits>

#include "chfpe.h"
#include "closure.h"
#include "kernels.h"

using namespace chfpe;

namespace {

thread_local std::string g_setup_error = "no error";

constexpr int kPBlockThreads = 256;  // k_pblock workgroup size (upper bound)
constexpr int kPBlockRPT = 4;        // rows per k_pblock thread
constexpr int kQThreadsMax = 512;    // largest k_qpass workgroup

// Kernel kinds for event timing; batched launches (several branch states per
// launch) are kept apart from single-state ones.
constexpr int kNumBase = 15;
constexpr int kNumKinds = 2 * kNumBase;
enum Kind : int {
  K_PBLOCK = 0,
  K_QACC = 1,
  K_QS1 = 2,
  K_QS2 = 3,
  K_QS3 = 4,
  K_QS4 = 5,
  K_OBSERVE = 6,
  K_PERTURB = 7,
  K_QOUT = 8,
  K_PCUBE = 9,
  K_HS1 = 10,  // Hermite basis: one k_hcube launch per RK4 stage
  K_HS2 = 11,
  K_HS3 = 12,
  K_HS4 = 13,
  K_HOUT = 14
};
const char *kKindNames[kNumKinds] = {
    "pblock_rhs", "qpass_acc", "qpass_rk4_s1", "qpass_rk4_s2", "qpass_rk4_s3", "qpass_rk4_s4", "observe",
    "perturb", "qpass_out", "pcube_rhs", "hcube_rk4_s1", "hcube_rk4_s2", "hcube_rk4_s3", "hcube_rk4_s4",
    "hcube_out", "batch_pblock_rhs", "batch_qpass_acc", "batch_qpass_rk4_s1",
    "batch_qpass_rk4_s2", "batch_qpass_rk4_s3", "batch_qpass_rk4_s4", "batch_observe", "batch_perturb",
    "batch_qpass_out", "batch_pcube_rhs", "batch_hcube_rk4_s1", "batch_hcube_rk4_s2", "batch_hcube_rk4_s3",
    "batch_hcube_rk4_s4", "batch_hcube_out"};
// state passes each kind reads plus writes (each input once, each output
// once): the first stage reads its input (y) and t and writes z1; later
// stages also read y (the last one reads and writes it in place); a
// Hermite stage reads its input (and y) and writes its output
const double kKindPasses[kNumBase] = {2, 3, 3, 4, 4, 4, 0.1, 2, 3, 2, 2, 3, 3, 3, 2};

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

struct Derived {
  int prec = 0, B = 1;    // precision of branch states; branches per wave
  bool batched = false;   // 2D responses use the batched branch buffers
  bool hermite = false;   // Hermite basis in p: P counts Hermite functions, layout [n][k][q]
  int M = 0, K = 0, ne = 0;
  int Nq[3] = {0, 0, 0}, Np[3] = {0, 0, 0};  // axes s >= M stay 0
  int Q = 0, P = 0;
  long long E, S;  // points per element, values per state
  std::vector<int> nvec;  // ne * M
};

// A dispatch's grid size counts work-items in 32 bits: every launch must stay
// within it (a larger one would wrap and leave tasks unrun).
constexpr long long kMaxGridItems = 0xFFFFFFFFLL;
constexpr int kMaxHcChunk = 1024;  // largest k_hcube XCD chunk (tasks)

// work-items of a launch of ntasks workgroups, padded to a multiple of 8
long long grid_items(long long ntasks, int threads) { return (ntasks + 7) / 8 * 8 * (long long)threads; }

// The k_pblock tile of the innermost p axes (one, or the last two): RG row
// groups of cols threads, each thread covering up to kPBlockRPT rows of a
// task's run of nb blocks.  RG divides rows (two or three modes), so a row
// batch lies in one block.  nb_hi: most blocks per task the row coverage and
// the LDS budget allow; nb_lo: fewest for which the launch over every state
// of the largest batch fits one dispatch.
struct PBShape {
  int NB, rows, cols, RG, nblocks, nb_lo, nb_hi;
  size_t blk_bytes;
  long long items(const Derived &d, int nb) const {
    const long long tasks = (long long)d.ne * (d.batched ? d.B : 1) * ((nblocks + nb - 1) / nb);
    return grid_items(tasks, RG * cols);
  }
};

PBShape pblock_shape(const Derived &d) {
  PBShape s{};
  const int M = d.M;
  s.NB = M == 1 ? 1 : 2;
  s.cols = d.Np[M - 1];
  s.rows = M == 1 ? 1 : d.Np[M - 2];
  s.RG = std::max(1, kPBlockThreads / s.cols);
  if (s.NB == 2)
    while (s.rows % s.RG) --s.RG;
  s.nblocks = (int)(d.E / ((long long)s.rows * s.cols));
  s.blk_bytes = (size_t)s.NB * s.rows * (s.cols + 1) * sizeof(double);
  long long hi = std::min<long long>((long long)kPBlockRPT * s.RG / s.rows, (long long)(80 * 1024 / s.blk_bytes));
  s.nb_hi = (int)std::max<long long>(1, std::min<long long>(hi, s.nblocks));
  s.nb_lo = 1;
  while (s.nb_lo < s.nb_hi && s.items(d, s.nb_lo) > kMaxGridItems) ++s.nb_lo;
  return s;
}

int nmax_bucket(int n) {
  return n <= 8 ? 8 : n <= 12 ? 12 : n <= 16 ? 16 : n <= 24 ? 24 : n <= 32 ? 32 : 48;
}

// The p block of k_pcube for two or three modes: p_1 lines (registers) of
// up to 32 points (three modes) or 48 (two modes), a (p_2, p_3) plane (two
// modes: a p_2 row) of threads within the workgroup bound, and the LDS copy
// of the block plus a round's planes within 160 KB (FP64).
int pcube_n3(const Derived &d) { return d.M == 3 ? d.Np[2] : 1; }
bool pcube_shape_ok(const Derived &d) {
  if (d.M < 2) return false;
  const int nb1 = nmax_bucket(d.Np[0]);
  const int plane = d.Np[1] * pcube_n3(d);
  const int maxthr = nb1 > 32 ? pcube_max_threads<double, 48>()
                     : nb1 >= 32 ? pcube_max_threads<double, 32>()
                     : nb1 >= 24 ? pcube_max_threads<double, 24>() : pcube_max_threads<double, 16>();
  const size_t lds = ((size_t)d.P + 2 * (size_t)pcube_planes(nb1) * d.Np[1] * (pcube_n3(d) + 1)) * sizeof(double);
  const long long items = ((long long)d.ne * d.Q * (d.batched ? d.B : 1) + 7) / 8 * 8 * ((plane + 63) / 64 * 64);
  return nb1 <= (d.M == 3 ? 32 : 48) && (plane + 63) / 64 * 64 <= maxthr && lds <= 160 * 1024 &&
         items <= 0xFFFFFFFFLL;
}

// The q cube of a k_hcube task (Hermite basis): q_1 lines (registers) of at
// most 48 points, a (q_2, q_3) plane (two modes: a q_2 row; one mode: one
// point) of threads within the workgroup bound of the q_1 bucket.
int hcube_n2(const Derived &d) { return d.M >= 2 ? d.Nq[1] : 1; }
int hcube_n3(const Derived &d) { return d.M == 3 ? d.Nq[2] : 1; }
int hcube_max_threads_for(int nb1) {
  return nb1 >= 48 ? hcube_max_threads<double, 48>()
         : nb1 >= 32 ? hcube_max_threads<double, 32>()
         : nb1 >= 24 ? hcube_max_threads<double, 24>() : hcube_max_threads<double, 16>();
}
bool hcube_shape_ok(const Derived &d, std::string &err) {
  const int nb1 = nmax_bucket(d.Nq[0]);
  const int thr = (hcube_n2(d) * hcube_n3(d) + 63) / 64 * 64;
  if (thr > hcube_max_threads_for(nb1)) {
    err = "Hermite basis: the (q_2, q_3) plane has more points than one workgroup for q_1 lines of " +
          std::to_string(d.Nq[0]) + " points allows";
    return false;
  }
  // (with room for the padding of the largest XCD chunk)
  const long long items = grid_items((long long)d.ne * d.P * (d.batched ? d.B : 1) + 8 * kMaxHcChunk, thr);
  if (items > kMaxGridItems) {
    err = "batch too large: a k_hcube launch over every branch state exceeds one dispatch (2^32 work-items)";
    return false;
  }
  return true;
}

bool derive(const chfpe_params *p, Derived &d, std::string &err) {
  if (!p) {
    err = "params is NULL";
    return false;
  }
  if (p->M < 1 || p->M > 3) {
    err = "M must be 1, 2 or 3";
    return false;
  }
  if (p->K < 0 || p->K > 12) {
    err = "K must be in [0, 12]";
    return false;
  }
  if (p->precision != CHFPE_FP64 && p->precision != CHFPE_FP32) {
    err = "precision must be CHFPE_FP64 or CHFPE_FP32";
    return false;
  }
  if (p->batch < 0 || p->batch > 1024) {
    err = "batch must be in [0, 1024]";
    return false;
  }
  if (p->basis != CHFPE_BASIS_GRID && p->basis != CHFPE_BASIS_HERMITE) {
    err = "basis must be CHFPE_BASIS_GRID or CHFPE_BASIS_HERMITE";
    return false;
  }
  d.hermite = p->basis == CHFPE_BASIS_HERMITE;
  d.prec = p->precision;
  d.B = p->batch > 0 ? p->batch : 1;
  d.batched = d.B > 1 || d.prec == CHFPE_FP32;
  d.M = p->M;
  d.K = p->K;
  d.Q = 1;
  d.P = 1;
  for (int s = 0; s < p->M; ++s) {
    const int np_lo = d.hermite ? 2 : 5;  // Hermite functions per mode, or p points
    if (p->Nq[s] < 5 || p->Nq[s] > kMaxAxis || p->Np[s] < np_lo || p->Np[s] > kMaxAxis) {
      err = d.hermite ? "every q axis needs 5 <= N <= 48 points and every mode 2 <= Nh <= 48 Hermite functions"
                      : "every axis needs 5 <= N <= 48 points";
      return false;
    }
    if (!(p->Lq[s] > 0) || (!d.hermite && !(p->Lp[s] > 0)) || !(p->m[s] > 0)) {
      err = "box half-widths and masses must be positive";
      return false;
    }
    d.Nq[s] = p->Nq[s];
    d.Np[s] = p->Np[s];
    d.Q *= p->Nq[s];
    d.P *= p->Np[s];
  }
  if (!(p->beta > 0)) {
    err = "beta must be positive";
    return false;
  }
  const double *scal[] = {p->omega, p->g3, p->g4, p->V_LL, p->V_SL, p->zeta, p->gamma};
  for (auto arr : scal)
    for (int s = 0; s < p->M; ++s)
      if (!std::isfinite(arr[s])) {
        err = "non-finite model parameter";
        return false;
      }
  for (int s = 0; s < p->M; ++s)
    for (int t = 0; t < p->M; ++t)
      if (!std::isfinite(p->g2[s][t]) || !std::isfinite(p->g21[s][t]) || !std::isfinite(p->g12[s][t])) {
        err = "non-finite coupling parameter";
        return false;
      }
  // hierarchy elements: |n| ascending, then n_1 largest first
  d.nvec.clear();
  std::vector<int> cur(d.M, 0);
  for (int deg = 0; deg <= d.K; ++deg) {
    // enumerate compositions of deg into M parts, lexicographically descending
    std::vector<int> n(d.M, 0);
    std::function<void(int, int)> rec = [&](int s, int left) {
      if (s == d.M - 1) {
        n[s] = left;
        d.nvec.insert(d.nvec.end(), n.begin(), n.end());
        return;
      }
      for (int v = left; v >= 0; --v) {
        n[s] = v;
        rec(s + 1, left - v);
      }
    };
    rec(0, deg);
  }
  d.ne = (int)(d.nvec.size() / d.M);
  if (d.ne > 4096) {
    err = "too many hierarchy elements";
    return false;
  }
  d.E = (long long)d.Q * d.P;
  d.S = d.E * d.ne;
  if (d.E >= (1LL << 29)) {  // byte offsets within an element fit 32 bits
    err = "one element must have fewer than 2^29 points";
    return false;
  }
  if (d.hermite) return hcube_shape_ok(d, err);
  const PBShape ps = pblock_shape(d);
  if (ps.rows > kPBlockRPT * ps.RG) {
    if (pcube_shape_ok(d)) return true;  // k_pcube takes the p block
    err = "the last two p axes (" + std::to_string(ps.rows) + " x " + std::to_string(ps.cols) +
          " points) cannot be tiled: N_{M-1} needs a divisor d with d * N_M <= 256 and N_{M-1} <= 4 d, "
          "and the p block does not fit one k_pcube workgroup";
    return false;
  }
  if (ps.items(d, ps.nb_lo) > kMaxGridItems) {
    if (pcube_shape_ok(d)) return true;
    err = "batch too large: the p-block launch over every branch state exceeds one dispatch (2^32 work-items)";
    return false;
  }
  return true;
}

constexpr int kStateBufs = 6;   // FP64: W_eq, U, y, xa, xb, t
constexpr int kBranchBufs = 4;  // per branch of a wave: y, xa, xb, t

// Workspace layout (byte offsets, 256-aligned).
struct Layout {
  size_t F, VpQ, Vp, pm, pg, gA, gB, gC, Cw, wp, sq, sp, up, dn, cc, tc, damp, partial, scal, flag, clos;
  size_t bufs[kStateBufs];
  size_t bbufs[kBranchBufs];  // batched branch buffers: y, xa, xb, t (B states each)
  size_t total;
};
constexpr int kPartials = 2048;

Layout layout(const Derived &d) {
  Layout L{};
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o = align_up(o + bytes, 256);
    return at;
  };
  L.F = take(sizeof(double) * 3 * d.Q);
  L.VpQ = take(sizeof(double) * 3 * d.Q);
  L.Vp = take(sizeof(double) * 3 * kTab);
  L.pm = take(sizeof(double) * 3 * kTab);
  L.pg = take(sizeof(double) * 3 * kTab);
  L.gA = take(sizeof(double) * 3 * d.Q);
  L.gB = take(sizeof(double) * 3 * d.Q);
  L.gC = take(sizeof(double) * 3 * d.Q);
  L.Cw = take(sizeof(double) * d.Q);
  L.wp = take(sizeof(double) * d.P);
  L.sq = take(sizeof(double) * d.Q);
  L.sp = take(sizeof(double) * d.P);
  L.up = take(sizeof(int) * 3 * d.ne);
  L.dn = take(sizeof(int) * 3 * d.ne);
  L.cc = take(sizeof(double) * 3 * d.ne);
  L.tc = take(sizeof(double) * 3 * d.ne);
  L.damp = take(sizeof(double) * d.ne);
  L.partial = take(sizeof(double) * kPartials);
  L.scal = take(sizeof(double) * 16);
  L.flag = take(sizeof(int) * 16);
  L.clos = take(sizeof(double) * 6 * 2 * kClosRows * kTab);  // closure weights [axis][orientation][6][kTab]
  for (int i = 0; i < kStateBufs; ++i) L.bufs[i] = take(sizeof(double) * (size_t)d.S);
  const size_t tsz = d.prec == CHFPE_FP32 ? sizeof(float) : sizeof(double);
  for (int i = 0; i < kBranchBufs; ++i) L.bbufs[i] = d.batched ? take(tsz * (size_t)d.S * d.B) : 0;
  L.total = o;
  return L;
}

struct Launch {
  PBlock pb{};
  size_t pb_lds = 0;
  int pb_threads = 256, pb_nmax = 48;
  int pb_rpt = 4;  // rows per k_pblock thread (3 where it tiles the 24-row blocks exactly)
  // strided-axis passes of one stage: qa (three modes only, accumulates into
  // t) then qf (applies the stage update); qx: the p_1 excitation pass of
  // three modes.
  QPass qa{}, qf{}, qx{};
  bool has_qa = false, qf_two = false, has_qx = false;
  // three modes: all p axes of a q point in one k_pcube task (then the q
  // passes are (q_2, q_3) and q_1 alone, and excitations need no qx)
  bool pcube = false, pcube_split = false, pcube_stream = false;
  PCube pcb{};
  // Hermite basis: k_hcube over the q cube of each (branch, element, k)
  bool hcube = false, hcube_split = false;
  PCube hcb{};
  int hcube_threads = 0, hcube_nb1 = 0;
  int pcube_threads = 0, pcube_nb1 = 0;
  size_t pcube_lds = 0;
  int qa_threads = 0, qf_threads = 0, qx_threads = 0;
  size_t qa_lds = 0, qf_lds = 0;
  int qa_nmax = 48, qf_nmax = 48, qx_nmax = 48;
};

int pad8(int n) { return (n + 7) / 8 * 8; }
// k_hcube grid: a multiple of 8 chunks when the tasks go to the XCDs in chunks
int hcube_nblk(int ntasks, int chunk) { return chunk > 0 ? (ntasks + 8 * chunk - 1) / (8 * chunk) * (8 * chunk) : pad8(ntasks); }

// Tile shapes the autotuner picked, kept per problem shape for the rest of
// the process (later contexts of the same shape start from them).
struct TileChoice {
  int pb_nb = 0, pb_split = -1, q_pc = 0, pb_run = 0;
};
std::mutex g_tune_mu;
std::map<std::vector<long long>, TileChoice> g_tuned;

std::vector<long long> tune_key(const Derived &d) {
  std::vector<long long> k = {d.M, d.K, d.prec, d.B, d.batched ? 1 : 0};
  for (int s = 0; s < 3; ++s) {
    k.push_back(s < d.M ? d.Nq[s] : 0);
    k.push_back(s < d.M ? d.Np[s] : 0);
  }
  return k;
}


}  // namespace

struct chfpe_ctx {
  chfpe_params prm;
  Derived d;
  Layout L;
  Launch ln;
  Geom g;
  Tabs tb;
  hipStream_t stream = nullptr;
  unsigned char *ws = nullptr;
  bool own_ws = false;
  double *F, *VpQ, *Vp, *pm, *pg, *gA, *gB, *gC, *Cw, *wp, *sq, *sp, *cc, *tc, *damp, *partial, *scal;
  int *up, *dn, *flag;
  double *weq, *u, *y, *xa, *xb, *t;
  void *bb[kBranchBufs] = {nullptr, nullptr, nullptr, nullptr};  // batched y, xa, xb, t
  // cached graph of one wave's t2 loop
  hipGraphExec_t wave_graph = nullptr;
  long long wave_key[6] = {0, 0, 0, 0, 0, 0};
  bool has_eq = false;
  double dV = 1.0;
  std::vector<double> qgrid[3], pgrid[3];
  std::vector<double> wq_host;  // q-point weights (product over q axes), Q entries
  std::vector<double> sq_host;  // exp(-beta U(q)/2), Q entries
  double *rbuf = nullptr;
  size_t rbuf_cap = 0;
  std::string err = "no error";
  int tune_pb_nb = 0;   // blocks per k_pblock task (0: automatic)
  int tune_q_pc = 0;    // run positions per two-axis k_qpass tile (0: automatic)
  int tune_pb_split = -1;  // k_pblock lines solved by lane pairs (-1: automatic)
  int tune_pb_run = 0;     // k_pblock consecutive block groups per state in task order (0: 1)
  int tune_pc_pad = 0;     // k_pcube LDS plane row pad (0: 1)
  int tune_pc_stream = -1;  // k_pcube_s (1) or k_pcube (0); -1: by the p_1 length
  int tune_hc_chunk = -1;   // k_hcube tasks per XCD chunk (0: one contiguous range per XCD; -1: automatic)
  int tune_hc_ktile = 0;    // k_hcube k_2 tile of the task order (0: automatic)
  bool capturing = false;  // a HIP graph is being captured: no event timing
  bool closure_on = false; // right-hand sides use the closure stencil weights (tb.clos)
  bool use_graphs = true;
  bool allow_pcube = true;  // three modes: k_pcube where the p block fits it
  // kernel timing
  int timing_every = 0;
  long long step_counter = 0;
  bool timing_now = false;
  struct Pending {
    hipEvent_t a, b;
    int kind;
    double bytes;
  };
  std::vector<Pending> pending;
  std::vector<hipEvent_t> event_pool;
  long long kcount[kNumKinds] = {0};
  double ktime[kNumKinds] = {0};
  double kbytes[kNumKinds] = {0};
};

namespace {

int fail(chfpe_ctx *c, int code, const std::string &msg) {
  if (c)
    c->err = msg;
  else
    g_setup_error = msg;
  return code;
}

#define HIPCHK(ctx, call)                                                                  \
  do {                                                                                     \
    hipError_t e_ = (call);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return fail(ctx, CHFPE_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

double coord(int i, int N, double L) { return -L + (i + 0.5) * (2.0 * L / N); }
double qw(int i, int N) { return (i == 0 || i == N - 1) ? 0.8 : 1.0; }

// Host tables of the right-hand side (FP64).
void build_tables(chfpe_ctx *c, std::vector<double> &F, std::vector<double> &Vp,
                  std::vector<double> &pm, std::vector<double> &pg, std::vector<double> &sq,
                  std::vector<double> &sp, std::vector<double> &wp, std::vector<int> &up,
                  std::vector<int> &dn, std::vector<double> &cc, std::vector<double> &tc,
                  std::vector<double> &damp) {
  const chfpe_params &p = c->prm;
  const Derived &d = c->d;
  const int M = d.M;
  for (int s = 0; s < M; ++s) {
    c->qgrid[s].resize(d.Nq[s]);
    c->pgrid[s].resize(d.Np[s]);
    for (int i = 0; i < d.Nq[s]; ++i) c->qgrid[s][i] = coord(i, d.Nq[s], p.Lq[s]);
    // Hermite basis: no p grid (the p tables are unused; zeros)
    for (int i = 0; i < d.Np[s]; ++i) c->pgrid[s][i] = d.hermite ? 0.0 : coord(i, d.Np[s], p.Lp[s]);
  }
  F.assign(3 * d.Q, 0.0);
  sq.assign(d.Q, 0.0);
  c->wq_host.assign(d.Q, 1.0);
  for (int ql = 0; ql < d.Q; ++ql) {
    double q[3] = {0, 0, 0};
    int rem = ql;
    double wgt = 1.0;
    for (int s = M - 1; s >= 0; --s) {
      const int j = rem % d.Nq[s];
      rem /= d.Nq[s];
      q[s] = c->qgrid[s][j];
      wgt *= qw(j, d.Nq[s]);
    }
    c->wq_host[ql] = wgt;
    double U = 0.0;
    for (int s = 0; s < M; ++s) {
      const double x = q[s], k2 = p.m[s] * p.omega[s] * p.omega[s];
      U += 0.5 * k2 * x * x + p.g3[s] * x * x * x / 6.0 + p.g4[s] * x * x * x * x / 24.0;
      F[s * d.Q + ql] = k2 * x + 0.5 * p.g3[s] * x * x + p.g4[s] * x * x * x / 6.0;
    }
    for (int s = 0; s < M; ++s)
      for (int t = s + 1; t < M; ++t) {
        const double a = q[s], b = q[t];
        U += p.g2[s][t] * a * b + (p.g21[s][t] * a * a * b + p.g12[s][t] * a * b * b) / 6.0;
        F[s * d.Q + ql] += p.g2[s][t] * b + (2.0 * p.g21[s][t] * a * b + p.g12[s][t] * b * b) / 6.0;
        F[t * d.Q + ql] += p.g2[s][t] * a + (p.g21[s][t] * a * a + 2.0 * p.g12[s][t] * a * b) / 6.0;
      }
    sq[ql] = std::exp(-0.5 * p.beta * U);
  }
  c->sq_host = sq;
  Vp.assign(3 * kTab, 0.0);
  pm.assign(3 * kTab, 0.0);
  pg.assign(3 * kTab, 0.0);
  for (int s = 0; s < M; ++s) {
    for (int j = 0; j < d.Nq[s]; ++j) Vp[s * kTab + j] = p.V_LL[s] + p.V_SL[s] * c->qgrid[s][j];
    for (int j = 0; j < d.Np[s]; ++j) {
      pg[s * kTab + j] = c->pgrid[s][j];
      pm[s * kTab + j] = c->pgrid[s][j] / p.m[s];
    }
  }
  sp.assign(d.P, 0.0);
  wp.assign(d.P, 1.0);
  for (int pi = 0; pi < d.P; ++pi) {
    int rem = pi;
    double ke = 0.0, wgt = 1.0;
    for (int s = M - 1; s >= 0; --s) {
      const int j = rem % d.Np[s];
      rem /= d.Np[s];
      const double x = c->pgrid[s][j];
      ke += x * x / (2.0 * p.m[s]);
      wgt *= qw(j, d.Np[s]);
    }
    sp[pi] = std::exp(-0.5 * p.beta * ke);
    wp[pi] = wgt * sp[pi];  // quadrature weight times the p part of exp(-beta H/2)
    if (d.hermite) sp[pi] = wp[pi] = 1.0;  // p is integrated exactly: sum over k = 0 only
  }
  const int ne = d.ne;
  up.assign(3 * ne, -1);
  dn.assign(3 * ne, -1);
  cc.assign(3 * ne, 0.0);
  tc.assign(3 * ne, 0.0);
  damp.assign(ne, 0.0);
  auto find = [&](const int *want) {
    for (int e = 0; e < ne; ++e) {
      bool ok = true;
      for (int s = 0; s < M; ++s) ok = ok && d.nvec[e * M + s] == want[s];
      if (ok) return e;
    }
    return -1;
  };
  for (int e = 0; e < ne; ++e) {
    const int *n = &d.nvec[e * M];
    for (int s = 0; s < M; ++s) {
      damp[e] += n[s] * p.gamma[s];
      int nb[3] = {0, 0, 0};
      for (int t = 0; t < M; ++t) nb[t] = n[t] + (t == s ? 1 : 0);
      up[e * 3 + s] = find(nb);
      if (n[s] > 0) {
        for (int t = 0; t < M; ++t) nb[t] = n[t] - (t == s ? 1 : 0);
        dn[e * 3 + s] = find(nb);
        cc[e * 3 + s] = n[s] * p.zeta[s] * p.gamma[s] * p.m[s] / p.beta;
        tc[e * 3 + s] = n[s] * p.zeta[s] * p.gamma[s];
      }
    }
  }
}

void make_geom(chfpe_ctx *c) {
  const Derived &d = c->d;
  Geom &g = c->g;
  std::memset(&g, 0, sizeof(g));
  g.M = d.M;
  g.ne = d.ne;
  g.nbatch = 1;
  g.Q = d.Q;
  g.P = d.P;
  g.E = d.E;
  const int NpM = d.Np[d.M - 1];
  int qs = 1, ps = 1;
  for (int s = d.M - 1; s >= 0; --s) {
    g.Nq[s] = d.Nq[s];
    g.Np[s] = d.Np[s];
    g.QS[s] = qs;
    g.PS[s] = ps;
    g.PSp[s] = (s == d.M - 1) ? 1 : ps / NpM * (NpM + 1);
    qs *= d.Nq[s];
    ps *= d.Np[s];
  }
  for (int s = 0; s < d.M; ++s) {
    const double hq = 2.0 * c->prm.Lq[s] / d.Nq[s];
    const double hp = d.hermite ? 0.0 : 2.0 * c->prm.Lp[s] / d.Np[s];
    g.bm[s] = c->prm.beta / (2.0 * c->prm.m[s]);
    g.dq_ca[s] = 7.0 / 9.0 / hq;
    g.dq_cb[s] = 1.0 / 36.0 / hq;
    g.dp_ca[s] = d.hermite ? 0.0 : 7.0 / 9.0 / hp;
    g.dp_cb[s] = d.hermite ? 0.0 : 1.0 / 36.0 / hp;
    const double a = std::sqrt(2.0 * c->prm.m[s] / c->prm.beta);  // Hermite width a_s
    g.ha[s] = a / (std::sqrt(2.0) * c->prm.m[s]);
    g.hf[s] = 1.0 / (std::sqrt(2.0) * a);
    g.hl[s] = std::sqrt(2.0) / a;
  }
  // dV = prod h (q axes only in the Hermite basis: p is integrated exactly)
  c->dV = 1.0;
  for (int s = 0; s < d.M; ++s)
    c->dV *= (2.0 * c->prm.Lq[s] / d.Nq[s]) * (d.hermite ? 1.0 : 2.0 * c->prm.Lp[s] / d.Np[s]);
}

// Axis ids: 0..M-1 are q_1..q_M, M..2M-1 are p_1..p_M.
int axis_len(const Derived &d, int ax) { return ax < d.M ? d.Nq[ax] : d.Np[ax - d.M]; }
int axis_stride(const Geom &g, int ax) { return ax < g.M ? g.QS[ax] * g.P : g.PS[ax - g.M]; }
double axis_ca(const Geom &g, int ax) { return ax < g.M ? g.dq_ca[ax] : g.dp_ca[ax - g.M]; }
double axis_cb(const Geom &g, int ax) { return ax < g.M ? g.dq_cb[ax] : g.dp_cb[ax - g.M]; }

// Pass over axes a (and b), tiling the innermost contiguous run of length
// `run` in chunks of pc; `rest` lists the remaining axes (outer first).
QPass make_qpass(chfpe_ctx *c, int a, int b, int run, std::vector<int> rest, int pc) {
  const Derived &d = c->d;
  const Geom &g = c->g;
  QPass q{};
  q.a = a;
  q.b = b;
  q.sa_mode = a % d.M;
  q.sb_mode = b >= 0 ? b % d.M : 0;
  q.Na = axis_len(d, a);
  q.Nb = b >= 0 ? axis_len(d, b) : 1;
  q.sa = axis_stride(g, a);
  q.sb = b >= 0 ? axis_stride(g, b) : 0;
  q.run = run;
  for (int i = 0; i < 3; ++i) {
    q.rN[i] = 1;
    q.rS[i] = 0;
  }
  const int nr = (int)rest.size();
  for (int i = 0; i < nr; ++i) {  // right-align: the last rest axis goes to slot 2
    q.rN[3 - nr + i] = axis_len(d, rest[i]);
    q.rS[3 - nr + i] = axis_stride(g, rest[i]);
  }
  q.nrest = q.rN[0] * q.rN[1] * q.rN[2];
  q.pc = std::min(pc, run);
  q.nchunk = (run + q.pc - 1) / q.pc;
  // (saturates: plan() then finds the launch too large for one dispatch)
  q.ntasks = (int)std::min<long long>((long long)d.ne * q.nrest * q.nchunk, 1LL << 30);
  q.nblk = pad8(q.ntasks);
  q.ca_a = axis_ca(g, a);
  q.cb_a = axis_cb(g, a);
  q.ca_b = b >= 0 ? axis_ca(g, b) : 0.0;
  q.cb_b = b >= 0 ? axis_cb(g, b) : 0.0;
  return q;
}

// two-axis tile: Na * Nb * pc values in LDS, max(Na, Nb) * pc threads
void plan_two(chfpe_ctx *c, int a, int b, int run, std::vector<int> rest, QPass &out, int &thr,
              size_t &lds, int &nmax) {
  const Derived &d = c->d;
  const int Na = axis_len(d, a), Nb = axis_len(d, b);
  int pc = c->tune_q_pc > 0 ? c->tune_q_pc : 16;
  const size_t lds_cap = 160 * 1024;  // a whole CU's LDS: one wide tile beats two narrow ones
  while (pc > 1 && ((size_t)Na * (Nb + 1) * pc * sizeof(double) > lds_cap || std::max(Na, Nb) * pc > kQThreadsMax))
    pc /= 2;
  out = make_qpass(c, a, b, run, rest, pc);
  thr = (std::max(Na, Nb) * out.pc + 63) / 64 * 64;
  lds = (size_t)Na * (Nb + 1) * out.pc * sizeof(double);
  nmax = nmax_bucket(std::max(Na, Nb));
}

void plan_one(chfpe_ctx *c, int a, int run, std::vector<int> rest, QPass &out, int &thr, int &nmax) {
  out = make_qpass(c, a, -1, run, rest, 256);
  thr = (out.pc + 63) / 64 * 64;
  nmax = nmax_bucket(axis_len(c->d, a));
}

// LDS of a k_pcube workgroup: a copy of the task's p block, and two fields
// of one round's (p_2, p_3) planes with rows of N_3 + pad values.  The
// streamed form (k_pcube_s) keeps no copy: its planes, and the first
// forward results of every p_1 line.
size_t pcube_lds_bytes(const Derived &d, size_t tsize, int pad, bool stream) {
  const int nb1 = nmax_bucket(d.Np[0]);
  const size_t rows = (size_t)d.Np[1] * (size_t)(pcube_n3(d) + pad);
  if (stream)
    return (kPCubeCF + 2 * (size_t)pcube_s_planes(nb1) * rows +
            (size_t)pcube_s_dlds((int)tsize, nb1) * d.Np[1] * pcube_n3(d)) * tsize;
  return ((size_t)d.P + 2 * (size_t)pcube_planes(nb1) * rows + (size_t)d.Np[0]) * tsize;  // + the p_1 table
}

// Three modes take k_pcube wherever its block fits (CHFPE_PCUBE=0 keeps the
// p-block path where that one tiles); two modes take it only for p blocks
// the p-block tile cannot cover (p axes above 32 points).
bool use_pcube(const chfpe_ctx *c) {
  const Derived &d = c->d;
  if (!pcube_shape_ok(d)) return false;
  const PBShape ps = pblock_shape(d);
  const bool pblock_ok = ps.rows <= kPBlockRPT * ps.RG && ps.items(d, ps.nb_lo) <= kMaxGridItems;
  return !pblock_ok || (d.M == 3 && c->allow_pcube);
}

// Choose tile shapes.  Returns false when a k_qpass launch over every state
// of the largest batch would exceed one dispatch (the k_pblock shape always
// fits: derive() checked it).
bool plan(chfpe_ctx *c) {
  const Derived &d = c->d;
  Launch &ln = c->ln;
  const int M = d.M;
  if (d.hermite) {
    // one k_hcube launch per stage; the grid tiles below are not used
    ln.hcube = true;
    PCube &h = ln.hcb;
    h.N1 = d.Nq[0];
    h.N2 = hcube_n2(d);
    h.N3 = hcube_n3(d);
    h.plane = h.N2 * h.N3;
    h.rs = h.N3 + 1;
    h.ntasks = d.ne * d.P;
    // task order (results do not depend on it): chunks of four Hermite
    // indices' elements per XCD in turn, k_2 tiles of three (measured on the
    // 24^3 x 12^3 workload: 7% over one contiguous range per XCD)
    h.chunk = c->tune_hc_chunk >= 0 ? std::min(kMaxHcChunk, c->tune_hc_chunk) : std::min(kMaxHcChunk, 4 * d.ne);
    h.ktile = M == 3 ? std::min(c->tune_hc_ktile > 0 ? c->tune_hc_ktile : 3, d.Np[1]) : 1;
    h.nblk = hcube_nblk(h.ntasks, h.chunk);
    ln.hcube_nb1 = nmax_bucket(h.N1);
    ln.hcube_threads = (h.plane + 63) / 64 * 64;
    ln.hcube_split = h.N1 == ln.hcube_nb1 && h.N2 == h.N1 && h.N3 == h.N1;
    return true;
  }
  const int NpM = d.Np[M - 1];
  // k_pblock: the innermost one (one mode) or two p axes
  PBlock &pb = ln.pb;
  const PBShape ps = pblock_shape(d);  // derive() checked rows <= kPBlockRPT RG and nb_lo's grid
  pb.NB = ps.NB;
  pb.cols = ps.cols;
  pb.rows = ps.rows;
  pb.B = pb.rows * pb.cols;
  pb.nblocks = ps.nblocks;
  pb.bpq = d.P / pb.B;
  pb.RG = ps.RG;  // row groups divide the rows: the block of a row batch is uniform
  // lines per task ~ threads, within [nb_lo, nb_hi] (row coverage, LDS, grid)
  const int lines_per_blk = pb.rows + (pb.NB == 2 ? pb.cols : 0);
  int nb = std::max(1, (pb.RG * pb.cols) / lines_per_blk);
  if (c->tune_pb_nb > 0) nb = c->tune_pb_nb;
  nb = std::max(ps.nb_lo, std::min(nb, ps.nb_hi));
  pb.nb = nb;
  pb.split = c->tune_pb_split >= 0 ? (c->tune_pb_split != 0) : 1;
  ln.pb_nmax = nmax_bucket(std::max(pb.rows, pb.cols));
  ln.pb_rpt = (ln.pb_nmax == 24 && pb.NB == 2 && nb * pb.rows == 3 * pb.RG) ? 3 : kPBlockRPT;
  // every thread row index rg + k RG (k < RPT) has an LDS slot
  const int tile_rows = std::max(nb * pb.rows, pb.RG * ln.pb_rpt);
  pb.tileP = tile_rows * (NpM + 1);
  // task order: runs of `run` consecutive block groups of one state (longer
  // contiguous reads), the (branch, element) index next; a run that would
  // push the launch past one dispatch falls back to 1
  const int ngroups = (pb.nblocks + nb - 1) / nb;
  const long long nbat = d.batched ? d.B : 1;
  pb.run = std::max(1, std::min(c->tune_pb_run > 0 ? c->tune_pb_run : 1, ngroups));
  auto pb_tasks = [&](int run) { return (long long)d.ne * ((ngroups + run - 1) / run) * run; };
  if (grid_items(pb_tasks(pb.run) * nbat, pb.RG * pb.cols) > kMaxGridItems) pb.run = 1;
  pb.ntasks = (int)pb_tasks(pb.run);
  pb.nblk = pad8(pb.ntasks);
  ln.pb_lds = (size_t)pb.NB * pb.tileP * sizeof(double);
  ln.pb_threads = pb.RG * pb.cols;
  // strided-axis passes
  if (M == 1) {
    ln.has_qa = false;
    ln.qf_two = false;
    plan_one(c, 0, d.P, {}, ln.qf, ln.qf_threads, ln.qf_nmax);
    ln.qf_lds = 0;
    ln.has_qx = false;
  } else if (use_pcube(c)) {
    // all p axes per q point (k_pcube); three modes then take (q_2, q_3)
    // over whole p-blocks and q_1 alone (lines in registers) with the stage
    // update, two modes (q_1, q_2)
    ln.pcube = true;
    PCube &pq = ln.pcb;
    pq.N1 = d.Np[0];
    pq.N2 = d.Np[1];
    pq.N3 = pcube_n3(d);
    pq.plane = pq.N2 * pq.N3;
    pq.ntasks = (int)std::min<long long>((long long)d.ne * d.Q, 1LL << 30);
    pq.nblk = pad8(pq.ntasks);
    ln.pcube_nb1 = nmax_bucket(pq.N1);
    ln.pcube_threads = (pq.plane + 63) / 64 * 64;
    // row pad of the LDS planes (CHFPE_TUNE_PC_PAD, 1..8), kept only while the LDS fits
    // the streamed form where its workgroups gain occupancy (p_1 up to 16
    // points: four-wave workgroups); CHFPE_TUNE_PC_STREAM=0/1 forces either
    ln.pcube_stream = c->tune_pc_stream >= 0 ? (c->tune_pc_stream > 0 && nmax_bucket(d.Np[0]) <= 32)
                                             : nmax_bucket(d.Np[0]) <= 16;
    pq.rs = pq.N3 + 1;
    if (!ln.pcube_stream && c->tune_pc_pad > 1 && pcube_lds_bytes(d, sizeof(double), c->tune_pc_pad, false) <= 160 * 1024)
      pq.rs = pq.N3 + c->tune_pc_pad;
    ln.pcube_lds = pcube_lds_bytes(d, sizeof(double), pq.rs - pq.N3, ln.pcube_stream);
    ln.pcube_split = pq.N1 == ln.pcube_nb1 && pq.N2 == pq.N1 && pq.N3 == pq.N1 && c->tune_pb_split != 0;
    pb.nb = 1;  // k_pblock is not launched: one shape for the autotuner
    pb.split = ln.pcube_split ? 1 : 0;
    pb.run = 1;
    ln.has_qx = false;
    if (M == 3) {
      ln.has_qa = true;
      plan_two(c, 1, 2, d.P, {0}, ln.qa, ln.qa_threads, ln.qa_lds, ln.qa_nmax);
      ln.qf_two = false;
      plan_one(c, 0, (d.Q / d.Nq[0]) * d.P, {}, ln.qf, ln.qf_threads, ln.qf_nmax);
      ln.qf_lds = 0;
    } else {
      ln.has_qa = false;
      ln.qf_two = true;
      plan_two(c, 0, 1, d.P, {}, ln.qf, ln.qf_threads, ln.qf_lds, ln.qf_nmax);
    }
  } else if (M == 2) {
    ln.has_qa = false;
    ln.qf_two = true;
    plan_two(c, 0, 1, d.P, {}, ln.qf, ln.qf_threads, ln.qf_lds, ln.qf_nmax);
    ln.has_qx = false;
  } else {
    // (q_2, q_3) over whole p-blocks, then (q_1, p_1) over (p_2, p_3) planes
    const int plane = d.Np[1] * d.Np[2];
    ln.has_qa = true;
    plan_two(c, 1, 2, d.P, {0}, ln.qa, ln.qa_threads, ln.qa_lds, ln.qa_nmax);
    ln.qf_two = true;
    plan_two(c, 0, M + 0, plane, {1, 2}, ln.qf, ln.qf_threads, ln.qf_lds, ln.qf_nmax);
    ln.has_qx = true;
    plan_one(c, M + 0, plane, {0, 1, 2}, ln.qx, ln.qx_threads, ln.qx_nmax);
  }
  auto fits = [&](const QPass &q, int thr) { return grid_items((long long)q.ntasks * nbat, thr) <= kMaxGridItems; };
  return fits(ln.qf, ln.qf_threads) && (!ln.has_qa || fits(ln.qa, ln.qa_threads)) &&
         (!ln.has_qx || fits(ln.qx, ln.qx_threads)) &&
         (!ln.pcube || grid_items((long long)ln.pcb.ntasks * nbat, ln.pcube_threads) <= kMaxGridItems);
}

// --------------------------------------------------------------------------
// kernel launch helpers (template dispatch on NMAX)
// --------------------------------------------------------------------------

hipEvent_t get_event(chfpe_ctx *c) {
  if (!c->event_pool.empty()) {
    hipEvent_t e = c->event_pool.back();
    c->event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

int drain_timing(chfpe_ctx *c) {
  if (c->pending.empty()) return CHFPE_OK;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  for (auto &pd : c->pending) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, pd.a, pd.b) == hipSuccess) {
      c->kcount[pd.kind] += 1;
      c->ktime[pd.kind] += ms;
      c->kbytes[pd.kind] += pd.bytes;
    }
    c->event_pool.push_back(pd.a);
    c->event_pool.push_back(pd.b);
  }
  c->pending.clear();
  return CHFPE_OK;
}

// Brackets one launch with events when the current RK4 step is timed.
// nstates x state_bytes is the state data the launch's kind touches per pass
// (the observe kind reads element 0 only, accounted by its pass factor).
struct TimedScope {
  chfpe_ctx *c;
  int kind;
  double bytes;
  hipEvent_t a = nullptr;
  TimedScope(chfpe_ctx *c_, int k, int nstates = 1, size_t tsize = sizeof(double))
      : c(c_), kind(k + (nstates > 1 ? kNumBase : 0)),
        bytes(kKindPasses[k] * (double)nstates * (double)c_->d.S * (double)tsize) {
    if (c->timing_now && !c->capturing) {
      a = get_event(c);
      if (a) (void)hipEventRecord(a, c->stream);
    }
  }
  ~TimedScope() {
    if (a) {
      hipEvent_t b = get_event(c);
      if (b) {
        (void)hipEventRecord(b, c->stream);
        c->pending.push_back({a, b, kind, bytes});
      } else {
        c->event_pool.push_back(a);
      }
    }
  }
};

template <typename K>
void allow_lds(K kern, size_t bytes) {
  if (bytes > 64 * 1024)
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

// A launch description for nb states stored back to back (t1 branches).
struct Batch {
  Geom g;
  PBlock pb;
  PCube pcb, hcb;
  QPass qa, qf, qx;
};

Batch batch_of(const chfpe_ctx *c, int nb) {
  Batch b;
  b.g = c->g;
  b.g.nbatch = nb;
  b.pb = c->ln.pb;
  b.pb.ntasks *= nb;
  b.pb.nblk = pad8(b.pb.ntasks);
  b.pcb = c->ln.pcb;
  b.pcb.ntasks *= nb;
  b.pcb.nblk = pad8(b.pcb.ntasks);
  b.hcb = c->ln.hcb;
  b.hcb.ntasks *= nb;
  b.hcb.nblk = hcube_nblk(b.hcb.ntasks, b.hcb.chunk);
  QPass *q[3] = {&b.qa, &b.qf, &b.qx};
  const QPass *s[3] = {&c->ln.qa, &c->ln.qf, &c->ln.qx};
  for (int i = 0; i < 3; ++i) {
    *q[i] = *s[i];
    q[i]->ntasks *= nb;
    q[i]->nblk = pad8(q[i]->ntasks);
  }
  return b;
}

// Closure variants of the kernels exist for FP64 states with every axis in a
// bucket of at most 16 points (chfpe_set_closure enforces this).
template <typename T, typename TO, int NMAX>
constexpr bool kClosureBuilt = std::is_same<T, double>::value && std::is_same<TO, double>::value && NMAX <= 16;

template <typename T, typename TO, int NMAX, int RPT, int MM, bool PERTURB>
void launch_pblock_rpt(chfpe_ctx *c, const Batch &b, const T *X, TO *out, const double *grad) {
  const Launch &ln = c->ln;
  if constexpr (kClosureBuilt<T, TO, NMAX>) {
    if (c->closure_on) {
      auto kern = k_pblock<T, TO, NMAX, RPT, MM, PERTURB, true>;
      allow_lds(kern, ln.pb_lds);
      hipLaunchKernelGGL(kern, dim3(b.pb.nblk), dim3(ln.pb_threads), ln.pb_lds, c->stream, b.g, c->tb, b.pb,
                         X, out, grad);
      return;
    }
  }
  auto kern = k_pblock<T, TO, NMAX, RPT, MM, PERTURB>;
  allow_lds(kern, ln.pb_lds);
  hipLaunchKernelGGL(kern, dim3(b.pb.nblk), dim3(ln.pb_threads), ln.pb_lds, c->stream, b.g, c->tb, b.pb, X,
                     out, grad);
}

template <typename T, typename TO, int NMAX, int MM, bool PERTURB>
void launch_pblock_nm(chfpe_ctx *c, const Batch &b, const T *X, TO *out, const double *grad) {
  if constexpr (NMAX == 24 && MM >= 2) {
    if (c->ln.pb_rpt == 3) {
      launch_pblock_rpt<T, TO, NMAX, 3, MM, PERTURB>(c, b, X, out, grad);
      return;
    }
  }
  launch_pblock_rpt<T, TO, NMAX, kPBlockRPT, MM, PERTURB>(c, b, X, out, grad);
}

template <typename T, typename TO, int NMAX, bool PERTURB>
void launch_pblock_n(chfpe_ctx *c, const Batch &b, const T *X, TO *out, const double *grad) {
  switch (c->d.M) {
    case 1: launch_pblock_nm<T, TO, NMAX, 1, PERTURB>(c, b, X, out, grad); break;
    case 2: launch_pblock_nm<T, TO, NMAX, 2, PERTURB>(c, b, X, out, grad); break;
    default: launch_pblock_nm<T, TO, NMAX, 3, PERTURB>(c, b, X, out, grad); break;
  }
}

template <typename T, typename TO, bool PERTURB>
void launch_pblock_t(chfpe_ctx *c, const Batch &b, const T *X, TO *out, const double *grad) {
  switch (c->ln.pb_nmax) {
    case 8: launch_pblock_n<T, TO, 8, PERTURB>(c, b, X, out, grad); break;
    case 12: launch_pblock_n<T, TO, 12, PERTURB>(c, b, X, out, grad); break;
    case 16: launch_pblock_n<T, TO, 16, PERTURB>(c, b, X, out, grad); break;
    case 24: launch_pblock_n<T, TO, 24, PERTURB>(c, b, X, out, grad); break;
    case 32: launch_pblock_n<T, TO, 32, PERTURB>(c, b, X, out, grad); break;
    default: launch_pblock_n<T, TO, 48, PERTURB>(c, b, X, out, grad); break;
  }
}

template <typename K, typename T, typename TO>
void launch_pcube_k(chfpe_ctx *c, K kern, size_t lds, const Batch &b, const T *X, TO *out, const double *grad) {
  allow_lds(kern, lds);
  hipLaunchKernelGGL(kern, dim3(b.pcb.nblk), dim3(c->ln.pcube_threads), lds, c->stream, b.g, c->tb, b.pcb,
                     X, out, grad);
}

// k_pcube, or its streamed form k_pcube_s where the plan chose it (p_1 axes
// up to 32 points, plain stencils; closure tables take k_pcube)
template <typename T, typename TO, int NB1, bool SPLIT, bool PERTURB>
void launch_pcube_s(chfpe_ctx *c, const Batch &b, const T *X, TO *out, const double *grad) {
  const int pad = b.pcb.rs - b.pcb.N3;
  if constexpr (kClosureBuilt<T, TO, NB1>) {
    if (c->closure_on) {
      launch_pcube_k(c, k_pcube<T, TO, NB1, SPLIT, PERTURB, true>, pcube_lds_bytes(c->d, sizeof(T), pad, false),
                     b, X, out, grad);
      return;
    }
  }
  if constexpr (NB1 <= 32) {
    if (c->ln.pcube_stream) {
      launch_pcube_k(c, k_pcube_s<T, TO, NB1, SPLIT, PERTURB>, pcube_lds_bytes(c->d, sizeof(T), pad, true), b, X,
                     out, grad);
      return;
    }
  }
  launch_pcube_k(c, k_pcube<T, TO, NB1, SPLIT, PERTURB>, pcube_lds_bytes(c->d, sizeof(T), pad, false), b, X, out,
                 grad);
}

template <typename T, typename TO, int NB1, bool PERTURB>
void launch_pcube_n(chfpe_ctx *c, const Batch &b, const T *X, TO *out, const double *grad) {
  if (c->ln.pcube_split)
    launch_pcube_s<T, TO, NB1, true, PERTURB>(c, b, X, out, grad);
  else
    launch_pcube_s<T, TO, NB1, false, PERTURB>(c, b, X, out, grad);
}

template <typename T, typename TO, bool PERTURB>
void launch_pcube_t(chfpe_ctx *c, const Batch &b, const T *X, TO *out, const double *grad) {
  switch (c->ln.pcube_nb1) {
    case 8: launch_pcube_n<T, TO, 8, PERTURB>(c, b, X, out, grad); break;
    case 12: launch_pcube_n<T, TO, 12, PERTURB>(c, b, X, out, grad); break;
    case 16: launch_pcube_n<T, TO, 16, PERTURB>(c, b, X, out, grad); break;
    case 24: launch_pcube_n<T, TO, 24, PERTURB>(c, b, X, out, grad); break;
    case 32: launch_pcube_n<T, TO, 32, PERTURB>(c, b, X, out, grad); break;
    default: launch_pcube_n<T, TO, 48, PERTURB>(c, b, X, out, grad); break;
  }
}

template <typename T, typename TO, int NMAX, bool TWO, int EPI, int FA, int FB>
void launch_q_n(chfpe_ctx *c, const Batch &b, const QPass &qp, int threads, size_t lds, const T *X, TO *Tacc,
                const TO *y, TO *xo, const double *grad, double cst) {
  if constexpr (kClosureBuilt<T, TO, NMAX>) {
    if (c->closure_on) {
      auto kern = k_qpass<T, TO, NMAX, TWO, EPI, FA, FB, true>;
      allow_lds(kern, lds);
      hipLaunchKernelGGL(kern, dim3(qp.nblk), dim3(threads), lds, c->stream, b.g, c->tb, qp, X, Tacc, y, xo,
                         grad, cst);
      return;
    }
  }
  auto kern = k_qpass<T, TO, NMAX, TWO, EPI, FA, FB>;
  allow_lds(kern, lds);
  hipLaunchKernelGGL(kern, dim3(qp.nblk), dim3(threads), lds, c->stream, b.g, c->tb, qp, X, Tacc, y, xo, grad,
                     cst);
}

template <typename T, typename TO, bool TWO, int EPI, int FA, int FB>
void launch_q_t(chfpe_ctx *c, const Batch &b, const QPass &qp, int threads, size_t lds, int nmax, const T *X,
                TO *Tacc, const TO *y, TO *xo, const double *grad, double cst) {
#define CHFPE_QN(N) launch_q_n<T, TO, N, TWO, EPI, FA, FB>(c, b, qp, threads, lds, X, Tacc, y, xo, grad, cst)
  switch (nmax) {
    case 8: CHFPE_QN(8); break;
    case 12: CHFPE_QN(12); break;
    case 16: CHFPE_QN(16); break;
    case 24: CHFPE_QN(24); break;
    case 32: CHFPE_QN(32); break;
    default: CHFPE_QN(48); break;
  }
#undef CHFPE_QN
}

// Hermite basis: one k_hcube launch computes the right-hand side of X and
// the stage update (EPI, coefficient cst) over every (branch, element, k).
template <typename T, int NB1, bool SPLIT, int EPI>
void launch_hcube_k(chfpe_ctx *c, const Batch &b, const T *X, const T *y, T *xo, double cst) {
  const size_t lds = (kHCubeCF + 2 * (size_t)kHCubePL * b.hcb.N2 * b.hcb.rs) * sizeof(T);
  auto kern = k_hcube<T, NB1, SPLIT, EPI>;
  allow_lds(kern, lds);
  hipLaunchKernelGGL(kern, dim3(b.hcb.nblk), dim3(c->ln.hcube_threads), lds, c->stream, b.g, c->tb, b.hcb, X, y,
                     xo, cst);
}

template <typename T, int NB1, int EPI>
void launch_hcube_n(chfpe_ctx *c, const Batch &b, const T *X, const T *y, T *xo, double cst) {
  if constexpr (NB1 <= 24) {  // cubes of 32 or 48 points exceed the workgroup: never lane pairs
    if (c->ln.hcube_split) {
      launch_hcube_k<T, NB1, true, EPI>(c, b, X, y, xo, cst);
      return;
    }
  }
  launch_hcube_k<T, NB1, false, EPI>(c, b, X, y, xo, cst);
}

template <typename T, int EPI>
void launch_hcube(chfpe_ctx *c, const Batch &b, const T *X, const T *y, T *xo, double cst) {
  switch (c->ln.hcube_nb1) {
    case 8: launch_hcube_n<T, 8, EPI>(c, b, X, y, xo, cst); break;
    case 12: launch_hcube_n<T, 12, EPI>(c, b, X, y, xo, cst); break;
    case 16: launch_hcube_n<T, 16, EPI>(c, b, X, y, xo, cst); break;
    case 24: launch_hcube_n<T, 24, EPI>(c, b, X, y, xo, cst); break;
    case 32: launch_hcube_n<T, 32, EPI>(c, b, X, y, xo, cst); break;
    default: launch_hcube_n<T, 48, EPI>(c, b, X, y, xo, cst); break;
  }
}

// One right-hand-side evaluation of X (t: partial right-hand side) fused with
// the stage epilogue EPI (coefficient cst); all buffers hold b.g.nbatch
// states.  kind: the timing kind of the stage-final launch.
template <typename T, int EPI>
void launch_stage(chfpe_ctx *c, const Batch &b, const T *X, T *t, const T *y, T *xo, double cst, int kind) {
  const Launch &ln = c->ln;
  if (ln.hcube) {  // Hermite basis: the whole stage in one launch
    const int hk = EPI == EPI_H1 ? K_HS1 : EPI == EPI_H4 ? K_HS4 : EPI == EPI_OUT ? K_HOUT
                   : kind == K_QS3 ? K_HS3 : K_HS2;
    TimedScope ts(c, hk, b.g.nbatch, sizeof(T));
    launch_hcube<T, EPI>(c, b, X, y, xo, cst);
    return;
  }
  if (ln.pcube) {
    TimedScope ts(c, K_PCUBE, b.g.nbatch, sizeof(T));
    launch_pcube_t<T, T, false>(c, b, X, t, nullptr);
  } else {
    TimedScope ts(c, K_PBLOCK, b.g.nbatch, sizeof(T));
    launch_pblock_t<T, T, false>(c, b, X, t, nullptr);
  }
  if (ln.has_qa) {
    TimedScope ts(c, K_QACC, b.g.nbatch, sizeof(T));
    launch_q_t<T, T, true, EPI_ACC, FQ, FQ>(c, b, b.qa, ln.qa_threads, ln.qa_lds, ln.qa_nmax, X, t, nullptr,
                                            nullptr, nullptr, 0.0);
  }
  TimedScope ts(c, kind, b.g.nbatch, sizeof(T));
  if (!ln.qf_two)  // one mode, or q_1 after k_pcube
    launch_q_t<T, T, false, EPI, FQ, FQ>(c, b, b.qf, ln.qf_threads, 0, ln.qf_nmax, X, t, y, xo, nullptr, cst);
  else if (c->d.M == 2)
    launch_q_t<T, T, true, EPI, FQ, FQ>(c, b, b.qf, ln.qf_threads, ln.qf_lds, ln.qf_nmax, X, t, y, xo, nullptr,
                                        cst);
  else
    launch_q_t<T, T, true, EPI, FQ, FP>(c, b, b.qf, ln.qf_threads, ln.qf_lds, ln.qf_nmax, X, t, y, xo, nullptr,
                                        cst);
}

// out = X^x W for every element of one state, arithmetic in FP64
// (grad: dX/dq_s table); out may be FP64 or the propagation type.
template <typename TO>
void launch_perturb(chfpe_ctx *c, const double *W, TO *out, const double *grad) {
  TimedScope ts(c, K_PERTURB);
  const Batch b = batch_of(c, 1);
  if (c->ln.hcube) {  // Hermite basis: a local raising of k, no derivative
    hipLaunchKernelGGL((k_hperturb<TO>), dim3(2048), dim3(256), 0, c->stream, b.g, W, out, grad);
    return;
  }
  if (c->ln.pcube) {
    launch_pcube_t<double, TO, true>(c, b, W, out, grad);
    return;
  }
  launch_pblock_t<double, TO, true>(c, b, W, out, grad);
  if (c->ln.has_qx)
    launch_q_t<double, TO, false, EPI_ACC, FX, FQ>(c, b, b.qx, c->ln.qx_threads, 0, c->ln.qx_nmax, W, out,
                                                   nullptr, nullptr, grad, 0.0);
}

int last_launch_error(chfpe_ctx *c) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(c, CHFPE_EDEVICE, std::string("kernel launch: ") + hipGetErrorString(e));
  return CHFPE_OK;
}

// The buffers of one RK4 integration: y (in place), the alternating stage
// states xa/xb, and the partial right-hand side t.
template <typename T>
struct RK4Bufs {
  T *y, *xa, *xb, *t;
};

// n RK4 steps on b.g.nbatch states (in place), each the degree-4 Taylor
// polynomial of dt L in nested form (see Epi in kernels.h).
template <typename T>
int rk4(chfpe_ctx *c, const Batch &b, const RK4Bufs<T> &r, long long nsteps, double dt) {
  for (long long st = 0; st < nsteps; ++st) {
    c->timing_now = c->timing_every > 0 && (c->step_counter % c->timing_every) == 0;
    ++c->step_counter;
    // xa = y + dt/4 L y
    launch_stage<T, EPI_H1>(c, b, r.y, r.t, nullptr, r.xa, 0.25 * dt, K_QS1);
    // xb = y + dt/3 L xa
    launch_stage<T, EPI_H2>(c, b, r.xa, r.t, r.y, r.xb, dt / 3.0, K_QS2);
    // xa = y + dt/2 L xb
    launch_stage<T, EPI_H2>(c, b, r.xb, r.t, r.y, r.xa, 0.5 * dt, K_QS3);
    // y = y + dt L xa
    launch_stage<T, EPI_H4>(c, b, r.xa, r.t, nullptr, r.y, dt, K_QS4);
    if (c->timing_now) {
      c->timing_now = false;
      if (c->pending.size() > 4096) {
        int rc = drain_timing(c);
        if (rc) return rc;
      }
    }
  }
  return last_launch_error(c);
}

// FP64 single-state integration on buffer yb
int rk4(chfpe_ctx *c, double *yb, long long nsteps, double dt) {
  const Batch b = batch_of(c, 1);
  return rk4<double>(c, b, RK4Bufs<double>{yb, c->xa, c->xb, c->t}, nsteps, dt);
}

// dst[b * dstride] = <C>(state b of W), b < nb (Cw holds the C table)
template <typename T>
void observe_batch(chfpe_ctx *c, const T *W, int nb, double *dst, int dstride) {
  TimedScope ts(c, K_OBSERVE, nb, sizeof(T));
  // element 0 of the grid basis: every (q, p); Hermite basis: the k = 0 slice,
  // the first Q values (p integrated exactly)
  const int P = c->d.hermite ? 1 : c->d.P;
  const int per = std::max(1, std::min(kPartials / nb, (int)(((long long)c->d.Q * P + 255) / 256)));
  hipLaunchKernelGGL((k_reduce_w0<T>), dim3(per, nb), dim3(256), 0, c->stream, W, c->Cw, c->wp, c->d.Q, P,
                     c->partial, (long long)c->d.S);
  hipLaunchKernelGGL(k_reduce_final, dim3(nb), dim3(256), 0, c->stream, c->partial, per, c->dV, dst, dstride);
}

int observe_to(chfpe_ctx *c, const double *W, double *dst) {
  observe_batch<double>(c, W, 1, dst, 1);
  return CHFPE_OK;
}

// The t2 loop of one wave: nb branch states in the batched buffers, each
// observed after every s2 steps; Rw[j2 * B + b] receives <C> of branch b.
template <typename T>
int enqueue_wave(chfpe_ctx *c, int nb, long long n_t2, int s2, double dt, double *Rw) {
  const Batch b = batch_of(c, nb);
  const RK4Bufs<T> r{(T *)c->bb[0], (T *)c->bb[1], (T *)c->bb[2], (T *)c->bb[3]};
  for (long long j2 = 0; j2 < n_t2; ++j2) {
    if (j2 > 0) {
      int rc = rk4<T>(c, b, r, s2, dt);
      if (rc) return rc;
    }
    observe_batch<T>(c, r.y, nb, Rw + j2 * c->d.B, 1);
  }
  return CHFPE_OK;
}

// Run one wave, as a captured HIP graph when possible.  The executable graph
// is kept for the next wave of the same shape (same buffers, nb, n_t2, s2,
// dt); without a stream of its own, or while kernel timing is on, the wave
// is enqueued directly.
template <typename T>
int run_wave(chfpe_ctx *c, int nb, long long n_t2, int s2, double dt, double *Rw) {
  if (!c->use_graphs || c->stream == nullptr || c->timing_every > 0)
    return enqueue_wave<T>(c, nb, n_t2, s2, dt, Rw);
  long long dtbits;
  std::memcpy(&dtbits, &dt, sizeof dtbits);
  const long long key[6] = {nb, n_t2, s2, dtbits, (long long)(uintptr_t)Rw, (long long)sizeof(T)};
  if (!c->wave_graph || std::memcmp(key, c->wave_key, sizeof key) != 0) {
    if (c->wave_graph) {
      HIPCHK(c, hipGraphExecDestroy(c->wave_graph));
      c->wave_graph = nullptr;
    }
    HIPCHK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    c->capturing = true;
    int rc = enqueue_wave<T>(c, nb, n_t2, s2, dt, Rw);
    c->capturing = false;
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(c->stream, &graph);
    if (rc) {
      if (graph) (void)hipGraphDestroy(graph);
      return rc;
    }
    if (e != hipSuccess) return fail(c, CHFPE_EDEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    e = hipGraphInstantiate(&c->wave_graph, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
      c->wave_graph = nullptr;
      return fail(c, CHFPE_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    }
    std::memcpy(c->wave_key, key, sizeof key);
  }
  HIPCHK(c, hipGraphLaunch(c->wave_graph, c->stream));
  return CHFPE_OK;
}

// All t1 branches in waves of B: U (FP64, buffer u) is advanced along t1 one
// branch start at a time; V_j1 = B^x U (FP64 arithmetic, stored in the branch
// type T) fills the wave's slots; the wave then runs its t2 loop.
template <typename T>
int branches_batched(chfpe_ctx *c, long long n_t1, long long n_t2, int s1, int s2, double dt) {
  const int B = c->d.B;
  double *Rw = c->rbuf + n_t1 * n_t2;
  long long cur = 0;
  for (long long j0 = 0; j0 < n_t1; j0 += B) {
    const int nb = (int)std::min<long long>(B, n_t1 - j0);
    for (int b = 0; b < nb; ++b) {
      const long long tgt = (j0 + b) * s1;
      if (tgt > cur) {
        int rc = rk4(c, c->u, tgt - cur, dt);
        if (rc) return rc;
        cur = tgt;
      }
      launch_perturb<T>(c, c->u, (T *)c->bb[0] + (size_t)b * c->d.S, c->gB);
    }
    int rc = run_wave<T>(c, nb, n_t2, s2, dt, Rw);
    if (rc) return rc;
    const int nthr = (int)(n_t2 * nb);
    hipLaunchKernelGGL(k_scatter_r, dim3((nthr + 255) / 256), dim3(256), 0, c->stream, Rw, c->rbuf, (int)n_t2,
                       B, nb, (int)n_t1, (int)j0);
  }
  return last_launch_error(c);
}

// upload grad tables (dX/dq_s on the q grid) for an optical operator
void grad_table(chfpe_ctx *c, const chfpe_optical *X, std::vector<double> &out) {
  const Derived &d = c->d;
  out.assign(3 * d.Q, 0.0);
  for (int ql = 0; ql < d.Q; ++ql) {
    double q[3] = {0, 0, 0};
    int rem = ql;
    for (int s = d.M - 1; s >= 0; --s) {
      q[s] = c->qgrid[s][rem % d.Nq[s]];
      rem /= d.Nq[s];
    }
    for (int s = 0; s < d.M; ++s) {
      double gv = X->lin[s];
      for (int t = 0; t < d.M; ++t) gv += 0.5 * (X->quad[s][t] + X->quad[t][s]) * q[t];
      out[s * d.Q + ql] = gv;
    }
  }
}

void value_table(chfpe_ctx *c, const chfpe_optical *X, std::vector<double> &out) {
  const Derived &d = c->d;
  out.assign(d.Q, 0.0);
  for (int ql = 0; ql < d.Q; ++ql) {
    double q[3] = {0, 0, 0};
    int rem = ql;
    for (int s = d.M - 1; s >= 0; --s) {
      q[s] = c->qgrid[s][rem % d.Nq[s]];
      rem /= d.Nq[s];
    }
    double v = 0.0;
    for (int s = 0; s < d.M; ++s) {
      v += X->lin[s] * q[s];
      for (int t = 0; t < d.M; ++t) v += 0.5 * X->quad[s][t] * q[s] * q[t];
    }
    out[ql] = v * c->wq_host[ql] * c->sq_host[ql];
  }
}

bool optical_ok(const chfpe_optical *X, int M) {
  if (!X) return false;
  for (int s = 0; s < M; ++s) {
    if (!std::isfinite(X->lin[s])) return false;
    for (int t = 0; t < M; ++t)
      if (!std::isfinite(X->quad[s][t])) return false;
  }
  return true;
}

int check_finite(chfpe_ctx *c, const double *W) {
  HIPCHK(c, hipMemsetAsync(c->flag, 0, sizeof(int), c->stream));
  hipLaunchKernelGGL((k_check_finite<double>), dim3(1024), dim3(256), 0, c->stream, W, c->d.S, c->flag);
  int h = 0;
  HIPCHK(c, hipMemcpyAsync(&h, c->flag, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (h) return fail(c, CHFPE_ENONFINITE, "state became non-finite (dt above the RK4 stability limit?)");
  return CHFPE_OK;
}

// Milliseconds per RK4 step of the path the context spends most time in:
// the batched branch buffers (branch type) when 2D responses are batched,
// else the FP64 single-state buffers with u as the state.  One untimed step
// first; returns < 0 on a launch or runtime error (message in c->err).
template <typename T>
double time_batched(chfpe_ctx *c, int n_steps, double dt) {
  const Batch b = batch_of(c, c->d.B);
  const RK4Bufs<T> r{(T *)c->bb[0], (T *)c->bb[1], (T *)c->bb[2], (T *)c->bb[3]};
  if (rk4<T>(c, b, r, 1, dt)) return -1.0;
  hipEvent_t e0 = get_event(c), e1 = get_event(c);
  if (!e0 || !e1) return -1.0;
  (void)hipEventRecord(e0, c->stream);
  const int rc = rk4<T>(c, b, r, n_steps, dt);
  (void)hipEventRecord(e1, c->stream);
  float ms = -1.f;
  if (rc == CHFPE_OK && hipEventSynchronize(e1) == hipSuccess) (void)hipEventElapsedTime(&ms, e0, e1);
  c->event_pool.push_back(e0);
  c->event_pool.push_back(e1);
  return rc ? -1.0 : (double)ms / n_steps;
}

double time_rk4_step(chfpe_ctx *c, int n_steps, double dt) {
  if (c->d.batched)
    return c->d.prec == CHFPE_FP32 ? time_batched<float>(c, n_steps, dt) : time_batched<double>(c, n_steps, dt);
  if (rk4(c, c->u, 1, dt)) return -1.0;
  hipEvent_t e0 = get_event(c), e1 = get_event(c);
  if (!e0 || !e1) return -1.0;
  (void)hipEventRecord(e0, c->stream);
  const int rc = rk4(c, c->u, n_steps, dt);
  (void)hipEventRecord(e1, c->stream);
  float ms = -1.f;
  if (rc == CHFPE_OK && hipEventSynchronize(e1) == hipSuccess) (void)hipEventElapsedTime(&ms, e0, e1);
  c->event_pool.push_back(e0);
  c->event_pool.push_back(e1);
  return rc ? -1.0 : (double)ms / n_steps;
}

int ensure_rbuf(chfpe_ctx *c, size_t n) {
  if (n <= c->rbuf_cap) return CHFPE_OK;
  if (c->rbuf) {
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipFree(c->rbuf));
    c->rbuf = nullptr;
    c->rbuf_cap = 0;
  }
  HIPCHK(c, hipMalloc(&c->rbuf, n * sizeof(double)));
  c->rbuf_cap = n;
  return CHFPE_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// closure helpers (host)
// ---------------------------------------------------------------------------
// Axis ids 0..M-1 are q_s, M..2M-1 are p_s; lengths and spacings per id.
void axis_table(const chfpe_params *p, int M, int *N, double *h, double *L) {
  for (int a = 0; a < 2 * M; ++a) {
    const int s = a % M;
    N[a] = a < M ? p->Nq[s] : p->Np[s];
    L[a] = a < M ? p->Lq[s] : p->Lp[s];
    h[a] = 2.0 * L[a] / N[a];
  }
}

// Lines along axis a of a state [element][axis 0..2M-1] with lengths N.
AxisLines axis_lines(const int *N, int nd, int a, long long ne) {
  AxisLines al{};
  long long stride = 1, E = 1;
  for (int d = nd - 1; d >= 0; --d) {
    if (d == a) al.inner = stride;
    stride *= N[d];
  }
  E = stride;
  al.N = N[a];
  al.E = E;
  al.outer = E / (al.inner * N[a]);
  al.nlines = ne * al.inner * al.outer;
  return al;
}

// A^{-1} and A^{-T} A^{-1} of the N x N matrix tridiag(1/3, 1, 1/3) (FP64,
// Gauss-Jordan on the small dense matrix).
void compact_inverse(int N, std::vector<double> &Ai, std::vector<double> &K) {
  std::vector<double> A(N * N, 0.0);
  Ai.assign(N * N, 0.0);
  for (int i = 0; i < N; ++i) {
    A[i * N + i] = 1.0;
    if (i > 0) A[i * N + i - 1] = 1.0 / 3.0;
    if (i + 1 < N) A[i * N + i + 1] = 1.0 / 3.0;
    Ai[i * N + i] = 1.0;
  }
  for (int col = 0; col < N; ++col) {  // diagonally dominant: no pivoting needed
    const double piv = A[col * N + col];
    for (int j = 0; j < N; ++j) {
      A[col * N + j] /= piv;
      Ai[col * N + j] /= piv;
    }
    for (int r = 0; r < N; ++r) {
      if (r == col) continue;
      const double f = A[r * N + col];
      if (f == 0.0) continue;
      for (int j = 0; j < N; ++j) {
        A[r * N + j] -= f * A[col * N + j];
        Ai[r * N + j] -= f * Ai[col * N + j];
      }
    }
  }
  K.assign(N * N, 0.0);
  for (int a = 0; a < N; ++a)
    for (int b = 0; b < N; ++b) {
      double v = 0.0;
      for (int n = 0; n < N; ++n) v += Ai[n * N + a] * Ai[n * N + b];
      K[a * N + b] = v;
    }
}

int nmax_of(int n) { return nmax_bucket(n); }

void launch_axis_deriv(hipStream_t st, const double *X, double *Y, const double *Yadd, double alpha,
                       const AxisLines &al, double h) {
  const double ca = 7.0 / 9.0 / h, cb = 1.0 / 36.0 / h;
  const dim3 grid((unsigned)((al.nlines + 255) / 256));
  switch (nmax_of(al.N)) {
    case 8: hipLaunchKernelGGL(k_axis_deriv<8>, grid, dim3(256), 0, st, X, Y, Yadd, alpha, al, ca, cb); break;
    case 12: hipLaunchKernelGGL(k_axis_deriv<12>, grid, dim3(256), 0, st, X, Y, Yadd, alpha, al, ca, cb); break;
    case 16: hipLaunchKernelGGL(k_axis_deriv<16>, grid, dim3(256), 0, st, X, Y, Yadd, alpha, al, ca, cb); break;
    case 24: hipLaunchKernelGGL(k_axis_deriv<24>, grid, dim3(256), 0, st, X, Y, Yadd, alpha, al, ca, cb); break;
    default: hipLaunchKernelGGL(k_axis_deriv<32>, grid, dim3(256), 0, st, X, Y, Yadd, alpha, al, ca, cb); break;
  }
}

// Device scratch owned by one closure call (freed on every exit path).
struct DevScratch {
  std::vector<void *> ptrs;
  ~DevScratch() {
    for (void *q : ptrs) (void)hipFree(q);
  }
  template <typename X>
  X *get(size_t n) {
    void *q = nullptr;
    if (hipMalloc(&q, std::max<size_t>(n, 1) * sizeof(X)) != hipSuccess) return nullptr;
    ptrs.push_back(q);
    return static_cast<X *>(q);
  }
};

// Rows of the closure network for a coarse problem: one per (axis, skew
// entry), axes in id order, entries S[i][i+k] for k = 1 .. kClosBands
// (i < N - k).
int closure_rows(const chfpe_params *p) {
  int n = 0;
  for (int a = 0; a < 2 * p->M; ++a) n += skew_entries(a < p->M ? p->Nq[a % p->M] : p->Np[a % p->M]);
  return n;
}

int fail_g(int code, const std::string &msg) { return fail(nullptr, code, msg); }

// ===========================================================================
// C ABI
// ===========================================================================

// ---------------------------------------------------------------------------
// Device scratch of chfpe_spectrum_2d_noalloc: a file-scope array, one copy
// per device, that holds R, two complex work arrays and I of one spectrum
// of at most kNoAllocMaxPoints points (48 bytes per point, 6 MiB).  Host
// code never passes the array's name to a kernel or copy: it takes the
// device address of each GPU's copy once (hipGetSymbolAddress, with that
// device current) and uses that address.
// ---------------------------------------------------------------------------
constexpr long long kNoAllocMaxPoints = 1LL << 17;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[48 * kNoAllocMaxPoints];

namespace {
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Address of the current device's scratch (resolved on first use per device).
int scratch_of_current_device(void **out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return CHFPE_EDEVICE;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return CHFPE_EDEVICE;
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return CHFPE_OK;
}
}  // namespace

extern "C" {

size_t chfpe_workspace_bytes(const chfpe_params *p) {
  Derived d;
  std::string err;
  if (!derive(p, d, err)) return 0;
  return layout(d).total;
}

int chfpe_setup(const chfpe_params *p, void *dev_workspace, size_t ws_bytes, void *hip_stream,
                chfpe_ctx **out) {
  if (!out) return fail(nullptr, CHFPE_EINVAL, "out is NULL");
  Derived d;
  std::string err;
  if (!derive(p, d, err)) return fail(nullptr, CHFPE_EINVAL, err);
  Layout L = layout(d);
  if (dev_workspace && ws_bytes < L.total)
    return fail(nullptr, CHFPE_ENOMEM, "workspace smaller than chfpe_workspace_bytes()");
  if (dev_workspace && (reinterpret_cast<uintptr_t>(dev_workspace) % 256) != 0)
    return fail(nullptr, CHFPE_EINVAL, "workspace must be 256-byte aligned");

  {
    void *sp = nullptr;  // the device's scratch address, taken once per device at set-up
    if (scratch_of_current_device(&sp) != CHFPE_OK)
      return fail(nullptr, CHFPE_EDEVICE, "hipGetSymbolAddress of the device scratch failed");
  }
  chfpe_ctx *c = new chfpe_ctx();
  c->prm = *p;
  c->d = d;
  c->L = L;
  c->stream = reinterpret_cast<hipStream_t>(hip_stream);
  if (dev_workspace) {
    c->ws = reinterpret_cast<unsigned char *>(dev_workspace);
  } else {
    hipError_t e = hipMalloc(&c->ws, L.total);
    if (e != hipSuccess) {
      delete c;
      return fail(nullptr, CHFPE_ENOMEM, std::string("hipMalloc workspace: ") + hipGetErrorString(e));
    }
    c->own_ws = true;
  }
  auto at = [&](size_t off) { return c->ws + off; };
  c->F = (double *)at(L.F);
  c->VpQ = (double *)at(L.VpQ);
  c->Vp = (double *)at(L.Vp);
  c->pm = (double *)at(L.pm);
  c->pg = (double *)at(L.pg);
  c->gA = (double *)at(L.gA);
  c->gB = (double *)at(L.gB);
  c->gC = (double *)at(L.gC);
  c->Cw = (double *)at(L.Cw);
  c->wp = (double *)at(L.wp);
  c->sq = (double *)at(L.sq);
  c->sp = (double *)at(L.sp);
  c->up = (int *)at(L.up);
  c->dn = (int *)at(L.dn);
  c->cc = (double *)at(L.cc);
  c->tc = (double *)at(L.tc);
  c->damp = (double *)at(L.damp);
  c->partial = (double *)at(L.partial);
  c->scal = (double *)at(L.scal);
  c->flag = (int *)at(L.flag);
  double **bp[kStateBufs] = {&c->weq, &c->u, &c->y, &c->xa, &c->xb, &c->t};
  for (int i = 0; i < kStateBufs; ++i) *bp[i] = (double *)at(L.bufs[i]);
  if (d.batched)
    for (int i = 0; i < kBranchBufs; ++i) c->bb[i] = at(L.bbufs[i]);

  make_geom(c);
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tuned.find(tune_key(d));
    if (it != g_tuned.end()) {
      c->tune_pb_nb = it->second.pb_nb;
      c->tune_pb_split = it->second.pb_split;
      c->tune_q_pc = it->second.q_pc;
      c->tune_pb_run = it->second.pb_run;
    }
  }
  if (const char *v = std::getenv("CHFPE_TUNE_PB_NB")) c->tune_pb_nb = std::atoi(v);
  if (const char *v = std::getenv("CHFPE_TUNE_Q_PC")) c->tune_q_pc = std::atoi(v);
  if (const char *v = std::getenv("CHFPE_TUNE_PB_SPLIT")) c->tune_pb_split = std::atoi(v);
  if (const char *v = std::getenv("CHFPE_TUNE_PB_RUN")) c->tune_pb_run = std::atoi(v);
  if (const char *v = std::getenv("CHFPE_TUNE_PC_PAD")) c->tune_pc_pad = std::max(0, std::min(8, std::atoi(v)));
  if (const char *v = std::getenv("CHFPE_TUNE_PC_STREAM")) c->tune_pc_stream = std::atoi(v);
  if (const char *v = std::getenv("CHFPE_TUNE_HC_CHUNK")) c->tune_hc_chunk = std::atoi(v);
  if (const char *v = std::getenv("CHFPE_TUNE_HC_KTILE")) c->tune_hc_ktile = std::atoi(v);
  if (const char *v = std::getenv("CHFPE_NO_GRAPH")) c->use_graphs = std::atoi(v) == 0;
  if (const char *v = std::getenv("CHFPE_PCUBE")) c->allow_pcube = std::atoi(v) != 0;
  std::vector<double> F, Vp, pm, pg, sq, sp, wp, cc, tc, damp;
  std::vector<int> up, dn;
  build_tables(c, F, Vp, pm, pg, sq, sp, wp, up, dn, cc, tc, damp);
  std::vector<double> VpQ(3 * (size_t)d.Q, 0.0);
  for (int ql = 0; ql < d.Q; ++ql) {
    int rem = ql;
    for (int s = d.M - 1; s >= 0; --s) {
      VpQ[(size_t)s * d.Q + ql] = Vp[s * kTab + rem % d.Nq[s]];
      rem /= d.Nq[s];
    }
  }
  {
    double smin = 1.0;
    for (double v : sq) smin = std::min(smin, v);
    for (double v : sp) smin = std::min(smin, v);
    if (!(smin > 1e-150)) {
      chfpe_destroy(c);
      return fail(nullptr, CHFPE_EINVAL, "box too large: exp(-beta H/2) underflows at its edge");
    }
  }
  if (!plan(c)) {  // requested q tiles too small for this batch: automatic ones
    c->tune_pb_nb = 0;
    c->tune_pb_split = -1;
    c->tune_q_pc = 0;
    c->tune_pb_run = 0;
    if (!plan(c)) {
      chfpe_destroy(c);
      return fail(nullptr, CHFPE_EINVAL,
                  "batch too large: a q-pass launch over every branch state exceeds one dispatch (2^32 work-items)");
    }
  }

  auto up_copy = [&](void *dst, const void *src, size_t bytes) {
    return hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, c->stream);
  };
  hipError_t e = hipSuccess;
  if (e == hipSuccess) e = up_copy(c->F, F.data(), F.size() * sizeof(double));
  if (e == hipSuccess) e = up_copy(c->VpQ, VpQ.data(), VpQ.size() * sizeof(double));
  if (e == hipSuccess) e = up_copy(c->Vp, Vp.data(), Vp.size() * sizeof(double));
  if (e == hipSuccess) e = up_copy(c->pm, pm.data(), pm.size() * sizeof(double));
  if (e == hipSuccess) e = up_copy(c->pg, pg.data(), pg.size() * sizeof(double));
  if (e == hipSuccess) e = up_copy(c->sq, sq.data(), sq.size() * sizeof(double));
  if (e == hipSuccess) e = up_copy(c->sp, sp.data(), sp.size() * sizeof(double));
  if (e == hipSuccess) e = up_copy(c->wp, wp.data(), wp.size() * sizeof(double));
  if (e == hipSuccess) e = up_copy(c->up, up.data(), up.size() * sizeof(int));
  if (e == hipSuccess) e = up_copy(c->dn, dn.data(), dn.size() * sizeof(int));
  if (e == hipSuccess) e = up_copy(c->cc, cc.data(), cc.size() * sizeof(double));
  if (e == hipSuccess) e = up_copy(c->tc, tc.data(), tc.size() * sizeof(double));
  if (e == hipSuccess) e = up_copy(c->damp, damp.data(), damp.size() * sizeof(double));
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);  // host vectors go out of scope
  if (e != hipSuccess) {
    std::string msg = std::string("table upload: ") + hipGetErrorString(e);
    chfpe_destroy(c);
    return fail(nullptr, CHFPE_EDEVICE, msg);
  }
  c->tb.F = c->F;
  c->tb.VpQ = c->VpQ;
  c->tb.Vp = c->Vp;
  c->tb.pm = c->pm;
  c->tb.pg = c->pg;
  c->tb.up = c->up;
  c->tb.dn = c->dn;
  c->tb.cc = c->cc;
  c->tb.tc = c->tc;
  c->tb.damp = c->damp;
  c->tb.clos = reinterpret_cast<const double *>(at(L.clos));
  *out = c;
  return CHFPE_OK;
}

int chfpe_equilibrate(chfpe_ctx *c, int64_t n_steps, double dt) {
  if (!c) return CHFPE_EINVAL;
  if (n_steps < 0 || !std::isfinite(dt) || (n_steps > 0 && !(dt > 0)))
    return fail(c, CHFPE_EINVAL, "need n_steps >= 0 and dt > 0");
  const int nb = 1024;
  // Hermite basis: c_{0,0} = e^{-beta U/2} / Z_q in the first Q values (a unit p block)
  const int P = c->d.hermite ? 1 : c->d.P;
  hipLaunchKernelGGL((k_boltzmann<double>), dim3(nb), dim3(256), 0, c->stream, c->y, c->sq, c->sp, c->d.Q,
                     P, c->d.S);
  // Z = dV sum w exp(-beta H) = dV sum (w_q sq)(w_p sp) h_0 with h_0 = sq sp
  std::vector<double> ones(c->d.Q);
  for (int ql = 0; ql < c->d.Q; ++ql) ones[ql] = c->wq_host[ql] * c->sq_host[ql];
  HIPCHK(c, hipMemcpyAsync(c->Cw, ones.data(), ones.size() * sizeof(double), hipMemcpyHostToDevice,
                           c->stream));
  {
    const int nbr = std::min(kPartials, std::max(1, (int)(((long long)c->d.Q * P + 255) / 256)));
    hipLaunchKernelGGL((k_reduce_w0<double>), dim3(nbr), dim3(256), 0, c->stream, c->y, c->Cw, c->wp,
                       c->d.Q, P, c->partial, (long long)c->d.S);
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(256), 0, c->stream, c->partial, nbr, 1.0, c->scal, 1);
    hipLaunchKernelGGL((k_normalise<double>), dim3(1024), dim3(256), 0, c->stream, c->y, c->scal, c->dV,
                       c->d.Q * P);
  }
  HIPCHK(c, hipStreamSynchronize(c->stream));  // `ones` is read by the async copy
  int rc = rk4(c, c->y, n_steps, dt);
  if (rc) return rc;
  rc = check_finite(c, c->y);
  if (rc) return rc;
  HIPCHK(c, hipMemcpyAsync(c->weq, c->y, c->d.S * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  c->has_eq = true;
  return last_launch_error(c);
}

int chfpe_propagate(chfpe_ctx *c, int64_t n_steps, double dt) {
  if (!c) return CHFPE_EINVAL;
  if (n_steps < 0 || !std::isfinite(dt) || (n_steps > 0 && !(dt > 0)))
    return fail(c, CHFPE_EINVAL, "need n_steps >= 0 and dt > 0");
  int rc = rk4(c, c->y, n_steps, dt);
  if (rc) return rc;
  return check_finite(c, c->y);
}

int chfpe_rhs(chfpe_ctx *c) {
  if (!c) return CHFPE_EINVAL;
  const Batch b = batch_of(c, 1);
  launch_stage<double, EPI_OUT>(c, b, c->y, c->t, nullptr, c->xa, 0.0, K_QOUT);
  std::swap(c->y, c->xa);
  return last_launch_error(c);
}

int chfpe_perturb(chfpe_ctx *c, const chfpe_optical *X) {
  if (!c) return CHFPE_EINVAL;
  if (!optical_ok(X, c->d.M)) return fail(c, CHFPE_EINVAL, "invalid optical operator");
  std::vector<double> gt;
  grad_table(c, X, gt);
  HIPCHK(c, hipMemcpyAsync(c->gA, gt.data(), gt.size() * sizeof(double), hipMemcpyHostToDevice, c->stream));
  launch_perturb<double>(c, c->y, c->xa, c->gA);
  std::swap(c->y, c->xa);
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return last_launch_error(c);
}

int chfpe_observe(chfpe_ctx *c, const chfpe_optical *X, double *value) {
  if (!c || !value) return CHFPE_EINVAL;
  if (!optical_ok(X, c->d.M)) return fail(c, CHFPE_EINVAL, "invalid optical operator");
  std::vector<double> ct;
  value_table(c, X, ct);
  HIPCHK(c, hipMemcpyAsync(c->Cw, ct.data(), ct.size() * sizeof(double), hipMemcpyHostToDevice, c->stream));
  observe_to(c, c->y, c->scal + 1);
  HIPCHK(c, hipMemcpyAsync(value, c->scal + 1, sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return last_launch_error(c);
}

int chfpe_response_1d(chfpe_ctx *c, const chfpe_optical *A, int64_t n_t, int32_t stride, double dt,
                      double *R) {
  if (!c) return CHFPE_EINVAL;
  if (!optical_ok(A, c->d.M) || n_t < 0 || stride < 0 || (n_t > 1 && stride < 1) || !R ||
      !std::isfinite(dt) || (n_t > 1 && !(dt > 0)))
    return fail(c, CHFPE_EINVAL, "invalid response arguments");
  if (!c->has_eq) return fail(c, CHFPE_ESTATE, "no equilibrium: call chfpe_equilibrate first");
  if (n_t == 0) return CHFPE_OK;
  int rc = ensure_rbuf(c, (size_t)n_t);
  if (rc) return rc;
  std::vector<double> gt, ct;
  grad_table(c, A, gt);
  value_table(c, A, ct);
  HIPCHK(c, hipMemcpyAsync(c->gA, gt.data(), gt.size() * sizeof(double), hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->Cw, ct.data(), ct.size() * sizeof(double), hipMemcpyHostToDevice, c->stream));
  launch_perturb<double>(c, c->weq, c->y, c->gA);
  for (int64_t j = 0; j < n_t; ++j) {
    if (j > 0) {
      rc = rk4(c, c->y, stride, dt);
      if (rc) return rc;
    }
    observe_to(c, c->y, c->rbuf + j);
  }
  HIPCHK(c, hipMemcpyAsync(R, c->rbuf, n_t * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  rc = last_launch_error(c);
  if (rc) return rc;
  for (int64_t j = 0; j < n_t; ++j)
    if (!std::isfinite(R[j])) return fail(c, CHFPE_ENONFINITE, "response became non-finite");
  return CHFPE_OK;
}

int chfpe_response_2d_range(chfpe_ctx *c, const chfpe_optical *A, const chfpe_optical *B,
                            const chfpe_optical *C, int64_t j1_begin, int64_t j1_end, int64_t n_t2, int32_t stride1,
                            int32_t stride2, double dt, double *R) {
  if (!c) return CHFPE_EINVAL;
  if (!optical_ok(A, c->d.M) || !optical_ok(B, c->d.M) || !optical_ok(C, c->d.M) || j1_begin < 0 ||
      j1_end < j1_begin || n_t2 < 0 || stride1 < 0 || stride2 < 0 || (j1_end > 1 && stride1 < 1) ||
      (n_t2 > 1 && stride2 < 1) || !R || !std::isfinite(dt) || ((j1_end > 1 || n_t2 > 1) && !(dt > 0)))
    return fail(c, CHFPE_EINVAL, "invalid response arguments");
  if (!c->has_eq) return fail(c, CHFPE_ESTATE, "no equilibrium: call chfpe_equilibrate first");
  const int64_t n_t1 = j1_end - j1_begin;  // columns computed here
  const int64_t n = n_t1 * n_t2;
  if (n == 0) return CHFPE_OK;
  int rc = ensure_rbuf(c, (size_t)(n + (c->d.batched ? (int64_t)c->d.B * n_t2 : 0)));
  if (rc) return rc;
  std::vector<double> ga, gb, ct;
  grad_table(c, A, ga);
  grad_table(c, B, gb);
  value_table(c, C, ct);
  HIPCHK(c, hipMemcpyAsync(c->gA, ga.data(), ga.size() * sizeof(double), hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->gB, gb.data(), gb.size() * sizeof(double), hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->Cw, ct.data(), ct.size() * sizeof(double), hipMemcpyHostToDevice, c->stream));
  // U = A^x W_eq, advanced to the first column's t1
  launch_perturb<double>(c, c->weq, c->u, c->gA);
  if (j1_begin > 0) {
    rc = rk4(c, c->u, j1_begin * stride1, dt);
    if (rc) return rc;
  }
  if (c->d.batched) {
    rc = c->d.prec == CHFPE_FP32 ? branches_batched<float>(c, n_t1, n_t2, stride1, stride2, dt)
                                 : branches_batched<double>(c, n_t1, n_t2, stride1, stride2, dt);
    if (rc) return rc;
  }
  for (int64_t j1 = 0; j1 < (c->d.batched ? 0 : n_t1); ++j1) {
    if (j1 > 0) {
      rc = rk4(c, c->u, stride1, dt);
      if (rc) return rc;
    }
    // V = B^x U
    launch_perturb<double>(c, c->u, c->y, c->gB);
    for (int64_t j2 = 0; j2 < n_t2; ++j2) {
      if (j2 > 0) {
        rc = rk4(c, c->y, stride2, dt);
        if (rc) return rc;
      }
      observe_to(c, c->y, c->rbuf + j2 * n_t1 + j1);
    }
  }
  HIPCHK(c, hipMemcpyAsync(R, c->rbuf, n * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  rc = last_launch_error(c);
  if (rc) return rc;
  for (int64_t j = 0; j < n; ++j)
    if (!std::isfinite(R[j])) return fail(c, CHFPE_ENONFINITE, "response became non-finite");
  return CHFPE_OK;
}

int chfpe_response_2d(chfpe_ctx *c, const chfpe_optical *A, const chfpe_optical *B, const chfpe_optical *C,
                      int64_t n_t1, int64_t n_t2, int32_t stride1, int32_t stride2, double dt, double *R) {
  if (!c) return CHFPE_EINVAL;
  if (n_t1 < 0) return fail(c, CHFPE_EINVAL, "invalid response arguments");
  return chfpe_response_2d_range(c, A, B, C, 0, n_t1, n_t2, stride1, stride2, dt, R);
}

int chfpe_response_3d(chfpe_ctx *c, const chfpe_optical *A, const chfpe_optical *B, const chfpe_optical *C,
                      const chfpe_optical *D, int64_t n_t1, int64_t t2_steps, int64_t n_t3, int32_t stride1,
                      int32_t stride3, double dt, double *R) {
  if (!c) return CHFPE_EINVAL;
  if (!optical_ok(A, c->d.M) || !optical_ok(B, c->d.M) || !optical_ok(C, c->d.M) || !optical_ok(D, c->d.M) ||
      n_t1 < 0 || t2_steps < 0 || n_t3 < 0 || stride1 < 0 || stride3 < 0 || (n_t1 > 1 && stride1 < 1) ||
      (n_t3 > 1 && stride3 < 1) || !R || !std::isfinite(dt) || ((n_t1 > 1 || n_t3 > 1 || t2_steps > 0) && !(dt > 0)))
    return fail(c, CHFPE_EINVAL, "invalid response arguments");
  if (!c->has_eq) return fail(c, CHFPE_ESTATE, "no equilibrium: call chfpe_equilibrate first");
  const int64_t n = n_t1 * n_t3;
  if (n == 0) return CHFPE_OK;
  int rc = ensure_rbuf(c, (size_t)n);
  if (rc) return rc;
  std::vector<double> ga, gb, gc, vd;
  grad_table(c, A, ga);
  grad_table(c, B, gb);
  grad_table(c, C, gc);
  value_table(c, D, vd);
  HIPCHK(c, hipMemcpyAsync(c->gA, ga.data(), ga.size() * sizeof(double), hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->gB, gb.data(), gb.size() * sizeof(double), hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->gC, gc.data(), gc.size() * sizeof(double), hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->Cw, vd.data(), vd.size() * sizeof(double), hipMemcpyHostToDevice, c->stream));
  // U = A^x W_eq, advanced along t1; each branch: B^x, the waiting time,
  // C^x, then the t3 samples of <D>
  launch_perturb<double>(c, c->weq, c->u, c->gA);
  for (int64_t j1 = 0; j1 < n_t1; ++j1) {
    if (j1 > 0) {
      rc = rk4(c, c->u, stride1, dt);
      if (rc) return rc;
    }
    launch_perturb<double>(c, c->u, c->y, c->gB);
    rc = rk4(c, c->y, t2_steps, dt);
    if (rc) return rc;
    launch_perturb<double>(c, c->y, c->xa, c->gC);
    std::swap(c->y, c->xa);  // the excited state becomes the propagated one
    for (int64_t j3 = 0; j3 < n_t3; ++j3) {
      if (j3 > 0) {
        rc = rk4(c, c->y, stride3, dt);
        if (rc) return rc;
      }
      observe_to(c, c->y, c->rbuf + j3 * n_t1 + j1);
    }
  }
  HIPCHK(c, hipMemcpyAsync(R, c->rbuf, n * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  rc = last_launch_error(c);
  if (rc) return rc;
  for (int64_t j = 0; j < n; ++j)
    if (!std::isfinite(R[j])) return fail(c, CHFPE_ENONFINITE, "response became non-finite");
  return CHFPE_OK;
}

int64_t chfpe_state_count(const chfpe_ctx *c) { return c ? c->d.S : 0; }

int chfpe_get_state(chfpe_ctx *c, double *host) {
  if (!c || !host) return CHFPE_EINVAL;
  // W = exp(-beta H/2) h, converted in a scratch buffer (the Hermite
  // coefficients are copied as they are)
  HIPCHK(c, hipMemcpyAsync(c->xb, c->y, c->d.S * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  if (!c->d.hermite)
    hipLaunchKernelGGL((k_sym_scale<double>), dim3(1024), dim3(256), 0, c->stream, c->xb, c->sq, c->sp, c->d.Q,
                       c->d.P, c->d.S, 1);
  HIPCHK(c, hipMemcpyAsync(host, c->xb, c->d.S * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return last_launch_error(c);
}

int chfpe_set_state(chfpe_ctx *c, const double *host) {
  if (!c || !host) return CHFPE_EINVAL;
  HIPCHK(c, hipMemcpyAsync(c->y, host, c->d.S * sizeof(double), hipMemcpyHostToDevice, c->stream));
  if (!c->d.hermite)
    hipLaunchKernelGGL((k_sym_scale<double>), dim3(1024), dim3(256), 0, c->stream, c->y, c->sq, c->sp, c->d.Q,
                       c->d.P, c->d.S, 0);
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return last_launch_error(c);
}

int chfpe_use_state_as_equilibrium(chfpe_ctx *c) {
  if (!c) return CHFPE_EINVAL;
  HIPCHK(c, hipMemcpyAsync(c->weq, c->y, c->d.S * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  c->has_eq = true;
  return CHFPE_OK;
}

// 64 workgroups of 256 threads per CU (256 CUs), fewer for small copies
static int stream_grid(long long n16) {
  return (int)std::max(1LL, std::min(16384LL, (n16 + 256LL * kStreamU - 1) / (256LL * kStreamU)));
}

int chfpe_stream_copy(void *dst, const void *src, size_t bytes, void *hip_stream) {
  if (!dst || !src || (bytes % 16) != 0) return CHFPE_EINVAL;
  const long long n16 = (long long)(bytes / 16);
  if (n16 == 0) return CHFPE_OK;
  hipLaunchKernelGGL(k_stream_copy, dim3(stream_grid(n16)), dim3(256), 0, reinterpret_cast<hipStream_t>(hip_stream),
                     reinterpret_cast<uint4 *>(dst), reinterpret_cast<const uint4 *>(src), n16);
  return hipGetLastError() == hipSuccess ? CHFPE_OK : CHFPE_EDEVICE;
}

int chfpe_stream_mix(void *dst, const void *a, const void *b, const void *c, int32_t nsrc, size_t bytes,
                     void *hip_stream) {
  if (!dst || nsrc < 0 || nsrc > 3 || (bytes % 16) != 0) return CHFPE_EINVAL;
  if ((nsrc >= 1 && !a) || (nsrc >= 2 && !b) || (nsrc >= 3 && !c)) return CHFPE_EINVAL;
  const long long n16 = (long long)(bytes / 16);
  if (n16 == 0) return CHFPE_OK;
  auto *d = reinterpret_cast<double2 *>(dst);
  auto *pa = reinterpret_cast<const double2 *>(a);
  auto *pb = reinterpret_cast<const double2 *>(b);
  auto *pc = reinterpret_cast<const double2 *>(c);
  const dim3 grid(stream_grid(n16));
  const hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  switch (nsrc) {
    case 0: hipLaunchKernelGGL(k_stream_mix<0>, grid, dim3(256), 0, st, d, pa, pb, pc, n16); break;
    case 1: hipLaunchKernelGGL(k_stream_mix<1>, grid, dim3(256), 0, st, d, pa, pb, pc, n16); break;
    case 2: hipLaunchKernelGGL(k_stream_mix<2>, grid, dim3(256), 0, st, d, pa, pb, pc, n16); break;
    default: hipLaunchKernelGGL(k_stream_mix<3>, grid, dim3(256), 0, st, d, pa, pb, pc, n16); break;
  }
  return hipGetLastError() == hipSuccess ? CHFPE_OK : CHFPE_EDEVICE;
}

namespace {
struct DevBuf {
  void *p = nullptr;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
};
}  // namespace

int chfpe_spectrum_1d(const double *R, int64_t n, double tau, double *omega, double *I, void *hip_stream) {
  if (!R || !I || n < 1 || n > (1LL << 24) || !(tau > 0) || !std::isfinite(tau)) return CHFPE_EINVAL;
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  DevBuf bR, bz, bo, bI;
  if (hipMalloc(&bR.p, n * sizeof(double)) != hipSuccess || hipMalloc(&bz.p, n * sizeof(double2)) != hipSuccess ||
      hipMalloc(&bo.p, n * sizeof(double2)) != hipSuccess || hipMalloc(&bI.p, n * sizeof(double)) != hipSuccess)
    return CHFPE_ENOMEM;
  if (hipMemcpyAsync(bR.p, R, n * sizeof(double), hipMemcpyHostToDevice, st) != hipSuccess) return CHFPE_EDEVICE;
  const int nb = (int)((n + 255) / 256);
  hipLaunchKernelGGL(k_to_complex, dim3(nb), dim3(256), 0, st, (const double *)bR.p, (double2 *)bz.p, n);
  // sum_j exp(+i omega_k t_j) R_j, omega_k = 2 pi k / (n tau)
  hipLaunchKernelGGL(k_dft_rows, dim3(nb), dim3(256), 0, st, (const double2 *)bz.p, (double2 *)bo.p, 1, (int)n,
                     (int)n, 1, (int)n, 1, 1.0);
  const double dw = 2.0 * M_PI / ((double)n * tau);
  hipLaunchKernelGGL(k_spectrum_out, dim3(nb), dim3(256), 0, st, (const double2 *)bo.p, (long long)n, (int)n,
                     tau, dw, 1, (double *)bI.p);
  if (hipMemcpyAsync(I, bI.p, n * sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess) return CHFPE_EDEVICE;
  if (hipStreamSynchronize(st) != hipSuccess) return CHFPE_EDEVICE;
  if (hipGetLastError() != hipSuccess) return CHFPE_EDEVICE;
  if (omega)
    for (int64_t k = 0; k < n; ++k) omega[k] = dw * (double)k;
  return CHFPE_OK;
}

}  // extern "C"

namespace {

// Im{tau_f tau_s sum_{j_s, j_f} exp(-i omega_f t_f + sign_s i omega_s t_s) R[j_s][j_f]}
// as two passes of discrete Fourier sums (fast axis, then slow axis), on
// device buffers dR (n doubles), dz, dout (n double2 each) and dI (n doubles).
int spectrum_2d_on(const double *R, long long n_f, long long n_s, double tau_f, double tau_s, double sign_s,
                   double *I, hipStream_t st, double *dR, double2 *dz, double2 *dout, double *dI) {
  const long long n = n_f * n_s;
  if (hipMemcpyAsync(dR, R, n * sizeof(double), hipMemcpyHostToDevice, st) != hipSuccess) return CHFPE_EDEVICE;
  const int nb = (int)((n + 255) / 256);
  hipLaunchKernelGGL(k_to_complex, dim3(nb), dim3(256), 0, st, (const double *)dR, dz, n);
  // along the fast axis (rows of length n_f), exp(-i omega t)
  hipLaunchKernelGGL(k_dft_rows, dim3(nb), dim3(256), 0, st, (const double2 *)dz, dout, (int)n_s, (int)n_f,
                     (int)n_f, 1, (int)n_f, 1, -1.0);
  // along the slow axis (columns, stride n_f), exp(sign_s i omega t)
  hipLaunchKernelGGL(k_dft_rows, dim3(nb), dim3(256), 0, st, (const double2 *)dout, dz, (int)n_f, (int)n_s, 1,
                     (int)n_f, 1, (int)n_f, sign_s);
  hipLaunchKernelGGL(k_spectrum_out, dim3(nb), dim3(256), 0, st, (const double2 *)dz, n, (int)n_f, tau_f * tau_s,
                     0.0, 0, dI);
  if (hipMemcpyAsync(I, dI, n * sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess) return CHFPE_EDEVICE;
  if (hipStreamSynchronize(st) != hipSuccess) return CHFPE_EDEVICE;
  if (hipGetLastError() != hipSuccess) return CHFPE_EDEVICE;
  return CHFPE_OK;
}

bool spectrum_args_ok(const double *R, const double *I, long long n_f, long long n_s, double tau_f, double tau_s) {
  return R && I && n_f >= 1 && n_s >= 1 && n_f * n_s <= (1LL << 26) && tau_f > 0 && tau_s > 0 &&
         std::isfinite(tau_f) && std::isfinite(tau_s);
}

// The same with device buffers allocated for the call.
int spectrum_2d_signed(const double *R, int64_t n_f, int64_t n_s, double tau_f, double tau_s, double sign_s,
                       double *I, void *hip_stream) {
  if (!spectrum_args_ok(R, I, n_f, n_s, tau_f, tau_s)) return CHFPE_EINVAL;
  const long long n = n_f * n_s;
  DevBuf bR, bz, bo, bI;
  if (hipMalloc(&bR.p, n * sizeof(double)) != hipSuccess || hipMalloc(&bz.p, n * sizeof(double2)) != hipSuccess ||
      hipMalloc(&bo.p, n * sizeof(double2)) != hipSuccess || hipMalloc(&bI.p, n * sizeof(double)) != hipSuccess)
    return CHFPE_ENOMEM;
  return spectrum_2d_on(R, n_f, n_s, tau_f, tau_s, sign_s, I, reinterpret_cast<hipStream_t>(hip_stream),
                        (double *)bR.p, (double2 *)bz.p, (double2 *)bo.p, (double *)bI.p);
}

}  // namespace

extern "C" {

int chfpe_spectrum_2d(const double *R, int64_t n_t1, int64_t n_t2, double tau1, double tau2, double *I,
                      void *hip_stream) {
  return spectrum_2d_signed(R, n_t1, n_t2, tau1, tau2, -1.0, I, hip_stream);
}

int chfpe_spectrum_2dir(const double *R, int64_t n_t1, int64_t n_t3, double tau1, double tau3, double *I,
                        void *hip_stream) {
  return spectrum_2d_signed(R, n_t1, n_t3, tau1, tau3, +1.0, I, hip_stream);
}

int chfpe_spectrum_2d_noalloc(const double *R, int64_t n_t1, int64_t n_t2, double tau1, double tau2, double *I,
                              void *hip_stream) {
  if (!spectrum_args_ok(R, I, n_t1, n_t2, tau1, tau2) || n_t1 * n_t2 > kNoAllocMaxPoints) return CHFPE_EINVAL;
  void *base = nullptr;
  int rc = scratch_of_current_device(&base);
  if (rc) return rc;
  const long long n = n_t1 * n_t2;
  // layout in the scratch: two complex arrays, then R and I (16-byte aligned)
  unsigned char *b = reinterpret_cast<unsigned char *>(base);
  double2 *dz = reinterpret_cast<double2 *>(b);
  double2 *dout = reinterpret_cast<double2 *>(b + 16 * n);
  double *dR = reinterpret_cast<double *>(b + 32 * n);
  double *dI = reinterpret_cast<double *>(b + 40 * n);
  return spectrum_2d_on(R, n_t1, n_t2, tau1, tau2, -1.0, I, reinterpret_cast<hipStream_t>(hip_stream), dR, dz,
                        dout, dI);
}

int chfpe_set_kernel_timing(chfpe_ctx *c, int32_t every) {
  if (!c || every < 0) return CHFPE_EINVAL;
  c->timing_every = every;
  c->step_counter = 0;
  return CHFPE_OK;
}

int chfpe_autotune(chfpe_ctx *c, int32_t n_steps) {
  if (!c) return CHFPE_EINVAL;
  if (n_steps < 1 || n_steps > 1000) return fail(c, CHFPE_EINVAL, "need 1 <= n_steps <= 1000");
  if (c->d.hermite) return CHFPE_OK;  // one k_hcube shape: nothing to choose
  const Derived &d = c->d;
  // the timed steps run on scratch buffers holding zeros (the work does not
  // depend on the values); the cached wave graph holds the old tile shapes
  HIPCHK(c, hipMemsetAsync(c->u, 0, sizeof(double) * (size_t)d.S, c->stream));
  if (d.batched)
    HIPCHK(c, hipMemsetAsync(c->bb[0], 0, (d.prec == CHFPE_FP32 ? 4 : 8) * (size_t)d.S * d.B, c->stream));
  if (c->wave_graph) {
    HIPCHK(c, hipGraphExecDestroy(c->wave_graph));
    c->wave_graph = nullptr;
  }
  const int timing = c->timing_every;
  c->timing_every = 0;
  const double dt = 1e-3;
  TileChoice best{c->tune_pb_nb, c->tune_pb_split, c->tune_q_pc, c->tune_pb_run};
  double best_ms = 1e300;
  auto restore = [&](int rc) {
    c->tune_pb_nb = best.pb_nb;
    c->tune_pb_split = best.pb_split;
    c->tune_q_pc = best.q_pc;
    c->tune_pb_run = best.pb_run;
    (void)plan(c);  // the starting shape, or one that fit when timed
    c->timing_every = timing;
    return rc;
  };
  auto trial = [&](const TileChoice &t, std::vector<std::vector<int>> &seen) -> int {
    c->tune_pb_nb = t.pb_nb;
    c->tune_pb_split = t.pb_split;
    c->tune_q_pc = t.q_pc;
    c->tune_pb_run = t.pb_run;
    if (!plan(c)) return CHFPE_OK;  // too large a launch for one dispatch: not a candidate
    const std::vector<int> eff = {c->ln.pb.nb, c->ln.pb.split, c->ln.qf.pc, c->ln.qa.pc, c->ln.pb.run};
    for (const auto &s : seen)
      if (s == eff) return CHFPE_OK;  // same launches as a shape already timed
    seen.push_back(eff);
    const double ms = time_rk4_step(c, n_steps, dt);
    if (ms < 0) return CHFPE_EDEVICE;
    if (ms < best_ms) {
      best_ms = ms;
      best = t;
    }
    return CHFPE_OK;
  };
  // k_pblock shapes first (q tiles automatic), then q tiles with the best,
  // then the k_pblock task order
  std::vector<std::vector<int>> seen;
  for (int split : {1, 0})
    for (int nb : {1, 2, 4, 8})
      if (trial(TileChoice{nb, split, best.q_pc, best.pb_run}, seen))
        return restore(fail(c, CHFPE_EDEVICE, "autotune step failed"));
  const TileChoice pbest = best;
  for (int pc : {4, 8, 16, 32})
    if (trial(TileChoice{pbest.pb_nb, pbest.pb_split, pc, pbest.pb_run}, seen))
      return restore(fail(c, CHFPE_EDEVICE, "autotune step failed"));
  const TileChoice qbest = best;
  for (int run : {1, 4, 8, 16, 32})
    if (trial(TileChoice{qbest.pb_nb, qbest.pb_split, qbest.q_pc, run}, seen))
      return restore(fail(c, CHFPE_EDEVICE, "autotune step failed"));
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tuned[tune_key(d)] = best;
  }
  return restore(last_launch_error(c));
}

int chfpe_tile_config(const chfpe_ctx *c, int32_t *out, int32_t n) {
  if (!c || !out || n < 0) return CHFPE_EINVAL;
  const int32_t v[15] = {c->ln.pb.nb,  c->ln.pb.split,    c->ln.pb_threads,
                         c->ln.qf.pc,  c->ln.has_qa ? c->ln.qa.pc : 0, c->ln.qf_threads,
                         c->tune_pb_nb, c->tune_pb_split, c->tune_q_pc, c->ln.pb.run, c->tune_pb_run,
                         c->ln.pcube ? 1 : 0, c->ln.pcube && c->ln.pcube_stream ? 1 : 0,
                         c->ln.hcube ? c->ln.hcb.chunk : 0, c->ln.hcube ? c->ln.hcb.ktile : 0};
  const int k = n < 15 ? n : 15;
  for (int i = 0; i < k; ++i) out[i] = v[i];
  return k;
}

int chfpe_kernel_times(chfpe_ctx *c, int32_t max_kinds, int64_t *counts, double *mean_ms,
                       double *mean_bytes, const char **names) {
  if (!c) return CHFPE_EINVAL;
  int rc = drain_timing(c);
  if (rc) return rc;
  int n = std::min<int>(max_kinds, kNumKinds);
  for (int i = 0; i < n; ++i) {
    if (counts) counts[i] = c->kcount[i];
    if (mean_ms) mean_ms[i] = c->kcount[i] ? c->ktime[i] / c->kcount[i] : 0.0;
    if (mean_bytes) mean_bytes[i] = c->kcount[i] ? c->kbytes[i] / c->kcount[i] : 0.0;
    if (names) names[i] = kKindNames[i];
  }
  return n;
}

const char *chfpe_last_error(const chfpe_ctx *c) { return c ? c->err.c_str() : g_setup_error.c_str(); }

void chfpe_destroy(chfpe_ctx *c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->stream);
  for (auto &pd : c->pending) {
    (void)hipEventDestroy(pd.a);
    (void)hipEventDestroy(pd.b);
  }
  for (auto ev : c->event_pool) (void)hipEventDestroy(ev);
  if (c->wave_graph) (void)hipGraphExecDestroy(c->wave_graph);
  if (c->rbuf) (void)hipFree(c->rbuf);
  if (c->own_ws && c->ws) (void)hipFree(c->ws);
  delete c;
}

// ---------------------------------------------------------------------------
// learned per-axis closure
// ---------------------------------------------------------------------------
int32_t chfpe_closure_rows(const chfpe_params *p) {
  Derived d;
  std::string err;
  if (!p || !derive(p, d, err)) return CHFPE_EINVAL;
  return closure_rows(p);
}

int chfpe_closure_features(const chfpe_params *p, float *feat, int32_t *axis_of_row) {
  Derived d;
  std::string err;
  if (!p || !feat || !derive(p, d, err)) return fail_g(CHFPE_EINVAL, err.empty() ? "invalid arguments" : err);
  const int M = p->M;
  int N[6];
  double h[6], L[6];
  axis_table(p, M, N, h, L);
  int row = 0;
  for (int a = 0; a < 2 * M; ++a) {
    const int s = a % M;
    const double m = p->m[s], om = p->omega[s], beta = p->beta;
    const double sig_q = 1.0 / (om * std::sqrt(beta * m));
    const double sig = a < M ? sig_q : std::sqrt(m / beta);
    for (int e = 0; e < skew_entries(N[a]); ++e) {
      int k = 1, i = e;
      while (i >= N[a] - k) {
        i -= N[a] - k;
        ++k;
      }
      const double xi = -L[a] + (i + 0.5) * h[a], xk = -L[a] + (i + k + 0.5) * h[a];
      const double u = 0.5 * (xi + xk) / L[a];
      const int edge = std::min(i, N[a] - 1 - (i + k));
      const double f[kClosFeat] = {u, u * u, std::fabs(u), k == 2 ? 1.0 : 0.0, a >= M ? 1.0 : 0.0, h[a] / sig,
                                   om / 1.6, p->g3[s] * sig_q / (m * om * om),
                                   p->g4[s] * sig_q * sig_q / (m * om * om), p->V_SL[s] * sig_q / p->V_LL[s],
                                   p->zeta[s], p->gamma[s], beta / 2.0, m, edge == 0 ? 1.0 : 0.0, 1.0};
      for (int q = 0; q < kClosFeat; ++q) feat[row * kClosFeat + q] = (float)f[q];
      if (axis_of_row) axis_of_row[row] = a;
      ++row;
    }
  }
  return CHFPE_OK;
}

int chfpe_closure_moments(chfpe_ctx *c, double *G, double *b, double *ct) {
  if (!c || !G || !b || !ct) return CHFPE_EINVAL;
  if (c->d.hermite) return fail(c, CHFPE_EINVAL, "the closure is defined for the grid basis only");
  const Derived &d = c->d;
  const int M = d.M, nd = 2 * M;
  int Nf[6], Nc[6];
  double hf[6], Lf[6];
  axis_table(&c->prm, M, Nf, hf, Lf);
  for (int a = 0; a < nd; ++a) {
    if (Nf[a] % 2 || Nf[a] / 2 < 5 || Nf[a] / 2 > 16)
      return fail(c, CHFPE_EINVAL, "closure moments need even fine axes with 10..32 points");
    Nc[a] = Nf[a] / 2;
  }
  const long long ne = d.ne;
  long long Ec = 1;
  for (int a = 0; a < nd; ++a) Ec *= Nc[a];
  // coarse x, T, r in xa (3 coarse states fit in one fine state buffer)
  double *xc = c->xa, *Tc = c->xa + ne * Ec, *rc = c->xa + 2 * ne * Ec;
  Restrict rs{};
  rs.nd = nd;
  {
    long long sc = 1, sf = 1;
    for (int a = nd - 1; a >= 0; --a) {
      rs.dc[a] = Nc[a];
      rs.sc[a] = sc;
      rs.sf[a] = sf;
      sc *= Nc[a];
      sf *= Nf[a];
    }
    rs.Ec = sc;
    rs.Ef = sf;
    rs.total = ne * sc;
  }
  const dim3 rgrid((unsigned)((rs.total + 255) / 256));
  hipLaunchKernelGGL(k_restrict, rgrid, dim3(256), 0, c->stream, c->y, xc, rs);
  DevScratch ds;
  size_t goff = 0, boff = 0;
  for (int a = 0; a < nd; ++a) {
    const int N = Nc[a], P = skew_entries(N);
    const double hc = 2.0 * hf[a];
    // target T = R(D_fine y) and residual r = T - D_coarse x
    launch_axis_deriv(c->stream, c->y, c->t, nullptr, 1.0, axis_lines(Nf, nd, a, ne), hf[a]);
    hipLaunchKernelGGL(k_restrict, rgrid, dim3(256), 0, c->stream, c->t, Tc, rs);
    const AxisLines al = axis_lines(Nc, nd, a, ne);
    launch_axis_deriv(c->stream, xc, rc, Tc, -1.0, al, hc);
    const long long lpb = std::max<long long>(kMomLines, (al.nlines + 1023) / 1024);
    const int nblk = (int)((al.nlines + lpb - 1) / lpb);
    const int nmom = 2 * N * N + 2;
    double *part = ds.get<double>((size_t)nblk * nmom);
    double *mom = ds.get<double>(nmom);
    double *dAi = ds.get<double>(N * N), *dK = ds.get<double>(N * N);
    double *dG = ds.get<double>(P * P), *db = ds.get<double>(P);
    if (!part || !mom || !dAi || !dK || !dG || !db) return fail(c, CHFPE_ENOMEM, "closure moments scratch");
    std::vector<double> Ai, K;
    compact_inverse(N, Ai, K);
    HIPCHK(c, hipMemcpyAsync(dAi, Ai.data(), N * N * sizeof(double), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(dK, K.data(), N * N * sizeof(double), hipMemcpyHostToDevice, c->stream));
    hipLaunchKernelGGL(k_line_moments, dim3(nblk), dim3(256), 0, c->stream, xc, rc, Tc, al, lpb, part);
    hipLaunchKernelGGL(k_sum_blocks, dim3((nmom + 255) / 256), dim3(256), 0, c->stream, part, nblk, nmom, mom);
    hipLaunchKernelGGL(k_gram, dim3((P * P + P + 255) / 256), dim3(256), 0, c->stream, mom, dAi, dK, N, hc, dG,
                       db);
    std::vector<double> hG(P * P), hb(P), hm(nmom);
    HIPCHK(c, hipMemcpyAsync(hG.data(), dG, P * P * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(hb.data(), db, P * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(hm.data(), mom, nmom * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (int v = 0; v < P * P; ++v) G[goff + v] += hG[v];
    for (int v = 0; v < P; ++v) b[boff + v] += hb[v];
    ct[2 * a] += hm[2 * N * N];
    ct[2 * a + 1] += hm[2 * N * N + 1];
    goff += (size_t)P * P;
    boff += P;
  }
  return last_launch_error(c);
}

// Converts host FP32 features to device BF16.
static short *upload_features(DevScratch &ds, const float *feat, int rows, hipStream_t st) {
  float *df = ds.get<float>((size_t)rows * kClosFeat);
  short *dh = ds.get<short>((size_t)rows * kClosFeat);
  if (!df || !dh) return nullptr;
  if (hipMemcpyAsync(df, feat, (size_t)rows * kClosFeat * sizeof(float), hipMemcpyHostToDevice, st) != hipSuccess)
    return nullptr;
  hipLaunchKernelGGL(k_to_bf16, dim3((rows * kClosFeat + 255) / 256), dim3(256), 0, st, df, dh, rows * kClosFeat);
  return dh;
}

int chfpe_closure_eval(const float *prm, const float *feat, int32_t rows, float *s, void *hip_stream) {
  if (!prm || !feat || !s || rows < 1 || rows > (1 << 20)) return fail_g(CHFPE_EINVAL, "invalid arguments");
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  DevScratch ds;
  short *dfeat = upload_features(ds, feat, rows, st);
  float *dp = ds.get<float>(kClosParams), *ds_ = ds.get<float>(rows);
  if (!dfeat || !dp || !ds_) return fail_g(CHFPE_ENOMEM, "closure eval scratch");
  if (hipMemcpyAsync(dp, prm, kClosParams * sizeof(float), hipMemcpyHostToDevice, st) != hipSuccess)
    return fail_g(CHFPE_EDEVICE, "copy");
  const int ntiles = (rows + 15) / 16;
  hipLaunchKernelGGL(k_clos_eval, dim3(std::min(1024, (ntiles + 3) / 4)), dim3(256), 0, st, dp, dfeat, rows, ds_);
  if (hipGetLastError() != hipSuccess) return fail_g(CHFPE_EDEVICE, "closure eval launch");
  if (hipMemcpyAsync(s, ds_, rows * sizeof(float), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return fail_g(CHFPE_EDEVICE, "closure eval copy");
  return CHFPE_OK;
}

int chfpe_closure_grad(const float *prm, const float *feat, int32_t rows, const float *gs, float *grad,
                       void *hip_stream) {
  if (!prm || !feat || !gs || !grad || rows < 1 || rows > (1 << 20))
    return fail_g(CHFPE_EINVAL, "invalid arguments");
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  DevScratch ds;
  short *dfeat = upload_features(ds, feat, rows, st);
  float *dp = ds.get<float>(kClosParams), *dgs = ds.get<float>(rows), *dg = ds.get<float>(kClosParams);
  if (!dfeat || !dp || !dgs || !dg) return fail_g(CHFPE_ENOMEM, "closure grad scratch");
  if (hipMemcpyAsync(dp, prm, kClosParams * sizeof(float), hipMemcpyHostToDevice, st) != hipSuccess ||
      hipMemcpyAsync(dgs, gs, rows * sizeof(float), hipMemcpyHostToDevice, st) != hipSuccess)
    return fail_g(CHFPE_EDEVICE, "copy");
  hipLaunchKernelGGL(k_clos_grad, dim3(1), dim3(256), 0, st, dp, dfeat, rows, dgs, dg);
  if (hipGetLastError() != hipSuccess) return fail_g(CHFPE_EDEVICE, "closure grad launch");
  if (hipMemcpyAsync(grad, dg, kClosParams * sizeof(float), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return fail_g(CHFPE_EDEVICE, "closure grad copy");
  return CHFPE_OK;
}

int chfpe_closure_train(const float *feat, int32_t rows, int32_t n_groups, const int32_t *group_start,
                        const double *G, const double *b, const double *ct, float *prm, float *adam_m,
                        float *adam_v, int32_t adam_t0, int32_t n_steps, float lr, float *loss, void *hip_stream) {
  if (!feat || !group_start || !G || !b || !ct || !prm || !adam_m || !adam_v || rows < 1 || rows > (1 << 20) ||
      n_groups < 1 || n_steps < 0 || n_steps > 1000000 || adam_t0 < 0 || !(lr > 0.f))
    return fail_g(CHFPE_EINVAL, "invalid arguments");
  if (group_start[0] != 0 || group_start[n_groups] != rows) return fail_g(CHFPE_EINVAL, "groups must cover the rows");
  std::vector<int> gof(rows);
  std::vector<long long> goff(n_groups);
  std::vector<int> boff(n_groups);
  long long gtot = 0;
  int btot = 0;
  for (int q = 0; q < n_groups; ++q) {
    const int P = group_start[q + 1] - group_start[q];
    if (P < 1) return fail_g(CHFPE_EINVAL, "empty group");
    goff[q] = gtot;
    boff[q] = btot;
    gtot += (long long)P * P;
    btot += P;
    for (int r = group_start[q]; r < group_start[q + 1]; ++r) gof[r] = q;
    if (!(ct[2 * q + 1] > 0.0)) return fail_g(CHFPE_EINVAL, "group target norm must be positive");
  }
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  DevScratch ds;
  short *dfeat = upload_features(ds, feat, rows, st);
  int *dgs = ds.get<int>(n_groups + 1), *dgof = ds.get<int>(rows), *dboff = ds.get<int>(n_groups);
  long long *dgoff = ds.get<long long>(n_groups);
  double *dG = ds.get<double>(gtot), *db = ds.get<double>(btot), *dct = ds.get<double>(2 * n_groups);
  float *dp = ds.get<float>(kClosParams), *dm = ds.get<float>(kClosParams), *dv = ds.get<float>(kClosParams);
  float *dsv = ds.get<float>(rows), *dgsv = ds.get<float>(rows), *dl = ds.get<float>(std::max(1, n_steps));
  if (!dfeat || !dgs || !dgof || !dboff || !dgoff || !dG || !db || !dct || !dp || !dm || !dv || !dsv || !dgsv || !dl)
    return fail_g(CHFPE_ENOMEM, "closure train scratch");
  auto up = [&](void *dst, const void *src, size_t bytes) {
    return hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st) == hipSuccess;
  };
  if (!up(dgs, group_start, (n_groups + 1) * sizeof(int)) || !up(dgof, gof.data(), rows * sizeof(int)) ||
      !up(dboff, boff.data(), n_groups * sizeof(int)) || !up(dgoff, goff.data(), n_groups * sizeof(long long)) ||
      !up(dG, G, gtot * sizeof(double)) || !up(db, b, btot * sizeof(double)) ||
      !up(dct, ct, 2 * n_groups * sizeof(double)) || !up(dp, prm, kClosParams * sizeof(float)) ||
      !up(dm, adam_m, kClosParams * sizeof(float)) || !up(dv, adam_v, kClosParams * sizeof(float)))
    return fail_g(CHFPE_EDEVICE, "closure train upload");
  ClosGroups gr{dgs, dgof, dgoff, dboff, dG, db, dct, n_groups};
  hipLaunchKernelGGL(k_clos_train, dim3(1), dim3(256), 0, st, dp, dm, dv, (int)adam_t0, dfeat, (int)rows, gr,
                     (int)n_steps, lr, dsv, dgsv, dl);
  if (hipGetLastError() != hipSuccess) return fail_g(CHFPE_EDEVICE, "closure train launch");
  bool ok = hipMemcpyAsync(prm, dp, kClosParams * sizeof(float), hipMemcpyDeviceToHost, st) == hipSuccess &&
            hipMemcpyAsync(adam_m, dm, kClosParams * sizeof(float), hipMemcpyDeviceToHost, st) == hipSuccess &&
            hipMemcpyAsync(adam_v, dv, kClosParams * sizeof(float), hipMemcpyDeviceToHost, st) == hipSuccess;
  if (ok && loss && n_steps > 0)
    ok = hipMemcpyAsync(loss, dl, n_steps * sizeof(float), hipMemcpyDeviceToHost, st) == hipSuccess;
  if (!ok || hipStreamSynchronize(st) != hipSuccess) return fail_g(CHFPE_EDEVICE, "closure train copy");
  return CHFPE_OK;
}

int chfpe_set_closure(chfpe_ctx *c, const double *sv) {
  if (!c) return CHFPE_EINVAL;
  if (!sv) {
    c->closure_on = false;
  } else {
    const Derived &d = c->d;
    if (d.hermite) return fail(c, CHFPE_EINVAL, "the closure is defined for the grid basis only");
    if (d.prec != CHFPE_FP64) return fail(c, CHFPE_EINVAL, "the closure runs with FP64 states only");
    const int M = d.M;
    int N[6];
    double h[6], L[6];
    axis_table(&c->prm, M, N, h, L);
    for (int a = 0; a < 2 * M; ++a)
      if (N[a] > 16) return fail(c, CHFPE_EINVAL, "the closure needs every axis to have at most 16 points");
    for (int r = 0; r < closure_rows(&c->prm); ++r)
      if (!std::isfinite(sv[r])) return fail(c, CHFPE_EINVAL, "closure entries must be finite");
    std::vector<double> tab(6 * 2 * kClosRows * kTab, 0.0);
    int row = 0;
    for (int a = 0; a < 2 * M; ++a) {
      const int n = N[a];
      // sk[k][i] = S[i][i+k]; zero where i + k is outside the line
      std::vector<double> sk[4];
      for (int k = 1; k <= 3; ++k) {
        sk[k].assign(n + 4, 0.0);
        if (k <= kClosBands)
          for (int i = 0; i < n - k; ++i) sk[k][i] = sv[row++];
      }
      const double base[4] = {0.0, 7.0 / 9.0, 1.0 / 36.0, 0.0};  // plain weights of f_{i+k} - f_{i-k}
      double *top = &tab[a * 2 * kClosRows * kTab], *mir = top + kClosRows * kTab;
      for (int i = 0; i < n; ++i) {
        const int j = n - 1 - i;  // position on the mirrored line
        for (int k = 1; k <= 3; ++k) {
          const double pk = (base[k] + sk[k][i]) / h[a];                      // weight of f_{i+k}
          const double mk = -(base[k] + (i >= k ? sk[k][i - k] : 0.0)) / h[a];  // weight of f_{i-k}
          top[(2 * k - 2) * kTab + i] = pk;
          top[(2 * k - 1) * kTab + i] = mk;
          // the mirrored line swaps the roles of the forward and backward neighbours
          mir[(2 * k - 2) * kTab + j] = mk;
          mir[(2 * k - 1) * kTab + j] = pk;
        }
      }
    }
    HIPCHK(c, hipMemcpyAsync(const_cast<double *>(c->tb.clos), tab.data(), tab.size() * sizeof(double),
                             hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->closure_on = true;
  }
  if (c->wave_graph) {  // captured with the other kernel variants
    HIPCHK(c, hipGraphExecDestroy(c->wave_graph));
    c->wave_graph = nullptr;
  }
  return CHFPE_OK;
}

}  // extern "C"
