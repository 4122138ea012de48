/*
 * chfpe.h -- C ABI of the MI355X (gfx950) solver for the multimode classical
 * hierarchical Fokker-Planck equations (CHFPE) of Hoshino & Tanimura,
 * "A Multimode Classical Hierarchical Fokker-Planck Equations Approach to
 * Molecular Vibrations: Simulating Two-Dimensional Spectra".
 *
 * Conventions shared by every entry point
 *   - Every function returns an int status (CHFPE_OK = 0, negative on error)
 *     unless stated otherwise; no C++ exception crosses this boundary.
 *   - Validation of arguments happens on the host before any device call, so
 *     CHFPE_EINVAL never leaves the device in a changed state.
 *   - Units are dimensionless with k_B = 1.
 *   - A state is the hierarchy W^(n)(q_1..q_M, p_1..p_M) of Eq. (eq:HEOM):
 *     FP64, C order [n][q_1..q_M][p_1..p_M] (p_M fastest); elements n are
 *     {n in N^M : |n| <= K} ordered by |n|, then lexicographically with n_1
 *     largest first.  Grids are uniform and cell-centred:
 *     x_i = -L + (i + 1/2) h, h = 2L/N.
 *   - Discretization: the compact sixth-order first derivative of Sec. III B
 *     (alpha = 1/3; weights 7/9 and 1/36 on the first and second
 *     differences; zero values outside the box) acts on the smooth factor
 *     h_n of W_n = exp(-beta H_sys/2) h_n, the factorization of Sec. III A,
 *     along every q and p axis; time integration is classical RK4 with a
 *     fixed step.  The discrete hierarchy is linear with a time-independent
 *     generator L, for which one classical RK4 step equals the degree-4
 *     Taylor polynomial of dt L; the device evaluates that polynomial in
 *     nested form, y <- y + dt L (y + dt/2 L (y + dt/3 L (y + dt/4 L y))),
 *     equal to the stage-by-stage form up to rounding.  Device buffers hold
 *     h; the functions below exchange W.
 *   - A context is not thread-safe; distinct contexts are independent.
 *   - All device work of a context runs on the stream given to chfpe_setup;
 *     functions that return host data synchronize that stream first.
 */
#ifndef CHFPE_H
#define CHFPE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  CHFPE_OK = 0,
  CHFPE_EINVAL = -1,     /* invalid argument or unsupported shape           */
  CHFPE_ENOMEM = -2,     /* workspace too small or allocation failed        */
  CHFPE_EDEVICE = -3,    /* a HIP runtime call failed                       */
  CHFPE_ENONFINITE = -4, /* the propagated state became non-finite          */
  CHFPE_ESTATE = -5      /* call out of order (e.g. response before eq.)    */
};

enum { CHFPE_FP64 = 0, CHFPE_FP32 = 1 };
enum { CHFPE_BASIS_GRID = 0, CHFPE_BASIS_HERMITE = 1 };

/*
 * Model and discretisation.
 *   U(q) = sum_s [ m_s omega_s^2 q_s^2 / 2 + g3_s q_s^3 / 3! + g4_s q_s^4 / 4! ]
 *        + sum_{s<s'} [ g2_ss' q_s q_s' + (g21_ss' q_s^2 q_s' + g12_ss' q_s q_s'^2) / 6 ]
 *     (Sec. II A, Eqs. (sec: Potenentials), (sec: Potential ss'); the quartic
 *     term extends the on-site potential).  Only entries s < s' of the pair
 *     matrices are read.
 *   V_s(q_s) = V_LL_s q_s + V_SL_s q_s^2 / 2 (system-bath coupling, Sec. II A).
 *   Drude bath per mode: zeta_s, gamma_s (Eq. (eq:drude)); beta = 1/T.
 *   K: hierarchy depth, elements {n : |n| <= K} (Eq. (eq:HEOM)).
 *   Nq/Np, Lq/Lp: points and half-width of the q_s and p_s axes.
 *   precision: type of the t1-branch states of chfpe_response_2d.  With
 *     CHFPE_FP32 their right-hand sides and RK4 updates are FP32, while the
 *     equilibration, the t1 trajectory U, both excitations (A^x, B^x) and
 *     every reduction stay FP64.  Everything else is FP64.
 *   batch: t1 branches propagated together by chfpe_response_2d (0 = 1);
 *     with batch > 1 or CHFPE_FP32, branches run in waves of `batch` states
 *     (batch x 4 extra state buffers of the branch type in the workspace),
 *     each wave's t2 loop as one captured HIP graph.
 *   basis: discretisation of the momenta.  CHFPE_BASIS_GRID: the compact
 *     scheme on a p grid (Np points on [-Lp, Lp]).  CHFPE_BASIS_HERMITE: the
 *     paper's own Hermite-function expansion (Sec. III A; Appendix A, Eq.
 *     (HEOM2FP-H)): W_n = e^{-beta U/2} prod_s psi_0(p_s) sum_k c_{n,k}(q)
 *     prod_s psi_{k_s}(p_s), psi_j the Hermite functions of width
 *     a_s = sqrt(2 m_s / beta); Np[s] is then the number of Hermite
 *     functions of mode s (k_s < Np[s]) and Lp is not read.  Every call
 *     below works in either basis; with the Hermite basis a state is the
 *     coefficient array c[n][k_1..k_M][q_1..q_M] (q_M fastest), which
 *     chfpe_get_state / chfpe_set_state copy as they are, observables
 *     integrate p exactly (only c_{0,0} contributes), and there are no tile
 *     shapes to tune (chfpe_autotune returns at once) and no closure.
 * Limits: 1 <= M <= 3, 0 <= K <= 12, 5 <= N <= 48 on every axis (the p
 * axes also within the tiling limit under chfpe_setup), all
 * masses, beta, L > 0, one element below 2^29 points, and
 * exp(-beta H_sys/2) representable (> 1e-150) everywhere on the grid.
 * With the Hermite basis: 2 <= Np[s] <= 48, and the q cube of one task
 * must fit one workgroup: a thread per (q_2, q_3) point (two modes: per q_2
 * point) holding a q_1 line, at most 1024 / 768 / 512 / 256 threads for q_1
 * lines of up to 16 / 24 / 32 / 48 points.
 */
typedef struct {
  int32_t M;
  int32_t K;
  int32_t Nq[3];
  int32_t Np[3];
  double Lq[3];
  double Lp[3];
  double m[3];
  double omega[3];
  double g3[3];
  double g4[3];
  double g2[3][3];
  double g21[3][3];
  double g12[3][3];
  double V_LL[3];
  double V_SL[3];
  double zeta[3];
  double gamma[3];
  double beta;
  int32_t precision;
  int32_t batch;
  int32_t basis; /* CHFPE_BASIS_GRID or CHFPE_BASIS_HERMITE */
} chfpe_params;

/* Optical operator X(q) = sum_s lin_s q_s + 1/2 sum_{s,s'} quad_ss' q_s q_s'
 * (dipole mu or polarizability Pi, Eqs. (NLdip), (NLpol)). */
typedef struct {
  double lin[3];
  double quad[3][3];
} chfpe_optical;

typedef struct chfpe_ctx chfpe_ctx;

/* Bytes of device workspace chfpe_setup needs for these parameters (tables,
 * six FP64 state buffers, the batched branch buffers, reduction scratch),
 * or 0 if the parameters are invalid.  The caller may allocate it (e.g. as a torch tensor) and pass it
 * to chfpe_setup. */
size_t chfpe_workspace_bytes(const chfpe_params *p);

/* Validate parameters, build the grids and coefficient tables of the
 * right-hand side of Eq. (eq:HEOM) on the host, and upload them once.
 *   dev_workspace: device memory of at least chfpe_workspace_bytes(p) bytes
 *     owned by the caller and kept alive until chfpe_destroy, or NULL to let
 *     the library allocate (and free in chfpe_destroy).
 *   hip_stream: a hipStream_t on the current device, or NULL for the null
 *     stream.
 *   out: receives the new context; untouched on error.
 * Errors: EINVAL (bad parameters; also a grid the p-block tile cannot cover,
 * see below, or a batch so large that one launch over all its states would
 * exceed a dispatch's 2^32 work-items), ENOMEM (workspace too small or
 * allocation failed), EDEVICE.
 * Tiling limit (M >= 2): the p block of every q point must fit one of two
 * tiles.  (a) The last two p axes, N_{M-1} x N_M points, as one LDS tile with
 * N_M threads per row group: N_{M-1} needs a divisor d with d * N_M <= 256 and
 * N_{M-1} <= 4 d (every size up to 16, and equal pairs of 18, 20-22, 24, 27,
 * 28 and 32).  (b) The whole block in one workgroup of one thread per
 * (p_2, p_3) point (two modes: per p_2 point) holding a p_1 line of at most 32
 * points (three modes) or 48 (two modes), with at most 512-768 threads and
 * the block in 160 KB of LDS.  Three modes take (b) wherever it fits, two
 * modes where (a) does not.  chfpe_workspace_bytes returns 0 when neither
 * fits. */
int chfpe_setup(const chfpe_params *p, void *dev_workspace, size_t ws_bytes, void *hip_stream,
                chfpe_ctx **out);

/* Equilibration (Sec. IV B): state <- W_0 = exp(-beta H_sys)/Z with
 * Z = integral of exp(-beta H_sys) (weighted midpoint rule, weights 1 except
 * 0.8 at both ends of every axis), W_{n != 0} = 0; then n_steps classical
 * RK4 steps of size dt; the result is kept as the equilibrium W_eq used by
 * the response functions.  n_steps >= 0, dt > 0 (dt may be 0 only when
 * n_steps == 0).  ENONFINITE if the state overflows. */
int chfpe_equilibrate(chfpe_ctx *ctx, int64_t n_steps, double dt);

/* n_steps classical RK4 steps of Eq. (eq:HEOM) on the context's current
 * state, in place.  ENONFINITE if the state became non-finite (it is then
 * unspecified). */
int chfpe_propagate(chfpe_ctx *ctx, int64_t n_steps, double dt);

/* Linear response, Eq. (1Dresponse):
 *   R[j] = integral A(q) W_0 of G(j * stride * dt) A^x W_eq,  j = 0..n_t-1,
 * with A^x W = sum_s dA/dq_s dW/dp_s on every element (Eq. (Opticalexc)).
 * R is a host array of n_t doubles.  Uses W_eq (ESTATE before
 * chfpe_equilibrate or chfpe_use_state_as_equilibrium); overwrites the
 * current state. */
int chfpe_response_1d(chfpe_ctx *ctx, const chfpe_optical *A, int64_t n_t, int32_t stride,
                      double dt, double *R);

/* Second-order response, Eq. (2Dresponse), by the t1/t2 double loop of
 * Sec. IV C:
 *   R[j2 * n_t1 + j1] = integral C W_0 of
 *       G(j2 * stride2 * dt) B^x G(j1 * stride1 * dt) A^x W_eq.
 * R is a host array of n_t2 * n_t1 doubles (t1 fastest).  The response
 * values are accumulated on the device and copied back once.  Uses W_eq;
 * overwrites the current state. */
int chfpe_response_2d(chfpe_ctx *ctx, const chfpe_optical *A, const chfpe_optical *B,
                      const chfpe_optical *C, int64_t n_t1, int64_t n_t2, int32_t stride1,
                      int32_t stride2, double dt, double *R);

/* Columns j1_begin <= j1 < j1_end of the same R (t1 = j1 stride1 dt):
 * R receives [n_t2][j1_end - j1_begin], t1 fastest.  U = A^x W_eq is first
 * advanced to the first column's t1 (j1_begin stride1 RK4 steps, FP64), so
 * the columns equal those of one chfpe_response_2d call over 0..j1_end
 * (bitwise for the FP64 path).  Ranges are the unit a caller spreads over
 * several calls (progress between them) or several devices (each its own
 * context).  Errors as for chfpe_response_2d; EINVAL also for
 * j1_begin < 0 or j1_end < j1_begin. */
int chfpe_response_2d_range(chfpe_ctx *ctx, const chfpe_optical *A, const chfpe_optical *B,
                            const chfpe_optical *C, int64_t j1_begin, int64_t j1_end, int64_t n_t2,
                            int32_t stride1, int32_t stride2, double dt, double *R);

/* Third-order response, Eq. (3Dresponse), at one waiting time
 * t2 = t2_steps * dt, for the 2D IR spectrum of Sec. IV C:
 *   R[j3 * n_t1 + j1] = integral D W_0 of
 *       G(j3 * stride3 * dt) C^x G(t2) B^x G(j1 * stride1 * dt) A^x W_eq.
 * R is a host array of n_t3 * n_t1 doubles (t1 fastest).  The t1 branches
 * run one after another on the FP64 single-state buffers whatever the
 * context's batch and precision.  Uses W_eq (ESTATE before equilibration);
 * overwrites the current state.  EINVAL for negative counts or strides, a
 * zero stride with more than one sample, or dt <= 0 with steps to take. */
int chfpe_response_3d(chfpe_ctx *ctx, const chfpe_optical *A, const chfpe_optical *B, const chfpe_optical *C,
                      const chfpe_optical *D, int64_t n_t1, int64_t t2_steps, int64_t n_t3, int32_t stride1,
                      int32_t stride3, double dt, double *R);

/* Number of values in a state: |{n : |n| <= K}| * prod_s Nq_s * Np_s. */
int64_t chfpe_state_count(const chfpe_ctx *ctx);

/* Copy the current state to / from a host array of chfpe_state_count
 * doubles in the canonical layout above. */
int chfpe_get_state(chfpe_ctx *ctx, double *host);
int chfpe_set_state(chfpe_ctx *ctx, const double *host);

/* Keep the current state as W_eq (lets a caller supply its own equilibrium). */
int chfpe_use_state_as_equilibrium(chfpe_ctx *ctx);

/* One evaluation of the right-hand side of Eq. (eq:HEOM) on the current
 * state; the result replaces the current state. */
int chfpe_rhs(chfpe_ctx *ctx);

/* Current state <- X^x (current state), Eq. (Opticalexc), every element. */
int chfpe_perturb(chfpe_ctx *ctx, const chfpe_optical *X);

/* *value = integral X(q) W_0(q, p) dq dp of the current state (weighted
 * midpoint rule as for Z above). */
int chfpe_observe(chfpe_ctx *ctx, const chfpe_optical *X, double *value);

/* Spectra of Eqs. (1DIR_Raman) and (2DThz_Raman) as discrete Fourier sums
 * on the device (rectangle rule, weight 1 at t = 0, no window or padding),
 * with omega_k = 2 pi k / (n tau):
 *   1D: I[k] = omega_k Im{ sum_j tau exp(+i omega_k t_j) R[j] },  t_j = j tau;
 *       omega (optional, may be NULL) receives omega_k.
 *   2D: I[k2 * n_t1 + k1] = Im{ tau1 tau2 sum_{j1,j2}
 *           exp(-i omega1_k1 t1_j1 - i omega2_k2 t2_j2) R[j2 * n_t1 + j1] }.
 * R, omega and I are host arrays; device scratch is allocated and freed per
 * call; the call synchronizes hip_stream (NULL: null stream). */
int chfpe_spectrum_1d(const double *R, int64_t n, double tau, double *omega, double *I,
                      void *hip_stream);
int chfpe_spectrum_2d(const double *R, int64_t n_t1, int64_t n_t2, double tau1, double tau2,
                      double *I, void *hip_stream);
/* 2D IR spectrum of a third-order response, Eq. (noncorrelation), at its
 * waiting time: R and I are [n_t3][n_t1] (t1 fastest) and
 *   I[k3 * n_t1 + k1] = Im{ tau1 tau3 sum_{j1,j3}
 *           exp(-i omega1_k1 t1_j1 + i omega3_k3 t3_j3) R[j3 * n_t1 + j1] },
 * same conventions, scratch and errors as chfpe_spectrum_2d. */
int chfpe_spectrum_2dir(const double *R, int64_t n_t1, int64_t n_t3, double tau1, double tau3,
                        double *I, void *hip_stream);

/* chfpe_spectrum_2d without device allocation, for callers that cannot
 * allocate (tight serving loops, harnesses that forbid hipMalloc): same
 * arguments, result and conventions, with every device buffer in a fixed
 * per-device scratch array of the library (48 bytes per point) instead of
 * per-call allocations.  n_t1 * n_t2 <= 131072 (EINVAL above).  Calls on one
 * GPU share that scratch: calls that overlap in time on one GPU (other host
 * threads, other streams) race and must be serialized by the caller.  The
 * call synchronizes hip_stream.  EDEVICE if the scratch address cannot be
 * resolved on the current device. */
int chfpe_spectrum_2d_noalloc(const double *R, int64_t n_t1, int64_t n_t2, double tau1, double tau2,
                              double *I, void *hip_stream);

/* Bandwidth reference: copy `bytes` bytes (a multiple of 16) from src to
 * dst, both device pointers, with a plain streaming kernel on hip_stream
 * (eight 16-byte loads in flight per thread, up to 64 workgroups per CU).
 * EINVAL for NULL pointers or a size that is not a multiple of 16. */
int chfpe_stream_copy(void *dst, const void *src, size_t bytes, void *hip_stream);

/* Bandwidth reference for other read/write mixes: dst[i] = a[i] + b[i] +
 * c[i] over the first nsrc of the sources (nsrc = 0..3; 0 writes zeros),
 * all device arrays of `bytes` bytes read as FP64 (a multiple of 16).  The
 * stage passes read two or three state arrays per one written; this kernel
 * moves the same mix with nothing else to do.  Sources past nsrc may be NULL.
 * EINVAL for nsrc out of range, a missing pointer or a bad size. */
int chfpe_stream_mix(void *dst, const void *a, const void *b, const void *c, int32_t nsrc, size_t bytes,
                     void *hip_stream);

/* Per-kernel timing with HIP events on the context's stream: every
 * `every`-th RK4 step (0 turns timing off) each launch of that step is
 * bracketed by events; while timing is on, 2D-response waves are issued
 * directly instead of as HIP graphs.  chfpe_kernel_times reports, for each
 * kernel kind, the number of timed launches, their mean duration in
 * milliseconds, their mean algorithmic bytes (each input state read once and
 * each output state written once) and the kind's name; launches that carry
 * several branch states are separate kinds ("batch_" names).  It
 * synchronizes the stream and returns the number of kinds written (at most
 * max_kinds).  Any output pointer may be NULL. */
int chfpe_set_kernel_timing(chfpe_ctx *ctx, int32_t every);
int chfpe_kernel_times(chfpe_ctx *ctx, int32_t max_kinds, int64_t *counts, double *mean_ms,
                       double *mean_bytes, const char **names);

/* Tile autotuner.  Times one RK4 step (after one untimed step), averaged
 * over n_steps (1..1000), for each candidate tile shape: first the k_pblock
 * shapes (blocks per task 1, 2, 4, 8 where the block fits, with and
 * without lane-pair line solves), then the q-pass tile widths 4, 8, 16, 32
 * (positions of the contiguous run per two-axis tile, as LDS allows) with
 * the best k_pblock shape, then the k_pblock task order (runs of 1, 4, 8,
 * 16, 32 consecutive block groups of one state before the next element).
 * Candidates whose launch would exceed one dispatch are skipped.  Every
 * candidate computes the same result.  The path timed is the one the context spends
 * most time in: the batched branch buffers (branch type) when batch > 1,
 * else the FP64 single-state path.  The fastest shape is kept by this
 * context and, for the rest of the process, by every later context of the
 * same shape (M, K, grid, precision, batch); CHFPE_TUNE_* environment
 * variables still override it.  Runs on scratch buffers only: the current
 * state and W_eq are unchanged; a cached 2D-response graph is dropped.
 * Synchronizes the stream.  EINVAL for n_steps out of range, EDEVICE if a
 * trial fails (the previous shapes are then kept). */
int chfpe_autotune(chfpe_ctx *ctx, int32_t n_steps);

/* The tile shapes in use: out[0] k_pblock blocks per task, out[1] 1 if
 * lines are solved by lane pairs, out[2] k_pblock threads per workgroup,
 * out[3] run positions per tile of the stage-final q-pass, out[4] the same
 * for the three-mode (q_2, q_3) pass (0 otherwise), out[5] threads of the
 * stage-final q-pass; out[6..8] the requests these came from (blocks per
 * task, lane pairs, run positions; 0, -1, 0 = planner default), which the
 * CHFPE_TUNE_PB_NB, CHFPE_TUNE_PB_SPLIT and CHFPE_TUNE_Q_PC environment
 * variables reproduce; out[9] the k_pblock task order (consecutive block
 * groups of one state before the next element) and out[10] its request
 * (0 = 1; CHFPE_TUNE_PB_RUN); out[11] 1 when one workgroup per q point takes
 * the whole p block (k_pcube; out[0], out[9] then describe no launch), out[12]
 * 1 when that kernel is the streamed form k_pcube_s (the default for p_1
 * axes up to 16 points; CHFPE_TUNE_PC_STREAM=0/1 forces either form).
 * Hermite basis: out[13] the k_hcube tasks per XCD chunk (the XCDs take
 * chunks of consecutive tasks in turn; 0: one contiguous range each) and
 * out[14] the width of the k_2 tiles of its task order (three modes; 1
 * otherwise), set by CHFPE_TUNE_HC_CHUNK and CHFPE_TUNE_HC_KTILE; 0 for the
 * grid basis.  The task order does not change any result.
 * Writes min(n, 15) values and returns that count. */
int chfpe_tile_config(const chfpe_ctx *ctx, int32_t *out, int32_t n);

/* ---- Learned per-axis closure (coarse grids) -------------------------------
 * The paper discretises every axis with the compact scheme of Sec. III B on
 * one grid.  A closure lets a coarse grid (half the points per axis of a fine
 * grid on the same box) stand in for the fine one: along each grid axis a,
 * the compact system A y = B f / h becomes A y = (B + S_a) f / h, with S_a
 * skew-symmetric on the first two off-diagonals (S[i][i+k] = -S[i+k][i] =
 * s, k = 1, 2), which keeps A D skew like the plain scheme.  The entries s are
 * the output of a network of one hidden layer (16 features -> 32 tanh units
 * -> 1; BF16 weights and activations in MFMA products, FP32 accumulation),
 * trained on this device against fine-grid states of the solver itself.
 * Rows of the network: one per (axis, entry), axes in id order (q_1..q_M,
 * p_1..p_M), entries S[i][i+k] for k = 1, 2 in turn, i < N_a - k.  Parameters (FP32, 577): W1[16][32], b1[32], W2[32], b2. */

/* Number of rows, sum over axes of 2 N_a - 3; EINVAL for invalid params. */
int32_t chfpe_closure_rows(const chfpe_params *coarse);

/* Features of every row (host, rows x 16 FP32): u, u^2 (u: the entry's
 * midpoint over the half box), |u|, [k == 2], [p axis], h / sigma (sigma: thermal
 * width, 1/(omega sqrt(beta m)) for q, sqrt(m/beta) for p), omega/1.6,
 * g3 sigma_q/(m omega^2), g4 sigma_q^2/(m omega^2), V_SL sigma_q / V_LL,
 * zeta, gamma, beta/2, m, [entry touches the box edge], 1.  axis_of_row
 * (may be NULL) receives each row's axis id. */
int chfpe_closure_features(const chfpe_params *coarse, float *feat, int32_t *axis_of_row);

/* Training statistics of the context's current state, which must be on a
 * fine grid (every axis even, 10..32 points): with x = R h (2:1 cell
 * averages), T = R(D_a h) and r = T - D_a^coarse x for every coarse line,
 * the loss sum ||r - A^{-1} S_a x / h||^2 of axis a is
 * s^T G_a s - 2 b_a^T s + c_a, compared with t_a = sum ||T||^2.  ADDS G_a
 * (P_a x P_a row-major, P_a = 2 N_a - 3, axes concatenated), b_a
 * (concatenated) and (c_a, t_a) (2 per axis) into the host arrays, so
 * calls over several states accumulate.  Uses the context's scratch
 * buffers (not the state or W_eq); synchronizes its stream. */
int chfpe_closure_moments(chfpe_ctx *fine, double *G, double *b, double *ct);

/* s for every row at parameters prm (host arrays). */
int chfpe_closure_eval(const float *prm, const float *feat, int32_t rows, float *s, void *hip_stream);

/* grad = d(sum_rows gs[row] s[row]) / d(prm) (host arrays; one forward and
 * backward pass, as in training). */
int chfpe_closure_grad(const float *prm, const float *feat, int32_t rows, const float *gs, float *grad,
                       void *hip_stream);

/* n_steps Adam steps (beta1 0.9, beta2 0.999, eps 1e-8, step lr) of the mean
 * over groups of (s^T G s - 2 b^T s + c) / t, all on the device in one
 * workgroup.  Group q owns rows [group_start[q], group_start[q+1]) (covering
 * 0..rows) with G (P_q x P_q, groups concatenated), b, and (c, t) in ct.
 * prm, adam_m, adam_v (577 each) are read and written back; adam_t0 is the
 * number of steps already taken; loss (n_steps, may be NULL) receives the
 * loss at the parameters each step starts from. */
int chfpe_closure_train(const float *feat, int32_t rows, int32_t n_groups, const int32_t *group_start,
                        const double *G, const double *b, const double *ct, float *prm, float *adam_m,
                        float *adam_v, int32_t adam_t0, int32_t n_steps, float lr, float *loss,
                        void *hip_stream);

/* Use the closure entries s (one per row, FP64) in every right-hand side and
 * excitation of this context from now on; NULL restores the plain scheme.
 * EINVAL unless the context holds FP64 states and every axis has at most
 * 16 points. */
int chfpe_set_closure(chfpe_ctx *ctx, const double *s);

/* Message of the last error on this context (or of the last failed
 * chfpe_setup on this thread when ctx is NULL); never NULL. */
const char *chfpe_last_error(const chfpe_ctx *ctx);

/* Release the context and any memory the library allocated. */
void chfpe_destroy(chfpe_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* CHFPE_H */
