/*
 * chfpe_oracle.c -- plain, slow, FP64 CPU oracle for the multimode classical
 * hierarchical Fokker-Planck equations (CHFPE) hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg load this library.  It shares no code,
 * header, table or constant with the HIP library.
 *
 * What it computes, and where the paper defines it:
 *   - model: modes with U_s = m nu^2 q^2/2 + g3 q^3/3! (+ g4 q^4/4!),
 *     pair couplings U_ss' = g_ss' q q' + (g_{s^2s'} q^2 q' + g_{ss'^2} q q'^2)/6,
 *     system-bath coupling V_s = V_LL q + V_SL q^2/2            (Sec. II A)
 *   - hierarchy equation of motion, Eq. (eq:HEOM), with the Liouvillian
 *     of Eq. (eq:CL_liouville) and the operators Phi, Theta of Eqs.
 *     (eq:Phi), (eq:Theta); the Theta coupling into element n carries the
 *     factor n_s (the appendix form, Eq. (HEOM2FP-H), and the Fokker-Planck
 *     derivation of the Drude bath both have it)                (Sec. II B)
 *   - the factorization of Sec. III A: every element is written as
 *     W_n = exp(-beta H_sys / 2) h_n (the paper's e^{-beta U/2} psi_0(p)
 *     prefactor); the smooth factor h_n is what is discretized.  In h the
 *     hierarchy reads (L is unchanged because L exp(-beta H/2) = 0)
 *       dh_n/dt = L h_n - sum_s n_s gamma_s h_n
 *               + sum_s V_s' (d/dp_s - beta p_s / 2 m_s) h_{n+e_s}
 *               + sum_s n_s (m_s zeta_s gamma_s / beta) V_s' (d/dp_s + beta p_s / 2 m_s) h_{n-e_s}
 *   - the compact sixth-order first derivative A f' = B f / h with
 *     alpha = 1/3 and right-hand-side weights 7/9 on f_{i+1}-f_{i-1} and
 *     1/36 on f_{i+2}-f_{i-2}, applied to h; values outside the box are
 *     zero (Sec. III B).  The tridiagonal systems are solved by the Thomas
 *     algorithm (the paper uses parallel cyclic reduction, Sec. III C; both
 *     solve the same system).
 *   - the optical excitation X^x W = sum_s dX/dq_s dW/dp_s, Eq. (Opticalexc)
 *   - response functions, Eqs. (1Dresponse) and (2Dresponse), with the
 *     equilibrium obtained by propagation (Sec. IV B) and the t1/t2 double
 *     loop of Sec. IV C.
 * Readings where the paper is silent (grid centring, quadrature weights,
 * integrator, element order) are listed in the design doc; in short: cell-centred
 * uniform grids, quadrature weights 1 except 0.8 at both ends of each axis,
 * classical RK4 with fixed dt, elements {n : |n| <= K} in graded
 * lexicographic order.
 *
 * Layout of a state: W[e][q_1..q_M][p_1..p_M], C order, p_M fastest.
 * States passed in and out are W; the right-hand side and the excitation
 * convert to h internally and back.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
  int32_t M, K;
  int32_t Nq[3], Np[3];
  double Lq[3], Lp[3];
  double m[3], omega[3], g3[3], g4[3];
  double g2[3][3], g21[3][3], g12[3][3];
  double VLL[3], VSL[3];
  double zeta[3], gamma[3];
  double beta;
} orc_params;

typedef struct {
  double lin[3];
  double quad[3][3];
} orc_optical;

/* ------------------------------------------------------------------ */
/* hierarchy index set                                                  */
/* ------------------------------------------------------------------ */

/* Enumerate {n in N^M : |n| <= K}: by |n| ascending, then lexicographically
 * descending (n_1 largest first).  Writes M ints per element into out (may
 * be NULL); returns the count. */
static int enum_rec(int M, int s, int left, int *cur, int *out, int count) {
  if (s == M - 1) {
    cur[s] = left;
    if (out) memcpy(out + (size_t)count * M, cur, sizeof(int) * M);
    return count + 1;
  }
  for (int v = left; v >= 0; --v) {
    cur[s] = v;
    count = enum_rec(M, s + 1, left - v, cur, out, count);
  }
  return count;
}

int orc_elements(const orc_params *P, int *out) {
  int cur[3] = {0, 0, 0};
  int count = 0;
  for (int d = 0; d <= P->K; ++d) count = enum_rec(P->M, 0, d, cur, out, count);
  return count;
}

static int find_element(const int *nvec, int ne, int M, const int *want) {
  for (int e = 0; e < ne; ++e) {
    int ok = 1;
    for (int s = 0; s < M; ++s)
      if (nvec[e * M + s] != want[s]) ok = 0;
    if (ok) return e;
  }
  return -1;
}

/* ------------------------------------------------------------------ */
/* grids                                                                */
/* ------------------------------------------------------------------ */

/* dims[0..M-1] = Nq, dims[M..2M-1] = Np */
static void get_dims(const orc_params *P, int *dims) {
  for (int s = 0; s < P->M; ++s) {
    dims[s] = P->Nq[s];
    dims[P->M + s] = P->Np[s];
  }
}

static int64_t element_size(const orc_params *P) {
  int64_t n = 1;
  for (int s = 0; s < P->M; ++s) n *= (int64_t)P->Nq[s] * P->Np[s];
  return n;
}

int64_t orc_points(const orc_params *P) { return element_size(P); }

/* cell-centred grid point i of an axis of N points on [-L, L] */
static double coord(int i, int N, double L) { return -L + (i + 0.5) * (2.0 * L / N); }

/* quadrature weight of point i on an axis of N points */
static double qweight(int i, int N) { return (i == 0 || i == N - 1) ? 0.8 : 1.0; }

/* decompose a point index into its 2M axis indices (p_M fastest) */
static void unravel(int64_t idx, const int *dims, int nd, int *ix) {
  for (int d = nd - 1; d >= 0; --d) {
    ix[d] = (int)(idx % dims[d]);
    idx /= dims[d];
  }
}

/* ------------------------------------------------------------------ */
/* model functions (Sec. II A)                                          */
/* ------------------------------------------------------------------ */

/* U(q) */
double orc_potential(const orc_params *P, const double *q) {
  double u = 0.0;
  for (int s = 0; s < P->M; ++s) {
    double x = q[s];
    u += 0.5 * P->m[s] * P->omega[s] * P->omega[s] * x * x + P->g3[s] * x * x * x / 6.0 +
         P->g4[s] * x * x * x * x / 24.0;
  }
  for (int s = 0; s < P->M; ++s)
    for (int t = s + 1; t < P->M; ++t)
      u += P->g2[s][t] * q[s] * q[t] +
           (P->g21[s][t] * q[s] * q[s] * q[t] + P->g12[s][t] * q[s] * q[t] * q[t]) / 6.0;
  return u;
}

/* dU/dq_s */
double orc_force(const orc_params *P, const double *q, int s) {
  double x = q[s];
  double f = P->m[s] * P->omega[s] * P->omega[s] * x + P->g3[s] * x * x / 2.0 +
             P->g4[s] * x * x * x / 6.0;
  for (int a = 0; a < P->M; ++a)
    for (int b = a + 1; b < P->M; ++b) {
      if (a == s)
        f += P->g2[a][b] * q[b] + (2.0 * P->g21[a][b] * q[a] * q[b] + P->g12[a][b] * q[b] * q[b]) / 6.0;
      if (b == s)
        f += P->g2[a][b] * q[a] + (P->g21[a][b] * q[a] * q[a] + 2.0 * P->g12[a][b] * q[a] * q[b]) / 6.0;
    }
  return f;
}

/* dV_s/dq_s for V_s = V_LL q + V_SL q^2 / 2 */
static double dV(const orc_params *P, int s, double x) { return P->VLL[s] + P->VSL[s] * x; }

/* exp(-beta H_sys(q, p) / 2): W_n = factor * h_n */
static double sym_factor(const orc_params *P, const double *q, const double *p) {
  double H = orc_potential(P, q);
  for (int s = 0; s < P->M; ++s) H += p[s] * p[s] / (2.0 * P->m[s]);
  return exp(-0.5 * P->beta * H);
}

/* dX/dq_s for X(q) = sum lin_s q_s + 1/2 sum_{s,s'} quad_ss' q_s q_s' */
double orc_optical_grad(const orc_params *P, const orc_optical *X, const double *q, int s) {
  double g = X->lin[s];
  for (int t = 0; t < P->M; ++t) g += 0.5 * (X->quad[s][t] + X->quad[t][s]) * q[t];
  return g;
}

double orc_optical_value(const orc_params *P, const orc_optical *X, const double *q) {
  double v = 0.0;
  for (int s = 0; s < P->M; ++s) {
    v += X->lin[s] * q[s];
    for (int t = 0; t < P->M; ++t) v += 0.5 * X->quad[s][t] * q[s] * q[t];
  }
  return v;
}

/* ------------------------------------------------------------------ */
/* compact sixth-order first derivative (Sec. III B)                    */
/* ------------------------------------------------------------------ */

/* y = A^{-1} B f / h on one line of N points; zero values outside the box. */
void orc_deriv_line(int N, double h, const double *f, double *y) {
  const double alpha = 1.0 / 3.0, a = 7.0 / 9.0, b = 1.0 / 36.0;
  double *cp = (double *)malloc(sizeof(double) * N);
  double *dp = (double *)malloc(sizeof(double) * N);
  for (int i = 0; i < N; ++i) {
    double fm2 = (i - 2 >= 0) ? f[i - 2] : 0.0;
    double fm1 = (i - 1 >= 0) ? f[i - 1] : 0.0;
    double fp1 = (i + 1 < N) ? f[i + 1] : 0.0;
    double fp2 = (i + 2 < N) ? f[i + 2] : 0.0;
    double r = (a * (fp1 - fm1) + b * (fp2 - fm2)) / h;
    /* Thomas forward elimination on tridiag(alpha, 1, alpha) */
    if (i == 0) {
      cp[0] = alpha;
      dp[0] = r;
    } else {
      double den = 1.0 - alpha * cp[i - 1];
      cp[i] = alpha / den;
      dp[i] = (r - alpha * dp[i - 1]) / den;
    }
  }
  y[N - 1] = dp[N - 1];
  for (int i = N - 2; i >= 0; --i) y[i] = dp[i] - cp[i] * y[i + 1];
  free(cp);
  free(dp);
}

/* Derivative along axis `ax` of an array with dims[0..nd-1] (C order). */
static void deriv_axis(const int *dims, int nd, int ax, double h, const double *in, double *out) {
  int64_t stride = 1;
  for (int d = ax + 1; d < nd; ++d) stride *= dims[d];
  int64_t total = 1;
  for (int d = 0; d < nd; ++d) total *= dims[d];
  int N = dims[ax];
  int64_t nlines = total / N;
#pragma omp parallel
  {
    double *f = (double *)malloc(sizeof(double) * N);
    double *y = (double *)malloc(sizeof(double) * N);
#pragma omp for schedule(static)
    for (int64_t l = 0; l < nlines; ++l) {
      int64_t base = (l / stride) * stride * N + (l % stride);
      for (int i = 0; i < N; ++i) f[i] = in[base + i * stride];
      orc_deriv_line(N, h, f, y);
      for (int i = 0; i < N; ++i) out[base + i * stride] = y[i];
    }
    free(f);
    free(y);
  }
}

/* ------------------------------------------------------------------ */
/* per-point coordinate tables                                          */
/* ------------------------------------------------------------------ */

typedef struct {
  int nd;
  int dims[6];
  int64_t E; /* points per element */
  double hq[3], hp[3];
} geom;

static void make_geom(const orc_params *P, geom *g) {
  g->nd = 2 * P->M;
  get_dims(P, g->dims);
  g->E = element_size(P);
  for (int s = 0; s < P->M; ++s) {
    g->hq[s] = 2.0 * P->Lq[s] / P->Nq[s];
    g->hp[s] = 2.0 * P->Lp[s] / P->Np[s];
  }
}

static void point_coords(const orc_params *P, const geom *g, int64_t idx, double *q, double *p) {
  int ix[6];
  unravel(idx, g->dims, g->nd, ix);
  for (int s = 0; s < P->M; ++s) {
    q[s] = coord(ix[s], P->Nq[s], P->Lq[s]);
    p[s] = coord(ix[P->M + s], P->Np[s], P->Lp[s]);
  }
}

/* ------------------------------------------------------------------ */
/* right-hand side of Eq. (eq:HEOM)                                     */
/* ------------------------------------------------------------------ */

/* h = W / exp(-beta H/2) for every element */
static void to_h(const orc_params *P, const geom *g, int ne, const double *W, double *h) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < g->E; ++i) {
    double q[3], p[3];
    point_coords(P, g, i, q, p);
    const double f = sym_factor(P, q, p);
    for (int e = 0; e < ne; ++e) h[(int64_t)e * g->E + i] = W[(int64_t)e * g->E + i] / f;
  }
}

/* out = exp(-beta H/2) * out for every element */
static void from_h(const orc_params *P, const geom *g, int ne, double *out) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < g->E; ++i) {
    double q[3], p[3];
    point_coords(P, g, i, q, p);
    const double f = sym_factor(P, q, p);
    for (int e = 0; e < ne; ++e) out[(int64_t)e * g->E + i] *= f;
  }
}

void orc_rhs(const orc_params *P, const double *W, double *out) {
  geom g;
  make_geom(P, &g);
  const int M = P->M;
  int nvec[3 * 512];
  int ne = orc_elements(P, nvec);
  const int64_t E = g.E;
  double *tmp = (double *)malloc(sizeof(double) * E);
  double *h = (double *)malloc(sizeof(double) * E * ne);
  to_h(P, &g, ne, W, h);

  for (int e = 0; e < ne; ++e) {
    const int *n = nvec + e * M;
    const double *he = h + (int64_t)e * E;
    double *oe = out + (int64_t)e * E;
    memset(oe, 0, sizeof(double) * E);

    /* L h_n = {H_sys, h_n} = sum_s dU/dq_s dh/dp_s - (p_s/m_s) dh/dq_s */
    for (int s = 0; s < M; ++s) {
      deriv_axis(g.dims, g.nd, M + s, g.hp[s], he, tmp);
#pragma omp parallel for schedule(static)
      for (int64_t i = 0; i < E; ++i) {
        double q[3], p[3];
        point_coords(P, &g, i, q, p);
        oe[i] += orc_force(P, q, s) * tmp[i];
      }
      deriv_axis(g.dims, g.nd, s, g.hq[s], he, tmp);
#pragma omp parallel for schedule(static)
      for (int64_t i = 0; i < E; ++i) {
        double q[3], p[3];
        point_coords(P, &g, i, q, p);
        oe[i] -= (p[s] / P->m[s]) * tmp[i];
      }
    }

    /* - sum_s n_s gamma_s h_n */
    double damp = 0.0;
    for (int s = 0; s < M; ++s) damp += n[s] * P->gamma[s];
    if (damp != 0.0) {
#pragma omp parallel for schedule(static)
      for (int64_t i = 0; i < E; ++i) oe[i] -= damp * he[i];
    }

    /* + sum_s Phi_s h_{n+e_s},  Phi_s -> V_s'(q_s) (d/dp_s - beta p_s / 2 m_s) */
    for (int s = 0; s < M; ++s) {
      int up[3] = {0, 0, 0};
      for (int t = 0; t < M; ++t) up[t] = n[t] + (t == s);
      int eu = find_element(nvec, ne, M, up);
      if (eu < 0) continue; /* outside the truncated set: W = 0 */
      const double *hu = h + (int64_t)eu * E;
      deriv_axis(g.dims, g.nd, M + s, g.hp[s], hu, tmp);
      const double bm = P->beta / (2.0 * P->m[s]);
#pragma omp parallel for schedule(static)
      for (int64_t i = 0; i < E; ++i) {
        double q[3], p[3];
        point_coords(P, &g, i, q, p);
        oe[i] += dV(P, s, q[s]) * (tmp[i] - bm * p[s] * hu[i]);
      }
    }

    /* + sum_s n_s Theta_s h_{n-e_s},
     *   Theta_s -> (m_s zeta_s gamma_s / beta) V_s' (d/dp_s + beta p_s / 2 m_s) */
    for (int s = 0; s < M; ++s) {
      if (n[s] == 0) continue;
      int dn[3] = {0, 0, 0};
      for (int t = 0; t < M; ++t) dn[t] = n[t] - (t == s);
      int ed = find_element(nvec, ne, M, dn);
      const double *hd = h + (int64_t)ed * E;
      deriv_axis(g.dims, g.nd, M + s, g.hp[s], hd, tmp);
      const double c1 = P->m[s] * P->zeta[s] * P->gamma[s] / P->beta;
      const double bm = P->beta / (2.0 * P->m[s]);
      const double ns = (double)n[s];
#pragma omp parallel for schedule(static)
      for (int64_t i = 0; i < E; ++i) {
        double q[3], p[3];
        point_coords(P, &g, i, q, p);
        oe[i] += ns * c1 * dV(P, s, q[s]) * (tmp[i] + bm * p[s] * hd[i]);
      }
    }
  }
  from_h(P, &g, ne, out);
  free(tmp);
  free(h);
}

/* The right-hand side at one point (element e, point index idx), computed
 * from the lines through that point only.  Same formulas as orc_rhs. */
double orc_rhs_point(const orc_params *P, const double *W, int e, int64_t idx) {
  geom g;
  make_geom(P, &g);
  const int M = P->M;
  int nvec[3 * 512];
  int ne = orc_elements(P, nvec);
  const int64_t E = g.E;
  const int *n = nvec + e * M;
  int ix[6];
  unravel(idx, g.dims, g.nd, ix);
  double q[3], p[3];
  point_coords(P, &g, idx, q, p);

  double f[64], y[64];
  /* derivative along axis ax of h of element ee, evaluated at this point */
#define LINE_DERIV(ee, ax, hh, result)                                        \
  do {                                                                        \
    int64_t st = 1;                                                           \
    for (int d = (ax) + 1; d < g.nd; ++d) st *= g.dims[d];                    \
    int64_t base = idx - (int64_t)ix[ax] * st;                                \
    const double *src = W + (int64_t)(ee) * E;                                \
    for (int i = 0; i < g.dims[ax]; ++i) {                                    \
      double qq[3], pp[3];                                                    \
      point_coords(P, &g, base + i * st, qq, pp);                             \
      f[i] = src[base + i * st] / sym_factor(P, qq, pp);                      \
    }                                                                         \
    orc_deriv_line(g.dims[ax], (hh), f, y);                                   \
    (result) = y[ix[ax]];                                                     \
  } while (0)

  const double fac = sym_factor(P, q, p);
  double acc = 0.0, d;
  for (int s = 0; s < M; ++s) {
    LINE_DERIV(e, M + s, g.hp[s], d);
    acc += orc_force(P, q, s) * d;
    LINE_DERIV(e, s, g.hq[s], d);
    acc -= (p[s] / P->m[s]) * d;
  }
  double damp = 0.0;
  for (int s = 0; s < M; ++s) damp += n[s] * P->gamma[s];
  acc -= damp * W[(int64_t)e * E + idx] / fac;
  for (int s = 0; s < M; ++s) {
    int up[3] = {0, 0, 0};
    for (int t = 0; t < M; ++t) up[t] = n[t] + (t == s);
    int eu = find_element(nvec, ne, M, up);
    if (eu < 0) continue;
    LINE_DERIV(eu, M + s, g.hp[s], d);
    const double hu = W[(int64_t)eu * E + idx] / fac;
    acc += dV(P, s, q[s]) * (d - P->beta / (2.0 * P->m[s]) * p[s] * hu);
  }
  for (int s = 0; s < M; ++s) {
    if (n[s] == 0) continue;
    int dn[3] = {0, 0, 0};
    for (int t = 0; t < M; ++t) dn[t] = n[t] - (t == s);
    int ed = find_element(nvec, ne, M, dn);
    LINE_DERIV(ed, M + s, g.hp[s], d);
    const double hd = W[(int64_t)ed * E + idx] / fac;
    acc += n[s] * P->m[s] * P->zeta[s] * P->gamma[s] / P->beta * dV(P, s, q[s]) *
           (d + P->beta / (2.0 * P->m[s]) * p[s] * hd);
  }
#undef LINE_DERIV
  return acc * fac;
}

/* ------------------------------------------------------------------ */
/* classical fourth-order Runge-Kutta, fixed dt                         */
/* ------------------------------------------------------------------ */

int64_t orc_state_size(const orc_params *P) {
  return (int64_t)orc_elements(P, NULL) * element_size(P);
}

void orc_rk4(const orc_params *P, double *y, int64_t nsteps, double dt) {
  int64_t S = orc_state_size(P);
  double *k1 = (double *)malloc(sizeof(double) * S);
  double *k2 = (double *)malloc(sizeof(double) * S);
  double *k3 = (double *)malloc(sizeof(double) * S);
  double *k4 = (double *)malloc(sizeof(double) * S);
  double *x = (double *)malloc(sizeof(double) * S);
  for (int64_t step = 0; step < nsteps; ++step) {
    orc_rhs(P, y, k1);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < S; ++i) x[i] = y[i] + 0.5 * dt * k1[i];
    orc_rhs(P, x, k2);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < S; ++i) x[i] = y[i] + 0.5 * dt * k2[i];
    orc_rhs(P, x, k3);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < S; ++i) x[i] = y[i] + dt * k3[i];
    orc_rhs(P, x, k4);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < S; ++i) y[i] += dt / 6.0 * (k1[i] + 2.0 * k2[i] + 2.0 * k3[i] + k4[i]);
  }
  free(k1);
  free(k2);
  free(k3);
  free(k4);
  free(x);
}

/* ------------------------------------------------------------------ */
/* equilibrium, excitation, observable                                  */
/* ------------------------------------------------------------------ */

static double point_weight(const orc_params *P, const geom *g, int64_t idx) {
  int ix[6];
  unravel(idx, g->dims, g->nd, ix);
  double w = 1.0;
  for (int d = 0; d < g->nd; ++d) w *= qweight(ix[d], g->dims[d]);
  return w;
}

static double cell_volume(const orc_params *P, const geom *g) {
  double v = 1.0;
  for (int s = 0; s < P->M; ++s) v *= g->hq[s] * g->hp[s];
  return v;
}

/* W_0 = exp(-beta H_sys) / Z, W_{n != 0} = 0, Z the quadrature of exp(-beta H_sys) */
void orc_boltzmann(const orc_params *P, double *W) {
  geom g;
  make_geom(P, &g);
  int64_t S = orc_state_size(P);
  memset(W, 0, sizeof(double) * S);
  double Z = 0.0;
  for (int64_t i = 0; i < g.E; ++i) {
    double q[3], p[3];
    point_coords(P, &g, i, q, p);
    double H = orc_potential(P, q);
    for (int s = 0; s < P->M; ++s) H += p[s] * p[s] / (2.0 * P->m[s]);
    W[i] = exp(-P->beta * H);
    Z += point_weight(P, &g, i) * W[i];
  }
  Z *= cell_volume(P, &g);
  for (int64_t i = 0; i < g.E; ++i) W[i] /= Z;
}

void orc_equilibrate(const orc_params *P, double *W, int64_t nsteps, double dt) {
  orc_boltzmann(P, W);
  orc_rk4(P, W, nsteps, dt);
}

/* (X^x W)_n = sum_s dX/dq_s dW_n/dp_s for every element n; with W = exp(-beta H/2) h
 * this is exp(-beta H/2) sum_s dX/dq_s (d/dp_s - beta p_s / 2 m_s) h_n */
void orc_perturb(const orc_params *P, const orc_optical *X, const double *W, double *out) {
  geom g;
  make_geom(P, &g);
  int ne = orc_elements(P, NULL);
  double *tmp = (double *)malloc(sizeof(double) * g.E);
  double *h = (double *)malloc(sizeof(double) * g.E * ne);
  to_h(P, &g, ne, W, h);
  for (int e = 0; e < ne; ++e) {
    const double *he = h + (int64_t)e * g.E;
    double *oe = out + (int64_t)e * g.E;
    memset(oe, 0, sizeof(double) * g.E);
    for (int s = 0; s < P->M; ++s) {
      deriv_axis(g.dims, g.nd, P->M + s, g.hp[s], he, tmp);
      const double bm = P->beta / (2.0 * P->m[s]);
#pragma omp parallel for schedule(static)
      for (int64_t i = 0; i < g.E; ++i) {
        double q[3], p[3];
        point_coords(P, &g, i, q, p);
        oe[i] += orc_optical_grad(P, X, q, s) * (tmp[i] - bm * p[s] * he[i]);
      }
    }
  }
  from_h(P, &g, ne, out);
  free(tmp);
  free(h);
}

/* <X>(W) = integral dq dp X(q) W_0(q, p) by the weighted midpoint rule */
double orc_observe(const orc_params *P, const orc_optical *X, const double *W) {
  geom g;
  make_geom(P, &g);
  double sum = 0.0;
  for (int64_t i = 0; i < g.E; ++i) {
    double q[3], p[3];
    point_coords(P, &g, i, q, p);
    sum += point_weight(P, &g, i) * orc_optical_value(P, X, q) * W[i];
  }
  return sum * cell_volume(P, &g);
}

/* integral of W_0 times 1, q_s, p_s, q_s^2, p_s^2, q_s p_s (mode s) */
void orc_moments(const orc_params *P, const double *W, int e, int s, double *mom6) {
  geom g;
  make_geom(P, &g);
  for (int k = 0; k < 6; ++k) mom6[k] = 0.0;
  const double *We = W + (int64_t)e * g.E;
  for (int64_t i = 0; i < g.E; ++i) {
    double q[3], p[3];
    point_coords(P, &g, i, q, p);
    double w = point_weight(P, &g, i) * We[i];
    mom6[0] += w;
    mom6[1] += w * q[s];
    mom6[2] += w * p[s];
    mom6[3] += w * q[s] * q[s];
    mom6[4] += w * p[s] * p[s];
    mom6[5] += w * q[s] * p[s];
  }
  double cv = cell_volume(P, &g);
  for (int k = 0; k < 6; ++k) mom6[k] *= cv;
}

/* integral of H_sys W_0 */
double orc_energy(const orc_params *P, const double *W) {
  geom g;
  make_geom(P, &g);
  double sum = 0.0;
  for (int64_t i = 0; i < g.E; ++i) {
    double q[3], p[3];
    point_coords(P, &g, i, q, p);
    double H = orc_potential(P, q);
    for (int s = 0; s < P->M; ++s) H += p[s] * p[s] / (2.0 * P->m[s]);
    sum += point_weight(P, &g, i) * H * W[i];
  }
  return sum * cell_volume(P, &g);
}

/* ------------------------------------------------------------------ */
/* response functions, Eqs. (1Dresponse), (2Dresponse), (3Dresponse)   */
/* ------------------------------------------------------------------ */

/* R[j] = <A>( G(j*stride*dt) A^x W_eq ),  j = 0..nt-1 */
void orc_response_1d(const orc_params *P, const orc_optical *A, const double *Weq, int64_t nt,
                     int stride, double dt, double *R) {
  int64_t S = orc_state_size(P);
  double *u = (double *)malloc(sizeof(double) * S);
  orc_perturb(P, A, Weq, u);
  for (int64_t j = 0; j < nt; ++j) {
    if (j > 0) orc_rk4(P, u, stride, dt);
    R[j] = orc_observe(P, A, u);
  }
  free(u);
}

/* R[j2 * nt1 + j1] = <C>( G(j2*s2*dt) B^x G(j1*s1*dt) A^x W_eq ) for the
 * listed t1 indices j1 (all of 0..nt1-1 when j1_list is NULL). */
/* j1_list, when given, must be ascending. */
void orc_response_2d(const orc_params *P, const orc_optical *A, const orc_optical *B,
                     const orc_optical *C, const double *Weq, int64_t nt1, int64_t nt2, int s1,
                     int s2, double dt, const int64_t *j1_list, int64_t n_j1, double *R) {
  int64_t S = orc_state_size(P);
  double *u = (double *)malloc(sizeof(double) * S);
  double *v = (double *)malloc(sizeof(double) * S);
  orc_perturb(P, A, Weq, u);
  int64_t done = 0; /* t1 steps already applied to u */
  int64_t count = j1_list ? n_j1 : nt1;
  for (int64_t c = 0; c < count; ++c) {
    int64_t j1 = j1_list ? j1_list[c] : c;
    if (j1 * s1 > done) {
      orc_rk4(P, u, j1 * s1 - done, dt);
      done = j1 * s1;
    }
    orc_perturb(P, B, u, v);
    for (int64_t j2 = 0; j2 < nt2; ++j2) {
      if (j2 > 0) orc_rk4(P, v, s2, dt);
      R[j2 * nt1 + j1] = orc_observe(P, C, v);
    }
  }
  free(u);
  free(v);
}

/* Third-order response, Eq. (3Dresponse), at one waiting time t2:
 *   R[j3 * nt1 + j1] = <D>( G(j3*s3*dt) C^x G(t2_steps*dt) B^x G(j1*s1*dt) A^x W_eq )
 * for the listed t1 indices j1 (all of 0..nt1-1 when j1_list is NULL;
 * j1_list ascending).  Each branch follows the excitations and free
 * propagations of the equation from right to left. */
void orc_response_3d(const orc_params *P, const orc_optical *A, const orc_optical *B,
                     const orc_optical *C, const orc_optical *D, const double *Weq, int64_t nt1,
                     int64_t t2_steps, int64_t nt3, int s1, int s3, double dt, const int64_t *j1_list,
                     int64_t n_j1, double *R) {
  int64_t S = orc_state_size(P);
  double *u = (double *)malloc(sizeof(double) * S);
  double *v = (double *)malloc(sizeof(double) * S);
  double *x = (double *)malloc(sizeof(double) * S);
  orc_perturb(P, A, Weq, u);
  int64_t done = 0; /* t1 steps already applied to u */
  int64_t count = j1_list ? n_j1 : nt1;
  for (int64_t c = 0; c < count; ++c) {
    int64_t j1 = j1_list ? j1_list[c] : c;
    if (j1 * s1 > done) {
      orc_rk4(P, u, j1 * s1 - done, dt);
      done = j1 * s1;
    }
    orc_perturb(P, B, u, v);
    orc_rk4(P, v, t2_steps, dt);
    orc_perturb(P, C, v, x);
    for (int64_t j3 = 0; j3 < nt3; ++j3) {
      if (j3 > 0) orc_rk4(P, x, s3, dt);
      R[j3 * nt1 + j1] = orc_observe(P, D, x);
    }
  }
  free(u);
  free(v);
  free(x);
}

int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
