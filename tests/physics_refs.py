"""Closed forms that pin the oracle, derived from the model's equations of motion.

None of these use the hierarchy or the grid: they come from the generalized
Langevin equation that the Drude bath of Eq. (eq:drude) with linear-linear
coupling produces (friction kernel m zeta gamma V_LL^2 e^{-gamma t}, bath
force f obeying df = -gamma f dt - zeta gamma V_LL p dt + sqrt(2 m zeta gamma^2/beta) dB),
from the Boltzmann distribution, and from plain Fourier sums.
"""
from __future__ import annotations

import numpy as np
from scipy import integrate
from scipy.linalg import expm


def chi_brownian(t, m, omega, zeta, gamma, V):
    """Impulse response of q for one harmonic mode with Drude friction.

    chi^(s) = (s + gamma) / (m [s^3 + gamma s^2 + (omega^2 + zeta gamma V^2) s + gamma omega^2]),
    inverted by residues at the three roots of the cubic.
    """
    c1 = omega ** 2 + zeta * gamma * V ** 2
    roots = np.roots([1.0, gamma, c1, gamma * omega ** 2])
    t = np.asarray(t, dtype=np.float64)
    out = np.zeros(t.shape, dtype=np.complex128)
    for r in roots:
        dP = 3 * r ** 2 + 2 * gamma * r + c1
        out += (r + gamma) * np.exp(r * t) / (m * dP)
    return np.real(out)


def linear_gle_matrix(w: dict):
    """Drift matrix of (q_1..q_M, p_1..p_M, f_1..f_M) for a harmonic potential
    with bilinear couplings g2 and LL coupling (mean dynamics of the GLE)."""
    M = w["M"]
    Kmat = np.zeros((M, M))
    for s in range(M):
        Kmat[s, s] = w["m"][s] * w["omega"][s] ** 2
        for t in range(s + 1, M):
            Kmat[s, t] += w["g2"][s][t]
            Kmat[t, s] += w["g2"][s][t]
    J = np.zeros((3 * M, 3 * M))
    for s in range(M):
        J[s, M + s] = 1.0 / w["m"][s]                     # dq/dt = p/m
        J[M + s, :M] = -Kmat[s]                           # dp/dt = -dU/dq + V f
        J[M + s, 2 * M + s] = w["VLL"][s]
        J[2 * M + s, 2 * M + s] = -w["gamma"][s]          # df/dt = -gamma f - zeta gamma V p
        J[2 * M + s, M + s] = -w["zeta"][s] * w["gamma"][s] * w["VLL"][s]
    return J


def linear_response_1d(w: dict, mu_lin, times):
    """R^(1)(t) = -sum_{s,s'} mu_s mu_s' chi_{s s'}(t) for the linear model,
    chi_{s s'}(t) = response of q_s to a unit momentum kick on mode s'."""
    M = w["M"]
    J = linear_gle_matrix(w)
    mu = np.asarray(mu_lin, dtype=np.float64)
    out = []
    for t in times:
        E = expm(J * t)
        Q = E[:M, M:2 * M]
        out.append(-mu @ Q @ mu)
    return np.array(out)


def lyapunov_moments(m, omega, zeta, gamma, V, beta, mean0, cov0, t):
    """Mean and covariance of (q, p, f) at time t for the one-mode linear SDE."""
    J = np.array([[0.0, 1.0 / m, 0.0],
                  [-m * omega ** 2, 0.0, V],
                  [0.0, -zeta * gamma * V, -gamma]])
    Q = np.diag([0.0, 0.0, 2.0 * m * zeta * gamma ** 2 / beta])
    n = 3
    L = np.kron(np.eye(n), J) + np.kron(J, np.eye(n))
    aug = np.zeros((n * n + 1, n * n + 1))
    aug[:n * n, :n * n] = L
    aug[:n * n, -1] = Q.reshape(-1)
    v = np.concatenate([np.asarray(cov0, dtype=np.float64).reshape(-1), [1.0]])
    cov = (expm(aug * t) @ v)[:n * n].reshape(n, n)
    mean = expm(J * t) @ np.asarray(mean0, dtype=np.float64)
    return mean, cov


def boltzmann_average_1d(U, g, beta, L):
    """<g(q)> under exp(-beta U(q)) on [-L, L], by adaptive quadrature."""
    num = integrate.quad(lambda q: g(q) * np.exp(-beta * U(q)), -L, L, epsabs=0, epsrel=1e-13,
                         limit=200)[0]
    den = integrate.quad(lambda q: np.exp(-beta * U(q)), -L, L, epsabs=0, epsrel=1e-13,
                         limit=200)[0]
    return num / den


# ---------------------------------------------------------------------------
# Gaussian closed forms of the nonlinear responses of the linear model
# ---------------------------------------------------------------------------
# For a harmonic potential (bilinear couplings allowed) with linear-linear
# system-bath coupling, the phase-space process x = (q, p, f) obeys the linear
# stochastic equation whose drift matrix is linear_gle_matrix(w), and its
# stationary density P_eq is Gaussian (Boltzmann in (q, p), f ~ N(0, m zeta
# gamma / beta) independent of them).  A density of the form poly(x) P_eq
# stays of that form: G(t)[p P_eq](x) = P_eq(x) E[p(x_0) | x_t = x] over the
# stationary process, a polynomial of the same degree.  The optical
# excitation maps poly * P_eq to poly' * P_eq, so every response function is
# a Gaussian expectation of polynomials, evaluated below by Isserlis' theorem.
# The hierarchy of Eq. (eq:HEOM) represents poly * P_eq exactly once its
# depth reaches the polynomial's degree in f.

class Poly:
    """Polynomial in variables x_0..x_{nv-1}: {sorted index tuple: coefficient}."""

    def __init__(self, terms=None):
        self.t = {} if terms is None else dict(terms)

    @staticmethod
    def const(c):
        return Poly({(): float(c)})

    @staticmethod
    def linear(vec, offset=0):
        return Poly({(offset + i,): float(v) for i, v in enumerate(vec) if v != 0.0})

    def __add__(self, other):
        out = dict(self.t)
        for k, v in other.t.items():
            out[k] = out.get(k, 0.0) + v
        return Poly(out)

    def scale(self, c):
        return Poly({k: c * v for k, v in self.t.items()})

    def __mul__(self, other):
        out = {}
        for k1, v1 in self.t.items():
            for k2, v2 in other.t.items():
                k = tuple(sorted(k1 + k2))
                out[k] = out.get(k, 0.0) + v1 * v2
        return Poly(out)

    def deriv(self, i):
        out = {}
        for k, v in self.t.items():
            c = k.count(i)
            if c:
                j = k.index(i)
                kk = k[:j] + k[j + 1:]
                out[kk] = out.get(kk, 0.0) + c * v
        return Poly(out)

    def degree(self):
        return max((len(k) for k in self.t), default=0)


def isserlis(idx, cov, memo):
    """E[prod_k z_{idx_k}] for a centred Gaussian z with covariance cov."""
    if len(idx) % 2:
        return 0.0
    if not idx:
        return 1.0
    key = tuple(sorted(idx))
    if key in memo:
        return memo[key]
    first, rest = key[0], key[1:]
    s = 0.0
    for j in range(len(rest)):
        c = cov[first, rest[j]]
        if c != 0.0:
            s += c * isserlis(rest[:j] + rest[j + 1:], cov, memo)
    memo[key] = s
    return s


def gauss_expect(P, cov):
    memo = {}
    return sum(v * isserlis(k, cov, memo) for k, v in P.t.items())


def stationary_covariance(w):
    """Covariance of (q, p, f) under P_eq for the linear model."""
    M = w["M"]
    Kmat = np.zeros((M, M))
    for s in range(M):
        Kmat[s, s] = w["m"][s] * w["omega"][s] ** 2
        for t in range(s + 1, M):
            Kmat[s, t] += w["g2"][s][t]
            Kmat[t, s] += w["g2"][s][t]
    S = np.zeros((3 * M, 3 * M))
    S[:M, :M] = np.linalg.inv(w["beta"] * Kmat)
    for s in range(M):
        S[M + s, M + s] = w["m"][s] / w["beta"]
        S[2 * M + s, 2 * M + s] = w["m"][s] * w["zeta"][s] * w["gamma"][s] / w["beta"]
    return S


def cond_expect(P, Mmat, Cc):
    """E[P(y) | x] with y = Mmat x + z, z ~ N(0, Cc) independent of x."""
    d = Mmat.shape[0]
    rows = [Poly.linear(Mmat[i]) for i in range(d)]
    out = Poly()
    memo = {}
    for k, v in P.t.items():
        n = len(k)
        for mask in range(1 << n):
            zi = [k[j] for j in range(n) if mask >> j & 1]
            ez = isserlis(zi, Cc, memo)
            if ez == 0.0:
                continue
            term = Poly.const(v * ez)
            for j in range(n):
                if not mask >> j & 1:
                    term = term * rows[k[j]]
            out = out + term
    return out


def optical_poly(X, M, offset=0):
    """X(q) = sum lin_s q_s + 1/2 sum quad_ss' q_s q_s' as a polynomial."""
    P = Poly.linear(X["lin"], offset)
    for s in range(M):
        for t in range(M):
            if X["quad"][s][t] != 0.0:
                P = P + Poly({tuple(sorted((offset + s, offset + t))): 0.5 * X["quad"][s][t]})
    return P


def excite(X, P, w):
    """Polynomial of X^x (P P_eq) / P_eq: sum_s dX/dq_s (dP/dp_s - P beta p_s / m_s)."""
    M = w["M"]
    Xp = optical_poly(X, M)
    out = Poly()
    for s in range(M):
        ps = M + s
        inner = P.deriv(ps) + (P * Poly.linear([1.0], ps)).scale(-w["beta"] / w["m"][s])
        out = out + Xp.deriv(s) * inner
    return out


def evolve(P, w, t, J, S, Sinv):
    """Polynomial of G(t)[P P_eq] / P_eq."""
    from scipy.linalg import expm as _expm
    E = _expm(J * t)
    Mmat = S @ E.T @ Sinv
    Cc = S - Mmat @ E @ S
    Cc = 0.5 * (Cc + Cc.T)
    return cond_expect(P, Mmat, Cc)


def response_2d_gaussian(w, A, B, C, t1s, t2s):
    """R[j2][j1] = <C>(G(t2_j2) B^x G(t1_j1) A^x W_eq), Eq. (2Dresponse), for
    the linear model (harmonic U with bilinear couplings, V_SL = 0)."""
    M = w["M"]
    J = linear_gle_matrix(w)
    S = stationary_covariance(w)
    Sinv = np.linalg.inv(S)
    pA = excite(A, Poly.const(1.0), w)
    Cp = optical_poly(C, M)
    d = 3 * M
    R = np.zeros((len(t2s), len(t1s)))
    from scipy.linalg import expm as _expm
    for j1, t1 in enumerate(t1s):
        g = excite(B, evolve(pA, w, t1, J, S, Sinv), w)
        for j2, t2 in enumerate(t2s):
            # E[C(x_t2) g(x_0)] over the stationary process: variables 0..d-1
            # are x_0, d..2d-1 are x_t2; Cov(x_t2, x_0) = e^{J t2} S
            E2S = _expm(J * t2) @ S
            cov = np.zeros((2 * d, 2 * d))
            cov[:d, :d] = S
            cov[d:, d:] = S
            cov[d:, :d] = E2S
            cov[:d, d:] = E2S.T
            R[j2, j1] = gauss_expect(Cp_shift(Cp, d) * g, cov)
    return R


def response_3d_gaussian(w, A, B, C, D, t1s, t2, t3s):
    """R[j3][j1] = <D>(G(t3_j3) C^x G(t2) B^x G(t1_j1) A^x W_eq), Eq. (3Dresponse),
    for the linear model: the chain of R^(2) with one more free propagation
    (the waiting time t2) and one more excitation."""
    M = w["M"]
    J = linear_gle_matrix(w)
    S = stationary_covariance(w)
    Sinv = np.linalg.inv(S)
    pA = excite(A, Poly.const(1.0), w)
    Dp = optical_poly(D, M)
    d = 3 * M
    R = np.zeros((len(t3s), len(t1s)))
    from scipy.linalg import expm as _expm
    for j1, t1 in enumerate(t1s):
        g = excite(C, evolve(excite(B, evolve(pA, w, t1, J, S, Sinv), w), w, t2, J, S, Sinv), w)
        for j3, t3 in enumerate(t3s):
            E3S = _expm(J * t3) @ S
            cov = np.zeros((2 * d, 2 * d))
            cov[:d, :d] = S
            cov[d:, d:] = S
            cov[d:, :d] = E3S
            cov[:d, d:] = E3S.T
            R[j3, j1] = gauss_expect(Cp_shift(Dp, d) * g, cov)
    return R


def Cp_shift(P, d):
    return Poly({tuple(i + d for i in k): v for k, v in P.t.items()})
