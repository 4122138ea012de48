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
