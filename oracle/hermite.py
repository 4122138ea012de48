"""Hermite-function form of the CHFPE -- TEST INFRASTRUCTURE.

Only ``tests/`` and the smoke check use this module; the HIP path never does.
Plain FP64 numpy, written for small grids (dense derivative matrices, loops
over hierarchy elements).

The paper's own discretisation (Sec. III A; Appendix A, Eq. (HEOM2FP-H))
expands each element in Hermite functions of the momenta,

    W_n(q, p) = e^{-beta U(q)/2} prod_s psi_0(p_s) sum_k c_{n,k}(q) prod_s psi_{k_s}(p_s),

    psi_j(p) = (2^j j! a sqrt(pi))^{-1/2} H_j(p/a) e^{-p^2/(2 a^2)},  a_s = sqrt(2 m_s / beta),

and evolves the coefficients c_{n,k}(q) on the q grid only.  Per mode s,
with k_s < Nh_s (the truncation; c = 0 beyond it) and n_s < 0 or n outside
the hierarchy meaning zero:

    dc_{n,k}/dt = - sum_s n_s gamma_s c_{n,k}
        + sum_s [ sqrt(k_s+1) D+_s c_{n,k+e_s} - sqrt(k_s) D-_s c_{n,k-e_s} ]
        - sum_s sqrt(2 k_s)/a_s V_s'(q_s) c_{n+e_s,k-e_s}
        + sum_s n_s zeta_s gamma_s (m_s/beta) sqrt(2 (k_s+1))/a_s V_s'(q_s) c_{n-e_s,k+e_s},

    D+-_s = F_s(q) / (sqrt(2) a_s) -+ a_s / (sqrt(2) m_s) d/dq_s,

F_s = dU/dq_s.  This is Eq. (HEOM2FP-H) with D^{+-}, Theta and Phi of the
appendix written out (a_s / sqrt(2) = sqrt(m_s k_B T)), and it is also what
the p-grid hierarchy of the h-form (W_n = e^{-beta H/2} h_n) becomes when
h_n is expanded in psi_k: (d/dp - p/a^2) raises k with factor
-sqrt(2(k+1))/a and (d/dp + p/a^2) lowers it with sqrt(2k)/a.  The
q derivatives are the compact sixth-order scheme of Sec. III B (values
outside the box are zero).  Excitation, Eq. (Opticalexc), raises k:
(X^x c)_{n,k} = - sum_s dX/dq_s sqrt(2 k_s)/a_s c_{n,k-e_s}.  Observables
integrate p exactly: <X> = int dq X(q) e^{-beta U/2} c_{0,0}(q) (weighted
midpoint rule in q, weights 1 except 0.8 at both ends).  The Boltzmann
state is c_{0,0} = e^{-beta U/2} / Z_q, Z_q = int dq e^{-beta U}, all
other coefficients zero.

State layout: C[e][k_1..k_M][q_1..q_M], C order (q_M fastest); the grid
oracle's Np[s] is read as Nh_s, the number of Hermite functions of mode s.
"""
from __future__ import annotations

from math import sqrt

import numpy as np

from . import elements, force, potential


def width(w: dict, s: int) -> float:
    """a_s = sqrt(2 m_s k_B T) (k_B = 1)."""
    return sqrt(2.0 * float(w["m"][s]) / float(w["beta"]))


def q_grid(w: dict, s: int) -> np.ndarray:
    """Cell-centred q_s grid: -L + (i + 1/2) h, h = 2 L / N."""
    N, L = int(w["Nq"][s]), float(w["Lq"][s])
    h = 2.0 * L / N
    return -L + (np.arange(N) + 0.5) * h


def deriv_matrix(N: int, h: float) -> np.ndarray:
    """Dense compact sixth-order first-derivative operator A^{-1} B / h
    (Sec. III B): A = tridiag(1/3, 1, 1/3), B with 7/9 on f_{i+1} - f_{i-1}
    and 1/36 on f_{i+2} - f_{i-2}; rows truncated at the box (zeros outside)."""
    A = np.eye(N)
    B = np.zeros((N, N))
    for i in range(N):
        if i > 0:
            A[i, i - 1] = 1.0 / 3.0
            B[i, i - 1] = -7.0 / 9.0
        if i + 1 < N:
            A[i, i + 1] = 1.0 / 3.0
            B[i, i + 1] = 7.0 / 9.0
        if i > 1:
            B[i, i - 2] = -1.0 / 36.0
        if i + 2 < N:
            B[i, i + 2] = 1.0 / 36.0
    return np.linalg.solve(A, B) / h


def shape(w: dict) -> tuple:
    M = int(w["M"])
    return (elements(w).shape[0],) + tuple(int(x) for x in w["Np"][:M]) + tuple(int(x) for x in w["Nq"][:M])


def _qpoints(w: dict) -> np.ndarray:
    M = int(w["M"])
    grids = np.meshgrid(*[q_grid(w, s) for s in range(M)], indexing="ij")
    return np.stack([g.ravel() for g in grids], axis=1)


def tables(w: dict) -> dict:
    """U(q), F_s(q) on the M-dimensional q grid (the grid oracle's potential
    and force, Sec. II A), V_s'(q_s) = V_LL + V_SL q_s, the derivative
    matrices and the quadrature weights times the cell volume."""
    M = int(w["M"])
    Nq = tuple(int(x) for x in w["Nq"][:M])
    pts = _qpoints(w)
    U = np.array([potential(w, q) for q in pts]).reshape(Nq)
    F = [np.array([force(w, q, s) for q in pts]).reshape(Nq) for s in range(M)]
    Vp = [float(w["VLL"][s]) + float(w["VSL"][s]) * q_grid(w, s) for s in range(M)]
    D = [deriv_matrix(Nq[s], 2.0 * float(w["Lq"][s]) / Nq[s]) for s in range(M)]
    wq = np.ones(Nq)
    for s in range(M):
        ws = np.ones(Nq[s])
        ws[0] = ws[-1] = 0.8
        wq = wq * ws.reshape([-1 if t == s else 1 for t in range(M)])
        wq = wq * (2.0 * float(w["Lq"][s]) / Nq[s])
    return {"U": U, "F": F, "Vp": Vp, "D": D, "wq": wq}


def _shift(c: np.ndarray, axis: int, d: int) -> np.ndarray:
    """out[..., k, ...] = c[..., k + d, ...] (zero where k + d is outside)."""
    out = np.zeros_like(c)
    n = c.shape[axis]
    src = [slice(None)] * c.ndim
    dst = [slice(None)] * c.ndim
    if d > 0:
        src[axis], dst[axis] = slice(d, n), slice(0, n - d)
    else:
        src[axis], dst[axis] = slice(0, n + d), slice(-d, n)
    out[tuple(dst)] = c[tuple(src)]
    return out


def _along(c: np.ndarray, axis: int, vec: np.ndarray) -> np.ndarray:
    """vec broadcast along one axis of an array shaped like c."""
    sh = [1] * c.ndim
    sh[axis] = vec.size
    return vec.reshape(sh)


def _apply(D: np.ndarray, c: np.ndarray, axis: int) -> np.ndarray:
    return np.moveaxis(np.tensordot(D, c, axes=([1], [axis])), 0, axis)


def rhs(w: dict, C, T=None) -> np.ndarray:
    """Right-hand side of Eq. (HEOM2FP-H) for every element and coefficient."""
    M = int(w["M"])
    T = tables(w) if T is None else T
    C = np.asarray(C, dtype=np.float64)
    assert C.shape == shape(w), (C.shape, shape(w))
    el = elements(w)
    index = {tuple(int(x) for x in n): e for e, n in enumerate(el)}
    beta = float(w["beta"])
    out = np.zeros_like(C)
    for e, n in enumerate(el):
        c = C[e]
        r = -sum(int(n[s]) * float(w["gamma"][s]) for s in range(M)) * c
        for s in range(M):
            ka, qa = s, M + s  # Hermite axis and q axis of mode s in c
            a, m = width(w, s), float(w["m"][s])
            k = np.arange(c.shape[ka], dtype=np.float64)
            sp, sm = _along(c, ka, np.sqrt(k + 1.0)), _along(c, ka, np.sqrt(k))
            up, dn = _shift(c, ka, +1), _shift(c, ka, -1)
            Fs = T["F"][s].reshape((1,) * M + T["F"][s].shape)
            Vp = _along(c, qa, T["Vp"][s])
            # D+ sqrt(k+1) c_{k+1} - D- sqrt(k) c_{k-1}: the force part and the q derivative
            r = r + Fs / (sqrt(2.0) * a) * (sp * up - sm * dn)
            r = r + _apply(T["D"][s], -a / (sqrt(2.0) * m) * (sp * up + sm * dn), qa)
            nu = tuple(int(n[t]) + (1 if t == s else 0) for t in range(M))
            if nu in index:  # Phi: n + e_s, lowered k
                r = r - np.sqrt(2.0) * sm / a * Vp * _shift(C[index[nu]], ka, -1)
            if n[s] > 0:  # Theta: n - e_s, raised k
                nd = tuple(int(n[t]) - (1 if t == s else 0) for t in range(M))
                cth = int(n[s]) * float(w["zeta"][s]) * float(w["gamma"][s]) * m / beta
                r = r + cth * np.sqrt(2.0) * sp / a * Vp * _shift(C[index[nd]], ka, +1)
        out[e] = r
    return out


def rk4(w: dict, C, nsteps: int, dt: float, T=None) -> np.ndarray:
    """nsteps classical RK4 steps (stage by stage)."""
    T = tables(w) if T is None else T
    y = np.array(C, dtype=np.float64)
    for _ in range(int(nsteps)):
        k1 = rhs(w, y, T)
        k2 = rhs(w, y + 0.5 * dt * k1, T)
        k3 = rhs(w, y + 0.5 * dt * k2, T)
        k4 = rhs(w, y + dt * k3, T)
        y = y + dt / 6.0 * (k1 + 2.0 * k2 + 2.0 * k3 + k4)
    return y


def boltzmann(w: dict, T=None) -> np.ndarray:
    """c_{0,0}(q) = e^{-beta U/2} / Z_q, every other coefficient zero."""
    T = tables(w) if T is None else T
    beta = float(w["beta"])
    C = np.zeros(shape(w))
    M = int(w["M"])
    Zq = float(np.sum(T["wq"] * np.exp(-beta * T["U"])))
    C[(0,) + (0,) * M] = np.exp(-0.5 * beta * T["U"]) / Zq
    return C


def equilibrate(w: dict, nsteps: int, dt: float, T=None) -> np.ndarray:
    T = tables(w) if T is None else T
    return rk4(w, boltzmann(w, T), nsteps, dt, T)


def _xvals(w: dict, X: dict):
    """X(q) and dX/dq_s on the q grid, X = sum lin_s q_s + 1/2 sum quad q_s q_t."""
    M = int(w["M"])
    Nq = tuple(int(x) for x in w["Nq"][:M])
    pts = _qpoints(w)
    lin = np.array([float(v) for v in X["lin"]][:M])
    Q = np.array([[float(v) for v in row[:M]] for row in X["quad"][:M]])
    val = pts @ lin + 0.5 * np.einsum("is,st,it->i", pts, Q, pts)
    grad = [(lin[s] + pts @ (0.5 * (Q[s] + Q[:, s]))).reshape(Nq) for s in range(M)]
    return val.reshape(Nq), grad


def perturb(w: dict, X: dict, C) -> np.ndarray:
    """(X^x c)_{n,k} = - sum_s dX/dq_s sqrt(2 k_s)/a_s c_{n,k-e_s} for every n."""
    M = int(w["M"])
    C = np.asarray(C, dtype=np.float64)
    _, grad = _xvals(w, X)
    out = np.zeros_like(C)
    for s in range(M):
        ka = 1 + s  # Hermite axis in C (axis 0 is the element)
        k = np.arange(C.shape[ka], dtype=np.float64)
        g = grad[s].reshape((1,) + (1,) * M + grad[s].shape)
        out = out - g * _along(C, ka, np.sqrt(2.0 * k) / width(w, s)) * _shift(C, ka, -1)
    return out


def observe(w: dict, X: dict, C, T=None) -> float:
    """<X> = int dq X(q) e^{-beta U/2} c_{0,0}(q) (p integrated exactly)."""
    T = tables(w) if T is None else T
    M = int(w["M"])
    val, _ = _xvals(w, X)
    c00 = np.asarray(C, dtype=np.float64)[(0,) + (0,) * M]
    return float(np.sum(T["wq"] * val * np.exp(-0.5 * float(w["beta"]) * T["U"]) * c00))


def response_1d(w: dict, A: dict, Ceq, n_t: int, stride: int, dt: float, T=None) -> np.ndarray:
    """R^(1)[j] of Eq. (1Dresponse) at t = j stride dt."""
    T = tables(w) if T is None else T
    u = perturb(w, A, Ceq)
    R = np.empty(int(n_t))
    for j in range(int(n_t)):
        if j > 0:
            u = rk4(w, u, stride, dt, T)
        R[j] = observe(w, A, u, T)
    return R


def response_2d(w: dict, A: dict, B: dict, Cop: dict, Ceq, n_t1: int, n_t2: int,
                stride1: int, stride2: int, dt: float, T=None) -> np.ndarray:
    """R^(2)[j2, j1] of Eq. (2Dresponse) (t1 fastest), the double loop of Sec. IV C."""
    T = tables(w) if T is None else T
    R = np.empty((int(n_t2), int(n_t1)))
    u = perturb(w, A, Ceq)
    for j1 in range(int(n_t1)):
        if j1 > 0:
            u = rk4(w, u, stride1, dt, T)
        v = perturb(w, B, u)
        for j2 in range(int(n_t2)):
            if j2 > 0:
                v = rk4(w, v, stride2, dt, T)
            R[j2, j1] = observe(w, Cop, v, T)
    return R


def response_3d(w: dict, A: dict, B: dict, Cop: dict, D: dict, Ceq, n_t1: int, t2_steps: int, n_t3: int,
                stride1: int, stride3: int, dt: float, T=None) -> np.ndarray:
    """R^(3)[j3, j1] of Eq. (3Dresponse) at the waiting time t2 = t2_steps dt
    (t1 fastest): each t1 branch follows B^x, the waiting time, C^x and the
    t3 samples of <D>."""
    T = tables(w) if T is None else T
    R = np.empty((int(n_t3), int(n_t1)))
    u = perturb(w, A, Ceq)
    for j1 in range(int(n_t1)):
        if j1 > 0:
            u = rk4(w, u, stride1, dt, T)
        v = rk4(w, perturb(w, B, u), t2_steps, dt, T)
        x = perturb(w, Cop, v)
        for j3 in range(int(n_t3)):
            if j3 > 0:
                x = rk4(w, x, stride3, dt, T)
            R[j3, j1] = observe(w, D, x, T)
    return R


def hermite_functions(kmax: int, p: np.ndarray, a: float) -> np.ndarray:
    """psi_0..psi_{kmax-1} at the points p (rows), by the three-term recurrence
    psi_{j+1} = sqrt(2/(j+1)) (p/a) psi_j - sqrt(j/(j+1)) psi_{j-1}."""
    x = np.asarray(p, dtype=np.float64) / a
    out = np.zeros((kmax, x.size))
    out[0] = np.exp(-0.5 * x * x) / sqrt(a * sqrt(np.pi))
    if kmax > 1:
        out[1] = sqrt(2.0) * x * out[0]
    for j in range(1, kmax - 1):
        out[j + 1] = sqrt(2.0 / (j + 1)) * x * out[j] - sqrt(j / (j + 1.0)) * out[j - 1]
    return out


def to_grid_h(w: dict, C, p_grids) -> np.ndarray:
    """The h-form element h_n(q, p) = prod_s (a_s sqrt(pi))^{-1/2} sum_k c_{n,k}(q) psi_k(p)
    (W_n = e^{-beta H/2} h_n) on the given p grids; shape [e][q...][p...]."""
    M = int(w["M"])
    C = np.asarray(C, dtype=np.float64)
    h = C
    for s in range(M):
        a = width(w, s)
        psi = hermite_functions(C.shape[1 + s], p_grids[s], a) / sqrt(a * sqrt(np.pi))
        # contract the leading remaining Hermite axis (axis 1) with psi; p_s is appended last
        h = np.tensordot(h, psi, axes=([1], [0]))
    return h
