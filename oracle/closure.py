"""FP64 CPU oracle of the learned per-axis closure -- TEST INFRASTRUCTURE.

Only ``tests/`` and the smoke check may import this module; the HIP library
never calls it.  It shares no code with the HIP path.

The paper computes on one grid and mentions machine learning only for
extracting model parameters from MD trajectories (Sec. V), so the closure is
a reading of this project (listed with the other readings in the design
notes):

* Closure form.  On a coarse grid, the compact first derivative of
  Sec. III B along grid axis a solves A y = (B + S_a) f / h_a instead of
  A y = B f / h_a.  S_a is skew-symmetric with nonzero entries only on the
  first two off-diagonals: S[i, i+k] = -S[i+k, i] (k = 1, 2, i < N - k),
  so P = 2N - 3 numbers per axis.  (A third off-diagonal fits the training
  derivatives better but gave larger spectrum errors on held-out draws.)
  Skew-symmetry keeps A D skew, as for the plain scheme (A symmetric, B
  skew), which keeps the generator stable; an unconstrained banded stencil
  fitted to the same data is not.
* Training pairs.  A fine grid has twice the points per axis on the same
  box (cell-centred nesting: fine cells 2i and 2i + 1 make coarse cell i).
  Restriction R averages the 2^(2M) fine values of each coarse cell, on the
  smooth factor h of W = exp(-beta H / 2) h.  For a fine state h_f the target
  of axis a is T = R(D_a^fine h_f); the coarse line values are x = R h_f and
  the residual of the plain coarse derivative is r = T - D_a^coarse x.
* Loss of one (draw, axis) group: ||r - A^{-1} S_a x / h_a||^2 summed over
  every line of every element of every snapshot, divided by ||T||^2.  As a
  function of s_a it is the quadratic s^T G s - 2 b^T s + c (divided by t),
  whose G and b follow from the moments Mx = sum x x^T and Cxr = sum x r^T.
* Network.  One row per (axis, skew entry): 16 features -> 32 tanh units ->
  1 output, the entry s.  Weights are stored in BF16 and products accumulate
  in FP32: features, W1, the hidden activations, W2 and, in the backward
  products, the gradients of the hidden layer and of s are rounded to BF16
  where the device rounds them (see ``bf16``).
"""
from __future__ import annotations

import numpy as np

from . import dense

NFEAT = 16
NHID = 32
KMAX = 2  # off-diagonals of the skew correction


# ---------------------------------------------------------------------------
# skew stencil correction
# ---------------------------------------------------------------------------
def skew_entries(N: int):
    """(i, k) of the free entries S[i, i+k]: k = 1 for i < N-1, then k = 2
    for i < N-2, and so on up to KMAX (this order is the order of s)."""
    return [(i, k) for k in range(1, KMAX + 1) for i in range(N - k)]


def n_entries(N: int) -> int:
    return sum(N - k for k in range(1, KMAX + 1))


def skew_matrix(N: int, s) -> np.ndarray:
    S = np.zeros((N, N))
    for (i, k), v in zip(skew_entries(N), s):
        S[i, i + k] += v
        S[i + k, i] -= v
    return S


def closure_derivative_matrix(N: int, h: float, s) -> np.ndarray:
    """D' = A^{-1} (B + S) / h, with A and B the compact matrices for h = 1."""
    A, B = dense.compact_matrices(N)
    return np.linalg.solve(A, B + skew_matrix(N, s)) / h


# ---------------------------------------------------------------------------
# restriction, axis derivatives, moments
# ---------------------------------------------------------------------------
def restrict(state: np.ndarray) -> np.ndarray:
    """2:1 cell average over every grid axis of [element, axis_0, axis_1, ...]."""
    a = np.asarray(state, dtype=np.float64)
    for d in range(1, a.ndim):
        shape = list(a.shape)
        if shape[d] % 2:
            raise ValueError("fine axes must have an even number of points")
        shape[d] //= 2
        shape.insert(d + 1, 2)
        a = a.reshape(shape).mean(axis=d + 1)
    return a


def along(Dm: np.ndarray, a: np.ndarray, d: int) -> np.ndarray:
    """Apply the matrix Dm to every line of a along array axis d."""
    return np.moveaxis(np.tensordot(Dm, np.moveaxis(a, d, 0), axes=(1, 0)), 0, d)


def axis_lengths(w: dict):
    M = w["M"]
    N = list(w["Nq"]) + list(w["Np"])
    L = list(w["Lq"]) + list(w["Lp"])
    return N, [2.0 * L[a] / N[a] for a in range(2 * M)], L


def moments(w_fine: dict, h_fine: np.ndarray, axis: int):
    """Moments of one fine state for coarse axis `axis` (0..M-1: q_s,
    M..2M-1: p_s): Mx = sum x x^T, Cxr = sum x r^T (N x N), c = sum r.r,
    t = sum T.T over every line of every element."""
    Nf, hf, _ = axis_lengths(w_fine)
    N, hc = Nf[axis] // 2, 2.0 * hf[axis]
    d = axis + 1
    T = restrict(along(dense.derivative_matrix(Nf[axis], hf[axis]), h_fine, d))
    x = restrict(h_fine)
    r = T - along(dense.derivative_matrix(N, hc), x, d)
    X = np.moveaxis(x, d, 0).reshape(N, -1)
    Rm = np.moveaxis(r, d, 0).reshape(N, -1)
    return X @ X.T, X @ Rm.T, float((r * r).sum()), float((T * T).sum())


def gram(N: int, h: float, Mx: np.ndarray, Cxr: np.ndarray):
    """G and b of the quadratic loss from the moments:
    v_e = A^{-1} E_e x / h for the skew basis E_e, G_ef = sum v_e.v_f,
    b_e = sum v_e.r."""
    A, _ = dense.compact_matrices(N)
    Ai = np.linalg.inv(A)
    K = Ai.T @ Ai
    P = n_entries(N)
    E = [skew_matrix(N, np.eye(P)[e]) for e in range(P)]
    P = len(E)
    G = np.empty((P, P))
    b = np.empty(P)
    for e in range(P):
        for f in range(P):
            G[e, f] = np.trace(E[e].T @ K @ E[f] @ Mx)
        b[e] = np.trace(Ai @ E[e] @ Cxr)
    return G / (h * h), b / h


def group_loss(s, G, b, c, t) -> float:
    s = np.asarray(s, dtype=np.float64)
    return float((s @ G @ s - 2.0 * b @ s + c) / t)


# ---------------------------------------------------------------------------
# features
# ---------------------------------------------------------------------------
def features(w_coarse: dict) -> np.ndarray:
    """Rows (axis, skew entry) of the coarse workload, in axis order then
    skew_entries order; 16 features each (the last is a constant 1)."""
    M = w_coarse["M"]
    N, h, L = axis_lengths(w_coarse)
    beta = w_coarse["beta"]
    rows = []
    for a in range(2 * M):
        s = a % M
        m, om = w_coarse["m"][s], w_coarse["omega"][s]
        sig_q = 1.0 / (om * np.sqrt(beta * m))
        sig = sig_q if a < M else np.sqrt(m / beta)
        x = -L[a] + (np.arange(N[a]) + 0.5) * h[a]
        for (i, k) in skew_entries(N[a]):
            u = 0.5 * (x[i] + x[i + k]) / L[a]
            edge = min(i, N[a] - 1 - (i + k))  # cells between the entry and the box edge
            rows.append([
                u, u * u, abs(u), float(k == 2), float(a >= M), h[a] / sig,
                om / 1.6, w_coarse["g3"][s] * sig_q / (m * om * om),
                w_coarse["g4"][s] * sig_q * sig_q / (m * om * om),
                w_coarse["VSL"][s] * sig_q / w_coarse["VLL"][s],
                w_coarse["zeta"][s], w_coarse["gamma"][s], beta / 2.0, m,
                float(edge == 0), 1.0])
    return np.array(rows, dtype=np.float64)


def row_axes(w_coarse: dict) -> np.ndarray:
    N, _, _ = axis_lengths(w_coarse)
    return np.concatenate([np.full(n_entries(N[a]), a) for a in range(2 * w_coarse["M"])])


# ---------------------------------------------------------------------------
# network (FP64 arithmetic with the device's BF16 rounding points)
# ---------------------------------------------------------------------------
def bf16(x) -> np.ndarray:
    """Round to the nearest BF16 value (ties to even), returned as float64.
    Values are first rounded to FP32, as the device holds them."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def init_params(seed: int) -> dict:
    """Seeded initial weights: W1 ~ N(0, 1/16), W2 ~ N(0, 1e-4), biases 0."""
    rng = np.random.default_rng(seed)
    return {"W1": rng.normal(0.0, 0.25, (NFEAT, NHID)), "b1": np.zeros(NHID),
            "W2": rng.normal(0.0, 0.01, NHID), "b2": 0.0}


def forward(p: dict, X: np.ndarray, rounding: bool = True):
    """s = tanh(X W1 + b1) W2 + b2, returning s and the cache for backward."""
    r = bf16 if rounding else (lambda v: np.asarray(v, dtype=np.float64))
    Xr, W1r, W2r = r(X), r(p["W1"]), r(p["W2"])
    Hpre = Xr @ W1r + p["b1"]
    A1 = np.tanh(Hpre)
    s = r(A1) @ W2r + p["b2"]
    return s, (Xr, W1r, W2r, A1)


def backward(p: dict, cache, gs: np.ndarray, rounding: bool = True) -> dict:
    """Gradients of sum(gs * s) with respect to the parameters."""
    r = bf16 if rounding else (lambda v: np.asarray(v, dtype=np.float64))
    Xr, W1r, W2r, A1 = cache
    gs = np.asarray(gs, dtype=np.float64)
    gW2 = r(A1).T @ r(gs)
    gb2 = float(gs.sum())
    gH = (gs[:, None] * W2r[None, :]) * (1.0 - A1 * A1)
    gW1 = Xr.T @ r(gH)
    gb1 = gH.sum(axis=0)
    return {"W1": gW1, "b1": gb1, "W2": gW2, "b2": gb2}


def loss_grad(s: np.ndarray, groups):
    """Mean group loss and its gradient with respect to s.  groups: list of
    (row indices, G, b, c, t)."""
    gs = np.zeros_like(s)
    tot = 0.0
    for idx, G, b, c, t in groups:
        v = s[idx]
        tot += (v @ G @ v - 2.0 * b @ v + c) / t
        gs[idx] = 2.0 * (G @ v - b) / t
    n = len(groups)
    return tot / n, gs / n


def adam_step(p: dict, g: dict, state: dict, lr: float, beta1=0.9, beta2=0.999, eps=1e-8) -> None:
    """One Adam step (Kingma & Ba) on the FP64 copies of the master weights."""
    state["t"] = state.get("t", 0) + 1
    t = state["t"]
    for k in ("W1", "b1", "W2", "b2"):
        m = state.get("m_" + k, np.zeros_like(np.asarray(p[k], dtype=np.float64)))
        v = state.get("v_" + k, np.zeros_like(np.asarray(p[k], dtype=np.float64)))
        m = beta1 * m + (1 - beta1) * np.asarray(g[k])
        v = beta2 * v + (1 - beta2) * np.square(g[k])
        state["m_" + k], state["v_" + k] = m, v
        mh = m / (1 - beta1 ** t)
        vh = v / (1 - beta2 ** t)
        p[k] = p[k] - lr * mh / (np.sqrt(vh) + eps)


# ---------------------------------------------------------------------------
# the coarse solver with a closure (small grids: sparse assembly)
# ---------------------------------------------------------------------------
def split_rows(w_coarse: dict, s):
    """The closure entries of each axis, in axis-id order."""
    N, _, _ = axis_lengths(w_coarse)
    out, o = [], 0
    for a in range(2 * w_coarse["M"]):
        P = n_entries(N[a])
        out.append(np.asarray(s[o:o + P], dtype=np.float64))
        o += P
    return out


def closure_deriv(w_coarse: dict, s):
    """deriv(axis, N, h) for dense.generator: D' = A^{-1}(B + S_axis)/h."""
    per_axis = split_rows(w_coarse, s)
    return lambda axis, N, h: closure_derivative_matrix(N, h, per_axis[axis])


def generator(w: dict, s=None):
    """(G, f) of the coarse problem with closure entries s (None: plain)."""
    return dense.generator(w, deriv=None if s is None else closure_deriv(w, s))


def rk4_h(G, x: np.ndarray, nsteps: int, dt: float) -> np.ndarray:
    """Classical RK4 on dx/dt = G x."""
    for _ in range(nsteps):
        k1 = G @ x
        k2 = G @ (x + 0.5 * dt * k1)
        k3 = G @ (x + 0.5 * dt * k2)
        k4 = G @ (x + dt * k3)
        x = x + dt / 6.0 * (k1 + 2.0 * k2 + 2.0 * k3 + k4)
    return x


def _grids(w: dict):
    M = w["M"]
    ax = [dense.grid(w["Nq"][s], w["Lq"][s]) for s in range(M)] + \
         [dense.grid(w["Np"][s], w["Lp"][s]) for s in range(M)]
    return np.meshgrid(*ax, indexing="ij")


def _hfactor(w: dict) -> np.ndarray:
    M = w["M"]
    mesh = _grids(w)
    q = [mesh[s] for s in range(M)]
    p = [mesh[M + s] for s in range(M)]
    H = dense.potential(w, q) + sum(p[s] ** 2 / (2.0 * w["m"][s]) for s in range(M))
    return np.exp(-0.5 * w["beta"] * H)


def perturb(w: dict, X: dict, W: np.ndarray, s=None) -> np.ndarray:
    """X^x W (Eq. (Opticalexc)) on every element, written for h and with the
    closure derivative along p when s is given; W-form in and out."""
    M = w["M"]
    mesh = _grids(w)
    q = [mesh[t] for t in range(M)]
    p = [mesh[M + t] for t in range(M)]
    f = _hfactor(w)
    h = np.asarray(W, dtype=np.float64) / f[None]
    per_axis = split_rows(w, s) if s is not None else None
    out = np.zeros_like(h)
    for t in range(M):
        dX = X["lin"][t] + sum(0.5 * (X["quad"][t][u] + X["quad"][u][t]) * q[u] for u in range(M))
        Np, hp = w["Np"][t], 2.0 * w["Lp"][t] / w["Np"][t]
        D = (closure_derivative_matrix(Np, hp, per_axis[M + t]) if per_axis is not None
             else dense.derivative_matrix(Np, hp))
        dh = along(D, h, 1 + M + t)
        out += dX[None] * (dh - (w["beta"] * p[t] / (2.0 * w["m"][t]))[None] * h)
    return out * f[None]


def response_2d(w: dict, A: dict, B: dict, C: dict, Weq: np.ndarray, n_t1: int, n_t2: int,
                s1: int, s2: int, dt: float, s=None) -> np.ndarray:
    """R[j2][j1] of the double loop of Sec. IV C with the closure s."""
    from . import observe
    G, _ = generator(w, s)
    shape = Weq.shape
    fW = _hfactor(w)[None] * np.ones(shape)
    U = perturb(w, A, Weq, s)
    R = np.zeros((n_t2, n_t1))
    for j1 in range(n_t1):
        if j1 > 0:
            U = (fW.ravel() * rk4_h(G, U.ravel() / fW.ravel(), s1, dt)).reshape(shape)
        V = perturb(w, B, U, s)
        for j2 in range(n_t2):
            if j2 > 0:
                V = (fW.ravel() * rk4_h(G, V.ravel() / fW.ravel(), s2, dt)).reshape(shape)
            R[j2, j1] = observe(w, C, V)
    return R


def propagate(w: dict, W: np.ndarray, nsteps: int, dt: float, s=None) -> np.ndarray:
    """nsteps RK4 steps of the W-form state with the closure s."""
    G, _ = generator(w, s)
    fW = (_hfactor(w)[None] * np.ones(W.shape)).ravel()
    return (fW * rk4_h(G, np.asarray(W, dtype=np.float64).ravel() / fW, nsteps, dt)).reshape(W.shape)
