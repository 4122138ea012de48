"""Second, independent assembly of the discrete CHFPE generator -- TEST INFRASTRUCTURE.

The generator is built as a sparse matrix from the Kronecker form of the
compact scheme (Sec. III B: (A_1 x I x I) dc/dq_1 = (B_1 x I x I) c, ...),
with the printed matrices A (alpha on the off-diagonals) and B (a on the
first, b on the second off-diagonals, antisymmetric) and the hierarchy
couplings of Eq. (eq:HEOM), acting on the smooth factor h_n of
W_n = exp(-beta H/2) h_n (the factorization of Sec. III A).  The force
dU/dq_s is taken from U itself by complex-step differentiation, so it does
not reuse the oracle's hand-written derivative of the potential.  Only small
grids are practical here.
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.sparse as sp

ALPHA = 1.0 / 3.0
A1 = 7.0 / 9.0    # weight of (f_{i+1} - f_{i-1}) / h
B1 = 1.0 / 36.0   # weight of (f_{i+2} - f_{i-2}) / h


def compact_matrices(N: int):
    """The N x N matrices A and B of the compact first-derivative scheme."""
    A = np.eye(N) + ALPHA * (np.eye(N, k=1) + np.eye(N, k=-1))
    B = A1 * (np.eye(N, k=1) - np.eye(N, k=-1)) + B1 * (np.eye(N, k=2) - np.eye(N, k=-2))
    return A, B


def derivative_matrix(N: int, h: float) -> np.ndarray:
    A, B = compact_matrices(N)
    return np.linalg.solve(A, B) / h


def grid(N: int, L: float) -> np.ndarray:
    return -L + (np.arange(N) + 0.5) * (2.0 * L / N)


def element_set(M: int, K: int):
    """{n : |n| <= K}, graded, lexicographically descending within a grade."""
    out = []
    for d in range(K + 1):
        grade = [n for n in itertools.product(range(d + 1), repeat=M) if sum(n) == d]
        grade.sort(reverse=True)
        out.extend(grade)
    return out


def potential(w: dict, q):
    """U(q) of Eqs. (sec: Potenentials), (sec: Potential ss') plus q^4/4! terms;
    q may be complex (used for complex-step differentiation)."""
    M = w["M"]
    u = 0.0
    for s in range(M):
        x = q[s]
        u = u + 0.5 * w["m"][s] * w["omega"][s] ** 2 * x ** 2 + w["g3"][s] * x ** 3 / 6.0 \
            + w["g4"][s] * x ** 4 / 24.0
    for s in range(M):
        for t in range(s + 1, M):
            u = u + w["g2"][s][t] * q[s] * q[t] + (w["g21"][s][t] * q[s] ** 2 * q[t]
                                                   + w["g12"][s][t] * q[s] * q[t] ** 2) / 6.0
    return u


def force(w: dict, q, s: int, eps: float = 1e-30):
    """dU/dq_s by complex-step differentiation (exact to rounding for polynomials)."""
    qc = [np.asarray(x, dtype=np.complex128) for x in q]
    qc[s] = qc[s] + 1j * eps
    return np.imag(potential(w, qc)) / eps


def generator(w: dict, symmetrised: bool = True, deriv=None):
    """(G, f): the sparse generator G acting on h (stacked elements) and the
    factor f = exp(-beta H/2) on the grid, so that dW/dt = f * (G @ (W / f)).

    With symmetrised=False the couplings of Eq. (eq:HEOM) are discretized on
    W itself (G then acts on W and f = 1); kept to show that form is unstable.
    deriv(axis, N, h), if given, supplies the first-derivative matrix of each
    grid axis (axis ids 0..M-1: q_s, M..2M-1: p_s) in place of the plain
    compact one (used for coarse grids with a closure).
    """
    M, K = w["M"], w["K"]
    Nq, Np = list(w["Nq"]), list(w["Np"])
    dims = Nq + Np
    nd = 2 * M
    beta = w["beta"]
    hq = [2.0 * w["Lq"][s] / Nq[s] for s in range(M)]
    hp = [2.0 * w["Lp"][s] / Np[s] for s in range(M)]
    axes = [grid(Nq[s], w["Lq"][s]) for s in range(M)] + [grid(Np[s], w["Lp"][s]) for s in range(M)]
    mesh = np.meshgrid(*axes, indexing="ij")
    q = [mesh[s].ravel() for s in range(M)]
    p = [mesh[M + s].ravel() for s in range(M)]

    def kron_axis(D, ax):
        mats = [sp.identity(dims[d], format="csr") if d != ax else sp.csr_matrix(D) for d in range(nd)]
        out = mats[0]
        for mat in mats[1:]:
            out = sp.kron(out, mat, format="csr")
        return out

    dm = deriv if deriv is not None else (lambda axis, N, h: derivative_matrix(N, h))
    Dq = [kron_axis(dm(s, Nq[s], hq[s]), s) for s in range(M)]
    Dp = [kron_axis(dm(M + s, Np[s], hp[s]), M + s) for s in range(M)]
    F = [force(w, q, s) for s in range(M)]
    Vp = [w["VLL"][s] + w["VSL"][s] * q[s] for s in range(M)]

    els = element_set(M, K)
    index = {n: i for i, n in enumerate(els)}
    E = int(np.prod(dims))
    blocks = [[None] * len(els) for _ in els]
    for i, n in enumerate(els):
        diag = sp.csr_matrix((E, E))
        for s in range(M):
            diag = diag + sp.diags(F[s]) @ Dp[s] - sp.diags(p[s] / w["m"][s]) @ Dq[s]
        diag = diag - sum(n[s] * w["gamma"][s] for s in range(M)) * sp.identity(E)
        blocks[i][i] = diag
        for s in range(M):
            bp = sp.diags(beta * p[s] / (2.0 * w["m"][s]))
            c1 = w["m"][s] * w["zeta"][s] * w["gamma"][s] / beta
            up = tuple(n[t] + (t == s) for t in range(M))
            if up in index:
                j = index[up]
                blk = sp.diags(Vp[s]) @ (Dp[s] - bp) if symmetrised else sp.diags(Vp[s]) @ Dp[s]
                blocks[i][j] = blk if blocks[i][j] is None else blocks[i][j] + blk
            if n[s] > 0:
                dn = tuple(n[t] - (t == s) for t in range(M))
                j = index[dn]
                if symmetrised:
                    blk = n[s] * c1 * (sp.diags(Vp[s]) @ (Dp[s] + bp))
                else:
                    c2 = w["zeta"][s] * w["gamma"][s]
                    blk = n[s] * (sp.diags(c1 * Vp[s]) @ Dp[s] + sp.diags(c2 * p[s] * Vp[s]))
                blocks[i][j] = blk if blocks[i][j] is None else blocks[i][j] + blk
    G = sp.bmat(blocks, format="csr")
    if not symmetrised:
        return G, np.ones(len(els) * E)
    H = potential(w, q) + sum(p[s] ** 2 / (2.0 * w["m"][s]) for s in range(M))
    f = np.tile(np.exp(-0.5 * beta * H), len(els))
    return G, f


def apply(w: dict, W: np.ndarray) -> np.ndarray:
    """dW/dt for a state W of the workload's shape."""
    G, f = generator(w)
    x = W.ravel()
    return (f * (G @ (x / f))).reshape(W.shape)
