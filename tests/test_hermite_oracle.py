"""Pins of the Hermite-function oracle (Sec. III A; Appendix A, Eq. (HEOM2FP-H)).

The Hermite form and the p-grid h-form are two discretisations of the same
hierarchy, Eq. (eq:HEOM).  On one q grid their q derivatives are the same
linear map, so a Hermite state reconstructed on a fine p grid must give,
through the independently pinned grid oracle, the Hermite oracle's
right-hand side, excitation and observables, up to the p grid's own error,
which falls at sixth order.  That fixes every ladder factor and sign of the
Hermite equations against the grid equations.  Further pins: the
derivative matrix against the C oracle's line derivative, the Hermite
function algebra, and stationarity of the Boltzmann state.
"""
import numpy as np
import pytest

import oracle as orc
import oracle.hermite as oh
import workloads as wl


def _w(M, Nq, Nh, K, Lq=None):
    w = wl.workload({1: "one_mode_48", 2: "two_mode_32", 3: "three_mode_24"}[M])
    w["Nq"] = [Nq] * M
    w["Np"] = [Nh] * M
    w["K"] = K
    if Lq is not None:
        w["Lq"] = [Lq] * M
    return w


def _state(w, seed, top_zero=True):
    """A seeded Hermite state: smooth in q, decaying in k; the highest
    Hermite function of each mode is left empty (so no raising term leaves
    the truncation)."""
    rng = np.random.default_rng(seed)
    M = w["M"]
    sh = oh.shape(w)
    C = np.zeros(sh)
    qs = np.meshgrid(*[oh.q_grid(w, s) for s in range(M)], indexing="ij")
    env = np.exp(-0.35 * sum((w["omega"][s] * qs[s]) ** 2 for s in range(M)))
    for idx in np.ndindex(*sh[:1 + M]):
        k = idx[1:]
        if top_zero and any(k[s] == w["Np"][s] - 1 for s in range(M)):
            continue
        amp = rng.normal() * 0.6 ** sum(k)
        phase = rng.normal(size=M)
        C[idx] = amp * env * (1.0 + 0.4 * sum(np.sin(0.7 * qs[s] + phase[s]) for s in range(M)))
    return C


def _grid_w(w, Np, Lp):
    g = dict(w)
    g["Np"] = [Np] * w["M"]
    g["Lp"] = [Lp] * w["M"]
    return g


def _p_grids(g):
    return [-g["Lp"][s] + (np.arange(g["Np"][s]) + 0.5) * 2.0 * g["Lp"][s] / g["Np"][s] for s in range(g["M"])]


def _weight(g):
    """e^{-beta H/2} on the grid of g, shape [q...][p...]: W_n = e^{-beta H/2} h_n."""
    M = g["M"]
    T = oh.tables(g)
    pg = _p_grids(g)
    kin = sum(((pg[s] ** 2) / (2.0 * g["m"][s])).reshape([-1 if t == s else 1 for t in range(M)])
              for s in range(M))
    return np.exp(-0.5 * g["beta"] * (T["U"].reshape(T["U"].shape + (1,) * M) + kin.reshape((1,) * M + kin.shape)))


def _to_W(g, w, C):
    return _weight(g)[None] * oh.to_grid_h(w, C, _p_grids(g))


def test_derivative_matrix_matches_the_c_oracle_line_derivative():
    rng = np.random.default_rng(0)
    for N, h in ((7, 0.3), (16, 0.25), (24, 0.5)):
        f = rng.normal(size=N)
        assert np.allclose(oh.deriv_matrix(N, h) @ f, orc.deriv_line(f, h), rtol=0, atol=1e-12)


def test_hermite_functions_are_orthonormal_and_obey_the_ladder_relations():
    """int psi_i psi_j dp = delta_ij; (d/dp - p/a^2) psi_k = -sqrt(2(k+1))/a psi_{k+1};
    (d/dp + p/a^2) psi_k = sqrt(2k)/a psi_{k-1}: the operators of the h-form."""
    a = 1.3
    p = np.linspace(-14 * a, 14 * a, 20001)
    dp = p[1] - p[0]
    psi = oh.hermite_functions(9, p, a)
    G = psi @ psi.T * dp
    assert np.allclose(G, np.eye(9), atol=1e-10)
    dpsi = np.gradient(psi, dp, axis=1, edge_order=2)
    for k in range(8):
        up = dpsi[k] - p / a ** 2 * psi[k]
        assert np.max(np.abs(up + np.sqrt(2 * (k + 1)) / a * psi[k + 1])) < 1e-5
        if k > 0:
            dn = dpsi[k] + p / a ** 2 * psi[k]
            assert np.max(np.abs(dn - np.sqrt(2 * k) / a * psi[k - 1])) < 1e-5


@pytest.mark.parametrize("M,Nq,Nh,K", [(1, 12, 6, 2), (2, 8, 5, 2)])
def test_hermite_rhs_matches_the_grid_oracle_on_reconstructed_states(M, Nq, Nh, K):
    """Hermite RHS, reconstructed on a p grid, against the grid oracle's RHS of
    the reconstructed state: the gap falls at the p grid's sixth order."""
    w = _w(M, Nq, Nh, K)
    C = _state(w, seed=1)
    R = oh.rhs(w, C)
    errs = []
    sizes = (24, 48) if M == 2 else (24, 48, 96)
    for Np in sizes:
        g = _grid_w(w, Np, 9.0)
        W = _to_W(g, w, C)
        ref = orc.rhs(g, W)
        got = _to_W(g, w, R)
        errs.append(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    print("rhs gaps", errs)
    for e0, e1 in zip(errs, errs[1:]):
        assert e0 / e1 > 30.0  # sixth order would give 64 per halving of h_p
    assert errs[-1] < (1e-5 if len(errs) == 3 else 5e-4)


@pytest.mark.parametrize("M,Nq,Nh,K", [(1, 12, 6, 2), (2, 8, 5, 1)])
def test_hermite_excitation_and_observable_match_the_grid_oracle(M, Nq, Nh, K):
    w = _w(M, Nq, Nh, K)
    C = _state(w, seed=2)
    X = wl.optical(M, lin=[1.0, -0.7][:M], quad=[[0.2, 0.05], [0.05, -0.1]][:M])
    X["quad"] = [r[:M] for r in X["quad"]]
    Xc = oh.perturb(w, X, C)
    errs, oerr = [], []
    for Np in (24, 48):
        g = _grid_w(w, Np, 9.0)
        W = _to_W(g, w, C)
        ref = orc.perturb(g, X, W)
        errs.append(np.linalg.norm(_to_W(g, w, Xc) - ref) / np.linalg.norm(ref))
        v_ref = orc.observe(g, X, W)
        oerr.append(abs(oh.observe(w, X, C) - v_ref) / abs(v_ref))
    print("perturb gaps", errs, "observe gaps", oerr)
    assert errs[0] / errs[1] > 30.0 and errs[1] < 5e-4
    assert oerr[1] < 1e-12  # p integrated exactly by psi_0; the grid's quadrature converges fast


def test_boltzmann_state_is_stationary_at_sixth_order():
    """c_00 = e^{-beta U/2}/Z_q: only the q derivative in D- c_00 is inexact
    (D- annihilates it in the continuum), so the right-hand side falls at the
    q grid's sixth order."""
    res = []
    for Nq in (16, 32, 64):
        w = _w(1, Nq, 6, 2, Lq=8.0)  # a box where e^{-beta U/2} has vanished
        C = oh.boltzmann(w)
        res.append(np.linalg.norm(oh.rhs(w, C)) / np.linalg.norm(C))
    print("Boltzmann residuals", res)
    assert res[0] / res[1] > 30.0 and res[1] / res[2] > 30.0


def test_boltzmann_observable_of_one_is_one():
    w = _w(2, 10, 4, 1)
    C = oh.boltzmann(w)
    T = oh.tables(w)
    unit = float(np.sum(T["wq"] * np.exp(-0.5 * w["beta"] * T["U"]) * C[0, 0, 0]))
    assert abs(unit - 1.0) < 1e-14


def test_rk4_is_the_degree_four_taylor_polynomial_of_the_hermite_generator():
    """One RK4 step equals sum_{j<=4} (dt L)^j/j! applied with the oracle's RHS."""
    w = _w(2, 6, 3, 1)
    C = _state(w, seed=3, top_zero=False)
    dt = 0.01
    T = oh.tables(w)
    term, acc = C.copy(), C.copy()
    for j in range(1, 5):
        term = dt * oh.rhs(w, term, T) / j
        acc = acc + term
    assert np.linalg.norm(oh.rk4(w, C, 1, dt, T) - acc) / np.linalg.norm(acc) < 1e-14


def test_hermite_linear_response_approaches_the_grid_result():
    """R^(1) of the one-mode workload model from the Hermite oracle against
    the grid oracle on a fine p grid (same q grid, equilibrated the same way):
    the two discretisations agree to the p grid's error."""
    w = _w(1, 16, 10, 2)
    g = _grid_w(w, 48, 9.0)
    A = wl.optical(1, lin=[1.0], quad=[[0.2]])
    dt, n_eq, n_t = 0.01, 200, 60
    Ch = oh.equilibrate(w, n_eq, dt)
    Rh = oh.response_1d(w, A, Ch, n_t, 2, dt)
    Wg = orc.equilibrate(g, n_eq, dt)
    Rg = orc.response_1d(g, A, Wg, n_t, 2, dt)
    err = np.linalg.norm(Rh - Rg) / np.linalg.norm(Rg)
    print("R1 Hermite vs grid", err)
    assert err < 1e-3


def test_hermite_third_order_response_approaches_the_grid_result():
    """R^(3) at one waiting time: the grid oracle's result on p grids of 48
    and 96 points (same q grid) converges to the Hermite oracle's at sixth
    order (three excitations spread the state over many Hermite functions,
    so the 48-point grid is still 6% off; the Hermite series with 10
    functions is within 1.3e-6 of one with 24)."""
    w = _w(1, 14, 10, 2)
    A = wl.optical(1, lin=[1.0], quad=[[0.2]])
    B = wl.optical(1, lin=[0.5], quad=[[0.1]])
    dt = 0.01
    Ch = oh.equilibrate(w, 100, dt)
    Rh = oh.response_3d(w, A, B, B, A, Ch, 6, 10, 12, 2, 2, dt)
    errs = []
    for Np in (48, 96):
        g = _grid_w(w, Np, 9.0)
        Rg = orc.response_3d(g, A, B, B, A, orc.equilibrate(g, 100, dt), 6, 10, 12, 2, 2, dt)
        errs.append(np.linalg.norm(Rg - Rh) / np.linalg.norm(Rh))
    print("R3 grid vs Hermite", errs)
    assert errs[0] / errs[1] > 30.0 and errs[1] < 2e-3
