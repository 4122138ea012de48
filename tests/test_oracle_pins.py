"""Pins of the FP64 CPU oracle against what the paper and the mathematics fix.

Each test names the passage of the paper it checks and what independent
fact it uses (a closed form, an identity, a textbook scheme property,
brute force on tiny grids).  None of them compares the oracle with itself.
"""
import numpy as np
import pytest

import oracle as orc
import workloads as wl
from oracle import dense
from physics_refs import (boltzmann_average_1d, chi_brownian, linear_response_1d,
                          lyapunov_moments, response_2d_gaussian, response_3d_gaussian)


def harmonic_ll(N=48, K=2, **kw):
    """One harmonic mode, linear-linear coupling only (V_SL = 0)."""
    return wl.workload("one_mode_48", Nq=[N], Np=[N], K=K, g3=[0.0], g4=[0.0], VSL=[0.0], **kw)


# ---------------------------------------------------------------------------
# hierarchy index set (Sec. II B): the set {n : |n| <= K} and its order
# ---------------------------------------------------------------------------

def test_element_set_and_order():
    w = wl.workload("three_mode_24", Nq=[5] * 3, Np=[5] * 3)
    got = [tuple(r) for r in orc.elements(w)]
    assert got == [(0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1), (2, 0, 0), (1, 1, 0),
                   (1, 0, 1), (0, 2, 0), (0, 1, 1), (0, 0, 2)]
    for M, K, count in [(1, 3, 4), (2, 3, 10), (3, 2, 10), (3, 4, 35)]:
        w = wl.workload("three_mode_24", M=M, K=K, Nq=[5] * M, Np=[5] * M)
        assert orc.elements(w).shape == (count, M)


# ---------------------------------------------------------------------------
# compact sixth-order derivative (Sec. III B)
# ---------------------------------------------------------------------------

def test_compact_derivative_matches_lele_modified_wavenumber():
    """Far from the box ends the truncated scheme acts like the periodic one,
    whose response to sin(k x) is k' cos(k x) with Lele's modified wavenumber
    k' h = (14/9 sin kh + 1/18 sin 2kh) / (1 + 2/3 cos kh).  Each k weighs
    alpha, the 7/9 and the 1/36 weights differently."""
    N, h = 240, 0.05
    x = np.arange(N) * h
    for kh in (0.3, 0.9, 1.7, 2.6):
        k = kh / h
        y = orc.deriv_line(np.sin(k * x), h)
        kmod = (14.0 / 9.0 * np.sin(kh) + 1.0 / 18.0 * np.sin(2 * kh)) / (1.0 + 2.0 / 3.0 * np.cos(kh)) / h
        mid = slice(90, 150)
        np.testing.assert_allclose(y[mid], kmod * np.cos(k * x[mid]), rtol=0, atol=1e-11 * k)


def test_compact_derivative_sixth_order_convergence():
    """Error on a Gaussian well inside the box falls by ~2^6 per halving of h."""
    errs = []
    for N in (24, 48, 96):
        L = 6.0
        h = 2 * L / N
        x = -L + (np.arange(N) + 0.5) * h
        y = orc.deriv_line(np.exp(-x ** 2), h)
        errs.append(np.abs(y + 2 * x * np.exp(-x ** 2)).max())
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates > 5.5), rates


def test_compact_derivative_zero_ghost_closure():
    """Rows 0 and N-1 are the truncated Toeplitz rows printed in Sec. III B:
    the line solve equals the dense solve of A y = B f / h."""
    rng = np.random.default_rng(0)
    for N in (5, 7, 12, 33):
        f = rng.standard_normal(N)
        A, B = dense.compact_matrices(N)
        np.testing.assert_allclose(orc.deriv_line(f, 0.3), np.linalg.solve(A, B @ f) / 0.3,
                                   rtol=1e-13, atol=1e-13)


# ---------------------------------------------------------------------------
# right-hand side of Eq. (eq:HEOM): two independent assemblies agree
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("case", ["m1", "m2", "m3"])
def test_rhs_matches_kronecker_assembly(case):
    if case == "m1":
        w = wl.workload("one_mode_48", Nq=[8], Np=[9], K=3)
    elif case == "m2":
        w = wl.workload("two_mode_32", Nq=[6, 5], Np=[5, 6], K=2)
        w["g21"][0][1], w["g12"][0][1] = 0.07, -0.04
        w["zeta"], w["gamma"], w["VSL"] = [0.3, 0.5], [1.0, 1.7], [0.3, -0.2]
    else:
        w = wl.workload("three_mode_24", Nq=[5, 6, 5], Np=[5, 5, 6], K=1)
    # a state of the physical shape: Boltzmann factor times seeded noise
    W = orc.boltzmann(w)[0][None] * (1.0 + 0.3 * wl.noise_state(w, seed=3))
    ref = dense.apply(w, W)
    got = orc.rhs(w, W)
    assert np.linalg.norm(got - ref) <= 1e-12 * np.linalg.norm(ref)


def test_rhs_point_matches_full_rhs():
    w = wl.workload("two_mode_32", Nq=[7, 6], Np=[6, 8], K=2)
    W = wl.noise_state(w, seed=5)
    full = orc.rhs(w, W).reshape(W.shape[0], -1)
    rng = np.random.default_rng(1)
    for _ in range(20):
        e = int(rng.integers(W.shape[0]))
        i = int(rng.integers(full.shape[1]))
        assert abs(orc.rhs_point(w, W, e, i) - full[e, i]) <= 1e-13 * np.abs(full).max()


# ---------------------------------------------------------------------------
# classical RK4: one step is the degree-4 Taylor polynomial of exp(dt L)
# ---------------------------------------------------------------------------

def test_rk4_is_fourth_order_taylor_of_generator():
    w = wl.workload("one_mode_48", Nq=[8], Np=[8], K=2)
    G, f = dense.generator(w)
    G = G.toarray()
    dt = 0.01
    X = dt * G
    T4 = np.eye(G.shape[0]) + X + X @ X / 2 + X @ X @ X / 6 + X @ X @ X @ X / 24
    W = orc.boltzmann(w)[0][None] * (1.0 + 0.3 * wl.noise_state(w, seed=7))
    ref = W.ravel() / f
    for _ in range(3):
        ref = T4 @ ref
    ref = f * ref
    got = orc.rk4(w, W, 3, dt).ravel()
    assert np.linalg.norm(got - ref) <= 1e-13 * np.linalg.norm(ref)


def test_symmetrised_discretization_is_stable():
    """Discretizing the hierarchy on W itself with the compact operator makes
    grid-scale modes grow (eigenvalues with real part ~ +6); on the factor h
    of W = exp(-beta H/2) h (Sec. III A) no eigenvalue of the generator has a
    positive real part (the conserved mode sits at zero)."""
    w = wl.workload("one_mode_48", Nq=[24], Np=[24], K=3)
    G_sym, _ = dense.generator(w, symmetrised=True)
    G_raw, _ = dense.generator(w, symmetrised=False)
    ev_sym = np.linalg.eigvals(G_sym.toarray())
    ev_raw = np.linalg.eigvals(G_raw.toarray())
    assert ev_raw.real.max() > 1.0
    assert ev_sym.real.max() < 1e-10


def test_one_mode_equilibration_stays_bounded():
    """The full equilibration of the one-mode workload (4000 RK4 steps,
    t = 20) keeps the state close to the Boltzmann start."""
    w = wl.workload("one_mode_48")
    W0 = orc.boltzmann(w)
    W = orc.rk4(w, W0, 4000, w["dt"])
    assert np.all(np.isfinite(W))
    assert np.abs(W - W0).max() < 1e-3 * np.abs(W0).max()


# ---------------------------------------------------------------------------
# Boltzmann stationarity and conservation (Sec. II B)
# ---------------------------------------------------------------------------

def test_boltzmann_is_stationary_to_sixth_order():
    """exp(-beta H) with W_{n>0} = 0 is an exact stationary state of the
    continuous hierarchy (L e^{-beta H} = 0 and Theta e^{-beta H} = 0), so the
    discrete residual must vanish at the scheme's order."""
    res = []
    for N in (24, 48, 96):
        w = wl.workload("one_mode_48", Nq=[N], Np=[N], K=2)
        W = orc.boltzmann(w)
        res.append(np.linalg.norm(orc.rhs(w, W)) / np.linalg.norm(W))
    rates = np.log2(np.array(res[:-1]) / np.array(res[1:]))
    assert np.all(rates > 5.5), (res, rates)
    # two coupled anharmonic modes with SL coupling
    w = wl.workload("two_mode_32", Nq=[24, 24], Np=[24, 24], K=2)
    W = orc.boltzmann(w)
    assert np.linalg.norm(orc.rhs(w, W)) / np.linalg.norm(W) < 2e-2


def test_boltzmann_normalisation_and_moments_match_quadrature():
    """Z and <q>, <q^2> of the discrete Boltzmann state against adaptive
    quadrature of exp(-beta U) (one anharmonic mode)."""
    w = wl.workload("one_mode_48")
    W = orc.boltzmann(w)
    mom = orc.moments(w, W, 0, 0)
    U = lambda q: 0.5 * q ** 2 - 0.15 * q ** 3 / 6 + 0.02 * q ** 4 / 24
    assert abs(mom[0] - 1.0) < 1e-13
    assert abs(mom[1] - boltzmann_average_1d(U, lambda q: q, 2.0, 6.0)) < 1e-9
    assert abs(mom[3] - boltzmann_average_1d(U, lambda q: q * q, 2.0, 6.0)) < 1e-9
    assert abs(mom[4] - 0.5) < 1e-9  # <p^2> = m / beta


def test_weighted_integral_of_w0_is_conserved():
    """Every n = 0 term of Eq. (eq:HEOM) is a p- or q-derivative of a flux, so
    the integral of W_0 is conserved.  The compact operator acts on the factor
    h of W = exp(-beta H/2) h, so the discrete product rule, and with it
    conservation, holds to the scheme's order: the defect falls at ~h^6, and
    vanishes to rounding for the Boltzmann state itself."""
    defects = []
    for N in (24, 48, 96):
        w = wl.workload("one_mode_48", Nq=[N], Np=[N], K=2)
        W = orc.boltzmann(w)
        r = orc.rhs(w, W)
        assert abs(orc.moments(w, r, 0, 0)[0]) < 1e-16
        grids = np.meshgrid(*[(np.arange(n) + 0.5) / n - 0.5 for n in w["Nq"] + w["Np"]], indexing="ij")
        poly = 1.0 + 0.4 * grids[0] - 0.3 * grids[1] + 0.5 * grids[0] * grids[1]
        W[1] = 0.3 * W[0] * poly               # non-stationary: polynomial times Boltzmann,
        W[0] = W[0] * (1.0 + 0.2 * grids[1])   # the shape the excitations produce
        r = orc.rhs(w, W)
        defects.append(abs(orc.moments(w, r, 0, 0)[0]) / orc.moments(w, np.abs(r), 0, 0)[0])
    rates = np.log2(np.array(defects[:-1]) / np.array(defects[1:]))
    assert defects[1] < 1e-7 and np.all(rates > 4.5), (defects, rates)


def test_weighted_integral_of_w0_is_conserved_in_time():
    """Time-integrated version on a resolved grid: Boltzmann start with a
    non-stationary first element; the integral of W_0 keeps its value to the
    scheme's accuracy on the 48 x 48 grid (~1e-9 over t = 1)."""
    w = wl.workload("one_mode_48", K=3)
    W = orc.boltzmann(w)
    W[1] = 0.3 * W[0]
    q0 = orc.moments(w, W, 0, 0)[0]
    q1 = orc.moments(w, orc.rk4(w, W, 200, 0.005), 0, 0)[0]
    assert abs(q1 - q0) < 1e-8


def test_liouvillian_conserves_energy():
    """d/dt int H W = int H {H, W} = 0 for zeta = 0: pins dU/dq_s against U,
    including the pair couplings g_ss', g_{s^2 s'}, g_{s s'^2}."""
    w = wl.workload("two_mode_32", Nq=[28, 28], Np=[28, 28], K=0, zeta=[0.0, 0.0])
    w["g21"][0][1], w["g12"][0][1] = 0.08, -0.05
    W = orc.boltzmann(w)
    # a non-stationary start: the Boltzmann state of a shifted potential
    W2 = np.roll(W, 2, axis=1)
    r = orc.rhs(w, W2)
    drift = abs(orc.energy(w, r))
    scale = orc.energy(w, np.abs(r))
    assert drift < 1e-6 * scale, (drift, scale)


# ---------------------------------------------------------------------------
# closed forms of the linear model: harmonic U, V = V_LL q
# ---------------------------------------------------------------------------

def order_and_last(errs, hs):
    errs, hs = np.asarray(errs), np.asarray(hs)
    rates = np.log(errs[:-1] / errs[1:]) / np.log(hs[:-1] / hs[1:])
    return rates, errs[-1]


@pytest.mark.parametrize("K", [1, 3])
def test_harmonic_ll_linear_response_closed_form(K):
    """R^(1)(t) = -mu^2 chi(t) with chi from the generalized Langevin equation;
    the hierarchy is exact at any K >= 1 for this model (Eqs. (1Dresponse),
    (eq:HEOM)), so the only error is the grid's: it falls at sixth order."""
    errs, hs = [], []
    t = np.arange(801) * 0.005
    ref = -1.3 ** 2 * chi_brownian(t, 1.0, 1.0, 0.3, 1.0, 1.0)
    for N in (40, 48, 64):
        w = harmonic_ll(N=N, K=K)
        A = wl.optical(1, lin=[1.3])
        R = orc.response_1d(w, A, orc.boltzmann(w), 801, 1, 0.005)
        errs.append(np.abs(R - ref).max() / np.abs(ref).max())
        hs.append(12.0 / N)
    rates, last = order_and_last(errs, hs)
    assert last < 1e-6 and np.all(rates > 5.0), (errs, rates)


def test_free_oscillator_response():
    """zeta = 0 and K = 0: R^(1)(t) = -mu^2 sin(omega t) / (m omega), to the
    grid's sixth-order accuracy."""
    errs, hs = [], []
    t = np.arange(601) * 0.005
    ref = -0.8 ** 2 * np.sin(1.4 * t) / 1.4
    for N in (40, 48, 64):
        w = wl.workload("one_mode_48", Nq=[N], Np=[N], K=0, g3=[0.0], g4=[0.0], zeta=[0.0],
                        omega=[1.4], Lq=[6.0 / 1.4])
        A = wl.optical(1, lin=[0.8])
        R = orc.response_1d(w, A, orc.boltzmann(w), 601, 1, 0.005)
        errs.append(np.abs(R - ref).max())
        hs.append(12.0 / N)
    rates, last = order_and_last(errs, hs)
    assert last < 1e-6 and np.all(rates > 5.0), (errs, rates)


def test_two_mode_bilinear_linear_response_closed_form():
    """Two harmonic modes coupled by g_12 q_1 q_2, each with its own Drude bath:
    R^(1) against the matrix exponential of the mean dynamics.  The p grid
    converges slowly (Sec. III A), so the check is the error level at N = 20
    and its fall from N = 16; doubling g_12 moves the closed form by 14%."""
    errs = []
    for N in (16, 20):
        w = wl.workload("two_mode_32", Nq=[N, N], Np=[N, N], K=1, g3=[0.0, 0.0], g4=[0.0, 0.0],
                        VSL=[0.0, 0.0])
        w["g2"][0][1] = 0.3
        A = wl.optical(2, lin=[1.0, 0.6])
        R = orc.response_1d(w, A, orc.boltzmann(w), 21, 10, 0.005)
        ref = linear_response_1d(w, [1.0, 0.6], np.arange(21) * 10 * 0.005)
        errs.append(np.abs(R - ref).max() / np.abs(ref).max())
    assert errs[1] < 1e-2 and errs[0] / errs[1] > 3.0, errs


@pytest.mark.parametrize("K", [2, 3])
def test_second_moments_pin_the_n_factor(K):
    """Second moments of W_0 from a hot, displaced Gaussian start follow the
    Lyapunov equation of the (q, p, f) stochastic process.  The moment system
    involves W_2, so a Theta coupling without the factor n_s (Eq. (eq:HEOM)
    as printed) misses by ~1e-2; with it the error is ~1e-6."""
    w = harmonic_ll(N=48, K=K)
    N, L = 48, 6.0
    x = -L + (np.arange(N) + 0.5) * (2 * L / N)
    q0, p0, s2 = 0.7, -0.4, 1.0
    g = lambda c: np.exp(-(x - c) ** 2 / (2 * s2)) / np.sqrt(2 * np.pi * s2)
    W = np.zeros(orc.state_shape(w))
    W[0] = np.outer(g(q0), g(p0))
    steps, dt = 400, 0.005
    mom = orc.moments(w, orc.rk4(w, W, steps, dt), 0, 0)
    mean, cov = lyapunov_moments(1.0, 1.0, 0.3, 1.0, 1.0, 2.0, [q0, p0, 0.0],
                                 np.diag([s2, s2, 0.3 / 2.0]), steps * dt)
    ref = [1.0, mean[0], mean[1], cov[0, 0] + mean[0] ** 2, cov[1, 1] + mean[1] ** 2,
           cov[0, 1] + mean[0] * mean[1]]
    np.testing.assert_allclose(mom, ref, rtol=0, atol=1e-5)


# ---------------------------------------------------------------------------
# excitation and observable: sum rules (Eqs. (Opticalexc), (1Dresponse), (2Dresponse))
# ---------------------------------------------------------------------------

def test_linear_response_sum_rules():
    """R^(1)(0) = 0 and dR^(1)/dt(0) = -<(dA/dq)^2>_Boltzmann / m (W_{n>0} = 0);
    the second to the grid's sixth-order accuracy."""
    U = lambda q: 0.5 * q ** 2 - 0.15 * q ** 3 / 6 + 0.02 * q ** 4 / 24
    ref = -boltzmann_average_1d(U, lambda q: (1 + 0.2 * q) ** 2, 2.0, 6.0)
    errs, hs = [], []
    for N in (40, 48, 64):
        w = wl.workload("one_mode_48", Nq=[N], Np=[N], K=2)
        Wb = orc.boltzmann(w)
        A = w["A"]  # q + 0.1 q^2
        u = orc.perturb(w, A, Wb)
        assert abs(orc.observe(w, A, u)) < 1e-13
        errs.append(abs(orc.observe(w, A, orc.rhs(w, u)) - ref) / abs(ref))
        hs.append(12.0 / N)
    rates, last = order_and_last(errs, hs)
    assert last < 1e-6 and np.all(rates > 5.0), (errs, rates)


def test_excitation_first_moment_in_p():
    """int p (X^x W) dq dp = -int dX/dq W dq dp (integration by parts in p),
    to the grid's sixth-order accuracy."""
    X = wl.optical(1, lin=[0.7], quad=[[0.2]])
    errs, hs = [], []
    for N in (32, 40, 48):
        w = wl.workload("one_mode_48", Nq=[N], Np=[N], K=1)
        W = orc.boltzmann(w)
        u = orc.perturb(w, X, W)
        lhs = orc.moments(w, u, 0, 0)[2]
        rhs = -(X["lin"][0] * orc.moments(w, W, 0, 0)[0] + X["quad"][0][0] * orc.moments(w, W, 0, 0)[1])
        errs.append(abs(lhs - rhs) / abs(rhs))
        hs.append(12.0 / N)
    rates, last = order_and_last(errs, hs)
    assert last < 1e-5 and np.all(rates > 5.0), (errs, rates)


def test_second_order_response_vanishes_at_t2_zero():
    """R^(2)(t2 = 0, t1) = sum_s int C dB/dq_s dU_0/dp_s = 0 (integration by
    parts in p); discretely the residue falls at the grid's order."""
    B = wl.optical(1, lin=[1.0], quad=[[0.1]])
    errs, hs = [], []
    for N in (32, 40, 48):
        w = wl.workload("one_mode_48", Nq=[N], Np=[N], K=2)
        R = orc.response_2d(w, w["A"], B, w["A"], orc.boltzmann(w), 6, 3, 40, 40, 0.005)
        assert np.abs(R[1:]).max() > 1e-3
        errs.append(np.abs(R[0]).max() / np.abs(R[1:]).max())
        hs.append(12.0 / N)
    rates, last = order_and_last(errs, hs)
    assert last < 1e-5 and np.all(rates > 5.0), (errs, rates)


def test_second_order_response_parity_zero():
    """Even U, odd V (V_SL = 0) and linear A, B, C on a symmetric grid: the
    dynamics commute with (q, p, f) -> -(q, p, f), A^x W_eq is odd, B^x maps
    odd to even, so R^(2) vanishes identically; quadratic B breaks it."""
    w = wl.workload("two_mode_32", Nq=[10, 10], Np=[10, 10], K=2, g3=[0.0, 0.0], VSL=[0.0, 0.0])
    Wb = orc.boltzmann(w)
    lin = wl.optical(2, lin=[1.0, 0.7])
    R0 = orc.response_2d(w, lin, lin, lin, Wb, 3, 4, 3, 3, 0.005)
    quadB = wl.optical(2, lin=[1.0, 0.7], quad=[[0.0, 0.3], [0.3, 0.0]])
    R1 = orc.response_2d(w, lin, quadB, lin, Wb, 3, 4, 3, 3, 0.005)
    assert np.abs(R1).max() > 1e-6
    assert np.abs(R0).max() < 1e-12 * np.abs(R1).max()


def _potential_np(w, Q):
    """U(q) of the model (Sec. II A, with the quartic on-site term) on arrays."""
    M = w["M"]
    U = 0.0
    for s in range(M):
        x = Q[s]
        U = U + 0.5 * w["m"][s] * w["omega"][s] ** 2 * x ** 2 + w["g3"][s] * x ** 3 / 6 + w["g4"][s] * x ** 4 / 24
        for t in range(s + 1, M):
            y = Q[t]
            U = U + w["g2"][s][t] * x * y + (w["g21"][s][t] * x * x * y + w["g12"][s][t] * x * y * y) / 6
    return U


def _boltzmann_average(w, f, n):
    """<f(q)> under exp(-beta U) over the q box, tensor Gauss-Legendre with n
    nodes per axis (independent of the oracle's grid and quadrature)."""
    M = w["M"]
    nodes, wts = [], []
    for s in range(M):
        x, wt = np.polynomial.legendre.leggauss(n)
        nodes.append(x * w["Lq"][s])
        wts.append(wt * w["Lq"][s])
    Q = np.meshgrid(*nodes, indexing="ij")
    Wt = np.ones_like(Q[0])
    for s in range(M):
        shape = [1] * M
        shape[s] = n
        Wt = Wt * wts[s].reshape(shape)
    b = Wt * np.exp(-w["beta"] * _potential_np(w, Q))
    return float((b * f(Q)).sum() / b.sum())


def _dX(X, s, Q):
    M = len(Q)
    return X["lin"][s] + sum(0.5 * (X["quad"][s][t] + X["quad"][t][s]) * Q[t] for t in range(M))


_X2 = wl.optical(2, lin=[1.0, 0.7], quad=[[0.2, 0.1], [0.1, -0.3]])
_X3 = wl.optical(3, lin=[1.0, 0.7, 0.5], quad=[[0.2, 0.1, 0.05], [0.1, -0.3, 0.08], [0.05, 0.08, 0.1]])


@pytest.mark.parametrize("M", [2, 3])
def test_linear_response_slope_sum_rule_multimode(M):
    """dR^(1)/dt(0) = -sum_s <(dA/dq_s)^2>_Boltzmann / m_s for anharmonic,
    coupled modes and an operator with cross terms quad_ss' q_s q_s'
    (Eqs. (Opticalexc), (1Dresponse)); the reference is a Gauss-Legendre
    average over the q box, and the oracle converges to it at sixth order."""
    name, X, Ns, K, nq = ("two_mode_32", _X2, (24, 32, 40), 1, 96) if M == 2 else \
        ("three_mode_24", _X3, (12, 14, 16), 0, 48)
    w0 = wl.workload(name)
    ref = -sum(_boltzmann_average(w0, lambda Q, s=s: _dX(X, s, Q) ** 2, nq) / w0["m"][s] for s in range(M))
    errs, hs = [], []
    for N in Ns:
        w = wl.workload(name, Nq=[N] * M, Np=[N] * M, K=K)
        u = orc.perturb(w, X, orc.boltzmann(w))
        errs.append(abs(orc.observe(w, X, orc.rhs(w, u)) - ref) / abs(ref))
        hs.append(1.0 / N)
    rates, last = order_and_last(errs, hs)
    assert last < (1e-5 if M == 2 else 3e-3) and np.all(rates > 5.5), (errs, rates)


@pytest.mark.parametrize("M", [2, 3])
def test_excitation_acts_on_every_element(M):
    """X^x acts on every hierarchy element (Eq. (Opticalexc) on the full
    density, whose f-moments are the elements): for each n and s,
    int p_s (X^x W)_n = -int dX/dq_s W_n, by parts in p.  The identity holds
    at every q point, so q stays coarse and p is refined; the error falls at
    sixth order.  An excitation of element 0 alone fails it for n >= 1."""
    name, X, Nq, Ns = ("two_mode_32", _X2, [6, 5], (24, 32, 40)) if M == 2 else \
        ("three_mode_24", _X3, [4, 3, 5], (16, 20, 24))
    errs, hs = [], []
    for N in Ns:
        w = wl.workload(name, Nq=Nq, Np=[N] * M, K=1)
        axes = [-w["Lq"][s] + (np.arange(w["Nq"][s]) + 0.5) * 2 * w["Lq"][s] / w["Nq"][s] for s in range(M)]
        axes += [-w["Lp"][s] + (np.arange(N) + 0.5) * 2 * w["Lp"][s] / N for s in range(M)]
        G = np.meshgrid(*axes, indexing="ij")
        Wb = orc.boltzmann(w)[0]
        W = np.zeros(orc.state_shape(w))
        rng = np.random.default_rng(4)
        for n in range(W.shape[0]):
            c = rng.uniform(-0.5, 0.5, size=2 * M)
            W[n] = Wb * (0.5 + n + sum(c[k] * G[k] for k in range(2 * M)) + 0.1 * G[M] * G[-1])
        u = orc.perturb(w, X, W)
        e = []
        for n in range(W.shape[0]):
            for s in range(M):
                lhs = orc.moments(w, u, n, s)[2]
                rhs = -(X["lin"][s] * orc.moments(w, W, n, s)[0]
                        + sum(0.5 * (X["quad"][s][t] + X["quad"][t][s]) * orc.moments(w, W, n, t)[1]
                              for t in range(M)))
                e.append(abs(lhs - rhs) / abs(rhs))
        errs.append(max(e))
        hs.append(1.0 / N)
    rates, last = order_and_last(errs, hs)
    assert last < (5e-6 if M == 2 else 1e-4) and np.all(rates > 5.5), (errs, rates)


def _harmonic_ll_w(N, K):
    return wl.workload("one_mode_48", Nq=[N], Np=[N], K=K, g3=[0.0], g4=[0.0], VSL=[0.0])


@pytest.mark.parametrize("case", ["quadB_K3", "linB_quadC_K2"])
def test_second_order_response_gaussian_closed_form(case):
    """The whole double loop of Eq. (2Dresponse) against a closed form.  For a
    harmonic mode with linear-linear coupling the density stays polynomial x
    P_eq(q, p, f), so R^(2) is a Gaussian expectation (tests/physics_refs.py).
    B^x then acts on hierarchy elements n >= 1 of G(t1) A^x W_eq, which are
    nonzero.  Quadratic B gives a cubic density (exact at depth 3); linear B
    with quadratic C a quadratic one (exact at depth 2).  Sixth-order
    convergence at two sets of strides; exciting element 0 alone misses by
    ~7e-3 at every N."""
    if case == "quadB_K3":
        A, B, C = wl.optical(1, lin=[1.0]), wl.optical(1, lin=[0.5], quad=[[0.6]]), \
            wl.optical(1, lin=[1.0], quad=[[0.2]])
        K, n1, n2, s1, s2 = 3, 4, 5, 40, 40
    else:
        A, B, C = wl.optical(1, lin=[1.0]), wl.optical(1, lin=[0.8]), wl.optical(1, lin=[0.3], quad=[[0.5]])
        K, n1, n2, s1, s2 = 2, 3, 4, 25, 60
    dt = 0.005
    ref = response_2d_gaussian(_harmonic_ll_w(48, K), A, B, C, np.arange(n1) * s1 * dt, np.arange(n2) * s2 * dt)
    assert np.abs(ref).max() > 1e-2
    errs, hs = [], []
    for N in (32, 40, 48):
        w = _harmonic_ll_w(N, K)
        R = orc.response_2d(w, A, B, C, orc.boltzmann(w), n1, n2, s1, s2, dt)
        errs.append(np.abs(R - ref).max() / np.abs(ref).max())
        hs.append(1.0 / N)
    rates, last = order_and_last(errs, hs)
    assert last < 1e-5 and np.all(rates > 5.5), (errs, rates)


def test_second_order_response_gaussian_closed_form_two_modes():
    """Two harmonic modes with a bilinear coupling and their own Drude baths,
    B with a cross term Pi_12 q_1 q_2: R^(2) against the Gaussian closed form.
    Depth 2 (the depth-3 terms move R by ~1e-10 here).  The p grid converges
    slowly (Sec. III A), so the check is the error at N = 20 and its
    sixth-order fall from N = 16."""
    A = wl.optical(2, lin=[1.0, 0.6])
    B = wl.optical(2, lin=[0.4, 0.3], quad=[[0.5, 0.3], [0.3, -0.2]])
    C = wl.optical(2, lin=[1.0, 0.6])
    n1, n2, s1, s2, dt = 2, 3, 10, 10, 0.02
    errs = []
    for N in (16, 20):
        w = wl.workload("two_mode_32", Nq=[N, N], Np=[N, N], K=2, g3=[0.0, 0.0], g4=[0.0, 0.0], VSL=[0.0, 0.0])
        w["g2"][0][1] = 0.3
        ref = response_2d_gaussian(w, A, B, C, np.arange(n1) * s1 * dt, np.arange(n2) * s2 * dt)
        R = orc.response_2d(w, A, B, C, orc.boltzmann(w), n1, n2, s1, s2, dt)
        errs.append(np.abs(R - ref).max() / np.abs(ref).max())
    assert errs[1] < 3e-3 and errs[0] / errs[1] > (20 / 16) ** 5.5, errs


@pytest.mark.parametrize("case", ["quad_BD", "quad_BCD"])
def test_third_order_response_gaussian_closed_form(case):
    """R^(3)(t3, t2, t1) of Eq. (3Dresponse) for one harmonic mode with
    linear-linear coupling against the Gaussian closed form, under grid
    refinement: sixth-order convergence.  With linear operators only, a
    linear system has no third-order response, and by parity a quadratic B
    alone leaves R^(3) zero too; the cases have a quadratic B and D, and a
    quadratic B, C and D.  The hierarchy holds the perturbed density exactly
    once its depth reaches the density's degree in f: four for a quadratic
    B and linear C (degrees 1, 3, 4 after A^x, B^x, C^x), five with C
    quadratic too.  An oracle that excites element 0 only, drops the
    waiting-time propagation or applies C^x before it misses by O(1)."""
    if case == "quad_BD":
        A, B, C, D = (wl.optical(1, lin=[1.0]), wl.optical(1, lin=[0.8], quad=[[0.5]]),
                      wl.optical(1, lin=[0.6]), wl.optical(1, lin=[1.0], quad=[[0.4]]))
        K, n1, t2s, n3, s1, s3 = 4, 3, 40, 4, 25, 30
    else:
        A, B, C, D = (wl.optical(1, lin=[1.0]), wl.optical(1, lin=[0.5], quad=[[0.4]]),
                      wl.optical(1, lin=[0.7], quad=[[-0.3]]), wl.optical(1, lin=[1.0], quad=[[0.2]]))
        K, n1, t2s, n3, s1, s3 = 5, 3, 20, 4, 40, 40
    dt = 0.005
    ref = response_3d_gaussian(_harmonic_ll_w(48, K), A, B, C, D, np.arange(n1) * s1 * dt, t2s * dt,
                               np.arange(n3) * s3 * dt)
    assert np.abs(ref).max() > 1e-3
    errs, hs = [], []
    for N in (40, 48, 56, 64):
        w = _harmonic_ll_w(N, K)
        R = orc.response_3d(w, A, B, C, D, orc.boltzmann(w), n1, t2s, n3, s1, s3, dt)
        errs.append(np.abs(R - ref).max() / np.abs(ref).max())
        hs.append(1.0 / N)
    rates, last = order_and_last(errs, hs)
    # the densities are polynomials of degree 4-5 in (q, p, f): the p grid
    # resolves them more slowly than R^(2)'s, so the grids run to N = 64
    # (the oracle has no axis limit) and the bar is the sixth-order fall
    assert last < 1e-3 and np.all(rates > 5.5), (errs, rates)


def test_third_order_response_columns_and_t3_zero():
    """The listed-column form of R^(3) equals the full one column by column,
    and R^(3)(t3 = 0) vanishes at the scheme's order (the integral of C^x V
    against D is a sum of p-derivatives): the t3 = 0 row falls at sixth
    order from N = 32 to 48, to below 2e-3 of the signal."""
    A, B, C, D = (wl.optical(1, lin=[1.0], quad=[[0.2]]), wl.optical(1, lin=[0.7], quad=[[0.3]]),
                  wl.optical(1, lin=[0.9]), wl.optical(1, lin=[1.0], quad=[[0.2]]))
    zero = []
    for N in (32, 48):
        w = _harmonic_ll_w(N, 3)
        Wb = orc.boltzmann(w)
        full = orc.response_3d(w, A, B, C, D, Wb, 4, 20, 5, 10, 10, 0.005)
        zero.append(np.abs(full[0]).max() / np.abs(full).max())
    part = orc.response_3d(w, A, B, C, D, Wb, 4, 20, 5, 10, 10, 0.005, j1_list=[1, 3])
    np.testing.assert_array_equal(part[:, [1, 3]], full[:, [1, 3]])
    assert np.all(np.isnan(part[:, [0, 2]]))
    rate = np.log(zero[0] / zero[1]) / np.log(48 / 32)
    assert zero[1] < 2e-3 and rate > 5.5, (zero, rate)


# ---------------------------------------------------------------------------
# spectra, Eqs. (1DIR_Raman), (2DThz_Raman): Fourier sums of known signals
# ---------------------------------------------------------------------------

def test_spectrum_1d_geometric_sum():
    n, tau, lam, Om = 256, 0.05, 0.3, 2.0
    t = np.arange(n) * tau
    R = np.exp(-lam * t) * np.sin(Om * t)
    omega, I = orc.spectrum_1d(R, tau)
    z = lambda wv: np.exp((1j * wv - lam) * tau)
    # sum_j e^{i w t_j} e^{-lam t_j} sin(Om t_j) = (S(w+Om) - S(w-Om)) / 2i
    S = lambda wv: (1 - z(wv) ** n) / (1 - z(wv))
    ref = omega * np.imag(tau * (S(omega + Om) - S(omega - Om)) / 2j)
    np.testing.assert_allclose(I, ref, rtol=0, atol=1e-10 * np.abs(ref).max())
    # and against numpy's inverse FFT (e^{+i} convention)
    ref2 = omega * np.imag(tau * n * np.fft.ifft(R))
    np.testing.assert_allclose(I, ref2, rtol=0, atol=1e-10 * np.abs(ref2).max())


def test_spectrum_2d_against_fft():
    rng = np.random.default_rng(2)
    R = rng.standard_normal((16, 8))
    _, _, I = orc.spectrum_2d(R, 0.1, 0.2)
    ref = np.imag(0.1 * 0.2 * np.fft.fft2(R))
    np.testing.assert_allclose(I, ref, rtol=0, atol=1e-12)


def test_spectrum_2dir_against_fft():
    """Eq. (noncorrelation): e^{-i omega1 t1} along t1 (numpy's forward FFT)
    and e^{+i omega3 t3} along t3 (n3 times its inverse FFT)."""
    rng = np.random.default_rng(3)
    R = rng.standard_normal((12, 10))
    w1, w3, I = orc.spectrum_2dir(R, 0.1, 0.2)
    ref = np.imag(0.1 * 0.2 * 12 * np.fft.ifft(np.fft.fft(R, axis=1), axis=0))
    np.testing.assert_allclose(I, ref, rtol=0, atol=1e-12)
    np.testing.assert_allclose(w1, 2 * np.pi * np.arange(10) / (10 * 0.1))
    np.testing.assert_allclose(w3, 2 * np.pi * np.arange(12) / (12 * 0.2))
