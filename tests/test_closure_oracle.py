"""Pins of the closure oracle (CPU): restriction, the quadratic loss and its
moments, the skew structure of the corrected derivative, the network's
gradients and BF16 rounding.  Each is checked against an independent
computation: exact values, brute force over explicit lines, finite
differences, or the C oracle."""
import numpy as np
import pytest

import oracle as orc
import oracle.closure as cl
import oracle.dense as dn
import workloads as wl


def test_restriction_is_exact_for_linear_functions():
    # cell-centred 2:1 nesting: the mean of two fine centres is the coarse centre
    L, Nf = 6.0, 12
    xf = dn.grid(Nf, L)
    xc = dn.grid(Nf // 2, L)
    q, p = np.meshgrid(xf, xf, indexing="ij")
    f = (1.5 * q - 0.7 * p + 0.3)[None]
    Qc, Pc = np.meshgrid(xc, xc, indexing="ij")
    assert np.allclose(cl.restrict(f)[0], 1.5 * Qc - 0.7 * Pc + 0.3, atol=1e-14)
    # and conserves the plain sum (interior weights)
    g = np.random.default_rng(0).standard_normal((2, 8, 6))
    assert abs(cl.restrict(g).sum() * 4 - g.sum()) < 1e-12


def test_corrected_derivative_keeps_the_skew_structure():
    N, h = 12, 0.5
    s = np.random.default_rng(1).normal(0, 0.1, cl.n_entries(N))
    A, B = dn.compact_matrices(N)
    D = cl.closure_derivative_matrix(N, h, s)
    X = A @ D * h
    assert np.abs((X + X.T)).max() < 1e-13          # A D h = B + S is skew
    assert np.allclose(cl.closure_derivative_matrix(N, h, np.zeros(cl.n_entries(N))),
                       dn.derivative_matrix(N, h), atol=1e-14)


def _lines(seed, N=7, n=40):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((N, n)), rng.standard_normal((N, n))


def test_gram_from_moments_matches_explicit_lines():
    N, h = 7, 0.8
    X, Rr = _lines(2, N)
    G, b = cl.gram(N, h, X @ X.T, X @ Rr.T)
    A, _ = dn.compact_matrices(N)
    P = cl.n_entries(N)
    Gb = np.zeros((P, P))
    bb = np.zeros(P)
    for col in range(X.shape[1]):
        x, r = X[:, col], Rr[:, col]
        V = np.stack([np.linalg.solve(A, cl.skew_matrix(N, np.eye(P)[e]) @ x) / h for e in range(P)])
        Gb += V @ V.T
        bb += V @ r
    assert np.allclose(G, Gb, rtol=1e-12, atol=1e-12)
    assert np.allclose(b, bb, rtol=1e-12, atol=1e-12)


def test_quadratic_loss_equals_the_residual_it_models():
    N, h = 7, 0.8
    X, Rr = _lines(3, N)
    G, b = cl.gram(N, h, X @ X.T, X @ Rr.T)
    s = np.random.default_rng(4).normal(0, 0.2, cl.n_entries(N))
    corr = (cl.closure_derivative_matrix(N, h, s) - dn.derivative_matrix(N, h)) @ X
    direct = float(((Rr - corr) ** 2).sum())
    assert abs(cl.group_loss(s, G, b, float((Rr ** 2).sum()), 1.0) - direct) < 1e-10 * direct


def test_planted_closure_is_recovered_by_least_squares():
    # targets made by a known closure: the quadratic's minimiser is that closure
    N, h = 8, 0.5
    rng = np.random.default_rng(5)
    s_true = rng.normal(0, 0.05, cl.n_entries(N))
    X = rng.standard_normal((N, 200))
    Rr = (cl.closure_derivative_matrix(N, h, s_true) - dn.derivative_matrix(N, h)) @ X
    G, b = cl.gram(N, h, X @ X.T, X @ Rr.T)
    assert np.allclose(np.linalg.solve(G, b), s_true, atol=1e-10)


def test_moments_of_a_state_match_the_definition():
    wf = wl.workload("one_mode_48", Nq=[12], Np=[12], K=1)
    h = orc.boltzmann(wf) * (1 + 0.1 * np.random.default_rng(6).standard_normal((2, 12, 12)))
    Mx, Cxr, c, t = cl.moments(wf, h, 1)
    x = cl.restrict(h)
    T = cl.restrict(cl.along(dn.derivative_matrix(12, 1.0), h, 2))
    r = T - cl.along(dn.derivative_matrix(6, 2.0), x, 2)
    xs = x.reshape(-1, 6)
    rs = r.reshape(-1, 6)
    assert np.allclose(Mx, xs.T @ xs) and np.allclose(Cxr, xs.T @ rs)
    assert np.isclose(c, (r * r).sum()) and np.isclose(t, (T * T).sum())


def test_network_gradients_match_finite_differences():
    rng = np.random.default_rng(7)
    X = rng.standard_normal((37, cl.NFEAT))
    p = cl.init_params(3)
    p["b1"] = rng.normal(0, 0.1, cl.NHID)
    p["b2"] = 0.05
    gs = rng.standard_normal(37)
    s, cache = cl.forward(p, X, rounding=False)
    g = cl.backward(p, cache, gs, rounding=False)
    eps = 1e-6
    for key, idx in (("W1", (3, 5)), ("W1", (15, 31)), ("b1", (7,)), ("W2", (11,)), ("b2", None)):
        q = {k: np.array(v, dtype=np.float64, copy=True) for k, v in p.items()}
        qm = {k: np.array(v, dtype=np.float64, copy=True) for k, v in p.items()}
        if idx is None:
            q[key] = q[key] + eps
            qm[key] = qm[key] - eps
            ga = g[key]
        else:
            q[key][idx] += eps
            qm[key][idx] -= eps
            ga = g[key][idx]
        fd = (gs @ cl.forward(q, X, False)[0] - gs @ cl.forward(qm, X, False)[0]) / (2 * eps)
        assert abs(fd - ga) < 1e-7 * max(1.0, abs(fd)), key


def test_bf16_rounding_ties_to_even():
    one = 1.0
    ulp = 2.0 ** -7
    vals = [one, one + ulp / 2, one + 3 * ulp / 2, one + ulp / 4, -(one + 3 * ulp / 2), 3.0 * 2 ** 100]
    want = [one, one, one + 2 * ulp, one, -(one + 2 * ulp), 3.0 * 2 ** 100]
    assert np.array_equal(cl.bf16(vals), np.array(want))


def test_plain_closure_solver_equals_the_c_oracle():
    # the sparse-assembled closure solver with the plain stencil reproduces
    # the independent C oracle (RK4 steps and the excitation)
    w = wl.workload("two_mode_32", Nq=[6, 7], Np=[6, 6], K=2)
    W = orc.boltzmann(w) * (1 + 0.1 * np.random.default_rng(8).standard_normal(orc.state_shape(w)))
    zero = np.zeros(len(cl.features(w)))
    assert np.linalg.norm(cl.propagate(w, W, 3, 0.002, zero) - orc.rk4(w, W, 3, 0.002)) \
        < 1e-13 * np.linalg.norm(W)
    A = w["A"]
    ref = orc.perturb(w, A, W)
    assert np.abs(cl.perturb(w, A, W, zero) - ref).max() < 1e-13 * np.abs(ref).max()


def test_features_follow_the_definition():
    w = wl.workload("two_mode_32", Nq=[8, 8], Np=[8, 8])
    F = cl.features(w)
    assert F.shape == (4 * (2 * 8 - 3), cl.NFEAT)
    assert np.all(F[:, -1] == 1.0)
    # first row: q_1 entry S[0][1], midpoint between the first two cells
    L, h = w["Lq"][0], 2 * w["Lq"][0] / 8
    u = (-L + h) / L
    assert np.isclose(F[0, 0], u) and np.isclose(F[0, 2], abs(u)) and F[0, 3] == 0.0 and F[0, 4] == 0.0
    assert F[0, 14] == 1.0
    # rows 7.. are S[i][i+2]
    assert F[7, 3] == 1.0 and F[6, 3] == 0.0
    assert np.allclose(cl.row_axes(w), np.repeat(np.arange(4), 13))


def test_adam_first_and_constant_gradient_steps_follow_the_published_update():
    """Facts of Adam (Kingma & Ba) that fix the update without retyping it:
    with bias correction, the first step has m_hat = g and v_hat = g^2, so a
    parameter with gradient g moves by -lr g / (|g| + eps), i.e.
    -lr sign(g) (1 - O(eps/|g|)), and one with g = 0 does not move; under a
    constant gradient every later step is the same, while a gradient that
    flips sign after many steps moves the parameter against the new sign
    only once the first moment has turned (it keeps the old direction for
    about ln 2 / (1 - beta1) ~ 7 steps)."""
    rng = np.random.default_rng(4)
    p0 = cl.init_params(5)
    g = {k: rng.standard_normal(np.shape(v)) for k, v in p0.items() if k != "b2"}
    g["b2"] = 0.3
    g["W1"][0, :4] = 0.0  # untouched entries
    lr = 1e-3
    p = {k: np.array(v, dtype=np.float64, copy=True) for k, v in p0.items()}
    st = {}
    cl.adam_step(p, g, st, lr)
    for k in p:
        d = np.asarray(p[k]) - np.asarray(p0[k])
        gk = np.asarray(g[k], dtype=np.float64)
        np.testing.assert_allclose(d, -lr * gk / (np.abs(gk) + 1e-8), rtol=1e-9, atol=1e-15)
    assert np.all(p["W1"][0, :4] == p0["W1"][0, :4])
    big = np.abs(g["W2"]) > 1e-3
    np.testing.assert_allclose((p["W2"] - p0["W2"])[big], -lr * np.sign(g["W2"][big]), rtol=1e-5)
    # constant gradient: steps 2..20 repeat the first one
    prev = {k: np.array(v, copy=True) for k, v in p.items()}
    for _ in range(19):
        cl.adam_step(p, g, st, lr)
        for k in p:
            gk = np.asarray(g[k], dtype=np.float64)
            np.testing.assert_allclose(np.asarray(p[k]) - prev[k], -lr * gk / (np.abs(gk) + 1e-8),
                                       rtol=1e-9, atol=1e-15)
            prev[k] = np.array(p[k], copy=True)
    # the gradient of one scalar flips after 20 steps
    x = {"W1": np.zeros((cl.NFEAT, cl.NHID)), "b1": np.zeros(cl.NHID), "W2": np.zeros(cl.NHID), "b2": 0.0}
    gx = {"W1": np.zeros((cl.NFEAT, cl.NHID)), "b1": np.zeros(cl.NHID), "W2": np.zeros(cl.NHID), "b2": 1.0}
    sx = {}
    for _ in range(20):
        cl.adam_step(x, gx, sx, lr)
    gx["b2"] = -1.0
    moves = []
    for _ in range(12):
        before = x["b2"]
        cl.adam_step(x, gx, sx, lr)
        moves.append(x["b2"] - before)
    first_up = next(i for i, mv in enumerate(moves) if mv > 0)
    assert all(mv < 0 for mv in moves[:first_up]) and 5 <= first_up <= 9, moves
