"""The learned closure on the GPU (through the C ABI) against the closure
oracle: features, training moments, the network's forward and backward
passes (the oracle rounds to BF16 where the device does), training steps,
and the coarse solver with a closure (right-hand side, RK4, excitation,
2D response) on small grids that take both line solvers."""
import copy
import sys

import numpy as np
import pytest

import oracle as orc
import oracle.closure as cl
import workloads as wl

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rel(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.fixture(scope="module")
def pk():
    import torch
    import paper_2509_25840_amd as pk
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    return pk


def phys_state(w, seed, noise=0.05):
    env = orc.boltzmann(w)[0]
    sm = wl.smooth_state(w, seed=seed)
    sm = sm / np.abs(sm).max()
    nz = wl.noise_state(w, seed=seed + 1000)
    return env[None] * (1.0 + 0.3 * sm + noise * nz)


COARSE = {
    "m1_n12": wl.workload("one_mode_48", Nq=[12], Np=[12], K=3),
    "m2_n8": wl.workload("two_mode_32", Nq=[8, 8], Np=[8, 8], K=2),       # lane-pair solves
    "m2_n6": wl.workload("two_mode_32", Nq=[6, 7], Np=[6, 6], K=2),       # one-lane solves
    "m3_n6": wl.workload("three_mode_24", Nq=[6, 6, 6], Np=[6, 6, 6], K=2),
    # cubic 8^3 p blocks: k_pcube's lane-pair plane solves with the closure
    "m3_c8": wl.workload("three_mode_24", Nq=[6, 7, 6], Np=[8, 8, 8], K=2),
}


def fine_of(w):
    f = copy.deepcopy(w)
    f["Nq"] = [2 * n for n in w["Nq"]]
    f["Np"] = [2 * n for n in w["Np"]]
    return f


@pytest.mark.parametrize("name", ["m1_n12", "m2_n8", "m3_n6"])
def test_features_match_the_oracle(pk, name):
    w = COARSE[name]
    feat, axis = pk.closure_features(pk.params_from_workload(w))
    ref = cl.features(w).astype(np.float32)
    assert np.array_equal(axis, cl.row_axes(w))
    assert np.allclose(feat, ref, rtol=1e-6, atol=1e-7)


@pytest.mark.parametrize("name", ["m1_n12", "m2_n6"])
def test_moments_match_the_oracle(pk, name):
    wc = COARSE[name]
    wf = fine_of(wc)
    say(f"[moments] {name} fine {wf['Nq']} {wf['Np']}")
    Wf = phys_state(wf, seed=11)
    with pk.Solver(pk.params_from_workload(wf)) as s:
        s.set_state(Wf)
        Gs, bs, ct = s.closure_moments()
    f = cl._hfactor(wf)
    h = Wf / f[None]
    N, hc, _ = cl.axis_lengths(wc)
    for a in range(2 * wc["M"]):
        Mx, Cxr, c, t = cl.moments(wf, h, a)
        G, b = cl.gram(N[a], hc[a], Mx, Cxr)
        assert rel(Gs[a], G) < 1e-10, a
        assert rel(bs[a], b) < 1e-10, a
        assert abs(ct[a, 0] - c) <= 1e-10 * c and abs(ct[a, 1] - t) <= 1e-10 * t


def _params(seed):
    p = cl.init_params(seed)
    rng = np.random.default_rng(seed + 100)
    p["b1"] = rng.normal(0, 0.1, cl.NHID)
    p["b2"] = 0.02
    return p


def _flat(p):
    return np.concatenate([np.ravel(p["W1"]), p["b1"], p["W2"], [p["b2"]]]).astype(np.float32)


def _unflat(v):
    v = np.asarray(v, dtype=np.float64)
    return {"W1": v[:512].reshape(16, 32), "b1": v[512:544], "W2": v[544:576], "b2": float(v[576])}


def test_network_forward_and_backward_match_the_oracle(pk):
    w = COARSE["m3_n6"]
    feat = cl.features(w).astype(np.float32)       # 54 rows: ragged last tile
    p = _unflat(_flat(_params(1)))
    s_dev = pk.closure_eval(_flat(p), feat)
    s_ref, cache = cl.forward(p, feat.astype(np.float64))
    assert rel(s_dev, s_ref) < 2e-6
    gs = np.random.default_rng(2).standard_normal(len(feat)).astype(np.float32)
    g_dev = pk.closure_grad(_flat(p), feat, gs)
    g_ref = cl.backward(p, cache, gs.astype(np.float64))
    g_ref = np.concatenate([np.ravel(g_ref["W1"]), g_ref["b1"], g_ref["W2"], [g_ref["b2"]]])
    assert rel(g_dev, g_ref) < 1e-4


def _bf16_bounds(p, X, gs):
    """Elementwise bounds on how far a network evaluated with BF16 operands
    (X, W1, tanh(H), W2 and the backward products rounded to BF16, FP32
    accumulation) can be from the exact FP64 network: each product of two
    rounded values has relative error at most 2u + u^2 with u = 2^-9 (half
    of BF16's 2^-8 step), tanh is 1-Lipschitz with slope 1 - tanh^2, and
    FP32 sums add 1e-6 of the absolute sums."""
    u = 2.0 ** -9
    e2 = 2 * u + u * u
    aX, aW1, aW2 = np.abs(X), np.abs(p["W1"]), np.abs(p["W2"])
    absH = aX @ aW1
    dH = (e2 + 1e-6) * absH
    A1 = np.tanh(X @ p["W1"] + p["b1"])
    dA1 = dH * np.minimum(1.0, 1.0 - A1 * A1 + 2.0 * dH)
    ds = ((np.abs(A1) + dA1) * e2 + dA1) @ aW2 + 1e-6 * (np.abs(A1) @ aW2 + abs(p["b2"]))
    ags = np.abs(gs)[:, None]
    dgW2 = (ags * ((np.abs(A1) + dA1) * e2 + dA1)).sum(axis=0) + 1e-6 * (ags * np.abs(A1)).sum(axis=0)
    gH = ags * aW2[None, :] * (1.0 - A1 * A1)
    dgH = ags * aW2[None, :] * (u * (1.0 - A1 * A1) + 2.0 * (np.abs(A1) + dA1) * dA1) * (1 + u)
    dgW1 = aX.T @ (gH * e2 + dgH * (1 + u) ** 2) + 1e-6 * (aX.T @ gH)
    dgb1 = dgH.sum(axis=0) + 1e-6 * gH.sum(axis=0)
    dgb2 = 1e-6 * np.abs(gs).sum()
    return ds, np.concatenate([np.ravel(dgW1), dgb1, dgW2, [dgb2]])


def test_network_matches_the_exact_fp64_network_within_bf16_bounds(pk):
    """The device network against the plain FP64 network (no rounding
    mirrored): every output and gradient entry within the bound BF16
    operands allow (_bf16_bounds), and the bound is tight enough to matter
    (the device differs from the exact network, by a fraction of it)."""
    w = COARSE["m3_n6"]
    feat = cl.features(w).astype(np.float32)
    p = _unflat(_flat(_params(1)))
    p["b1"] = np.float32(np.random.default_rng(3).normal(0, 0.1, 32)).astype(np.float64)
    X = feat.astype(np.float64)
    s_dev = pk.closure_eval(_flat(p), feat)
    s_ex, cache = cl.forward(p, X, rounding=False)
    gs = np.random.default_rng(2).standard_normal(len(feat)).astype(np.float32)
    g_dev = pk.closure_grad(_flat(p), feat, gs)
    g_ex = cl.backward(p, cache, gs.astype(np.float64), rounding=False)
    g_ex = np.concatenate([np.ravel(g_ex["W1"]), g_ex["b1"], g_ex["W2"], [g_ex["b2"]]])
    ds, dg = _bf16_bounds(p, X, gs.astype(np.float64))
    es = np.abs(s_dev - s_ex)
    eg = np.abs(g_dev - g_ex)
    say(f"    forward: max err/bound {np.max(es / ds):.3f}; backward: {np.max(eg / (dg + 1e-30)):.3f}")
    assert np.all(es <= ds) and np.all(eg <= dg + 1e-30)
    assert np.max(es) > 0.0 and np.max(es / ds) > 1e-3  # BF16 rounding is in effect


def _groups(pk, wc, seeds):
    """Training groups (draw, axis) from fine states of draws of wc."""
    feats, gstart, Gs, bs, cts = [], [0], [], [], []
    for sd in seeds:
        wd = wl.draw_perturbed(wc, sd)
        wf = fine_of(wd)
        with pk.Solver(pk.params_from_workload(wf)) as s:
            s.set_state(phys_state(wf, seed=sd, noise=0.0))
            G, b, ct = s.closure_moments()
        f, axis = pk.closure_features(pk.params_from_workload(wd))
        feats.append(f)
        for a in range(2 * wc["M"]):
            gstart.append(gstart[-1] + len(b[a]))
            Gs.append(G[a].ravel())
            bs.append(b[a])
            cts.append(ct[a])
    return (np.concatenate(feats), np.array(gstart, dtype=np.int32), np.concatenate(Gs), np.concatenate(bs),
            np.concatenate(cts))


def test_training_steps_match_the_oracle_and_reduce_the_loss(pk):
    wc = COARSE["m2_n6"]
    feat, gstart, G, b, ct = _groups(pk, wc, [0, 1])
    p0 = _params(4)
    tr = pk.ClosureTrainer(_flat(p0))
    loss = tr.train(feat, gstart, G, b, ct, n_steps=5, lr=1e-3)
    # oracle: the same five steps
    p = _unflat(_flat(p0))
    groups, go, bo = [], 0, 0
    for q in range(len(gstart) - 1):
        P = gstart[q + 1] - gstart[q]
        groups.append((np.arange(gstart[q], gstart[q + 1]), G[go:go + P * P].reshape(P, P), b[bo:bo + P],
                       ct[2 * q], ct[2 * q + 1]))
        go += P * P
        bo += P
    st = {}
    ref_loss = []
    for _ in range(5):
        s, cache = cl.forward(p, feat.astype(np.float64))
        L, gs = cl.loss_grad(s, groups)
        ref_loss.append(L)
        g = cl.backward(p, cache, np.float32(gs).astype(np.float64))
        cl.adam_step(p, g, st, 1e-3)
    say(f"    loss dev {loss} ref {ref_loss}")
    assert np.allclose(loss, ref_loss, rtol=1e-4)
    assert rel(tr.prm, _flat(p)) < 1e-4
    more = tr.train(feat, gstart, G, b, ct, n_steps=300, lr=3e-3)
    assert more[-1] < 0.9 * loss[0]


@pytest.mark.parametrize("run", ["0", "3"])
@pytest.mark.parametrize("name", list(COARSE))
def test_coarse_solver_with_closure_matches_the_oracle(pk, monkeypatch, name, run):
    # run: k_pblock task order (consecutive block groups per state; 0 = default)
    monkeypatch.setenv("CHFPE_TUNE_PB_RUN", run)
    w = COARSE[name]
    say(f"[closure solver] {name} run {run}")
    n = len(cl.features(w))
    sv = np.random.default_rng(9).normal(0, 0.02, n)
    W = phys_state(w, seed=12)
    M = w["M"]
    X = {"lin": [1.0, -0.6, 0.4][:M], "quad": [[0.2, 0.05, 0.0], [0.05, -0.1, 0.02], [0.0, 0.02, 0.3]][:M]}
    X["quad"] = [r[:M] for r in X["quad"]]
    with pk.Solver(pk.params_from_workload(w)) as s:
        s.set_closure(sv)
        s.set_state(W)
        s.propagate(3, 0.002)
        got = s.get_state().reshape(W.shape)
        s.set_state(W)
        s.perturb(X)
        got_p = s.get_state().reshape(W.shape)
        s.set_closure(None)
        s.set_state(W)
        s.propagate(3, 0.002)
        plain = s.get_state().reshape(W.shape)
    ref = cl.propagate(w, W, 3, 0.002, sv)
    assert rel(got, ref) < 1e-13
    assert rel(got_p, cl.perturb(w, X, W, sv)) < 1e-13
    assert rel(plain, orc.rk4(w, W, 3, 0.002)) < 1e-13
    assert rel(got, plain) > 1e-8  # the closure is in effect


def test_closure_response_2d_matches_the_oracle(pk):
    w = COARSE["m2_n8"]
    sv = np.random.default_rng(10).normal(0, 0.02, len(cl.features(w)))
    A, B, C = wl.response_types(w)["TRT"]
    Weq = cl.propagate(w, orc.boltzmann(w), 10, 0.004, sv)
    ref = cl.response_2d(w, A, B, C, Weq, 4, 5, 2, 2, 0.004, sv)
    for batch in (1, 3):
        with pk.Solver(pk.params_from_workload(w, batch=batch)) as s:
            s.set_closure(sv)
            s.equilibrate(10, 0.004)
            got = s.response_2d(A, B, C, 4, 5, 2, 2, 0.004)
        assert rel(got, ref) < 1e-10, batch


def test_trained_closure_beats_the_plain_coarse_grid(pk):
    """Ablation, in the configuration bench.py --mode closure runs: a closure
    trained on fine 32^4 runs of sixteen seeded draws brings the 16^4 coarse
    2D spectrum of the nominal workload (not a training draw) closer to the
    fine FP64 spectrum than the plain coarse grid, over the full 64 x 256
    response after full equilibration."""
    import paper_2509_25840_amd.closure as clo
    w = wl.workload("two_mode_32")
    wc = copy.deepcopy(w)
    wc["Nq"], wc["Np"] = [16, 16], [16, 16]
    dt = w["dt"]
    draws = []
    for sd in range(16):
        wd = wl.draw_perturbed(wc, sd)
        draws.append((wd, clo.fine_moments(wd, 1000, 400, 50, dt)))
    tr, hist = clo.train(clo.training_set(draws), 3000, 3e-3)
    say(f"    loss {hist[0]:.3e} -> {hist[-1]:.3e}")
    assert hist[-1] < 0.5 * hist[0]

    def spectrum(wk, sv=None):
        with pk.Solver(pk.params_from_workload(wk, batch=64)) as s:
            if sv is not None:
                s.set_closure(sv)
            s.equilibrate(w["eq_steps"], dt)
            R = s.response_2d(wk["A"], wk["B"], wk["C"], w["n_t1"], w["n_t2"], 1, 1, dt)
        return pk.spectrum_2d(R, dt, dt)

    I_fine = spectrum(clo.fine_of(wc))
    e_plain = rel(spectrum(wc), I_fine)
    e_clos = rel(spectrum(wc, clo.entries(tr.prm, wc)), I_fine)
    say(f"    spectrum error plain {e_plain:.3e} closure {e_clos:.3e}")
    assert e_clos < 0.5 * e_plain
