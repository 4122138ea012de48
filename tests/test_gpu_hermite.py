"""Parity of the Hermite-basis path (CHFPE_BASIS_HERMITE: k_hcube, k_hperturb)
with the Hermite oracle (``oracle.hermite``, Sec. III A; Appendix A,
Eq. (HEOM2FP-H)), through the C ABI.

Bar: the FP64 bar of the grid path (relative L2 <= 1e-13 for one right-hand
side, a few RK4 steps and the excitation; <= 1e-10 for responses), and 1e-4
for FP32 branch waves.  Grids: one, two and three modes, ragged q cubes and
cubic ones (8, 12 and 24 points: the lane-pair plane solves), Hermite counts
2..6 per mode, hierarchy depths 1..3.
"""
import sys

import numpy as np
import pytest

import oracle.hermite as oh
import workloads as wl

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-10


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.fixture(scope="module")
def pk():
    import torch
    import paper_2509_25840_amd as pk
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    return pk


def hw(base, Nq, Nh, K):
    return wl.workload(base, Nq=list(Nq), Np=list(Nh), K=K, basis="hermite")


SMALL = {
    "h1_n12": hw("one_mode_48", [12], [6], 3),
    "h2_n10": hw("two_mode_32", [10, 9], [5, 6], 2),
    "h3_n8": hw("three_mode_24", [8, 7, 8], [4, 3, 5], 2),
    "h3_c8": hw("three_mode_24", [8, 8, 8], [4, 4, 4], 2),
    "h3_c12": hw("three_mode_24", [12, 12, 12], [3, 3, 3], 2),
    "h3_c24": hw("three_mode_24", [24, 24, 24], [3, 2, 3], 1),
    # edge shapes: a 48-point q_1 line (the largest bucket), depth 0 (no
    # hierarchy neighbours), the minimum of two Hermite functions
    "h1_n48": hw("one_mode_48", [48], [4], 2),
    "h2_k0": hw("two_mode_32", [7, 11], [2, 3], 0),
    "h3_nh2": hw("three_mode_24", [6, 9, 5], [2, 2, 2], 2),
}


def hstate(w, seed):
    """A seeded Hermite state: smooth in q with the Boltzmann envelope's
    width, decaying with the Hermite index, on every element."""
    rng = np.random.default_rng(seed)
    M = w["M"]
    sh = oh.shape(w)
    qs = np.meshgrid(*[oh.q_grid(w, s) for s in range(M)], indexing="ij")
    env = np.exp(-0.35 * sum((w["omega"][s] * qs[s]) ** 2 for s in range(M)))
    C = np.zeros(sh)
    for idx in np.ndindex(*sh[:1 + M]):
        ph = rng.normal(size=M)
        C[idx] = rng.normal() * 0.6 ** sum(idx[1:]) * env * (
            1.0 + 0.4 * sum(np.sin(0.7 * qs[s] + ph[s]) for s in range(M)))
    return C


def optical(M):
    X = wl.optical(M, lin=[1.0, -0.7, 0.4][:M],
                   quad=[[0.2, 0.05, -0.03], [0.05, -0.1, 0.02], [-0.03, 0.02, 0.3]][:M])
    X["quad"] = [r[:M] for r in X["quad"]]
    return X


@pytest.mark.parametrize("name", list(SMALL))
def test_hermite_rhs_rk4_and_excitation_match_the_oracle(pk, name):
    w = SMALL[name]
    M = w["M"]
    say(f"[hermite] {name} shape={oh.shape(w)}")
    T = oh.tables(w)
    C = hstate(w, seed=5)
    X = optical(M)
    with pk.Solver(pk.params_from_workload(w)) as s:
        cfg = s.tile_config()
        assert cfg["pcube"] == 0
        s.set_state(C)
        s.rhs()
        e_rhs = rel_l2(s.get_state(), oh.rhs(w, C, T))
        s.set_state(C)
        s.propagate(3, 0.002)
        e_rk4 = rel_l2(s.get_state(), oh.rk4(w, C, 3, 0.002, T))
        s.set_state(C)
        v = s.observe(X)
        v_ref = oh.observe(w, X, C, T)
        s.perturb(X)
        e_x = rel_l2(s.get_state(), oh.perturb(w, X, C))
    say(f"    rhs {e_rhs:.2e} rk4 {e_rk4:.2e} perturb {e_x:.2e} observe {abs(v - v_ref) / abs(v_ref):.2e}")
    assert e_rhs < 1e-13 and e_rk4 < 1e-13 and e_x < 1e-13
    assert abs(v - v_ref) <= 1e-13 * abs(v_ref)


@pytest.mark.parametrize("name", ["h1_n12", "h2_n10", "h3_n8"])
def test_hermite_equilibration_matches_the_oracle(pk, name):
    w = SMALL[name]
    say(f"[hermite equilibrate] {name}")
    ref = oh.equilibrate(w, 30, 0.004)
    with pk.Solver(pk.params_from_workload(w)) as s:
        s.equilibrate(30, 0.004)
        got = s.get_state()
    assert rel_l2(got, ref) < 1e-12


def test_hermite_one_mode_linear_response_matches_the_oracle(pk):
    w = hw("one_mode_48", [24], [10], 3)
    A = wl.optical(1, lin=[1.0], quad=[[0.2]])
    say("[hermite response_1d] one mode 24 x 10, depth 3")
    T = oh.tables(w)
    Ceq = oh.equilibrate(w, 200, 0.005, T)
    ref = oh.response_1d(w, A, Ceq, 120, 2, 0.005, T)
    with pk.Solver(pk.params_from_workload(w)) as s:
        s.equilibrate(200, 0.005)
        assert rel_l2(s.get_state(), Ceq) < 1e-11
        got = s.response_1d(A, 120, 2, 0.005)
    assert rel_l2(got, ref) < FP64_TOL


@pytest.mark.parametrize("name,batch,prec", [("h2_n10", 0, "f64"), ("h3_n8", 0, "f64"),
                                             ("h2_n10", 3, "f64"), ("h3_c8", 4, "f64"),
                                             ("h2_n10", 3, "f32"), ("h3_c8", 4, "f32")])
def test_hermite_second_order_response_matches_the_oracle(pk, name, batch, prec):
    """R^(2) of Eq. (2Dresponse) (THz-Raman-THz operators) on the single-state
    path and in batched FP64 and FP32 branch waves."""
    w = SMALL[name]
    M = w["M"]
    base = wl.workload({2: "two_mode_32", 3: "three_mode_24"}[M])
    A, B = base["A"], base["B"]
    say(f"[hermite response_2d] {name} batch={batch} {prec}")
    T = oh.tables(w)
    Ceq = oh.equilibrate(w, 10, 0.004, T)
    ref = oh.response_2d(w, A, B, A, Ceq, 5, 6, 2, 3, 0.004, T)
    code = pk.CHFPE_FP32 if prec == "f32" else pk.CHFPE_FP64
    with pk.Solver(pk.params_from_workload(w, precision=code, batch=batch)) as s:
        s.equilibrate(10, 0.004)
        got = s.response_2d(A, B, A, 5, 6, 2, 3, 0.004)
    err = rel_l2(got, ref)
    say(f"    R2 rel L2 {err:.2e}")
    assert err < (1e-4 if prec == "f32" else FP64_TOL)


def test_hermite_workload_shape_is_accepted_and_planned(pk):
    """The three-mode 24^3 x 12^3 Hermite workload sets up (one k_hcube launch
    per stage; the lane-pair plane solves for its cubic q grid)."""
    w = wl.workload("three_mode_24_hermite")
    with pk.Solver(pk.params_from_workload(w)) as s:
        assert s.count == oh.shape(w)[0] * 12 ** 3 * 24 ** 3
        s.equilibrate(2, 0.005)
        v = s.observe(w["A"])
    assert np.isfinite(v)


@pytest.mark.parametrize("name", ["h1_n12", "h3_n8"])
def test_hermite_third_order_response_matches_the_oracle(pk, name):
    """R^(3) of Eq. (3Dresponse) at one waiting time in the Hermite basis."""
    w = SMALL[name]
    M = w["M"]
    A = optical(M)
    B = wl.optical(M, lin=[0.5, 0.8, -0.3][:M], quad=[[0.1, 0.0, 0.05], [0.0, 0.2, 0.0], [0.05, 0.0, -0.1]][:M])
    B["quad"] = [r[:M] for r in B["quad"]]
    say(f"[hermite response_3d] {name}")
    T = oh.tables(w)
    Ceq = oh.equilibrate(w, 10, 0.004, T)
    ref = oh.response_3d(w, A, B, B, A, Ceq, 4, 3, 5, 2, 2, 0.004, T)
    with pk.Solver(pk.params_from_workload(w)) as s:
        s.equilibrate(10, 0.004)
        got = s.response_3d(A, B, B, A, 4, 3, 5, 2, 2, 0.004)
    err = rel_l2(got, ref)
    say(f"    R3 rel L2 {err:.2e}")
    assert err < FP64_TOL


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_hermite_graph_and_eager_waves_agree(pk, monkeypatch, prec):
    """Hermite-basis waves captured as HIP graphs and issued directly give
    identical R, over three calls that replay the cached graph."""
    w = SMALL["h3_c8"]
    base = wl.workload("three_mode_24")
    A, B = base["A"], base["B"]
    code = pk.CHFPE_FP64 if prec == "f64" else pk.CHFPE_FP32
    say(f"[hermite graph vs eager] {prec}")
    monkeypatch.setenv("CHFPE_NO_GRAPH", "1")
    with pk.Solver(pk.params_from_workload(w, precision=code, batch=3)) as s:
        s.equilibrate(5, 0.004)
        eager = s.response_2d(A, B, A, 7, 5, 1, 2, 0.004)
    monkeypatch.setenv("CHFPE_NO_GRAPH", "0")
    with pk.Solver(pk.params_from_workload(w, precision=code, batch=3)) as s:
        s.equilibrate(5, 0.004)
        for rep in range(3):
            got = s.response_2d(A, B, A, 7, 5, 1, 2, 0.004)
            assert np.array_equal(got, eager), rep
            s.set_state(s.get_state())
            s.observe(A)


def test_hermite_context_has_no_tiles_to_tune_and_no_closure(pk):
    """chfpe_autotune returns at once on a Hermite context (one k_hcube shape)
    and leaves the results unchanged; the closure calls are refused (EINVAL),
    as the closure is defined for the p grid."""
    w = SMALL["h2_n10"]
    C = hstate(w, seed=9)
    with pk.Solver(pk.params_from_workload(w)) as s:
        s.set_state(C)
        s.rhs()
        before = s.get_state()
        cfg = s.autotune(2)
        assert cfg["pcube"] == 0
        s.set_state(C)
        s.rhs()
        assert np.array_equal(s.get_state(), before)
        for call in (lambda: s.set_closure(np.zeros(4)), lambda: s.closure_moments()):
            with pytest.raises(pk.ChfpeError):
                call()


@pytest.mark.parametrize("name", ["h3_n8", "h3_c12", "h2_n10"])
def test_hermite_task_order_does_not_change_results(pk, monkeypatch, name):
    """k_hcube's task order (XCD chunks, k_2 tiles) only schedules the tasks:
    RK4 steps and a batched 2D response are bitwise equal under the default
    order, one contiguous range per XCD, and chunks of 3 with k_2 tiles of 2
    (ragged last tiles)."""
    w = SMALL[name]
    M = w["M"]
    base = wl.workload({2: "two_mode_32", 3: "three_mode_24"}[M])
    A, B = base["A"], base["B"]
    C = hstate(w, seed=11)
    ne = oh.shape(w)[0]
    res = {}
    for chunk, ktile in ((None, None), ("0", "0"), ("3", "2")):
        for var, val in (("CHFPE_TUNE_HC_CHUNK", chunk), ("CHFPE_TUNE_HC_KTILE", ktile)):
            if val is None:
                monkeypatch.delenv(var, raising=False)
            else:
                monkeypatch.setenv(var, val)
        say(f"[hermite task order] {name} chunk={chunk} ktile={ktile}")
        with pk.Solver(pk.params_from_workload(w)) as s:
            cfg = s.tile_config()
            want_chunk = 4 * ne if chunk is None else int(chunk)
            want_tile = (min(3, w["Np"][1]) if ktile in (None, "0") else min(int(ktile), w["Np"][1])) if M == 3 else 1
            assert (cfg["hcube_chunk"], cfg["hcube_ktile"]) == (want_chunk, want_tile), cfg
            s.set_state(C)
            s.propagate(2, 0.003)
            st = s.get_state()
        with pk.Solver(pk.params_from_workload(w, batch=3)) as s:
            s.equilibrate(4, 0.004)
            r2 = s.response_2d(A, B, A, 4, 3, 1, 2, 0.004)
        res[(chunk, ktile)] = (st, r2)
    ref = res[(None, None)]
    for key, (st, r2) in res.items():
        assert np.array_equal(st, ref[0]) and np.array_equal(r2, ref[1]), key
