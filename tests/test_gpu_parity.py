"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Bar (FP64 path): relative L2 error <= 1e-10 on states, responses and
observables; one right-hand side and a few RK4 steps agree to ~1e-14.
Sizes: small grids that span several tiles with ragged tails, the one-mode
workload at full size, the two-mode 32^4 workload at full size in the
launch configuration its benchmark times (one 64-branch FP64 wave, sampled
t1 columns), and the three-mode workloads at full size (12^6 and 16^6
whole states, 16^6 responses in batched FP64 and FP32 waves on a t1 subset,
24^6 at sampled points of one right-hand side and one whole RK4 step).
"""
import sys

import numpy as np
import pytest

import oracle as orc
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


def solver(pk, w):
    return pk.Solver(pk.params_from_workload(w))


def phys_state(w, seed, noise=0.05):
    """A seeded state with the physical shape: the Boltzmann envelope of the
    model (from the oracle) on every element, times 1 + smooth + noise."""
    env = orc.boltzmann(w)[0]
    sm = wl.smooth_state(w, seed=seed)
    sm = sm / np.abs(sm).max()
    nz = wl.noise_state(w, seed=seed + 1000)
    return env[None] * (1.0 + 0.3 * sm + noise * nz)


SMALL = {
    "m1_n12_k3": wl.workload("one_mode_48", Nq=[12], Np=[13], K=3),
    "m2_n10_k2": wl.workload("two_mode_32", Nq=[10, 9], Np=[11, 10], K=2),
    "m2_n12_k3": wl.workload("two_mode_32", Nq=[12, 12], Np=[12, 12], K=3),
    # p blocks beyond the two-axis LDS tile: k_pcube with a unit third axis
    "m2_p40_k2": wl.workload("two_mode_32", Nq=[6, 7], Np=[40, 36], K=2),
    "m2_p48_k2": wl.workload("two_mode_32", Nq=[5, 6], Np=[48, 48], K=2),
    "m2_p25_k2": wl.workload("two_mode_32", Nq=[6, 5], Np=[25, 25], K=2),
    "m3_n8_k2": wl.workload("three_mode_24", Nq=[8, 7, 8], Np=[8, 9, 7], K=2),
    "m3_n6_k3": wl.workload("three_mode_24", Nq=[6, 6, 6], Np=[6, 6, 6], K=3),
    # square 8 x 8 (p_2, p_3) blocks: lane-pair line solves, ragged q and p_1
    "m3_p8_k2": wl.workload("three_mode_24", Nq=[7, 6, 8], Np=[9, 8, 8], K=2),
    # 24 x 24 (p_2, p_3) blocks as in the 24^6 workload: three rows per thread
    # (a 576-thread plane with 5-point p_1 lines exceeds k_pcube's FP64
    # workgroup: the p-block + (q_1, p_1) path)
    "m3_p24_k2": wl.workload("three_mode_24", Nq=[5, 6, 5], Np=[5, 24, 24], K=2),
    # cubic p blocks: k_pcube with lane-pair plane solves (8^3, 12^3, 24^3)
    "m3_c8_k2": wl.workload("three_mode_24", Nq=[5, 6, 7], Np=[8, 8, 8], K=2),
    "m3_c12_k2": wl.workload("three_mode_24", Nq=[5, 5, 6], Np=[12, 12, 12], K=2),
    "m3_c24_k2": wl.workload("three_mode_24", Nq=[5, 5, 5], Np=[24, 24, 24], K=2),
}

THREE = [n for n in SMALL if n.startswith("m3")]


def test_the_planner_takes_k_pcube_where_it_should(pk):
    """Three modes take k_pcube wherever its block fits; two modes only for
    p blocks the two-axis tile cannot cover; one mode never."""
    want = {"m1_n12_k3": 0, "m2_n10_k2": 0, "m2_n12_k3": 0, "m2_p40_k2": 1, "m2_p48_k2": 1,
            "m2_p25_k2": 1, "m3_n8_k2": 1, "m3_p24_k2": 0, "m3_c24_k2": 1}
    for name, flag in want.items():
        with solver(pk, SMALL[name]) as s:
            assert s.tile_config()["pcube"] == flag, name


@pytest.mark.parametrize("name", THREE)
def test_three_mode_p_block_path_matches_the_oracle(pk, monkeypatch, name):
    """Three modes with k_pcube switched off (CHFPE_PCUBE=0): the p-block,
    (q_2, q_3) and (q_1, p_1) passes, and the two-launch excitation, still
    give the oracle's right-hand side, RK4 steps and X^x."""
    monkeypatch.setenv("CHFPE_PCUBE", "0")
    w = SMALL[name]
    say(f"[p-block path] {name}")
    W = phys_state(w, seed=11)
    X = wl.optical(3, lin=[1.0, -0.7, 0.4], quad=[[0.2, 0.05, -0.03], [0.05, -0.1, 0.02], [-0.03, 0.02, 0.3]])
    with solver(pk, w) as s:
        s.set_state(W)
        s.rhs()
        e_rhs = rel_l2(s.get_state(), orc.rhs(w, W))
        s.set_state(W)
        s.propagate(2, 0.002)
        e_rk4 = rel_l2(s.get_state(), orc.rk4(w, W, 2, 0.002))
        s.set_state(W)
        s.perturb(X)
        e_x = rel_l2(s.get_state(), orc.perturb(w, X, W))
    say(f"    rhs {e_rhs:.2e} rk4 {e_rk4:.2e} perturb {e_x:.2e}")
    assert e_rhs < 1e-13 and e_rk4 < 1e-13 and e_x < 1e-13


PCUBE = ["m3_n8_k2", "m3_p8_k2", "m3_n6_k3", "m3_c8_k2", "m3_c12_k2", "m3_c24_k2", "m2_p25_k2"]


@pytest.mark.parametrize("stream", [0, 1])
@pytest.mark.parametrize("name", PCUBE)
def test_both_k_pcube_forms_match_the_oracle(pk, monkeypatch, name, stream):
    """k_pcube (a copy of the p block in LDS) and k_pcube_s (one streamed
    sweep over the planes), each forced with CHFPE_TUNE_PC_STREAM, give the
    oracle's right-hand side, RK4 steps and X^x (cubic blocks with lane-pair
    plane solves, ragged blocks, and a two-mode block with a unit third axis)."""
    monkeypatch.setenv("CHFPE_TUNE_PC_STREAM", str(stream))
    w = SMALL[name]
    M = w["M"]
    say(f"[k_pcube stream={stream}] {name}")
    W = phys_state(w, seed=12)
    X = wl.optical(M, lin=[1.0, -0.7, 0.4][:M],
                   quad=[r[:M] for r in [[0.2, 0.05, -0.03], [0.05, -0.1, 0.02], [-0.03, 0.02, 0.3]][:M]])
    with solver(pk, w) as s:
        cfg = s.tile_config()
        assert cfg["pcube"] == 1 and cfg["pcube_stream"] == stream, cfg
        s.set_state(W)
        s.rhs()
        e_rhs = rel_l2(s.get_state(), orc.rhs(w, W))
        s.set_state(W)
        s.propagate(2, 0.002)
        e_rk4 = rel_l2(s.get_state(), orc.rk4(w, W, 2, 0.002))
        s.set_state(W)
        s.perturb(X)
        e_x = rel_l2(s.get_state(), orc.perturb(w, X, W))
    say(f"    rhs {e_rhs:.2e} rk4 {e_rk4:.2e} perturb {e_x:.2e}")
    assert e_rhs < 1e-13 and e_rk4 < 1e-13 and e_x < 1e-13


@pytest.mark.parametrize("name", list(SMALL))
def test_rhs_parity_small(pk, name):
    w = SMALL[name]
    say(f"[rhs] {name} shape={orc.state_shape(w)}")
    W = phys_state(w, seed=1)
    ref = orc.rhs(w, W)
    with solver(pk, w) as s:
        s.set_state(W)
        s.rhs()
        got = s.get_state().reshape(W.shape)
    assert rel_l2(got, ref) < 1e-13


@pytest.mark.parametrize("name", list(SMALL))
def test_rk4_parity_small(pk, name):
    w = SMALL[name]
    say(f"[rk4] {name}")
    W = phys_state(w, seed=3)
    ref = orc.rk4(w, W, 3, 0.002)
    with solver(pk, w) as s:
        s.set_state(W)
        s.propagate(3, 0.002)
        got = s.get_state().reshape(W.shape)
    assert rel_l2(got, ref) < 1e-13


@pytest.mark.parametrize("name", list(SMALL))
def test_perturb_and_observe_parity_small(pk, name):
    w = SMALL[name]
    M = w["M"]
    say(f"[perturb] {name}")
    X = wl.optical(M, lin=[1.0, -0.7, 0.4][:M],
                   quad=[[0.2, 0.05, -0.03], [0.05, -0.1, 0.02], [-0.03, 0.02, 0.3]][:M])
    X["quad"] = [row[:M] for row in X["quad"]]
    W = phys_state(w, seed=4)
    ref = orc.perturb(w, X, W)
    with solver(pk, w) as s:
        s.set_state(W)
        v_gpu = s.observe(X)
        s.perturb(X)
        got = s.get_state().reshape(W.shape)
    assert rel_l2(got, ref) < 1e-13
    v_ref = orc.observe(w, X, W)
    assert abs(v_gpu - v_ref) <= 1e-13 * max(abs(v_ref), 1e-300)


@pytest.mark.parametrize("name", ["m1_n12_k3", "m2_n10_k2", "m3_n8_k2"])
def test_equilibrate_parity_small(pk, name):
    w = SMALL[name]
    say(f"[equilibrate] {name}")
    ref = orc.equilibrate(w, 40, 0.004)
    with solver(pk, w) as s:
        s.equilibrate(40, 0.004)
        got = s.get_state().reshape(ref.shape)
    assert rel_l2(got, ref) < 1e-12


def test_response_1d_parity_one_mode_full(pk):
    """The one-mode 48 x 48, depth-3 workload: equilibration and 1D response
    (shortened to 600 + 800 steps so that the oracle stays fast)."""
    w = wl.workload("one_mode_48")
    say("[response_1d] one_mode_48")
    Weq = orc.equilibrate(w, 600, w["dt"])
    ref = orc.response_1d(w, w["A"], Weq, 800, 1, w["dt"])
    with solver(pk, w) as s:
        s.equilibrate(600, w["dt"])
        assert rel_l2(s.get_state(), Weq) < 1e-11
        got = s.response_1d(w["A"], 800, 1, w["dt"])
    assert rel_l2(got, ref) < FP64_TOL


@pytest.mark.parametrize("name", ["m2_n10_k2", "m3_n8_k2", "m3_n6_k3"])
def test_response_2d_parity_small(pk, name):
    w = SMALL[name]
    M = w["M"]
    A = wl.workload("three_mode_24")["A"]
    B = wl.workload("three_mode_24")["B"]
    A = {"lin": A["lin"][:M], "quad": [r[:M] for r in A["quad"][:M]]}
    B = {"lin": B["lin"][:M], "quad": [r[:M] for r in B["quad"][:M]]}
    say(f"[response_2d] {name}")
    Weq = orc.equilibrate(w, 10, 0.004)
    ref = orc.response_2d(w, A, B, A, Weq, 5, 6, 2, 3, 0.004)
    with solver(pk, w) as s:
        s.equilibrate(10, 0.004)
        got = s.response_2d(A, B, A, 5, 6, 2, 3, 0.004)
    assert rel_l2(got, ref) < FP64_TOL


def test_two_mode_full_size_rhs_and_steps(pk):
    """Two modes, 32^4, depth 3 (10 elements): one right-hand side and two RK4
    steps on a seeded smooth state."""
    w = wl.workload("two_mode_32")
    say("[full] two_mode_32 rhs + 2 steps")
    W = phys_state(w, seed=5, noise=0.0)
    ref_rhs = orc.rhs(w, W)
    ref_2 = orc.rk4(w, W, 2, w["dt"])
    with solver(pk, w) as s:
        s.set_state(W)
        s.rhs()
        assert rel_l2(s.get_state(), ref_rhs) < 1e-13
        s.set_state(W)
        s.propagate(2, w["dt"])
        assert rel_l2(s.get_state(), ref_2) < 1e-13


@pytest.mark.timeout(900)
def test_two_mode_full_size_response_2d_sampled(pk):
    """The two-mode 2D THz-Raman run (64 t1 x 256 t2, stride 1) in the launch
    configuration its benchmark times: all 64 t1 branches in one batched
    FP64 wave (a captured HIP graph).  Columns spread across the wave
    (j1 = 0, 21, 42, 63) over the first 16 t2 rows against the oracle, both
    starting from the same equilibrium (the discrete Boltzmann state); the
    rest of R must be finite."""
    w = wl.workload("two_mode_32")
    say("[full] two_mode_32 response_2d 64x256, one 64-branch wave, sampled")
    Wb = orc.boltzmann(w)
    cols = [0, 21, 42, 63]
    ref = orc.response_2d(w, w["A"], w["B"], w["C"], Wb, 64, 16, 1, 1, w["dt"], j1_list=cols)
    say("    oracle done")
    with pk.Solver(pk.params_from_workload(w, precision=pk.CHFPE_FP64, batch=64)) as s:
        s.set_state(Wb)
        s.use_state_as_equilibrium()
        got = s.response_2d(w["A"], w["B"], w["C"], 64, 256, 1, 1, w["dt"])
    assert np.all(np.isfinite(got))
    err = rel_l2(got[:16, cols], ref[:16, cols])
    say(f"    sampled columns rel L2 {err:.2e}")
    assert err < FP64_TOL


def test_spectra_parity(pk):
    """Device Fourier sums of Eqs. (1DIR_Raman), (2DThz_Raman) against the
    oracle's plain sums, on seeded signals of the response shapes."""
    say("[spectra]")
    rng = np.random.default_rng(9)
    R1 = rng.standard_normal(500)
    om_ref, I_ref = orc.spectrum_1d(R1, 0.005)
    om, I = pk.spectrum_1d(R1, 0.005)
    assert rel_l2(om, om_ref) < 1e-14
    assert rel_l2(I, I_ref) < 1e-12
    R2 = rng.standard_normal((256, 64))
    _, _, I2_ref = orc.spectrum_2d(R2, 0.005, 0.005)
    I2 = pk.spectrum_2d(R2, 0.005, 0.005)
    assert rel_l2(I2, I2_ref) < 1e-12
    R3 = rng.standard_normal((7, 5))  # ragged, odd sizes
    _, _, I3_ref = orc.spectrum_2d(R3, 0.3, 0.1)
    assert rel_l2(pk.spectrum_2d(R3, 0.3, 0.1), I3_ref) < 1e-12


# ---------------------------------------------------------------------------
# batched t1 branches (waves of B states), HIP graphs, FP32 branch states
# ---------------------------------------------------------------------------

def _ops(M):
    A = wl.workload("three_mode_24")["A"]
    B = wl.workload("three_mode_24")["B"]
    A = {"lin": A["lin"][:M], "quad": [r[:M] for r in A["quad"][:M]]}
    B = {"lin": B["lin"][:M], "quad": [r[:M] for r in B["quad"][:M]]}
    return A, B


@pytest.mark.parametrize("name", ["m2_n10_k2", "m3_n8_k2"])
def test_response_2d_batched_fp64_parity(pk, name):
    """Seven t1 branches in waves of 3, 3 and 1 (graph replays with eager
    work in between, a smaller last wave), FP64, against the oracle."""
    w = SMALL[name]
    A, B = _ops(w["M"])
    say(f"[batched fp64] {name}")
    Weq = orc.equilibrate(w, 10, 0.004)
    ref = orc.response_2d(w, A, B, A, Weq, 7, 5, 2, 3, 0.004)
    with pk.Solver(pk.params_from_workload(w, precision=pk.CHFPE_FP64, batch=3)) as s:
        s.equilibrate(10, 0.004)
        got = s.response_2d(A, B, A, 7, 5, 2, 3, 0.004)
        again = s.response_2d(A, B, A, 7, 5, 2, 3, 0.004)  # cached graph, second use
    assert rel_l2(got, ref) < FP64_TOL
    assert np.array_equal(got, again)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_graph_and_eager_waves_agree(pk, monkeypatch, prec):
    """Waves captured as HIP graphs (the solver's own stream) and the same
    launches issued directly give identical R (deterministic kernels,
    fixed-order reductions).  The graph context replays its cached graphs in
    three calls with eager work and synchronizations in between (a state
    round trip, an observable); every replay must equal the eager result."""
    w = SMALL["m2_n12_k3"]
    A, B = _ops(2)
    code = pk.CHFPE_FP64 if prec == "f64" else pk.CHFPE_FP32
    say(f"[graph vs eager] {prec}")
    monkeypatch.setenv("CHFPE_NO_GRAPH", "1")
    with pk.Solver(pk.params_from_workload(w, precision=code, batch=4)) as s:
        assert s.stream.cuda_stream != 0
        s.equilibrate(5, 0.004)
        eager = s.response_2d(A, B, A, 9, 6, 1, 2, 0.004)
    monkeypatch.setenv("CHFPE_NO_GRAPH", "0")
    with pk.Solver(pk.params_from_workload(w, precision=code, batch=4)) as s:
        s.equilibrate(5, 0.004)
        for rep in range(3):
            got = s.response_2d(A, B, A, 9, 6, 1, 2, 0.004)
            assert np.array_equal(got, eager), rep
            s.set_state(s.get_state())
            s.observe(A)


@pytest.mark.parametrize("name", ["m2_n12_k3", "m3_n8_k2"])
def test_response_2d_fp32_branches(pk, name):
    """FP32 branch states (FP64 equilibrium, t1 trajectory, excitations and
    reductions) against the FP64 oracle: relative L2 <= 1e-4."""
    w = SMALL[name]
    A, B = _ops(w["M"])
    say(f"[fp32 branches] {name}")
    Weq = orc.equilibrate(w, 10, 0.004)
    ref = orc.response_2d(w, A, B, A, Weq, 6, 8, 2, 2, 0.004)
    with pk.Solver(pk.params_from_workload(w, precision=pk.CHFPE_FP32, batch=4)) as s:
        s.equilibrate(10, 0.004)
        got = s.response_2d(A, B, A, 6, 8, 2, 2, 0.004)
    err = rel_l2(got, ref)
    say(f"    fp32 rel L2 = {err:.2e}")
    assert err < 1e-4


@pytest.mark.parametrize("kind", ["RTT", "TRT", "TTR", "TTT"])
def test_response_2d_orderings_and_resolved_stride(pk, kind):
    """The three THz-Raman orderings (operator swaps through the same entry
    point) with a physically resolved stride of 8 RK4 steps per sample."""
    w = SMALL["m2_n12_k3"]
    A, B, C = wl.response_types(w)[kind]
    say(f"[ordering] {kind}")
    Weq = orc.equilibrate(w, 10, 0.004)
    ref = orc.response_2d(w, A, B, C, Weq, 4, 5, 8, 8, 0.004)
    with solver(pk, w) as s:
        s.equilibrate(10, 0.004)
        got = s.response_2d(A, B, C, 4, 5, 8, 8, 0.004)
    assert rel_l2(got, ref) < FP64_TOL


@pytest.mark.parametrize("split", ["0", "1"])
def test_pblock_line_solvers_agree(pk, monkeypatch, split):
    """Lane-pair and single-lane line solves of k_pblock both match the oracle
    (two-mode 12^4 and one-mode 48-point lines)."""
    monkeypatch.setenv("CHFPE_TUNE_PB_SPLIT", split)
    for name, w in (("m2_n12_k3", SMALL["m2_n12_k3"]), ("m1_n48", wl.workload("one_mode_48"))):
        say(f"[pblock split={split}] {name}")
        W = phys_state(w, seed=6)
        ref = orc.rk4(w, W, 2, 0.002)
        with solver(pk, w) as s:
            s.set_state(W)
            s.propagate(2, 0.002)
            got = s.get_state().reshape(W.shape)
        assert rel_l2(got, ref) < 1e-13


def test_autotune_keeps_state_and_results(pk):
    """chfpe_autotune times tile shapes on scratch buffers: the state is
    unchanged, the chosen shapes are reported, later steps and batched
    responses still match the oracle, and a new context of the same shape
    starts from the tuned shapes."""
    w = SMALL["m2_n12_k3"]
    A, B = _ops(2)
    say("[autotune]")
    Weq = orc.equilibrate(w, 10, 0.004)
    ref = orc.response_2d(w, A, B, A, Weq, 5, 4, 1, 2, 0.004)
    W = phys_state(w, seed=7)
    ref_steps = orc.rk4(w, W, 2, 0.002)
    p = pk.params_from_workload(w, precision=pk.CHFPE_FP64, batch=5)
    with pk.Solver(p) as s:
        s.equilibrate(10, 0.004)
        s.set_state(W)
        before = s.get_state()
        cfg = s.autotune(1)
        say(f"    tuned {cfg}")
        assert cfg["pblock_blocks_per_task"] >= 1 and cfg["qpass_positions"] >= 1
        assert cfg["pblock_split_lines"] in (0, 1)
        assert np.array_equal(s.get_state(), before)
        s.propagate(2, 0.002)
        assert rel_l2(s.get_state().reshape(W.shape), ref_steps) < 1e-13
        got = s.response_2d(A, B, A, 5, 4, 1, 2, 0.004)
    assert rel_l2(got, ref) < FP64_TOL
    with pk.Solver(p) as s2:
        assert s2.tile_config() == cfg


@pytest.mark.parametrize("batch", [1, 3])
def test_response_2d_range_equals_the_full_columns(pk, batch):
    """Column ranges of R (chfpe_response_2d_range) reproduce the columns of
    one full call bitwise, single-state and in batched waves."""
    w = SMALL["m2_n12_k3"]
    A, B = _ops(2)
    say(f"[range] batch {batch}")
    with pk.Solver(pk.params_from_workload(w, precision=pk.CHFPE_FP64, batch=batch)) as s:
        s.equilibrate(5, 0.004)
        full = s.response_2d(A, B, A, 7, 4, 2, 2, 0.004)
        parts = [s.response_2d_range(A, B, A, j0, j1, 4, 2, 2, 0.004) for j0, j1 in ((0, 3), (3, 4), (4, 7))]
    assert np.array_equal(full, np.concatenate(parts, axis=1))


TILE_CANDIDATES = [
    {"CHFPE_TUNE_PB_NB": "1"}, {"CHFPE_TUNE_PB_NB": "2"}, {"CHFPE_TUNE_PB_NB": "8"},
    {"CHFPE_TUNE_PB_SPLIT": "0"},
    {"CHFPE_TUNE_Q_PC": "4"}, {"CHFPE_TUNE_Q_PC": "8"}, {"CHFPE_TUNE_Q_PC": "32"},
    {"CHFPE_TUNE_PB_RUN": "4"}, {"CHFPE_TUNE_PB_RUN": "32"},
]


@pytest.mark.parametrize("name", ["m2_n12_k3", "m3_p8_k2", "m3_n8_k2", "m3_n16_k2"])
def test_every_autotuner_tile_shape_matches_the_oracle(pk, monkeypatch, name):
    """Each tile shape chfpe_autotune may pick gives the oracle's RK4 steps."""
    w = SMALL[name] if name in SMALL else wl.workload("three_mode_24", Nq=[5, 6, 16], Np=[6, 16, 16], K=2)
    W = phys_state(w, seed=21)
    ref = orc.rk4(w, W, 2, 0.002)
    bad = []
    for env in TILE_CANDIDATES:
        for k in ("CHFPE_TUNE_PB_NB", "CHFPE_TUNE_PB_SPLIT", "CHFPE_TUNE_Q_PC", "CHFPE_TUNE_PB_RUN"):
            monkeypatch.delenv(k, raising=False)
        for k, v in env.items():
            monkeypatch.setenv(k, v)
        with solver(pk, w) as s:
            s.set_state(W)
            s.propagate(2, 0.002)
            err = rel_l2(s.get_state().reshape(W.shape), ref)
            cfg = s.tile_config()
        say(f"[tiles] {name} {env} -> {cfg} err {err:.2e}")
        if not err < 1e-13:
            bad.append((env, cfg, err))
    assert not bad, bad


def test_batched_launch_stays_within_one_dispatch(pk, monkeypatch):
    """Ten elements of 16^6 points in a wave of 32 FP32 branch states on the
    p-block path: at one p-block per task that launch would pass 2^32
    work-items (a dispatch's limit), so the planner raises the request to two
    blocks per task.  The 32 columns then match the single-state FP64 solver
    (which keeps one)."""
    import torch
    monkeypatch.setenv("CHFPE_TUNE_PB_NB", "1")
    monkeypatch.setenv("CHFPE_PCUBE", "0")  # the p-block launch is the one at the limit
    w = wl.workload("three_mode_16")
    dt = w["dt"]
    A, B, C = w["A"], w["B"], w["C"]
    n_eq, nc, n2 = 50, 32, 3
    say("[dispatch] three_mode_16 single FP64")
    with pk.Solver(pk.params_from_workload(w, precision=pk.CHFPE_FP64, batch=1)) as s:
        assert s.tile_config()["pblock_blocks_per_task"] == 1
        s.equilibrate(n_eq, dt)
        R1 = s.response_2d_range(A, B, C, 0, nc, n2, 1, 1, dt)
    torch.cuda.empty_cache()
    say("[dispatch] three_mode_16 batch 32 FP32")
    with pk.Solver(pk.params_from_workload(w, precision=pk.CHFPE_FP32, batch=32)) as sb:
        cfg = sb.tile_config()
        assert cfg["pblock_blocks_per_task"] == 2, cfg
        sb.equilibrate(n_eq, dt)
        RB = sb.response_2d_range(A, B, C, 0, nc, n2, 1, 1, dt)
    torch.cuda.empty_cache()
    err = float(np.abs(RB - R1).max() / np.abs(R1).max())
    say(f"[dispatch] max rel diff {err:.3e}")
    assert err < 1e-4


@pytest.mark.parametrize("name,steps", [("three_mode_12", 2), ("three_mode_16", 1)])
def test_three_mode_full_size_rhs_and_steps(pk, name, steps):
    """Three modes at full size (12^6 and 16^6 grids, depth 2, 10 elements):
    one right-hand side and RK4 steps on a seeded state, every value against
    the oracle."""
    import torch
    w = wl.workload(name)
    say(f"[full] {name}: rhs + {steps} RK4 steps")
    W = phys_state(w, seed=7, noise=0.0)
    ref_rhs = orc.rhs(w, W)
    say(f"    oracle rhs done; {steps} oracle RK4 steps")
    ref = orc.rk4(w, W, steps, w["dt"])
    say("    oracle done; GPU")
    with solver(pk, w) as s:
        s.set_state(W)
        s.rhs()
        e_rhs = rel_l2(s.get_state(), ref_rhs)
        s.set_state(W)
        s.propagate(steps, w["dt"])
        e_rk4 = rel_l2(s.get_state(), ref)
    torch.cuda.empty_cache()
    say(f"    rhs {e_rhs:.2e}  rk4 {e_rk4:.2e}")
    assert e_rhs < 1e-13 and e_rk4 < 1e-13


@pytest.mark.timeout(900)
def test_three_mode_24_full_size_rhs_sampled(pk):
    """Three modes on the full 24^6 grid (10 elements, 1.9e9 values): one
    right-hand side on the GPU, checked at 96 seeded points and at the first
    and last point of every element against the oracle's evaluation of the
    same point (which reads only the lines through it)."""
    import torch
    w = wl.workload("three_mode_24")
    say("[full] three_mode_24: building the state")
    # element e: Boltzmann envelope of element 0 (a depth-0 call gives one
    # element) times 1 + 0.3 x a seeded smooth field, built one element at a
    # time to keep host memory near one state
    w0 = {**w, "K": 0}
    env = orc.boltzmann(w0)[0]
    ne = orc.state_shape(w)[0]
    W = np.empty(orc.state_shape(w))
    for e in range(ne):
        sm = wl.smooth_state(w0, seed=9 + e)[0]
        sm *= 0.3 / np.abs(sm).max()
        sm += 1.0
        np.multiply(env, sm, out=W[e])
        say(f"    element {e} built")
    del env, sm
    E = W[0].size
    rng = np.random.default_rng(10)
    pts = [(int(rng.integers(ne)), int(rng.integers(E))) for _ in range(96)]
    pts += [(e, 0) for e in range(ne)] + [(e, E - 1) for e in range(ne)]
    say("[full] three_mode_24: oracle points")
    ref = np.array([orc.rhs_point(w, W, e, i) for e, i in pts])
    with solver(pk, w) as s:
        s.set_state(W)
        say("[full] three_mode_24: rhs on the GPU")
        s.rhs()
        del W
        got = s.get_state().reshape(ne, E)
    torch.cuda.empty_cache()
    g = np.array([got[e, i] for e, i in pts])
    del got
    err = float(np.abs(g - ref).max() / np.abs(ref).max())
    say(f"    max error / max |rhs| over {len(pts)} points: {err:.2e}")
    assert err < 1e-13


@pytest.mark.timeout(900)
def test_three_mode_16_response_2d_waves_against_the_oracle(pk):
    """The three-mode 16^6 workload's 2D response on a t1 subset, in batched
    waves as its benchmark runs them: FP64 waves against the oracle at the
    FP64 bar and FP32 waves at the FP32 bar.  Columns j1 = 0..2 (waves of 3)
    over 4 t2 rows, from the discrete Boltzmann state as W_eq; columns 0
    and 2 are compared (the oracle skips column 1)."""
    import torch
    w = wl.workload("three_mode_16")
    dt = w["dt"]
    say("[full] three_mode_16 response: oracle columns 0, 2 x 4 rows")
    Wb = orc.boltzmann(w)
    cols = [0, 2]
    ref = orc.response_2d(w, w["A"], w["B"], w["C"], Wb, 3, 4, 1, 1, dt, j1_list=cols)
    say("    oracle done")
    for prec, tol in ((pk.CHFPE_FP64, FP64_TOL), (pk.CHFPE_FP32, 1e-4)):
        with pk.Solver(pk.params_from_workload(w, precision=prec, batch=3)) as s:
            s.set_state(Wb)
            s.use_state_as_equilibrium()
            got = s.response_2d(w["A"], w["B"], w["C"], 3, 4, 1, 1, dt)
        torch.cuda.empty_cache()
        err = rel_l2(got[:, cols], ref[:, cols])
        say(f"    precision {prec}: rel L2 {err:.2e}")
        assert err < tol


@pytest.mark.timeout(900)
def test_three_mode_24_full_size_rk4_step(pk):
    """One whole RK4 step of the full 24^6 three-mode state (1.9e9 values)
    against the oracle, every value.  The oracle's step is taken as its four
    right-hand sides with the classical RK4 combination (one call each, so
    that progress shows between them); about 95 GB of host memory (six
    states: input, GPU result, sum, stage input, slope, and the oracle's
    own copy in h-form)."""
    import psutil
    import torch
    need = 110e9
    if psutil.virtual_memory().available < need:
        pytest.skip(f"needs {need / 1e9:.0f} GB of free host memory for the oracle at 24^6")
    w = wl.workload("three_mode_24")
    dt = w["dt"]
    say("[full] three_mode_24 rk4 step: building the state")
    w0 = {**w, "K": 0}
    env = orc.boltzmann(w0)[0]
    ne = orc.state_shape(w)[0]
    y = np.empty(orc.state_shape(w))
    for e in range(ne):
        sm = wl.smooth_state(w0, seed=30 + e)[0]
        sm *= 0.3 / np.abs(sm).max()
        sm += 1.0
        np.multiply(env, sm, out=y[e])
    del env, sm
    say("    GPU step")
    with solver(pk, w) as s:
        s.set_state(y)
        s.propagate(1, dt)
        got = s.get_state()
    torch.cuda.empty_cache()
    acc = y.copy()
    x = None
    for st, (cx, cw) in enumerate(((0.5, 1.0), (0.5, 2.0), (1.0, 2.0), (None, 1.0))):
        k = orc.rhs(w, y if x is None else x)
        say(f"    oracle stage {st + 1}/4 done")
        if cx is not None:  # next stage input y + cx dt k, in place
            if x is None:
                x = np.empty_like(y)
            np.multiply(k, cx * dt, out=x)
            x += y
        np.multiply(k, dt / 6.0 * cw, out=k)
        acc += k
        del k
    del x
    err = rel_l2(got, acc)
    say(f"    rel L2 {err:.2e}")
    assert err < 1e-13


# ---------------------------------------------------------------------------
# third-order response, Eq. (3Dresponse), and the 2D IR spectrum
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("name", ["m1_n12_k3", "m2_n10_k2", "m3_n8_k2", "m3_c8_k2"])
def test_response_3d_parity_small(pk, name):
    """R^(3)(t3, t2, t1) at one waiting time against the oracle (FP64 bar),
    with quadratic operators (dipole, polarizability) in the TRRT-like order
    A = mu, B = Pi, C = Pi, D = mu; also from a batched FP32 context, whose
    third-order branches run on the FP64 single-state buffers."""
    w = SMALL[name]
    A, B = _ops(w["M"])
    say(f"[response_3d] {name}")
    Weq = orc.equilibrate(w, 10, 0.004)
    ref = orc.response_3d(w, A, B, B, A, Weq, 4, 6, 5, 2, 3, 0.004)
    for prec, batch in ((pk.CHFPE_FP64, 1), (pk.CHFPE_FP32, 3)):
        with pk.Solver(pk.params_from_workload(w, precision=prec, batch=batch)) as s:
            s.equilibrate(10, 0.004)
            got = s.response_3d(A, B, B, A, 4, 6, 5, 2, 3, 0.004)
        assert rel_l2(got, ref) < FP64_TOL, prec


def test_spectrum_2dir_parity(pk):
    """Device Fourier sums of Eq. (noncorrelation) against the oracle's."""
    rng = np.random.default_rng(11)
    for shape in ((256, 64), (7, 5)):
        R = rng.standard_normal(shape)
        _, _, ref = orc.spectrum_2dir(R, 0.005, 0.01)
        assert rel_l2(pk.spectrum_2dir(R, 0.005, 0.01), ref) < 1e-12
