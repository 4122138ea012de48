"""Benchmark of the CHFPE hot path on one MI355X.

One step = the whole hot path once on the two-mode 32^4 depth-3 workload
(10 hierarchy elements, 10,485,760 values per state, FP64):
  coefficient tables and upload (chfpe_setup into a resident workspace),
  equilibration (Boltzmann start + 4000 RK4 steps),
  2D THz-Raman response R(t2, t1) over 64 t1 x 256 t2 samples (stride 1,
  dt = 0.005), and the 2D spectrum of R.
That is 4000 + 63 + 64 * 255 = 20383 RK4 steps per bench step.

Prints one JSON line: hierarchy-gridpoint RK4 updates/s over the timed
steps, the roofline of the dominant kernel (HIP-event timing of sampled RK4
steps inside the timed region; algorithmic bytes per launch from the
library), and the FP64 CPU oracle timed on a bounded sample of the same
workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "hierarchy-gridpoint RK4 updates/s + % HBM peak; 2D spectrum time at ≤1e-3 error"
HBM_PEAK_GBPS = 8000.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def source_hash() -> str:
    h = hashlib.sha256()
    for rel in ("paper_2509_25840_amd/csrc/kernels.h", "paper_2509_25840_amd/csrc/chfpe.hip"):
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def rk4_steps(w) -> int:
    return (int(w["eq_steps"]) + (int(w["n_t1"]) - 1) * int(w["stride1"])
            + int(w["n_t1"]) * (int(w["n_t2"]) - 1) * int(w["stride2"]))


def launches_per_rk4_step(M: int) -> dict:
    d = {"pblock_rhs": 4, "qpass_rk4_s1": 1, "qpass_rk4_s2": 1, "qpass_rk4_s3": 1, "qpass_rk4_s4": 1}
    if M == 3:
        d["qpass_acc"] = 4
    return d


def cpu_baseline(w, pk, target_s: float, sample_note: str):
    """Time the oracle's RK4 on this workload's state for ~target_s seconds
    and compare the GPU's result for the same steps."""
    import numpy as np
    import oracle as orc
    W0 = orc.boltzmann(w)
    W0[1] = 0.2 * W0[0]  # a non-stationary start so the steps do real work
    t0 = time.perf_counter()
    W1 = orc.rk4(w, W0, 1, w["dt"])
    t1 = time.perf_counter() - t0
    n = max(1, min(64, int(target_s / max(t1, 1e-3)) - 1))
    t0 = time.perf_counter()
    Wn = orc.rk4(w, W1, n, w["dt"])
    tn = time.perf_counter() - t0
    S = W0.size
    with pk.Solver(pk.params_from_workload(w)) as s:
        s.set_state(W0)
        s.propagate(n + 1, w["dt"])
        got = s.get_state()
    err = float(np.linalg.norm(got - Wn.ravel()) / np.linalg.norm(Wn.ravel()))
    return {
        "value": S * n / tn,
        "unit": "updates/s",
        "cores": orc.num_threads(),
        "kind": "oracle",
        "sample": f"{n} FP64 RK4 steps ({tn:.1f} s) of the {w['M']}-mode state ({S} values) "
                  f"{sample_note}",
    }, err, n + 1


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="two_mode_32")
    ap.add_argument("--timing-every", type=int, default=64,
                    help="bracket every k-th RK4 step's launches with HIP events")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--batch", type=int, default=1, help="t1 branches propagated together")
    ap.add_argument("--precision", choices=["f64", "f32"], default="f64",
                    help="type of the propagated t1-branch states")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--mode", choices=["bench", "kernels", "rk4"], default="bench",
                    help="kernels: a few RK4 steps of the workload plus a plain copy of known "
                         "size, for hardware-counter runs")
    ap.add_argument("--rk4-steps", type=int, default=4, help="RK4 steps in --mode kernels")
    args = ap.parse_args(argv)

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (--gpus {args.gpus} requested): the build targets a "
              f"single MI355X; sharding over t1 branches is described in DESIGN.md", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import paper_2509_25840_amd as pk
    import workloads as wl

    w = wl.workload(args.workload)
    dt = float(w["dt"])
    if args.mode == "bench" and w["kind"] != "2d":
        print(f"bench mode needs a 2D-response workload ({args.workload} is {w['kind']})", file=sys.stderr)
        return 2
    steps_per = rk4_steps(w) if w["kind"] == "2d" else int(w["eq_steps"]) + int(w["n_t"]) - 1
    torch.cuda.init()
    prec = pk.CHFPE_FP32 if args.precision == "f32" else pk.CHFPE_FP64
    solver = pk.Solver(pk.params_from_workload(w, precision=prec, batch=args.batch))
    S = solver.count
    log(f"[bench] workload={args.workload} values/state={S} rk4_steps/step={steps_per}")

    if args.mode == "rk4":
        # time RK4 propagation alone (tile sweeps); one JSON line per call
        solver.equilibrate(0, 0.0)
        solver.propagate(20, dt)
        torch.cuda.synchronize()
        solver.set_kernel_timing(8)
        t0 = time.perf_counter()
        solver.propagate(args.rk4_steps, dt)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        kt = solver.kernel_times()
        print(json.dumps({"mode": "rk4", "workload": args.workload, "rk4_steps": args.rk4_steps,
                          "ms_per_rk4_step": 1000 * el / args.rk4_steps,
                          "updates_per_s": S * args.rk4_steps / el,
                          "alg_frac_16pass": 16 * 8 * S * args.rk4_steps / el / 1e9 / HBM_PEAK_GBPS,
                          "env": {k: v for k, v in os.environ.items() if k.startswith("CHFPE_TUNE")},
                          "kernels": {k: {"ms": v[1], "GBps": v[2] / (v[1] * 1e-3) / 1e9}
                                      for k, v in kt.items() if v[0] > 0}}), flush=True)
        solver.close()
        return 0

    if args.mode == "kernels":
        # the same kernels as a bench step, a few RK4 steps only; then a plain
        # copy of a known byte count as the counter calibration reference
        solver.equilibrate(0, 0.0)  # Boltzmann start on the device
        solver.propagate(args.rk4_steps, dt)
        torch.cuda.synchronize()
        nbytes = 1 << 30
        src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            pk.stream_copy(dst, src, nbytes)
        torch.cuda.synchronize()
        print(json.dumps({"mode": "kernels", "workload": args.workload, "rk4_steps": args.rk4_steps,
                          "values_per_state": S, "copy_bytes": nbytes, "copies": 3}), flush=True)
        solver.close()
        return 0

    def one_step(timing_every=0):
        solver.rebuild()
        if timing_every:
            solver.set_kernel_timing(timing_every)
        solver.equilibrate(int(w["eq_steps"]), dt)
        R = solver.response_2d(w["A"], w["B"], w["C"], int(w["n_t1"]), int(w["n_t2"]),
                               int(w["stride1"]), int(w["stride2"]), dt)
        I = pk.spectrum_2d(R, int(w["stride1"]) * dt, int(w["stride2"]) * dt)
        return R, I

    for i in range(args.warmup):
        log(f"[bench] warmup {i + 1}/{args.warmup}")
        one_step()
    torch.cuda.synchronize()

    times = []
    kcount, ktime, kbyte = {}, {}, {}
    for i in range(args.steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        one_step(args.timing_every)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        # the events of this step's context (read before the next rebuild)
        for k, (cnt, mean, mb) in solver.kernel_times().items():
            kcount[k] = kcount.get(k, 0) + cnt
            ktime[k] = ktime.get(k, 0.0) + cnt * mean
            kbyte[k] = kbyte.get(k, 0.0) + cnt * mb
        log(f"[bench] step {i + 1}/{args.steps}: {times[-1]:.3f} s")
    kt = {k: (kcount[k], ktime[k] / kcount[k] if kcount[k] else 0.0) for k in kcount}
    kb = {k: (kbyte[k] / kcount[k] if kcount[k] else 0.0) for k in kcount}
    total = float(sum(times))
    ms_per_step = 1000.0 * total / args.steps
    updates = float(S) * steps_per * args.steps
    value = updates / total

    # roofline of the dominant kernel (largest share of the timed launches' time)
    share = {k: kt[k][0] * kt[k][1] for k in kt if kt[k][0] > 0}
    roofline = None
    if share:
        dom = max(share, key=share.get)
        mean_ms = kt[dom][1]
        achieved = kb[dom] / (mean_ms * 1e-3) / 1e9
        traffic = None
        tf = os.path.join(ROOT, "profiles", f"traffic_{args.workload}.json")
        if os.path.exists(tf):
            try:
                rec = json.load(open(tf))
                if (rec.get("source_hash") == source_hash() and dom in rec.get("bytes_per_launch", {})
                        and rec.get("batch") == args.batch and rec.get("precision") == args.precision):
                    traffic = float(rec["bytes_per_launch"][dom])
            except (OSError, ValueError):
                traffic = None
        roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1),
                    "peak": HBM_PEAK_GBPS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 4),
                    "traffic": traffic, "mean_ms": mean_ms, "bytes_per_launch": kb[dom],
                    "timed_launches": kt[dom][0]}
    # whole hot path against the 16-pass algorithmic floor of classical RK4
    tb = 4 if args.precision == "f32" else 8
    n_branch = int(w["n_t1"]) * (int(w["n_t2"]) - 1) * int(w["stride2"])
    n_fp64 = steps_per - n_branch
    alg_bytes = 16.0 * S * (8 * n_fp64 + tb * n_branch) * args.steps
    step_alg = {"algorithmic_GBps": alg_bytes / total / 1e9,
                "frac": alg_bytes / total / 1e9 / HBM_PEAK_GBPS}

    cpu = None
    parity = None
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle)")
        cpu, parity, nst = cpu_baseline(w, pk, args.cpu_seconds,
                                        f"of the {steps_per} per bench step")
    solver.close()

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.precision,
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: 2 modes, 32^4 (q,p) grid, depth 3 (10 elements), "
                               f"equilibration 4000 + 2D THz-Raman 64 t1 x 256 t2 RK4 steps, dt {dt}",
                   "values_per_state": S, "rk4_steps_per_step": steps_per,
                   "branch_batch": args.batch, "branch_precision": args.precision},
        "roofline": roofline,
        "path_roofline_16pass": step_alg,
        "cpu_baseline": cpu,
        "spectrum_time_s": ms_per_step / 1000.0,
        "parity_rel_l2_vs_oracle": parity,
        "kernel_mean_ms": {k: v[1] for k, v in kt.items() if v[0] > 0},
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
