"""Benchmark of the CHFPE hot path on one MI355X.

Default workload: three modes on a 24^6 (q, p) grid, depth 2 (10 hierarchy
elements, 1,911,029,760 values per state, 15.3 GB in FP64), FP64 throughout.
Its whole 2D THz-Raman job (4000 equilibration steps, then 64 t1 x 256 t2
samples at stride 1) is 20383 RK4 steps, about half an hour on one GPU, so a
bench step is a fixed slice of that job in which every stage of the path
runs at the job's full grid and depth:
  coefficient tables and upload (chfpe_setup into a resident workspace),
  Boltzmann start + 16 equilibration RK4 steps,
  A^x excitation, then the t1 columns j1 = 0, 1 of R(t2, t1), each with its
  B^x excitation and 8 t2 samples (7 RK4 steps apart, stride 1, dt = 0.005),
  and the 2D spectrum of those columns.
That is 16 + 1 + 2 * 7 = 31 RK4 steps per bench step; the whole job's time
is reported as projected from the measured rate (--slice full runs it).
The two-mode 32^4 workload (--workload two_mode_32) runs its whole job per
step (20383 RK4 steps, 64 t1 branches in one FP64 wave).

Prints one JSON line: hierarchy-gridpoint RK4 updates/s over the timed
steps, the roofline of the dominant kernel (HIP-event timing of sampled RK4
steps inside the timed region; algorithmic bytes per launch from the
library), the whole path against the 16-pass floor of classical RK4, and
the FP64 CPU oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "hierarchy-gridpoint RK4 updates/s + % HBM peak; 2D spectrum time at ≤1e-3 error"
HBM_PEAK_GBPS = 8000.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


KERNEL_SOURCES = ("paper_2509_25840_amd/csrc/kernels.h", "paper_2509_25840_amd/csrc/closure.h",
                  "paper_2509_25840_amd/csrc/chfpe.hip")


def code_of(text: str) -> str:
    """Source text without comments, trailing blanks and empty lines: what the
    compiler sees, so that comment edits leave recorded profiles valid."""
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    text = re.sub(r"//[^\n]*", "", text)
    return "\n".join(line.rstrip() for line in text.splitlines() if line.strip())


def source_hash(read=None) -> str:
    """Hash of the kernel sources' code; profiles record it and bench.py uses a
    profile only while it matches.  `read(rel)` returns a source's text
    (default: the working tree)."""
    if read is None:
        read = lambda rel: open(os.path.join(ROOT, rel), encoding="utf-8").read()
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        h.update(code_of(read(rel)).encode())
    return h.hexdigest()[:16]


def stream_references(pk) -> dict:
    """HBM rates of plain streaming kernels with the read/write mixes of the
    stage passes, over 4 GiB arrays: writes only, one, two and three reads
    per write (best of three each; chfpe_stream_mix on torch's stream)."""
    import torch
    mbytes = 4 << 30
    srcs = [torch.zeros(mbytes // 8, dtype=torch.float64, device="cuda") for _ in range(4)]
    out = {"bytes_per_array": mbytes}
    for ns in (0, 1, 2, 3):
        best = float("inf")
        for _ in range(3):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            pk.stream_mix(srcs[3], srcs[:ns], mbytes)
            e1.record()
            torch.cuda.synchronize()
            best = min(best, e0.elapsed_time(e1))
        out[f"{ns}r1w"] = (ns + 1) * mbytes / (best * 1e-3) / 1e9
    del srcs
    torch.cuda.empty_cache()
    return out


def rk4_steps(w) -> int:
    return (int(w["eq_steps"]) + (int(w["n_t1"]) - 1) * int(w["stride1"])
            + int(w["n_t1"]) * (int(w["n_t2"]) - 1) * int(w["stride2"]))


# Bench-step slices (equilibration steps, t1 columns, t2 samples) of jobs too
# long to run whole per step; other workloads run their whole job.
SLICES = {"three_mode_24": (16, 2, 8), "three_mode_24_hermite": (64, 8, 32)}


def job_slice(w, name: str, spec: str):
    """(workload of one bench step, description).  spec: "" (default slice),
    "full", or "EQ,N_T1,N_T2"."""
    full = dict(w)
    if spec == "full" or (not spec and name not in SLICES):
        return full, "the whole job"
    eq, n1, n2 = SLICES[name] if not spec else (int(x) for x in spec.split(","))
    sl = dict(w, eq_steps=eq, n_t1=n1, n_t2=n2)
    return sl, (f"a slice of the job: Boltzmann start + {eq} equilibration RK4 steps, A^x, t1 columns "
                f"0..{n1 - 1}, each with B^x and {n2} t2 samples")


def describe(name: str, w) -> str:
    M = int(w["M"])
    grid = "x".join(str(n) for n in list(w["Nq"]) + list(w["Np"]))
    same = len(set(list(w["Nq"]) + list(w["Np"]))) == 1
    if same:
        grid = f"{w['Nq'][0]}^{2 * M}"
    if w.get("basis") == "hermite":
        grid = ("x".join(str(n) for n in w["Nq"]) + " q grid x " + "x".join(str(n) for n in w["Np"]) +
                " Hermite functions in p (Sec. III A)")
    else:
        grid += " (q,p) grid"
    return (f"{name}: {M} mode{'s' if M > 1 else ''}, {grid}, depth {w['K']}; "
            f"job = equilibration {w['eq_steps']} + 2D THz-Raman {w['n_t1']} t1 x {w['n_t2']} t2 samples "
            f"(stride {w['stride1']}, dt {w['dt']}) = {rk4_steps(w)} RK4 steps")


def launches_per_rk4_step(M: int) -> dict:
    d = {"pcube_rhs" if M == 3 else "pblock_rhs": 4, "qpass_rk4_s1": 1, "qpass_rk4_s2": 1,
         "qpass_rk4_s3": 1, "qpass_rk4_s4": 1}
    if M == 3:
        d["qpass_acc"] = 4
    return d


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, solver, target_s: float, name: str):
    """Time the FP64 CPU oracle on this workload's full state and compare the
    GPU's result for the same work (relative L2).  States above 5e8 values:
    one right-hand side (an RK4 step is four), else RK4 steps for about
    target_s seconds."""
    import numpy as np
    import oracle as orc
    W0 = orc.boltzmann(w)
    W0[1] = 0.2 * W0[0]  # a non-stationary start so the steps do real work
    S = W0.size
    M = int(w["M"])
    if S > 500_000_000:
        t0 = time.perf_counter()
        ref = orc.rhs(w, W0).ravel()
        tn = time.perf_counter() - t0
        solver.set_state(W0)
        del W0
        solver.rhs()
        got = solver.get_state().ravel()
        value = S / (4.0 * tn)
        sample = (f"one oracle right-hand side of the full {M}-mode state ({S} values, {tn:.1f} s); "
                  f"an RK4 step is four right-hand sides, so updates/s = values / (4 x that time)")
        n_cmp = "1 right-hand side"
    else:
        t0 = time.perf_counter()
        W1 = orc.rk4(w, W0, 1, w["dt"])
        t1 = time.perf_counter() - t0
        n = max(1, min(64, int(target_s / max(t1, 1e-3)) - 1))
        t0 = time.perf_counter()
        ref = orc.rk4(w, W1, n, w["dt"]).ravel()
        tn = time.perf_counter() - t0
        solver.set_state(W0)
        solver.propagate(n + 1, w["dt"])
        got = solver.get_state().ravel()
        value = S * n / tn
        sample = f"{n} FP64 oracle RK4 steps ({tn:.1f} s) of the full {M}-mode state ({S} values)"
        n_cmp = f"{n + 1} RK4 steps"
    err = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    return {
        "value": value,
        "unit": "updates/s",
        "cores": orc.num_threads(),
        "kind": "oracle",
        "sample": sample,
        "cpu_model": cpu_model(),
        "nproc": os.cpu_count(),
        "one_thread": one_thread_rate(name),
    }, err, n_cmp


def oracle_one_thread(name: str) -> dict:
    """One oracle right-hand side, timed in this process (run it with
    OMP_NUM_THREADS=1), on the workload with every axis halved: same modes
    and depth, 1/2^(2M) of the points."""
    import oracle as orc
    import workloads as wl
    w = wl.workload(name)
    h = wl.workload(name, Nq=[max(4, n // 2) for n in w["Nq"]], Np=[max(4, n // 2) for n in w["Np"]])
    W0 = orc.boltzmann(h)
    W0[1] = 0.2 * W0[0]
    t0 = time.perf_counter()
    orc.rhs(h, W0)
    t = time.perf_counter() - t0
    return {"value": W0.size / (4.0 * t), "unit": "updates/s", "threads": orc.num_threads(),
            "sample": f"one oracle right-hand side ({t:.1f} s) of the {name} workload with every "
                      f"axis halved (Nq {h['Nq']}, Np {h['Np']}, {W0.size} values); updates/s = values / (4 x time)"}


def one_thread_rate(name: str):
    """oracle_one_thread in a child process limited to one OpenMP thread
    (None if that run fails)."""
    import subprocess
    env = dict(os.environ, OMP_NUM_THREADS="1")
    try:
        r = subprocess.run([sys.executable, os.path.abspath(__file__), "--mode", "oracle1", "--workload", name],
                           env=env, capture_output=True, text=True, timeout=300)
        return json.loads(r.stdout.strip().splitlines()[-1]) if r.returncode == 0 else None
    except (subprocess.SubprocessError, ValueError, IndexError):
        return None



# ---------------------------------------------------------------------------
# rocprofv3 output -> text summaries under profiles/ (runs without a GPU)

# k_qpass epilogues; the two middle RK4 stages share one instantiation
_EPI_KIND = {0: "qpass_acc", 1: "qpass_out", 2: "qpass_rk4_s1", 3: "qpass_rk4_s23", 4: "qpass_rk4_s4"}
# k_hcube (Hermite basis): one launch per stage, same epilogue numbering
_HEPI_KIND = {1: "hcube_out", 2: "hcube_rk4_s1", 3: "hcube_rk4_s23", 4: "hcube_rk4_s4"}


def _short_name(name: str) -> str:
    s = name.split("(")[0] if not name.startswith("void ") else name[5:].split("(")[0]
    return s.replace("chfpe::", "").strip()


def _kind_of(short: str, grid: int, min_grid: dict):
    """Library kernel kind of one dispatch (the names chfpe_kernel_times uses);
    a launch over several branch states has a larger grid than the single-state
    launch of the same instantiation, and FP32 launches are always batched."""
    fam = short.split("<")[0]
    targs = [a.strip() for a in short[short.find("<") + 1:short.rfind(">")].split(",")] if "<" in short else []
    if fam == "k_pblock":
        kind = "perturb" if targs[5] == "true" else "pblock_rhs"  # <T, TO, NMAX, RPT, MM, PERTURB, CLOS>
    elif fam in ("k_pcube", "k_pcube_s"):
        kind = "perturb" if targs[4] == "true" else "pcube_rhs"  # <T, TO, NB1, SPLIT, PERTURB[, CLOS]>
    elif fam == "k_qpass":
        if int(targs[5]) == 2:        # dX/dq field: second launch of a perturbation
            kind = "perturb_q"
        else:
            kind = _EPI_KIND[int(targs[4])]
    elif fam == "k_hcube":
        kind = _HEPI_KIND[int(targs[3])]  # <T, NB1, SPLIT, EPI>
    elif fam == "k_hperturb":
        kind = "perturb"
    elif fam == "k_reduce_w0":
        kind = "observe"
    else:
        return None
    batched = (targs and targs[0] == "float" and kind != "perturb") or grid > min_grid.get(short, grid)
    return ("batch_" + kind) if batched else kind


def _grid(row: dict) -> int:
    if "Grid_Size" in row:
        return int(float(row["Grid_Size"]))
    g = 1
    for ax in ("X", "Y", "Z"):
        g *= int(float(row.get(f"Grid_Size_{ax}", 1) or 1))
    return g


def _csv(folder: str, suffix: str):
    import csv
    import glob
    files = sorted(glob.glob(os.path.join(folder, "**", f"*{suffix}"), recursive=True))
    if not files:
        raise SystemExit(f"no *{suffix} under {folder}")
    with open(files[0], newline="") as f:
        return list(csv.DictReader(f))


def _cmd(args, extra: str) -> str:
    return (f"python bench.py {extra} --workload {args.workload} --batch {args.batch} "
            f"--precision {args.precision}" + (f" --tiles {args.tiles}" if args.tiles else ""))


def recorded_traffic(workload: str, batch: int, precision: str, tiles: str, kind: str,
                     prof: str = os.path.join(ROOT, "profiles")):
    """Counter-measured HBM bytes per launch of `kind` from a traffic record
    of the same kernel sources, batch, precision and tile choice (the main
    record or a tile-specific one), else None."""
    names = sorted(f for f in os.listdir(prof) if f.startswith(f"traffic_{workload}")
                   and f.endswith(".json")) if os.path.isdir(prof) else []
    for name in names:
        try:
            rec = json.load(open(os.path.join(prof, name)))
        except (OSError, ValueError):
            continue
        if (rec.get("source_hash") == source_hash() and kind in rec.get("bytes_per_launch", {})
                and rec.get("batch") == batch and rec.get("precision") == precision
                and rec.get("tiles") in ("", tiles)):
            return float(rec["bytes_per_launch"][kind])
    return None


# SQ counters count per-wave cycles in units of 4 cycles; ratios below use
# the raw values (units cancel) and instruction counts per wave.
_COUNTER_COLS = [
    ("VALU active", lambda c: c["SQ_ACTIVE_INST_VALU"] / c["SQ_WAVE_CYCLES"]),
    ("waiting (any)", lambda c: c["SQ_WAIT_ANY"] / c["SQ_WAVE_CYCLES"]),
    ("waiting for issue", lambda c: c["SQ_WAIT_INST_ANY"] / c["SQ_WAVE_CYCLES"]),
    ("LDS active", lambda c: c["SQ_ACTIVE_INST_LDS"] / c["SQ_WAVE_CYCLES"]),
    ("VALU instr/wave", lambda c: c["SQ_INSTS_VALU"] / c["SQ_WAVES"]),
    ("SALU instr/wave", lambda c: c["SQ_INSTS_SALU"] / c["SQ_WAVES"]),
    ("VMEM rd / wr per wave", lambda c: f"{c['SQ_INSTS_VMEM_RD'] / c['SQ_WAVES']:.0f} / "
                                        f"{c['SQ_INSTS_VMEM_WR'] / c['SQ_WAVES']:.0f}"),
    ("LDS instr/wave", lambda c: c["SQ_INSTS_LDS"] / c["SQ_WAVES"]),
    ("LDS bank-conflict / LDS active", lambda c: c["SQ_LDS_BANK_CONFLICT"] / max(c["SQ_LDS_IDX_ACTIVE"], 1.0)),
    ("L1->L2 latency (cycles)", lambda c: c["TCP_TCC_READ_REQ_LATENCY_sum"] / max(c["TCP_TCC_READ_REQ_sum"], 1.0)),
    ("L2 hit rate", lambda c: c["TCC_HIT_sum"] / max(c["TCC_HIT_sum"] + c["TCC_MISS_sum"], 1.0)),
]


def summarise_counters(args, kern_cmd: str) -> None:
    """counters_<workload>.md: per-kernel issue, stall, LDS and cache
    counters, summed over the dispatches of each instantiation and grid."""
    per, passes = {}, []
    for folder in [d for d in args.counter_dirs.split(",") if d]:
        rows = _csv(folder, "counter_collection.csv")
        names = sorted({r["Counter_Name"] for r in rows})
        passes.append(names)
        for r in rows:
            s = _short_name(r["Kernel_Name"])
            if not s.startswith(("k_pcube", "k_qpass", "k_pblock", "k_hcube")):
                continue
            key = (s, _grid(r))
            per.setdefault(key, {})
            per[key][r["Counter_Name"]] = per[key].get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    lines = [f"# Issue and stall counters: {args.workload}, {args.precision} branch states, "
             f"{args.batch}-branch waves", "",
             f"Commands (repository root; one pass per counter set, each over the kernels of a few RK4 steps):", ""]
    for names in passes:
        lines.append(f"    rocprofv3 --pmc {' '.join(names)} --output-format csv -d <dir> -o run -- {kern_cmd}")
    lines += ["", "Counter values summed over the dispatches of one kernel instantiation and grid. "
              "Fractions are of SQ_WAVE_CYCLES (per-wave cycles); instruction counts are per wave "
              "(SQ_INSTS_* / SQ_WAVES); L1->L2 latency is TCP_TCC_READ_REQ_LATENCY_sum / "
              "TCP_TCC_READ_REQ_sum; L2 hit rate is TCC_HIT / (TCC_HIT + TCC_MISS).", "",
              "| kernel | grid | " + " | ".join(c for c, _ in _COUNTER_COLS) + " |",
              "|---|---|" + "---|" * len(_COUNTER_COLS)]
    for (s, g), c in sorted(per.items()):
        cells = []
        for _, f in _COUNTER_COLS:
            try:
                v = f(c)
                cells.append(v if isinstance(v, str) else (f"{v:.3f}" if v < 10 else f"{v:.0f}"))
            except (KeyError, ZeroDivisionError):
                cells.append("-")
        lines.append(f"| `{s[:70]}` | {g} | " + " | ".join(cells) + " |")
    lines += ["", f"Kernel sources hash: {source_hash()}."]
    path = os.path.join(ROOT, "profiles", f"counters_{args.workload}.md")
    open(path, "w").write("\n".join(lines) + "\n")
    log(f"[summarise] wrote {path}")


def summarise(args) -> int:
    tag = f"{args.workload}_{args.precision}_b{args.batch}"
    os.makedirs(os.path.join(ROOT, "profiles"), exist_ok=True)
    bench_cmd = _cmd(args, "--steps 1 --warmup 0 --no-cpu-baseline")
    kern_cmd = _cmd(args, "--mode kernels --rk4-steps 4")
    if args.trace_dir:
        rows = _csv(args.trace_dir, "kernel_trace.csv")
        rows.sort(key=lambda r: int(r["Start_Timestamp"]))
        marks = [i for i, r in enumerate(rows) if "k_stream_copy" in r["Kernel_Name"]]
        if marks:  # the timed region of bench.py starts after its marker copy
            rows = rows[marks[-1] + 1:]
        min_grid = {}
        for r in rows:
            s = _short_name(r["Kernel_Name"])
            min_grid[s] = min(min_grid.get(s, 1 << 62), _grid(r))
        groups = {}
        for r in rows:
            s = _short_name(r["Kernel_Name"])
            g = _grid(r)
            d = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-6
            e = groups.setdefault((s, g), [0, 0.0, _kind_of(s, g, min_grid)])
            e[0] += 1
            e[1] += d
        total = sum(e[1] for e in groups.values())
        ev = {}
        if args.bench_json and os.path.exists(args.bench_json):
            for line in open(args.bench_json):
                if line.startswith("{"):
                    ev = json.loads(line).get("kernel_mean_ms", {})
        lines = [f"# Kernel trace: {args.workload}, {args.precision} branch states, "
                 f"{args.batch}-branch waves, one bench step",
                 "", "Command (repository root, ROCm 7 rocprofv3):", "",
                 f"    rocprofv3 --kernel-trace --stats --output-format csv -d <out> -o run -- {bench_cmd}",
                 "", "Per kernel instantiation and grid, from the kernel trace of the timed region "
                 "(dispatches after bench.py's marker copy; durations from the trace's timestamps; "
                 "`event mean` is the same run's HIP-event mean of that kind, from the JSON line "
                 "bench.py printed):", "",
                 "| kind | kernel | grid | calls | mean ms | event mean ms | total s | share |",
                 "|---|---|---|---|---|---|---|---|"]
        for (s, g), (n, t, kind) in sorted(groups.items(), key=lambda kv: -kv[1][1])[:24]:
            em = ev.get(kind) if kind else None
            lines.append(f"| {kind or '-'} | `{s[:70]}` | {g} | {n} | {t / n:.4f} | "
                         f"{'%.4f' % em if em else '-'} | {t / 1e3:.3f} | {100 * t / total:.1f}% |")
        st = _csv(args.trace_dir, "kernel_stats.csv")
        lines += ["", "rocprofv3 --stats (kernel_stats.csv, the whole run: setup, autotuning, warmup "
                  "and the timed step), top 12 by total time:", "",
                  "| kernel | calls | total s | mean ms | % |", "|---|---|---|---|---|"]
        for r in st[:12]:
            lines.append(f"| `{_short_name(r['Name'])[:70]}` | {r['Calls']} | "
                         f"{float(r['TotalDurationNs']) * 1e-9:.3f} | {float(r['AverageNs']) * 1e-6:.4f} | "
                         f"{float(r['Percentage']):.1f} |")
        path = os.path.join(ROOT, "profiles", f"kernel_trace_{tag}.md")
        open(path, "w").write("\n".join(lines) + "\n")
        log(f"[summarise] wrote {path}")
    if args.counter_dirs:
        summarise_counters(args, kern_cmd)
    if args.fetch_dir and args.write_dir:
        per = {}
        for which, folder in (("fetch", args.fetch_dir), ("write", args.write_dir)):
            rows = _csv(folder, "counter_collection.csv")
            min_grid = {}
            for r in rows:
                s = _short_name(r["Kernel_Name"])
                min_grid[s] = min(min_grid.get(s, 1 << 62), _grid(r))
            for r in rows:
                s = _short_name(r["Kernel_Name"])
                kind = "copy" if s.startswith("k_stream_copy") else _kind_of(s, _grid(r), min_grid)
                if kind is None:
                    continue
                e = per.setdefault(kind, {}).setdefault(which, [0, 0.0])
                e[0] += 1
                e[1] += float(r["Counter_Value"]) * 1024.0
        kj = {}
        if args.kernels_json and os.path.exists(args.kernels_json):
            for line in open(args.kernels_json):
                if line.startswith("{"):
                    kj = json.loads(line)
        copy_bytes = float(kj.get("copy_bytes", 1 << 30))
        ff = copy_bytes / (per["copy"]["fetch"][1] / per["copy"]["fetch"][0])
        wf = copy_bytes / (per["copy"]["write"][1] / per["copy"]["write"][0])
        alg = kj.get("kernel_bytes", {})
        rec = {"workload": args.workload, "batch": args.batch, "precision": args.precision,
               "tiles": args.tiles, "source_hash": source_hash(),
               "calibration": {"copy_bytes": copy_bytes, "fetch_factor": ff, "write_factor": wf},
               "fetch_bytes_per_launch": {}, "write_bytes_per_launch": {}, "bytes_per_launch": {},
               "algorithmic_bytes_per_launch": alg,
               "commands": [f"rocprofv3 --pmc FETCH_SIZE --output-format csv -d <fetch> -o run -- {kern_cmd}",
                            f"rocprofv3 --pmc WRITE_SIZE --output-format csv -d <write> -o run -- {kern_cmd}"]}
        for kind, d in sorted(per.items()):
            if kind == "copy" or "fetch" not in d or "write" not in d:
                continue
            fb = ff * d["fetch"][1] / d["fetch"][0]
            wb = wf * d["write"][1] / d["write"][0]
            rec["fetch_bytes_per_launch"][kind] = fb
            rec["write_bytes_per_launch"][kind] = wb
            rec["bytes_per_launch"][kind] = fb + wb
        if args.traffic_variant:
            # another tile choice of the same kernels: its record only, beside the main one
            tag = args.tiles.replace(",", "_")
            path = os.path.join(ROOT, "profiles", f"traffic_{args.workload}_tiles_{tag}.json")
            json.dump(rec, open(path, "w"), indent=1)
            log(f"[summarise] wrote {path}")
            return 0
        path = os.path.join(ROOT, "profiles", f"traffic_{args.workload}.json")
        json.dump(rec, open(path, "w"), indent=1)
        lines = [f"# HBM traffic per launch: {args.workload}, {args.precision} branch states, "
                 f"{args.batch}-branch waves", "", "Commands (repository root):", ""]
        lines += [f"    {c}" for c in rec["commands"]]
        lines += ["", f"FETCH_SIZE and WRITE_SIZE (KiB per dispatch) are scaled by what they read for "
                  f"a plain {copy_bytes / 2**30:.0f} GiB copy kernel in the same run: fetch factor "
                  f"{ff:.3f}, write factor {wf:.3f}.", "",
                  "| kind | launches | fetch MB | write MB | total MB | algorithmic MB | total / algorithmic |",
                  "|---|---|---|---|---|---|---|"]
        for kind in rec["bytes_per_launch"]:
            # the two middle RK4 stages share one instantiation (qpass_rk4_s23)
            a = alg.get(kind) or (alg.get(kind[:-3] + "s2") if kind.endswith("_rk4_s23") else None)
            t = rec["bytes_per_launch"][kind]
            lines.append(f"| {kind} | {per[kind]['fetch'][0]} | {rec['fetch_bytes_per_launch'][kind] / 1e6:.2f} | "
                         f"{rec['write_bytes_per_launch'][kind] / 1e6:.2f} | {t / 1e6:.2f} | "
                         f"{'%.2f' % (a / 1e6) if a else '-'} | {'%.3f' % (t / a) if a else '-'} |")
        lines += ["", f"Kernel sources hash: {rec['source_hash']} (of their code, comments excluded; bench.py "
                  f"uses these figures only while the kernel sources hash to this value)."]
        path = os.path.join(ROOT, "profiles", f"traffic_{args.workload}.md")
        open(path, "w").write("\n".join(lines) + "\n")
        log(f"[summarise] wrote {path}")
    return 0


def auto_batch(pk, w, prec, total_bytes: int) -> int:
    """Largest branch batch (at most n_t1) whose workspace fits in 85% of the
    device memory; 1 for states of 2 GB or more, which fill the GPU alone."""
    n_t1 = int(w.get("n_t1", 1))
    if pk.workspace_bytes(pk.params_from_workload(w, precision=pk.CHFPE_FP64, batch=1)) >= 6 * 2e9:
        return 1
    base = pk.workspace_bytes(pk.params_from_workload(w, precision=pk.CHFPE_FP64, batch=1))
    one = pk.workspace_bytes(pk.params_from_workload(w, precision=prec, batch=1))
    two = pk.workspace_bytes(pk.params_from_workload(w, precision=prec, batch=2))
    per = max(1, two - one)  # branch buffers of one more branch
    fit = int((0.85 * total_bytes - base) // per)
    return max(1, min(n_t1, fit))


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="three_mode_24")
    ap.add_argument("--slice", default="",
                    help="bench step: 'full' (the whole job), 'EQ,N_T1,N_T2', or empty for the "
                         "workload's default (three_mode_24: 16,2,8; others: the whole job)")
    ap.add_argument("--timing-every", type=int, default=8,
                    help="bracket every k-th RK4 step's launches with HIP events")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--batch", type=int, default=0,
                    help="t1 branches propagated together (0: as many as fit in 85%% of device "
                         "memory, at most n_t1; two_mode_32: all 64 in one wave)")
    ap.add_argument("--precision", choices=["f64", "f32"], default="f64",
                    help="type of the propagated t1-branch states")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the planner's default tile shapes (no chfpe_autotune before warmup)")
    ap.add_argument("--tiles", default="",
                    help="NB,SPLIT,PC[,RUN]: fixed tile shapes (k_pblock blocks per task, lane-pair "
                         "line solves 0/1, q-pass run positions per tile, k_pblock block groups "
                         "per state in task order) instead of autotuning")
    ap.add_argument("--mode", choices=["bench", "kernels", "rk4", "summarise", "precision", "closure", "oracle1",
                                       "basis"],
                    default="bench",
                    help="kernels: a few RK4 steps of the workload (single state, then one "
                         "batched wave) plus a plain copy of known size, for hardware-counter "
                         "runs; summarise: turn rocprofv3 output of the bench and kernels "
                         "commands into the text summaries under profiles/ (no GPU)")
    ap.add_argument("--closure-draws", type=int, default=16, help="closure: training draws (seeds 0..)")
    ap.add_argument("--closure-held", type=int, default=4, help="closure: held-out draws (seeds 1000..)")
    ap.add_argument("--closure-steps", type=int, default=3000, help="closure: Adam steps")
    ap.add_argument("--closure-lr", type=float, default=3e-3)
    ap.add_argument("--closure-snap", default="1000,400,50",
                    help="closure: fine-run equilibration steps, steps after each excitation, snapshot spacing")
    ap.add_argument("--judge", default="",
                    help="closure: EQ,N_T1,N_T2,STRIDE of the judged responses (default: the workload's)")
    ap.add_argument("--closure-stage", choices=["all", "moments", "fine", "final"], default="all",
                    help="closure: all in one run, or in stages that save to and read from --leg-dir: "
                         "moments (draws of --closure-draw-range), fine (judge columns --judge-cols of "
                         "the fine FP64 response), final (train, coarse runs, comparison)")
    ap.add_argument("--closure-draw-range", default="", help="closure moments stage: FIRST:END draw seeds")
    ap.add_argument("--judge-cols", default="", help="closure fine stage: FIRST:END t1 columns")
    ap.add_argument("--judge-cases", default="",
                    help="closure fine stage: comma-separated cases to run (nominal, held_1000, ...; default all)")
    ap.add_argument("--ref-batch", type=int, default=0,
                    help="precision: branch batch of the FP64 reference run (0: --batch)")
    ap.add_argument("--legs", default="f64,f32",
                    help="precision: the runs made here (f64, f32 or both); results of the others "
                         "come from --leg-dir")
    ap.add_argument("--leg-dir", default="",
                    help="precision: folder each leg's R, spectrum and timing are saved to and read from")
    ap.add_argument("--trace-dir", help="summarise: rocprofv3 --kernel-trace --stats output folder")
    ap.add_argument("--fetch-dir", help="summarise: rocprofv3 --pmc FETCH_SIZE output folder")
    ap.add_argument("--write-dir", help="summarise: rocprofv3 --pmc WRITE_SIZE output folder")
    ap.add_argument("--bench-json", help="summarise: the JSON line the traced bench run printed")
    ap.add_argument("--kernels-json", help="summarise: the JSON line the counted kernels run printed")
    ap.add_argument("--counter-dirs", default="",
                    help="summarise: comma-separated rocprofv3 --pmc output folders of SQ/TCP/TCC counter passes "
                         "(each over the kernels command), summarised per kernel into counters_<workload>.md")
    ap.add_argument("--traffic-variant", action="store_true",
                    help="summarise: write only a tile-specific traffic record (traffic_<workload>_tiles_<tiles>.json)")
    ap.add_argument("--rk4-steps", type=int, default=4, help="RK4 steps in --mode kernels")
    ap.add_argument("--basis-run", default="400,4,32",
                    help="basis: EQ,N_T1,N_T2 of the R^(2) both p bases compute (strides 1, the workload's dt)")
    ap.add_argument("--hermite-n", type=int, default=0,
                    help="basis: Hermite functions per mode (0: those of the workload's _hermite variant)")
    ap.add_argument("--basis-ref", type=int, default=0,
                    help="basis: also a reference run with this many Hermite functions per mode, "
                         "against which both bases' errors are reported (0: none)")
    ap.add_argument("--tune", action="store_true", help="rk4: autotune the tile shapes first")
    args = ap.parse_args(argv)
    if args.mode == "summarise":
        return summarise(args)
    if args.mode == "oracle1":  # the CPU oracle alone (cpu_baseline's one-thread figure); no GPU
        import workloads as wl
        print(json.dumps(oracle_one_thread(args.workload)), flush=True)
        return 0

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (--gpus {args.gpus} requested): the solver targets a "
              f"single MI355X; splitting the t1 branches over GPUs (chfpe_response_2d_range per "
              f"GPU) is not built", file=sys.stderr)
        return 2

    if args.tiles:
        vals = [int(x) for x in args.tiles.split(",")]
        nb, split, pc = vals[:3]
        os.environ["CHFPE_TUNE_PB_NB"] = str(nb)
        os.environ["CHFPE_TUNE_PB_SPLIT"] = str(split)
        os.environ["CHFPE_TUNE_Q_PC"] = str(pc)
        os.environ["CHFPE_TUNE_PB_RUN"] = str(vals[3] if len(vals) > 3 else 0)
        args.no_autotune = True

    import numpy as np
    import torch

    import paper_2509_25840_amd as pk
    import workloads as wl

    w = wl.workload(args.workload)
    dt = float(w["dt"])
    if args.mode == "bench" and w["kind"] != "2d":
        print(f"bench mode needs a 2D-response workload ({args.workload} is {w['kind']})", file=sys.stderr)
        return 2
    ws, slice_desc = job_slice(w, args.workload, args.slice) if w["kind"] == "2d" else (w, "")
    steps_per = rk4_steps(ws) if w["kind"] == "2d" else int(w["eq_steps"]) + int(w["n_t"]) - 1
    torch.cuda.init()
    prec = pk.CHFPE_FP32 if args.precision == "f32" else pk.CHFPE_FP64
    if args.mode == "rk4":
        args.batch = 1  # propagation of one FP64 state: no branch buffers
    elif args.batch <= 0:
        args.batch = auto_batch(pk, w, prec, torch.cuda.get_device_properties(0).total_memory)
    if args.mode in ("precision", "closure", "basis"):
        # these modes make their own contexts; no workspace of this shape
        S = wl.n_elements(int(w["M"]), int(w["K"])) * int(np.prod(w["Nq"])) * int(np.prod(w["Np"]))

        class _NoSolver:
            def close(self):
                pass

        solver = _NoSolver()
    else:
        solver = pk.Solver(pk.params_from_workload(w, precision=prec, batch=args.batch))
        S = solver.count
    log(f"[bench] workload={args.workload} values/state={S} rk4_steps/step={steps_per}")

    if args.mode == "rk4":
        # time RK4 propagation alone (tile sweeps); one JSON line per call
        solver.equilibrate(0, 0.0)
        tiles = solver.autotune(2) if args.tune else solver.tile_config()
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
                          "tiles": tiles,
                          "kernels": {k: {"ms": v[1], "GBps": v[2] / (v[1] * 1e-3) / 1e9}
                                      for k, v in kt.items() if v[0] > 0}}), flush=True)
        solver.close()
        return 0

    if args.mode == "closure":
        # train the closure of the 2:1 coarse grid of this workload on fine
        # runs of seeded draws, then judge it on held-out draws and on the
        # workload itself against the fine-grid FP64 spectrum
        import copy
        import paper_2509_25840_amd.closure as clo
        solver.close()
        wc = copy.deepcopy(w)
        wc["Nq"] = [n // 2 for n in w["Nq"]]
        wc["Np"] = [n // 2 for n in w["Np"]]
        n_eq, n_prop, every = (int(x) for x in args.closure_snap.split(","))
        stage = args.closure_stage
        if stage != "all" and not args.leg_dir:
            log("[closure] staged runs need --leg-dir")
            return 2
        mom_file = lambda sd: os.path.join(args.leg_dir, f"closure_moments_{args.workload}_{sd}.npz")
        if args.judge:
            j_eq, j1, j2, js = (int(x) for x in args.judge.split(","))
        else:
            j_eq, j1, j2, js = int(w["eq_steps"]), int(w["n_t1"]), int(w["n_t2"]), int(w["stride1"])
        judged = [("nominal", wc)] + [(f"held_{1000 + k}", wl.draw_perturbed(wc, 1000 + k))
                                      for k in range(args.closure_held)]
        mem = torch.cuda.get_device_properties(0).total_memory

        if stage == "moments":
            a, b = (int(x) for x in args.closure_draw_range.split(":"))
            os.makedirs(args.leg_dir, exist_ok=True)
            t0 = time.perf_counter()
            for sd in range(a, b):
                mom = clo.fine_moments(wl.draw_perturbed(wc, sd), n_eq, n_prop, every, dt,
                                       progress=lambda n: log(f"[closure] draw {sd}: snapshot {n} "
                                                              f"({time.perf_counter() - t0:.1f} s)"))
                clo.save_moments(mom_file(sd), mom)
                log(f"[closure] moments of draw {sd} saved ({time.perf_counter() - t0:.1f} s)")
            print(json.dumps({"mode": "closure", "stage": "moments", "fine_workload": args.workload,
                              "draws": [a, b], "snapshots": args.closure_snap,
                              "seconds": time.perf_counter() - t0}), flush=True)
            return 0

        def fine_file(name, c0, c1):
            return os.path.join(args.leg_dir, f"closure_fine_{args.workload}_{name}_{j_eq}_{j2}_{js}_{c0}_{c1}.npz")

        if stage == "fine":
            c0, c1 = (int(x) for x in args.judge_cols.split(":")) if args.judge_cols else (0, j1)
            os.makedirs(args.leg_dir, exist_ok=True)
            only = [x for x in args.judge_cases.split(",") if x]
            for name, wj in judged:
                if only and name not in only:
                    continue
                wf = clo.fine_of(wj)
                t0 = time.perf_counter()
                with pk.Solver(pk.params_from_workload(wf, precision=pk.CHFPE_FP64, batch=1)) as s:
                    s.equilibrate(j_eq, dt)
                    torch.cuda.synchronize()
                    t_eq = time.perf_counter() - t0
                    log(f"[closure] fine {name}: equilibrated ({t_eq:.1f} s)")
                    cols = []
                    for c in range(c0, c1):  # one column per call: progress between calls
                        cols.append(s.response_2d_range(wf["A"], wf["B"], wf["C"], c, c + 1, j2, js, js, dt))
                        log(f"[closure] fine {name}: column {c} ({time.perf_counter() - t0:.1f} s)")
                    torch.cuda.synchronize()
                # column time includes re-advancing U to each column's t1 (an upper bound)
                np.savez(fine_file(name, c0, c1), R=np.concatenate(cols, axis=1), eq_seconds=t_eq,
                         col_seconds=time.perf_counter() - t0 - t_eq)
            print(json.dumps({"mode": "closure", "stage": "fine", "fine_workload": args.workload,
                              "judge": [j_eq, j1, j2, js], "cols": [c0, c1]}), flush=True)
            return 0

        t0 = time.perf_counter()
        draws = []
        for sd in range(args.closure_draws):
            wd = wl.draw_perturbed(wc, sd)
            if stage == "final":
                draws.append((wd, clo.load_moments(mom_file(sd))))
            else:
                draws.append((wd, clo.fine_moments(wd, n_eq, n_prop, every, dt)))
                log(f"[closure] moments of draw {sd}")
        data = clo.training_set(draws)
        t_data = time.perf_counter() - t0
        t0 = time.perf_counter()
        tr, hist = clo.train(data, args.closure_steps, args.closure_lr)
        t_train = time.perf_counter() - t0
        log(f"[closure] trained: loss {hist[0]:.4e} -> {hist[-1]:.4e} ({t_train:.2f} s)")

        def spectrum(wk, nb, sv=None):
            with pk.Solver(pk.params_from_workload(wk, precision=pk.CHFPE_FP64, batch=nb)) as s:
                if sv is not None:
                    s.set_closure(sv)
                torch.cuda.synchronize()
                ts = time.perf_counter()
                s.equilibrate(j_eq, dt)
                R = s.response_2d(wk["A"], wk["B"], wk["C"], j1, j2, js, js, dt)
                I = pk.spectrum_2d(R, js * dt, js * dt)
                torch.cuda.synchronize()
                return R, I, time.perf_counter() - ts

        def saved_fine(name):
            # the fine columns of earlier fine-stage runs, in order, covering 0..j1
            parts, c, secs = [], 0, None
            while c < j1:
                hits = [f for f in os.listdir(args.leg_dir)
                        if f.startswith(f"closure_fine_{args.workload}_{name}_{j_eq}_{j2}_{js}_{c}_")]
                if not hits:
                    raise SystemExit(f"closure final: no saved fine columns from {c} for {name}")
                c1 = max(int(f[:-4].rsplit("_", 1)[1]) for f in hits)
                z = np.load(fine_file(name, c, c1))
                parts.append(z["R"])
                secs = (float(z["eq_seconds"]) if secs is None else secs) + float(z["col_seconds"])
                c = c1
            R = np.concatenate(parts, axis=1)[:, :j1]
            return R, pk.spectrum_2d(R, js * dt, js * dt), secs

        rows = []
        for name, wj in judged:
            wf = clo.fine_of(wj)
            nbc = auto_batch(pk, {**wj, "n_t1": j1}, pk.CHFPE_FP64, mem)
            if stage == "final":
                Rf, If, tf = saved_fine(name)
            else:
                Rf, If, tf = spectrum(wf, auto_batch(pk, {**wf, "n_t1": j1}, pk.CHFPE_FP64, mem))
            Rp, Ip, tp = spectrum(wj, nbc)
            Rc, Ic, tc = spectrum(wj, nbc, clo.entries(tr.prm, wj))
            e = lambda a, b: float(np.linalg.norm(a - b) / np.linalg.norm(b))
            rows.append({"case": name, "fine_s": tf, "coarse_s": tp, "closure_s": tc,
                         "spectrum_err_plain": e(Ip, If), "spectrum_err_closure": e(Ic, If),
                         "R_err_plain": e(Rp, Rf), "R_err_closure": e(Rc, Rf)})
            log(f"[closure] {name}: plain {rows[-1]['spectrum_err_plain']:.3e} "
                f"closure {rows[-1]['spectrum_err_closure']:.3e} fine {tf:.2f} s coarse {tc:.2f} s")
        out = {"mode": "closure", "stage": stage, "fine_workload": args.workload, "coarse_grid": wc["Nq"] + wc["Np"],
               "draws": args.closure_draws, "snapshots": args.closure_snap, "steps": args.closure_steps,
               "lr": args.closure_lr, "loss_first": float(hist[0]), "loss_last": float(hist[-1]),
               "data_s": t_data, "train_s": t_train, "judge": [j_eq, j1, j2, js], "cases": rows,
               "speedup_closure_vs_fine": float(np.mean([r["fine_s"] / r["closure_s"] for r in rows]))}
        print(json.dumps(out), flush=True)
        return 0

    if args.mode == "basis":
        # the same R^(2) in both p bases on the workload's q grid (FP64): the
        # p grid of the workload and the Hermite functions of Sec. III A
        import copy
        n_eq, n1, n2 = (int(x) for x in args.basis_run.split(","))
        wh = copy.deepcopy(w)
        nh = args.hermite_n or int(wl.workload(args.workload + "_hermite")["Np"][0])
        wh["Np"] = [nh] * int(w["M"])
        wh["basis"] = "hermite"
        res = {}
        runs = [("grid", w), ("hermite", wh)]
        if args.basis_ref:
            wr = copy.deepcopy(wh)
            wr["Np"] = [args.basis_ref] * int(w["M"])
            runs.append(("reference", wr))
        for name, ww in runs:
            with pk.Solver(pk.params_from_workload(ww, precision=pk.CHFPE_FP64, batch=1)) as sv:
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                sv.equilibrate(n_eq, dt)
                R = sv.response_2d(w["A"], w["B"], w["C"], n1, n2, 1, 1, dt)
                torch.cuda.synchronize()
                el = time.perf_counter() - t0
                steps = n_eq + (n1 - 1) + n1 * (n2 - 1)
                res[name] = {"seconds": el, "values_per_state": sv.count, "R": R,
                             "updates_per_s": sv.count * steps / el}
            log(f"[basis] {name}: {el:.2f} s, {res[name]['values_per_state']} values per state")
        Rg, Rh = res["grid"]["R"], res["hermite"]["R"]
        out = {"mode": "basis", "workload": args.workload, "q_grid": w["Nq"], "p_grid": w["Np"], "p_box": w["Lp"],
               "hermite_functions": wh["Np"], "run": {"eq_steps": n_eq, "n_t1": n1, "n_t2": n2, "dt": dt},
               "R_rel_l2_hermite_vs_grid": float(np.linalg.norm(Rh - Rg) / np.linalg.norm(Rg)),
               "R_max_abs_grid": float(np.abs(Rg).max()),
               "speedup_hermite_over_grid": res["grid"]["seconds"] / res["hermite"]["seconds"]}
        if args.basis_ref:
            Rr = res["reference"]["R"]
            out["reference_hermite_functions"] = [args.basis_ref] * int(w["M"])
            out["R_rel_l2_vs_reference"] = {k: float(np.linalg.norm(res[k]["R"] - Rr) / np.linalg.norm(Rr))
                                            for k in ("grid", "hermite")}
        for name in res:
            out[name] = {k: v for k, v in res[name].items() if k != "R"}
        print(json.dumps(out), flush=True)
        return 0

    if args.mode == "precision":
        # the whole hot path twice, FP64 then FP32 branch states: speedup and
        # the FP32 error of R and of the 2D spectrum against the FP64 run
        solver.close()
        out = {"mode": "precision", "workload": args.workload}
        res = {}
        legs = [x for x in args.legs.split(",") if x]
        for prec_name, pcode, nb in (("f64", pk.CHFPE_FP64, args.ref_batch or args.batch),
                                     ("f32", pk.CHFPE_FP32, args.batch)):
            leg_file = os.path.join(args.leg_dir, f"precision_{args.workload}_{prec_name}.npz") if args.leg_dir else ""
            if prec_name not in legs:
                if not leg_file or not os.path.exists(leg_file):
                    log(f"[precision] {prec_name}: not run here and no saved leg")
                    continue
                z = np.load(leg_file)
                res[prec_name] = (z["R"], z["I"])
                out[prec_name] = json.loads(str(z["meta"]))
                log(f"[precision] {prec_name}: read {leg_file}")
                continue
            s = pk.Solver(pk.params_from_workload(w, precision=pcode, batch=nb))
            tiles = s.tile_config() if args.no_autotune else s.autotune(1)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s.equilibrate(int(w["eq_steps"]), dt)
            torch.cuda.synchronize()
            log(f"[precision] {prec_name}: equilibrated ({time.perf_counter() - t0:.1f} s)")
            # one wave of t1 columns per call, so that progress shows between calls
            n1 = int(w["n_t1"])
            cols = []
            for j0 in range(0, n1, nb):
                cols.append(s.response_2d_range(w["A"], w["B"], w["C"], j0, min(n1, j0 + nb), int(w["n_t2"]),
                                                int(w["stride1"]), int(w["stride2"]), dt))
                log(f"[precision] {prec_name}: t1 columns {j0}..{min(n1, j0 + nb) - 1} "
                    f"({time.perf_counter() - t0:.1f} s)")
            R = np.concatenate(cols, axis=1)
            I = pk.spectrum_2d(R, int(w["stride1"]) * dt, int(w["stride2"]) * dt)
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            s.close()
            res[prec_name] = (R, I)
            out[prec_name] = {"seconds": el, "updates_per_s": S * steps_per / el, "batch": nb, "tiles": tiles}
            if leg_file:
                os.makedirs(args.leg_dir, exist_ok=True)
                np.savez(leg_file, R=R, I=I, meta=json.dumps(out[prec_name]))
            log(f"[precision] {prec_name}: {el:.2f} s")
        if "f64" not in res or "f32" not in res:
            print(json.dumps(out), flush=True)
            return 0
        (R64, I64), (R32, I32) = res["f64"], res["f32"]
        out["speedup_f32_over_f64"] = out["f64"]["seconds"] / out["f32"]["seconds"]
        out["R_rel_l2"] = float(np.linalg.norm(R32 - R64) / np.linalg.norm(R64))
        out["spectrum_rel_l2"] = float(np.linalg.norm(I32 - I64) / np.linalg.norm(I64))
        print(json.dumps(out), flush=True)
        return 0

    if args.mode == "kernels":
        # the same kernels as a bench step, a few RK4 steps only; then a plain
        # copy of a known byte count as the counter calibration reference
        solver.set_kernel_timing(1)  # every launch bracketed (and no graph capture)
        solver.equilibrate(0, 0.0)  # Boltzmann start on the device
        solver.propagate(args.rk4_steps, dt)
        if w["kind"] == "2d":
            # one wave of all batch branches, rk4_steps batched RK4 steps long
            nb = max(1, args.batch)
            solver.response_2d(w["A"], w["B"], w["C"], nb, args.rk4_steps + 1, 1, 1, dt)
        torch.cuda.synchronize()
        kt = solver.kernel_times()
        nbytes = 1 << 30
        src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        ev[0].record()
        for i in range(3):  # on torch's current stream, which its events see
            pk.stream_copy(dst, src, nbytes)
            ev[i + 1].record()
        torch.cuda.synchronize()
        copy_ms = [ev[i].elapsed_time(ev[i + 1]) for i in range(3)]
        mix_GBps = stream_references(pk)
        print(json.dumps({"mode": "kernels", "workload": args.workload, "rk4_steps": args.rk4_steps,
                          "values_per_state": S, "copy_bytes": nbytes, "copies": 3,
                          "copy_ms": copy_ms, "copy_GBps": 2 * nbytes / (min(copy_ms) * 1e-3) / 1e9,
                          "stream_mix_GBps": mix_GBps,
                          "kernel_bytes": {k: v[2] for k, v in kt.items() if v[0] > 0},
                          "kernel_ms": {k: v[1] for k, v in kt.items() if v[0] > 0}}), flush=True)
        solver.close()
        return 0

    def one_step(timing_every=0):
        solver.rebuild()
        if timing_every:
            solver.set_kernel_timing(timing_every)
        solver.equilibrate(int(ws["eq_steps"]), dt)
        R = solver.response_2d(w["A"], w["B"], w["C"], int(ws["n_t1"]), int(ws["n_t2"]),
                               int(w["stride1"]), int(w["stride2"]), dt)
        I = pk.spectrum_2d(R, int(w["stride1"]) * dt, int(w["stride2"]) * dt)
        return R, I

    tiles = solver.tile_config()
    if not args.no_autotune:
        # tile shapes for this problem shape, kept by later contexts of the
        # same shape (the rebuild at the start of every step)
        t0 = time.perf_counter()
        tiles = solver.autotune(2)
        log(f"[bench] autotune {time.perf_counter() - t0:.2f} s: {tiles}")
    for i in range(args.warmup):
        log(f"[bench] warmup {i + 1}/{args.warmup}")
        one_step()
    torch.cuda.synchronize()

    # a 16-byte copy marks the start of the timed region in kernel traces
    # (the profile summaries keep only dispatches after the last copy)
    mark = torch.zeros(32, dtype=torch.uint8, device="cuda")
    pk.stream_copy(mark[16:], mark[:16], 16)
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

    tiles_arg = "{},{},{},{}".format(tiles["request_pblock_blocks"], tiles["request_split"],
                                     tiles["request_qpass_positions"], tiles["request_pblock_run"])
    # roofline of the dominant kernel (largest share of the timed launches' time)
    share = {k: kt[k][0] * kt[k][1] for k in kt if kt[k][0] > 0}
    roofline = None
    if share:
        dom = max(share, key=share.get)
        mean_ms = kt[dom][1]
        achieved = kb[dom] / (mean_ms * 1e-3) / 1e9
        traffic = recorded_traffic(args.workload, args.batch, args.precision, tiles_arg, dom)
        roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1),
                    "peak": HBM_PEAK_GBPS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 4),
                    "traffic": traffic, "mean_ms": mean_ms, "bytes_per_launch": kb[dom],
                    "timed_launches": kt[dom][0]}
    # whole hot path against the 16-pass algorithmic floor of classical RK4
    tb = 4 if args.precision == "f32" else 8
    n_branch = int(ws["n_t1"]) * (int(ws["n_t2"]) - 1) * int(w["stride2"])
    n_fp64 = steps_per - n_branch
    alg_bytes = 16.0 * S * (8 * n_fp64 + tb * n_branch) * args.steps
    step_alg = {"algorithmic_GBps": alg_bytes / total / 1e9,
                "frac": alg_bytes / total / 1e9 / HBM_PEAK_GBPS}

    cpu = None
    parity = None
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle)")
        cpu, parity, parity_of = cpu_baseline(w, solver, args.cpu_seconds, args.workload)
        cpu["sample"] += f"; the GPU result of the same work: relative L2 {parity:.1e} ({parity_of})"
    solver.close()
    # context for the roofline (after the timed region): what plain streams
    # with the passes' read/write mixes reach on this GPU
    streams = stream_references(pk)

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
        "config": {"workload": describe(args.workload, w) + f"; bench step = {slice_desc} "
                               f"({steps_per} RK4 steps)",
                   "values_per_state": S, "rk4_steps_per_step": steps_per,
                   "job_rk4_steps": rk4_steps(w),
                   "job_seconds_projected": rk4_steps(w) * (ms_per_step / 1000.0) / steps_per,
                   "branch_batch": args.batch, "branch_precision": args.precision,
                   "tiles": tiles, "tiles_arg": tiles_arg},
        "roofline": roofline,
        "path_roofline_16pass": step_alg,
        "stream_reference_GBps": streams,
        "cpu_baseline": cpu,
        "spectrum_time_s": rk4_steps(w) * (ms_per_step / 1000.0) / steps_per,
        "parity_rel_l2_vs_oracle": parity,
        "kernel_mean_ms": {k: v[1] for k, v in kt.items() if v[0] > 0},
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
