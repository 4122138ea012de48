"""Host logic of bench.py that needs no GPU: finding the counter-measured
traffic record of a run's tile choice."""
import json

import bench


def test_committed_traffic_records_are_found_only_for_their_own_runs():
    """Every committed traffic record is used by bench.py exactly for its own
    workload, batch, precision and tile choice while the kernel sources hash
    to its recorded value, and is ignored otherwise."""
    import glob
    import os
    recs = sorted(glob.glob(os.path.join(bench.ROOT, "profiles", "traffic_*.json")))
    for path in recs:
        rec = json.load(open(path))
        current = rec["source_hash"] == bench.source_hash()
        tiles = rec["tiles"] or "1,1,0,1"
        for kind, b in rec["bytes_per_launch"].items():
            got = bench.recorded_traffic(rec["workload"], rec["batch"], rec["precision"], tiles, kind)
            if current:
                assert got is not None
                alg = rec.get("algorithmic_bytes_per_launch", {}).get(kind)
                if alg:  # counters within a few percent of the kernel's own bytes or above
                    assert got / alg > 0.95, (path, kind, got, alg)
            other = bench.recorded_traffic(rec["workload"], rec["batch"] + 1, rec["precision"], tiles, kind)
            assert other is None


def test_stale_or_broken_records_are_ignored(tmp_path):
    rec = {"workload": "w", "batch": 2, "precision": "f64", "tiles": "1,1,0,1",
           "source_hash": bench.source_hash(), "bytes_per_launch": {"k": 123.0}}
    (tmp_path / "traffic_w.json").write_text(json.dumps({**rec, "source_hash": "0"}))
    (tmp_path / "traffic_w_tiles_x.json").write_text("{not json")
    assert bench.recorded_traffic("w", 2, "f64", "1,1,0,1", "k", prof=str(tmp_path)) is None
    (tmp_path / "traffic_w_tiles_1_1_0_1.json").write_text(json.dumps(rec))
    assert bench.recorded_traffic("w", 2, "f64", "1,1,0,1", "k", prof=str(tmp_path)) == 123.0
    assert bench.recorded_traffic("w", 2, "f64", "1,1,0,1", "other", prof=str(tmp_path)) is None


def test_source_hash_follows_code_not_comments():
    base = {rel: open(f"{bench.ROOT}/{rel}", encoding="utf-8").read() for rel in bench.KERNEL_SOURCES}
    h0 = bench.source_hash(lambda rel: base[rel])
    assert h0 == bench.source_hash()
    rel = bench.KERNEL_SOURCES[0]
    commented = dict(base)
    commented[rel] = "// a new comment\n/* and a block\n   comment */\n" + base[rel].replace("\n", "  // note\n", 3)
    assert bench.source_hash(lambda r: commented[r]) == h0
    changed = dict(base)
    changed[rel] = base[rel] + "\nconstexpr int kProbe = 1;\n"
    assert bench.source_hash(lambda r: changed[r]) != h0
