"""Host logic of bench.py that needs no GPU: finding the counter-measured
traffic record of a run's tile choice."""
import json

import bench


def test_committed_traffic_records_match_their_tile_choices():
    # the committed records were taken with the current kernel sources
    main = bench.recorded_traffic("two_mode_32", 64, "f64", "1,1,0,32", "batch_pblock_rhs")
    r8 = bench.recorded_traffic("two_mode_32", 64, "f64", "1,1,0,8", "batch_pblock_rhs")
    r16 = bench.recorded_traffic("two_mode_32", 64, "f64", "1,1,0,16", "batch_pblock_rhs")
    alg = 2 * 64 * 10 * 32 ** 4 * 8          # read X, write t: 64 states of 10 x 32^4 FP64 values
    for t in (main, r8, r16):
        assert t is not None and abs(t / alg - 1) < 0.01
    assert bench.recorded_traffic("two_mode_32", 64, "f64", "1,1,0,4", "batch_pblock_rhs") is None
    assert bench.recorded_traffic("two_mode_32", 32, "f64", "1,1,0,32", "batch_pblock_rhs") is None
    assert bench.recorded_traffic("two_mode_32", 64, "f32", "1,1,0,32", "batch_pblock_rhs") is None


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
