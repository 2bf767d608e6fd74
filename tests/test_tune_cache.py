"""The committed launch-shape cache and the committed traffic record of the
headline kernel (CPU only: no kernel runs).

bench.py reports `roofline.traffic` from profiles/traffic_fused_swe16384_f32.json
only while the fused kernel's sources hash to the value stored there and the
headline's tuned shape is the one the counters were taken with; these tests
fail when either drifts (a kernel edit or a re-tune without re-profiling),
instead of the bench line quietly reporting null."""
import importlib.util
import json
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CACHE = os.path.join(ROOT, "paper_1107_2157_amd", "tune_cache_gfx950.txt")
TRAFFIC = os.path.join(ROOT, "profiles", "traffic_fused_swe16384_f32.json")
FIELDS = ("variant", "rows", "vec", "occupancy", "prefetch", "order")
KEY = re.compile(r"^gfx950:\d+:(f32|f64):[01]:(\d+x\d+(:fixeddt)?|batch\d+:\d+)$")


def bench_module():
    spec = importlib.util.spec_from_file_location("bench_for_tests", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def entries():
    out = {}
    for line in open(CACHE).read().splitlines():
        if not line.strip():
            continue
        parts = line.split()
        assert len(parts) == 8, line
        assert KEY.match(parts[0]), line
        shape = dict(zip(FIELDS, (int(v) for v in parts[1:7])))
        assert float(parts[7]) > 0, line
        assert parts[0] not in out, f"duplicate key {parts[0]}"
        out[parts[0]] = shape
    return out


def test_cache_lines_are_well_formed():
    for key, t in entries().items():
        if ":batch" in key:
            assert t["variant"] == 2 and t["order"] in (0, 1, 2), key
        elif key.endswith(":fixeddt"):
            assert t["variant"] in (2, 3), key
        else:
            assert t["variant"] == 2, key           # CFL runs: the fused kernel
        if t["variant"] == 2:
            assert t["rows"] >= 1 and t["prefetch"] in (1, 2, 3) and t["occupancy"] in (0, 3, 4), key
            assert t["vec"] in ((1, 2) if ":f64:" in key else (1, 2, 4)), key


def test_headline_traffic_record_matches_sources_and_shape():
    rec = json.load(open(TRAFFIC))
    bench = bench_module()
    assert rec["source_sha256_16"] == bench.source_hash(bench.FUSED_SRC)
    assert rec["tuning"] == entries()["gfx950:256:f32:0:16384x16384"]
    alg = 16384 * 16384 * 24
    assert 1.0 <= rec["bytes_per_launch"] / alg < 1.05
    assert abs(rec["read_bytes"] + rec["write_bytes"] - rec["bytes_per_launch"]) < 1.0
