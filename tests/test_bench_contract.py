"""Host-side checks of the benchmark's contract (no GPU): more than one GPU
is refused with a message; the roofline traffic record is keyed to the
stage kernels' sources and holds one value per launch-order candidate; the per-launch byte table covers every stage; the fused kernels are booked as one kernel each."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_traffic_records_are_used_only_for_their_kernel_sources():
    # a committed counter record holds one value per launch-order candidate
    # and is used only while it was taken on the current kernel code
    import glob

    import bench
    paths = glob.glob(os.path.join(ROOT, "profiles", "traffic_*.json"))
    assert paths
    for path in paths:
        rec = json.load(open(path))
        assert len(rec["bytes_per_launch_by_candidate"]) == 16
        current = rec["sources_sha256"] == bench.kernel_source_hash()
        for c in range(16):
            t = bench.measured_traffic(rec["kernel"], rec["form"], c, rec.get("workload"))
            if current:
                assert t == rec["bytes_per_launch_by_candidate"][c] and t > 0
            else:
                assert t is None
    assert bench.measured_traffic("riem1", "fp64", 0) is None


def test_bytes_per_launch_for_every_stage():
    import bench
    for st in ("prim", "flat", "trace", "riem0", "riem1", "riem2", "update"):
        assert bench.bytes_per_launch(st, 256, 4) > 0
        assert bench.bytes_per_launch(st, 256, 8) > bench.bytes_per_launch(st, 256, 4)


def test_source_hash_ignores_comments_and_layout():
    import bench
    a = "int f(int x) {  // one\n  return x + 1; /* two\n lines */ }\n"
    b = "int f(int x) {\n/* other */ return x + 1; }"
    assert bench._code_tokens(a) == bench._code_tokens(b) == "int f(int x) { return x + 1; }"
    assert bench._code_tokens("a - b") != bench._code_tokens("a + b")


def test_fused_stage_accounting():
    # a fused launch is reported as its first stage by the library's events
    # (the second stage's interval empty); the benchmark books it as one
    # kernel, "front" (trace + riem0) or "final" (riem2 + update), with both
    # stages' algorithmic flops together
    import bench
    table = bench.flop_table("box512_stress")
    shapes = [(64, 64, 64)] * 2
    stage_ms = {"prim": 1.0, "flat": 1.0, "trace": 2.0, "riem0": 3.0, "riem1": 6.0,
                "riem2": 4.5, "update": 0.001}
    assert bench.kernel_stages(True) == ("prim", "flat", "front", "riem1", "final")
    assert bench.kernel_ms(stage_ms, "final") == 4.501
    assert bench.kernel_ms(stage_ms, "front") == 5.0
    assert bench.kernel_flops(table, "front", shapes, 3.4) == (
        bench.stage_flops(table, "trace", shapes, 3.4) + bench.stage_flops(table, "riem0", shapes, 3.4))
    fl = bench.kernel_flops(table, "final", shapes, 3.4)
    assert fl == (bench.stage_flops(table, "riem2", shapes, 3.4) +
                  bench.stage_flops(table, "update", shapes, 3.4)) and fl > 0
    rates = bench.stage_rates(stage_ms, table, shapes, 3.4, fused=True)
    assert set(rates) == set(bench.FUSED_STAGES)
    roof, _ = bench.roofline_of(stage_ms, table, shapes, 3.4, 20.0, 4, "mixed",
                                "box512_stress_patches", fused=True)
    assert roof["kernel"] == "riem1" and roof["bound"] == "alu"
    stage_ms["riem2"] = 9.0
    roof, _ = bench.roofline_of(stage_ms, table, shapes, 3.4, 20.0, 4, "mixed",
                                "box512_stress_patches", fused=True)
    assert roof["kernel"] == "final" and roof["traffic"] is None
    assert abs(roof["ms_per_launch"] - 9.001) < 1e-9
    stage_ms["riem0"] = 8.0
    roof, _ = bench.roofline_of(stage_ms, table, shapes, 3.4, 20.0, 4, "mixed",
                                "box512_stress_patches", fused=True)
    assert roof["kernel"] == "front" and roof["bound"] == "alu" and roof["traffic"] is None
