"""CPU checks of the benchmark's contract: one GPU only, the committed counter record
belongs to the sweep sources as they stand, and the recorded studies parse."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr


def test_traffic_record_matches_the_sweep_sources():
    """profiles/traffic_counters.json was taken on the sweep kernel built from the
    current sources (the bench line reports its traffic only then)."""
    from paper_2606_00641_amd.pmc_traffic import kernel_source_hash
    with open(os.path.join(ROOT, "profiles", "traffic_counters.json")) as fh:
        rec = json.load(fh)
    assert rec["kernel_hash"] == kernel_source_hash()
    r = rec["records"]["resistive_256/f32"]
    assert 0.99 < r["ratio_to_algorithmic"] < 1.1


def test_recorded_studies_parse():
    import bench
    studies = bench.recorded_studies()
    for key in ("precision_slab_512", "learned_coarse_2d", "learned_coarse_3d", "learned_coarse_3d_f16",
                "learned_coarse_3d_bf16"):
        assert key in studies, key
    for key in ("learned_coarse_2d", "learned_coarse_3d"):
        s = studies[key]
        assert s["speedup_vs_fine_fp32"] > 1.0
        err = s["rel_l2_vs_restricted_fine"]
        assert err["learned_coarse"]["m"] < err["plain_coarse"]["m"]
