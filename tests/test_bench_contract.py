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


def _counter_csv(path, counter, rows):
    """A counter file in rocprofv3's layout: (kernel name, KiB) per dispatch."""
    import csv
    with open(path, "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(["Correlation_Id", "Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        for j, (name, kib) in enumerate(rows):
            w.writerow([j + 1, j + 1, name, counter, kib])


def test_traffic_tool_selects_the_kernel_forms(tmp_path):
    """pmc_traffic scales each counter by what it reads for the copy kernel of known
    size (FETCH counts half the copy's 4 GiB here, WRITE all of it) and averages the
    parities of the kernel form asked for -- the one-cell sweep, the plain two-cell
    sweep, or its body form, which stores nothing for the body's box -- ignoring the
    other forms in the same run."""
    from paper_2606_00641_amd import pmc_traffic as P
    ns = "void vlbm::(anonymous namespace)::"
    args = "(vlbm::Grid, vlbm::Phys, vlbm::Codec, vlbm::Body, vlbm::Inflow)"
    copy = (ns + "k_copy(HIP_vector_type<unsigned int, 4u>*, HIP_vector_type<unsigned int, 4u> const*, unsigned long)")
    kib = lambda b: b / 1024.0
    rows_f = [(copy, kib(2 << 30)),
              (ns + "k_sweep2<2, 3, 0, 0, 0, false, false>" + args, kib(500)),
              (ns + "k_sweep2<2, 3, 0, 1, 0, false, false>" + args, kib(700)),
              (ns + "k_sweep2<2, 3, 0, 0, 0, true, true>" + args, kib(1000)),
              (ns + "k_sweep2<2, 3, 0, 1, 0, true, true>" + args, kib(1200)),
              (ns + "k_sweep2<2, 3, 0, 1, 1, true, true>" + args, kib(9999)),  # two-rate: not selected
              (ns + "k_sweep<1, 3, 1, 0, 0, 0, false, false, false, 0>(vlbm::Grid)", kib(300)),
              (ns + "k_sweep<1, 3, 1, 1, 0, 0, false, false, false, 0>(vlbm::Grid)", kib(500))]
    rows_w = [(copy, kib(4 << 30))] + [(n, v / 2) for n, v in rows_f[1:]]
    fetch, write = tmp_path / "f.csv", tmp_path / "w.csv"
    _counter_csv(fetch, "FETCH_SIZE", rows_f)
    _counter_csv(write, "WRITE_SIZE", rows_w)
    out = tmp_path / "t.json"

    def run(*extra):
        r = subprocess.run([sys.executable, "-m", "paper_2606_00641_amd.pmc_traffic", "--fetch", str(fetch),
                            "--write", str(write), "--out", str(out), *extra], capture_output=True, text=True,
                           cwd=ROOT, timeout=120)
        assert r.returncode == 0, r.stderr
        return json.load(open(out))

    t = run("--key", "a", "--cells", "10", "--bytes-per-cell", "100")  # one-cell resistive sweep
    rec = t["records"]["a"]
    assert rec["fetch_bytes_per_launch"] == 2 * 400 and rec["write_bytes_per_launch"] == 200
    assert rec["algorithmic_bytes_per_launch"] == 1000 and rec["ratio_to_algorithmic"] == 1.0
    t = run("--key", "b", "--kernel", "pair", "--storage", "2", "--model", "0", "--cells", "10",
            "--bytes-per-cell", "180")
    rec = t["records"]["b"]
    assert rec["fetch_bytes_per_launch"] == 2 * 600 and rec["write_bytes_per_launch"] == 300
    t = run("--key", "c", "--kernel", "pair_body", "--storage", "2", "--model", "0", "--cells", "20",
            "--store-cells", "16", "--bytes-per-cell", "100")
    rec = t["records"]["c"]
    assert rec["fetch_bytes_per_launch"] == 2 * 1100 and rec["write_bytes_per_launch"] == 550
    assert rec["algorithmic_bytes_per_launch"] == (20 + 16) * 50 and rec["cells_stored"] == 16
