"""Host-side checks of the benchmark and profile plumbing (no GPU): the
single-GPU refusal, the algorithmic byte count of the paper-scale step, the
committed traffic figure and the rule that makes it stale."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_algorithmic_bytes_of_the_paper_scale_step():
    """A synchronous step stores no counters (every counter is the
    generation number): trait and 64 one-bit sites (12 bytes) read and
    written per agent, one 16-byte migrant entry written and read per
    island."""
    import bench
    from paper_2404_10861_amd import workloads as wl
    agents, islands = 512 * 1024 * 32, 512 * 1024
    want = 2 * agents * 12 + 2 * islands * 16
    assert want == 419_430_400
    assert bench.algorithmic_bytes_per_generation(wl.c2()) == want
    assert want / agents == 25.0          # bytes per agent-replication


def test_record_model_bytes_of_the_paper_scale_step():
    """The same generation priced with a stored counter per record (16-byte
    records) and a 32-byte migrant entry per island."""
    import bench
    from paper_2404_10861_amd import workloads as wl
    agents, islands = 512 * 1024 * 32, 512 * 1024
    want = 2 * agents * 16 + islands * 32
    assert want == 553_648_128
    assert bench.record_model_bytes_per_generation(wl.c2()) == want


def test_traffic_is_reported_only_for_the_profiled_code(monkeypatch):
    import bench
    from paper_2404_10861_amd import profiling
    from paper_2404_10861_amd import workloads as wl
    with open(bench.TRAFFIC_FILE) as f:
        rec = json.load(f)
    # measured traffic within 1 % of the bytes the step must move
    assert abs(rec["bytes_per_launch"] / bench.algorithmic_bytes_per_generation(wl.c2()) - 1) < 0.01
    # reported for the profiled code, null for any other
    monkeypatch.setattr(profiling, "kernel_hash", lambda sources=None: rec["kernel_hash"])
    assert bench.measured_traffic(wl.c2()) == rec["bytes_per_launch"]
    monkeypatch.setattr(profiling, "kernel_hash", lambda sources=None: "0" * 16)
    assert bench.measured_traffic(wl.c2()) is None


def test_valu_is_reported_only_for_the_profiled_code(monkeypatch):
    import bench
    from paper_2404_10861_amd import profiling
    with open(bench.SQ_FILE) as f:
        rec = json.load(f)
    assert 0 < rec["valu_issue_estimate"] < 1.5 and rec["valu_instructions_per_wave"] > 100
    monkeypatch.setattr(profiling, "kernel_hash", lambda sources=None: rec["kernel_hash"])
    v = bench.measured_valu()
    assert v["issue_estimate"] == rec["valu_issue_estimate"]
    monkeypatch.setattr(profiling, "kernel_hash", lambda sources=None: "0" * 16)
    assert bench.measured_valu() is None


def test_code_hash_ignores_comments_and_layout_only(tmp_path):
    from paper_2404_10861_amd import profiling
    texts = {
        "a": "int f(int a) { // one\n  return a + 1; /* two\n three */ }\n",
        "same": "int f(int a) {\n  // another comment\n    return a + 1;\n}\n",
        "other": "int f(int a) { return a + 2; }\n",
    }
    h = {}
    for k, t in texts.items():
        p = tmp_path / f"{k}.hip"
        p.write_text(t)
        h[k] = profiling.kernel_hash([str(p)])
    assert h["a"] == h["same"]
    assert h["a"] != h["other"]


def test_small_run_baseline_compares_final_records():
    """The CPU-scale leg times the whole run on the oracle and reports
    whether the records it is handed equal the oracle's, word for word."""
    import numpy as np
    sys.path.insert(0, os.path.join(ROOT, "oracle"))
    import hsga_oracle as orc
    import bench
    from paper_2404_10861_amd import workloads as wl
    spec = wl.c1()
    spec.generations = 30
    r = orc.Run(spec.grid_w, spec.grid_h, spec.pop_per_island, spec.surface_sites,
                orc.KINDS[spec.surface_kind], spec.tournament_size, spec.mut_threshold,
                spec.mut_lo, spec.mut_hi, spec.migrants_per_island, spec.seed)
    r.step(30)
    final = [np.array(x, copy=True) for x in r.agents()]
    r.close()
    rec = bench.cpu_baseline_small(spec, final)
    assert rec["final_records_equal_gpu"] and rec["cores"] == 1 and rec["value"] > 0
    final[0][17] ^= 1
    assert not bench.cpu_baseline_small(spec, final)["final_records_equal_gpu"]
