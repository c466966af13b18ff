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
    import bench
    from paper_2404_10861_amd import workloads as wl
    spec = wl.c2()
    agents, islands, rec = 512 * 1024 * 32, 512 * 1024, 4 + 4 + 64 // 8
    # every parent record read and every child record written; each island's
    # outbox entry (record + direction word) written once and read once
    want = 2 * agents * rec + 2 * islands * (rec + 4)
    assert want == 557_842_432
    assert bench.algorithmic_bytes_per_generation(spec) == want



def test_design_bytes_of_the_paper_scale_step():
    """A synchronous step keeps no counter plane: trait and 64 one-bit sites
    (12 bytes) read and written per agent, one 16-byte outbox entry written
    and read per island."""
    import bench
    from paper_2404_10861_amd import workloads as wl
    agents, islands = 512 * 1024 * 32, 512 * 1024
    want = 2 * agents * 12 + 2 * islands * 16
    assert want == 419_430_400
    assert bench.design_bytes_per_generation(wl.c2()) == want

def test_traffic_is_reported_only_for_the_profiled_code(monkeypatch):
    import bench
    from paper_2404_10861_amd import profiling
    from paper_2404_10861_amd import workloads as wl
    with open(bench.TRAFFIC_FILE) as f:
        rec = json.load(f)
    # below the algorithmic bytes: no counter plane read, 16-byte outbox entries
    assert rec["bytes_per_launch"] < rec["algorithmic_bytes_per_launch"]
    # reported for the profiled code, null for any other
    monkeypatch.setattr(profiling, "kernel_hash", lambda sources=None: rec["kernel_hash"])
    assert bench.measured_traffic(wl.c2()) == rec["bytes_per_launch"]
    monkeypatch.setattr(profiling, "kernel_hash", lambda sources=None: "0" * 16)
    assert bench.measured_traffic(wl.c2()) is None


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
