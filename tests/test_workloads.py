"""The seeded workload generators produce the configured run sets."""
import numpy as np

from paper_2404_10861_amd import workloads as wl


def test_plain_workloads():
    assert wl.c1().agents == 2048 and wl.c1().generations == 1000
    assert wl.c2().agents == 16777216 and wl.c2().surface_kind == "hybrid"
    assert wl.c2().surface_sites == 64
    a, b = wl.c3(True), wl.c3(False)
    assert a.agents == 4194304 and a.tournament_size == 2 and b.tournament_size == 0
    assert a.seed == b.seed == 1 and a.sample == 4096


def test_batched_run_set():
    runs = wl.c4()
    assert len(runs) == 64
    assert [r.seed for r in runs] == list(range(1, 65))
    assert sum(r.tournament_size == 2 for r in runs) == 32
    assert all(r.generations == 5000 for r in runs)
    assert {(r.grid_w, r.grid_h) for r in runs} <= set(wl.C4_GRIDS)
    assert {r.pop_per_island for r in runs} <= {16, 32, 64}
    assert len({r.surface_kind for r in runs}) == 3
    assert wl.c4() == runs                          # seeded: reproducible


def test_served_request_list():
    reqs = wl.c5()
    n = len(reqs)
    assert 2000 < n < 2800                          # about 20/s over 120 s
    arrivals = np.array([r.arrival for r in reqs])
    assert np.all(np.diff(arrivals) > 0) and arrivals[-1] < 120
    assert wl.log_uniform_check([r.grid_w for r in reqs], 8, 256)
    assert wl.log_uniform_check([r.grid_h for r in reqs], 8, 512)
    assert wl.log_uniform_check([r.generations for r in reqs], 1000, 20000)
    assert all(r.pop_per_island == 32 and r.sample == 1024 for r in reqs)
    assert [r.seed for r in reqs] == list(range(1, n + 1))
    # log-uniform generations: median near 1000 * sqrt(20)
    med = np.median([r.generations for r in reqs])
    assert 3500 < med < 5500


def test_saved_lists_are_the_generated_ones():
    """The committed run lists are the workloads; they were written from
    the seeded generators, which still reproduce them."""
    assert wl.c4_saved() == wl.c4()
    saved, drawn = wl.c5_saved(), wl.c5()
    assert len(saved) == len(drawn) == 2398
    for x, y in zip(saved, drawn):
        assert abs(x.arrival - y.arrival) < 1e-8
        assert (x.grid_w, x.grid_h, x.generations, x.surface_kind, x.surface_sites, x.seed) == \
            (y.grid_w, y.grid_h, y.generations, y.surface_kind, y.surface_sites, y.seed)
    assert len(wl.c5_saved(20.0)) == sum(r.arrival < 20.0 for r in drawn)
