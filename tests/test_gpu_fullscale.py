"""Full-size GPU parity over many generations (opt-in: set
HSGA_FULL_PARITY=1; the oracle needs minutes of host time): the
paper-scale workload (512x1024 islands x 32, hybrid-64, tournament of two)
for 300 generations and the treatment pair's torus (256x256 x 64,
tilted-32) for 2,000 generations of each treatment, every agent word, the
layout and every outbox entry against the oracle, in the launch
configuration the benchmark uses."""
import os
import sys
import time

import numpy as np
import pytest

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(os.environ.get("HSGA_FULL_PARITY") != "1",
                                 reason="opt-in: HSGA_FULL_PARITY=1")]


@pytest.fixture(scope="module")
def hs():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2404_10861_amd as hs
    hs.load_library()
    return hs


def oracle_steps(o, G, label):
    """Step the oracle G generations, printing progress now and then."""
    t0 = time.perf_counter()
    done = 0
    while done < G:
        k = min(50, G - done)
        o.step(k)
        done += k
        print(f"{label}: oracle at generation {done} ({time.perf_counter() - t0:.0f} s)",
              file=sys.stderr, flush=True)


@pytest.mark.parametrize("W,H,N,S,kind,tour,G", [
    (512, 1024, 32, 64, "hybrid", 2, 300),
    (256, 256, 64, 32, "tilted", 2, 2000),
    (256, 256, 64, 32, "tilted", 0, 2000),
])
def test_full_size_runs_match_oracle(hs, orc, W, H, N, S, kind, tour, G):
    kinds = {"steady": 0, "tilted": 1, "hybrid": 2}
    cfg = hs.Config(W, H, N, S, kind, tournament_size=tour, seed=1)
    run = hs.Run(cfg)
    run.step(G)
    run.sync()
    o = orc.Run(W, H, N, S, kinds[kind], tournament=tour, seed=1)
    oracle_steps(o, G, f"{W}x{H}x{N} {kind}-{S} tournament {tour}")
    for name, x, y in zip(("trait", "counter", "surface"), run.agents(), o.agents()):
        assert np.array_equal(x, y), name
    assert np.array_equal(run.layout(), o.layout())
    for x, y in zip(run.outbox(), o.outbox()):
        assert np.array_equal(x, y)
    o.close()
