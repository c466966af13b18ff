"""GPU parity of trie reconstruction and phylometrics against the oracle
(zero tolerance on the integer results): samples of evolved runs of every
surface kind, ragged and tiny sample sizes, identical annotations, and the
refused cases (counters that differ, past the horizon)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

KIND = {"steady": 0, "tilted": 1, "hybrid": 2}


@pytest.fixture(scope="module")
def hs():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2404_10861_amd as hs
    hs.load_library()
    return hs


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, np.uint32).view(np.int32)).cuda()


def check(hs, orc, kind, S, counters, surf):
    got = hs.phylo_metrics(kind, S, dev(counters), dev(surf))
    assert got["status"] == 0 and got["n"] == len(counters)
    sbl, pairs, root, internal, ed = orc.phylo_metrics(kind, S, counters, surf)
    assert (got["sum_branch_length"], got["pair_sum"], got["root_time"],
            got["internal_nodes"]) == (sbl, pairs, root, internal)
    assert got["mean_ed"] == pytest.approx(ed.mean(), rel=1e-12)
    return got


@pytest.mark.parametrize("kind", ["steady", "tilted", "hybrid"])
@pytest.mark.parametrize("S", [32, 64])
@pytest.mark.parametrize("tournament", [0, 2])
def test_evolved_samples(hs, orc, kind, S, tournament):
    cfg = hs.Config(16, 16, 32, S, kind, tournament_size=tournament, seed=11 + S)
    run = hs.Run(cfg)
    run.step(900)
    _, cnt, srf = run.sample(2000)
    check(hs, orc, KIND[kind], S, hs.as_u32(cnt), hs.as_u32(srf))


@pytest.mark.parametrize("n", [1, 2, 3, 5, 63, 64, 65, 257, 1000, 1025])
def test_ragged_with_identical(hs, orc, n):
    rng = np.random.default_rng(100 + n)
    counters = np.full(n, 4000, np.uint32)
    surf = rng.integers(0, 2**32, size=(n, 2), dtype=np.uint64).astype(np.uint32)
    surf[: n // 3] = surf[0]                       # a polytomy
    surf[n // 3: n // 2, 0] = surf[0, 0]           # shares a long prefix with it
    check(hs, orc, KIND["hybrid"], 64, counters, surf)


@pytest.mark.parametrize("T", [0, 1, 7, 31, 32, 33])
def test_fill_phase_and_founders(hs, orc, T):
    rng = np.random.default_rng(T)
    counters = np.full(40, T, np.uint32)
    surf = rng.integers(0, 2**32, size=(40, 1), dtype=np.uint64).astype(np.uint32)
    check(hs, orc, KIND["tilted"], 32, counters, surf)


def test_all_identical(hs, orc):
    counters = np.full(50, 1234, np.uint32)
    surf = np.full((50, 2), 0xdeadbeef, np.uint32)
    got = check(hs, orc, KIND["steady"], 64, counters, surf)
    assert got["internal_nodes"] == 1 and got["root_time"] == 1234
    assert got["sum_branch_length"] == 0 and got["pair_sum"] == 0


def test_full_sample_of_a_large_run(hs, orc):
    """65,535 annotations (the largest query) of a 64x64-island hybrid run."""
    cfg = hs.Config(64, 64, 32, 64, "hybrid", tournament_size=2, seed=77)
    run = hs.Run(cfg)
    run.step(3000)
    _, cnt, srf = run.sample(65535)
    check(hs, orc, KIND["hybrid"], 64, hs.as_u32(cnt), hs.as_u32(srf))


def test_refused(hs, orc):
    got = hs.phylo_metrics(0, 32, dev(np.array([7, 8, 7], np.uint32)),
                           dev(np.zeros((3, 1), np.uint32)))
    assert got["status"] == 1 and got["sum_branch_length"] == 0
    past = 2 * (2**16 - 2) + 4
    got = hs.phylo_metrics(2, 32, dev(np.full(4, past, np.uint32)),
                           dev(np.zeros((4, 1), np.uint32)))
    assert got["status"] == 2
    with pytest.raises(ValueError):                 # the oracle refuses it too
        orc.phylo_metrics(2, 32, np.full(4, past, np.uint32), np.zeros((4, 1), np.uint32))
    orc.phylo_metrics(2, 32, np.full(4, past - 1, np.uint32), np.zeros((4, 1), np.uint32))
    with pytest.raises(hs.HsgaError):
        hs.phylo_metrics(0, 48, dev(np.zeros(2, np.uint32)), dev(np.zeros((2, 1), np.uint32)))


def test_selection_shortens_the_tree(hs):
    """Sweeps make common ancestry recent: at equal T the selected run's
    tree has a shorter sum of branch lengths and a later root."""
    res = {}
    for tour in (0, 2):
        run = hs.Run(hs.Config(32, 32, 32, 64, "hybrid", tournament_size=tour, seed=5))
        run.step(2000)
        _, cnt, srf = run.sample(4096)
        res[tour] = hs.phylo_metrics("hybrid", 64, cnt, srf)
    assert res[2]["sum_branch_length"] < res[0]["sum_branch_length"]
    assert res[2]["mean_pairwise_distance"] < res[0]["mean_pairwise_distance"]


# --------------------------------------------------------------------------
# The reconstructed tree itself: canonical Newick text from the device's
# node and leaf parents equals the oracle's, character for character.

@pytest.mark.parametrize("kind,S,bits,interval", [("steady", 32, 1, 1), ("tilted", 64, 1, 1),
                                                  ("hybrid", 64, 1, 3), ("steady", 8, 8, 1),
                                                  ("tilted", 8, 8, 2)])
def test_tree_newick_matches_oracle(hs, orc, kind, S, bits, interval):
    cfg = hs.Config(16, 16, 32, S, kind, tournament_size=0, seed=19, differentia_bits=bits,
                    ingest_interval=interval)
    G = min(800, orc.horizon_gen(KIND[kind], S, interval) + 1)
    run = hs.Run(cfg)
    run.step(G)
    _, cnt, srf = run.sample(1500)
    tree = hs.phylo_tree(kind, S, cnt, srf, bits=bits, interval=interval)
    assert tree["status"] == 0
    want = orc.phylo_newick(KIND[kind], S, hs.as_u32(cnt), hs.as_u32(srf), bits=bits,
                            interval=interval)
    assert hs.newick(tree) == want
    nodes = tree["node_parent"] != hs.binding.PHYLO_NOT_NODE
    assert int(nodes.sum()) == tree["internal_nodes"]
    assert int((tree["node_parent"] == hs.binding.PHYLO_ROOT).sum()) == 1


@pytest.mark.parametrize("n", [1, 2, 3, 64, 65, 257, 1025])
def test_tree_ragged_many_way_and_polytomies(hs, orc, n):
    rng = np.random.default_rng(7 * n)
    counters = np.full(n, 8, np.uint32)
    vals = rng.integers(0, 3, size=(n, 8)).astype(np.uint32)
    vals[: n // 4] = vals[0]
    words = np.zeros((n, 2), np.uint32)
    for k in range(8):
        words[:, k // 4] |= vals[:, k] << (8 * (k % 4))
    tree = hs.phylo_tree("steady", 8, dev(counters), dev(words), bits=8)
    assert hs.newick(tree) == orc.phylo_newick(0, 8, counters, words, bits=8)


def test_tree_of_a_large_sample(hs, orc):
    cfg = hs.Config(64, 64, 32, 64, "hybrid", tournament_size=2, seed=77)
    run = hs.Run(cfg)
    run.step(3000)
    _, cnt, srf = run.sample(65535)
    tree = hs.phylo_tree("hybrid", 64, cnt, srf)
    assert hs.newick(tree) == orc.phylo_newick(2, 64, hs.as_u32(cnt), hs.as_u32(srf))
