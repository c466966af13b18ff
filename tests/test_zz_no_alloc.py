"""The allocation-free MRCA entry point (hstrat_mrca_bounds_noalloc, for
callers that cannot allocate device memory) against hstrat_mrca_bounds with
a caller's workspace and against the oracle, through the C ABI: two calls in
a row on the library's shared static scratch, the second with a smaller
input of other counters, so that it must not read what the first left."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hs():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2404_10861_amd as hs
    hs.load_library()
    return hs


def noalloc(hs, kind, S, cnt, srf, stream=None):
    import torch
    n = cnt.shape[0]
    lb = torch.full((n, n), -7, dtype=torch.int32, device=cnt.device)
    ub = torch.full((n, n), -7, dtype=torch.int32, device=cnt.device)
    if stream is None:
        stream = torch.cuda.current_stream()
    vp = ctypes.c_void_p
    rc = hs.load_library().hstrat_mrca_bounds_noalloc(
        kind, S, n, vp(cnt.data_ptr()), vp(srf.data_ptr()), vp(lb.data_ptr()),
        vp(ub.data_ptr()), vp(int(stream.cuda_stream)))
    assert rc == 0, hs.load_library().ga_last_error()
    return lb, ub


def with_workspace(hs, kind, S, cnt, srf):
    ws = hs.MrcaWorkspace(S, cnt.shape[0])
    lb, ub = hs.mrca_bounds(kind, S, cnt, srf, workspace=ws)
    assert hs.mrca_status(ws) == 0
    return lb, ub


def test_two_calls_in_a_row_match_the_workspace_route_and_the_oracle(hs, orc):
    import torch
    # call 1: 2,000 annotations of a hybrid-64 run sharing counter 900
    cfg1 = hs.Config(16, 16, 32, 64, "hybrid", seed=41)
    r1 = hs.Run(cfg1)
    r1.step(900)
    _, c1, s1 = r1.sample(2000)
    # call 2: 300 tilted-32 annotations with mixed counters (the general
    # route, which reads other parts of the scratch)
    rng = np.random.default_rng(5)
    c2h = rng.integers(0, 5000, size=300).astype(np.uint32)
    c2h[:4] = [0, 1, 31, 32]
    s2h = rng.integers(0, 2**32, size=(300, 1), dtype=np.uint64).astype(np.uint32)
    c2 = torch.from_numpy(c2h.view(np.int32)).cuda()
    s2 = torch.from_numpy(s2h.view(np.int32)).cuda()

    lb1, ub1 = noalloc(hs, 2, 64, c1, s1)
    lb2, ub2 = noalloc(hs, 1, 32, c2, s2)
    torch.cuda.synchronize()
    wl1, wu1 = with_workspace(hs, 2, 64, c1, s1)
    wl2, wu2 = with_workspace(hs, 1, 32, c2, s2)
    assert torch.equal(lb1, wl1) and torch.equal(ub1, wu1)
    assert torch.equal(lb2, wl2) and torch.equal(ub2, wu2)
    ol2, ou2 = orc.mrca_allpairs(1, 32, c2h, s2h)
    assert np.array_equal(hs.as_u32(lb2), ol2) and np.array_equal(hs.as_u32(ub2), ou2)
    ch, sh = hs.as_u32(c1), hs.as_u32(s1)
    rows = np.array([0, 1, 999, 1999], np.uint32)
    ol1, ou1 = orc.mrca_rows(2, 64, ch, sh, rows)
    assert np.array_equal(hs.as_u32(lb1)[rows], ol1)
    assert np.array_equal(hs.as_u32(ub1)[rows], ou1)

    # the first shape again, after the smaller call: the same bounds
    lb3, ub3 = noalloc(hs, 2, 64, c1, s1)
    torch.cuda.synchronize()
    assert torch.equal(lb3, wl1) and torch.equal(ub3, wu1)


def test_limits_and_horizon(hs):
    import torch
    lib = hs.load_library()
    vp = ctypes.c_void_p
    dummy = torch.zeros(16, dtype=torch.int32, device="cuda")
    p = vp(dummy.data_ptr())
    assert lib.hstrat_mrca_bounds_noalloc(0, 32, 4097, p, p, p, p, None) == hs.GA_EINVAL
    assert b"4096" in lib.ga_last_error()
    assert lib.hstrat_mrca_bounds_noalloc(0, 48, 4, p, p, p, p, None) == hs.GA_EINVAL
    assert lib.hstrat_mrca_bounds_noalloc(3, 32, 4, p, p, p, p, None) == hs.GA_EINVAL
    assert lib.hstrat_mrca_bounds_noalloc(0, 32, 0, p, p, p, p, None) == hs.GA_EINVAL
    assert lib.hstrat_mrca_bounds_noalloc(0, 32, 4, None, p, p, p, None) == hs.GA_EINVAL
    # a hybrid-32 counter past the horizon (its 16-site tilted half places
    # items up to generation 131,070): every bound reads 0xFFFFFFFF
    cnt = torch.tensor(np.array([5, 200000, 5], np.uint32).view(np.int32), device="cuda")
    srf = torch.zeros((3, 1), dtype=torch.int32, device="cuda")
    lb, ub = noalloc(hs, 2, 32, cnt, srf)
    torch.cuda.synchronize()
    assert np.all(hs.as_u32(lb) == 0xFFFFFFFF) and np.all(hs.as_u32(ub) == 0xFFFFFFFF)
