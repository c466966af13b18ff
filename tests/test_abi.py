"""The C-ABI library loads and exports every entry point include/hsga.h
declares, and the Python binding names the same set.  No compute call is
made, so this runs without a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hsga.h")
LIB = os.path.join(ROOT, "paper_2404_10861_amd", "libhsga.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    names = re.findall(r"^[A-Za-z_][\w\s\*]*?\b((?:ga|hstrat)_\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("ga_create", "ga_step", "ga_read_agents", "hstrat_mrca_bounds"):
        assert required in names
    assert len(names) >= 15


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        pytest.skip("libhsga.so not built")
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_names_match_header():
    import paper_2404_10861_amd.binding as b
    assert sorted(b.EXPORTS) == declared_functions()


def test_config_struct_layout():
    import paper_2404_10861_amd.binding as b
    # 12 uint32/int32 fields, a uint64 seed, the six float-treatment and
    # scheme words, the asynchronous activity and a reserved word: 88 bytes
    assert ctypes.sizeof(b.ga_config) == 88
    assert b.ga_config.async_activity.offset == 80
    assert b.ga_config.seed.offset == 48
    assert b.ga_config.fitness_model.offset == 56
    assert b.ga_config.del_sigma.offset == 68 and b.ga_config.differentia_bits.offset == 76
    assert b.ga_config.ingest_interval.offset == 44
    assert ctypes.sizeof(b.hstrat_scheme) == 16


def test_footprint_without_gpu():
    if not os.path.exists(LIB):
        pytest.skip("libhsga.so not built")
    import paper_2404_10861_amd as hs
    cfg = hs.Config(512, 1024, 32, 64, "hybrid")
    n = hs.footprint_bytes(cfg)
    # a synchronous run: two populations of trait and surface words (no
    # counter plane: every counter is the generation count), plus outboxes,
    # layout, the site rule's two constant-time tables (about 25 KB each)
    # and the schedule of a launch batch (4 bytes per generation)
    base = 2 * cfg.agents * 12 + 2 * cfg.islands * 32
    assert base + 40 * 1024 + 4096 * 4 < n < base + (1 << 20)
    assert hs.footprint_bytes(cfg, 8192) - n == 4096 * 4
    # an asynchronous run keeps its counter planes as well, and a ring of
    # 4,096 sites in place of the 4,096-generation schedule
    acfg = hs.Config(512, 1024, 32, 64, "hybrid", async_activity=1 << 31)
    assert hs.footprint_bytes(acfg) - (n + 2 * cfg.agents * 4) == 0
    # and no tick bound: the same bytes whatever the launch batch
    assert hs.footprint_bytes(acfg, 16) == hs.footprint_bytes(acfg, 1 << 20)
    with pytest.raises(hs.HsgaError):
        hs.footprint_bytes(hs.Config(0, 4))


def test_config_versions_and_float_validation_without_gpu():
    """Host-side validation: a 56-byte config (no float fields) is read as
    the integer model; float-treatment fields are range-checked."""
    if not os.path.exists(LIB):
        pytest.skip("libhsga.so not built")
    import paper_2404_10861_amd as hs
    import paper_2404_10861_amd.binding as b
    lib = b.load_library()
    base = hs.Config(8, 8, 32, 32, "tilted")
    c = base.to_c()
    full = lib.ga_footprint_bytes(ctypes.byref(c), 0)
    assert full > 0
    c.struct_size = 56
    c.fitness_model = 7            # beyond a 56-byte config: never read
    assert lib.ga_footprint_bytes(ctypes.byref(c), 0) == full
    c.struct_size = 80
    c.fitness_model = 0
    c.async_activity = 9           # beyond an 80-byte config: never read
    assert lib.ga_footprint_bytes(ctypes.byref(c), 0) == full
    c.struct_size = 60
    assert lib.ga_footprint_bytes(ctypes.byref(c), 0) == 0
    good = dict(fitness_model="float", tournament_size=5, del_threshold=1417339207,
                ben_threshold=12884901, del_sigma=1.0, ben_sigma=1.0)
    assert hs.footprint_bytes(hs.Config(8, 8, 32, 32, "tilted", **good)) == full
    for bad in (dict(tournament_size=6), dict(del_threshold=2**31, ben_threshold=2**31 + 1),
                dict(del_sigma=float("nan")), dict(ben_sigma=-0.5), dict(del_sigma=2.0**21)):
        kw = dict(good)
        kw.update(bad)
        with pytest.raises(hs.HsgaError):
            hs.footprint_bytes(hs.Config(8, 8, 32, 32, "tilted", **kw))
    with pytest.raises(hs.HsgaError):
        hs.footprint_bytes(hs.Config(8, 8, 32, 32, "tilted", tournament_size=5))


def test_checkpoint_and_run_query_arguments_without_gpu():
    """Host-side argument checks of the checkpoint and run-bound query entry
    points: a NULL run is refused before any device work."""
    if not os.path.exists(LIB):
        pytest.skip("libhsga.so not built")
    import paper_2404_10861_amd.binding as b
    lib = b.load_library()
    assert lib.ga_state_bytes(None) == 0
    assert lib.ga_export_state(None, None, 0) == b.GA_EINVAL
    assert lib.ga_import_state(None, None, 0) == b.GA_EINVAL
    assert lib.ga_mrca_bounds(None, 1, None, None, None, None, None, 0) == b.GA_EINVAL
    assert b"run is NULL" in lib.ga_last_error()
    assert lib.ga_phylo_tree(None, 1, None, None, None, None, None, None, None, 0) == b.GA_EINVAL


def test_launch_form_arguments_without_gpu():
    """The resident-form and pool-split settings refuse NULL handles."""
    if not os.path.exists(LIB):
        pytest.skip("libhsga.so not built")
    import ctypes
    import paper_2404_10861_amd.binding as b
    lib = b.load_library()
    assert lib.ga_set_resident(None, 1) == b.GA_EINVAL
    t = ctypes.c_uint32(7)
    assert lib.ga_resident_threads(None, ctypes.byref(t)) == b.GA_EINVAL
    assert lib.ga_pool_set_split(None, 0) == b.GA_EINVAL
    assert b"pool is NULL" in lib.ga_last_error()


def test_missing_library_fails_loudly():
    """No CPU fallback: without the built library every entry point of the
    binding refuses to run."""
    import subprocess
    import sys
    code = (
        "import paper_2404_10861_amd.binding as b\n"
        "b.LIB_PATH = '/nonexistent/libhsga.so'\n"
        "b._lib = None\n"
        "import paper_2404_10861_amd as hs\n"
        "try:\n"
        "    hs.footprint_bytes(hs.Config(8, 8, 32, 32, 'steady'))\n"
        "except RuntimeError as e:\n"
        "    print('refused:', e)\n"
        "else:\n"
        "    print('ran')\n")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, cwd=ROOT,
                       timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    assert "refused: HIP library not built" in r.stdout
