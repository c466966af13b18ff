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
    # 12 uint32/int32 fields then a uint64 seed: 56 bytes, seed at offset 48
    assert ctypes.sizeof(b.ga_config) == 56
    assert b.ga_config.seed.offset == 48


def test_footprint_without_gpu():
    if not os.path.exists(LIB):
        pytest.skip("libhsga.so not built")
    import paper_2404_10861_amd as hs
    cfg = hs.Config(512, 1024, 32, 64, "hybrid")
    n = hs.footprint_bytes(cfg)
    # two populations of 16 B records plus outboxes, layout and schedule
    assert n >= 2 * cfg.agents * 16 + 2 * cfg.islands * 32
    assert n < 2 * cfg.agents * 16 + 2 * cfg.islands * 32 + (1 << 20)
    with pytest.raises(hs.HsgaError):
        hs.footprint_bytes(hs.Config(0, 4))
