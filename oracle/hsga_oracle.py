"""ctypes front end of the plain CPU oracle (``hsga_oracle.c``).

TEST INFRASTRUCTURE ONLY.  The test suite, the smoke check and the
CPU-baseline leg of the benchmark are the only callers.  The product library
never imports this module, and this module imports nothing from the product
package.

``build()`` compiles the oracle with gcc into ``liboracle.so`` next to this
file; ``load()`` loads the built library and fails loudly if it is missing.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "hsga_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

EMPTY = 0xFFFFFFFF
STEADY, TILTED, HYBRID = 0, 1, 2
KINDS = {"steady": STEADY, "tilted": TILTED, "hybrid": HYBRID}
BIRTH, EMIGRATE, IMMIGRATE, SAMPLE, BIRTH_B, FOUNDER, ACTIVITY = 0, 1, 2, 3, 4, 5, 6
INT_TRAIT, FLOAT_FITNESS, FOUNDER_TAG = 0, 1, 2

_lib = None

u32p = ctypes.POINTER(ctypes.c_uint32)
i32p = ctypes.POINTER(ctypes.c_int32)
u8p = ctypes.POINTER(ctypes.c_uint8)


def build() -> str:
    """Compile the oracle (plain C, -O2, scalar) into liboracle.so."""
    cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-pthread", "-Wall", "-Wextra", "-shared",
           "-fPIC", "-o", LIB + ".tmp", SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB):
        raise RuntimeError(f"oracle library not built: {LIB} (run build())")
    lib = ctypes.CDLL(LIB)
    lib.orc_philox.argtypes = [ctypes.c_uint32] * 4 + [ctypes.c_uint64, u32p]
    lib.orc_philox.restype = None
    lib.orc_mulhi.argtypes = [ctypes.c_uint32, ctypes.c_uint32]
    lib.orc_mulhi.restype = ctypes.c_uint32
    lib.orc_in_D.argtypes = [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint64,
                             ctypes.c_uint64]
    lib.orc_in_D.restype = ctypes.c_int
    lib.orc_horizon.argtypes = [ctypes.c_uint32, ctypes.c_uint32]
    lib.orc_horizon.restype = ctypes.c_uint64
    lib.orc_place.argtypes = [ctypes.c_uint32, ctypes.c_uint32, u32p,
                              ctypes.c_uint32]
    lib.orc_place.restype = ctypes.c_int
    lib.orc_layout.argtypes = [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
                               u32p]
    lib.orc_layout.restype = ctypes.c_int
    lib.orc_site_sequence.argtypes = [ctypes.c_uint32, ctypes.c_uint32,
                                      ctypes.c_uint32, ctypes.c_uint32, i32p]
    lib.orc_site_sequence.restype = ctypes.c_int
    lib.orc_create.argtypes = ([ctypes.c_uint32] * 7 + [ctypes.c_int32] * 2 +
                               [ctypes.c_uint32, ctypes.c_uint64,
                                ctypes.c_uint32])
    lib.orc_create.restype = ctypes.c_void_p
    lib.orc_create_ex.argtypes = ([ctypes.c_uint32] * 7 + [ctypes.c_int32] * 2 +
                                  [ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint32,
                                   ctypes.c_uint32, ctypes.c_uint32])
    lib.orc_create_ex.restype = ctypes.c_void_p
    lib.orc_set_async.argtypes = [ctypes.c_void_p, ctypes.c_uint32]
    lib.orc_set_async.restype = ctypes.c_int
    lib.orc_set_threads.argtypes = [ctypes.c_void_p, ctypes.c_uint32]
    lib.orc_set_threads.restype = ctypes.c_int
    lib.orc_horizon_gen.argtypes = [ctypes.c_uint32] * 3
    lib.orc_horizon_gen.restype = ctypes.c_uint64
    lib.orc_mrca_rows_x.argtypes = ([ctypes.c_uint32] * 5 + [u32p, u32p, ctypes.c_uint32, u32p,
                                                             u32p, u32p])
    lib.orc_mrca_rows_x.restype = ctypes.c_int
    lib.orc_mrca_allpairs_x.argtypes = [ctypes.c_uint32] * 5 + [u32p] * 4
    lib.orc_mrca_allpairs_x.restype = ctypes.c_int
    lib.orc_phylo_metrics_x.argtypes = ([ctypes.c_uint32] * 5 +
                                        [u32p, u32p, ctypes.POINTER(ctypes.c_uint64),
                                         ctypes.POINTER(ctypes.c_double)])
    lib.orc_phylo_metrics_x.restype = ctypes.c_int
    lib.orc_phylo_newick_x.argtypes = ([ctypes.c_uint32] * 5 +
                                       [u32p, u32p, ctypes.c_char_p, ctypes.c_size_t])
    lib.orc_phylo_newick_x.restype = ctypes.c_long
    lib.orc_set_fitness.argtypes = [ctypes.c_void_p] + [ctypes.c_uint32] * 4 + [ctypes.c_float] * 2
    lib.orc_set_fitness.restype = ctypes.c_int
    lib.orc_half_normal.argtypes = [ctypes.c_uint32, ctypes.c_uint32]
    lib.orc_half_normal.restype = ctypes.c_double
    lib.orc_step.argtypes = [ctypes.c_void_p, ctypes.c_uint32]
    lib.orc_step.restype = ctypes.c_int
    lib.orc_generation.argtypes = [ctypes.c_void_p]
    lib.orc_generation.restype = ctypes.c_uint32
    lib.orc_num_agents.argtypes = [ctypes.c_void_p]
    lib.orc_num_agents.restype = ctypes.c_uint32
    lib.orc_read_agents.argtypes = [ctypes.c_void_p, u32p, u32p, u32p]
    lib.orc_read_agents.restype = None
    lib.orc_read_outbox.argtypes = [ctypes.c_void_p, u32p, u32p, u32p, u32p,
                                    u32p]
    lib.orc_read_outbox.restype = ctypes.c_int
    lib.orc_read_layout.argtypes = [ctypes.c_void_p, u32p]
    lib.orc_read_layout.restype = None
    lib.orc_read_pedigree.argtypes = [ctypes.c_void_p, ctypes.c_uint32, u32p,
                                      u8p]
    lib.orc_read_pedigree.restype = ctypes.c_int
    lib.orc_destroy.argtypes = [ctypes.c_void_p]
    lib.orc_destroy.restype = None
    lib.orc_sample.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
                               ctypes.c_uint32, u32p]
    lib.orc_sample.restype = ctypes.c_uint32
    lib.orc_mrca_pair.argtypes = [ctypes.c_uint32, ctypes.c_uint32, u32p, u32p,
                                  ctypes.c_uint32, u32p, u32p, u32p, u32p]
    lib.orc_mrca_pair.restype = ctypes.c_int
    lib.orc_mrca_allpairs.argtypes = [ctypes.c_uint32, ctypes.c_uint32,
                                      ctypes.c_uint32, u32p, u32p, u32p, u32p]
    lib.orc_mrca_allpairs.restype = ctypes.c_int
    lib.orc_mrca_rows.argtypes = [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
                                  u32p, u32p, ctypes.c_uint32, u32p, u32p, u32p]
    lib.orc_mrca_rows.restype = ctypes.c_int
    lib.orc_phylo_metrics.argtypes = [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
                                      u32p, u32p, ctypes.POINTER(ctypes.c_uint64),
                                      ctypes.POINTER(ctypes.c_double)]
    lib.orc_phylo_metrics.restype = ctypes.c_int
    _lib = lib
    return lib


def _p(arr, typ=u32p):
    return arr.ctypes.data_as(typ)


# --------------------------------------------------------------------------
# Philox and integer mappings

def philox(c0: int, c1: int, c2: int, c3: int, seed: int) -> tuple:
    out = np.zeros(4, np.uint32)
    load().orc_philox(c0, c1, c2, c3, seed, _p(out))
    return tuple(int(x) for x in out)


def mulhi(w: int, n: int) -> int:
    return int(load().orc_mulhi(w, n))


def half_normal(w_radius: int, w_angle: int) -> float:
    """|Z| of one Box-Muller draw from two Philox words (float treatments)."""
    return float(load().orc_half_normal(w_radius, w_angle))


def as_f32(words) -> np.ndarray:
    """binary32 view of trait words."""
    return np.ascontiguousarray(words, np.uint32).view(np.float32)


# --------------------------------------------------------------------------
# Site rule

def in_D(policy: int, m: int, u: int, t: int) -> bool:
    return bool(load().orc_in_D(policy, m, u, t))


def horizon(kind: int, S: int) -> int:
    return int(load().orc_horizon(kind, S))


def layout(kind: int, S: int, T: int) -> np.ndarray:
    """Deposit time held by each site after T ingests (EMPTY if unfilled)."""
    L = np.zeros(S, np.uint32)
    rc = load().orc_layout(kind, S, T, _p(L))
    if rc:
        raise ValueError("beyond the horizon")
    return L


def place(kind: int, S: int, L: np.ndarray, T: int) -> int:
    L = np.ascontiguousarray(L, np.uint32)
    return int(load().orc_place(kind, S, _p(L), T))


def site_sequence(kind: int, S: int, T0: int, n: int) -> np.ndarray:
    out = np.zeros(n, np.int32)
    rc = load().orc_site_sequence(kind, S, T0, n, _p(out, i32p))
    if rc:
        raise ValueError("beyond the horizon")
    return out


# --------------------------------------------------------------------------
# GA runs

class Run:
    """One oracle run.  Parameters mirror the GA configuration."""

    def __init__(self, W, H, N, S, kind, tournament=2, mut_thr=42949672,
                 mut_lo=-8, mut_hi=8, migrants=1, seed=1, pedigree_gens=0,
                 fitness_model=INT_TRAIT, del_thr=0, ben_thr=0, del_sigma=1.0,
                 ben_sigma=1.0, bits=1, interval=1, activity=0, threads=0):
        lib = load()
        h = lib.orc_create_ex(W, H, N, S, kind,
                              tournament if fitness_model == INT_TRAIT else 0,
                              mut_thr, mut_lo, mut_hi, migrants, seed, pedigree_gens, bits,
                              interval)
        if not h:
            raise ValueError("invalid oracle configuration")
        self._h = h
        if lib.orc_set_fitness(h, fitness_model, tournament, del_thr, ben_thr, del_sigma,
                               ben_sigma):
            self.close()
            raise ValueError("invalid oracle fitness configuration")
        if lib.orc_set_async(h, activity):
            self.close()
            raise ValueError("invalid asynchronous configuration")
        if lib.orc_set_threads(h, threads):
            self.close()
            raise ValueError("invalid thread count")
        self.W, self.H, self.N, self.S, self.kind = W, H, N, S, kind
        self.bits, self.interval = bits, interval
        self.I = W * H
        self.A = self.I * N
        self.SW = S * bits // 32
        self.seed = seed

    def close(self):
        if self._h:
            load().orc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def generation(self) -> int:
        return int(load().orc_generation(self._h))

    def step(self, n: int = 1):
        rc = load().orc_step(self._h, n)
        if rc:
            raise RuntimeError(f"oracle step failed ({rc})")

    def agents(self):
        """(trait, counter, surface[A, SW]) of the current population."""
        t = np.zeros(self.A, np.uint32)
        c = np.zeros(self.A, np.uint32)
        s = np.zeros((self.A, self.SW), np.uint32)
        load().orc_read_agents(self._h, _p(t), _p(c), _p(s))
        return t, c, s

    def outbox(self):
        """(dir, trait, counter, surface[I, SW], src) of O_g, or None."""
        d = np.zeros(self.I, np.uint32)
        t = np.zeros(self.I, np.uint32)
        c = np.zeros(self.I, np.uint32)
        s = np.zeros((self.I, self.SW), np.uint32)
        src = np.zeros(self.I, np.uint32)
        ok = load().orc_read_outbox(self._h, _p(d), _p(t), _p(c), _p(s), _p(src))
        if not ok:
            return None
        return d, t, c, s, src

    def layout(self) -> np.ndarray:
        L = np.zeros(self.S, np.uint32)
        load().orc_read_layout(self._h, _p(L))
        return L

    def pedigree(self, gen: int):
        """(parent index in P_{gen-1}, drawn differentia bit) of generation gen."""
        p = np.zeros(self.A, np.uint32)
        b = np.zeros(self.A, np.uint8)
        rc = load().orc_read_pedigree(self._h, gen, _p(p), _p(b, u8p))
        if rc:
            raise ValueError("no pedigree for that generation")
        return p, b


# --------------------------------------------------------------------------
# Sampling and MRCA bounds

def sample(seed: int, A: int, n: int, T: int) -> np.ndarray:
    idx = np.zeros(max(n, 1), np.uint32)
    k = load().orc_sample(seed, A, n, T, _p(idx))
    return idx[:k].copy()


def mrca_pair(S: int, Ta: int, sa, Tb: int, sb, kind: int):
    sa = np.ascontiguousarray(sa, np.uint32)
    sb = np.ascontiguousarray(sb, np.uint32)
    La = layout(kind, S, Ta)
    Lb = layout(kind, S, Tb)
    lb = np.zeros(1, np.uint32)
    ub = np.zeros(1, np.uint32)
    load().orc_mrca_pair(S, Ta, _p(sa), _p(La), Tb, _p(sb), _p(Lb), _p(lb),
                         _p(ub))
    return int(lb[0]), int(ub[0])


def horizon_gen(kind: int, S: int, interval: int = 1) -> int:
    """Last generation a run can step with this ingest interval."""
    return int(load().orc_horizon_gen(kind, S, interval))


def mrca_allpairs(kind: int, S: int, counters, surfaces, bits: int = 1, interval: int = 1):
    """lb, ub (n x n, row-major) over every ordered pair."""
    counters = np.ascontiguousarray(counters, np.uint32)
    surfaces = np.ascontiguousarray(surfaces, np.uint32).reshape(-1)
    n = counters.shape[0]
    lb = np.zeros((n, n), np.uint32)
    ub = np.zeros((n, n), np.uint32)
    rc = load().orc_mrca_allpairs_x(kind, S, bits, interval, n, _p(counters), _p(surfaces),
                                    _p(lb), _p(ub))
    if rc:
        raise ValueError("beyond the horizon or invalid scheme")
    return lb, ub


def mrca_rows(kind: int, S: int, counters, surfaces, rows, bits: int = 1, interval: int = 1):
    """Rows `rows` of the all-pairs matrices (len(rows) x n)."""
    counters = np.ascontiguousarray(counters, np.uint32)
    surfaces = np.ascontiguousarray(surfaces, np.uint32).reshape(-1)
    rows = np.ascontiguousarray(rows, np.uint32)
    n = counters.shape[0]
    lb = np.zeros((len(rows), n), np.uint32)
    ub = np.zeros((len(rows), n), np.uint32)
    rc = load().orc_mrca_rows_x(kind, S, bits, interval, n, _p(counters), _p(surfaces),
                                len(rows), _p(rows), _p(lb), _p(ub))
    if rc:
        raise ValueError("beyond the horizon, invalid scheme or row out of range")
    return lb, ub


def phylo_metrics(kind: int, S: int, counters, surfaces, bits: int = 1, interval: int = 1):
    """Trie reconstruction of annotations sharing a counter: (sum of branch
    lengths, sum over pairs of T - MRCA time, root time, internal nodes,
    per-leaf evolutionary distinctiveness)."""
    counters = np.ascontiguousarray(counters, np.uint32)
    surfaces = np.ascontiguousarray(surfaces, np.uint32).reshape(-1)
    n = counters.shape[0]
    out = np.zeros(4, np.uint64)
    ed = np.zeros(max(n, 1), np.float64)
    rc = load().orc_phylo_metrics_x(kind, S, bits, interval, n, _p(counters), _p(surfaces),
                                    out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                                    ed.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    if rc:
        raise ValueError("counters differ, past the horizon, invalid scheme, or no memory")
    return int(out[0]), int(out[1]), int(out[2]), int(out[3]), ed[:n].copy()


def phylo_newick(kind: int, S: int, counters, surfaces, bits: int = 1,
                 interval: int = 1) -> str:
    """The reconstructed tree as canonical Newick text (leaves = indices)."""
    counters = np.ascontiguousarray(counters, np.uint32)
    surfaces = np.ascontiguousarray(surfaces, np.uint32).reshape(-1)
    n = counters.shape[0]
    cap = 64 * max(n, 1) + 64
    buf = ctypes.create_string_buffer(cap)
    rc = load().orc_phylo_newick_x(kind, S, bits, interval, n, _p(counters), _p(surfaces),
                                   buf, cap)
    if rc < 0:
        raise ValueError("counters differ, past the horizon, invalid scheme, or no memory")
    return buf.value.decode()


# --------------------------------------------------------------------------
# The paper's 96-bit validation genome (Supplemental Material, genome layout
# figure): bytes 0-1 founder tag, bytes 2-3 generation counter, bytes 4-11
# surface, little-endian.

def unpack_genome96(b: bytes):
    if len(b) != 12:
        raise ValueError("a 96-bit genome has 12 bytes")
    tag = int.from_bytes(b[0:2], "little")
    counter = int.from_bytes(b[2:4], "little")
    surface = int.from_bytes(b[4:12], "little")
    return tag, counter, surface
