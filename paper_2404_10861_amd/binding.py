"""ctypes binding of libhsga.so (declared in include/hsga.h).

Argument marshalling only: every step of the method runs in the library's
HIP kernels.  PyTorch provides device memory (uint8 arenas, output tensors)
and streams.  There is no CPU fallback: loading fails loudly when the built
library is missing.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np
import torch  # imported first: the library then binds to torch's HIP runtime

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libhsga.so")

GA_OK, GA_EINVAL, GA_ENOMEM, GA_EHORIZON, GA_EDEVICE, GA_EBUSY = 0, -1, -2, -3, -4, -5
STEADY, TILTED, HYBRID = 0, 1, 2
KINDS = {"steady": STEADY, "tilted": TILTED, "hybrid": HYBRID}
EMPTY_SITE = 0xFFFFFFFF

# Every exported entry point of include/hsga.h.
EXPORTS = (
    "ga_footprint_bytes", "ga_create", "ga_step", "ga_sync", "ga_generation",
    "ga_read_agents", "ga_read_outbox", "ga_read_layout", "ga_sample",
    "ga_state_bytes", "ga_export_state", "ga_import_state",
    "ga_destroy", "ga_last_error", "hstrat_mrca_workspace_bytes",
    "hstrat_mrca_bounds", "hstrat_mrca_status", "ga_set_kernel_timing",
    "ga_kernel_time", "ga_set_launch_shape", "ga_probe_copy",
    "ga_pool_overhead_bytes", "ga_pool_create", "ga_pool_footprint", "ga_pool_admit",
    "ga_pool_advance", "ga_pool_poll", "ga_pool_run", "ga_pool_release", "ga_pool_sync",
    "ga_pool_set_launch", "ga_pool_info", "ga_pool_destroy",
    "hstrat_phylo_workspace_bytes", "hstrat_phylo_metrics",
    "hstrat_mrca_bounds_ex", "hstrat_phylo_metrics_ex", "hstrat_phylo_tree_ex",
    "ga_mrca_bounds", "ga_phylo_tree", "hstrat_mrca_bounds_noalloc",
    "hstrat_layout", "hstrat_mrca_bounds_pair", "hstrat_mrca_bounds_pair_ex", "hstrat_sites",
    "hstrat_phylo_newick", "ga_set_resident", "ga_resident_threads", "ga_pool_set_split",
)


class HsgaError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{message} (status {status})")
        self.status = status


class ga_config(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32),
        ("grid_w", ctypes.c_uint32),
        ("grid_h", ctypes.c_uint32),
        ("pop_per_island", ctypes.c_uint32),
        ("surface_sites", ctypes.c_uint32),
        ("surface_kind", ctypes.c_uint32),
        ("tournament_size", ctypes.c_uint32),
        ("mut_threshold", ctypes.c_uint32),
        ("mut_lo", ctypes.c_int32),
        ("mut_hi", ctypes.c_int32),
        ("migrants_per_island", ctypes.c_uint32),
        ("ingest_interval", ctypes.c_uint32),
        ("seed", ctypes.c_uint64),
        ("fitness_model", ctypes.c_uint32),
        ("del_threshold", ctypes.c_uint32),
        ("ben_threshold", ctypes.c_uint32),
        ("del_sigma", ctypes.c_float),
        ("ben_sigma", ctypes.c_float),
        ("differentia_bits", ctypes.c_uint32),
        ("async_activity", ctypes.c_uint32),
        ("reserved", ctypes.c_uint32),
    ]


class hstrat_scheme(ctypes.Structure):
    _fields_ = [
        ("kind", ctypes.c_uint32),
        ("sites", ctypes.c_uint32),
        ("differentia_bits", ctypes.c_uint32),
        ("ingest_interval", ctypes.c_uint32),
    ]


FITNESS_MODELS = {"int": 0, "float": 1, "tag": 2}


_lib = None
_u32p = ctypes.POINTER(ctypes.c_uint32)
_vp = ctypes.c_void_p


def load_library():
    """Load libhsga.so (built in-tree by paper_2404_10861_amd.build)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"HIP library not built: {LIB_PATH}; run python -m paper_2404_10861_amd.build")
    lib = ctypes.CDLL(LIB_PATH)
    cfgp = ctypes.POINTER(ga_config)
    sig = {
        "ga_footprint_bytes": (ctypes.c_size_t, [cfgp, ctypes.c_uint32]),
        "ga_create": (ctypes.c_int, [cfgp, _vp, ctypes.c_size_t, ctypes.c_uint32, _vp,
                                     ctypes.POINTER(_vp)]),
        "ga_step": (ctypes.c_int, [_vp, ctypes.c_uint32]),
        "ga_sync": (ctypes.c_int, [_vp]),
        "ga_generation": (ctypes.c_int, [_vp, _u32p]),
        "ga_read_agents": (ctypes.c_int, [_vp, ctypes.c_uint32, ctypes.c_uint32, _vp, _vp, _vp]),
        "ga_read_outbox": (ctypes.c_int, [_vp, ctypes.c_uint32, ctypes.c_uint32, _vp, _vp, _vp,
                                          _vp, ctypes.POINTER(ctypes.c_int)]),
        "ga_read_layout": (ctypes.c_int, [_vp, _vp]),
        "ga_sample": (ctypes.c_int, [_vp, ctypes.c_uint32, _vp, _vp, _vp, _u32p]),
        "ga_state_bytes": (ctypes.c_size_t, [_vp]),
        "ga_export_state": (ctypes.c_int, [_vp, _vp, ctypes.c_size_t]),
        "ga_import_state": (ctypes.c_int, [_vp, _vp, ctypes.c_size_t]),
        "ga_destroy": (None, [_vp]),
        "ga_last_error": (ctypes.c_char_p, []),
        "hstrat_mrca_workspace_bytes": (ctypes.c_size_t, [ctypes.c_uint32, ctypes.c_uint32]),
        "hstrat_mrca_bounds": (ctypes.c_int, [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
                                              _vp, _vp, _vp, _vp, _vp, ctypes.c_size_t, _vp]),
        "hstrat_mrca_status": (ctypes.c_int, [_vp, _vp]),
        "hstrat_layout": (ctypes.c_int, [_vp, ctypes.c_uint32, _vp]),
        "hstrat_sites": (ctypes.c_int, [_vp, ctypes.c_uint32, ctypes.c_uint32, _vp]),
        "hstrat_phylo_newick": (ctypes.c_int, [ctypes.c_uint32, ctypes.c_uint32, _vp, _vp, _vp,
                                               ctypes.c_char_p, ctypes.c_size_t,
                                               ctypes.POINTER(ctypes.c_size_t)]),
        "hstrat_mrca_bounds_pair": (ctypes.c_int, [ctypes.c_uint32, ctypes.c_uint32,
                                                   ctypes.c_uint32, _vp, ctypes.c_uint32, _vp,
                                                   _vp, _vp]),
        "hstrat_mrca_bounds_pair_ex": (ctypes.c_int, [_vp, ctypes.c_uint32, _vp,
                                                      ctypes.c_uint32, _vp, _vp, _vp]),
        "hstrat_mrca_bounds_noalloc": (ctypes.c_int, [ctypes.c_uint32, ctypes.c_uint32,
                                                      ctypes.c_uint32, _vp, _vp, _vp, _vp, _vp]),
        "ga_set_kernel_timing": (ctypes.c_int, [_vp, ctypes.c_int]),
        "ga_kernel_time": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_double),
                                          ctypes.POINTER(ctypes.c_uint64), ctypes.c_int]),
        "ga_set_launch_shape": (ctypes.c_int, [_vp, ctypes.c_uint32, ctypes.c_uint32]),
        "ga_set_resident": (ctypes.c_int, [_vp, ctypes.c_int]),
        "ga_pool_set_split": (ctypes.c_int, [_vp, ctypes.c_uint64]),
        "ga_resident_threads": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_uint32)]),
        "ga_probe_copy": (ctypes.c_int, [_vp, _vp, ctypes.c_size_t, _vp]),
        "ga_pool_overhead_bytes": (ctypes.c_size_t, [ctypes.c_uint32]),
        "ga_pool_create": (ctypes.c_int, [_vp, ctypes.c_size_t, ctypes.c_uint32, ctypes.c_uint32,
                                          _vp, ctypes.POINTER(_vp)]),
        "ga_pool_footprint": (ctypes.c_size_t, [_vp, cfgp]),
        "ga_pool_admit": (ctypes.c_int, [_vp, cfgp, ctypes.c_uint32, _u32p]),
        "ga_pool_advance": (ctypes.c_int, [_vp, ctypes.c_uint32, _u32p]),
        "ga_pool_poll": (ctypes.c_int, [_vp, _vp, ctypes.c_uint32, _u32p]),
        "ga_pool_run": (ctypes.c_int, [_vp, ctypes.c_uint32, ctypes.POINTER(_vp)]),
        "ga_pool_release": (ctypes.c_int, [_vp, ctypes.c_uint32]),
        "ga_pool_sync": (ctypes.c_int, [_vp]),
        "ga_pool_set_launch": (ctypes.c_int, [_vp, ctypes.c_uint32, ctypes.c_int]),
        "ga_pool_info": (ctypes.c_int, [_vp, _u32p, _u32p, ctypes.POINTER(ctypes.c_size_t),
                                        ctypes.POINTER(ctypes.c_size_t)]),
        "ga_pool_destroy": (None, [_vp]),
        "hstrat_phylo_workspace_bytes": (ctypes.c_size_t, [ctypes.c_uint32, ctypes.c_uint32]),
        "hstrat_phylo_metrics": (ctypes.c_int, [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
                                                _vp, _vp, _vp, _vp, ctypes.c_size_t, _vp]),
        "hstrat_phylo_tree_ex": (ctypes.c_int, [_vp, ctypes.c_uint32, _vp, _vp, _vp, _vp, _vp,
                                                _vp, _vp, ctypes.c_size_t, _vp]),
        "ga_mrca_bounds": (ctypes.c_int, [_vp, ctypes.c_uint32, _vp, _vp, _vp, _vp, _vp,
                                          ctypes.c_size_t]),
        "ga_phylo_tree": (ctypes.c_int, [_vp, ctypes.c_uint32, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                                         ctypes.c_size_t]),
        "hstrat_mrca_bounds_ex": (ctypes.c_int, [_vp, ctypes.c_uint32, _vp, _vp, _vp, _vp, _vp,
                                                 ctypes.c_size_t, _vp]),
        "hstrat_phylo_metrics_ex": (ctypes.c_int, [_vp, ctypes.c_uint32, _vp, _vp, _vp, _vp,
                                                   ctypes.c_size_t, _vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(rc: int):
    if rc != GA_OK:
        raise HsgaError(rc, load_library().ga_last_error().decode())


def _stream_handle(stream) -> int:
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream)


def _ptr(arr: np.ndarray):
    return arr.ctypes.data_as(_vp)


@dataclass
class Config:
    """GA configuration (ga_config).  Kinds: 'steady', 'tilted', 'hybrid'.

    fitness_model 'int' is the integer trait (tournament_size 0 or 2, the
    mut_* fields); 'float' is the paper's float treatments (tournament_size
    0..5, del_threshold / ben_threshold class probabilities times 2^32,
    del_sigma / ben_sigma scales of the half-normal change); 'tag' gives
    founders random 16-bit tags, inherited unchanged (tournament_size 0).
    differentia_bits 1 (surface_sites 32 or 64) or 8 (surface_sites 4 or
    8); ingest_interval n deposits every n-th generation only.
    async_activity p * 2^32 (0: synchronous) runs asynchronous ticks: each
    island runs a generation with probability p per tick, agents keep their
    own counters."""
    grid_w: int
    grid_h: int
    pop_per_island: int = 32
    surface_sites: int = 32
    surface_kind: str = "steady"
    tournament_size: int = 2
    mut_threshold: int = 42949672
    mut_lo: int = -8
    mut_hi: int = 8
    migrants_per_island: int = 1
    seed: int = 1
    fitness_model: str = "int"
    del_threshold: int = 0
    ben_threshold: int = 0
    del_sigma: float = 1.0
    ben_sigma: float = 1.0
    differentia_bits: int = 1
    ingest_interval: int = 1
    async_activity: int = 0

    @property
    def kind(self) -> int:
        return KINDS[self.surface_kind]

    @property
    def surface_words(self) -> int:
        return self.surface_sites * self.differentia_bits // 32

    @property
    def scheme(self) -> dict:
        """Keyword arguments of mrca_bounds / phylo_metrics for this run."""
        return {"bits": self.differentia_bits, "interval": self.ingest_interval}

    @property
    def islands(self) -> int:
        return self.grid_w * self.grid_h

    @property
    def agents(self) -> int:
        return self.islands * self.pop_per_island

    def to_c(self) -> ga_config:
        c = ga_config()
        c.struct_size = ctypes.sizeof(ga_config)
        c.grid_w, c.grid_h = self.grid_w, self.grid_h
        c.pop_per_island = self.pop_per_island
        c.surface_sites = self.surface_sites
        c.surface_kind = self.kind
        c.tournament_size = self.tournament_size
        c.mut_threshold = self.mut_threshold
        c.mut_lo, c.mut_hi = self.mut_lo, self.mut_hi
        c.migrants_per_island = self.migrants_per_island
        c.ingest_interval = self.ingest_interval
        c.seed = self.seed
        c.fitness_model = FITNESS_MODELS[self.fitness_model]
        c.del_threshold = self.del_threshold
        c.ben_threshold = self.ben_threshold
        c.del_sigma = self.del_sigma
        c.ben_sigma = self.ben_sigma
        c.differentia_bits = self.differentia_bits
        c.async_activity = self.async_activity
        c.reserved = 0
        return c


def footprint_bytes(cfg: Config, max_gens_per_launch: int = 0) -> int:
    c = cfg.to_c()
    n = load_library().ga_footprint_bytes(ctypes.byref(c), max_gens_per_launch)
    if n == 0:
        raise HsgaError(GA_EINVAL, load_library().ga_last_error().decode())
    return int(n)


def _aligned_bytes(nbytes: int, device) -> tuple:
    """A uint8 device tensor with a 256-byte aligned window of nbytes."""
    buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
    off = (-buf.data_ptr()) % 256
    return buf, buf.data_ptr() + off


class RunHandle:
    """Read and sample operations on a run handle (owned or borrowed)."""

    _h = None

    def _setup(self, cfg: Config, device):
        self.cfg = cfg
        self.device = torch.device(device)
        self.S = cfg.surface_sites
        self.SW = cfg.surface_words
        self.A = cfg.agents
        self.I = cfg.islands

    @property
    def generation(self) -> int:
        T = ctypes.c_uint32()
        _check(load_library().ga_generation(self._h, ctypes.byref(T)))
        return T.value

    def agents(self, first: int = 0, count: int | None = None):
        """(trait, counter, surface[count, S/32]) as numpy uint32 (blocking)."""
        if count is None:
            count = self.A - first
        t = np.zeros(count, np.uint32)
        c = np.zeros(count, np.uint32)
        s = np.zeros((count, self.SW), np.uint32)
        _check(load_library().ga_read_agents(self._h, first, count, _ptr(t), _ptr(c), _ptr(s)))
        return t, c, s

    def outbox(self, first: int = 0, count: int | None = None):
        """(dir, trait, counter, surface[count, S/32]) or None (blocking)."""
        if count is None:
            count = self.I - first
        d = np.zeros(count, np.uint32)
        t = np.zeros(count, np.uint32)
        c = np.zeros(count, np.uint32)
        s = np.zeros((count, self.SW), np.uint32)
        valid = ctypes.c_int()
        _check(load_library().ga_read_outbox(self._h, first, count, _ptr(d), _ptr(t), _ptr(c),
                                             _ptr(s), ctypes.byref(valid)))
        return (d, t, c, s) if valid.value else None

    def layout(self) -> np.ndarray:
        L = np.zeros(self.S, np.uint32)
        _check(load_library().ga_read_layout(self._h, _ptr(L)))
        return L

    def export_state(self) -> np.ndarray:
        """The run's state at the generation enqueued so far, as a uint8
        host array (blocking); ``Run.import_state`` resumes from it."""
        lib = load_library()
        nbytes = lib.ga_state_bytes(self._h)
        words = np.zeros(nbytes // 4, np.uint32)
        _check(lib.ga_export_state(self._h, _ptr(words), nbytes))
        return words.view(np.uint8)

    def mrca_bounds(self, counter: torch.Tensor, surface_words: torch.Tensor,
                    workspace: "MrcaWorkspace | None" = None, lb=None, ub=None):
        """mrca_bounds of annotations taken from this run, with its scheme and
        on its stream: when every counter is the run's generation count, the
        run's own layout is used as it stands."""
        n = counter.shape[0]
        if counter.dtype != torch.int32 or surface_words.dtype != torch.int32:
            raise ValueError("counter and surface_words must be int32 tensors")
        with torch.cuda.stream(self.stream):
            counter = counter.contiguous()
            surface_words = surface_words.contiguous()
            if workspace is None or workspace.n < n or workspace.S < self.S:
                workspace = MrcaWorkspace(self.S, n, self.device)
            if lb is None:
                lb = torch.empty((n, n), dtype=torch.int32, device=self.device)
            if ub is None:
                ub = torch.empty((n, n), dtype=torch.int32, device=self.device)
            _check(load_library().ga_mrca_bounds(
                self._h, n, _vp(counter.data_ptr()), _vp(surface_words.data_ptr()),
                _vp(lb.data_ptr()), _vp(ub.data_ptr()), _vp(workspace.ptr), workspace.nbytes))
        return lb, ub

    def phylo_tree(self, counter: torch.Tensor, surface_words: torch.Tensor,
                   tree: bool = True) -> dict:
        """phylo_tree (tree=False: phylo_metrics) of annotations taken from
        this run, with its scheme and on its stream, using the run's own
        layout when every counter is its generation count."""
        n = counter.shape[0]
        if counter.dtype != torch.int32 or surface_words.dtype != torch.int32:
            raise ValueError("counter and surface_words must be int32 tensors")
        lib = load_library()
        with torch.cuda.stream(self.stream):
            counter = counter.contiguous()
            surface_words = surface_words.contiguous()
            need = int(lib.hstrat_phylo_workspace_bytes(self.S, n))
            buf, ptr = _aligned_bytes(need, self.device)
            out = torch.zeros(8, dtype=torch.int64, device=self.device)
            leaf = node_parent = node_time = None
            if tree:
                leaf = torch.empty(n, dtype=torch.int32, device=self.device)
                node_parent = torch.empty(max(n - 1, 1), dtype=torch.int32, device=self.device)
                node_time = torch.empty(max(n - 1, 1), dtype=torch.int32, device=self.device)
            ptr_of = lambda t: _vp(t.data_ptr()) if t is not None else None   # noqa: E731
            _check(lib.ga_phylo_tree(self._h, n, _vp(counter.data_ptr()),
                                     _vp(surface_words.data_ptr()), ptr_of(leaf),
                                     ptr_of(node_parent), ptr_of(node_time),
                                     _vp(out.data_ptr()), _vp(ptr), need))
            res = _phylo_result(out.cpu().numpy().view(np.uint64), n)
            if tree:
                res.update({"leaf_parent": as_u32(leaf),
                            "node_parent": as_u32(node_parent)[:n - 1],
                            "node_time": as_u32(node_time)[:n - 1],
                            "T": int(counter[0].item()) & 0xFFFFFFFF})
            del buf
        return res

    def sample(self, n: int, out=None):
        """Stratified sample on the device: (idx, counter, surface[n, S/32])
        as int32 CUDA tensors holding the uint32 bit patterns."""
        if out is None:
            idx = torch.empty(n, dtype=torch.int32, device=self.device)
            cnt = torch.empty(n, dtype=torch.int32, device=self.device)
            srf = torch.empty((n, self.SW), dtype=torch.int32, device=self.device)
        else:
            idx, cnt, srf = out
        taken = ctypes.c_uint32()
        _check(load_library().ga_sample(self._h, n, _vp(idx.data_ptr()), _vp(cnt.data_ptr()),
                                        _vp(srf.data_ptr()), ctypes.byref(taken)))
        k = taken.value
        return idx[:k], cnt[:k], srf[:k]


class Run(RunHandle):
    """One GA run on the GPU; the arena is a torch uint8 tensor it owns
    (or the caller's, via ``arena``)."""

    def __init__(self, cfg: Config, max_gens_per_launch: int = 0, device="cuda",
                 stream=None, arena: torch.Tensor | None = None):
        lib = load_library()
        self._setup(cfg, device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        need = footprint_bytes(cfg, max_gens_per_launch)
        if arena is None:
            self._arena, ptr = _aligned_bytes(need, self.device)
            nbytes = need
        else:
            if arena.dtype != torch.uint8 or not arena.is_cuda:
                raise ValueError("arena must be a CUDA uint8 tensor")
            self._arena, ptr, nbytes = arena, arena.data_ptr(), arena.numel()
        self._c = cfg.to_c()
        h = _vp()
        _check(lib.ga_create(ctypes.byref(self._c), _vp(ptr), nbytes, max_gens_per_launch,
                             _vp(_stream_handle(self.stream)), ctypes.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            load_library().ga_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, n: int = 1):
        _check(load_library().ga_step(self._h, n))

    def sync(self):
        _check(load_library().ga_sync(self._h))

    def set_kernel_timing(self, enable: bool = True):
        _check(load_library().ga_set_kernel_timing(self._h, 1 if enable else 0))

    def kernel_time(self, reset: bool = False):
        """(milliseconds, launches) of the timed step kernels (blocking)."""
        ms = ctypes.c_double()
        n = ctypes.c_uint64()
        _check(load_library().ga_kernel_time(self._h, ctypes.byref(ms), ctypes.byref(n),
                                             1 if reset else 0))
        return ms.value, n.value

    def set_launch_shape(self, block_threads: int = 0, agents_per_thread: int = 0):
        _check(load_library().ga_set_launch_shape(self._h, block_threads, agents_per_thread))

    def set_resident(self, enable: bool = True):
        """The resident form for a run that fits one workgroup (default on);
        False: one launch per generation at the launch shape."""
        _check(load_library().ga_set_resident(self._h, 1 if enable else 0))

    @property
    def resident_threads(self) -> int:
        """Workgroup size of the resident form, 0 if the run does not use it."""
        t = ctypes.c_uint32()
        _check(load_library().ga_resident_threads(self._h, ctypes.byref(t)))
        return t.value

    def import_state(self, state):
        """Replace this run's state by one exported from a run of the same
        configuration (a uint8 array or bytes); the run continues from
        there exactly as the exporting run would (blocking)."""
        raw = np.frombuffer(bytes(state), np.uint8) if not isinstance(state, np.ndarray) \
            else np.ascontiguousarray(state).reshape(-1).view(np.uint8)
        words = np.zeros((raw.size + 3) // 4, np.uint32)      # a 4-byte aligned copy
        words.view(np.uint8)[: raw.size] = raw
        _check(load_library().ga_import_state(self._h, _ptr(words), raw.size))


class PoolRun(RunHandle):
    """A run admitted to a Pool (borrowed handle, valid until released)."""

    def __init__(self, pool: "Pool", run_id: int, cfg: Config):
        h = _vp()
        _check(load_library().ga_pool_run(pool._h, run_id, ctypes.byref(h)))
        self._h = h
        self.id = run_id
        self.stream = pool.stream
        self._setup(cfg, pool.device)


class Pool:
    """Batched / served runs sharing one device arena and one stream."""

    def __init__(self, arena_bytes: int, max_runs: int = 256, max_gens_per_launch: int = 0,
                 device="cuda", stream=None, block_threads: int = 64, use_graph: bool = False):
        lib = load_library()
        self.device = torch.device(device)
        if stream is None:
            stream = torch.cuda.Stream(self.device)
        self.stream = stream
        self._arena, ptr = _aligned_bytes(arena_bytes, self.device)
        h = _vp()
        _check(lib.ga_pool_create(_vp(ptr), arena_bytes, max_runs, max_gens_per_launch,
                                  _vp(_stream_handle(stream)), ctypes.byref(h)))
        self._h = h
        self.cfgs: dict[int, Config] = {}
        self._c: dict[int, ga_config] = {}
        self.set_launch(block_threads, use_graph)

    def close(self):
        if getattr(self, "_h", None):
            load_library().ga_pool_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_launch(self, block_threads: int = 0, use_graph: bool = False):
        _check(load_library().ga_pool_set_launch(self._h, block_threads, 1 if use_graph else 0))

    def set_split(self, min_words: int):
        """Generations reading at least min_words trait and surface words
        launch as two groups side by side (0: always)."""
        _check(load_library().ga_pool_set_split(self._h, min_words))

    def footprint(self, cfg: Config) -> int:
        c = cfg.to_c()
        return int(load_library().ga_pool_footprint(self._h, ctypes.byref(c)))

    def admit(self, cfg: Config, n_generations: int):
        """The new run's id, or None when its footprint does not fit now."""
        c = cfg.to_c()
        rid = ctypes.c_uint32()
        rc = load_library().ga_pool_admit(self._h, ctypes.byref(c), n_generations,
                                          ctypes.byref(rid))
        if rc == GA_EBUSY:
            return None
        _check(rc)
        self.cfgs[rid.value] = cfg
        self._c[rid.value] = c
        return rid.value

    def advance(self, max_gens: int) -> int:
        n = ctypes.c_uint32()
        _check(load_library().ga_pool_advance(self._h, max_gens, ctypes.byref(n)))
        return n.value

    def poll(self) -> list[int]:
        ids = (ctypes.c_uint32 * 256)()
        n = ctypes.c_uint32()
        _check(load_library().ga_pool_poll(self._h, ctypes.cast(ids, _vp), 256, ctypes.byref(n)))
        return [ids[i] for i in range(n.value)]

    def run(self, run_id: int) -> PoolRun:
        return PoolRun(self, run_id, self.cfgs[run_id])

    def release(self, run_id: int):
        _check(load_library().ga_pool_release(self._h, run_id))
        self.cfgs.pop(run_id, None)
        self._c.pop(run_id, None)

    def sync(self):
        _check(load_library().ga_pool_sync(self._h))

    def info(self) -> dict:
        a = ctypes.c_uint32()
        u = ctypes.c_uint32()
        fb = ctypes.c_size_t()
        lf = ctypes.c_size_t()
        _check(load_library().ga_pool_info(self._h, ctypes.byref(a), ctypes.byref(u),
                                           ctypes.byref(fb), ctypes.byref(lf)))
        return {"active": a.value, "admitted": u.value, "free_bytes": fb.value,
                "largest_free": lf.value}


def pool_overhead_bytes(max_runs: int) -> int:
    return int(load_library().ga_pool_overhead_bytes(max_runs))


class MrcaWorkspace:
    """Device workspace for mrca_bounds, reusable across calls."""

    def __init__(self, S: int, n: int, device="cuda"):
        need = int(load_library().hstrat_mrca_workspace_bytes(S, n))
        self._buf, self.ptr = _aligned_bytes(need, device)
        self.nbytes = need
        self.S, self.n = S, n


def _scheme(kind: int, S: int, bits: int, interval: int) -> hstrat_scheme:
    sc = hstrat_scheme()
    sc.kind, sc.sites, sc.differentia_bits, sc.ingest_interval = kind, S, bits, interval
    return sc


def mrca_bounds(kind, S: int, counter: torch.Tensor, surface_words: torch.Tensor,
                workspace: MrcaWorkspace | None = None, stream=None,
                lb: torch.Tensor | None = None, ub: torch.Tensor | None = None,
                bits: int = 1, interval: int = 1):
    """All ordered pairs of MRCA-generation bounds on the device.

    counter: int32 CUDA tensor [n] (uint32 bit patterns); surface_words:
    int32 CUDA tensor [n, S * bits / 32].  bits / interval: the annotation
    scheme (Config.scheme).  Returns (lb, ub) int32 CUDA tensors [n, n].
    """
    if isinstance(kind, str):
        kind = KINDS[kind]
    n = counter.shape[0]
    dev = counter.device
    if counter.dtype != torch.int32 or surface_words.dtype != torch.int32:
        raise ValueError("counter and surface_words must be int32 tensors")
    counter = counter.contiguous()
    surface_words = surface_words.contiguous()
    if workspace is None or workspace.n < n or workspace.S < S:
        workspace = MrcaWorkspace(S, n, dev)
    if lb is None:
        lb = torch.empty((n, n), dtype=torch.int32, device=dev)
    if ub is None:
        ub = torch.empty((n, n), dtype=torch.int32, device=dev)
    lib = load_library()
    if bits == 1 and interval == 1:
        _check(lib.hstrat_mrca_bounds(kind, S, n, _vp(counter.data_ptr()),
                                      _vp(surface_words.data_ptr()), _vp(lb.data_ptr()),
                                      _vp(ub.data_ptr()), _vp(workspace.ptr), workspace.nbytes,
                                      _vp(_stream_handle(stream))))
    else:
        sc = _scheme(kind, S, bits, interval)
        _check(lib.hstrat_mrca_bounds_ex(ctypes.byref(sc), n, _vp(counter.data_ptr()),
                                         _vp(surface_words.data_ptr()), _vp(lb.data_ptr()),
                                         _vp(ub.data_ptr()), _vp(workspace.ptr),
                                         workspace.nbytes, _vp(_stream_handle(stream))))
    return lb, ub


def phylo_metrics(kind, S: int, counter: torch.Tensor, surface_words: torch.Tensor,
                  stream=None, bits: int = 1, interval: int = 1) -> dict:
    """Trie reconstruction of annotations sharing a counter, on the device.

    Returns the library's eight result words (blocking copy to the host):
    sum_branch_length, pair_sum, root_time, internal_nodes, status, n,
    mean_ed (= sum_branch_length / n under fair proportion) and
    mean_pairwise_distance."""
    if isinstance(kind, str):
        kind = KINDS[kind]
    n = counter.shape[0]
    dev = counter.device
    if counter.dtype != torch.int32 or surface_words.dtype != torch.int32:
        raise ValueError("counter and surface_words must be int32 tensors")
    if stream is None:
        stream = torch.cuda.current_stream(dev)
    lib = load_library()
    with torch.cuda.stream(stream):     # allocation, launch and copy in one stream order
        counter = counter.contiguous()
        surface_words = surface_words.contiguous()
        need = int(lib.hstrat_phylo_workspace_bytes(S, n))
        buf, ptr = _aligned_bytes(need, dev)
        out = torch.zeros(8, dtype=torch.int64, device=dev)
        if bits == 1 and interval == 1:
            _check(lib.hstrat_phylo_metrics(kind, S, n, _vp(counter.data_ptr()),
                                            _vp(surface_words.data_ptr()), _vp(out.data_ptr()),
                                            _vp(ptr), need, _vp(_stream_handle(stream))))
        else:
            sc = _scheme(kind, S, bits, interval)
            _check(lib.hstrat_phylo_metrics_ex(ctypes.byref(sc), n, _vp(counter.data_ptr()),
                                               _vp(surface_words.data_ptr()),
                                               _vp(out.data_ptr()), _vp(ptr), need,
                                               _vp(_stream_handle(stream))))
        w = out.cpu().numpy().view(np.uint64)
        del buf
    return _phylo_result(w, n)


def _phylo_result(w, n: int) -> dict:
    """The eight result words of a reconstruction (the last two are the
    library's binary64 means)."""
    means = np.ascontiguousarray(w[6:8], np.uint64).view(np.float64)
    return {"sum_branch_length": int(w[0]), "pair_sum": int(w[1]), "root_time": int(w[2]),
            "internal_nodes": int(w[3]), "status": int(w[4]), "n": int(w[5]),
            "mean_ed": float(means[0]), "mean_pairwise_distance": float(means[1])}


PHYLO_ROOT, PHYLO_NOT_NODE = 0xFFFFFFFF, 0xFFFFFFFE


def phylo_tree(kind, S: int, counter: torch.Tensor, surface_words: torch.Tensor,
               stream=None, bits: int = 1, interval: int = 1) -> dict:
    """The reconstructed tree on the device: {"leaf_parent", "node_parent",
    "node_time"} numpy uint32 arrays (nodes named by boundary indices, see
    hstrat_phylo_tree_ex) plus the metrics of phylo_metrics."""
    if isinstance(kind, str):
        kind = KINDS[kind]
    n = counter.shape[0]
    dev = counter.device
    if counter.dtype != torch.int32 or surface_words.dtype != torch.int32:
        raise ValueError("counter and surface_words must be int32 tensors")
    if stream is None:
        stream = torch.cuda.current_stream(dev)
    lib = load_library()
    with torch.cuda.stream(stream):
        counter = counter.contiguous()
        surface_words = surface_words.contiguous()
        need = int(lib.hstrat_phylo_workspace_bytes(S, n))
        buf, ptr = _aligned_bytes(need, dev)
        out = torch.zeros(8, dtype=torch.int64, device=dev)
        leaf = torch.empty(n, dtype=torch.int32, device=dev)
        node_parent = torch.empty(max(n - 1, 1), dtype=torch.int32, device=dev)
        node_time = torch.empty(max(n - 1, 1), dtype=torch.int32, device=dev)
        sc = _scheme(kind, S, bits, interval)
        _check(lib.hstrat_phylo_tree_ex(ctypes.byref(sc), n, _vp(counter.data_ptr()),
                                        _vp(surface_words.data_ptr()), _vp(leaf.data_ptr()),
                                        _vp(node_parent.data_ptr()), _vp(node_time.data_ptr()),
                                        _vp(out.data_ptr()), _vp(ptr), need,
                                        _vp(_stream_handle(stream))))
        w = out.cpu().numpy().view(np.uint64)
        res = {"leaf_parent": as_u32(leaf), "node_parent": as_u32(node_parent)[:n - 1],
               "node_time": as_u32(node_time)[:n - 1]}
        del buf
    res.update(_phylo_result(w, n))
    res["T"] = int(counter[0].item()) & 0xFFFFFFFF
    return res


def newick(tree: dict) -> str:
    """Canonical Newick text of a phylo_tree result (formatted by the
    library's hstrat_phylo_newick): leaves are annotation indices, branch
    lengths generations, children ordered by the smallest annotation index
    below them, no length on the root."""
    lib = load_library()
    n = len(tree["leaf_parent"])
    leaf = np.ascontiguousarray(tree["leaf_parent"], np.uint32)
    npar = np.ascontiguousarray(tree["node_parent"], np.uint32)
    ntime = np.ascontiguousarray(tree["node_time"], np.uint32)
    length = ctypes.c_size_t()
    _check(lib.hstrat_phylo_newick(n, tree["T"], _ptr(leaf), _ptr(npar), _ptr(ntime), None, 0,
                                   ctypes.byref(length)))
    buf = ctypes.create_string_buffer(length.value + 1)
    _check(lib.hstrat_phylo_newick(n, tree["T"], _ptr(leaf), _ptr(npar), _ptr(ntime), buf,
                                   length.value + 1, ctypes.byref(length)))
    return buf.value.decode()

def layout(kind, S: int, T: int, bits: int = 1, interval: int = 1) -> np.ndarray:
    """Deposit generation held by each site of an annotation with counter T
    (host, constant time per site; EMPTY_SITE when unfilled)."""
    if isinstance(kind, str):
        kind = KINDS[kind]
    sc = _scheme(kind, S, bits, interval)
    L = np.zeros(S, np.uint32)
    _check(load_library().hstrat_layout(ctypes.byref(sc), T, _ptr(L)))
    return L


def sites(kind, S: int, tau0: int, n: int) -> np.ndarray:
    """Sites of the rule's items tau0 .. tau0 + n - 1 (host, constant time
    per item)."""
    if isinstance(kind, str):
        kind = KINDS[kind]
    sc = _scheme(kind, S, 1, 1)
    out = np.zeros(n, np.uint32)
    _check(load_library().hstrat_sites(ctypes.byref(sc), tau0, n, _ptr(out)))
    return out


def mrca_bounds_pair(kind, S: int, Ta: int, sa, Tb: int, sb, bits: int = 1,
                     interval: int = 1) -> tuple:
    """(lb, ub) of one pair of annotations on the host."""
    if isinstance(kind, str):
        kind = KINDS[kind]
    a = np.ascontiguousarray(sa, np.uint32)
    b = np.ascontiguousarray(sb, np.uint32)
    lb, ub = ctypes.c_uint32(), ctypes.c_uint32()
    lib = load_library()
    if bits == 1 and interval == 1:
        _check(lib.hstrat_mrca_bounds_pair(kind, S, Ta, _ptr(a), Tb, _ptr(b),
                                           ctypes.byref(lb), ctypes.byref(ub)))
    else:
        sc = _scheme(kind, S, bits, interval)
        _check(lib.hstrat_mrca_bounds_pair_ex(ctypes.byref(sc), Ta, _ptr(a), Tb, _ptr(b),
                                              ctypes.byref(lb), ctypes.byref(ub)))
    return lb.value, ub.value


def mrca_status(workspace: MrcaWorkspace, stream=None) -> int:
    rc = load_library().hstrat_mrca_status(_vp(workspace.ptr), _vp(_stream_handle(stream)))
    return rc


def probe_copy(src: torch.Tensor, dst: torch.Tensor, stream=None):
    """Plain 16-byte-per-lane device copy of src into dst (instrumentation)."""
    nbytes = min(src.numel() * src.element_size(), dst.numel() * dst.element_size()) & ~15
    _check(load_library().ga_probe_copy(_vp(src.data_ptr()), _vp(dst.data_ptr()), nbytes,
                                        _vp(_stream_handle(stream))))
    return nbytes


def as_u32(t: torch.Tensor) -> np.ndarray:
    """Device int32 tensor -> host numpy uint32 (bit-preserving)."""
    return t.detach().cpu().numpy().view(np.uint32)
