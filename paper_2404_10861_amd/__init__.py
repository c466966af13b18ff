"""MI355X-native island-model GA with hereditary-stratigraphy surface
annotations (Moreno et al., "Trackable Agent-based Evolution Models at Wafer
Scale").  The kernels live in libhsga.so (csrc/, C ABI in include/hsga.h);
``binding`` marshals arguments to it from Python."""
from .binding import (  # noqa: F401
    Config, Run, RunHandle, Pool, PoolRun, pool_overhead_bytes, MrcaWorkspace, HsgaError, mrca_bounds, mrca_status, phylo_metrics, phylo_tree, newick, footprint_bytes,
    load_library, as_u32, probe_copy, KINDS, STEADY, TILTED, HYBRID, EMPTY_SITE, EXPORTS,
    layout, sites, mrca_bounds_pair,
    GA_OK, GA_EINVAL, GA_ENOMEM, GA_EHORIZON, GA_EDEVICE, GA_EBUSY,
)
