// hsga_pool.cpp -- batched and served runs (include/hsga.h, ga_pool_*): a
// first-fit allocator over the caller's arena, a device-resident run table,
// and one launch per generation for all active runs (optionally replayed
// from a captured hipGraph).  The per-run arithmetic is step_tile and
// schedule_sites, the same device code as the plain runs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <new>
#include <string>
#include <vector>

#include "hsga_host.hpp"

using namespace hsga_host;

namespace {

struct Slot {
    bool used = false;
    bool reported = false;
    uint32_t target = 0;   // generation count at which the run stops
    size_t off = 0, bytes = 0;
    ga_run run;
};

struct GraphKey {
    uint32_t nruns = 0, tiles = 0, gens = 0, block = 0;
    size_t lds = 0;
    bool with_float = false;
    bool operator==(const GraphKey& o) const {
        return nruns == o.nruns && tiles == o.tiles && gens == o.gens && block == o.block &&
               lds == o.lds && with_float == o.with_float;
    }
};

size_t table_bytes(uint32_t max_runs) {
    return align_up(sizeof(hsga::BatchRun) * max_runs) + align_up(4 * (size_t)(max_runs + 1));
}

}  // namespace

struct ga_pool {
    hipStream_t stream;
    uint8_t* arena;
    size_t arena_bytes;
    uint32_t max_runs, gens;
    hsga::BatchRun* d_table;
    uint32_t* d_tile0;
    size_t data_off;
    hsga::BatchRun* h_table;   // pinned staging
    uint32_t* h_tile0;         // pinned staging
    hipEvent_t staged;         // the last table upload has been consumed
    bool staged_pending;
    std::vector<Slot> slots;
    std::map<size_t, size_t> free_ranges;   // offset -> bytes, coalesced
    uint32_t block;
    bool use_graph;
    GraphKey key;
    hipGraphExec_t exec;
};

namespace {

void free_range(ga_pool* p, size_t off, size_t bytes) {
    auto it = p->free_ranges.emplace(off, bytes).first;
    auto next = std::next(it);
    if (next != p->free_ranges.end() && it->first + it->second == next->first) {
        it->second += next->second;
        p->free_ranges.erase(next);
    }
    if (it != p->free_ranges.begin()) {
        auto prev = std::prev(it);
        if (prev->first + prev->second == it->first) {
            prev->second += it->second;
            p->free_ranges.erase(it);
        }
    }
}

bool take_range(ga_pool* p, size_t bytes, size_t* off) {
    for (auto it = p->free_ranges.begin(); it != p->free_ranges.end(); ++it) {
        if (it->second >= bytes) {
            *off = it->first;
            const size_t rest = it->second - bytes;
            const size_t at = it->first + bytes;
            p->free_ranges.erase(it);
            if (rest) p->free_ranges.emplace(at, rest);
            return true;
        }
    }
    return false;
}

void drop_graph(ga_pool* p) {
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    p->exec = nullptr;
    p->key = GraphKey{};
}

uint32_t variant_of(const ga_run& r) {
    uint32_t v = 0;
    if (r.SW == 2) v |= 1u;
    v |= birth_model(r.cfg) << 1;
    if (r.cfg.migrants_per_island) v |= 8u;
    const uint32_t apt_log2 = r.apt == 4 ? 2u : (r.apt == 2 ? 1u : 0u);
    return v | (apt_log2 << 4);
}

int enqueue_launches(ga_pool* p, uint32_t nruns, uint32_t tiles, uint32_t gens, size_t lds,
                     bool with_float) {
    hipError_t e = hsga::launch_batch_sites(p->d_table, nruns, gens, p->stream);
    if (e != hipSuccess) return hip_fail(e, "batched site schedule launch");
    for (uint32_t k = 0; k < gens; ++k) {
        e = hsga::launch_batch_step(p->d_table, p->d_tile0, nruns, tiles, k, p->block, lds,
                                    with_float, p->stream);
        if (e != hipSuccess) return hip_fail(e, "batched step launch");
    }
    return GA_OK;
}

}  // namespace

extern "C" {

size_t ga_pool_overhead_bytes(uint32_t max_runs) { return table_bytes(max_runs); }

int ga_pool_create(void* dev_arena, size_t arena_bytes, uint32_t max_runs,
                   uint32_t max_gens_per_launch, void* hip_stream, ga_pool** out) {
    if (!out) return fail(GA_EINVAL, "out is NULL");
    *out = nullptr;
    if (!dev_arena || (uintptr_t)dev_arena % kAlign)
        return fail(GA_EINVAL, "arena NULL or not 256-byte aligned");
    if (max_runs == 0 || max_runs > hsga::kMaxBatchRuns)
        return fail(GA_EINVAL, "max_runs must be 1..256");
    const size_t over = table_bytes(max_runs);
    if (arena_bytes < over) return fail(GA_ENOMEM, "arena smaller than the pool's tables");
    ga_pool* p = new (std::nothrow) ga_pool();
    if (!p) return fail(GA_ENOMEM, "host allocation failed");
    p->stream = static_cast<hipStream_t>(hip_stream);
    p->arena = static_cast<uint8_t*>(dev_arena);
    p->arena_bytes = arena_bytes;
    p->max_runs = max_runs;
    p->gens = max_gens_per_launch ? max_gens_per_launch : kDefaultGens;
    p->d_table = reinterpret_cast<hsga::BatchRun*>(p->arena);
    p->d_tile0 = reinterpret_cast<uint32_t*>(p->arena +
                                             align_up(sizeof(hsga::BatchRun) * max_runs));
    p->data_off = over;
    p->slots.resize(max_runs);
    if (arena_bytes > over) p->free_ranges.emplace(over, arena_bytes - over);
    p->block = 64;
    p->use_graph = false;
    p->exec = nullptr;
    p->staged_pending = false;
    hipError_t e = hipHostMalloc(reinterpret_cast<void**>(&p->h_table),
                                 sizeof(hsga::BatchRun) * max_runs, hipHostMallocDefault);
    if (e != hipSuccess) {
        delete p;
        return hip_fail(e, "hipHostMalloc table staging");
    }
    e = hipHostMalloc(reinterpret_cast<void**>(&p->h_tile0), 4 * (size_t)(max_runs + 1),
                      hipHostMallocDefault);
    if (e != hipSuccess) {
        (void)hipHostFree(p->h_table);
        delete p;
        return hip_fail(e, "hipHostMalloc tile staging");
    }
    e = hipEventCreateWithFlags(&p->staged, hipEventDisableTiming);
    if (e != hipSuccess) {
        (void)hipHostFree(p->h_table);
        (void)hipHostFree(p->h_tile0);
        delete p;
        return hip_fail(e, "hipEventCreate");
    }
    *out = p;
    return GA_OK;
}

size_t ga_pool_footprint(const ga_pool* p, const ga_config* in) {
    ga_config cfg;
    if (!p || validate(in, &cfg) != GA_OK) return 0;
    return carve(cfg, p->gens).total;
}

int ga_pool_admit(ga_pool* p, const ga_config* in, uint32_t n_generations, uint32_t* id) {
    if (!p || !id) return fail(GA_EINVAL, "NULL argument");
    ga_config cfg_copy;
    int rc = validate(in, &cfg_copy);
    const ga_config* cfg = &cfg_copy;
    if (rc != GA_OK) return rc;
    if (n_generations == 0) return fail(GA_EINVAL, "a run needs at least one generation");
    if (cfg->async_activity)
        return fail(GA_EINVAL, "asynchronous runs use the plain API, not a pool");
    if ((uint64_t)n_generations - 1 >
        hsga::horizon_gen_of(cfg->surface_kind, cfg->surface_sites, cfg->ingest_interval))
        return fail(GA_EHORIZON, "generation count past the site rule's horizon");
    uint32_t slot = p->max_runs;
    for (uint32_t s = 0; s < p->max_runs; ++s)
        if (!p->slots[s].used) {
            slot = s;
            break;
        }
    if (slot == p->max_runs) return fail(GA_EBUSY, "no free run slot");
    const size_t need = ga_pool_footprint(p, cfg);
    size_t off = 0;
    if (!take_range(p, need, &off)) return fail(GA_EBUSY, "no free range of the run's footprint");
    Slot& s = p->slots[slot];
    s.run = ga_run();
    rc = run_init(&s.run, cfg, p->arena + off, p->gens, p->stream);
    if (rc != GA_OK) {
        free_range(p, off, need);
        return rc;
    }
    s.run.block = p->block;
    s.run.pooled = true;
    s.used = true;
    s.reported = false;
    s.target = n_generations;
    s.off = off;
    s.bytes = need;
    *id = slot;
    return GA_OK;
}

int ga_pool_advance(ga_pool* p, uint32_t max_gens, uint32_t* gens_enqueued) {
    if (!p) return fail(GA_EINVAL, "pool is NULL");
    if (gens_enqueued) *gens_enqueued = 0;
    const uint32_t G = std::min(max_gens, p->gens);
    if (G == 0) return GA_OK;
    std::vector<uint32_t> active;
    for (uint32_t s = 0; s < p->max_runs; ++s)
        if (p->slots[s].used && p->slots[s].run.T < p->slots[s].target) active.push_back(s);
    if (active.empty()) return GA_OK;
    // runs of one kernel specialisation side by side: their tiles run
    // together on the CUs, which then share one variant's code in the
    // instruction cache (the order changes no result)
    std::stable_sort(active.begin(), active.end(), [&](uint32_t a, uint32_t b) {
        return variant_of(p->slots[a].run) < variant_of(p->slots[b].run);
    });
    if (p->staged_pending) {
        hipError_t e = hipEventSynchronize(p->staged);
        if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
        p->staged_pending = false;
    }
    uint32_t tiles = 0, gens = 0;
    size_t lds = 0;
    bool with_float = false;
    const uint32_t nruns = (uint32_t)active.size();
    for (uint32_t i = 0; i < nruns; ++i) {
        Slot& s = p->slots[active[i]];
        ga_run& r = s.run;
        r.block = p->block;
        const uint32_t g = std::min(G, s.target - r.T);
        const hsga::StepParams sp = step_params(&r, r.T, hsga::ingests_of(r.T, r.cfg.ingest_interval));
        // the island pass takes one island per thread
        if (sp.tile_isl == 0 || sp.tile_isl > p->block)
            return fail(GA_EINVAL, "tile has more islands than the workgroup has threads");
        hsga::BatchRun& b = p->h_table[i];
        for (int q = 0; q < 2; ++q) {
            b.trait[q] = r.trait[q];
            b.counter[q] = r.counter[q];
            b.surf[q] = r.surf[q];
            b.outbox[q] = r.outbox[q];
        }
        b.sites = r.sites;
        b.layout = r.layout;
        b.rules = r.rules;
        b.W = sp.W; b.H = sp.H; b.N = sp.N; b.I = sp.I; b.A = sp.A;
        b.T0 = r.T;
        b.gens = g;
        b.k0 = sp.k0; b.k1 = sp.k1;
        b.mut_thr = sp.mut_thr; b.mut_lo = sp.mut_lo; b.mut_span = sp.mut_span;
        b.kind = r.cfg.surface_kind;
        b.S = r.S;
        b.variant = variant_of(r);
        with_float = with_float || birth_model(r.cfg) == hsga::kBirthFloat;
        b.tour = sp.tour;
        b.del_thr = sp.del_thr; b.ben_thr = sp.ben_thr;
        b.del_sigma = sp.del_sigma; b.ben_sigma = sp.ben_sigma;
        b.interval = r.cfg.ingest_interval;
        b.diff_log2 = sp.diff_log2;
        b.tile_isl = sp.tile_isl;
        b.div_magic = sp.div_magic;
        b.w_magic = sp.w_magic;
        b.w_shift = sp.w_shift;
        b.tile0 = tiles;
        p->h_tile0[i] = tiles;
        const uint32_t rt = (r.I + sp.tile_isl - 1) / sp.tile_isl;
        tiles += rt;
        gens = std::max(gens, g);
        lds = std::max(lds, hsga::step_lds_bytes(sp.tile_isl, r.N, r.SW,
                                                 birth_model(r.cfg) == hsga::kBirthFloat,
                                                 p->block, r.apt));
    }
    if (lds > kMaxStepLds) return fail(GA_EINVAL, "batched tiles need more than 64 KiB of LDS");
    p->h_tile0[nruns] = tiles;
    hipError_t e = hipMemcpyAsync(p->d_table, p->h_table, sizeof(hsga::BatchRun) * nruns,
                                  hipMemcpyHostToDevice, p->stream);
    if (e != hipSuccess) return hip_fail(e, "table upload");
    e = hipMemcpyAsync(p->d_tile0, p->h_tile0, 4 * (size_t)(nruns + 1), hipMemcpyHostToDevice,
                       p->stream);
    if (e != hipSuccess) return hip_fail(e, "tile table upload");
    e = hipEventRecord(p->staged, p->stream);
    if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
    p->staged_pending = true;

    const GraphKey key{nruns, tiles, gens, p->block, lds, with_float};
    int rc = GA_OK;
    if (p->use_graph && p->stream) {
        if (!(p->exec && p->key == key)) {
            drop_graph(p);
            e = hipStreamBeginCapture(p->stream, hipStreamCaptureModeThreadLocal);
            if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
            rc = enqueue_launches(p, nruns, tiles, gens, lds, with_float);
            hipGraph_t graph = nullptr;
            e = hipStreamEndCapture(p->stream, &graph);
            if (rc != GA_OK) {
                if (graph) (void)hipGraphDestroy(graph);
                return rc;
            }
            if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
            e = hipGraphInstantiate(&p->exec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            if (e != hipSuccess) {
                p->exec = nullptr;
                return hip_fail(e, "hipGraphInstantiate");
            }
            p->key = key;
        }
        e = hipGraphLaunch(p->exec, p->stream);
        if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
    } else {
        rc = enqueue_launches(p, nruns, tiles, gens, lds, with_float);
        if (rc != GA_OK) return rc;
    }
    for (uint32_t i = 0; i < nruns; ++i) {
        Slot& s = p->slots[active[i]];
        s.run.T += p->h_table[i].gens;
    }
    if (gens_enqueued) *gens_enqueued = gens;
    return GA_OK;
}

int ga_pool_poll(ga_pool* p, uint32_t* ids, uint32_t cap, uint32_t* n) {
    if (!p || !n || (cap && !ids)) return fail(GA_EINVAL, "NULL argument");
    uint32_t k = 0;
    for (uint32_t s = 0; s < p->max_runs && k < cap; ++s) {
        Slot& sl = p->slots[s];
        if (sl.used && !sl.reported && sl.run.T >= sl.target) {
            sl.reported = true;
            ids[k++] = s;
        }
    }
    *n = k;
    return GA_OK;
}

int ga_pool_run(ga_pool* p, uint32_t id, ga_run** run) {
    if (!p || !run) return fail(GA_EINVAL, "NULL argument");
    if (id >= p->max_runs || !p->slots[id].used) return fail(GA_EINVAL, "no such run");
    *run = &p->slots[id].run;
    return GA_OK;
}

int ga_pool_release(ga_pool* p, uint32_t id) {
    if (!p) return fail(GA_EINVAL, "pool is NULL");
    if (id >= p->max_runs || !p->slots[id].used) return fail(GA_EINVAL, "no such run");
    Slot& s = p->slots[id];
    free_range(p, s.off, s.bytes);
    s.used = false;
    s.reported = false;
    return GA_OK;
}

int ga_pool_sync(ga_pool* p) {
    if (!p) return fail(GA_EINVAL, "pool is NULL");
    hipError_t e = hipStreamSynchronize(p->stream);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    p->staged_pending = false;
    return GA_OK;
}

int ga_pool_set_launch(ga_pool* p, uint32_t block_threads, int use_graph) {
    if (!p) return fail(GA_EINVAL, "pool is NULL");
    if (block_threads) {
        if (block_threads % 64 || block_threads > 256)
            return fail(GA_EINVAL, "block_threads must be a multiple of 64, at most 256");
        p->block = block_threads;
    }
    if (use_graph && !p->stream)
        return fail(GA_EINVAL, "graph replay needs a created stream, not the null stream");
    p->use_graph = use_graph != 0;
    if (!p->use_graph) drop_graph(p);
    return GA_OK;
}

int ga_pool_info(const ga_pool* p, uint32_t* active, uint32_t* admitted, size_t* free_bytes,
                 size_t* largest_free) {
    if (!p) return fail(GA_EINVAL, "pool is NULL");
    uint32_t a = 0, u = 0;
    for (const Slot& s : p->slots) {
        if (!s.used) continue;
        ++u;
        if (s.run.T < s.target) ++a;
    }
    size_t fb = 0, lf = 0;
    for (const auto& fr : p->free_ranges) {
        fb += fr.second;
        lf = std::max(lf, fr.second);
    }
    if (active) *active = a;
    if (admitted) *admitted = u;
    if (free_bytes) *free_bytes = fb;
    if (largest_free) *largest_free = lf;
    return GA_OK;
}

void ga_pool_destroy(ga_pool* p) {
    if (!p) return;
    drop_graph(p);
    (void)hipEventDestroy(p->staged);
    (void)hipHostFree(p->h_table);
    (void)hipHostFree(p->h_tile0);
    delete p;
}

}  // extern "C"
