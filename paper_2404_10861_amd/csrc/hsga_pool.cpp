// hsga_pool.cpp -- batched and served runs (include/hsga.h, ga_pool_*): a
// first-fit allocator over the caller's arena, a device-resident run table,
// and per generation one launch per group of active runs, the groups on
// streams of their own that run side by side (optionally replayed from
// captured hipGraphs).  The per-run arithmetic is step_tile and run_sites,
// the same device code as the plain runs.
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

// An advance cuts the active runs, in table order, into kGroups
// contiguous groups of about equal bytes per generation and gives each
// group one launch per generation on a stream of its own.  The groups'
// runs are independent, so the streams run side by side and one group's
// launch tail (its last, partly filled wave of workgroups, and the gap
// before its next launch) overlaps the others' work.  Only generations
// that read at least kSplitWords trait and surface words are split: below
// that a launch is short, its tail small, and the second launch per
// generation costs more than it hides (a served run set, about 0.5 M words
// per generation, had its median latency 10 % longer split in two; the
// treatment pair, 16.8 M words, and the 64-run batch, 55 M, gain).
// ga_pool_set_split changes the threshold.
constexpr uint32_t kGroups = 2;
constexpr uint64_t kSplitWords = 1u << 22;

// The runs of one launch: table entries first .. first + count - 1, and
// their tiles' workgroups dealt over the XCDs in the xcd table from word
// 2 * kXcds * first on.
struct Group {
    uint32_t first = 0, count = 0, tiles = 0;
    size_t lds = 0;
    bool with_float = false;
    bool operator==(const Group& o) const {
        return first == o.first && count == o.count && tiles == o.tiles && lds == o.lds &&
               with_float == o.with_float;
    }
};

// One advance's launches (a group may be empty).
struct GraphKey {
    Group grp[kGroups];
    uint32_t gens = 0, block = 0;
    bool operator==(const GraphKey& o) const {
        for (uint32_t q = 0; q < kGroups; ++q)
            if (!(grp[q] == o.grp[q])) return false;
        return gens == o.gens && block == o.block;
    }
};

// words of the xcd tables (launch_batch_step) of up to max_runs runs
size_t xcd_words(uint32_t max_runs) { return 2 * (size_t)hsga::kXcds * max_runs; }

// the run table, then the xcd tables
size_t table_bytes(uint32_t max_runs) {
    return align_up(sizeof(hsga::BatchRun) * max_runs) + align_up(4 * xcd_words(max_runs));
}

}  // namespace

struct ga_pool {
    hipStream_t stream;
    hipStream_t side[kGroups - 1];   // groups 1.. launch here
    hipEvent_t fork;                 // the sides wait for stream
    hipEvent_t join[kGroups - 1];    // then stream for each side
    uint8_t* arena;
    size_t arena_bytes;
    uint32_t max_runs, gens;
    hsga::BatchRun* d_table;
    uint32_t* d_xtab;          // the groups' xcd tables
    size_t data_off;
    hsga::BatchRun* h_table;   // pinned staging
    uint32_t* h_xtab;          // pinned staging
    hipEvent_t staged;         // the last table upload has been consumed
    bool staged_pending;
    std::vector<Slot> slots;
    std::map<size_t, size_t> free_ranges;   // offset -> bytes, coalesced
    uint32_t block;
    bool use_graph;
    GraphKey key;
    bool captured;                   // exec holds key's launches
    bool broken;                     // an advance failed after enqueueing work
    uint64_t split_words;            // generations from this size on are split
    hipGraphExec_t exec[kGroups];    // each group's launches, replayed on its stream
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
    for (hipGraphExec_t& x : p->exec) {
        if (x) (void)hipGraphExecDestroy(x);
        x = nullptr;
    }
    p->key = GraphKey{};
    p->captured = false;
}

void release_handles(ga_pool* p) {
    for (hipStream_t& x : p->side)
        if (x) (void)hipStreamDestroy(x);
    for (hipEvent_t& x : p->join)
        if (x) (void)hipEventDestroy(x);
    if (p->fork) (void)hipEventDestroy(p->fork);
    if (p->staged) (void)hipEventDestroy(p->staged);
    (void)hipHostFree(p->h_xtab);
    (void)hipHostFree(p->h_table);
}

// words a run reads or writes per agent and generation: its trait and
// surface words, in and out (the balance of the launch groups)
uint64_t words_per_generation(const ga_run& r) { return (uint64_t)r.A * (1 + r.SW); }

uint32_t variant_of(const ga_run& r) {
    uint32_t v = 0;
    if (r.SW == 2) v |= 1u;
    v |= birth_model(r.cfg) << 1;
    if (r.cfg.migrants_per_island) v |= 8u;
    const uint32_t apt_log2 = r.apt == 4 ? 2u : (r.apt == 2 ? 1u : 0u);
    return v | (apt_log2 << 4);
}

hipStream_t stream_of(const ga_pool* p, uint32_t q) { return q ? p->side[q - 1] : p->stream; }

hipError_t launch_group(ga_pool* p, const GraphKey& key, uint32_t q, uint32_t k) {
    const Group& g = key.grp[q];
    return hsga::launch_batch_step(p->d_table + g.first, p->d_xtab + xcd_words(g.first), g.count,
                                   g.tiles, k, p->block, g.lds, g.with_float, stream_of(p, q));
}

// Group q's launches of every generation, captured on its stream into
// exec[q]: one linear graph per stream.
int capture_group(ga_pool* p, const GraphKey& key, uint32_t q) {
    const hipStream_t s = stream_of(p, q);
    hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
    hipError_t le = hipSuccess;
    for (uint32_t k = 0; k < key.gens && le == hipSuccess; ++k) le = launch_group(p, key, q, k);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(s, &graph);
    if (le == hipSuccess && e == hipSuccess)
        e = hipGraphInstantiate(&p->exec[q], graph, nullptr, nullptr, 0);
    if (graph) (void)hipGraphDestroy(graph);
    if (le != hipSuccess || e != hipSuccess) {
        p->exec[q] = nullptr;
        return hip_fail(le != hipSuccess ? le : e, "capture of the batched launches");
    }
    return GA_OK;
}

// The site schedules of all runs on the pool's stream, then the groups'
// launches, groups 1.. on the side streams: forked after the schedules and
// joined back at the end, so that work enqueued on the pool's stream later
// sees the whole advance.  Replayed, each stream replays its own group's
// graph.
int enqueue_launches(ga_pool* p, const GraphKey& key) {
    uint32_t nruns = 0;
    for (const Group& g : key.grp) nruns += g.count;
    hipError_t e = hsga::launch_batch_sites(p->d_table, nruns, key.gens, p->stream);
    if (e != hipSuccess) return hip_fail(e, "batched site schedule launch");
    const bool graph = p->use_graph && p->stream;
    if (graph && !(p->captured && p->key == key)) {
        drop_graph(p);
        for (uint32_t q = 0; q < kGroups; ++q) {
            if (key.grp[q].count == 0) continue;
            const int rc = capture_group(p, key, q);
            if (rc != GA_OK) {
                drop_graph(p);
                return rc;
            }
        }
        p->key = key;
        p->captured = true;
    }
    bool forked = false;
    for (uint32_t q = 1; q < kGroups; ++q) {
        if (key.grp[q].count == 0) continue;
        if (!forked) {
            e = hipEventRecord(p->fork, p->stream);
            if (e != hipSuccess) return hip_fail(e, "fork to the side streams");
            forked = true;
        }
        e = hipStreamWaitEvent(p->side[q - 1], p->fork, 0);
        if (e != hipSuccess) return hip_fail(e, "fork to the side streams");
    }
    hipError_t le = hipSuccess;
    if (graph) {
        for (uint32_t q = 0; q < kGroups && le == hipSuccess; ++q)
            if (key.grp[q].count) le = hipGraphLaunch(p->exec[q], stream_of(p, q));
    } else {
        for (uint32_t k = 0; k < key.gens && le == hipSuccess; ++k)
            for (uint32_t q = 0; q < kGroups && le == hipSuccess; ++q)
                if (key.grp[q].count) le = launch_group(p, key, q, k);
    }
    // joined even after a failed launch, so that the pool's stream orders
    // whatever was enqueued
    for (uint32_t q = 1; q < kGroups; ++q) {
        if (key.grp[q].count == 0) continue;
        e = hipEventRecord(p->join[q - 1], p->side[q - 1]);
        if (e == hipSuccess) e = hipStreamWaitEvent(p->stream, p->join[q - 1], 0);
        if (e != hipSuccess) return hip_fail(e, "join from the side streams");
    }
    if (le != hipSuccess) return hip_fail(le, graph ? "hipGraphLaunch" : "batched step launch");
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
    p->d_xtab = reinterpret_cast<uint32_t*>(p->arena +
                                            align_up(sizeof(hsga::BatchRun) * max_runs));
    p->data_off = over;
    p->slots.resize(max_runs);
    if (arena_bytes > over) p->free_ranges.emplace(over, arena_bytes - over);
    p->block = 64;
    p->use_graph = false;
    p->captured = false;
    p->broken = false;
    p->split_words = kSplitWords;
    p->staged_pending = false;
    hipError_t e = hipHostMalloc(reinterpret_cast<void**>(&p->h_table),
                                 sizeof(hsga::BatchRun) * max_runs, hipHostMallocDefault);
    if (e != hipSuccess) {
        delete p;
        return hip_fail(e, "hipHostMalloc table staging");
    }
    e = hipHostMalloc(reinterpret_cast<void**>(&p->h_xtab), 4 * xcd_words(max_runs),
                      hipHostMallocDefault);
    if (e != hipSuccess) {
        (void)hipHostFree(p->h_table);
        delete p;
        return hip_fail(e, "hipHostMalloc tile staging");
    }
    e = hipEventCreateWithFlags(&p->staged, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&p->fork, hipEventDisableTiming);
    for (uint32_t q = 0; q + 1 < kGroups && e == hipSuccess; ++q) {
        e = hipEventCreateWithFlags(&p->join[q], hipEventDisableTiming);
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&p->side[q], hipStreamNonBlocking);
    }
    if (e != hipSuccess) {
        release_handles(p);
        delete p;
        return hip_fail(e, "pool event or stream creation");
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
    if (p->broken) return fail(GA_EDEVICE, "an earlier advance failed part-way");
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
    // the groups: run i joins the group its bytes' midpoint falls in (the
    // lower one on a boundary, so that a lone run stays on the pool's
    // stream)
    uint64_t total_words = 0;
    for (uint32_t s : active) total_words += words_per_generation(p->slots[s].run);
    const uint32_t groups = total_words >= p->split_words ? kGroups : 1u;
    if (p->staged_pending) {
        hipError_t e = hipEventSynchronize(p->staged);
        if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
        p->staged_pending = false;
    }
    GraphKey key;
    key.block = p->block;
    const uint32_t nruns = (uint32_t)active.size();
    std::vector<uint32_t> run_tiles(nruns);
    uint64_t words_before = 0;
    for (uint32_t i = 0; i < nruns; ++i) {
        Slot& s = p->slots[active[i]];
        ga_run& r = s.run;
        const uint64_t w = words_per_generation(r);
        const uint32_t q = (uint32_t)std::min<uint64_t>(
            groups - 1, ((2 * words_before + w) * groups - 1) / (2 * total_words));
        words_before += w;
        Group& grp = key.grp[q];
        r.block = p->block;
        const uint32_t g = std::min(G, s.target - r.T);
        const hsga::StepParams sp =
            step_params(&r, r.T, hsga::ingests_of(r.T, r.cfg.ingest_interval));
        // the island pass takes one island per thread
        if (sp.tile_isl == 0 || sp.tile_isl > p->block)
            return fail(GA_EINVAL, "tile has more islands than the workgroup has threads");
        hsga::BatchRun& b = p->h_table[i];
        for (int j = 0; j < 2; ++j) {
            b.trait[j] = r.trait[j];
            b.counter[j] = r.counter[j];
            b.surf[j] = r.surf[j];
            b.outbox[j] = r.outbox[j];
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
        grp.with_float = grp.with_float || birth_model(r.cfg) == hsga::kBirthFloat;
        b.tour = sp.tour;
        b.del_thr = sp.del_thr; b.ben_thr = sp.ben_thr;
        b.del_sigma = sp.del_sigma; b.ben_sigma = sp.ben_sigma;
        b.interval = r.cfg.ingest_interval;
        b.diff_log2 = sp.diff_log2;
        b.tile_isl = sp.tile_isl;
        b.div_magic = sp.div_magic;
        b.w_magic = sp.w_magic;
        b.w_shift = sp.w_shift;
        const uint32_t rt = (r.I + sp.tile_isl - 1) / sp.tile_isl;
        run_tiles[i] = rt;
        grp.tiles += rt;
        ++grp.count;
        key.gens = std::max(key.gens, g);
        grp.lds = std::max(grp.lds, hsga::step_lds_bytes(sp.tile_isl, r.N, r.SW,
                                                         birth_model(r.cfg) == hsga::kBirthFloat,
                                                         p->block, r.apt));
    }
    // each group's xcd table, group after group
    uint32_t first = 0;
    for (uint32_t q = 0; q < kGroups; ++q) {
        Group& grp = key.grp[q];
        if (grp.lds > kMaxStepLds)
            return fail(GA_EINVAL, "batched tiles need more than 64 KiB of LDS");
        grp.first = first;
        if (!hsga::deal_tiles(run_tiles.data() + first, grp.count, grp.tiles,
                        p->h_xtab + xcd_words(first)))
            return fail(GA_EINVAL, "tiles could not be dealt over the XCDs");
        first += grp.count;
    }
    hipError_t e = hipMemcpyAsync(p->d_table, p->h_table, sizeof(hsga::BatchRun) * nruns,
                                  hipMemcpyHostToDevice, p->stream);
    if (e != hipSuccess) return hip_fail(e, "table upload");
    e = hipMemcpyAsync(p->d_xtab, p->h_xtab, 4 * xcd_words(nruns), hipMemcpyHostToDevice,
                       p->stream);
    if (e != hipSuccess) return hip_fail(e, "tile table upload");
    e = hipEventRecord(p->staged, p->stream);
    if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
    p->staged_pending = true;

    const int rc = enqueue_launches(p, key);
    if (rc != GA_OK) {
        // some of the runs' generations may be enqueued while their
        // generation counts stay: no later advance can be consistent
        p->broken = true;
        return rc;
    }
    for (uint32_t i = 0; i < nruns; ++i) {
        Slot& s = p->slots[active[i]];
        s.run.T += p->h_table[i].gens;
    }
    if (gens_enqueued) *gens_enqueued = key.gens;
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

int ga_pool_set_split(ga_pool* p, uint64_t min_words) {
    if (!p) return fail(GA_EINVAL, "pool is NULL");
    p->split_words = min_words;
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
    (void)hipStreamSynchronize(p->stream);
    drop_graph(p);
    release_handles(p);
    delete p;
}

}  // extern "C"
