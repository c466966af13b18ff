// hsga_api.cpp -- the C ABI of libhsga.so (include/hsga.h): configuration
// checks, arena carving, launch sequencing and error reporting.  All
// arithmetic of the method runs in the kernels of hsga_kernels.hip; this
// file only validates, carves memory and enqueues.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstddef>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "hsga_host.hpp"

namespace hsga_host {

namespace {
thread_local std::string g_last_error;
}

int fail(int status, const std::string& msg) {
    g_last_error = msg;
    return status;
}

int hip_fail(hipError_t e, const char* what) {
    return fail(GA_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

const char* last_error() { return g_last_error.c_str(); }

Carve carve(const ga_config& cfg, uint32_t gens) {
    const size_t I = (size_t)cfg.grid_w * cfg.grid_h;
    const size_t A = I * cfg.pop_per_island;
    const size_t SW = surface_words(cfg);
    Carve c;
    size_t off = 0;
    c.trait = off;   off += 2 * align_up(A * 4);
    c.counter = 0;
    if (cfg.async_activity) {
        c.counter = off;
        off += 2 * align_up(A * 4);
    }
    c.surf = off;    off += 2 * align_up(SW * A * 4);
    c.outbox = off;  off += 2 * align_up((size_t)I * hsga::kOutboxWords * 4);
    c.layout = off;  off += align_up(64 * 4);
    c.rules = off;   off += align_up(2 * sizeof(hsga::RuleTable));
    c.sites = off;
    off += cfg.async_activity ? 4 * hsga::kSiteRing : align_up((size_t)gens * 4);
    c.total = off;
    return c;
}

int validate(const ga_config* in, ga_config* out) {
    if (!in) return fail(GA_EINVAL, "config is NULL");
    constexpr uint32_t kIntOnlySize = offsetof(ga_config, fitness_model);
    constexpr uint32_t kSyncOnlySize = offsetof(ga_config, async_activity);
    if (in->struct_size != sizeof(ga_config) && in->struct_size != kIntOnlySize &&
        in->struct_size != kSyncOnlySize)
        return fail(GA_EINVAL, "config struct_size does not match this library");
    ga_config c;
    std::memset(&c, 0, sizeof c);
    std::memcpy(&c, in, in->struct_size);
    c.struct_size = sizeof(ga_config);
    const ga_config* cfg = &c;
    if (cfg->grid_w == 0 || cfg->grid_h == 0) return fail(GA_EINVAL, "empty torus");
    if (cfg->grid_w > 65535 || cfg->grid_h > 65535)
        return fail(GA_EINVAL, "torus side above 65535 islands");
    if (cfg->pop_per_island == 0 || cfg->pop_per_island > 64)
        return fail(GA_EINVAL, "pop_per_island must be 1..64");
    const uint64_t A = (uint64_t)cfg->grid_w * cfg->grid_h * cfg->pop_per_island;
    if (A > (1ull << 30)) return fail(GA_EINVAL, "more than 2^30 agents");
    if (c.differentia_bits == 0) c.differentia_bits = 1;
    if (c.ingest_interval == 0) c.ingest_interval = 1;
    if (cfg->differentia_bits != 1 && cfg->differentia_bits != 8)
        return fail(GA_EINVAL, "differentia_bits must be 1 or 8");
    if (cfg->surface_sites * cfg->differentia_bits != 32 &&
        cfg->surface_sites * cfg->differentia_bits != 64)
        return fail(GA_EINVAL, "surface_sites * differentia_bits must be 32 or 64");
    if (cfg->surface_kind > GA_HYBRID) return fail(GA_EINVAL, "unknown surface kind");
    if (cfg->fitness_model > GA_FOUNDER_TAG) return fail(GA_EINVAL, "unknown fitness model");
    if (cfg->fitness_model == GA_FOUNDER_TAG && cfg->tournament_size != 0)
        return fail(GA_EINVAL, "founder tags need neutral selection (tournament_size 0)");
    if (cfg->fitness_model == GA_INT_TRAIT) {
        if (cfg->tournament_size != 0 && cfg->tournament_size != 2)
            return fail(GA_EINVAL, "tournament_size must be 2 (tournament) or 0 (neutral)");
        if (cfg->mut_lo > cfg->mut_hi) return fail(GA_EINVAL, "mut_lo > mut_hi");
        if ((int64_t)cfg->mut_hi - cfg->mut_lo + 1 > 0xffffffffll)
            return fail(GA_EINVAL, "mutation range wider than 2^32 - 1");
    } else {
        if (cfg->tournament_size > 5) return fail(GA_EINVAL, "tournament_size must be 0..5");
        if ((uint64_t)cfg->del_threshold + cfg->ben_threshold > (1ull << 32))
            return fail(GA_EINVAL, "deleterious and beneficial thresholds sum above 2^32");
        if (!(cfg->del_sigma >= 0.0f && cfg->del_sigma <= 1048576.0f) ||
            !(cfg->ben_sigma >= 0.0f && cfg->ben_sigma <= 1048576.0f))
            return fail(GA_EINVAL, "mutation scales must lie in [0, 2^20]");
    }
    if (cfg->migrants_per_island > 1) return fail(GA_EINVAL, "migrants_per_island must be 0 or 1");
    if (cfg->reserved != 0) return fail(GA_EINVAL, "reserved must be 0");
    if (out) *out = c;
    return GA_OK;
}

namespace {
// Pinned host copies of the cached rule tables, made on first use and kept
// until the process ends, so that a query's upload of them is an ordinary
// stream copy (a copy from pageable memory may hold the host until the
// stream has drained).  Pageable tables when pinned memory is refused.
std::mutex g_pinned_mutex;
std::vector<std::pair<const hsga::RuleTable*, hsga::RuleTable*>> g_pinned;

const hsga::RuleTable* pinned_table(const hsga::RuleTable* t) {
    std::lock_guard<std::mutex> lock(g_pinned_mutex);
    for (auto& pr : g_pinned)
        if (pr.first == t) return pr.second ? pr.second : t;
    void* p = nullptr;
    if (hipHostMalloc(&p, sizeof(hsga::RuleTable), hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        p = nullptr;
    } else {
        std::memcpy(p, t, sizeof(hsga::RuleTable));
    }
    g_pinned.emplace_back(t, static_cast<hsga::RuleTable*>(p));
    return p ? static_cast<hsga::RuleTable*>(p) : t;
}

}  // namespace

// Enqueue the upload of the tables of a surface of `kind` and S sites (one,
// or two for hybrid) to dev on `stream`, from the pinned host copies.
hipError_t upload_tables(uint32_t kind, uint32_t S, hsga::RuleTable* dev, hipStream_t stream) {
    const hsga::RuleTable* tabs[2] = {nullptr, nullptr};
    if (!hsga::scheme_rules(kind, S, tabs)) return hipErrorInvalidValue;
    for (int k = 0; k < 2 && tabs[k]; ++k) {
        hipError_t e = hipMemcpyAsync(dev + k, pinned_table(tabs[k]), sizeof(hsga::RuleTable),
                                      hipMemcpyHostToDevice, stream);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

namespace {
uint32_t default_agents_per_thread(uint32_t N) {
    return N % 4 == 0 ? 4u : (N % 2 == 0 ? 2u : 1u);
}
}  // namespace

int run_init(ga_run* r, const ga_config* cfg, uint8_t* base, uint32_t gens, hipStream_t stream) {
    const uint32_t I = cfg->grid_w * cfg->grid_h;
    const Carve c = carve(*cfg, gens);
    r->cfg = *cfg;
    r->I = I;
    r->N = cfg->pop_per_island;
    r->A = I * r->N;
    r->S = cfg->surface_sites;
    r->SW = surface_words(*cfg);
    r->stream = stream;
    const size_t A = r->A;
    for (int b = 0; b < 2; ++b) {
        r->trait[b] = reinterpret_cast<uint32_t*>(base + c.trait + b * align_up(A * 4));
        r->counter[b] = cfg->async_activity ? reinterpret_cast<uint32_t*>(
                                                  base + c.counter + b * align_up(A * 4))
                                            : nullptr;
        r->surf[b] = reinterpret_cast<uint32_t*>(base + c.surf + b * align_up(r->SW * A * 4));
        r->outbox[b] = reinterpret_cast<uint32_t*>(
            base + c.outbox + b * align_up((size_t)I * hsga::kOutboxWords * 4));
    }
    r->layout = reinterpret_cast<uint32_t*>(base + c.layout);
    r->rules = reinterpret_cast<hsga::RuleTable*>(base + c.rules);
    r->sites = cfg->async_activity ? nullptr : reinterpret_cast<uint32_t*>(base + c.sites);
    r->ring = cfg->async_activity ? reinterpret_cast<uint32_t*>(base + c.sites) : nullptr;
    r->ring_hi = 0;
    r->gens = gens;
    r->T = 0;
    r->horizon = hsga::horizon_gen_of(cfg->surface_kind, r->S, cfg->ingest_interval);
    r->apt = default_agents_per_thread(r->N);
    // integer births with four agents per thread: small tiles, more
    // workgroups in flight per CU -- 64 threads for synchronous runs on
    // two-word surfaces, 128 for one-word ones and for asynchronous ticks
    // (3 to 5 KB of records per tile, which measured fastest: the treatment
    // pair's selection run 3-6 % faster at 128 than at 64, asynchronous
    // ticks 1.4-2.2 %, the paper-scale run about 1 % slower); float births
    // (VALU-bound) and the rest: 256 threads, which measured faster for them
    const bool narrow = r->SW == 2 && cfg->async_activity == 0;
    r->block = r->apt == 4 && birth_model(*cfg) != hsga::kBirthFloat ? (narrow ? 64u : 128u)
                                                                        : 256u;
    r->timing = false;
    hipError_t e = hsga::launch_founders(r->trait[0], r->counter[0], r->surf[0], r->A, r->SW,
                                         r->layout, r->S, cfg->fitness_model == GA_FOUNDER_TAG,
                                         (uint32_t)cfg->seed, (uint32_t)(cfg->seed >> 32),
                                         r->stream);
    if (e != hipSuccess) return hip_fail(e, "founders launch");
    // the rule's tables: a synchronous run's launch batches take their sites
    // and layouts from them, an asynchronous birth its site from its
    // parent's counter
    e = upload_tables(cfg->surface_kind, r->S, r->rules, r->stream);
    if (e != hipSuccess) return hip_fail(e, "site rule tables upload");
    return GA_OK;
}

int set_run_layout(ga_run* r, uint32_t T) {
    // the layout after the run's ingests up to generation (tick) T, in
    // ingest units, from the rule's closed form
    uint32_t L[64];
    hsga::scheme_layout_items(r->cfg.surface_kind, r->S,
                              hsga::ingests_of(T, r->cfg.ingest_interval), L);
    hipError_t e = hsga::launch_set_layout(r->layout, L, r->S, r->stream);
    if (e != hipSuccess) return hip_fail(e, "layout launch");
    return GA_OK;
}

hsga::StepParams step_params(const ga_run* r, uint32_t g, uint32_t tau0) {
    const ga_config& cfg = r->cfg;
    const int src = g & 1, dst = (g + 1) & 1;
    hsga::StepParams p;
    p.in_trait = r->trait[src];
    p.in_counter = r->counter[src];
    p.in_surf = r->surf[src];
    p.out_trait = r->trait[dst];
    p.out_counter = r->counter[dst];
    p.out_surf = r->surf[dst];
    p.ob_in = r->outbox[src];
    p.ob_out = r->outbox[dst];
    const uint32_t n = cfg.ingest_interval;
    p.site = g % n == 0 && r->sites ? r->sites + (g / n - tau0) : nullptr;
    p.diff_log2 = cfg.differentia_bits == 8 ? 3u : 0u;
    p.async_thr = cfg.async_activity;
    p.rules = r->rules;
    p.ring = r->ring;
    p.ring_lo = r->ring_hi > hsga::kSiteRing ? r->ring_hi - hsga::kSiteRing : 0u;
    p.kind = cfg.surface_kind;
    p.S = r->S;
    p.interval = n;
    p.W = cfg.grid_w;
    p.H = cfg.grid_h;
    p.N = r->N;
    p.I = r->I;
    p.A = r->A;
    p.g = g;
    p.k0 = (uint32_t)cfg.seed;
    p.k1 = (uint32_t)(cfg.seed >> 32);
    // founder tags: neutral, inherited unchanged
    p.mut_thr = cfg.fitness_model == GA_FOUNDER_TAG ? 0u : cfg.mut_threshold;
    p.mut_lo = cfg.mut_lo;
    p.mut_span = (uint32_t)((int64_t)cfg.mut_hi - cfg.mut_lo + 1);
    p.has_inbox = (cfg.migrants_per_island != 0 && g > 0) ? 1u : 0u;
    p.tile_isl = tile_islands(r->block, r->apt, r->N);
    p.div_magic = ((1u << 20) + r->N - 1) / r->N;
    hsga::column_magic(cfg.grid_w, &p.w_magic, &p.w_shift);
    p.tour = cfg.tournament_size > 1 ? cfg.tournament_size : 1u;
    p.del_thr = cfg.del_threshold;
    p.ben_thr = cfg.ben_threshold;
    p.del_sigma = cfg.del_sigma;
    p.ben_sigma = cfg.ben_sigma;
    return p;
}

uint32_t birth_model(const ga_config& cfg) {
    if (cfg.fitness_model == GA_FLOAT_FITNESS) return hsga::kBirthFloat;
    if (cfg.fitness_model == GA_FOUNDER_TAG) return hsga::kBirthIntNeutral;
    return cfg.tournament_size == 2 ? hsga::kBirthIntTournament : hsga::kBirthIntNeutral;
}

}  // namespace hsga_host

using namespace hsga_host;

namespace {

// Exported state: header words (magic "HSGS", version, sizeof(ga_config), T).
constexpr uint32_t kStateMagic = 0x53475348u;
constexpr uint32_t kStateVersion = 1;
constexpr size_t kStateHeaderWords = 4;
static_assert(sizeof(ga_config) % 4 == 0, "the state holds the config as whole words");

// Words of one outbox entry as the device holds it.
uint32_t entry_words(const ga_run* r) {
    return r->cfg.async_activity ? hsga::kOutboxWords : hsga::kSyncOutboxWords;
}

bool has_outbox(const ga_run* r) { return r->cfg.migrants_per_island != 0 && r->T > 0; }

hipEvent_t take_event(ga_run* r) {
    if (!r->spare.empty()) {
        hipEvent_t e = r->spare.back();
        r->spare.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

int step_enqueue(ga_run* r, uint32_t n);

}  // namespace

extern "C" {

size_t ga_footprint_bytes(const ga_config* in, uint32_t max_gens_per_launch) {
    ga_config cfg;
    if (validate(in, &cfg) != GA_OK) return 0;
    const uint32_t gens = max_gens_per_launch ? max_gens_per_launch : kDefaultGens;
    return carve(cfg, gens).total;
}

int ga_create(const ga_config* in, void* dev_arena, size_t arena_bytes,
              uint32_t max_gens_per_launch, void* hip_stream, ga_run** out) {
    if (!out) return fail(GA_EINVAL, "out is NULL");
    *out = nullptr;
    ga_config cfg_copy;
    int rc = validate(in, &cfg_copy);
    const ga_config* cfg = &cfg_copy;
    if (rc != GA_OK) return rc;
    if (!dev_arena) return fail(GA_EINVAL, "arena is NULL");
    if ((uintptr_t)dev_arena % kAlign) return fail(GA_EINVAL, "arena not 256-byte aligned");
    const uint32_t gens = max_gens_per_launch ? max_gens_per_launch : kDefaultGens;
    const Carve c = carve(*cfg, gens);
    if (arena_bytes < c.total)
        return fail(GA_ENOMEM, "arena of " + std::to_string(arena_bytes) + " bytes, need " +
                                   std::to_string(c.total));
    ga_run* r = new (std::nothrow) ga_run();
    if (!r) return fail(GA_ENOMEM, "host allocation failed");
    rc = run_init(r, cfg, static_cast<uint8_t*>(dev_arena), gens, static_cast<hipStream_t>(hip_stream));
    if (rc != GA_OK) {
        delete r;
        return rc;
    }
    *out = r;
    return GA_OK;
}

int ga_step(ga_run* r, uint32_t n) {
    if (!r) return fail(GA_EINVAL, "run is NULL");
    if (r->pooled) return fail(GA_EINVAL, "a run of a pool advances with ga_pool_advance");
    if (r->broken)
        return fail(GA_EDEVICE, "an earlier ga_step failed part-way; import a state first");
    if (n == 0) return GA_OK;
    // a failure after the first launch leaves the run between generations
    // (its layout already advanced): refuse further steps until a state is
    // imported
    const int rc = step_enqueue(r, n);
    if (rc == GA_EDEVICE) r->broken = true;
    return rc;
}

}  // extern "C"

namespace {

// Workgroup size of the resident form for this run: the fewest multiple of
// 64 threads that holds every agent at the run's agents per thread, so that
// the whole torus is one tile; 0 when the run steps one launch per
// generation instead (the form is off, the run is asynchronous or larger
// than kResidentMaxAgents, or the tile would not fit the LDS).
uint32_t resident_block(const ga_run* r) {
    if (!r->resident || r->cfg.async_activity || r->A > kResidentMaxAgents) return 0;
    const uint32_t block = ((r->A + r->apt - 1) / r->apt + 63) / 64 * 64;
    const uint32_t tile_isl = tile_islands(block, r->apt, r->N);
    if (block > 1024 || tile_isl < r->I || tile_isl > block) return 0;
    if (hsga::step_lds_bytes(tile_isl, r->N, r->SW, birth_model(r->cfg) == hsga::kBirthFloat,
                             block, r->apt) > kMaxStepLds)
        return 0;
    return block;
}

int step_enqueue(ga_run* r, uint32_t n) {
    if ((uint64_t)r->T + n - 1 > r->horizon)
        return fail(GA_EHORIZON, "generation " + std::to_string((uint64_t)r->T + n - 1) +
                                     " is past the site rule's horizon " +
                                     std::to_string(r->horizon));
    const ga_config& cfg = r->cfg;
    const uint32_t model = birth_model(cfg);
    const bool mig = cfg.migrants_per_island != 0;
    if (cfg.async_activity) {
        // asynchronous ticks: one launch per tick; each birth finds its site
        // from its parent's counter in the rule's tables
        ga_run::Span span{nullptr, nullptr, n};
        if (r->timing) {
            span.start = take_event(r);
            span.stop = take_event(r);
            if (!span.start || !span.stop) return fail(GA_EDEVICE, "hipEventCreate failed");
            hipError_t e = hipEventRecord(span.start, r->stream);
            if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
        }
        for (uint32_t k = 0; k < n; ++k) {
            if ((k & (hsga::kSiteRing / 2 - 1)) == 0) {
                // the ring takes the ingests the next half ring of ticks can
                // reach (a parent's counter is at most the tick)
                const uint32_t last = (uint32_t)std::min<uint64_t>(
                    (uint64_t)r->T + k + hsga::kSiteRing / 2, (uint64_t)r->T + n);
                const uint32_t hi = hsga::ingests_of(last, cfg.ingest_interval);
                if (hi > r->ring_hi) {
                    const uint32_t lo = std::max(r->ring_hi, hi > hsga::kSiteRing
                                                                 ? hi - hsga::kSiteRing : 0u);
                    hipError_t e = hsga::launch_fill_site_ring(r->rules, cfg.surface_kind, r->S,
                                                               r->ring, lo, hi - lo, r->stream);
                    if (e != hipSuccess) return hip_fail(e, "site ring launch");
                    r->ring_hi = hi;
                }
            }
            const hsga::StepParams p = step_params(r, r->T + k, 0);
            hipError_t e = hsga::launch_step(p, r->SW, model, mig, r->apt, r->block, r->stream);
            if (e != hipSuccess) return hip_fail(e, "step launch");
        }
        if (r->timing) {
            hipError_t e = hipEventRecord(span.stop, r->stream);
            if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
            r->spans.push_back(span);
        }
        r->T += n;
        // the run's layout (what every agent of counter T holds), for the
        // run-bound queries
        return set_run_layout(r, r->T);
    }
    while (n > 0) {
        const uint32_t G = n < r->gens ? n : r->gens;
        const uint32_t tau0 = hsga::ingests_of(r->T, cfg.ingest_interval);
        const uint32_t count = hsga::ingests_of(r->T + G, cfg.ingest_interval) - tau0;
        hipError_t e = hsga::launch_run_sites(r->rules, cfg.surface_kind, r->S, r->sites,
                                              r->layout, tau0, count, r->stream);
        if (e != hipSuccess) return hip_fail(e, "site schedule launch");
        ga_run::Span span{nullptr, nullptr, G};
        if (r->timing) {
            span.start = take_event(r);
            span.stop = take_event(r);
            if (!span.start || !span.stop) return fail(GA_EDEVICE, "hipEventCreate failed");
            e = hipEventRecord(span.start, r->stream);
            if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
        }
        const uint32_t rb = resident_block(r);
        if (rb) {
            // the whole batch in one workgroup
            hsga::StepParams p = step_params(r, r->T, tau0);
            p.tile_isl = tile_islands(rb, r->apt, r->N);
            e = hsga::launch_resident_step(p, G, r->sites, tau0, r->SW, model, mig, r->apt, rb,
                                           r->stream);
            if (e != hipSuccess) return hip_fail(e, "resident step launch");
        } else {
            for (uint32_t k = 0; k < G; ++k) {
                const hsga::StepParams p = step_params(r, r->T + k, tau0);
                e = hsga::launch_step(p, r->SW, model, mig, r->apt, r->block, r->stream);
                if (e != hipSuccess) return hip_fail(e, "step launch");
            }
        }
        if (r->timing) {
            e = hipEventRecord(span.stop, r->stream);
            if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
            r->spans.push_back(span);
        }
        r->T += G;
        n -= G;
    }
    return GA_OK;
}

}  // namespace

extern "C" {

int ga_sync(ga_run* r) {
    if (!r) return fail(GA_EINVAL, "run is NULL");
    hipError_t e = hipStreamSynchronize(r->stream);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    return GA_OK;
}

int ga_generation(const ga_run* r, uint32_t* T) {
    if (!r || !T) return fail(GA_EINVAL, "NULL argument");
    *T = r->T;
    return GA_OK;
}

int ga_read_agents(ga_run* r, uint32_t first, uint32_t count, uint32_t* trait, uint32_t* counter,
                   uint32_t* surface_words) {
    if (!r) return fail(GA_EINVAL, "run is NULL");
    if ((uint64_t)first + count > r->A) return fail(GA_EINVAL, "agent range out of bounds");
    if (count == 0) return GA_OK;
    const int cur = r->T & 1;
    hipError_t e = hipStreamSynchronize(r->stream);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    if (trait) {
        e = hipMemcpy(trait, r->trait[cur] + first, (size_t)count * 4, hipMemcpyDeviceToHost);
        if (e != hipSuccess) return hip_fail(e, "hipMemcpy trait");
    }
    if (counter && r->counter[cur]) {
        e = hipMemcpy(counter, r->counter[cur] + first, (size_t)count * 4, hipMemcpyDeviceToHost);
        if (e != hipSuccess) return hip_fail(e, "hipMemcpy counter");
    } else if (counter) {
        std::fill(counter, counter + count, r->T);   // synchronous: every counter is T
    }
    if (surface_words) {
        std::vector<uint32_t> plane(count);
        for (uint32_t w = 0; w < r->SW; ++w) {
            e = hipMemcpy(plane.data(), r->surf[cur] + (size_t)w * r->A + first, (size_t)count * 4,
                          hipMemcpyDeviceToHost);
            if (e != hipSuccess) return hip_fail(e, "hipMemcpy surface");
            for (uint32_t k = 0; k < count; ++k) surface_words[(size_t)k * r->SW + w] = plane[k];
        }
    }
    return GA_OK;
}

int ga_read_outbox(ga_run* r, uint32_t first, uint32_t count, uint32_t* dir, uint32_t* trait,
                   uint32_t* counter, uint32_t* surface_words, int* valid) {
    if (!r || !valid) return fail(GA_EINVAL, "NULL argument");
    if ((uint64_t)first + count > r->I) return fail(GA_EINVAL, "island range out of bounds");
    *valid = (r->cfg.migrants_per_island != 0 && r->T > 0) ? 1 : 0;
    if (!*valid || count == 0) return GA_OK;
    hipError_t e = hipStreamSynchronize(r->stream);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    // asynchronous entries: dir, trait, counter, surface; synchronous ones
    // leave the counter out (every emigrant's counter is T)
    const bool async = r->cfg.async_activity != 0;
    const uint32_t words = async ? hsga::kOutboxWords : hsga::kSyncOutboxWords;
    const uint32_t surf0 = async ? 3 : 2;
    std::vector<uint32_t> entries((size_t)count * words);
    e = hipMemcpy(entries.data(), r->outbox[r->T & 1] + (size_t)first * words,
                  entries.size() * 4, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy outbox");
    for (uint32_t k = 0; k < count; ++k) {
        const uint32_t* en = &entries[(size_t)k * words];
        if (dir) dir[k] = en[0];
        if (trait) trait[k] = en[1];
        if (counter) counter[k] = async ? en[2] : r->T;
        if (surface_words)
            for (uint32_t w = 0; w < r->SW; ++w)
                surface_words[(size_t)k * r->SW + w] = en[surf0 + w];
    }
    return GA_OK;
}

int ga_read_layout(ga_run* r, uint32_t* layout) {
    if (!r || !layout) return fail(GA_EINVAL, "NULL argument");
    hipError_t e = hipStreamSynchronize(r->stream);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    e = hipMemcpy(layout, r->layout, (size_t)r->S * 4, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy layout");
    // the device layout holds ingest indices; report deposit generations
    for (uint32_t k = 0; k < r->S; ++k)
        if (layout[k] != GA_EMPTY_SITE) layout[k] *= r->cfg.ingest_interval;
    return GA_OK;
}

int ga_sample(ga_run* r, uint32_t n, uint32_t* dev_idx, uint32_t* dev_counter,
              uint32_t* dev_surface_words, uint32_t* n_taken) {
    if (!r || !n_taken) return fail(GA_EINVAL, "NULL argument");
    if (n == 0 || !dev_idx || !dev_counter || !dev_surface_words)
        return fail(GA_EINVAL, "empty sample or NULL buffer");
    const int cur = r->T & 1;
    hipError_t e = hsga::launch_sample(r->counter[cur], r->surf[cur], r->A, r->SW, n, r->T,
                                       (uint32_t)r->cfg.seed, (uint32_t)(r->cfg.seed >> 32),
                                       dev_idx, dev_counter, dev_surface_words, r->stream);
    if (e != hipSuccess) return hip_fail(e, "sample launch");
    *n_taken = r->A <= n ? r->A : n;
    return GA_OK;
}

size_t ga_state_bytes(const ga_run* r) {
    if (!r) return 0;
    return 4 * (kStateHeaderWords + sizeof(ga_config) / 4 + (size_t)r->A * (2 + r->SW) +
                (size_t)r->I * entry_words(r));
}

int ga_export_state(ga_run* r, void* host, size_t bytes) {
    if (!r || !host) return fail(GA_EINVAL, "NULL argument");
    if ((uintptr_t)host % 4) return fail(GA_EINVAL, "state buffer not 4-byte aligned");
    const size_t need = ga_state_bytes(r);
    if (bytes < need)
        return fail(GA_EINVAL, "state buffer of " + std::to_string(bytes) + " bytes, need " +
                                   std::to_string(need));
    hipError_t e = hipStreamSynchronize(r->stream);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    uint32_t* w = static_cast<uint32_t*>(host);
    w[0] = kStateMagic;
    w[1] = kStateVersion;
    w[2] = sizeof(ga_config);
    w[3] = r->T;
    std::memcpy(w + kStateHeaderWords, &r->cfg, sizeof(ga_config));
    uint32_t* at = w + kStateHeaderWords + sizeof(ga_config) / 4;
    const int cur = r->T & 1;
    const size_t A = r->A;
    // a synchronous run keeps no counter plane: every counter is T
    const struct { const uint32_t* src; size_t words; } planes[] = {
        {r->trait[cur], A}, {r->counter[cur], A}, {r->surf[cur], r->SW * A}};
    for (const auto& pl : planes) {
        if (pl.src) {
            e = hipMemcpy(at, pl.src, pl.words * 4, hipMemcpyDeviceToHost);
            if (e != hipSuccess) return hip_fail(e, "hipMemcpy state");
        } else {
            std::fill(at, at + pl.words, r->T);
        }
        at += pl.words;
    }
    const size_t ob = (size_t)r->I * entry_words(r);
    if (has_outbox(r)) {
        e = hipMemcpy(at, r->outbox[cur], ob * 4, hipMemcpyDeviceToHost);
        if (e != hipSuccess) return hip_fail(e, "hipMemcpy outbox");
    } else {
        std::memset(at, 0, ob * 4);
    }
    return GA_OK;
}

int ga_import_state(ga_run* r, const void* host, size_t bytes) {
    if (!r || !host) return fail(GA_EINVAL, "NULL argument");
    if (r->pooled) return fail(GA_EINVAL, "a run of a pool cannot import a state");
    if ((uintptr_t)host % 4) return fail(GA_EINVAL, "state buffer not 4-byte aligned");
    if (bytes != ga_state_bytes(r))
        return fail(GA_EINVAL, "state of " + std::to_string(bytes) + " bytes; this run's has " +
                                   std::to_string(ga_state_bytes(r)));
    const uint32_t* w = static_cast<const uint32_t*>(host);
    if (w[0] != kStateMagic || w[1] != kStateVersion || w[2] != sizeof(ga_config))
        return fail(GA_EINVAL, "not a run state of this format version");
    if (std::memcmp(w + kStateHeaderWords, &r->cfg, sizeof(ga_config)) != 0)
        return fail(GA_EINVAL, "state exported under another configuration");
    const uint32_t T = w[3];
    const bool async = r->cfg.async_activity != 0;
    if ((uint64_t)T > r->horizon + 1)
        return fail(GA_EHORIZON, "state generation " + std::to_string(T) +
                                     " is past the site rule's horizon");
    const size_t A = r->A;
    const uint32_t* trait = w + kStateHeaderWords + sizeof(ga_config) / 4;
    const uint32_t* counter = trait + A;
    const uint32_t* surf = counter + A;
    const uint32_t* ob = surf + r->SW * A;
    // every later launch indexes the site table by counters: check them
    for (size_t a = 0; a < A; ++a)
        if (async ? counter[a] > T : counter[a] != T)
            return fail(GA_EINVAL, "agent " + std::to_string(a) + " has counter " +
                                       std::to_string(counter[a]) + " at generation " +
                                       std::to_string(T));
    const uint32_t E = entry_words(r);
    const bool outbox = r->cfg.migrants_per_island != 0 && T > 0;
    if (outbox)
        for (uint32_t i = 0; i < r->I; ++i) {
            const uint32_t* en = ob + (size_t)i * E;
            if (en[0] > 4 || (async && en[2] > T))
                return fail(GA_EINVAL, "outbox entry " + std::to_string(i) + " out of range");
        }
    hipError_t e = hipStreamSynchronize(r->stream);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    const int cur = T & 1;
    const struct { uint32_t* dst; const uint32_t* src; size_t words; } planes[] = {
        {r->trait[cur], trait, A}, {r->counter[cur], counter, A}, {r->surf[cur], surf, r->SW * A},
        {r->outbox[cur], ob, outbox ? (size_t)r->I * E : 0}};
    for (const auto& pl : planes) {
        if (pl.words == 0 || !pl.dst) continue;      // no counter plane when synchronous
        e = hipMemcpy(pl.dst, pl.src, pl.words * 4, hipMemcpyHostToDevice);
        if (e != hipSuccess) return hip_fail(e, "hipMemcpy state");
    }
    // the layout after ingests_of(T) ingests, from the rule's closed form
    // (a function of the scheme and T alone, nothing of the state)
    int rc = set_run_layout(r, T);
    if (rc != GA_OK) return rc;
    r->ring_hi = 0;     // the next ticks refill the ring
    e = hipStreamSynchronize(r->stream);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    r->T = T;
    r->broken = false;
    return GA_OK;
}

void ga_destroy(ga_run* r) {
    if (!r) return;
    if (r->pooled) {
        // the handle lives in the pool's slot table: ga_pool_release frees it
        (void)fail(GA_EINVAL, "ga_destroy of a run of a pool ignored (use ga_pool_release)");
        return;
    }
    for (auto& s : r->spans) {
        (void)hipEventDestroy(s.start);
        (void)hipEventDestroy(s.stop);
    }
    for (auto e : r->spare) (void)hipEventDestroy(e);
    delete r;
}

const char* ga_last_error(void) { return last_error(); }

namespace {
// Query workspaces: the MRCA or reconstruction workspace proper, then the
// surface's site rule tables, which the query kernels read to lay out an
// annotation in constant time.
size_t aligned256(size_t x) { return (x + 255) & ~(size_t)255; }
size_t mrca_total_bytes(uint32_t S, uint32_t n) {
    return aligned256(hsga::MrcaWorkspace::bytes(S, n)) + hsga::kRuleRegionBytes;
}
size_t phylo_total_bytes(uint32_t S, uint32_t n) {
    return aligned256(hsga::phylo_workspace_bytes(S, n)) + hsga::kRuleRegionBytes;
}

// Enqueue the upload of the scheme's tables to `region` (kRuleRegionBytes,
// 256-byte aligned) on `stream`; the LayoutHint that reads them.
hipError_t upload_rules(const hsga::Scheme& sc, uint8_t* region, hipStream_t stream,
                        hsga::LayoutHint* hint) {
    auto* dev = reinterpret_cast<hsga::RuleTable*>(region);
    hipError_t e = upload_tables(sc.kind, sc.S, dev, stream);
    if (e != hipSuccess) return e;
    hint->rules = dev;
    return hipSuccess;
}
}  // namespace

size_t hstrat_mrca_workspace_bytes(uint32_t S, uint32_t n) { return mrca_total_bytes(S, n); }

namespace {
int check_scheme(const hstrat_scheme* sc, hsga::Scheme* out) {
    if (!sc) return fail(GA_EINVAL, "scheme is NULL");
    if (sc->kind > GA_HYBRID) return fail(GA_EINVAL, "unknown surface kind");
    if (sc->differentia_bits != 1 && sc->differentia_bits != 8)
        return fail(GA_EINVAL, "differentia_bits must be 1 or 8");
    if (sc->sites * sc->differentia_bits != 32 && sc->sites * sc->differentia_bits != 64)
        return fail(GA_EINVAL, "sites * differentia_bits must be 32 or 64");
    if (sc->ingest_interval == 0) return fail(GA_EINVAL, "ingest_interval must be >= 1");
    *out = hsga::Scheme{sc->kind, sc->sites, sc->differentia_bits, sc->ingest_interval};
    return GA_OK;
}
}  // namespace

int hstrat_mrca_bounds_ex(const hstrat_scheme* scheme, uint32_t n, const uint32_t* counter,
                          const uint32_t* surface_words, uint32_t* lb, uint32_t* ub,
                          void* workspace, size_t workspace_bytes, void* hip_stream) {
    hsga::Scheme sc;
    int rc = check_scheme(scheme, &sc);
    if (rc != GA_OK) return rc;
    if (n == 0 || n > 65535) return fail(GA_EINVAL, "n must be 1..65535");
    if (!counter || !surface_words || !lb || !ub || !workspace)
        return fail(GA_EINVAL, "NULL buffer");
    if ((uintptr_t)workspace % kAlign) return fail(GA_EINVAL, "workspace not 256-byte aligned");
    if (workspace_bytes < mrca_total_bytes(sc.S, n)) return fail(GA_ENOMEM, "workspace too small");
    const auto stream = static_cast<hipStream_t>(hip_stream);
    hsga::LayoutHint hint;
    hipError_t e = upload_rules(sc, static_cast<uint8_t*>(workspace) +
                                        aligned256(hsga::MrcaWorkspace::bytes(sc.S, n)),
                                stream, &hint);
    if (e != hipSuccess) return hip_fail(e, "site rule upload");
    e = hsga::launch_mrca(sc, n, counter, surface_words, lb, ub, workspace, stream, hint);
    if (e != hipSuccess) return hip_fail(e, "mrca launch");
    return GA_OK;
}

int ga_mrca_bounds(ga_run* r, uint32_t n, const uint32_t* counter,
                   const uint32_t* surface_words, uint32_t* lb, uint32_t* ub, void* workspace,
                   size_t workspace_bytes) {
    if (!r) return fail(GA_EINVAL, "run is NULL");
    const hsga::Scheme sc{r->cfg.surface_kind, r->S, r->cfg.differentia_bits,
                          r->cfg.ingest_interval};
    if (n == 0 || n > 65535) return fail(GA_EINVAL, "n must be 1..65535");
    if (!counter || !surface_words || !lb || !ub || !workspace)
        return fail(GA_EINVAL, "NULL buffer");
    if ((uintptr_t)workspace % kAlign) return fail(GA_EINVAL, "workspace not 256-byte aligned");
    if (workspace_bytes < mrca_total_bytes(sc.S, n)) return fail(GA_ENOMEM, "workspace too small");
    // on the run's stream: the layout is read after the steps enqueued so
    // far and before any later ones advance it
    // the run's own tables (in its arena) lay out annotations of other counts
    const hsga::LayoutHint hint{r->layout, r->T, r->rules};
    hipError_t e =
        hsga::launch_mrca(sc, n, counter, surface_words, lb, ub, workspace, r->stream, hint);
    if (e != hipSuccess) return hip_fail(e, "mrca launch");
    return GA_OK;
}

int ga_phylo_tree(ga_run* r, uint32_t n, const uint32_t* counter, const uint32_t* surface_words,
                  uint32_t* leaf_parent, uint32_t* node_parent, uint32_t* node_time,
                  uint64_t* out, void* workspace, size_t workspace_bytes) {
    if (!r) return fail(GA_EINVAL, "run is NULL");
    const hsga::Scheme sc{r->cfg.surface_kind, r->S, r->cfg.differentia_bits,
                          r->cfg.ingest_interval};
    if (n == 0 || n > 65535) return fail(GA_EINVAL, "n must be 1..65535");
    if (!counter || !surface_words || !out || !workspace ||
        (leaf_parent && n > 1 && (!node_parent || !node_time)))
        return fail(GA_EINVAL, "NULL buffer");
    if ((uintptr_t)workspace % kAlign) return fail(GA_EINVAL, "workspace not 256-byte aligned");
    if (workspace_bytes < phylo_total_bytes(sc.S, n))
        return fail(GA_ENOMEM, "workspace too small");
    const hsga::LayoutHint hint{r->layout, r->T, r->rules};
    hipError_t e = hsga::launch_phylo(sc, n, counter, surface_words, out, workspace, r->stream,
                                      leaf_parent, node_parent, node_time, hint);
    if (e != hipSuccess) return hip_fail(e, "phylo launch");
    return GA_OK;
}

int hstrat_mrca_bounds(uint32_t kind, uint32_t S, uint32_t n, const uint32_t* counter,
                       const uint32_t* surface_words, uint32_t* lb, uint32_t* ub, void* workspace,
                       size_t workspace_bytes, void* hip_stream) {
    if (S != 32 && S != 64) return fail(GA_EINVAL, "S must be 32 or 64");
    const hstrat_scheme sc{kind, S, 1, 1};
    return hstrat_mrca_bounds_ex(&sc, n, counter, surface_words, lb, ub, workspace,
                                 workspace_bytes, hip_stream);
}

int hstrat_mrca_bounds_noalloc(uint32_t kind, uint32_t S, uint32_t n, const uint32_t* counter,
                               const uint32_t* surface_words, uint32_t* lb, uint32_t* ub,
                               void* hip_stream) {
    if (S != 32 && S != 64) return fail(GA_EINVAL, "S must be 32 or 64");
    if (kind > GA_HYBRID) return fail(GA_EINVAL, "unknown surface kind");
    if (n == 0 || n > hsga::kNoAllocMaxN)
        return fail(GA_EINVAL, "n must be 1.." + std::to_string(hsga::kNoAllocMaxN) +
                                   " (the library's static scratch)");
    if (!counter || !surface_words || !lb || !ub) return fail(GA_EINVAL, "NULL buffer");
    const hsga::Scheme sc{kind, S, 1, 1};
    hipError_t e = hsga::launch_mrca_noalloc(sc, n, counter, surface_words, lb, ub,
                                             static_cast<hipStream_t>(hip_stream));
    if (e != hipSuccess) return hip_fail(e, "mrca launch (static scratch)");
    return GA_OK;
}

size_t hstrat_phylo_workspace_bytes(uint32_t S, uint32_t n) { return phylo_total_bytes(S, n); }

int hstrat_phylo_metrics_ex(const hstrat_scheme* scheme, uint32_t n, const uint32_t* counter,
                            const uint32_t* surface_words, uint64_t* out, void* workspace,
                            size_t workspace_bytes, void* hip_stream) {
    hsga::Scheme sc;
    int rc = check_scheme(scheme, &sc);
    if (rc != GA_OK) return rc;
    if (n == 0 || n > 65535) return fail(GA_EINVAL, "n must be 1..65535");
    if (!counter || !surface_words || !out || !workspace) return fail(GA_EINVAL, "NULL buffer");
    if ((uintptr_t)workspace % kAlign) return fail(GA_EINVAL, "workspace not 256-byte aligned");
    if (workspace_bytes < phylo_total_bytes(sc.S, n))
        return fail(GA_ENOMEM, "workspace too small");
    const auto stream = static_cast<hipStream_t>(hip_stream);
    hsga::LayoutHint hint;
    hipError_t e = upload_rules(sc, static_cast<uint8_t*>(workspace) +
                                        aligned256(hsga::phylo_workspace_bytes(sc.S, n)),
                                stream, &hint);
    if (e != hipSuccess) return hip_fail(e, "site rule upload");
    e = hsga::launch_phylo(sc, n, counter, surface_words, out, workspace, stream, nullptr,
                           nullptr, nullptr, hint);
    if (e != hipSuccess) return hip_fail(e, "phylo launch");
    return GA_OK;
}

int hstrat_phylo_tree_ex(const hstrat_scheme* scheme, uint32_t n, const uint32_t* counter,
                         const uint32_t* surface_words, uint32_t* leaf_parent,
                         uint32_t* node_parent, uint32_t* node_time, uint64_t* out,
                         void* workspace, size_t workspace_bytes, void* hip_stream) {
    hsga::Scheme sc;
    int rc = check_scheme(scheme, &sc);
    if (rc != GA_OK) return rc;
    if (n == 0 || n > 65535) return fail(GA_EINVAL, "n must be 1..65535");
    if (!counter || !surface_words || !out || !workspace || !leaf_parent ||
        (n > 1 && (!node_parent || !node_time)))
        return fail(GA_EINVAL, "NULL buffer");
    if ((uintptr_t)workspace % kAlign) return fail(GA_EINVAL, "workspace not 256-byte aligned");
    if (workspace_bytes < phylo_total_bytes(sc.S, n))
        return fail(GA_ENOMEM, "workspace too small");
    const auto stream = static_cast<hipStream_t>(hip_stream);
    hsga::LayoutHint hint;
    hipError_t e = upload_rules(sc, static_cast<uint8_t*>(workspace) +
                                        aligned256(hsga::phylo_workspace_bytes(sc.S, n)),
                                stream, &hint);
    if (e != hipSuccess) return hip_fail(e, "site rule upload");
    e = hsga::launch_phylo(sc, n, counter, surface_words, out, workspace, stream, leaf_parent,
                           node_parent, node_time, hint);
    if (e != hipSuccess) return hip_fail(e, "phylo tree launch");
    return GA_OK;
}

int hstrat_phylo_metrics(uint32_t kind, uint32_t S, uint32_t n, const uint32_t* counter,
                         const uint32_t* surface_words, uint64_t* out, void* workspace,
                         size_t workspace_bytes, void* hip_stream) {
    if (S != 32 && S != 64) return fail(GA_EINVAL, "S must be 32 or 64");
    const hstrat_scheme sc{kind, S, 1, 1};
    return hstrat_phylo_metrics_ex(&sc, n, counter, surface_words, out, workspace,
                                   workspace_bytes, hip_stream);
}

int hstrat_mrca_status(const void* workspace, void* hip_stream) {
    if (!workspace) return fail(GA_EINVAL, "workspace is NULL");
    hipError_t e = hipStreamSynchronize(static_cast<hipStream_t>(hip_stream));
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    uint32_t status = 0;
    e = hipMemcpy(&status, workspace, 4, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy status");
    if (status == 2) return fail(GA_EHORIZON, "a counter is past the site rule's horizon");
    return GA_OK;
}

int ga_set_kernel_timing(ga_run* r, int enable) {
    if (!r) return fail(GA_EINVAL, "run is NULL");
    r->timing = enable != 0;
    return GA_OK;
}

int ga_kernel_time(ga_run* r, double* ms, uint64_t* launches, int reset) {
    if (!r || !ms || !launches) return fail(GA_EINVAL, "NULL argument");
    double total = 0.0;
    uint64_t count = 0;
    for (auto& s : r->spans) {
        hipError_t e = hipEventSynchronize(s.stop);
        if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
        float span_ms = 0.f;
        e = hipEventElapsedTime(&span_ms, s.start, s.stop);
        if (e != hipSuccess) return hip_fail(e, "hipEventElapsedTime");
        total += span_ms;
        count += s.launches;
    }
    *ms = total;
    *launches = count;
    if (reset) {
        for (auto& s : r->spans) {
            r->spare.push_back(s.start);
            r->spare.push_back(s.stop);
        }
        r->spans.clear();
    }
    return GA_OK;
}

int ga_probe_copy(const void* src, void* dst, size_t bytes, void* hip_stream) {
    if (!src || !dst) return fail(GA_EINVAL, "NULL pointer");
    if (bytes % 16 || (uintptr_t)src % 16 || (uintptr_t)dst % 16)
        return fail(GA_EINVAL, "copy needs 16-byte multiples and alignment");
    hipError_t e = hsga::launch_probe_copy(src, dst, bytes, static_cast<hipStream_t>(hip_stream));
    if (e != hipSuccess) return hip_fail(e, "copy launch");
    return GA_OK;
}

int ga_set_launch_shape(ga_run* r, uint32_t block_threads, uint32_t agents_per_thread) {
    if (!r) return fail(GA_EINVAL, "run is NULL");
    const uint32_t block = block_threads ? block_threads : r->block;
    const uint32_t apt = agents_per_thread ? agents_per_thread : r->apt;
    if (block % 64 || block < 64 || block > 1024)
        return fail(GA_EINVAL, "block_threads must be a multiple of 64 in 64..1024");
    if ((apt != 1 && apt != 2 && apt != 4) || r->N % apt)
        return fail(GA_EINVAL, "agents_per_thread must be 1, 2 or 4 and divide pop_per_island");
    if (hsga::step_lds_bytes(tile_islands(block, apt, r->N), r->N, r->SW,
                             birth_model(r->cfg) == hsga::kBirthFloat, block, apt) > kMaxStepLds)
        return fail(GA_EINVAL, "tile needs more than 64 KiB of LDS");
    r->block = block;
    r->apt = apt;
    return GA_OK;
}

int ga_set_resident(ga_run* r, int enable) {
    if (!r) return fail(GA_EINVAL, "run is NULL");
    r->resident = enable != 0;
    return GA_OK;
}

int ga_resident_threads(const ga_run* r, uint32_t* threads) {
    if (!r || !threads) return fail(GA_EINVAL, "NULL argument");
    *threads = resident_block(r);
    return GA_OK;
}

}  // extern "C"
