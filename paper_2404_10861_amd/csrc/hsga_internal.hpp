// hsga_internal.hpp -- launchers shared between the kernel translation unit
// and the C-ABI host runtime.  Not part of the public interface.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hsga_rule.hpp"

namespace hsga {

// An annotation scheme (Distributed Phylogenetic Tracking: one-bit or byte
// differentiae; Results, Surface Algorithm Benchmark: annotations updated
// only every n-th generation): surface kind, S sites of `bits` bits (1 or
// 8) filling S * bits / 32 words, one deposit every `interval` generations.
// The site rule runs in ingest units: item tau is deposited at generation
// tau * interval, and layouts hold tau.
struct Scheme {
    uint32_t kind, S, bits, interval;
};

// How a birth picks its parent and changes the trait word.
enum BirthModel : uint32_t {
    kBirthIntNeutral = 0,      // integer trait, one uniform draw
    kBirthIntTournament = 1,   // integer trait, tournament of two
    kBirthFloat = 2,           // binary32 fitness, tournament of `tour`, half-normal mutations
};

struct StepParams {
    const uint32_t* in_trait;
    const uint32_t* in_counter;
    const uint32_t* in_surf;   // S/32 planes of A words
    uint32_t* out_trait;
    uint32_t* out_counter;
    uint32_t* out_surf;
    const uint32_t* ob_in;     // I entries of 8 words (read at generation g)
    uint32_t* ob_out;          // I entries of 8 words (written for g + 1)
    const uint32_t* site;      // this generation's surface site; nullptr: no deposit
    uint32_t W, H, N, I, A;
    uint32_t g;
    uint32_t k0, k1;           // Philox key (seed)
    uint32_t mut_thr;
    int32_t mut_lo;
    uint32_t mut_span;         // mut_hi - mut_lo + 1
    uint32_t has_inbox;        // outboxes of generation g exist
    uint32_t tile_isl;         // islands per workgroup tile
    uint32_t div_magic;        // ceil(2^20 / N): la / N == (la * div_magic) >> 20 for la < 4096
    uint32_t w_magic, w_shift; // isl / W by multiplication (column_magic)
    uint32_t diff_log2;        // log2 of the differentia width: 0 (bit) or 3 (byte)
    uint32_t async_thr;        // asynchronous ticks: island activity threshold; 0: synchronous
    const RuleTable* rules;    // asynchronous ticks: the surface's site rule tables
    const uint32_t* ring;      // asynchronous ticks: sites of ingests ring_lo .. (ring of
                               // kSiteRing words, ingest tau at tau % kSiteRing)
    uint32_t ring_lo;
    uint32_t kind, S;          // asynchronous ticks: the surface
    uint32_t interval;         // asynchronous ticks: the ingest interval
    uint32_t tour;             // float model: tournament draws, 1..5
    uint32_t del_thr, ben_thr; // float model: mutation class thresholds
    float del_sigma, ben_sigma;
};

// One run of a batched launch: a device-resident table entry, written by the
// host before each batch.  The step of generation T0 + k uses ping-pong
// buffers (T0 + k) & 1 -> (T0 + k + 1) & 1 and site sites[k]; a run with
// k >= gens sits the launch out.
struct BatchRun {
    uint32_t* trait[2];
    uint32_t* counter[2];
    uint32_t* surf[2];
    uint32_t* outbox[2];
    uint32_t* sites;           // this batch's site schedule
    uint32_t* layout;          // the run's layout (S words)
    const RuleTable* rules;    // the surface's site rule tables (device)
    uint32_t W, H, N, I, A;
    uint32_t T0, gens;
    uint32_t k0, k1;
    uint32_t mut_thr;
    int32_t mut_lo;
    uint32_t mut_span;
    uint32_t kind, S;
    uint32_t variant;          // bit 0: S = 64, bits 1..2: BirthModel, bit 3: migration,
                               // bits 4..5: log2(agents per thread)
    uint32_t tour, del_thr, ben_thr;
    float del_sigma, ben_sigma;
    uint32_t interval;         // one deposit every `interval` generations
    uint32_t diff_log2;        // 0: one-bit differentiae, 3: bytes
    uint32_t tile_isl, div_magic;
    uint32_t w_magic, w_shift;
};

// Division of any 32-bit n by a fixed d >= 1 as a multiply-high and
// shifts (the round-down method with an add indicator, Granlund and
// Montgomery 1994): with l = ceil(log2 d), magic = floor(2^32 (2^l - d) / d)
// + 1 (0 when d is a power of two) and t = mulhi(n, magic),
// n / d = (t + ((n - t) >> s1)) >> s2, s1 = min(l, 1), s2 = max(l - 1, 0);
// shift packs s1 | s2 << 8.
inline void column_magic(uint32_t d, uint32_t* magic, uint32_t* shift) {
    uint32_t l = 0;
    while ((1ull << l) < d) ++l;
    *magic = (d & (d - 1)) == 0 ? 0u
                                : (uint32_t)((((1ull << l) - d) << 32) / d + 1);
    *shift = (l ? 1u : 0u) | ((l ? l - 1 : 0u) << 8);
}

constexpr uint32_t kMaxBatchRuns = 256;

// LDS bytes of one step workgroup.
size_t step_lds_bytes(uint32_t tile_isl, uint32_t N, uint32_t SW);
// ... and with the float births' draw queues (8 bytes per agent slot of the
// workgroup, block_threads * apt).
size_t step_lds_bytes(uint32_t tile_isl, uint32_t N, uint32_t SW, bool float_births,
                      uint32_t block_threads, uint32_t apt);

// tags: founders' trait words are random 16-bit founder tags (key k0, k1);
// counter may be nullptr (a synchronous run keeps no counter plane).
hipError_t launch_founders(uint32_t* trait, uint32_t* counter, uint32_t* surf, uint32_t A,
                           uint32_t SW, uint32_t* layout, uint32_t S, bool tags, uint32_t k0,
                           uint32_t k1, hipStream_t stream);

// Sites of ingests tau0 .. tau0 + count - 1 (ingest units) into
// sites[0 .. count - 1], one thread per ingest, and the run's layout after
// them (S words, ingest units), from the rule's constant-time tables
// (rules: the surface's one or two tables on the device).
hipError_t launch_run_sites(const RuleTable* rules, uint32_t kind, uint32_t S, uint32_t* sites,
                            uint32_t* layout, uint32_t tau0, uint32_t count, hipStream_t stream);

// agents_per_thread (1, 2 or 4) must divide N; tile_isl * N <= block_threads *
// agents_per_thread.
// Asynchronous runs keep the sites of their most recent kSiteRing ingests
// in a ring (filled from the rule's tables) for the common case, a parent
// counter near the tick; older counters take the tables directly.
constexpr uint32_t kSiteRing = 4096;
hipError_t launch_fill_site_ring(const RuleTable* rules, uint32_t kind, uint32_t S,
                                 uint32_t* ring, uint32_t tau0, uint32_t count,
                                 hipStream_t stream);

// Writes a run's layout (S words, given on the host) on the stream.
hipError_t launch_set_layout(uint32_t* layout, const uint32_t* words, uint32_t S,
                             hipStream_t stream);

hipError_t launch_step(const StepParams& p, uint32_t SW, uint32_t birth_model, bool migration,
                       uint32_t agents_per_thread, uint32_t block_threads, hipStream_t stream);
// The resident form: gens generations of a synchronous run whose torus is
// one tile (p.tile_isl >= p.I at block_threads), in one workgroup, from
// generation p.g on; sites holds the launch batch's schedule from ingest
// tau0 (launch_run_sites).
hipError_t launch_resident_step(const StepParams& p, uint32_t gens, const uint32_t* sites,
                                uint32_t tau0, uint32_t SW, uint32_t birth_model, bool migration,
                                uint32_t agents_per_thread, uint32_t block_threads,
                                hipStream_t stream);

// Batched forms.  Every run's sites for its generations T0 .. T0 + gens - 1 and its layout
// after them (launch_run_sites per run); max_gens bounds every run's gens.
hipError_t launch_batch_sites(const BatchRun* runs, uint32_t nruns, uint32_t max_gens,
                              hipStream_t stream);
// One generation of every run: total_tiles workgroups, workgroup b on XCD
// b mod kXcds as its (b / kXcds)-th.  xcd_tab (2 * kXcds * nruns words):
// for each XCD x, pre[x][i] = the offset of run i's chunk among x's
// workgroups (ascending in i, pre[x][0] = 0); then for each XCD x,
// first[x][i] = run i's first tile in that chunk.  The chunks of run i
// over all XCDs tile it exactly, and XCD x's chunks fill exactly its
// ceil((total_tiles - x) / kXcds) workgroups.
// with_float: some run of the batch uses kBirthFloat (a separate kernel, so
// that integer-only batches keep the integer kernel's register budget).
constexpr uint32_t kXcds = 8;
hipError_t launch_batch_step(const BatchRun* runs, const uint32_t* xcd_tab, uint32_t nruns,
                             uint32_t total_tiles, uint32_t k, uint32_t block_threads,
                             size_t lds_bytes, bool with_float, hipStream_t stream);

// Cut each of n runs' tiles (tiles[i], total T) into kXcds contiguous
// chunks, one per XCD, that fill exactly XCD x's ceil((T - x) / kXcds)
// workgroups, and write the xcd table launch_batch_step takes.  Each run
// gives every XCD tiles / kXcds of its tiles, and its tiles % kXcds
// remaining ones go one each to the XCDs with the most workgroups still
// unfilled.  The unfilled counts then never differ by more than one
// between XCDs, so none goes below zero and all reach zero together.
inline bool deal_tiles(const uint32_t* tiles, uint32_t n, uint32_t T, uint32_t* tab) {
    constexpr uint32_t X = kXcds;
    uint32_t left[X], filled[X];
    for (uint32_t x = 0; x < X; ++x) {
        left[x] = T > x ? (T - x + X - 1) / X : 0u;
        filled[x] = 0;
    }
    for (uint32_t i = 0; i < n; ++i) {
        uint32_t take[X];
        for (uint32_t x = 0; x < X; ++x) take[x] = tiles[i] / X;
        for (uint32_t r = 0; r < tiles[i] % X; ++r) {
            // the XCD with the most left after what it takes so far, ties
            // going round from a run-dependent start
            uint32_t best = X;
            for (uint32_t d = 0; d < X; ++d) {
                const uint32_t x = (i + d) % X;
                if (take[x] != tiles[i] / X) continue;      // has its extra tile
                if (best == X ||
                    (int64_t)left[x] - take[x] > (int64_t)left[best] - take[best])
                    best = x;
            }
            ++take[best];
        }
        uint32_t first = 0;
        for (uint32_t x = 0; x < X; ++x) {
            if (take[x] > left[x]) return false;
            tab[x * n + i] = filled[x];
            tab[(X + x) * n + i] = first;
            first += take[x];
            filled[x] += take[x];
            left[x] -= take[x];
        }
    }
    for (uint32_t x = 0; x < X; ++x)
        if (left[x]) return false;
    return true;
}

hipError_t launch_sample(const uint32_t* counter, const uint32_t* surf, uint32_t A, uint32_t SW,
                         uint32_t n, uint32_t T, uint32_t k0, uint32_t k1, uint32_t* idx_out,
                         uint32_t* counter_out, uint32_t* surf_out, hipStream_t stream);

hipError_t launch_probe_copy(const void* src, void* dst, size_t bytes, hipStream_t stream);

// Workspace layout of the MRCA kernels (bytes).
struct MrcaWorkspace {
    static constexpr size_t kHeader = 2048;   // flags, T, F, rank tables
    static constexpr size_t bytes(uint32_t S, uint32_t n) {
        const size_t ranked = ((size_t)n * 8 + 255) & ~(size_t)255;
        const size_t layouts = ((size_t)n * S * 4 + 255) & ~(size_t)255;
        const size_t sites = ((size_t)n * S + 255) & ~(size_t)255;
        return kHeader + ranked + layouts + sites;
    }
};

// A run's own layout (device, S words in ingest units) after the ingests of
// generation count T; the queries use it as it stands when every
// annotation's counter is T.
struct LayoutHint {
    const uint32_t* layout = nullptr;
    uint32_t T = 0;
    // the surface's site rule tables on the device (one, or two for hybrid)
    // in scheme_site's order: layouts from their closed form; nullptr:
    // replayed one placement per ingest
    const RuleTable* rules = nullptr;
};

// Bytes a query's workspace keeps for the rule's tables (after the
// MRCA or reconstruction workspace proper).
constexpr size_t kRuleRegionBytes = (2 * sizeof(RuleTable) + 255) & ~(size_t)255;

size_t phylo_workspace_bytes(uint32_t S, uint32_t n);
// leaf_parent (n), node_parent and node_time (n - 1), all device: the tree
// itself; NULL leaf_parent computes the metrics only.
hipError_t launch_phylo(const Scheme& sc, uint32_t n, const uint32_t* counter,
                        const uint32_t* surf, uint64_t* out, void* workspace, hipStream_t stream,
                        uint32_t* leaf_parent = nullptr, uint32_t* node_parent = nullptr,
                        uint32_t* node_time = nullptr, LayoutHint hint = {});

hipError_t launch_mrca(const Scheme& sc, uint32_t n, const uint32_t* counter,
                       const uint32_t* surf, uint32_t* lb, uint32_t* ub, void* workspace,
                       hipStream_t stream, LayoutHint hint = {});

// launch_mrca with the library's own static device scratch in place of a
// caller's workspace (at most kNoAllocMaxN annotations of up to 64 sites):
// no device memory is allocated.  The scratch's address on the current
// device is looked up once per device.
constexpr uint32_t kNoAllocMaxN = 4096;
constexpr size_t kNoAllocScratchBytes = MrcaWorkspace::bytes(64, kNoAllocMaxN);
hipError_t launch_mrca_noalloc(const Scheme& sc, uint32_t n, const uint32_t* counter,
                               const uint32_t* surf, uint32_t* lb, uint32_t* ub,
                               hipStream_t stream);

}  // namespace hsga
