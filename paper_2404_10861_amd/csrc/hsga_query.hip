// hsga_query.hip -- gfx950 kernels of the end-of-run queries and their
// launchers: the stratified sample, the MRCA-generation bounds of all pairs,
// and trie reconstruction (tree metrics and the tree itself).
#include <mutex>

#include "hsga_device.hpp"
#include "hsga_internal.hpp"

namespace hsga {

// ---------------------------------------------------------------------------
// Stratified end-of-run sample (Results, On-hardware Trial): agent k is
// drawn uniformly from the k-th of n equal strata; every agent when A <= n.
// counter == nullptr: a synchronous run, whose every counter is T.
__global__ __launch_bounds__(256) void sample_kernel(const uint32_t* __restrict__ counter,
                                                    const uint32_t* __restrict__ surf, uint32_t A,
                                                    uint32_t SW, uint32_t n, uint32_t T,
                                                    uint32_t k0, uint32_t k1,
                                                    uint32_t* __restrict__ idx_out,
                                                    uint32_t* __restrict__ counter_out,
                                                    uint32_t* __restrict__ surf_out) {
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t taken = A <= n ? A : n;
    if (k >= taken) return;
    uint32_t a = k;
    if (A > n) {
        const uint32_t lo = (uint32_t)((uint64_t)k * A / n);
        const uint32_t hi = (uint32_t)((uint64_t)(k + 1) * A / n);
        const uint4 w = philox4x32_10(make_uint4(k, 0u, T, kSample), k0, k1);
        a = lo + word_below(w.x, hi - lo);
    }
    idx_out[k] = a;
    counter_out[k] = counter ? counter[a] : T;
    for (uint32_t w = 0; w < SW; ++w) surf_out[(size_t)k * SW + w] = surf[(size_t)w * A + a];
}

hipError_t launch_sample(const uint32_t* counter, const uint32_t* surf, uint32_t A, uint32_t SW,
                         uint32_t n, uint32_t T, uint32_t k0, uint32_t k1, uint32_t* idx_out,
                         uint32_t* counter_out, uint32_t* surf_out, hipStream_t stream) {
    const uint32_t taken = A <= n ? A : n;
    const uint32_t blocks = (taken + 255) / 256;
    hipLaunchKernelGGL(sample_kernel, dim3(blocks ? blocks : 1), dim3(256), 0, stream, counter,
                       surf, A, SW, n, T, k0, k1, idx_out, counter_out, surf_out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// MRCA-generation bounds (Distributed Phylogenetic Tracking: mismatching
// differentiae delimit common ancestry).
//
// Workspace header words.
constexpr uint32_t kWsStatus = 0;  // 0 all counters equal, 1 mixed, 2 past horizon
constexpr uint32_t kWsT = 1;
constexpr uint32_t kWsF = 2;
constexpr uint32_t kWsPerm = 64;    // site of each time rank (ascending time)
constexpr uint32_t kWsTimes = 128;  // deposit time of each rank
constexpr uint32_t kWsLbTab = 192;  // 65 entries: lb when the first mismatch is rank r (64: none)
constexpr uint32_t kWsUbTab = 320;  // 65 entries: ub likewise
constexpr uint32_t kWsStatusMixed = 1, kWsStatusHorizon = 2;

// Rank of this lane's time among the S lanes (ascending; empty sites last,
// ties by lane).  All 64 lanes call it.
__device__ __forceinline__ uint32_t time_rank(uint32_t held, uint32_t lane, uint32_t S) {
    uint32_t rank = 0;
    for (uint32_t q = 0; q < S; ++q) {
        const uint32_t tq = __shfl(held, (int)q);
        rank += (tq < held || (tq == held && q < lane)) ? 1u : 0u;
    }
    return rank;
}

// Layout after T ingests, replayed in the wavefront (lane = site).
__device__ __forceinline__ uint32_t replay_layout(uint32_t kind, uint32_t S, uint32_t T,
                                                  uint32_t lane) {
    uint32_t held = kEmpty, leave = 0;
    place_items(kind, S, 0, T, held, leave, lane, [](uint32_t, int) {});
    return held;
}

// The item lane's site holds after T ingests: from the rule's tables when
// the query has them (constant time per site), else by the replay.
__device__ __forceinline__ uint32_t layout_lane(const RuleTable* rules, uint32_t kind, uint32_t S,
                                                uint32_t T, uint32_t lane) {
    if (rules) return scheme_item_at(rules, kind, S, T, lane);
    return replay_layout(kind, S, T, lane);
}

// Classify the counters (four wavefronts); when all are equal, wavefront 0
// lays out the shared layout once (in ingest units: from the rule's tables,
// or by replaying the placements when the caller has none), orders its
// sites by deposit time and tabulates the bounds, in generations, for every
// possible first-mismatch rank.  A run's own layout (hint, S words in
// ingest units, the layout after the ingests of generation count hint_T) is
// used as it stands when every counter is hint_T: the layout is a function
// of the scheme and the count alone, so all three give the same words.
constexpr uint32_t kPrepareThreads = 256;   // 4 wavefronts classify; wave 0 does the rest
__global__ __launch_bounds__(kPrepareThreads) void mrca_prepare_kernel(
    Scheme sc, uint32_t n, const uint32_t* __restrict__ counter, uint32_t* __restrict__ ws,
    const uint32_t* __restrict__ hint, uint32_t hint_T, const RuleTable* __restrict__ rules) {
    const uint32_t tid = threadIdx.x;
    const uint32_t lane = tid & 63u;
    const uint32_t S = sc.S;
    const uint32_t T0 = counter[0];
    const uint64_t hz = horizon_of(sc.kind, S);
    // past_hz: an item past the site rule's horizon; long: more ingests
    // than a replay may take (no limit when the run's layout is used)
    bool same = true, past_hz = false, long_replay = false;
    // 16 loads in flight per thread before any is used
    constexpr uint32_t kBatch = 16;
    for (uint32_t k0 = tid; k0 < n; k0 += kPrepareThreads * kBatch) {
        uint32_t c[kBatch];
#pragma unroll
        for (uint32_t j = 0; j < kBatch; ++j) {
            const uint32_t k = k0 + kPrepareThreads * j;
            c[j] = k < n ? counter[k] : T0;
        }
#pragma unroll
        for (uint32_t j = 0; j < kBatch; ++j) {
            const uint32_t ing = ingests_of(c[j], sc.interval);
            same = same && c[j] == T0;
            past_hz = past_hz || (ing > 0 && (uint64_t)(ing - 1) > hz);
            long_replay = long_replay || ing > kMaxReplayGenerations;
        }
    }
    // the four wavefronts' findings, combined through LDS
    __shared__ uint32_t flags[kPrepareThreads / 64];
    const uint32_t f_wave = (__ballot(!same) != 0 ? 1u : 0u) | (__ballot(past_hz) != 0 ? 2u : 0u) |
                            (__ballot(long_replay) != 0 ? 4u : 0u);
    if (lane == 0) flags[tid >> 6] = f_wave;
    __syncthreads();
    uint32_t f = 0;
#pragma unroll
    for (uint32_t w = 0; w < kPrepareThreads / 64; ++w) f |= flags[w];
    const bool all_same = (f & 1u) == 0;
    const bool hinted = all_same && hint && T0 == hint_T;
    const bool any_past = (f & 2u) != 0 || (!hinted && !rules && (f & 4u) != 0);
    if (any_past || !all_same) {                 // the same decision in every thread
        if (tid == 0) {
            ws[kWsStatus] = any_past ? kWsStatusHorizon : kWsStatusMixed;
            ws[kWsT] = T0;
        }
        return;
    }
    __shared__ uint32_t times[64];
    uint32_t F = 0;
    if (tid < 64) {                              // wavefront 0: lane = site
        const uint32_t held = hinted ? (lane < S ? hint[lane] : kEmpty)
                                     : layout_lane(rules, sc.kind, S,
                                                   ingests_of(T0, sc.interval), lane);
        const uint32_t rank = time_rank(held, lane, S);
        F = (uint32_t)__popcll(__ballot(lane < S && held != kEmpty));
        if (lane < S) {
            const uint32_t gen = held == kEmpty ? kEmpty : held * sc.interval;   // deposit generation
            times[rank] = gen;
            ws[kWsPerm + rank] = lane;
            ws[kWsTimes + rank] = gen;
        }
    }
    __syncthreads();
    if (tid >= 64) return;
    // first mismatch at rank r: ub = times[r], lb = times[r-1] + 1 (0 if r = 0);
    // no mismatch (entry 64): ub = T, lb = times[F-1] + 1 (0 if F = 0)
    ws[kWsLbTab + lane] = lane == 0 ? 0u : (lane < S ? times[lane - 1] + 1u : 0u);
    ws[kWsUbTab + lane] = lane < S ? times[lane] : 0u;
    if (lane == 0) {
        ws[kWsLbTab + 64] = F > 0 ? times[F - 1] + 1u : 0u;
        ws[kWsUbTab + 64] = T0;
        ws[kWsT] = T0;
        ws[kWsF] = F;
        ws[kWsStatus] = 0;
    }
}

// The annotation's surface words as one 64-bit value.
__device__ __forceinline__ uint64_t surface64(const uint32_t* __restrict__ surf, uint32_t SW,
                                              uint32_t a) {
    return SW == 2 ? ((uint64_t)surf[(size_t)a * 2 + 1] << 32) | surf[(size_t)a * 2]
                   : (uint64_t)surf[a];
}

// Fast route: each annotation's differentiae in ascending-time order, packed
// in 64 bits (rank r at bit r for one-bit differentiae, at byte r for bytes).
__global__ __launch_bounds__(256) void mrca_rank_kernel(uint32_t S, uint32_t diff_log2,
                                                       uint32_t n,
                                                       const uint32_t* __restrict__ surf,
                                                       const uint32_t* __restrict__ ws,
                                                       uint64_t* __restrict__ ranked) {
    if (ws[kWsStatus] != 0) return;
    __shared__ uint32_t perm[64];
    if (threadIdx.x < 64) perm[threadIdx.x] = ws[kWsPerm + threadIdx.x];
    __syncthreads();
    const uint32_t a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= n) return;
    const uint32_t F = ws[kWsF];
    const uint64_t s = surface64(surf, (S << diff_log2) >> 5, a);
    const uint64_t mask = diff_log2 ? 0xffull : 1ull;
    uint64_t packed = 0;
    for (uint32_t r = 0; r < F; ++r)
        packed |= ((s >> (perm[r] << diff_log2)) & mask) << (r << diff_log2);
    ranked[a] = packed;
}

// Fast route, all ordered pairs: x = P_a xor P_b; the first set bit gives
// the rank of the first mismatch (its bit index, or its byte index).  Each thread owns 4 adjacent columns of 4
// rows, so stores are 16-byte and a wavefront writes 1 KiB contiguously.
constexpr uint32_t kPairRows = 4;
__global__ __launch_bounds__(256) void mrca_allpairs_kernel(uint32_t n, uint32_t diff_log2,
                                                           const uint64_t* __restrict__ ranked,
                                                           const uint32_t* __restrict__ ws,
                                                           uint32_t* __restrict__ lb,
                                                           uint32_t* __restrict__ ub) {
    const uint32_t status = ws[kWsStatus];
    if (status == kWsStatusHorizon) {
        // a counter past the horizon: every bound reads 0xFFFFFFFF, a value
        // no valid bound takes (bounds are at most 2^32 - 2)
        const uint32_t c0 = (blockIdx.x * blockDim.x + threadIdx.x) * 4u;
        for (uint32_t rr = 0; rr < kPairRows; ++rr) {
            const uint32_t a = blockIdx.y * kPairRows + rr;
            for (uint32_t q = 0; q < 4; ++q) {
                if (a < n && c0 + q < n) {
                    lb[(size_t)a * n + c0 + q] = kEmpty;
                    ub[(size_t)a * n + c0 + q] = kEmpty;
                }
            }
        }
        return;
    }
    if (status != 0) return;
    __shared__ uint32_t lbt[65], ubt[65];
    if (threadIdx.x < 65) {
        lbt[threadIdx.x] = ws[kWsLbTab + threadIdx.x];
        ubt[threadIdx.x] = ws[kWsUbTab + threadIdx.x];
    }
    __syncthreads();
    const uint32_t c0 = (blockIdx.x * blockDim.x + threadIdx.x) * 4u;
    if (c0 >= n) return;
    const uint32_t a0 = blockIdx.y * kPairRows;
    uint64_t pb[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) pb[q] = c0 + q < n ? ranked[c0 + q] : 0ull;
    const bool vec = (n & 3u) == 0;
    for (uint32_t rr = 0; rr < kPairRows; ++rr) {
        const uint32_t a = a0 + rr;
        if (a >= n) break;
        const uint64_t pa = ranked[a];
        uint32_t l[4], u[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const uint64_t x = pa ^ pb[q];
            const uint32_t idx =
                x ? ((uint32_t)(__ffsll((long long)x) - 1) >> diff_log2) : 64u;
            l[q] = lbt[idx];
            u[q] = ubt[idx];
        }
        const size_t off = (size_t)a * n + c0;
        if (vec) {
            *reinterpret_cast<uint4*>(lb + off) = make_uint4(l[0], l[1], l[2], l[3]);
            *reinterpret_cast<uint4*>(ub + off) = make_uint4(u[0], u[1], u[2], u[3]);
        } else {
            for (uint32_t q = 0; q < 4 && c0 + q < n; ++q) {
                lb[off + q] = l[q];
                ub[off + q] = u[q];
            }
        }
    }
}

// General route (counters differ): one wavefront per annotation lays out
// its own layout (from the rule's tables, else by replay) and stores its
// retained deposit generations in ascending order with their sites.
__global__ __launch_bounds__(64) void mrca_layouts_kernel(Scheme sc,
                                                         const uint32_t* __restrict__ counter,
                                                         const uint32_t* __restrict__ ws,
                                                         uint32_t* __restrict__ times,
                                                         uint8_t* __restrict__ sites,
                                                         const RuleTable* __restrict__ rules) {
    if (ws[kWsStatus] != kWsStatusMixed) return;
    const uint32_t a = blockIdx.x;
    const uint32_t lane = threadIdx.x;
    const uint32_t S = sc.S;
    const uint32_t held = layout_lane(rules, sc.kind, S, ingests_of(counter[a], sc.interval), lane);
    const uint32_t rank = time_rank(held, lane, S);
    if (lane < S) {
        times[(size_t)a * S + rank] = held == kEmpty ? kEmpty : held * sc.interval;
        sites[(size_t)a * S + rank] = (uint8_t)lane;
    }
}

// General route, all ordered pairs: merge the two ascending time lists,
// comparing differentiae on common times until the first mismatch.
constexpr uint32_t kGeneralPairRows = 512;   // grid rows of the general pairs kernel
__global__ __launch_bounds__(256) void mrca_general_pairs_kernel(
    uint32_t S, uint32_t diff_log2, uint32_t n, const uint32_t* __restrict__ counter,
    const uint32_t* __restrict__ surf, const uint32_t* __restrict__ times,
    const uint8_t* __restrict__ sites, const uint32_t* __restrict__ ws, uint32_t* __restrict__ lb,
    uint32_t* __restrict__ ub) {
    if (ws[kWsStatus] != kWsStatusMixed) return;
    const uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n) return;
    const uint32_t SW = (S << diff_log2) >> 5;
    const uint64_t sb = surface64(surf, SW, b);
    const uint64_t mask = diff_log2 ? 0xffull : 1ull;
    const uint32_t* tb = times + (size_t)b * S;
    const uint8_t* kb = sites + (size_t)b * S;
    const uint32_t Tb = counter[b];
    // rows a = blockIdx.y, blockIdx.y + gridDim.y, ...: a small grid, so that
    // the shared-counter route, which skips this kernel, pays little for it
    for (uint32_t a = blockIdx.y; a < n; a += gridDim.y) {
        const uint64_t sa = surface64(surf, SW, a);
        const uint32_t* ta = times + (size_t)a * S;
        const uint8_t* ka = sites + (size_t)a * S;
        uint32_t i = 0, k = 0;
        bool have_last = false, mismatch = false;
        uint32_t last = 0, tstar = 0;
        while (i < S && k < S) {
            const uint32_t x = ta[i], y = tb[k];
            if (x == kEmpty || y == kEmpty) break;
            if (x == y) {
                if (((sa >> ((uint32_t)ka[i] << diff_log2)) & mask) !=
                    ((sb >> ((uint32_t)kb[k] << diff_log2)) & mask)) {
                    mismatch = true;
                    tstar = x;
                    break;
                }
                have_last = true;
                last = x;
                ++i;
                ++k;
            } else if (x < y) {
                ++i;
            } else {
                ++k;
            }
        }
        const uint32_t Ta = counter[a];
        const size_t off = (size_t)a * n + b;
        ub[off] = mismatch ? tstar : (Ta < Tb ? Ta : Tb);
        lb[off] = have_last ? last + 1u : 0u;
    }
}

// ---------------------------------------------------------------------------
// Trie reconstruction and phylometrics of annotations sharing a counter
// (Distributed Phylogenetic Tracking: reconstruction is a trie over the
// record of differentiae; Results, On-hardware Trial: sum branch length and
// mean evolutionary distinctiveness).  Annotations read as their
// differentiae in ascending deposit time are sorted lexicographically;
// neighbours in that order share a prefix of d_i = LCP(i, i+1) retained
// items, and the trie's branching nodes are exactly these boundaries.  A
// node at depth d sits at time tau(d) = t_d (the MRCA upper bound of the
// pairs it separates), tau(F) = T (identical annotations).
//   boundaries of one node: equal depth d with nothing shallower between
//     (a many-way split, or a run of identical annotations); the node
//     starts at the boundary whose nearest not-deeper left neighbour is
//     strictly shallower;
//   leaf i hangs from the deeper of boundaries i-1, i;
//   a node hangs from the deeper of its nearest strictly shallower
//   boundaries on either side (none: the root);
//   pairs (a, b) meet at the shallowest boundary between them, so the sum
//   over pairs of T - tau(MRCA) is a sum over all boundary ranges of their
//   minimum, counted by nearest-smaller spans.
// Six result words: sum of branch lengths, pair sum, root time, internal
// nodes, status, n.

// Sort keys: rank 0 most significant (bit-reversed for one-bit
// differentiae, byte-reversed for bytes).
__global__ __launch_bounds__(256) void phylo_keys_kernel(uint32_t n, uint32_t npad,
                                                        uint32_t diff_log2,
                                                        const uint64_t* __restrict__ ranked,
                                                        const uint32_t* __restrict__ ws,
                                                        uint64_t* __restrict__ keys,
                                                        uint32_t* __restrict__ idx) {
    if (ws[kWsStatus] != 0) return;
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npad) return;
    uint64_t key = ~0ull;
    if (i < n) key = diff_log2 ? __builtin_bswap64(ranked[i]) : __brevll(ranked[i]);
    keys[i] = key;
    idx[i] = i < n ? i : 0xffffffffu;
}

// Bitonic sort of (key, index) over npad (a power of two) entries, ascending
// by key then index.  The network is the usual one: for k = 2, 4, .., npad
// and j = k/2, .., 1, entries i and i + j (i with bit j clear) are ordered
// ascending where bit k of i is clear and descending where it is set.
// Stages with j < kSortChunk stay inside aligned chunks of kSortChunk
// entries, so each workgroup runs them in LDS: all stages of k <= the chunk
// at once (phylo_sort_local_kernel), and for each larger k its strides
// below the chunk after the strides at or above it, which take one launch
// each over the whole array (phylo_sort_global_kernel).
constexpr uint32_t kSortChunk = 2048;

__device__ __forceinline__ void sort_exchange(uint64_t& ka, uint32_t& ia, uint64_t& kb,
                                              uint32_t& ib, bool up) {
    const bool greater = ka > kb || (ka == kb && ia > ib);
    if (greater == up) {
        const uint64_t tk = ka;
        ka = kb;
        kb = tk;
        const uint32_t ti = ia;
        ia = ib;
        ib = ti;
    }
}

// One chunk of `chunk` entries (a power of two, at most kSortChunk) per
// workgroup of chunk / 2 threads.  k_only = 0: every stage with k <= chunk;
// otherwise the stages j = chunk/2 .. 1 of k = k_only.
__global__ __launch_bounds__(kSortChunk / 2) void phylo_sort_local_kernel(
    uint32_t chunk, uint32_t k_only, const uint32_t* __restrict__ ws, uint64_t* __restrict__ keys,
    uint32_t* __restrict__ idx) {
    if (ws[kWsStatus] != 0) return;
    __shared__ uint64_t sk[kSortChunk];
    __shared__ uint32_t si[kSortChunk];
    const uint32_t base = blockIdx.x * chunk;
    const uint32_t t = threadIdx.x;
    sk[t] = keys[base + t];
    si[t] = idx[base + t];
    sk[t + chunk / 2] = keys[base + t + chunk / 2];
    si[t + chunk / 2] = idx[base + t + chunk / 2];
    __syncthreads();
    const uint32_t k_first = k_only ? k_only : 2u;
    const uint32_t k_last = k_only ? k_only : chunk;
    for (uint32_t k = k_first; k <= k_last; k <<= 1) {
        for (uint32_t j = (k_only ? chunk : k) >> 1; j > 0; j >>= 1) {
            const uint32_t i = (t / j) * 2 * j + (t % j);
            const bool up = ((base + i) & k) == 0;
            sort_exchange(sk[i], si[i], sk[i + j], si[i + j], up);
            __syncthreads();
        }
    }
    keys[base + t] = sk[t];
    idx[base + t] = si[t];
    keys[base + t + chunk / 2] = sk[t + chunk / 2];
    idx[base + t + chunk / 2] = si[t + chunk / 2];
}

// Stage (k, j) over the whole array, one pair per thread (npad / 2 threads).
__global__ __launch_bounds__(256) void phylo_sort_global_kernel(uint32_t npad, uint32_t k,
                                                                uint32_t j,
                                                                const uint32_t* __restrict__ ws,
                                                                uint64_t* __restrict__ keys,
                                                                uint32_t* __restrict__ idx) {
    if (ws[kWsStatus] != 0) return;
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= npad / 2) return;
    const uint32_t i = (t / j) * 2 * j + (t % j);
    const uint32_t l = i + j;
    uint64_t ki = keys[i], kl = keys[l];
    uint32_t ii = idx[i], il = idx[l];
    sort_exchange(ki, ii, kl, il, (i & k) == 0);
    keys[i] = ki;
    keys[l] = kl;
    idx[i] = ii;
    idx[l] = il;
}

void launch_phylo_sort(uint32_t npad, const uint32_t* ws, uint64_t* keys, uint32_t* idx,
                       hipStream_t stream) {
    if (npad < 2) return;
    const uint32_t chunk = npad < kSortChunk ? npad : kSortChunk;
    const uint32_t chunks = npad / chunk;
    hipLaunchKernelGGL(phylo_sort_local_kernel, dim3(chunks), dim3(chunk / 2), 0, stream, chunk,
                       0u, ws, keys, idx);
    for (uint32_t k = 2 * chunk; k <= npad; k <<= 1) {
        for (uint32_t j = k >> 1; j >= chunk; j >>= 1)
            hipLaunchKernelGGL(phylo_sort_global_kernel, dim3((npad / 2 + 255) / 256), dim3(256),
                               0, stream, npad, k, j, ws, keys, idx);
        hipLaunchKernelGGL(phylo_sort_local_kernel, dim3(chunks), dim3(chunk / 2), 0, stream,
                           chunk, k, ws, keys, idx);
    }
}

// Boundary depths and the tree, in parallel.  tab[k][i] = the minimum depth
// over boundaries [i, i + 2^k) (a sparse table); the nearest boundary to the
// left or right of b shallower than a depth is found by binary lifting over
// it, one thread per boundary.  Sums go to 64-bit accumulators.
constexpr uint32_t kPhyloMaxLevels = 17;   // 2^16 > 65534 boundaries
constexpr uint32_t kNoBoundary = 0xffffffffu;

struct PhyloAcc {
    unsigned long long sbl, pairs, internal, dmin;
};

__device__ __forceinline__ uint64_t phylo_tau(const uint32_t* ws, uint32_t d) {
    const uint32_t F = ws[kWsF];
    return d < F ? (uint64_t)ws[kWsTimes + d] : (uint64_t)ws[kWsT];
}

__global__ __launch_bounds__(256) void phylo_depth_kernel(uint32_t n, uint32_t diff_log2,
                                                         const uint32_t* __restrict__ ws,
                                                         const uint64_t* __restrict__ keys,
                                                         uint8_t* __restrict__ depth,
                                                         PhyloAcc* __restrict__ acc) {
    if (ws[kWsStatus] != 0) return;
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t F = ws[kWsF];
    if (i == 0) {
        acc->sbl = 0;
        acc->pairs = 0;
        acc->internal = 0;
        acc->dmin = F;
    }
    if (i + 1 < n) {
        const uint64_t x = keys[i] ^ keys[i + 1];
        const uint32_t d = x ? ((uint32_t)__clzll((long long)x) >> diff_log2) : 64u;
        depth[i] = (uint8_t)(d < F ? d : F);
    }
}

// Level k of the sparse table from level k - 1 (m boundaries per level).
__global__ __launch_bounds__(256) void phylo_table_kernel(uint32_t m, uint32_t k,
                                                         const uint32_t* __restrict__ ws,
                                                         uint8_t* __restrict__ tab) {
    if (ws[kWsStatus] != 0) return;
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t half = 1u << (k - 1);
    if (i + 2 * half > m) return;
    const uint8_t* prev = tab + (size_t)(k - 1) * m;
    const uint8_t a = prev[i], b = prev[i + half];
    tab[(size_t)k * m + i] = a < b ? a : b;
}

// Nearest boundary i < b with depth[i] < d.
__device__ __forceinline__ uint32_t phylo_left_below(const uint8_t* tab, uint32_t m,
                                                     uint32_t levels, uint32_t b, uint32_t d) {
    uint32_t pos = b;   // every boundary in [pos, b) is at depth >= d
    for (uint32_t k = levels; k-- > 0;) {
        const uint32_t len = 1u << k;
        if (pos >= len && tab[(size_t)k * m + pos - len] >= d) pos -= len;
    }
    return pos == 0 ? kNoBoundary : pos - 1;
}

// Nearest boundary i > b with depth[i] < d.
__device__ __forceinline__ uint32_t phylo_right_below(const uint8_t* tab, uint32_t m,
                                                      uint32_t levels, uint32_t b, uint32_t d) {
    uint32_t pos = b + 1;   // every boundary in (b, pos) is at depth >= d
    for (uint32_t k = levels; k-- > 0;) {
        const uint32_t len = 1u << k;
        if (pos + len <= m && tab[(size_t)k * m + pos] >= d) pos += len;
    }
    return pos >= m ? kNoBoundary : pos;
}

__device__ __forceinline__ void phylo_add(PhyloAcc* acc, uint64_t sbl, uint64_t pairs,
                                          uint64_t internal, uint32_t dmin) {
    __shared__ unsigned long long s_sbl, s_pairs, s_internal;
    __shared__ uint32_t s_dmin;
    if (threadIdx.x == 0) {
        s_sbl = 0;
        s_pairs = 0;
        s_internal = 0;
        s_dmin = 0xffffffffu;
    }
    __syncthreads();
    if (sbl) atomicAdd(&s_sbl, (unsigned long long)sbl);
    if (pairs) atomicAdd(&s_pairs, (unsigned long long)pairs);
    if (internal) atomicAdd(&s_internal, (unsigned long long)internal);
    if (dmin != 0xffffffffu) atomicMin(&s_dmin, dmin);
    __syncthreads();
    if (threadIdx.x == 0) {
        if (s_sbl) atomicAdd(&acc->sbl, s_sbl);
        if (s_pairs) atomicAdd(&acc->pairs, s_pairs);
        if (s_internal) atomicAdd(&acc->internal, s_internal);
        if (s_dmin != 0xffffffffu) atomicMin(&acc->dmin, (unsigned long long)s_dmin);
    }
}

// One thread per boundary b (depth d):
//   pairs meeting at b (b the rightmost shallowest boundary between them):
//     (b - L) (Rq - b), L = nearest left shallower (-1 if none), Rq =
//     nearest right not deeper (m if none), each adding T - tau(d);
//   a tree node starts at b unless the nearest not-deeper boundary on its
//   left has the same depth (one many-way node, or a run of identical
//   annotations); the node hangs from the deeper of its nearest shallower
//   boundaries (none on either side: the root).
__global__ __launch_bounds__(256) void phylo_boundary_kernel(uint32_t m, uint32_t levels,
                                                            const uint32_t* __restrict__ ws,
                                                            const uint8_t* __restrict__ tab,
                                                            PhyloAcc* __restrict__ acc) {
    if (ws[kWsStatus] != 0) return;
    const uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
    uint64_t sbl = 0, pairs = 0, internal = 0;
    uint32_t dmin = 0xffffffffu;
    if (b < m) {
        const uint8_t* depth = tab;
        const uint32_t d = depth[b];
        const uint64_t T = ws[kWsT];
        const uint32_t L = phylo_left_below(tab, m, levels, b, d);
        const uint32_t Lq = phylo_left_below(tab, m, levels, b, d + 1);
        const uint32_t R = phylo_right_below(tab, m, levels, b, d);
        const uint32_t Rq = phylo_right_below(tab, m, levels, b, d + 1);
        const uint64_t nl = (uint64_t)b - (L == kNoBoundary ? (uint64_t)-1 : L);
        const uint64_t nr = (uint64_t)(Rq == kNoBoundary ? m : Rq) - b;
        pairs = (T - phylo_tau(ws, d)) * nl * nr;
        dmin = d;
        if (Lq == kNoBoundary || depth[Lq] < d) {
            internal = 1;
            if (L != kNoBoundary || R != kNoBoundary) {
                uint32_t pd;
                if (L == kNoBoundary) pd = depth[R];
                else if (R == kNoBoundary) pd = depth[L];
                else pd = depth[L] > depth[R] ? depth[L] : depth[R];
                sbl = phylo_tau(ws, d) - phylo_tau(ws, pd);
            }
        }
    }
    phylo_add(acc, sbl, pairs, internal, dmin);
}

// One thread per leaf: its edge from the deeper adjacent boundary to T.
__global__ __launch_bounds__(256) void phylo_leaf_kernel(uint32_t n,
                                                        const uint32_t* __restrict__ ws,
                                                        const uint8_t* __restrict__ depth,
                                                        PhyloAcc* __restrict__ acc) {
    if (ws[kWsStatus] != 0) return;
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    uint64_t sbl = 0;
    if (i < n && n > 1) {
        const uint32_t m = n - 1;
        uint32_t pd = i > 0 ? depth[i - 1] : 0u;
        if (i < m && (i == 0 || depth[i] > pd)) pd = depth[i];
        sbl = (uint64_t)ws[kWsT] - phylo_tau(ws, pd);
    }
    phylo_add(acc, sbl, 0, 0, 0xffffffffu);
}

__global__ __launch_bounds__(64) void phylo_finish_kernel(uint32_t n,
                                                         const uint32_t* __restrict__ ws,
                                                         const PhyloAcc* __restrict__ acc,
                                                         uint64_t* __restrict__ out) {
    if (threadIdx.x != 0) return;
    const uint32_t status = ws[kWsStatus];
    if (status != 0) {
        out[0] = out[1] = out[2] = out[3] = out[6] = out[7] = 0;
    } else {
        out[0] = acc->sbl;
        out[1] = acc->pairs;
        out[2] = n > 1 ? phylo_tau(ws, (uint32_t)acc->dmin) : ws[kWsT];
        out[3] = acc->internal;
        // the means, as binary64: mean evolutionary distinctiveness under
        // fair proportion (each edge shared equally by the leaves below it)
        // is the sum of branch lengths over n; the mean pairwise distance
        // is twice the pair sum over the n(n-1)/2 pairs (a path runs from
        // each leaf up to their MRCA)
        const double pairs = (double)n * (double)(n - 1) * 0.5;
        const double ed = (double)acc->sbl / (double)n;
        const double mpd = n > 1 ? 2.0 * (double)acc->pairs / pairs : 0.0;
        out[6] = (uint64_t)__double_as_longlong(ed);
        out[7] = (uint64_t)__double_as_longlong(mpd);
    }
    out[4] = status;
    out[5] = n;
}

// The tree itself.  A node is named by the first boundary of its run (the
// first boundary after its nearest shallower left boundary L that is not
// deeper than it).
constexpr uint32_t kPhyloRoot = 0xffffffffu, kPhyloNotNode = 0xfffffffeu;

__device__ __forceinline__ uint32_t phylo_node_of(const uint8_t* tab, uint32_t m,
                                                  uint32_t levels, uint32_t b) {
    const uint32_t d = tab[b];
    const uint32_t L = phylo_left_below(tab, m, levels, b, d);
    if (L == kNoBoundary) return tab[0] <= d ? 0u : phylo_right_below(tab, m, levels, 0, d + 1);
    return phylo_right_below(tab, m, levels, L, d + 1);
}

// One thread per boundary: node_parent[b] = the parent node (kPhyloRoot for
// the root) when b starts a node, kPhyloNotNode otherwise; node_time[b] =
// the time of b's node.
__global__ __launch_bounds__(256) void phylo_tree_kernel(uint32_t m, uint32_t levels,
                                                        const uint32_t* __restrict__ ws,
                                                        const uint8_t* __restrict__ tab,
                                                        uint32_t* __restrict__ node_parent,
                                                        uint32_t* __restrict__ node_time) {
    if (ws[kWsStatus] != 0) return;
    const uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= m) return;
    const uint32_t d = tab[b];
    node_time[b] = (uint32_t)phylo_tau(ws, d);
    const uint32_t Lq = phylo_left_below(tab, m, levels, b, d + 1);
    if (Lq != kNoBoundary && tab[Lq] == d) {
        node_parent[b] = kPhyloNotNode;
        return;
    }
    const uint32_t L = phylo_left_below(tab, m, levels, b, d);
    const uint32_t R = phylo_right_below(tab, m, levels, b, d);
    if (L == kNoBoundary && R == kNoBoundary) {
        node_parent[b] = kPhyloRoot;
        return;
    }
    uint32_t p;
    if (L == kNoBoundary) p = R;
    else if (R == kNoBoundary) p = L;
    else p = tab[L] >= tab[R] ? L : R;
    node_parent[b] = phylo_node_of(tab, m, levels, p);
}

// One thread per sorted position i: the annotation idx[i] hangs from the
// node of the deeper adjacent boundary.
__global__ __launch_bounds__(256) void phylo_tree_leaf_kernel(uint32_t n, uint32_t levels,
                                                             const uint32_t* __restrict__ ws,
                                                             const uint8_t* __restrict__ tab,
                                                             const uint32_t* __restrict__ idx,
                                                             uint32_t* __restrict__ leaf_parent) {
    if (ws[kWsStatus] != 0) return;
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (n == 1) {
        leaf_parent[idx[i]] = kPhyloRoot;
        return;
    }
    const uint32_t m = n - 1;
    uint32_t pb;
    if (i == 0) pb = 0;
    else if (i == m) pb = m - 1;
    else pb = tab[i] > tab[i - 1] ? i : i - 1;
    leaf_parent[idx[i]] = phylo_node_of(tab, m, levels, pb);
}

size_t phylo_workspace_bytes(uint32_t S, uint32_t n) {
    size_t npad = 1;
    while (npad < n) npad <<= 1;
    const size_t a = (MrcaWorkspace::bytes(S, n) + 255) & ~(size_t)255;
    return a + npad * 8 + npad * 4 + 256 + (size_t)kPhyloMaxLevels * n + 1024;
}

hipError_t launch_phylo(const Scheme& scm, uint32_t n, const uint32_t* counter,
                        const uint32_t* surf, uint64_t* out, void* workspace,
                        hipStream_t stream, uint32_t* leaf_parent, uint32_t* node_parent,
                        uint32_t* node_time, LayoutHint hint) {
    const uint32_t diff_log2 = scm.bits == 8 ? 3u : 0u;
    uint8_t* base = static_cast<uint8_t*>(workspace);
    uint32_t* ws = reinterpret_cast<uint32_t*>(base);
    uint64_t* ranked = reinterpret_cast<uint64_t*>(base + MrcaWorkspace::kHeader);
    size_t npad = 1;
    while (npad < n) npad <<= 1;
    size_t off = (MrcaWorkspace::bytes(scm.S, n) + 255) & ~(size_t)255;
    uint64_t* keys = reinterpret_cast<uint64_t*>(base + off);   off += npad * 8;
    uint32_t* idx = reinterpret_cast<uint32_t*>(base + off);    off += npad * 4;
    off = (off + 255) & ~(size_t)255;
    PhyloAcc* acc = reinterpret_cast<PhyloAcc*>(base + off);    off += 256;
    uint8_t* tab = base + off;                                  // levels x m bytes
    const uint32_t m = n - 1;
    uint32_t levels = 1;
    while (levels < kPhyloMaxLevels && (2u << (levels - 1)) <= m) ++levels;
    const uint32_t gn = (n + 255) / 256;
    hipLaunchKernelGGL(mrca_prepare_kernel, dim3(1), dim3(kPrepareThreads), 0, stream, scm, n,
                       counter, ws, hint.layout, hint.T, hint.rules);
    hipLaunchKernelGGL(mrca_rank_kernel, dim3(gn), dim3(256), 0, stream, scm.S, diff_log2, n,
                       surf, ws, ranked);
    hipLaunchKernelGGL(phylo_keys_kernel, dim3((uint32_t)((npad + 255) / 256)), dim3(256), 0,
                       stream, n, (uint32_t)npad, diff_log2, ranked, ws, keys, idx);
    launch_phylo_sort((uint32_t)npad, ws, keys, idx, stream);
    hipLaunchKernelGGL(phylo_depth_kernel, dim3(gn), dim3(256), 0, stream, n, diff_log2, ws, keys,
                       tab, acc);
    for (uint32_t k = 1; k < levels; ++k)
        hipLaunchKernelGGL(phylo_table_kernel, dim3(gn), dim3(256), 0, stream, m, k, ws, tab);
    if (m > 0)
        hipLaunchKernelGGL(phylo_boundary_kernel, dim3((m + 255) / 256), dim3(256), 0, stream, m,
                           levels, ws, tab, acc);
    hipLaunchKernelGGL(phylo_leaf_kernel, dim3(gn), dim3(256), 0, stream, n, ws, tab, acc);
    hipLaunchKernelGGL(phylo_finish_kernel, dim3(1), dim3(64), 0, stream, n, ws, acc, out);
    if (leaf_parent) {
        if (m > 0)
            hipLaunchKernelGGL(phylo_tree_kernel, dim3((m + 255) / 256), dim3(256), 0, stream, m,
                               levels, ws, tab, node_parent, node_time);
        hipLaunchKernelGGL(phylo_tree_leaf_kernel, dim3(gn), dim3(256), 0, stream, n, levels, ws,
                           tab, idx, leaf_parent);
    }
    return hipGetLastError();
}

hipError_t launch_mrca(const Scheme& scm, uint32_t n, const uint32_t* counter,
                       const uint32_t* surf, uint32_t* lb, uint32_t* ub, void* workspace,
                       hipStream_t stream, LayoutHint hint) {
    const uint32_t S = scm.S;
    const uint32_t diff_log2 = scm.bits == 8 ? 3u : 0u;
    uint8_t* base = static_cast<uint8_t*>(workspace);
    uint32_t* ws = reinterpret_cast<uint32_t*>(base);
    uint64_t* ranked = reinterpret_cast<uint64_t*>(base + MrcaWorkspace::kHeader);
    const size_t ranked_bytes = ((size_t)n * 8 + 255) & ~(size_t)255;
    uint32_t* times = reinterpret_cast<uint32_t*>(base + MrcaWorkspace::kHeader + ranked_bytes);
    const size_t times_bytes = ((size_t)n * S * 4 + 255) & ~(size_t)255;
    uint8_t* sites = base + MrcaWorkspace::kHeader + ranked_bytes + times_bytes;

    hipLaunchKernelGGL(mrca_prepare_kernel, dim3(1), dim3(kPrepareThreads), 0, stream, scm, n,
                       counter, ws, hint.layout, hint.T, hint.rules);
    hipLaunchKernelGGL(mrca_rank_kernel, dim3((n + 255) / 256), dim3(256), 0, stream, S,
                       diff_log2, n, surf, ws, ranked);
    hipLaunchKernelGGL(mrca_allpairs_kernel, dim3((n + 1023) / 1024, (n + kPairRows - 1) / kPairRows),
                       dim3(256), 0, stream, n, diff_log2, ranked, ws, lb, ub);
    hipLaunchKernelGGL(mrca_layouts_kernel, dim3(n), dim3(64), 0, stream, scm, counter, ws,
                       times, sites, hint.rules);
    const uint32_t rows = n < kGeneralPairRows ? n : kGeneralPairRows;
    hipLaunchKernelGGL(mrca_general_pairs_kernel, dim3((n + 255) / 256, rows), dim3(256), 0,
                       stream, S, diff_log2, n, counter, surf, times, sites, ws, lb, ub);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Allocation-free MRCA bounds: the workspace is a static device array that
// the library holds, one copy per device (the array's name is a host-side
// stand-in, so kernels take its device address, looked up once per device
// with that device current).  Every call on a device shares its copy: calls
// that overlap on one device race.  Nothing in the workspace needs clearing
// first: the prepare kernel writes every word the later kernels read.
static __device__ __align__(256) uint8_t scratch[kNoAllocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t launch_mrca_noalloc(const Scheme& scm, uint32_t n, const uint32_t* counter,
                               const uint32_t* surf, uint32_t* lb, uint32_t* ub,
                               hipStream_t stream) {
    if (n == 0 || n > kNoAllocMaxN || scm.S > 64) return hipErrorInvalidValue;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    void* ptr = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_scratch_mutex);
        if (!g_scratch_ptr[dev]) {
            e = hipGetSymbolAddress(&g_scratch_ptr[dev], HIP_SYMBOL(scratch));
            if (e != hipSuccess) {
                g_scratch_ptr[dev] = nullptr;
                return e;
            }
        }
        ptr = g_scratch_ptr[dev];
    }
    return launch_mrca(scm, n, counter, surf, lb, ub, ptr, stream);
}

}  // namespace hsga
