// hsga_kernels.hip -- gfx950 kernels of the island-model GA with
// hereditary-stratigraphy surface annotations (founders, site schedule, the
// generation step, its batched form), and their launchers.  The end-of-run
// queries live in hsga_query.hip.
//
// Device state is structure-of-arrays: trait[A], the S/32 surface word
// planes [S/32][A] and, for asynchronous runs only, counter[A] (in a
// synchronous run every counter is the generation number), agent a =
// island * N + slot.  Consecutive
// lanes own consecutive agents, so every population read and write is a
// contiguous 256-byte wavefront access per plane.
#include "hsga_device.hpp"
#include "hsga_internal.hpp"

namespace hsga {

// ---------------------------------------------------------------------------
// Founders (Genome Model; Distributed Phylogenetic Tracking): trait 0,
// counter 0 (written only when the run keeps a counter plane), every site
// 0, and an empty layout.  Founders carry no
// differentia; item g is deposited by generation g's births.  With founder
// tags (Results, Clade Reconstruction Trial) the trait word is instead a
// random 16-bit identifier: the low half of the first word of Philox block
// (a, 0, 0, founder).
__global__ __launch_bounds__(256) void founders_kernel(uint32_t* __restrict__ trait,
                                                      uint32_t* __restrict__ counter,
                                                      uint32_t* __restrict__ surf, uint32_t A,
                                                      uint32_t SW, uint32_t* __restrict__ layout,
                                                      uint32_t S, uint32_t tags, uint32_t k0,
                                                      uint32_t k1) {
    const uint32_t stride = gridDim.x * blockDim.x;
    const uint32_t first = blockIdx.x * blockDim.x + threadIdx.x;
    for (uint32_t a = first; a < A; a += stride) {
        trait[a] = tags ? philox4x32_10(make_uint4(a, 0u, 0u, kFounder), k0, k1).x & 0xffffu : 0u;
        if (counter) counter[a] = 0u;
        for (uint32_t w = 0; w < SW; ++w) surf[(size_t)w * A + a] = 0u;
    }
    if (first < S) layout[first] = kEmpty;
}

hipError_t launch_founders(uint32_t* trait, uint32_t* counter, uint32_t* surf, uint32_t A,
                           uint32_t SW, uint32_t* layout, uint32_t S, bool tags, uint32_t k0,
                           uint32_t k1, hipStream_t stream) {
    uint32_t blocks = (A + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    if (blocks == 0) blocks = 1;
    hipLaunchKernelGGL(founders_kernel, dim3(blocks), dim3(256), 0, stream, trait, counter, surf,
                       A, SW, layout, S, tags ? 1u : 0u, k0, k1);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Site schedule.  In a synchronous run every parent of generation T carries
// counter T, so the surface site is the same for the whole population and
// is computed once per generation (Results, Surface Algorithm Benchmark:
// synchronous simulations can cache placements for a whole
// subpopulation).  The sites of a launch batch's ingests come from the
// rule's constant-time tables, one thread per ingest, and the first
// wavefront writes the run's layout after them (lane = site), for the
// run-bound queries and the read calls.
__device__ __forceinline__ void run_sites(const RuleTable* rules, uint32_t kind, uint32_t S,
                                          uint32_t* sites, uint32_t* layout, uint32_t tau0,
                                          uint32_t count, uint32_t k) {
    if (k < count) sites[k] = scheme_site(rules, kind, S, tau0 + k);
    if (k < S) layout[k] = scheme_item_at(rules, kind, S, (uint64_t)tau0 + count, k);
}

__global__ __launch_bounds__(256) void run_sites_kernel(const RuleTable* __restrict__ rules,
                                                       uint32_t kind, uint32_t S,
                                                       uint32_t* __restrict__ sites,
                                                       uint32_t* __restrict__ layout,
                                                       uint32_t tau0, uint32_t count) {
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    run_sites(rules, kind, S, sites, layout, tau0, count, k);
}

hipError_t launch_run_sites(const RuleTable* rules, uint32_t kind, uint32_t S, uint32_t* sites,
                            uint32_t* layout, uint32_t tau0, uint32_t count,
                            hipStream_t stream) {
    if (S > 64) return hipErrorInvalidValue;
    const uint32_t blocks = count > 256 ? (count + 255) / 256 : 1u;
    hipLaunchKernelGGL(run_sites_kernel, dim3(blocks), dim3(256), 0, stream, rules, kind, S,
                       sites, layout, tau0, count);
    return hipGetLastError();
}

// Sites of ingests tau0 .. tau0 + count - 1 into an asynchronous run's
// ring, one thread per ingest, from the rule's constant-time tables.
__global__ __launch_bounds__(256) void fill_site_ring_kernel(const RuleTable* __restrict__ rules,
                                                            uint32_t kind, uint32_t S,
                                                            uint32_t* __restrict__ ring,
                                                            uint32_t tau0, uint32_t count) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const uint32_t tau = tau0 + i;
    ring[tau & (kSiteRing - 1u)] = scheme_site(rules, kind, S, tau);
}

hipError_t launch_fill_site_ring(const RuleTable* rules, uint32_t kind, uint32_t S,
                                 uint32_t* ring, uint32_t tau0, uint32_t count,
                                 hipStream_t stream) {
    if (count == 0) return hipSuccess;
    if (count > kSiteRing) return hipErrorInvalidValue;
    hipLaunchKernelGGL(fill_site_ring_kernel, dim3((count + 255) / 256), dim3(256), 0, stream,
                       rules, kind, S, ring, tau0, count);
    return hipGetLastError();
}

// A run's layout set from the host through the kernel's arguments (so no
// host buffer has to outlive the call).
struct LayoutWords {
    uint32_t w[64];
};

__global__ __launch_bounds__(64) void set_layout_kernel(uint32_t* __restrict__ layout,
                                                        LayoutWords words, uint32_t S) {
    if (threadIdx.x < S) layout[threadIdx.x] = words.w[threadIdx.x];
}

hipError_t launch_set_layout(uint32_t* layout, const uint32_t* words, uint32_t S,
                             hipStream_t stream) {
    if (S > 64) return hipErrorInvalidValue;
    LayoutWords lw{};
    for (uint32_t k = 0; k < S; ++k) lw.w[k] = words[k];
    hipLaunchKernelGGL(set_layout_kernel, dim3(1), dim3(64), 0, stream, layout, lw, S);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// One generation, (P_g, O_g) -> (P_{g+1}, O_{g+1}) (Methods, Asynchronous
// Island-model Genetic Algorithm).
//
// One workgroup per tile of whole islands; the tile's population is staged
// in LDS as structure-of-arrays planes.
//  1. Each thread issues one 16-byte (APT = 4) non-temporal load per plane
//     for its APT consecutive agents: traits and surface words, counters
//     only for asynchronous ticks (in a synchronous run every counter is the
//     generation number).  In the same round thread t issues the loads of
//     island t's four neighbour outbox entries (direction word and record
//     together), the island pass draws the immigration and emigration
//     Philox blocks, and, while the loads are in flight, each thread draws
//     the Philox blocks of its births.
//  2. Records go to LDS; after a barrier, the thread of each island copies
//     the neighbours' emigrants addressed to it over the drawn slots,
//     north, south, west, east (a later one wins).
//  3. After a second barrier each thread gives birth to its APT agents: a
//     tournament of two over the island's LDS traits, the parent record
//     copied from LDS, trait mutation, counter + 1 and the differentia bit
//     written at this generation's site.  After the loop the thread holding
//     the island's emigrant posts its copy to the outbox for g + 1.
//     Children leave with one 16-byte store per plane (the counter plane
//     only for asynchronous ticks).
// Immigration slots: bits 6d .. 6d+5 = slot for direction d.  Emigration
// word: bits 0..7 = slot, 8..10 = direction (4: none, an idle island).
// Plan word (asynchronous ticks): bit 31 = the island is active.
template <int APT>
struct Lanes {
    uint32_t v[APT];
};

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

// Population planes stream through once per generation: global accesses
// carry the non-temporal hint.  LDS accesses are APT-word aligned.
template <int APT>
__device__ __forceinline__ Lanes<APT> load_lanes(const uint32_t* __restrict__ src) {
    Lanes<APT> r;
    if constexpr (APT == 4) {
        const u32x4 x = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(src));
        r.v[0] = x.x; r.v[1] = x.y; r.v[2] = x.z; r.v[3] = x.w;
    } else if constexpr (APT == 2) {
        const u32x2 x = __builtin_nontemporal_load(reinterpret_cast<const u32x2*>(src));
        r.v[0] = x.x; r.v[1] = x.y;
    } else {
        r.v[0] = __builtin_nontemporal_load(src);
    }
    return r;
}

template <int APT>
__device__ __forceinline__ void store_lanes(uint32_t* __restrict__ dst, const Lanes<APT>& r) {
    if constexpr (APT == 4) {
        u32x4 x = {r.v[0], r.v[1], r.v[2], r.v[3]};
        __builtin_nontemporal_store(x, reinterpret_cast<u32x4*>(dst));
    } else if constexpr (APT == 2) {
        u32x2 x = {r.v[0], r.v[1]};
        __builtin_nontemporal_store(x, reinterpret_cast<u32x2*>(dst));
    } else {
        __builtin_nontemporal_store(r.v[0], dst);
    }
}

template <int APT>
__device__ __forceinline__ void lds_store_lanes(uint32_t* dst, const Lanes<APT>& r) {
    if constexpr (APT == 4) {
        *reinterpret_cast<u32x4*>(__builtin_assume_aligned(dst, 16)) =
            u32x4{r.v[0], r.v[1], r.v[2], r.v[3]};
    } else if constexpr (APT == 2) {
        *reinterpret_cast<u32x2*>(__builtin_assume_aligned(dst, 8)) = u32x2{r.v[0], r.v[1]};
    } else {
        *dst = r.v[0];
    }
}

// Column of island isl on a torus W wide: isl mod W, the quotient by the
// run's multiplier (column_magic).
__device__ __forceinline__ uint32_t column_of(uint32_t isl, uint32_t W, uint32_t magic,
                                              uint32_t shift) {
    const uint32_t t = __umulhi(isl, magic);
    const uint32_t q = (t + ((isl - t) >> (shift & 0xffu))) >> (shift >> 8);
    return isl - q * W;
}

// Island index of a neighbour: 0 north, 1 south, 2 west, 3 east (torus).
__device__ __forceinline__ uint32_t neighbour_of(uint32_t isl, uint32_t x, uint32_t d, uint32_t W,
                                                 uint32_t I) {
    if (d == 0) return isl >= W ? isl - W : isl + I - W;
    if (d == 1) return isl + W < I ? isl + W : isl + W - I;
    if (d == 2) return x > 0 ? isl - 1 : isl + W - 1;
    return x + 1 < W ? isl + 1 : isl + 1 - W;
}

// Set bits of a wave mask on lanes below this one.
__device__ __forceinline__ uint32_t lanes_below(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

extern __shared__ __attribute__((aligned(16))) uint32_t g_step_lds[];

// The Philox blocks of a thread's APT births (and the second blocks of
// float births), computed as interleaved chains.  Their counter words
// (slot, island, generation, purpose) need no population data, so the tile
// computes them while its loads are in flight.
template <uint32_t BM, int APT>
struct BirthDraws {
    static constexpr int NB = BM == kBirthFloat ? 2 * APT : APT;
    uint4 blk[NB];
    __device__ __forceinline__ void compute(const StepParams& p, uint32_t j0, uint32_t isl) {
#pragma unroll
        for (int q = 0; q < APT; ++q) {
            blk[q] = make_uint4(j0 + q, isl, p.g, kBirth);
            if constexpr (BM == kBirthFloat) blk[APT + q] = make_uint4(j0 + q, isl, p.g, kBirthB);
        }
        philox4x32_10_multi<NB>(blk, p.k0, p.k1);
    }
};

// Births of this thread's APT agents.  APT divides N, so they share one
// island (il of the tile, slots j0 .. j0+APT-1).
template <int SW, uint32_t BM, bool MIGR, int APT, bool ASYNC, bool POW2>
__device__ __forceinline__ void step_births(const StepParams& p, uint32_t first_isl,
                                            uint32_t la0, uint32_t il, uint32_t j0,
                                            const BirthDraws<BM, APT>& draws,
                                            uint32_t site_word, uint32_t site_shift,
                                            uint32_t diff_mask, uint32_t n_shift) {
    uint32_t* lds = g_step_lds;
    const uint32_t N = p.N;
    const uint32_t TA = (p.tile_isl * N + 3u) & ~3u;
    const uint32_t* l_trait = lds;
    const uint32_t* l_count = lds + TA;
    const uint32_t* l_surf = lds + 2 * TA;
    const uint32_t* l_plan = lds + (2 + SW) * TA;
    const uint32_t* l_emig = l_plan + p.tile_isl;
    const size_t a0 = (size_t)first_isl * N;
    const size_t A = p.A;
    auto pick = [&](uint32_t w) -> uint32_t {
        if constexpr (POW2) return w >> n_shift;   // = mulhi(w, N) for N = 2^(32 - n_shift)
        else return word_below(w, N);
    };
    const uint32_t isl = first_isl + il;
    const uint32_t base = il * N;
    const uint4* blk = draws.blk;
    Lanes<APT> ctr, ccn, csf[SW];
    // Float births: the half-normal draws of the mutating births are queued
    // in the wave's LDS area (cosine cases from the front, sine cases from
    // the back) and evaluated after the loop in rounds of the wave's lanes,
    // so the draw runs once per mutating birth rather than once per birth
    // for the whole wave, and no round mixes the two series.
    // The loop itself has only wave-uniform branches; the mutation class of
    // each birth is read again from its draw words after the loop, where the
    // queue is filled.
    constexpr uint32_t QC = 64u * APT;                  // queue capacity of a wave
    uint2* wq = nullptr;
    uint32_t fslot = 0, ncos = 0, nsin = 0;
    if constexpr (BM == kBirthFloat)
        wq = reinterpret_cast<uint2*>(lds + ((((2 + SW) * TA + 2 * p.tile_isl) + 3u) & ~3u)) +
             (threadIdx.x >> 6) * QC;
#pragma unroll
    for (int q = 0; q < APT; ++q) {
        const uint32_t la = la0 + q;
        bool act = true;
        if constexpr (ASYNC) act = (l_plan[il] >> 31) != 0u;
        if (!act) {
            // idle island: the same individual on the next tick
            ctr.v[q] = l_trait[la];
            ccn.v[q] = l_count[la];
#pragma unroll
            for (int w = 0; w < SW; ++w) csf[w].v[q] = l_surf[w * TA + la];
        } else {
            const uint4 r = blk[q];
            uint32_t par = base + pick(r.x);
            uint32_t bit;
            if constexpr (BM == kBirthFloat) {
                // tournament of p.tour draws (words r.x, r.y, r.z, r.w, v.x),
                // the first of maximal fitness winning; mutation class from
                // v.y, |Z| from v.z and v.w, differentia the low bits of v.w
                const uint4 v = blk[APT + q];
                float best = __uint_as_float(l_trait[par]);
                const uint32_t words[4] = {r.y, r.z, r.w, v.x};
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    if ((uint32_t)c + 1u < p.tour) {
                        const uint32_t cb = base + pick(words[c]);
                        const float fc = __uint_as_float(l_trait[cb]);
                        if (fc > best) {
                            best = fc;
                            par = cb;
                        }
                    }
                }
                ctr.v[q] = __float_as_uint(best);        // the draw is applied after the loop
                bit = v.w & diff_mask;
            } else {
                uint32_t ptrait = l_trait[par];
                if constexpr (BM == kBirthIntTournament) {
                    const uint32_t pb = base + pick(r.y);
                    const uint32_t tb = l_trait[pb];
                    if ((int32_t)tb > (int32_t)ptrait) {
                        par = pb;
                        ptrait = tb;
                    }
                }
                const uint32_t delta =
                    r.z < p.mut_thr ? (uint32_t)((int32_t)word_below(r.w, p.mut_span) + p.mut_lo)
                                    : 0u;
                ctr.v[q] = ptrait + delta;
                bit = r.w & diff_mask;
            }
            // synchronous generations: every member's counter is g
            const uint32_t T = ASYNC ? l_count[par] : p.g;
            ccn.v[q] = T + 1u;
            uint32_t dep_word = site_word, dep_shift = site_shift;
            if constexpr (ASYNC) {
                // the parent's own counter picks the item and, in constant
                // time through the rule's tables, its site
                const uint32_t tau = p.interval == 1u ? T : T / p.interval;
                dep_word = 0xffu;
                if (tau * p.interval == T) {
                    const uint32_t site = tau >= p.ring_lo
                                              ? p.ring[tau & (kSiteRing - 1u)]
                                              : scheme_site(p.rules, p.kind, p.S, tau);
                    dep_word = site >> (5u - p.diff_log2);
                    dep_shift = (site << p.diff_log2) & 31u;
                }
            }
#pragma unroll
            for (int w = 0; w < SW; ++w) {
                const uint32_t word = l_surf[w * TA + par];
                csf[w].v[q] = (uint32_t)w == dep_word
                                  ? (word & ~(diff_mask << dep_shift)) | (bit << dep_shift)
                                  : word;
            }
        }
    }
    if constexpr (BM == kBirthFloat) {
        // mutating births: deleterious below del_thr, beneficial in the top
        // ben_thr words (idle islands of a tick draw nothing)
        bool act = true;
        if constexpr (ASYNC) act = (l_plan[il] >> 31) != 0u;
        const bool ben_on = p.ben_thr != 0u;
        const uint32_t ben_lo = 0u - p.ben_thr;
        auto needs = [&](const uint4& v) {
            return act && (v.y < p.del_thr || (ben_on && v.y >= ben_lo));
        };
#pragma unroll
        for (int q = 0; q < APT; ++q) {
            const uint4 vq = blk[APT + q];
            const bool nd = needs(vq);
            const bool sn = vq.w >= 0x80000000u;          // the draw's sine case
            const uint64_t mc = __ballot(nd && !sn);
            const uint64_t ms = __ballot(nd && sn);
            if (nd) {
                const uint32_t slot = sn ? QC - 1u - (nsin + lanes_below(ms))
                                         : ncos + lanes_below(mc);
                wq[slot] = make_uint2(vq.z, vq.w);
                fslot |= slot << (8 * q);
            }
            ncos += (uint32_t)__popcll(mc);
            nsin += (uint32_t)__popcll(ms);
        }
        // the queued draws in rounds of the active lanes (one wavefront: its
        // LDS writes land before its later reads), then each birth's fitness
        const uint64_t ex = __ballot(true);
        const uint32_t me = lanes_below(ex), na = (uint32_t)__popcll(ex);
        for (uint32_t b0 = 0; b0 < ncos; b0 += na) {
            if (b0 + me < ncos) {
                const uint2 e = wq[b0 + me];
                const double z = half_normal_case<false>(e.x, e.y);
                const uint64_t zb = (uint64_t)__double_as_longlong(z);
                wq[b0 + me] = make_uint2((uint32_t)zb, (uint32_t)(zb >> 32));
            }
        }
        for (uint32_t b0 = 0; b0 < nsin; b0 += na) {
            if (b0 + me < nsin) {
                const uint32_t i = QC - 1u - (b0 + me);
                const uint2 e = wq[i];
                const double z = half_normal_case<true>(e.x, e.y);
                const uint64_t zb = (uint64_t)__double_as_longlong(z);
                wq[i] = make_uint2((uint32_t)zb, (uint32_t)(zb >> 32));
            }
        }
#pragma unroll
        for (int q = 0; q < APT; ++q) {
            const uint4 vq = blk[APT + q];
            if (needs(vq)) {
                const uint2 e = wq[(fslot >> (8 * q)) & 0xffu];
                const double z =
                    __longlong_as_double((long long)(((uint64_t)e.y << 32) | e.x));
                ctr.v[q] = __float_as_uint(apply_half_normal(__uint_as_float(ctr.v[q]),
                                                             vq.y < p.del_thr, p.del_sigma,
                                                             p.ben_sigma, z));
            }
        }
    }
    if (MIGR) {
        // the island's emigrant, if it is one of this thread's agents (after
        // the loop, so that the loop body has no branch and the agents' LDS
        // reads overlap)
        const uint32_t em = l_emig[il];
        const uint32_t qe = (em & 0xffu) - j0;          // >= APT: another thread's
        constexpr uint32_t OBW = ASYNC ? kOutboxWords : kSyncOutboxWords;
        if (qe < (uint32_t)APT) {
            uint32_t e_tr = ctr.v[0], e_cn = ccn.v[0], e_s0 = csf[0].v[0],
                     e_s1 = csf[SW - 1].v[0];
#pragma unroll
            for (int q = 1; q < APT; ++q) {
                if (qe == (uint32_t)q) {
                    e_tr = ctr.v[q];
                    e_cn = ccn.v[q];
                    e_s0 = csf[0].v[q];
                    e_s1 = csf[SW - 1].v[q];
                }
            }
            uint32_t* o = p.ob_out + (size_t)isl * OBW;
            const uint32_t dir = (em >> 8) & 7u;
            if constexpr (!ASYNC) {
                // synchronous: always a direction below 4, counter implied
                *reinterpret_cast<uint4*>(o) = make_uint4(dir, e_tr, e_s0, SW > 1 ? e_s1 : 0u);
            } else if (dir < 4u) {
                *reinterpret_cast<uint4*>(o) = make_uint4(dir, e_tr, e_cn, e_s0);
                *reinterpret_cast<uint4*>(o + 4) = make_uint4(SW > 1 ? e_s1 : 0u, 0u, 0u, 0u);
            } else {
                *reinterpret_cast<uint4*>(o) = make_uint4(dir, 0u, 0u, 0u);
                *reinterpret_cast<uint4*>(o + 4) = make_uint4(0u, 0u, 0u, 0u);
            }
        }
    }
    store_lanes<APT>(p.out_trait + a0 + la0, ctr);
    // a synchronous run keeps no counter plane: every counter is g + 1
    if constexpr (ASYNC) store_lanes<APT>(p.out_counter + a0 + la0, ccn);
#pragma unroll
    for (int w = 0; w < SW; ++w) store_lanes<APT>(p.out_surf + w * A + a0 + la0, csf[w]);
}


// One tile of one run.  Shared by the plain kernel (one run per launch) and
// the batched kernel (many runs per launch).
template <int SW, uint32_t BM, bool MIGR, int APT, bool ASYNC = false>
__device__ __forceinline__ void step_tile(const StepParams& p, uint32_t tile) {
    uint32_t* lds = g_step_lds;
    const uint32_t N = p.N, W = p.W;
    const uint32_t TA = (p.tile_isl * N + 3u) & ~3u;   // plane stride (16-byte multiple)
    uint32_t* l_trait = lds;
    uint32_t* l_count = lds + TA;
    uint32_t* l_surf = lds + 2 * TA;                   // SW planes of TA words
    uint32_t* l_plan = lds + (2 + SW) * TA;            // tile_isl words
    uint32_t* l_emig = l_plan + p.tile_isl;            // tile_isl words

    const uint32_t first_isl = tile * p.tile_isl;
    const uint32_t nisl = min(p.tile_isl, p.I - first_isl);
    const uint32_t nag = nisl * N;
    const size_t a0 = (size_t)first_isl * N;
    const size_t A = p.A;
    const uint32_t t = threadIdx.x;
    const uint32_t la0 = t * APT;
    const bool mine = la0 < nag;

    // this generation's deposit: word and bit offset of the site, none
    // (no word matches) between ingests
    uint32_t site_word = 0xffu, site_shift = 0u;
    if (p.site) {
        const uint32_t site = *p.site;
        site_word = site >> (5u - p.diff_log2);
        site_shift = (site << p.diff_log2) & 31u;
    }
    // A wave issues its loads at the highest priority and then drops back:
    // when a fresh wave arrives, its loads go out ahead of the arithmetic of
    // waves already holding data, which keeps more bytes in flight.
    __builtin_amdgcn_s_setprio(3);
    // 1. this thread's agents, every plane
    Lanes<APT> tr, ct, sf[SW];
    if (mine) {
        tr = load_lanes<APT>(p.in_trait + a0 + la0);
        // only asynchronous runs keep a counter plane: in synchronous
        // generations every agent's counter is the generation number
        // (founders 0, each birth one above a parent of the same
        // generation)
        if (ASYNC) ct = load_lanes<APT>(p.in_counter + a0 + la0);
#pragma unroll
        for (int w = 0; w < SW; ++w) sf[w] = load_lanes<APT>(p.in_surf + w * A + a0 + la0);
    }
    // Island pass: thread t takes island t for immigration (and the activity
    // draw) and thread blockDim-1-t takes island t for emigration; the host
    // keeps tile_isl <= blockDim.  Each neighbour's whole outbox entry is
    // read together with the tile (the record shares the direction word's
    // cache line), so the immigrants need no second round trip; the loads
    // are issued outside any branch (lanes without an island read entry 0;
    // before the first generation the entries are read but not used) so
    // that nothing waits for them before the birth draws.  Only wavefronts
    // holding an island lane work out neighbour indices (a wave-uniform
    // test: most wavefronts of a large tile hold none); the loads stay after
    // the branch, since loads inside it would be waited for at its end.
    constexpr uint32_t OBW = ASYNC ? kOutboxWords : kSyncOutboxWords;
    uint4 in_lo[4], in_hi[4];
    uint32_t imm_slots = 0;        // the four directions' slots, 6 bits each
    bool imm_take = false;         // this lane's island takes immigrants
    if (MIGR) {
        size_t e[4] = {0, 0, 0, 0};
        if ((uint32_t)__builtin_amdgcn_readfirstlane((int)t) < nisl) {
            const bool lane_isl = t < nisl;
            const uint32_t isl = first_isl + (lane_isl ? t : 0u);
            const uint32_t x = column_of(isl, W, p.w_magic, p.w_shift);
#pragma unroll
            for (int d = 0; d < 4; ++d)
                e[d] = lane_isl ? (size_t)neighbour_of(isl, x, (uint32_t)d, W, p.I) * OBW : 0;
        }
#pragma unroll
        for (int d = 0; d < 4; ++d) {
            in_lo[d] = *reinterpret_cast<const uint4*>(p.ob_in + e[d]);
            if (ASYNC && SW > 1) in_hi[d] = *reinterpret_cast<const uint4*>(p.ob_in + e[d] + 4);
        }
    }
    __builtin_amdgcn_s_setprio(0);
    if (MIGR && !ASYNC && 2u * nisl <= blockDim.x) {
        // one Philox evaluation for both island draws: lanes t < nisl draw
        // island t's immigration block, lanes nisl .. 2 nisl - 1 the
        // emigration block of island t - nisl (the same blocks as two
        // separate passes, without a second divergent evaluation)
        const bool imm_lane = t < nisl;
        if (t < 2u * nisl) {
            const uint32_t il = imm_lane ? t : t - nisl;
            const uint32_t isl = first_isl + il;
            const uint4 w4 = philox4x32_10(
                make_uint4(0u, isl, p.g, imm_lane ? kImmigrate : kEmigrate), p.k0, p.k1);
            if (!imm_lane) {
                l_emig[il] = word_below(w4.x, N) | ((w4.y >> 30) << 8);
            } else if (p.has_inbox) {
                imm_slots = word_below(w4.x, N) | (word_below(w4.y, N) << 6) |
                            (word_below(w4.z, N) << 12) | (word_below(w4.w, N) << 18);
                imm_take = true;
            }
        }
    } else if (MIGR || ASYNC) {
        // asynchronous ticks: an island runs a generation iff its activity
        // draw is below the threshold (plan bit 31); an idle island takes no
        // immigrants and posts no emigrant (direction 4)
        if (t < nisl) {
            const uint32_t isl = first_isl + t;
            bool act = true;
            if constexpr (ASYNC)
                act = philox4x32_10(make_uint4(0u, isl, p.g, kActivity), p.k0, p.k1).x <
                      p.async_thr;
            if (MIGR && act && p.has_inbox) {
                const uint4 w4 = philox4x32_10(make_uint4(0u, isl, p.g, kImmigrate), p.k0, p.k1);
                imm_slots = word_below(w4.x, N) | (word_below(w4.y, N) << 6) |
                            (word_below(w4.z, N) << 12) | (word_below(w4.w, N) << 18);
                imm_take = true;
            }
            if constexpr (ASYNC) l_plan[t] = act ? 1u << 31 : 0u;
        }
        if (MIGR) {
            const uint32_t il = blockDim.x - 1u - t;
            if (il < nisl) {
                const uint32_t isl = first_isl + il;
                bool act = true;
                if constexpr (ASYNC)
                    act = philox4x32_10(make_uint4(0u, isl, p.g, kActivity), p.k0, p.k1).x <
                          p.async_thr;
                const uint4 w4 = philox4x32_10(make_uint4(0u, isl, p.g, kEmigrate), p.k0, p.k1);
                l_emig[il] = word_below(w4.x, N) | ((act ? (w4.y >> 30) : 4u) << 8);
            }
        }
    }

    // this thread's island and first slot (one division: la0 < 4096), and
    // its birth draws while the loads are in flight (integer births; the
    // float births' two blocks per agent would cost a wave per SIMD, so
    // they are drawn after the staging)
    const uint32_t il = (la0 * p.div_magic) >> 20;
    const uint32_t j0 = la0 - il * N;
    BirthDraws<BM, APT> draws;
    if constexpr (BM != kBirthFloat)
        if (mine) draws.compute(p, j0, first_isl + il);

    // 2. stage the tile in LDS, then overwrite immigrant slots (north,
    // south, west, east: a later direction overwrites an earlier one)
    if (mine) {
        lds_store_lanes<APT>(l_trait + la0, tr);
        if (ASYNC) lds_store_lanes<APT>(l_count + la0, ct);
#pragma unroll
        for (int w = 0; w < SW; ++w) lds_store_lanes<APT>(l_surf + w * TA + la0, sf[w]);
    }
    __syncthreads();
    if (MIGR) {
        if (imm_take) {
            // a neighbour delivers when its emigrant was sent our way
            const uint32_t arrivals = (in_lo[0].x == 1u ? 1u : 0u) | (in_lo[1].x == 0u ? 2u : 0u) |
                                      (in_lo[2].x == 3u ? 4u : 0u) | (in_lo[3].x == 2u ? 8u : 0u);
#pragma unroll
            for (int d = 0; d < 4; ++d) {
                if ((arrivals >> d) & 1u) {
                    const uint32_t la = t * N + ((imm_slots >> (6 * d)) & 63u);
                    l_trait[la] = in_lo[d].y;
                    if constexpr (ASYNC) {
                        l_count[la] = in_lo[d].z;
                        l_surf[la] = in_lo[d].w;
                        if (SW > 1) l_surf[TA + la] = in_hi[d].x;
                    } else {
                        l_surf[la] = in_lo[d].z;
                        if (SW > 1) l_surf[TA + la] = in_lo[d].w;
                    }
                }
            }
        }
        __syncthreads();
    }

    // 3. births (no barrier follows, so threads without agents may skip
    // them; the resident form's next generation waits for every thread)
    const uint32_t diff_mask = p.diff_log2 ? 0xffu : 1u;
    if (mine) {
        if constexpr (BM == kBirthFloat) draws.compute(p, j0, first_isl + il);
        // draws onto [0, N): a shift when N is a power of two above 1 (a
        // wave-uniform choice between two copies of the births)
        const uint32_t n_shift =
            (N > 1u && (N & (N - 1u)) == 0u) ? 32u - __builtin_ctz(N) : 0u;
        if (n_shift)
            step_births<SW, BM, MIGR, APT, ASYNC, true>(p, first_isl, la0, il, j0, draws,
                                                        site_word, site_shift, diff_mask, n_shift);
        else
            step_births<SW, BM, MIGR, APT, ASYNC, false>(p, first_isl, la0, il, j0, draws,
                                                         site_word, site_shift, diff_mask, n_shift);
    }
}

template <int SW, uint32_t BM, bool MIGR, int APT, bool ASYNC>
__global__ __launch_bounds__(1024) void step_kernel(const StepParams p) {
    step_tile<SW, BM, MIGR, APT, ASYNC>(p, xcd_local_block(blockIdx.x, gridDim.x));
}

// The resident form of a small synchronous run: its whole torus is one
// tile, and one workgroup takes it through all gens generations of a launch
// batch, with a workgroup barrier between generations where the plain form
// has a kernel boundary.  A generation then costs neither a launch nor the
// chip-wide cache write-back and invalidation between kernels, and its
// planes and outboxes stay in this CU's caches.  p is generation p.g's;
// sites holds the batch's schedule from ingest tau0.
template <int SW, uint32_t BM, bool MIGR, int APT>
__global__ __launch_bounds__(1024) void resident_step_kernel(StepParams p, const uint32_t gens,
                                                            const uint32_t* __restrict__ sites,
                                                            const uint32_t tau0) {
    for (uint32_t k = 0; k < gens; ++k) {
        if (k > 0) {
            // the previous generation's children and emigrants are this
            // one's parents and immigrants: every thread's stores and LDS
            // reads are done before any thread loads or stages again
            __syncthreads();
            // the ping-pong buffers swap roles (the read side is typed const)
            uint32_t* t = const_cast<uint32_t*>(p.in_trait);
            p.in_trait = p.out_trait;
            p.out_trait = t;
            t = const_cast<uint32_t*>(p.in_surf);
            p.in_surf = p.out_surf;
            p.out_surf = t;
            t = const_cast<uint32_t*>(p.ob_in);
            p.ob_in = p.ob_out;
            p.ob_out = t;
            ++p.g;
            p.has_inbox = MIGR ? 1u : 0u;
            p.site = p.g % p.interval == 0u ? sites + (p.g / p.interval - tau0) : nullptr;
        }
        step_tile<SW, BM, MIGR, APT, false>(p, 0u);
    }
}

size_t step_lds_bytes(uint32_t tile_isl, uint32_t N, uint32_t SW) {
    const size_t TA = ((size_t)tile_isl * N + 3) & ~(size_t)3;
    return ((2 + SW) * TA + 2 * (size_t)tile_isl) * 4;
}

size_t step_lds_bytes(uint32_t tile_isl, uint32_t N, uint32_t SW, bool float_births,
                      uint32_t block_threads, uint32_t apt) {
    const size_t b = step_lds_bytes(tile_isl, N, SW);
    if (!float_births) return b;
    return ((b + 15) & ~(size_t)15) + (size_t)block_threads * apt * 8;   // the draw queues
}

// rs.gens == 0: one generation over the run's tiles; otherwise the resident
// form (rs.gens generations of a synchronous run that is one tile).
struct Resident {
    uint32_t gens;
    const uint32_t* sites;
    uint32_t tau0;
};

template <int SW, uint32_t BM, bool MIGR, int APT, bool ASYNC>
static hipError_t launch_step_t(const StepParams& p, uint32_t block_threads, const Resident& rs,
                                hipStream_t stream) {
    if (p.tile_isl == 0 || p.tile_isl > block_threads) return hipErrorInvalidValue;
    const uint32_t tiles = (p.I + p.tile_isl - 1) / p.tile_isl;
    const size_t lds =
        step_lds_bytes(p.tile_isl, p.N, SW, BM == kBirthFloat, block_threads, APT);
    if (rs.gens) {
        if constexpr (ASYNC) return hipErrorInvalidValue;
        if (tiles != 1 || !rs.sites) return hipErrorInvalidValue;
        hipLaunchKernelGGL((resident_step_kernel<SW, BM, MIGR, APT>), dim3(1),
                           dim3(block_threads), lds, stream, p, rs.gens, rs.sites, rs.tau0);
    } else {
        hipLaunchKernelGGL((step_kernel<SW, BM, MIGR, APT, ASYNC>), dim3(tiles),
                           dim3(block_threads), lds, stream, p);
    }
    return hipGetLastError();
}

template <int SW, uint32_t BM, bool MIGR, bool ASYNC>
static hipError_t launch_step_apt(const StepParams& p, uint32_t apt, uint32_t block_threads,
                                  const Resident& rs, hipStream_t stream) {
    if (apt == 4) return launch_step_t<SW, BM, MIGR, 4, ASYNC>(p, block_threads, rs, stream);
    if (apt == 2) return launch_step_t<SW, BM, MIGR, 2, ASYNC>(p, block_threads, rs, stream);
    return launch_step_t<SW, BM, MIGR, 1, ASYNC>(p, block_threads, rs, stream);
}

template <int SW, uint32_t BM, bool ASYNC>
static hipError_t launch_step_mig(const StepParams& p, bool migration, uint32_t apt,
                                  uint32_t block_threads, const Resident& rs,
                                  hipStream_t stream) {
    return migration ? launch_step_apt<SW, BM, true, ASYNC>(p, apt, block_threads, rs, stream)
                     : launch_step_apt<SW, BM, false, ASYNC>(p, apt, block_threads, rs, stream);
}

template <int SW, bool ASYNC>
static hipError_t launch_step_model(const StepParams& p, uint32_t birth_model, bool migration,
                                    uint32_t apt, uint32_t block_threads, const Resident& rs,
                                    hipStream_t stream) {
    if (birth_model == kBirthFloat)
        return launch_step_mig<SW, kBirthFloat, ASYNC>(p, migration, apt, block_threads, rs,
                                                       stream);
    if (birth_model == kBirthIntTournament)
        return launch_step_mig<SW, kBirthIntTournament, ASYNC>(p, migration, apt, block_threads,
                                                               rs, stream);
    return launch_step_mig<SW, kBirthIntNeutral, ASYNC>(p, migration, apt, block_threads, rs,
                                                        stream);
}

template <bool ASYNC>
static hipError_t launch_step_sw(const StepParams& p, uint32_t SW, uint32_t birth_model,
                                 bool migration, uint32_t apt, uint32_t block_threads,
                                 const Resident& rs, hipStream_t stream) {
    if (SW == 1)
        return launch_step_model<1, ASYNC>(p, birth_model, migration, apt, block_threads, rs,
                                           stream);
    return launch_step_model<2, ASYNC>(p, birth_model, migration, apt, block_threads, rs, stream);
}

hipError_t launch_step(const StepParams& p, uint32_t SW, uint32_t birth_model, bool migration,
                       uint32_t agents_per_thread, uint32_t block_threads, hipStream_t stream) {
    const Resident none{0u, nullptr, 0u};
    if (p.async_thr)
        return launch_step_sw<true>(p, SW, birth_model, migration, agents_per_thread,
                                    block_threads, none, stream);
    return launch_step_sw<false>(p, SW, birth_model, migration, agents_per_thread, block_threads,
                                 none, stream);
}

hipError_t launch_resident_step(const StepParams& p, uint32_t gens, const uint32_t* sites,
                                uint32_t tau0, uint32_t SW, uint32_t birth_model, bool migration,
                                uint32_t agents_per_thread, uint32_t block_threads,
                                hipStream_t stream) {
    if (gens == 0) return hipSuccess;
    if (p.async_thr) return hipErrorInvalidValue;
    return launch_step_sw<false>(p, SW, birth_model, migration, agents_per_thread, block_threads,
                                 Resident{gens, sites, tau0}, stream);
}

// ---------------------------------------------------------------------------
// Batched forms: many runs of different sizes, surfaces, treatments and
// agents per thread in one launch per generation, sharing step_tile and
// run_sites with the plain forms.
__global__ __launch_bounds__(256) void batch_sites_kernel(const BatchRun* __restrict__ runs) {
    const BatchRun& R = runs[blockIdx.y];
    const uint32_t tau0 = ingests_of(R.T0, R.interval);
    const uint32_t count = ingests_of(R.T0 + R.gens, R.interval) - tau0;
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    run_sites(R.rules, R.kind, R.S, R.sites, R.layout, tau0, count, k);
}

hipError_t launch_batch_sites(const BatchRun* runs, uint32_t nruns, uint32_t max_gens,
                              hipStream_t stream) {
    if (nruns == 0) return hipSuccess;
    const uint32_t blocks = max_gens > 256 ? (max_gens + 255) / 256 : 1u;
    hipLaunchKernelGGL(batch_sites_kernel, dim3(blocks, nruns), dim3(256), 0, stream, runs);
    return hipGetLastError();
}

template <int SW, uint32_t BM, bool MIGR>
__device__ __forceinline__ void step_tile_apt(const StepParams& p, uint32_t tile, uint32_t apt_log2) {
    if (apt_log2 == 2) step_tile<SW, BM, MIGR, 4>(p, tile);
    else if (apt_log2 == 1) step_tile<SW, BM, MIGR, 2>(p, tile);
    else step_tile<SW, BM, MIGR, 1>(p, tile);
}

template <uint32_t BM>
__device__ __forceinline__ void step_tile_variant(const StepParams& p, uint32_t tile,
                                                  uint32_t variant) {
    const uint32_t apt_log2 = (variant >> 4) & 3u;
    const bool mig = (variant >> 3) & 1u;
    if (variant & 1u) {
        if (mig) step_tile_apt<2, BM, true>(p, tile, apt_log2);
        else step_tile_apt<2, BM, false>(p, tile, apt_log2);
    } else {
        if (mig) step_tile_apt<1, BM, true>(p, tile, apt_log2);
        else step_tile_apt<1, BM, false>(p, tile, apt_log2);
    }
}

// WITH_FLOAT: the batch may hold float-treatment runs.  Integer-only
// batches use the instantiation without them, which needs fewer registers.
template <bool WITH_FLOAT>
__global__ __launch_bounds__(1024) void batch_step_kernel(const BatchRun* __restrict__ runs,
                                                         const uint32_t* __restrict__ xcd_tab,
                                                         uint32_t nruns, uint32_t k) {
    // Workgroup b runs on XCD x = b mod 8 as the XCD's j-th workgroup, j =
    // b / 8 (the dispatcher deals workgroups to the XCDs in turn).  Every
    // run's tiles are cut into 8 contiguous chunks, one per XCD, so
    // each XCD gets an equal share of every run: a launch of runs of
    // unequal cost per tile then finishes on all XCDs together, while torus
    // neighbours within a chunk still share an L2.  xcd_tab holds, per
    // XCD, the ascending offsets of the runs' chunks among its workgroups
    // (nruns words), then per XCD the first tile of each run's chunk.
    const uint32_t x = blockIdx.x % kXcds, j = blockIdx.x / kXcds;
    const uint32_t* __restrict__ pre = xcd_tab + x * nruns;
    // the run owning this workgroup: the number of runs whose chunk starts
    // at or before j, less one (a run with an empty chunk shares its
    // offset with the next and is passed over) -- one load per lane and a
    // ballot per 64 runs in every wavefront, with no LDS round trip or
    // barrier before the run's parameters can be fetched
    const uint32_t lane = threadIdx.x & 63u;
    uint32_t before = 0;
    for (uint32_t b0 = 0; b0 < nruns; b0 += 64) {
        const uint32_t i = b0 + lane;
        const bool le = i < nruns && pre[i] <= j;
        before += (uint32_t)__popcll(__ballot(le));
    }
    const uint32_t lo = before - 1u;       // pre[0] = 0: at least one run
    const BatchRun& R = runs[lo];
    const uint32_t t = xcd_tab[(kXcds + x) * nruns + lo] + (j - pre[lo]);
    if (k >= R.gens) return;
    const uint32_t g = R.T0 + k;
    const uint32_t src = g & 1u, dst = (g + 1u) & 1u;
    StepParams p;
    p.in_trait = R.trait[src];
    p.in_counter = R.counter[src];
    p.in_surf = R.surf[src];
    p.out_trait = R.trait[dst];
    p.out_counter = R.counter[dst];
    p.out_surf = R.surf[dst];
    p.ob_in = R.outbox[src];
    p.ob_out = R.outbox[dst];
    // deposit iff g is a multiple of the interval; its site is entry
    // g / interval - tau0 of this batch's schedule
    p.site = g % R.interval == 0 ? R.sites + (g / R.interval - ingests_of(R.T0, R.interval))
                                 : nullptr;
    p.diff_log2 = R.diff_log2;
    p.W = R.W; p.H = R.H; p.N = R.N; p.I = R.I; p.A = R.A;
    p.g = g;
    p.k0 = R.k0; p.k1 = R.k1;
    p.mut_thr = R.mut_thr; p.mut_lo = R.mut_lo; p.mut_span = R.mut_span;
    const bool mig = (R.variant >> 3) & 1u;
    p.has_inbox = (mig && g > 0) ? 1u : 0u;
    p.tile_isl = R.tile_isl;
    p.div_magic = R.div_magic;
    p.w_magic = R.w_magic;
    p.w_shift = R.w_shift;
    p.async_thr = 0u;          // batched runs are synchronous
    p.rules = nullptr;
    p.ring = nullptr;
    p.ring_lo = 0u;
    p.kind = R.kind;
    p.S = R.S;
    p.interval = R.interval;
    p.tour = R.tour;
    p.del_thr = R.del_thr; p.ben_thr = R.ben_thr;
    p.del_sigma = R.del_sigma; p.ben_sigma = R.ben_sigma;
    const uint32_t model = (R.variant >> 1) & 3u;
    if (model == kBirthIntTournament) step_tile_variant<kBirthIntTournament>(p, t, R.variant);
    else if (WITH_FLOAT && model == kBirthFloat) step_tile_variant<kBirthFloat>(p, t, R.variant);
    else step_tile_variant<kBirthIntNeutral>(p, t, R.variant);
}

hipError_t launch_batch_step(const BatchRun* runs, const uint32_t* xcd_tab, uint32_t nruns,
                             uint32_t total_tiles, uint32_t k, uint32_t block_threads,
                             size_t lds_bytes, bool with_float, hipStream_t stream) {
    if (nruns == 0 || total_tiles == 0) return hipSuccess;
    if (with_float)
        hipLaunchKernelGGL(batch_step_kernel<true>, dim3(total_tiles), dim3(block_threads),
                           lds_bytes, stream, runs, xcd_tab, nruns, k);
    else
        hipLaunchKernelGGL(batch_step_kernel<false>, dim3(total_tiles), dim3(block_threads),
                           lds_bytes, stream, runs, xcd_tab, nruns, k);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Plain streaming copy (instrumentation): one 16-byte non-temporal load
// and store per thread over a grid that covers the buffer (the fastest of
// the simple copy forms on this chip, so the attainable-bandwidth figure
// is not understated).
__global__ __launch_bounds__(256) void probe_copy_kernel(const u32x4* __restrict__ src,
                                                        u32x4* __restrict__ dst, size_t n16) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n16) __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

hipError_t launch_probe_copy(const void* src, void* dst, size_t bytes, hipStream_t stream) {
    const size_t n16 = bytes / 16;
    const size_t blocks = (n16 + 255) / 256;
    if (blocks == 0) return hipSuccess;
    if (blocks > 0xffffffffull) return hipErrorInvalidValue;
    hipLaunchKernelGGL(probe_copy_kernel, dim3((uint32_t)blocks), dim3(256), 0, stream,
                       static_cast<const u32x4*>(src), static_cast<u32x4*>(dst), n16);
    return hipGetLastError();
}

}  // namespace hsga
