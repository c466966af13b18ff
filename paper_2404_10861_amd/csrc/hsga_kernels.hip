// hsga_kernels.hip -- gfx950 kernels of the island-model GA with
// hereditary-stratigraphy surface annotations, and their launchers.
//
// Device state is structure-of-arrays: trait[A], counter[A] and the S/32
// surface word planes [S/32][A], agent a = island * N + slot.  Consecutive
// lanes own consecutive agents, so every population read and write is a
// contiguous 256-byte wavefront access per plane.
#include "hsga_device.hpp"
#include "hsga_internal.hpp"

namespace hsga {

// ---------------------------------------------------------------------------
// Founders (Genome Model; Distributed Phylogenetic Tracking): trait 0,
// counter 0, every site 0, and an empty layout.  Founders carry no
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
        counter[a] = 0u;
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
// subpopulation).  One wavefront, lane k = site k: for ingests
// tau = tau0 .. tau0+count-1 (ingest units; every generation when the
// interval is 1) the placement is a ballot over the lanes whose item left
// the target, then a bit scan; the run's layout is carried in registers and
// written back at the end.
__device__ __forceinline__ void schedule_sites(uint32_t kind, uint32_t S, uint32_t* layout,
                                               uint32_t* sites, uint32_t tau0, uint32_t count) {
    const uint32_t lane = threadIdx.x;
    uint32_t held = lane < S ? layout[lane] : kEmpty;
    uint32_t leave = lane_leave_time(kind, S, lane, held);
    place_items(kind, S, tau0, count, held, leave, lane,
                [&](uint32_t k, int site) { sites[k] = (uint32_t)site; });
    if (lane < S) layout[lane] = held;
}

__global__ __launch_bounds__(64) void site_schedule_kernel(uint32_t kind, uint32_t S,
                                                           uint32_t* __restrict__ layout,
                                                           uint32_t* __restrict__ sites,
                                                           uint32_t tau0, uint32_t count) {
    schedule_sites(kind, S, layout, sites, tau0, count);
}

hipError_t launch_site_schedule(uint32_t kind, uint32_t S, uint32_t* layout, uint32_t* sites,
                                uint32_t tau0, uint32_t count, hipStream_t stream) {
    if (count == 0) return hipSuccess;
    hipLaunchKernelGGL(site_schedule_kernel, dim3(1), dim3(64), 0, stream, kind, S, layout,
                       sites, tau0, count);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// One generation, (P_g, O_g) -> (P_{g+1}, O_{g+1}) (Methods, Asynchronous
// Island-model Genetic Algorithm).
//
// One workgroup per tile of whole islands; the tile's population is staged
// in LDS as structure-of-arrays planes.
//  1. Each thread loads APT consecutive agents of every plane with one
//     16-byte (APT = 4) load per plane; meanwhile the island pass draws one
//     immigration and one emigration Philox block per island and reads the
//     four neighbours' outbox directions.
//  2. Records go to LDS; after a barrier, one thread per island copies the
//     neighbours' emigrants that were addressed to it over the chosen slots,
//     north, south, west, east (a later one wins).
//  3. After a second barrier each thread gives birth to its APT agents: one
//     Philox block each, a tournament of two read from the island's LDS
//     traits, the parent record copied from LDS, trait mutation, counter
//     increment and the differentia bit written at this generation's site.
//     The thread holding the chosen emigrant posts its copy to the outbox
//     for g + 1.  Children leave with one 16-byte store per plane.
// Immigration plan word: bits 0..3 = direction d delivers, bits 4+6d ..
// 9+6d = slot for direction d.  Emigration word: bits 0..7 = slot, 8..9 =
// direction.
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

// Island index of a neighbour: 0 north, 1 south, 2 west, 3 east (torus).
__device__ __forceinline__ uint32_t neighbour_of(uint32_t isl, uint32_t x, uint32_t d, uint32_t W,
                                                 uint32_t I) {
    if (d == 0) return isl >= W ? isl - W : isl + I - W;
    if (d == 1) return isl + W < I ? isl + W : isl + W - I;
    if (d == 2) return x > 0 ? isl - 1 : isl + W - 1;
    return x + 1 < W ? isl + 1 : isl + 1 - W;
}

extern __shared__ __attribute__((aligned(16))) uint32_t g_step_lds[];

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

    // 1. this thread's agents, every plane
    Lanes<APT> tr, ct, sf[SW];
    if (mine) {
        tr = load_lanes<APT>(p.in_trait + a0 + la0);
        ct = load_lanes<APT>(p.in_counter + a0 + la0);
#pragma unroll
        for (int w = 0; w < SW; ++w) sf[w] = load_lanes<APT>(p.in_surf + w * A + a0 + la0);
    }
    if (MIGR || ASYNC) {
        // asynchronous ticks: an island runs a generation iff its activity
        // draw is below the threshold (plan bit 31); an idle island takes no
        // immigrants and posts no emigrant (direction 4)
        const uint32_t passes = MIGR ? 2 * nisl : nisl;
        for (uint32_t b = t; b < passes; b += blockDim.x) {
            const bool imm = b < nisl;
            const uint32_t il = imm ? b : b - nisl;
            const uint32_t isl = first_isl + il;
            bool act = true;
            if constexpr (ASYNC)
                act = philox4x32_10(make_uint4(0u, isl, p.g, kActivity), p.k0, p.k1).x <
                      p.async_thr;
            if (imm) {
                uint32_t plan = 0;
                if (MIGR && act && p.has_inbox) {
                    const uint4 w4 =
                        philox4x32_10(make_uint4(0u, isl, p.g, kImmigrate), p.k0, p.k1);
                    const uint32_t x = isl % W;
                    // a neighbour delivers when its emigrant was sent our way
                    const uint32_t dn = p.ob_in[(size_t)neighbour_of(isl, x, 0, W, p.I) * kOutboxWords];
                    const uint32_t ds = p.ob_in[(size_t)neighbour_of(isl, x, 1, W, p.I) * kOutboxWords];
                    const uint32_t dw = p.ob_in[(size_t)neighbour_of(isl, x, 2, W, p.I) * kOutboxWords];
                    const uint32_t de = p.ob_in[(size_t)neighbour_of(isl, x, 3, W, p.I) * kOutboxWords];
                    plan = (dn == 1u ? 1u : 0u) | (ds == 0u ? 2u : 0u) | (dw == 3u ? 4u : 0u) |
                           (de == 2u ? 8u : 0u);
                    plan |= word_below(w4.x, N) << 4;
                    plan |= word_below(w4.y, N) << 10;
                    plan |= word_below(w4.z, N) << 16;
                    plan |= word_below(w4.w, N) << 22;
                }
                if (ASYNC && act) plan |= 1u << 31;
                l_plan[il] = plan;
            } else {
                const uint4 w4 = philox4x32_10(make_uint4(0u, isl, p.g, kEmigrate), p.k0, p.k1);
                l_emig[il] = word_below(w4.x, N) | ((act ? (w4.y >> 30) : 4u) << 8);
            }
        }
    }

    // 2. stage the tile in LDS, then overwrite immigrant slots
    if (mine) {
        lds_store_lanes<APT>(l_trait + la0, tr);
        lds_store_lanes<APT>(l_count + la0, ct);
#pragma unroll
        for (int w = 0; w < SW; ++w) lds_store_lanes<APT>(l_surf + w * TA + la0, sf[w]);
    }
    __syncthreads();
    if (MIGR) {
        if (p.has_inbox) {
            for (uint32_t il = t; il < nisl; il += blockDim.x) {
                const uint32_t plan = l_plan[il];
                if ((plan & 15u) == 0) continue;
                const uint32_t isl = first_isl + il;
                const uint32_t x = isl % W;
                uint4 lo[4], hi[4];
#pragma unroll
                for (int d = 0; d < 4; ++d) {
                    if ((plan >> d) & 1u) {
                        const uint32_t* e =
                            p.ob_in + (size_t)neighbour_of(isl, x, d, W, p.I) * kOutboxWords;
                        lo[d] = *reinterpret_cast<const uint4*>(e);
                        if (SW > 1) hi[d] = *reinterpret_cast<const uint4*>(e + 4);
                    }
                }
#pragma unroll
                for (int d = 0; d < 4; ++d) {
                    if ((plan >> d) & 1u) {
                        const uint32_t la = il * N + ((plan >> (4 + 6 * d)) & 63u);
                        l_trait[la] = lo[d].y;
                        l_count[la] = lo[d].z;
                        l_surf[la] = lo[d].w;
                        if (SW > 1) l_surf[TA + la] = hi[d].x;
                    }
                }
            }
        }
        __syncthreads();
    }

    // 3. births
    // this generation's deposit: word and bit offset of the site, none
    // (no word matches) between ingests
    uint32_t site_word = 0xffu, site_shift = 0u;
    if (p.site) {
        const uint32_t site = *p.site;
        site_word = site >> (5u - p.diff_log2);
        site_shift = (site << p.diff_log2) & 31u;
    }
    const uint32_t diff_mask = p.diff_log2 ? 0xffu : 1u;
    if (!mine) return;
    Lanes<APT> ctr, ccn, csf[SW];
#pragma unroll
    for (int q = 0; q < APT; ++q) {
        const uint32_t la = la0 + q;
        const uint32_t il = (la * p.div_magic) >> 20;   // la / N, exact for la < 4096
        const uint32_t j = la - il * N;
        const uint32_t isl = first_isl + il;
        bool act = true;
        if constexpr (ASYNC) act = (l_plan[il] >> 31) != 0u;
        if (!act) {
            // idle island: the same individual on the next tick
            ctr.v[q] = l_trait[la];
            ccn.v[q] = l_count[la];
#pragma unroll
            for (int w = 0; w < SW; ++w) csf[w].v[q] = l_surf[w * TA + la];
        } else {
            const uint4 r = philox4x32_10(make_uint4(j, isl, p.g, kBirth), p.k0, p.k1);
            const uint32_t base = il * N;
            uint32_t par = base + word_below(r.x, N);
            uint32_t bit;
            if constexpr (BM == kBirthFloat) {
                // tournament of p.tour draws (words r.x, r.y, r.z, r.w, v.x),
                // the first of maximal fitness winning; mutation class from
                // v.y, |Z| from v.z and v.w, differentia the low bits of v.w
                const uint4 v = philox4x32_10(make_uint4(j, isl, p.g, kBirthB), p.k0, p.k1);
                float best = __uint_as_float(l_trait[par]);
                const uint32_t words[4] = {r.y, r.z, r.w, v.x};
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    if ((uint32_t)c + 1u < p.tour) {
                        const uint32_t cb = base + word_below(words[c], N);
                        const float fc = __uint_as_float(l_trait[cb]);
                        if (fc > best) {
                            best = fc;
                            par = cb;
                        }
                    }
                }
                const bool del = v.y < p.del_thr;
                const bool ben = !del && p.ben_thr != 0u && v.y >= 0u - p.ben_thr;
                ctr.v[q] = (del || ben) ? __float_as_uint(mutate_fitness(best, del, p.del_sigma,
                                                                         p.ben_sigma, v.z, v.w))
                                        : __float_as_uint(best);
                bit = v.w & diff_mask;
            } else {
                uint32_t ptrait = l_trait[par];
                if constexpr (BM == kBirthIntTournament) {
                    const uint32_t pb = base + word_below(r.y, N);
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
            const uint32_t T = l_count[par];
            ccn.v[q] = T + 1u;
            uint32_t dep_word = site_word, dep_shift = site_shift;
            if constexpr (ASYNC) {
                // the parent's own counter picks the item and, through the
                // site table, its site
                const uint32_t tau = p.interval == 1u ? T : T / p.interval;
                dep_word = 0xffu;
                if (tau * p.interval == T) {
                    const uint32_t site = p.site_tab[tau];
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
        if (MIGR) {
            const uint32_t em = l_emig[il];
            if (j == (em & 0xffu)) {
                uint32_t* o = p.ob_out + (size_t)isl * kOutboxWords;
                const uint32_t dir = (em >> 8) & 7u;
                if (dir < 4u) {
                    *reinterpret_cast<uint4*>(o) = make_uint4(dir, ctr.v[q], ccn.v[q], csf[0].v[q]);
                    *reinterpret_cast<uint4*>(o + 4) =
                        make_uint4(SW > 1 ? csf[SW - 1].v[q] : 0u, 0u, 0u, 0u);
                } else {
                    *reinterpret_cast<uint4*>(o) = make_uint4(dir, 0u, 0u, 0u);
                    *reinterpret_cast<uint4*>(o + 4) = make_uint4(0u, 0u, 0u, 0u);
                }
            }
        }
    }
    store_lanes<APT>(p.out_trait + a0 + la0, ctr);
    store_lanes<APT>(p.out_counter + a0 + la0, ccn);
#pragma unroll
    for (int w = 0; w < SW; ++w) store_lanes<APT>(p.out_surf + w * A + a0 + la0, csf[w]);
}

template <int SW, uint32_t BM, bool MIGR, int APT, bool ASYNC>
__global__ __launch_bounds__(1024) void step_kernel(const StepParams p) {
    step_tile<SW, BM, MIGR, APT, ASYNC>(p, xcd_local_block(blockIdx.x, gridDim.x));
}

size_t step_lds_bytes(uint32_t tile_isl, uint32_t N, uint32_t SW) {
    const size_t TA = ((size_t)tile_isl * N + 3) & ~(size_t)3;
    return ((2 + SW) * TA + 2 * (size_t)tile_isl) * 4;
}

template <int SW, uint32_t BM, bool MIGR, int APT, bool ASYNC>
static hipError_t launch_step_t(const StepParams& p, uint32_t block_threads, hipStream_t stream) {
    const uint32_t tiles = (p.I + p.tile_isl - 1) / p.tile_isl;
    const size_t lds = step_lds_bytes(p.tile_isl, p.N, SW);
    hipLaunchKernelGGL((step_kernel<SW, BM, MIGR, APT, ASYNC>), dim3(tiles), dim3(block_threads),
                       lds, stream, p);
    return hipGetLastError();
}

template <int SW, uint32_t BM, bool MIGR, bool ASYNC>
static hipError_t launch_step_apt(const StepParams& p, uint32_t apt, uint32_t block_threads,
                                  hipStream_t stream) {
    if (apt == 4) return launch_step_t<SW, BM, MIGR, 4, ASYNC>(p, block_threads, stream);
    if (apt == 2) return launch_step_t<SW, BM, MIGR, 2, ASYNC>(p, block_threads, stream);
    return launch_step_t<SW, BM, MIGR, 1, ASYNC>(p, block_threads, stream);
}

template <int SW, uint32_t BM, bool ASYNC>
static hipError_t launch_step_mig(const StepParams& p, bool migration, uint32_t apt,
                                  uint32_t block_threads, hipStream_t stream) {
    return migration ? launch_step_apt<SW, BM, true, ASYNC>(p, apt, block_threads, stream)
                     : launch_step_apt<SW, BM, false, ASYNC>(p, apt, block_threads, stream);
}

template <int SW, bool ASYNC>
static hipError_t launch_step_model(const StepParams& p, uint32_t birth_model, bool migration,
                                    uint32_t apt, uint32_t block_threads, hipStream_t stream) {
    if (birth_model == kBirthFloat)
        return launch_step_mig<SW, kBirthFloat, ASYNC>(p, migration, apt, block_threads, stream);
    if (birth_model == kBirthIntTournament)
        return launch_step_mig<SW, kBirthIntTournament, ASYNC>(p, migration, apt, block_threads,
                                                               stream);
    return launch_step_mig<SW, kBirthIntNeutral, ASYNC>(p, migration, apt, block_threads, stream);
}

template <bool ASYNC>
static hipError_t launch_step_sw(const StepParams& p, uint32_t SW, uint32_t birth_model,
                                 bool migration, uint32_t apt, uint32_t block_threads,
                                 hipStream_t stream) {
    if (SW == 1)
        return launch_step_model<1, ASYNC>(p, birth_model, migration, apt, block_threads, stream);
    return launch_step_model<2, ASYNC>(p, birth_model, migration, apt, block_threads, stream);
}

hipError_t launch_step(const StepParams& p, uint32_t SW, uint32_t birth_model, bool migration,
                       uint32_t agents_per_thread, uint32_t block_threads, hipStream_t stream) {
    if (p.async_thr)
        return launch_step_sw<true>(p, SW, birth_model, migration, agents_per_thread,
                                    block_threads, stream);
    return launch_step_sw<false>(p, SW, birth_model, migration, agents_per_thread, block_threads,
                                 stream);
}

// ---------------------------------------------------------------------------
// Batched forms: many runs of different sizes, surfaces, treatments and
// agents per thread in one launch per generation, sharing step_tile and
// schedule_sites with the plain forms.
__global__ __launch_bounds__(64) void batch_site_schedule_kernel(
    const BatchRun* __restrict__ runs) {
    const BatchRun& R = runs[blockIdx.x];
    const uint32_t tau0 = ingests_of(R.T0, R.interval);
    const uint32_t count = ingests_of(R.T0 + R.gens, R.interval) - tau0;
    schedule_sites(R.kind, R.S, R.layout, R.sites, tau0, count);
}

hipError_t launch_batch_site_schedule(const BatchRun* runs, uint32_t nruns, hipStream_t stream) {
    if (nruns == 0) return hipSuccess;
    hipLaunchKernelGGL(batch_site_schedule_kernel, dim3(nruns), dim3(64), 0, stream, runs);
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
                                                         const uint32_t* __restrict__ tile0,
                                                         uint32_t nruns, uint32_t k) {
    __shared__ uint32_t s_tile0[kMaxBatchRuns + 1];
    for (uint32_t i = threadIdx.x; i <= nruns; i += blockDim.x) s_tile0[i] = tile0[i];
    __syncthreads();
    const uint32_t tile = xcd_local_block(blockIdx.x, gridDim.x);
    // the run owning this tile: last r with tile0[r] <= tile
    uint32_t lo = 0, hi = nruns;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (s_tile0[mid] <= tile) lo = mid;
        else hi = mid;
    }
    const BatchRun& R = runs[lo];
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
    p.async_thr = 0u;          // batched runs are synchronous
    p.site_tab = nullptr;
    p.interval = R.interval;
    p.tour = R.tour;
    p.del_thr = R.del_thr; p.ben_thr = R.ben_thr;
    p.del_sigma = R.del_sigma; p.ben_sigma = R.ben_sigma;
    const uint32_t t = tile - s_tile0[lo];
    const uint32_t model = (R.variant >> 1) & 3u;
    if (model == kBirthIntTournament) step_tile_variant<kBirthIntTournament>(p, t, R.variant);
    else if (WITH_FLOAT && model == kBirthFloat) step_tile_variant<kBirthFloat>(p, t, R.variant);
    else step_tile_variant<kBirthIntNeutral>(p, t, R.variant);
}

hipError_t launch_batch_step(const BatchRun* runs, const uint32_t* tile0, uint32_t nruns,
                             uint32_t total_tiles, uint32_t k, uint32_t block_threads,
                             size_t lds_bytes, bool with_float, hipStream_t stream) {
    if (nruns == 0 || total_tiles == 0) return hipSuccess;
    if (with_float)
        hipLaunchKernelGGL(batch_step_kernel<true>, dim3(total_tiles), dim3(block_threads),
                           lds_bytes, stream, runs, tile0, nruns, k);
    else
        hipLaunchKernelGGL(batch_step_kernel<false>, dim3(total_tiles), dim3(block_threads),
                           lds_bytes, stream, runs, tile0, nruns, k);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Plain streaming copy (instrumentation): one 16-byte load and store per
// lane per iteration, grid-stride.
__global__ __launch_bounds__(256) void probe_copy_kernel(const uint4* __restrict__ src,
                                                        uint4* __restrict__ dst, size_t n16) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride)
        dst[i] = src[i];
}

hipError_t launch_probe_copy(const void* src, void* dst, size_t bytes, hipStream_t stream) {
    const size_t n16 = bytes / 16;
    size_t blocks = (n16 + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(probe_copy_kernel, dim3((uint32_t)blocks), dim3(256), 0, stream,
                       static_cast<const uint4*>(src), static_cast<uint4*>(dst), n16);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Stratified end-of-run sample (Results, On-hardware Trial): agent k is
// drawn uniformly from the k-th of n equal strata; every agent when A <= n.
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
    counter_out[k] = counter[a];
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

// One wavefront: classify the counters; when all are equal, replay the
// shared layout once (in ingest units), order its sites by deposit time and
// tabulate the bounds, in generations, for every possible first-mismatch
// rank.
__global__ __launch_bounds__(64) void mrca_prepare_kernel(Scheme sc, uint32_t n,
                                                         const uint32_t* __restrict__ counter,
                                                         uint32_t* __restrict__ ws) {
    const uint32_t lane = threadIdx.x;
    const uint32_t S = sc.S;
    const uint32_t T0 = counter[0];
    const uint64_t hz = horizon_of(sc.kind, S);
    bool same = true, past = false;
    for (uint32_t k = lane; k < n; k += 64) {
        const uint32_t c = counter[k];
        const uint32_t ing = ingests_of(c, sc.interval);
        same = same && c == T0;
        past = past || ing > kMaxReplayGenerations || (ing > 0 && (uint64_t)(ing - 1) > hz);
    }
    const bool any_past = __ballot(past) != 0;
    const bool all_same = __ballot(!same) == 0;
    if (any_past || !all_same) {
        if (lane == 0) {
            ws[kWsStatus] = any_past ? kWsStatusHorizon : kWsStatusMixed;
            ws[kWsT] = T0;
        }
        return;
    }
    const uint32_t held = replay_layout(sc.kind, S, ingests_of(T0, sc.interval), lane);
    const uint32_t rank = time_rank(held, lane, S);
    const uint32_t F = (uint32_t)__popcll(__ballot(lane < S && held != kEmpty));
    __shared__ uint32_t times[64];
    if (lane < S) {
        const uint32_t gen = held == kEmpty ? kEmpty : held * sc.interval;   // deposit generation
        times[rank] = gen;
        ws[kWsPerm + rank] = lane;
        ws[kWsTimes + rank] = gen;
    }
    __syncthreads();
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
    if (ws[kWsStatus] != 0) return;
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

// General route (counters differ): one wavefront per annotation replays its
// own layout and stores its retained deposit generations in ascending order
// with their sites.
__global__ __launch_bounds__(64) void mrca_layouts_kernel(Scheme sc, uint32_t n,
                                                         const uint32_t* __restrict__ counter,
                                                         const uint32_t* __restrict__ ws,
                                                         uint32_t* __restrict__ times,
                                                         uint8_t* __restrict__ sites) {
    if (ws[kWsStatus] != kWsStatusMixed) return;
    const uint32_t a = blockIdx.x;
    const uint32_t lane = threadIdx.x;
    const uint32_t S = sc.S;
    const uint32_t held = replay_layout(sc.kind, S, ingests_of(counter[a], sc.interval), lane);
    const uint32_t rank = time_rank(held, lane, S);
    if (lane < S) {
        times[(size_t)a * S + rank] = held == kEmpty ? kEmpty : held * sc.interval;
        sites[(size_t)a * S + rank] = (uint8_t)lane;
    }
}

// General route, all ordered pairs: merge the two ascending time lists,
// comparing differentiae on common times until the first mismatch.
__global__ __launch_bounds__(256) void mrca_general_pairs_kernel(
    uint32_t S, uint32_t diff_log2, uint32_t n, const uint32_t* __restrict__ counter,
    const uint32_t* __restrict__ surf, const uint32_t* __restrict__ times,
    const uint8_t* __restrict__ sites, const uint32_t* __restrict__ ws, uint32_t* __restrict__ lb,
    uint32_t* __restrict__ ub) {
    if (ws[kWsStatus] != kWsStatusMixed) return;
    const uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t a = blockIdx.y;
    if (b >= n) return;
    const uint32_t SW = (S << diff_log2) >> 5;
    const uint64_t sa = surface64(surf, SW, a);
    const uint64_t sb = surface64(surf, SW, b);
    const uint64_t mask = diff_log2 ? 0xffull : 1ull;
    const uint32_t* ta = times + (size_t)a * S;
    const uint32_t* tb = times + (size_t)b * S;
    const uint8_t* ka = sites + (size_t)a * S;
    const uint8_t* kb = sites + (size_t)b * S;
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
    const uint32_t Ta = counter[a], Tb = counter[b];
    const size_t off = (size_t)a * n + b;
    ub[off] = mismatch ? tstar : (Ta < Tb ? Ta : Tb);
    lb[off] = have_last ? last + 1u : 0u;
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
constexpr uint32_t kPhyloOutWords = 6;   // sbl, pair sum, root, internal, status, n

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

// One workgroup: bitonic sort of (key, index) over npad (a power of two)
// entries held in global memory.
__global__ __launch_bounds__(1024) void phylo_sort_kernel(uint32_t npad,
                                                         const uint32_t* __restrict__ ws,
                                                         uint64_t* __restrict__ keys,
                                                         uint32_t* __restrict__ idx) {
    if (ws[kWsStatus] != 0) return;
    for (uint32_t k = 2; k <= npad; k <<= 1) {
        for (uint32_t j = k >> 1; j > 0; j >>= 1) {
            for (uint32_t t = threadIdx.x; t < npad / 2; t += blockDim.x) {
                const uint32_t i = (t / j) * 2 * j + (t % j);
                const uint32_t l = i + j;
                const bool up = (i & k) == 0;
                const uint64_t ki = keys[i], kl = keys[l];
                const uint32_t ii = idx[i], il = idx[l];
                const bool greater = ki > kl || (ki == kl && ii > il);
                if (greater == up) {
                    keys[i] = kl; keys[l] = ki;
                    idx[i] = il; idx[l] = ii;
                }
            }
            __syncthreads();
        }
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
        out[0] = out[1] = out[2] = out[3] = 0;
    } else {
        out[0] = acc->sbl;
        out[1] = acc->pairs;
        out[2] = n > 1 ? phylo_tau(ws, (uint32_t)acc->dmin) : ws[kWsT];
        out[3] = acc->internal;
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
                        uint32_t* node_time) {
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
    hipLaunchKernelGGL(mrca_prepare_kernel, dim3(1), dim3(64), 0, stream, scm, n, counter, ws);
    hipLaunchKernelGGL(mrca_rank_kernel, dim3(gn), dim3(256), 0, stream, scm.S, diff_log2, n,
                       surf, ws, ranked);
    hipLaunchKernelGGL(phylo_keys_kernel, dim3((uint32_t)((npad + 255) / 256)), dim3(256), 0,
                       stream, n, (uint32_t)npad, diff_log2, ranked, ws, keys, idx);
    hipLaunchKernelGGL(phylo_sort_kernel, dim3(1), dim3(1024), 0, stream, (uint32_t)npad, ws,
                       keys, idx);
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
                       hipStream_t stream) {
    const uint32_t S = scm.S;
    const uint32_t diff_log2 = scm.bits == 8 ? 3u : 0u;
    uint8_t* base = static_cast<uint8_t*>(workspace);
    uint32_t* ws = reinterpret_cast<uint32_t*>(base);
    uint64_t* ranked = reinterpret_cast<uint64_t*>(base + MrcaWorkspace::kHeader);
    const size_t ranked_bytes = ((size_t)n * 8 + 255) & ~(size_t)255;
    uint32_t* times = reinterpret_cast<uint32_t*>(base + MrcaWorkspace::kHeader + ranked_bytes);
    const size_t times_bytes = ((size_t)n * S * 4 + 255) & ~(size_t)255;
    uint8_t* sites = base + MrcaWorkspace::kHeader + ranked_bytes + times_bytes;

    hipLaunchKernelGGL(mrca_prepare_kernel, dim3(1), dim3(64), 0, stream, scm, n, counter, ws);
    hipLaunchKernelGGL(mrca_rank_kernel, dim3((n + 255) / 256), dim3(256), 0, stream, S,
                       diff_log2, n, surf, ws, ranked);
    hipLaunchKernelGGL(mrca_allpairs_kernel, dim3((n + 1023) / 1024, (n + kPairRows - 1) / kPairRows),
                       dim3(256), 0, stream, n, diff_log2, ranked, ws, lb, ub);
    hipLaunchKernelGGL(mrca_layouts_kernel, dim3(n), dim3(64), 0, stream, scm, n, counter, ws,
                       times, sites);
    hipLaunchKernelGGL(mrca_general_pairs_kernel, dim3((n + 255) / 256, n), dim3(256), 0, stream,
                       S, diff_log2, n, counter, surf, times, sites, ws, lb, ub);
    return hipGetLastError();
}

}  // namespace hsga
