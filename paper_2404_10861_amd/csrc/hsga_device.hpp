// hsga_device.hpp -- device building blocks for gfx950 (wave64):
// Philox4x32-10, the integer maps, and the surface site rule evaluated
// across one wavefront (lane k owns site k).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hsga {

constexpr uint32_t kEmpty = 0xffffffffu;
constexpr uint32_t kSteady = 0, kTilted = 1, kHybrid = 2;
// Fourth Philox counter word: what the draw is for.
constexpr uint32_t kBirth = 0, kEmigrate = 1, kImmigrate = 2, kSample = 3;
// Outbox entry: dir, trait, counter, surface words (up to 2), padding.
constexpr uint32_t kOutboxWords = 8;

// Philox4x32-10 (Salmon et al., SC'11).  Counter (c.x, c.y, c.z, c.w), key
// (k0, k1).  Each round forms the two 32x32->64 products of counter words
// 0 and 2 with the Philox multipliers, swaps the halves across the two
// lanes of the block and folds in the key; the key advances by the Weyl
// increments after every round.  The key is wave-uniform, so its schedule
// stays in scalar registers.  Each three-way XOR is one v_bitop3_b32
// (truth table 0x96) on gfx950.
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint64_t prod0 = (uint64_t)c.x * 0xD2511F53u;
        const uint64_t prod1 = (uint64_t)c.z * 0xCD9E8D57u;
        const uint32_t hi0 = (uint32_t)(prod0 >> 32), lo0 = (uint32_t)prod0;
        const uint32_t hi1 = (uint32_t)(prod1 >> 32), lo1 = (uint32_t)prod1;
        c = make_uint4(xor3(hi1, c.y, k0), lo1, xor3(hi0, c.w, k1), lo0);
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

// A uniform 32-bit word mapped onto [0, n).
__device__ __forceinline__ uint32_t word_below(uint32_t w, uint32_t n) {
    return __umulhi(w, n);
}

// Number of significant bits.
__device__ __forceinline__ uint32_t bit_length64(uint64_t x) {
    return x ? 64u - (uint32_t)__clzll((long long)x) : 0u;
}

// Sub-surface that deposit time T belongs to (hybrid: even T on the steady
// half [0, S/2) with local time T/2, odd T on the tilted half [S/2, S) with
// local time (T-1)/2; otherwise one surface of S sites with local time T).
struct SubSurface {
    uint32_t policy, m, offset, u;
};

__device__ __forceinline__ SubSurface sub_surface(uint32_t kind, uint32_t S, uint32_t T) {
    SubSurface s;
    if (kind == kHybrid) {
        s.m = S >> 1;
        if ((T & 1u) == 0) { s.policy = kSteady; s.u = T >> 1; s.offset = 0; }
        else { s.policy = kTilted; s.u = (T - 1) >> 1; s.offset = S >> 1; }
    } else {
        s.policy = kind; s.m = S; s.u = T; s.offset = 0;
    }
    return s;
}

// Is item t (local time, t <= u) part of the retention target D(u) of an
// m-site sub-surface?  Steady: multiples of 2^bitlen(u/(m-1)), plus u.
// Tilted: on each level h = ctz(t+1) keep the floor(m/bitlen(u+1)) most
// recent items.
__device__ __forceinline__ bool retained_target(uint32_t policy, uint32_t m, uint32_t u,
                                                uint32_t t) {
    if (policy == kSteady) {
        const uint32_t q = u / (m - 1u);
        const uint32_t spacing_bits = q ? 32u - (uint32_t)__clz((int)q) : 0u;  // < 30 for m >= 16
        return ((t & ((1u << spacing_bits) - 1u)) == 0u) || t == u;
    }
    const uint32_t r = m / bit_length64((uint64_t)u + 1u);
    const uint32_t h = (uint32_t)__ffs((int)(t + 1u)) - 1u;
    const uint64_t c = ((uint64_t)t + 1u) >> (h + 1);
    const uint64_t n_h = ((uint64_t)u + 1u + (1ull << h)) >> (h + 1);
    return c + r >= n_h;
}

// One placement across the wavefront: lane k holds the deposit time of
// site k (global time, kEmpty if unfilled).  Returns the site that item T
// goes to: T's own local slot while its sub-surface fills, otherwise the
// lowest site of the sub-surface whose item has left the target (ballot +
// bit scan).  Returns -1 when no site is evictable (past the horizon).
// Must be called by all 64 lanes with a uniform T.
__device__ __forceinline__ int place_in_wave(uint32_t kind, uint32_t S, uint32_t T,
                                             uint32_t lane_time, uint32_t lane) {
    const SubSurface s = sub_surface(kind, S, T);
    if (s.u < s.m)
        return (int)(s.offset + s.u);
    bool evictable = false;
    if (lane >= s.offset && lane < s.offset + s.m) {
        if (lane_time == kEmpty) {
            evictable = true;
        } else {
            const uint32_t t_local = kind == kHybrid ? lane_time >> 1 : lane_time;
            evictable = !retained_target(s.policy, s.m, s.u, t_local);
        }
    }
    const uint64_t mask = __ballot(evictable);
    if (mask == 0)
        return -1;
    return (int)(__ffsll((long long)mask) - 1);
}

// The MRCA kernels replay layouts on the device, one placement per
// generation; counters above this bound are refused.
constexpr uint32_t kMaxReplayGenerations = 1u << 24;

// Last deposit time the rule can place for (kind, S): tilted needs
// bitlen(u+1) <= m; the 32-bit counter caps every kind at 2^32 - 2.
__host__ __device__ inline uint64_t horizon_of(uint32_t kind, uint32_t S) {
    const uint64_t cap = 0xfffffffeull;
    uint64_t h = cap;
    if (kind == kTilted && S < 33) h = (1ull << S) - 2;
    if (kind == kHybrid && (S >> 1) < 33) h = 2 * ((1ull << (S >> 1)) - 2) + 2;
    return h < cap ? h : cap;
}

// Maps workgroup IDs so that consecutive logical tiles land on the same XCD
// (the dispatcher hands workgroups to the 8 XCDs round-robin); torus
// neighbours then share an L2.  A bijection on [0, nblocks).
__device__ __forceinline__ uint32_t xcd_local_block(uint32_t b, uint32_t nblocks) {
    const uint32_t full = nblocks & ~7u;
    if (b >= full) return b;
    return (b & 7u) * (full >> 3) + (b >> 3);
}

}  // namespace hsga
