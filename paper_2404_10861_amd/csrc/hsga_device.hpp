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

// Local time at which item t (local deposit time) leaves the retention
// target D(u) of an m-site sub-surface, kNever if it stays as long as the
// 32-bit counter runs.  Membership is monotone (D(u) without u is a subset
// of D(u-1)), so "t is out of D(u)" is exactly "u >= leave_time(t)".
//   Steady, D(u) = multiples of g(u) = 2^bitlen(floor(u/(m-1))) plus u:
//     for u > t, t stays while g(u) divides t, i.e. floor(u/(m-1)) <
//     2^ctz(t), i.e. u < (m-1) * 2^ctz(t); item 0 never leaves.
//   Tilted, D(u) = the r(u) = floor(m / bitlen(u+1)) most recent items of
//     each level h = ctz(t+1), t+1 = (2c+1) 2^h: t leaves at the first u
//     with n_h(u) = (u + 1 + 2^h) >> (h+1) > c + r(u).  Within one epoch of
//     bitlen(u+1) = B, r is constant, so that u is
//     max((c+r+1) 2^(h+1) - 2^h - 1, first u of the epoch).
constexpr uint32_t kNever = 0xffffffffu;

__host__ __device__ inline uint32_t leave_time(uint32_t policy, uint32_t m, uint32_t t) {
    if (policy == kSteady) {
        if (t == 0) return kNever;
        const uint64_t e = (uint64_t)(m - 1) << __builtin_ctz(t);
        const uint64_t x = e > (uint64_t)t + 1 ? e : (uint64_t)t + 1;
        return x >= kNever ? kNever : (uint32_t)x;
    }
    const uint32_t h = (uint32_t)__builtin_ctz(t + 1u);
    const uint64_t c = ((uint64_t)t + 1) >> (h + 1);
    const uint64_t t1 = (uint64_t)t + 1;
    uint32_t B = 64u - (uint32_t)__builtin_clzll(t1 + 1);   // epoch of u = t + 1
    for (; B <= m && B < 34; ++B) {
        const uint64_t r = m / B;
        const uint64_t need = ((c + r + 1) << (h + 1)) - (1ull << h) - 1;
        const uint64_t first = (1ull << (B - 1)) - 1;
        uint64_t u = need > first ? need : first;
        if (u < t1) u = t1;
        if (u <= (1ull << B) - 2) return u >= kNever ? kNever : (uint32_t)u;
    }
    return kNever;   // stays until past the horizon
}

// One placement across the wavefront: lane k holds the deposit time of
// site k (global time, kEmpty if unfilled) and the local time its item
// leaves the target (0 if unfilled).  Item T goes to its own local slot
// while its sub-surface fills, otherwise to the lowest site of the
// sub-surface whose item has left the target (ballot + bit scan); -1 if
// none (past the horizon).  The chosen lane takes (T, new_leave), the leave
// time of item T.  Must be called by all 64 lanes with uniform arguments.
__device__ __forceinline__ int place_in_wave(uint32_t kind, uint32_t S, uint32_t T,
                                             uint32_t new_leave, uint32_t& lane_time,
                                             uint32_t& lane_leave, uint32_t lane) {
    const SubSurface s = sub_surface(kind, S, T);
    int site;
    if (s.u < s.m) {
        site = (int)(s.offset + s.u);
    } else {
        const bool evictable = lane >= s.offset && lane < s.offset + s.m && s.u >= lane_leave;
        const uint64_t mask = __ballot(evictable);
        site = mask ? (int)(__ffsll((long long)mask) - 1) : -1;
    }
    if ((int)lane == site) {
        lane_time = T;
        lane_leave = new_leave;
    }
    return site;
}

// Leave time of item T in its own sub-surface.
__device__ __forceinline__ uint32_t item_leave_time(uint32_t kind, uint32_t S, uint32_t T) {
    const SubSurface s = sub_surface(kind, S, T);
    return leave_time(s.policy, s.m, s.u);
}

// Places items T0 .. T0+G-1 in blocks of 64: each lane first computes the
// leave time of one item of the block (in parallel), then the 64 serial
// placements read it with readlane.  site_out(k, site) is called by lane
// k % 64 once per item.  Must be called by all 64 lanes.
template <typename SiteOut>
__device__ __forceinline__ void place_items(uint32_t kind, uint32_t S, uint32_t T0, uint32_t G,
                                            uint32_t& lane_time, uint32_t& lane_leave,
                                            uint32_t lane, SiteOut site_out) {
    for (uint32_t base = 0; base < G; base += 64) {
        const uint32_t n = G - base < 64 ? G - base : 64;
        const uint32_t mine = lane < n ? item_leave_time(kind, S, T0 + base + lane) : 0u;
        int my_site = -1;
        for (uint32_t j = 0; j < n; ++j) {
            const uint32_t nl = (uint32_t)__builtin_amdgcn_readlane((int)mine, (int)j);
            const int site = place_in_wave(kind, S, T0 + base + j, nl, lane_time, lane_leave, lane);
            if (lane == j) my_site = site;
        }
        if (lane < n) site_out(base + lane, my_site);
    }
}

// Leave time of the item a lane holds (at the start of a schedule or replay).
__device__ __forceinline__ uint32_t lane_leave_time(uint32_t kind, uint32_t S, uint32_t lane,
                                                    uint32_t lane_time) {
    if (lane_time == kEmpty || lane >= S) return 0u;
    if (kind == kHybrid) {
        const bool tilted_half = lane >= (S >> 1);
        return leave_time(tilted_half ? kTilted : kSteady, S >> 1, lane_time >> 1);
    }
    return leave_time(kind, S, lane_time);
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
