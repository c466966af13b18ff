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
// Second block of a float-treatment birth; founder tags; whether an island
// is active on a tick of an asynchronous run.
constexpr uint32_t kBirthB = 4, kFounder = 5, kActivity = 6;
// Outbox entry of an asynchronous run: dir, trait, counter, surface words
// (up to 2), padding.  A synchronous run's emigrant carries counter T, the
// generation count, so its entry is dir, trait, surface words (up to 2):
// 16 bytes.  The arena reserves the larger size.
constexpr uint32_t kOutboxWords = 8;
constexpr uint32_t kSyncOutboxWords = 4;

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

// K independent Philox4x32-10 blocks under one key, advanced round by
// round together so that their multiply chains overlap in the pipeline.
template <int K>
__device__ __forceinline__ void philox4x32_10_multi(uint4 (&c)[K], uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int round = 0; round < 10; ++round) {
#pragma unroll
        for (int q = 0; q < K; ++q) {
            const uint64_t prod0 = (uint64_t)c[q].x * 0xD2511F53u;
            const uint64_t prod1 = (uint64_t)c[q].z * 0xCD9E8D57u;
            const uint32_t hi0 = (uint32_t)(prod0 >> 32), lo0 = (uint32_t)prod0;
            const uint32_t hi1 = (uint32_t)(prod1 >> 32), lo1 = (uint32_t)prod1;
            c[q] = make_uint4(xor3(hi1, c[q].y, k0), lo1, xor3(hi0, c[q].w, k1), lo0);
        }
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

// A uniform 32-bit word mapped onto [0, n).
__device__ __forceinline__ uint32_t word_below(uint32_t w, uint32_t n) {
    return __umulhi(w, n);
}

// ---------------------------------------------------------------------------
// Half-normal draw of the float treatments (Results, On-hardware Trial:
// mutations change fitness by normally distributed amounts).  Box and
// Muller (1958) give |Z| the law of sqrt(-2 ln U1) cos(pi/2 U2) for U1, U2
// uniform on (0, 1); here U1 = (w_radius + 1/2) 2^-32 and U2 = (w_angle +
// 1/2) 2^-32.  The draw is defined by one fixed binary64 evaluation made
// only of correctly rounded +, -, *, fma and exact power-of-two scalings, so
// every IEEE-754 machine that takes the same steps gets the same bits:
//   ln U1: U1 = m 2^(e-33) with m in [sqrt(1/2), sqrt(2)]; ln m = 2 atanh s,
//          s = (m-1)/(m+1), 1/(m+1) by five Newton steps from 1/2, atanh by
//          its odd series through s^21;
//   sqrt:  y = q 4^k, q in [1, 4); 1/sqrt q by six Newton steps from
//          9/8 - 3q/16, sqrt q = q (1/sqrt q) plus one correction;
//   cos:   cos(pi/2 U2) by its series through x^18 when U2 < 1/2, else
//          sin(pi/2 (1 - U2)) by its series through x^19.
// Contraction is off: every fused multiply-add below is written out.
constexpr uint64_t kMantissa = 0x000FFFFFFFFFFFFFull;   // binary64 fraction bits
constexpr uint64_t kExpZero = 0x3FF0000000000000ull;    // biased exponent of 2^0

// The series coefficients of the half-normal evaluation, read through
// scalar loads (so that a loop over draws keeps them in scalar registers):
// atanh 1/(2k+1) for k = 10 .. 0, then sine 1/(2k+1)! with alternating
// signs for k = 9 .. 0, then cosine 1/(2k)! for k = 10 .. 1 (the last
// cosine term, 1, is written out).
__constant__ double kHalfNormalSeries[31] = {
    1.0 / 21.0, 1.0 / 19.0, 1.0 / 17.0, 1.0 / 15.0, 1.0 / 13.0, 1.0 / 11.0,
    1.0 / 9.0, 1.0 / 7.0, 1.0 / 5.0, 1.0 / 3.0, 1.0,
    -1.0 / 121645100408832000.0, 1.0 / 355687428096000.0, -1.0 / 1307674368000.0,
    1.0 / 6227020800.0, -1.0 / 39916800.0, 1.0 / 362880.0, -1.0 / 5040.0, 1.0 / 120.0,
    -1.0 / 6.0, 1.0,
    -1.0 / 6402373705728000.0, 1.0 / 20922789888000.0, -1.0 / 87178291200.0,
    1.0 / 479001600.0, -1.0 / 3628800.0, 1.0 / 40320.0, -1.0 / 720.0, 1.0 / 24.0,
    -1.0 / 2.0, 1.0,
};

// The draw for an angle word of a known case: SIN for w_angle >= 2^31 (the
// sine series), else the cosine series.
template <bool SIN>
__device__ __forceinline__ double half_normal_case(uint32_t w_radius, uint32_t w_angle) {
#pragma clang fp contract(off)
    const double* K = kHalfNormalSeries;
    // ln U1.  v = 2 w_radius + 1 < 2^33 is exact in binary64; its exponent
    // is floor(log2 v), and setting the exponent to 0 gives v 2^-e exactly
    const double vd = __builtin_fma(2.0, (double)w_radius, 1.0);
    const uint64_t vb = (uint64_t)__double_as_longlong(vd);
    int e = (int)(vb >> 52) - 1023;
    double m = __longlong_as_double((long long)((vb & kMantissa) | kExpZero));
    if (m > 1.4142135623730951) {
        m = m * 0.5;
        e = e + 1;
    }
    const double d = m + 1.0;
    double r = 0.5;
#pragma unroll
    for (int k = 0; k < 5; ++k) r = __builtin_fma(r, __builtin_fma(-d, r, 1.0), r);
    const double sv = (m - 1.0) * r;
    const double z = sv * sv;
    double p = K[0];
#pragma unroll
    for (int k = 1; k < 11; ++k) p = __builtin_fma(p, z, K[k]);
    const double ln_u = __builtin_fma((double)e - 33.0, 0.6931471805599453, (sv + sv) * p);
    // sqrt(-2 ln U1)
    const double y = -2.0 * ln_u;
    const uint64_t yb = (uint64_t)__double_as_longlong(y);
    const int ex = (int)((yb >> 52) & 0x7ff) - 1023;                        // floor(log2 y)
    const int kq = ex >> 1;                                                 // floor(ex / 2)
    // q = y 4^-kq exactly: its exponent becomes ex - 2 kq, that is 0 or 1
    const double q =
        __longlong_as_double((long long)((yb & kMantissa) | ((uint64_t)(1023 + (ex & 1)) << 52)));
    const double h = 0.5 * q;
    double rs = __builtin_fma(-0.1875, q, 1.125);
#pragma unroll
    for (int i = 0; i < 6; ++i) rs = __builtin_fma(rs, __builtin_fma(-h, rs * rs, 0.5), rs);
    double sq = q * rs;
    sq = __builtin_fma(__builtin_fma(-sq, sq, q), 0.5 * rs, sq);
    const double radius = __builtin_ldexp(sq, kq);                          // exact scaling
    // cos(pi/2 U2).  2 w_angle + 1, or 2^33 - (2 w_angle + 1) in the sine
    // case, is an exact binary64 integer; the 2^-33 is folded into pi/2
    // (an exact power-of-two scaling of it, so the product rounds the same)
    const double wad = (double)w_angle;
    const double va = SIN ? __builtin_fma(-2.0, wad, 8589934591.0) : __builtin_fma(2.0, wad, 1.0);
    const double x = va * (1.5707963267948966 * 0x1p-33);
    const double x2 = x * x;
    double c;
    if constexpr (SIN) {
        c = K[11];
#pragma unroll
        for (int k = 12; k < 21; ++k) c = __builtin_fma(c, x2, K[k]);
        c = x * c;
    } else {
        c = K[21];
#pragma unroll
        for (int k = 22; k < 31; ++k) c = __builtin_fma(c, x2, K[k]);
    }
    return radius * c;
}

// The fitness after a draw: f - del_sigma |Z| (deleterious) or
// f + ben_sigma |Z|, in binary64, rounded to binary32.  Written as one
// product and one sum with the sign folded into the factor: negation is
// exact and rounding is symmetric, so f + (-s) z rounds as f - s z.
__device__ __forceinline__ float apply_half_normal(float f, bool deleterious, float del_sigma,
                                                   float ben_sigma, double z) {
#pragma clang fp contract(off)
    const double s = deleterious ? -(double)del_sigma : (double)ben_sigma;
    return (float)((double)f + s * z);
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

// Places items T0 .. T0+G-1 across the wavefront.  Lane k holds the deposit
// time of site k (global time, kEmpty if unfilled) and the local time its
// item leaves the target (0 if unfilled).  Item T goes to its own local
// slot while its sub-surface fills, otherwise to the lowest site of the
// sub-surface whose item has left the target; -1 if none (past the
// horizon).  The chosen lane takes (T, the leave time of item T).
// Items go in blocks of 64: each lane first works out one item of the
// block (sub-surface, local time, leave time) in parallel; the serial
// placements then read them with readlane and reduce to a compare, a
// ballot, a bit scan and two selects.  site_out(k, site) is called by
// lane k % 64 once per item.  Must be called by all 64 lanes with uniform
// arguments.
template <typename SiteOut>
__device__ __forceinline__ void place_items(uint32_t kind, uint32_t S, uint32_t T0, uint32_t G,
                                            uint32_t& lane_time, uint32_t& lane_leave,
                                            uint32_t lane, SiteOut site_out) {
    // sites of the sub-surfaces: the whole surface, or the halves of a
    // hybrid one (steady below, tilted above)
    const uint32_t half = S >> 1;
    const uint64_t all = S >= 64 ? ~0ull : (1ull << S) - 1;
    const uint64_t lower = kind == kHybrid ? (1ull << half) - 1 : all;
    const uint64_t upper = ((1ull << half) - 1) << half;
    for (uint32_t base = 0; base < G; base += 64) {
        const uint32_t n = G - base < 64 ? G - base : 64;
        // item T0+base+lane: local time, leave time, and a word holding its
        // fill-phase site (bits 0-7), "still filling" (bit 8) and "upper
        // half" (bit 9)
        uint32_t my_u = 0, my_leave = 0, my_info = 0;
        if (lane < n) {
            const SubSurface sb = sub_surface(kind, S, T0 + base + lane);
            my_u = sb.u;
            my_leave = leave_time(sb.policy, sb.m, sb.u);
            my_info = (sb.u < sb.m ? ((sb.offset + sb.u) | 0x100u) : 0u) |
                      (sb.offset != 0 ? 0x200u : 0u);
        }
        int my_site = -1;
        for (uint32_t j = 0; j < n; ++j) {
            const uint32_t u = (uint32_t)__builtin_amdgcn_readlane((int)my_u, (int)j);
            const uint32_t nl = (uint32_t)__builtin_amdgcn_readlane((int)my_leave, (int)j);
            const uint32_t info = (uint32_t)__builtin_amdgcn_readlane((int)my_info, (int)j);
            const uint64_t range = (info & 0x200u) ? upper : lower;
            const uint64_t left = __ballot(u >= lane_leave) & range;
            const int site = (info & 0x100u) ? (int)(info & 0xffu)
                                              : (left ? (int)__builtin_ctzll(left) : -1);
            if ((int)lane == site) {
                lane_time = T0 + base + j;
                lane_leave = nl;
            }
            if (lane == j) my_site = site;
        }
        if (lane < n) site_out(base + lane, my_site);
    }
}

// Leave time of the item a lane holds (at the start of a replay).
__device__ __forceinline__ uint32_t lane_leave_time(uint32_t kind, uint32_t S, uint32_t lane,
                                                    uint32_t lane_time) {
    if (lane_time == kEmpty || lane >= S) return 0u;
    if (kind == kHybrid) {
        const bool tilted_half = lane >= (S >> 1);
        return leave_time(tilted_half ? kTilted : kSteady, S >> 1, lane_time >> 1);
    }
    return leave_time(kind, S, lane_time);
}

// Without the rule's tables (the allocation-free query) the MRCA kernels
// replay layouts on the device, one placement per ingest; annotations with
// more ingests than this are then refused.
constexpr uint32_t kMaxReplayGenerations = 1u << 24;

// Deposits made by an annotation with counter T (generations 0, interval,
// 2 interval, ... below T).
__host__ __device__ inline uint32_t ingests_of(uint32_t T, uint32_t interval) {
    return (uint32_t)(((uint64_t)T + interval - 1) / interval);
}

// Last deposit time the rule can place for (kind, S): tilted needs
// bitlen(u+1) <= m; the 32-bit counter caps every kind at 2^32 - 2.
__host__ __device__ inline uint64_t horizon_of(uint32_t kind, uint32_t S) {
    const uint64_t cap = 0xfffffffeull;
    uint64_t h = cap;
    if (kind == kTilted && S < 33) h = (1ull << S) - 2;
    if (kind == kHybrid && (S >> 1) < 33) h = 2 * ((1ull << (S >> 1)) - 2) + 2;
    return h < cap ? h : cap;
}

// Last generation a run may step (inclusive): the next deposit after it
// would be past the rule's horizon, or the counter would overflow.
__host__ __device__ inline uint64_t horizon_gen_of(uint32_t kind, uint32_t S, uint32_t interval) {
    const uint64_t g = (horizon_of(kind, S) + 1) * (uint64_t)interval - 1;
    return g < 0xfffffffeull ? g : 0xfffffffeull;
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
