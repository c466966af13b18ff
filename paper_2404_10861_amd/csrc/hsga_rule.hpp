// hsga_rule.hpp -- constant-time form of the surface site rule (Methods,
// Surface-based Hereditary Stratigraphy Algorithms: a surface is indexed in
// constant time from the generation count; Distributed Phylogenetic
// Tracking: deposit times follow from the site index and the count).
//
// The rule places item u of an m-site sub-surface at site u while the
// sub-surface fills, then at the lowest site whose item has left the
// retention target D(u).  Its history collapses into a few tables:
//
//   steady, D(u) = multiples of 2^j plus u, j = bitlen(floor(u/(m-1))):
//     within epoch j (u from E_j = max((m-1) 2^(j-1), m) to (m-1) 2^j - 1)
//     nothing leaves but the newest item when it is not a multiple of 2^j.
//     So the sites evictable at E_j, in ascending order (the pool P_j),
//     are used one by one: u goes to P_j[c], c = the number of multiples
//     of 2^j in [E_j, u), and a non-multiple frees its own site again.
//
//   tilted, D(u) = the r = floor(m/B) newest items of each level h =
//     ctz(t+1), B = bitlen(u+1): within epoch B (r constant) the level-h
//     item of index c (t+1 = (2c+1) 2^h) pushes out the level-h item of
//     index c - r.  Group each level's items by c mod r into chains: a
//     chain's retained item always sits at one site, and a new item
//     takes that site again unless a lower site is free (or the chain is
//     new).  Those exceptions -- events -- are rare (at most 40 in any
//     epoch at m = 64, 245 up to 2^32) and are found by jumping from one
//     to the next.  So u goes to its chain's site at the epoch start,
//     updated by the chain's events up to u.
//
// Tables cover local times up to the rule's horizon (capped at 2^32 - 2).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hsga {

constexpr uint32_t kRuleEpochs = 34;     // steady j <= 32, tilted B <= 33
constexpr uint32_t kRuleEvents = 512;
constexpr uint8_t kRuleNoSite = 0xff;

// One sub-surface (policy, m sites).  Epoch e of the tables is the epoch
// index (j or B) minus `first`.
struct RuleTable {
    uint32_t policy, m, first, n_epochs;
    uint32_t start[kRuleEpochs];           // steady: E_j; tilted: first u of the epoch
    uint32_t r[kRuleEpochs];               // tilted: floor(m / B)
    uint16_t ev_begin[kRuleEpochs][65];    // tilted: events of chain key k are
                                           // ev_begin[e][k] .. ev_begin[e][k+1] - 1
    uint8_t site0[kRuleEpochs][64];        // steady: pool P_j; tilted: chain sites at
                                           // the epoch start by key h * r + c % r
    uint32_t ev_u[kRuleEvents];            // tilted: event times, by chain, ascending
    uint8_t ev_site[kRuleEvents];          // tilted: the chain's site from that time on
    // layouts
    uint32_t layout0[kRuleEpochs][64];     // the items the sites hold at the epoch start
                                           // (steady: at E_j; tilted: free sites' too)
    uint8_t pool_pos[kRuleEpochs][64];     // steady: site k's position in P_j (kRuleNoSite:
                                           // none)
    uint8_t chain_of[kRuleEpochs][64];     // tilted: the chain key holding site k at the
                                           // epoch start (kRuleNoSite: a free site)
    uint16_t evt_begin[kRuleEpochs + 1];   // tilted: the events in time order, epoch e's
    uint32_t evt_u[kRuleEvents];           // at evt_begin[e] .. evt_begin[e + 1] - 1
    uint8_t evt_key[kRuleEvents];
    uint8_t evt_site[kRuleEvents];
};

__host__ __device__ inline uint32_t rule_bitlen(uint64_t x) {
    return x ? 64u - (uint32_t)__builtin_clzll(x) : 0u;
}

// Site of local item u (u within the tables' range).
__host__ __device__ inline uint32_t rule_site(const RuleTable& R, uint32_t u) {
    const uint32_t m = R.m;
    if (u < m) return u;
    if (R.policy == 0) {
        const uint32_t j = rule_bitlen(u / (m - 1));
        const uint32_t e = j - R.first;
        const uint64_t step = 1ull << j;
        const uint64_t c = (((uint64_t)u + step - 1) >> j) - (((uint64_t)R.start[e] + step - 1) >> j);
        return R.site0[e][c];
    }
    const uint32_t B = rule_bitlen((uint64_t)u + 1);
    const uint32_t e = B - R.first;
    const uint32_t r = R.r[e];
    const uint32_t h = (uint32_t)__builtin_ctzll((uint64_t)u + 1);
    const uint64_t c = ((uint64_t)u + 1) >> (h + 1);
    const uint32_t key = h * r + (uint32_t)(c % r);
    uint32_t s = R.site0[e][key];
    for (uint32_t i = R.ev_begin[e][key]; i < R.ev_begin[e][key + 1]; ++i) {
        if (R.ev_u[i] > u) break;
        s = R.ev_site[i];
    }
    return s;
}

// Item (local time) held by site `site` of a sub-surface after U items
// (0 .. U-1), kRuleEmptyItem if unfilled or site >= m.  The same layout as
// placing every item in turn: steady, the epoch-start layout with the pool's
// first sites holding this epoch's multiples of 2^j and the next one the
// newest item; tilted, the epoch-start assignment of sites to chains moved
// by the epoch's events up to U - 1 (a chain's old site keeps the item it
// held), each chain's site holding its newest item.  O(1) for steady, O(the
// epoch's events) for tilted.
constexpr uint32_t kRuleEmptyItem = 0xffffffffu;

__host__ __device__ inline uint32_t rule_item_at(const RuleTable& R, uint64_t U, uint32_t site) {
    const uint32_t m = R.m;
    if (site >= m) return kRuleEmptyItem;
    if (U <= m) return site < U ? site : kRuleEmptyItem;
    const uint64_t u = U - 1;                        // the newest item
    if (R.policy == 0) {
        const uint32_t j = rule_bitlen(u / (m - 1));
        const uint32_t e = j - R.first;
        const uint64_t step = 1ull << j;
        const uint64_t first = ((uint64_t)R.start[e] + step - 1) >> j;
        const uint64_t cnt = ((u + step - 1) >> j) - first;   // multiples in [E_j, u)
        const uint32_t pos = R.pool_pos[e][site];
        if (pos != kRuleNoSite && pos < cnt) return (uint32_t)((first + pos) << j);
        if (pos != kRuleNoSite && pos == cnt) return (uint32_t)u;
        return R.layout0[e][site];
    }
    const uint32_t B = rule_bitlen(u + 1);
    const uint32_t e = B - R.first;
    const uint32_t r = R.r[e];
    uint32_t key = R.chain_of[e][site];
    uint32_t held = R.layout0[e][site];
    for (uint32_t i = R.evt_begin[e]; i < R.evt_begin[e + 1]; ++i) {
        const uint32_t ue = R.evt_u[i];
        if (ue > u) break;
        const uint32_t k = R.evt_key[i], s = R.evt_site[i];
        if (key == k && site != s) {
            // the chain leaves this site, which keeps the chain's item
            // index c - r (the one the event's item pushed out)
            const uint32_t h = (uint32_t)__builtin_ctzll((uint64_t)ue + 1);
            const uint64_t c = ((uint64_t)ue + 1) >> (h + 1);
            key = kRuleNoSite;
            held = (uint32_t)(((2 * (c - r) + 1) << h) - 1);
        }
        if (site == s) key = k;
    }
    if (key == kRuleNoSite) return held;
    const uint32_t h = key / r, q = key % r;
    const uint64_t cmax = ((U >> h) - 1) / 2;           // newest level-h index below U
    const uint64_t c = cmax - (cmax + r - q) % r;
    return (uint32_t)(((2 * c + 1) << h) - 1);
}

// Site of item tau of a surface of `kind` and S sites: rules[0] is the
// steady or tilted table of a plain surface; a hybrid surface's even items
// go to its steady half (rules[0], local time tau / 2) and its odd items to
// its tilted half (rules[1], local time (tau - 1) / 2, sites S/2 .. S-1).
__host__ __device__ inline uint32_t scheme_site(const RuleTable* rules, uint32_t kind,
                                                uint32_t S, uint32_t tau) {
    if (kind == 2)
        return (tau & 1u) == 0 ? rule_site(rules[0], tau >> 1)
                               : (S >> 1) + rule_site(rules[1], (tau - 1) >> 1);
    return rule_site(rules[0], tau);
}

// Item (in ingest units) held by `site` of a surface of `kind` and S sites
// after tau items, kRuleEmptyItem if unfilled: hybrid sites below S/2 are
// the steady half (even items 2u), the rest the tilted half (odd items
// 2u + 1).
__host__ __device__ inline uint32_t scheme_item_at(const RuleTable* rules, uint32_t kind,
                                                   uint32_t S, uint64_t tau, uint32_t site) {
    if (site >= S) return kRuleEmptyItem;
    if (kind == 2) {
        const uint32_t h = S >> 1;
        if (site < h) {
            const uint32_t v = rule_item_at(rules[0], (tau + 1) >> 1, site);
            return v == kRuleEmptyItem ? v : 2 * v;
        }
        const uint32_t v = rule_item_at(rules[1], tau >> 1, site - h);
        return v == kRuleEmptyItem ? v : 2 * v + 1;
    }
    return rule_item_at(rules[0], tau, site);
}

// Host side.  Tables of (policy, m), built once and cached; NULL when the
// policy or m is invalid.  Thread-safe.
const RuleTable* rule_table(uint32_t policy, uint32_t m);

// Layout of a sub-surface after U items (0 .. U-1): the local item held by
// each of its m sites, kRuleEmpty when unfilled.  U - 1 must lie within the
// tables' range.  O(m + the events of one epoch).
constexpr uint32_t kRuleEmpty = 0xffffffffu;
void rule_layout(uint32_t policy, uint32_t m, uint64_t U, uint32_t* L);

// Last local time the tables cover (the horizon capped at 2^32 - 2).
uint64_t rule_last(uint32_t policy, uint32_t m);

// The tables of a surface of `kind` and S sites in scheme_site's order
// (one for steady or tilted, two for hybrid) into out; false if invalid.
bool scheme_rules(uint32_t kind, uint32_t S, const RuleTable** out);

// Layout of a surface of `kind` and S sites after tau items, in item
// (ingest) units, kRuleEmpty when unfilled: the run's layout form.
void scheme_layout_items(uint32_t kind, uint32_t S, uint64_t tau, uint32_t* L);

}  // namespace hsga
