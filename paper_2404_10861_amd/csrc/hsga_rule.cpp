// hsga_rule.cpp -- host builder of the constant-time site rule tables
// (hsga_rule.hpp), layouts from them, and the host entry points that use
// them: hstrat_layout and hstrat_mrca_bounds_pair (include/hsga.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "hsga_host.hpp"
#include "hsga_rule.hpp"

namespace hsga {

namespace {

uint32_t ctz64(uint64_t x) { return (uint32_t)__builtin_ctzll(x); }

// Item t of level h, index c: t + 1 = (2c + 1) 2^h.
uint64_t level_item(uint32_t h, uint64_t c) { return ((2 * c + 1) << h) - 1; }

// The tables of one sub-surface and the last local time they cover.
struct RuleHost {
    RuleTable t;
    uint64_t last = 0;
    struct Event {
        uint64_t u;
        uint32_t key;
        uint32_t site;
    };
};

uint64_t horizon_local(uint32_t policy, uint32_t m) {
    uint64_t h = 0xfffffffeull;
    if (policy == kTilted && m < 33) h = (1ull << m) - 2;
    return h < 0xfffffffeull ? h : 0xfffffffeull;
}

// Is item t (t < u) in D(u)?  Membership is monotone, so t is in D(u)
// exactly while u is below the local time at which t leaves.
bool retained(uint32_t policy, uint32_t m, uint64_t u, uint64_t t) {
    return u < (uint64_t)leave_time(policy, m, (uint32_t)t);
}

void build_steady(RuleHost& H, uint32_t m) {
    RuleTable& T = H.t;
    std::vector<uint32_t> L(m);
    for (uint32_t k = 0; k < m; ++k) L[k] = k;       // the fill: item k at site k
    uint32_t j = rule_bitlen(m / (m - 1));          // epoch of u = m
    T.first = j;
    for (;; ++j) {
        const uint64_t E = std::max<uint64_t>((uint64_t)(m - 1) << (j - 1), m);
        if (E > H.last) break;
        const uint32_t e = j - T.first;
        T.start[e] = (uint32_t)E;
        std::vector<uint32_t> pool;
        for (uint32_t k = 0; k < m; ++k)
            if (!retained(kSteady, m, E, L[k])) pool.push_back(k);
        for (uint32_t k = 0; k < 64; ++k) {
            T.site0[e][k] = k < pool.size() ? (uint8_t)pool[k] : kRuleNoSite;
            T.layout0[e][k] = k < m ? L[k] : kRuleEmptyItem;
            T.pool_pos[e][k] = kRuleNoSite;
        }
        for (uint32_t k = 0; k < pool.size(); ++k) T.pool_pos[e][pool[k]] = (uint8_t)k;
        T.n_epochs = e + 1;
        // the layout at the next epoch start: the multiples of 2^j of this
        // epoch on the pool's first sites, its last item on the next one
        const uint64_t end = std::min<uint64_t>((uint64_t)(m - 1) << j, H.last + 1);
        const uint64_t step = 1ull << j;
        const uint64_t first = (E + step - 1) >> j;                  // multiples from first * 2^j
        const uint64_t cnt = ((end - 1 + step - 1) >> j) - first;    // those below end - 1
        for (uint64_t k = 0; k < cnt; ++k) L[pool[k]] = (uint32_t)((first + k) << j);
        L[pool[cnt]] = (uint32_t)(end - 1);
    }
}

void build_tilted(RuleHost& H, uint32_t m) {
    RuleTable& T = H.t;
    std::vector<uint64_t> L(m);
    for (uint32_t k = 0; k < m; ++k) L[k] = k;
    uint64_t u = m;
    T.first = rule_bitlen(u + 1);
    uint32_t n_ev = 0;
    while (u <= H.last) {
        const uint32_t B = rule_bitlen(u + 1);
        const uint32_t r = m / B;
        if (r == 0) break;
        const uint32_t e = B - T.first;
        T.start[e] = (uint32_t)u;
        T.r[e] = r;
        T.n_epochs = e + 1;
        // the state at u: each retained item heads its chain (level, index
        // mod r); every other site is free and keeps its item
        uint8_t chain[64];
        std::memset(chain, kRuleNoSite, sizeof chain);
        uint64_t free_mask = 0;
        std::vector<uint32_t> stale(m, 0);
        for (uint32_t k = 0; k < 64; ++k) {
            T.chain_of[e][k] = kRuleNoSite;
            T.layout0[e][k] = k < m ? (uint32_t)L[k] : kRuleEmptyItem;
        }
        for (uint32_t k = 0; k < m; ++k) {
            const uint64_t t = L[k];
            if (retained(kTilted, m, u, t)) {
                const uint32_t h = ctz64(t + 1);
                const uint64_t c = (t + 1) >> (h + 1);
                chain[h * r + (uint32_t)(c % r)] = (uint8_t)k;
                T.chain_of[e][k] = (uint8_t)(h * r + (uint32_t)(c % r));
            } else {
                free_mask |= 1ull << k;
                stale[k] = (uint32_t)t;
            }
        }
        std::memcpy(T.site0[e], chain, sizeof chain);
        std::vector<RuleHost::Event> events;
        const uint64_t u_end = std::min<uint64_t>((1ull << B) - 1, H.last + 1);
        // jump from event to event: between events every item takes its
        // chain's site and nothing else changes
        while (true) {
            const uint32_t g = free_mask ? ctz64(free_mask) : 64u;
            uint64_t best = u_end;
            for (uint32_t h = 0; h < B; ++h) {
                const uint64_t step = 1ull << h;
                const uint64_t c0 = u + 1 >= step ? ((u + 1) - step + 2 * step - 1) >> (h + 1) : 0;
                for (uint32_t q = 0; q < r; ++q) {
                    const uint64_t cq = c0 + (q + r - (uint32_t)(c0 % r)) % r;
                    const uint64_t t = level_item(h, cq);
                    if (t >= best) continue;
                    const uint32_t k = chain[h * r + q];
                    if (k == kRuleNoSite || g < k) best = t;   // a new chain, or a lower free site
                }
            }
            if (best >= u_end) break;
            u = best;
            const uint32_t h = ctz64(u + 1);
            const uint64_t c = (u + 1) >> (h + 1);
            const uint32_t key = h * r + (uint32_t)(c % r);
            uint64_t F = free_mask;
            if (c >= r && chain[key] != kRuleNoSite) {
                F |= 1ull << chain[key];           // its chain's item c - r leaves now
                stale[chain[key]] = (uint32_t)level_item(h, c - r);
            }
            const uint32_t s = ctz64(F);
            free_mask = F & ~(1ull << s);
            chain[key] = (uint8_t)s;
            events.push_back({u, key, s});
            ++u;
        }
        // the layout at the end of the epoch: each chain's newest item
        const uint64_t U = u_end;
        for (uint32_t key = 0; key < B * r; ++key) {
            if (chain[key] == kRuleNoSite) continue;
            const uint32_t h = key / r, q = key % r;
            const uint64_t cmax = ((U >> h) - 1) / 2;     // newest level-h index below U
            L[chain[key]] = level_item(h, cmax - (cmax + r - q) % r);
        }
        for (uint32_t k = 0; k < m; ++k)
            if ((free_mask >> k) & 1) L[k] = stale[k];
        // events grouped by chain for the constant-time lookup, and in time
        // order for layouts
        if (n_ev + events.size() > kRuleEvents) {
            T.n_epochs = 0;                 // more events than the table holds
            return;
        }
        T.evt_begin[e] = (uint16_t)n_ev;
        for (size_t i = 0; i < events.size(); ++i) {
            T.evt_u[n_ev + i] = (uint32_t)events[i].u;
            T.evt_key[n_ev + i] = (uint8_t)events[i].key;
            T.evt_site[n_ev + i] = (uint8_t)events[i].site;
        }
        T.evt_begin[e + 1] = (uint16_t)(n_ev + events.size());
        uint32_t pos = n_ev;
        for (uint32_t key = 0; key <= 64; ++key) {
            T.ev_begin[e][key] = (uint16_t)pos;
            if (key == 64) break;
            for (const auto& ev : events)
                if (ev.key == key) {
                    T.ev_u[pos] = (uint32_t)ev.u;
                    T.ev_site[pos] = (uint8_t)ev.site;
                    ++pos;
                }
        }
        n_ev = pos;
        u = (1ull << B) - 1;
    }
}

std::mutex g_rule_mutex;
std::map<uint64_t, std::unique_ptr<RuleHost>> g_rules;

const RuleHost* rule_host(uint32_t policy, uint32_t m) {
    if ((policy != kSteady && policy != kTilted) || m < 2 || m > 64) return nullptr;
    std::lock_guard<std::mutex> lock(g_rule_mutex);
    const uint64_t key = ((uint64_t)policy << 32) | m;
    auto it = g_rules.find(key);
    if (it != g_rules.end()) return it->second.get();
    auto H = std::make_unique<RuleHost>();
    std::memset(&H->t, 0, sizeof H->t);
    H->t.policy = policy;
    H->t.m = m;
    H->last = horizon_local(policy, m);
    if (policy == kSteady) build_steady(*H, m);
    else build_tilted(*H, m);
    if (H->t.n_epochs == 0) return nullptr;
    const RuleHost* out = H.get();
    g_rules.emplace(key, std::move(H));
    return out;
}

}  // namespace

const RuleTable* rule_table(uint32_t policy, uint32_t m) {
    const RuleHost* H = rule_host(policy, m);
    return H ? &H->t : nullptr;
}

uint64_t rule_last(uint32_t policy, uint32_t m) { return horizon_local(policy, m); }

void rule_layout(uint32_t policy, uint32_t m, uint64_t U, uint32_t* L) {
    const RuleHost* H = rule_host(policy, m);
    for (uint32_t k = 0; k < m; ++k)
        L[k] = H ? rule_item_at(H->t, U, k) : (k < U ? k : kRuleEmpty);
}

bool scheme_rules(uint32_t kind, uint32_t S, const RuleTable** out) {
    if (kind == kHybrid) {
        out[0] = rule_table(kSteady, S / 2);
        out[1] = rule_table(kTilted, S / 2);
        return out[0] && out[1];
    }
    out[0] = rule_table(kind, S);
    return out[0] != nullptr;
}

void scheme_layout_items(uint32_t kind, uint32_t S, uint64_t tau, uint32_t* L) {
    if (kind == kHybrid) {
        const uint32_t h = S / 2;
        uint32_t lo[32] = {}, hi[32] = {};
        rule_layout(kSteady, h, (tau + 1) / 2, lo);
        rule_layout(kTilted, h, tau / 2, hi);
        for (uint32_t k = 0; k < h; ++k) {
            L[k] = lo[k] == kRuleEmpty ? kRuleEmpty : 2 * lo[k];
            L[h + k] = hi[k] == kRuleEmpty ? kRuleEmpty : 2 * hi[k] + 1;
        }
        return;
    }
    rule_layout(kind, S, tau, L);
}

}  // namespace hsga

using namespace hsga_host;

namespace {

// Layout of an annotation of `scheme` with counter T, in deposit
// generations (GA_EMPTY_SITE when unfilled).  GA_EHORIZON past the horizon.
int scheme_layout(const hstrat_scheme& sc, uint32_t T, uint32_t* L) {
    const uint32_t tau = hsga::ingests_of(T, sc.ingest_interval);   // items 0 .. tau - 1
    if (tau > 0 && (uint64_t)(tau - 1) > hsga::horizon_of(sc.kind, sc.sites))
        return fail(GA_EHORIZON, "counter " + std::to_string(T) +
                                     " holds an item past the site rule's horizon");
    const uint32_t S = sc.sites;
    const hsga::RuleTable* rules[2];
    if (!hsga::scheme_rules(sc.kind, S, rules))
        return fail(GA_EINVAL, "no site rule tables for this surface");
    // hybrid: even items on the steady half (local time tau / 2), odd ones
    // on the tilted half (local time (tau - 1) / 2)
    hsga::scheme_layout_items(sc.kind, S, tau, L);
    for (uint32_t k = 0; k < S; ++k)
        if (L[k] != GA_EMPTY_SITE) L[k] *= sc.ingest_interval;
    return GA_OK;
}

int check_host_scheme(const hstrat_scheme* sc) {
    if (!sc) return fail(GA_EINVAL, "scheme is NULL");
    if (sc->kind > GA_HYBRID) return fail(GA_EINVAL, "unknown surface kind");
    if (sc->differentia_bits != 1 && sc->differentia_bits != 8)
        return fail(GA_EINVAL, "differentia_bits must be 1 or 8");
    if (sc->sites * sc->differentia_bits != 32 && sc->sites * sc->differentia_bits != 64)
        return fail(GA_EINVAL, "sites * differentia_bits must be 32 or 64");
    if (sc->ingest_interval == 0) return fail(GA_EINVAL, "ingest_interval must be >= 1");
    return GA_OK;
}

uint32_t site_value(const uint32_t* s, uint32_t k, uint32_t bits) {
    const uint32_t per = 32 / bits;
    const uint32_t mask = bits == 8 ? 0xffu : 1u;
    return (s[k / per] >> ((k % per) * bits)) & mask;
}

}  // namespace

extern "C" {

int hstrat_layout(const hstrat_scheme* scheme, uint32_t T, uint32_t* layout) {
    // a layout does not depend on the differentia width, so any surface of
    // 2..64 sites (hybrid: an even number, at least 4) is accepted here
    if (!scheme) return fail(GA_EINVAL, "scheme is NULL");
    if (scheme->kind > GA_HYBRID) return fail(GA_EINVAL, "unknown surface kind");
    if (scheme->sites < 2 || scheme->sites > 64 ||
        (scheme->kind == GA_HYBRID && (scheme->sites % 2 || scheme->sites < 4)))
        return fail(GA_EINVAL, "sites must be 2..64 (hybrid: even, at least 4)");
    if (scheme->ingest_interval == 0) return fail(GA_EINVAL, "ingest_interval must be >= 1");
    if (!layout) return fail(GA_EINVAL, "layout is NULL");
    return scheme_layout(*scheme, T, layout);
}

int hstrat_sites(const hstrat_scheme* scheme, uint32_t tau0, uint32_t n, uint32_t* sites) {
    if (!scheme) return fail(GA_EINVAL, "scheme is NULL");
    const uint32_t S = scheme->sites;
    if (scheme->kind > GA_HYBRID) return fail(GA_EINVAL, "unknown surface kind");
    if (S < 2 || S > 64 || (scheme->kind == GA_HYBRID && (S % 2 || S < 4)))
        return fail(GA_EINVAL, "sites must be 2..64 (hybrid: even, at least 4)");
    if (n && !sites) return fail(GA_EINVAL, "sites is NULL");
    if (n && (uint64_t)tau0 + n - 1 > hsga::horizon_of(scheme->kind, S))
        return fail(GA_EHORIZON, "an item past the site rule's horizon");
    const hsga::RuleTable* rules[2];
    if (!hsga::scheme_rules(scheme->kind, S, rules))
        return fail(GA_EINVAL, "no site rule tables for this surface");
    // the tables side by side, as a run's device copy holds them
    hsga::RuleTable pair[2];
    pair[0] = *rules[0];
    if (scheme->kind == GA_HYBRID) pair[1] = *rules[1];
    for (uint32_t i = 0; i < n; ++i) sites[i] = hsga::scheme_site(pair, scheme->kind, S, tau0 + i);
    return GA_OK;
}

int hstrat_mrca_bounds_pair_ex(const hstrat_scheme* scheme, uint32_t Ta, const uint32_t* sa,
                               uint32_t Tb, const uint32_t* sb, uint32_t* lb, uint32_t* ub) {
    int rc = check_host_scheme(scheme);
    if (rc != GA_OK) return rc;
    if (!sa || !sb || !lb || !ub) return fail(GA_EINVAL, "NULL argument");
    uint32_t La[64], Lb[64];
    if ((rc = scheme_layout(*scheme, Ta, La)) != GA_OK) return rc;
    if ((rc = scheme_layout(*scheme, Tb, Lb)) != GA_OK) return rc;
    // deposit times held by both, ascending, with their sites in each
    const uint32_t S = scheme->sites;
    struct Common { uint32_t t, ka, kb; };
    Common c[64];
    uint32_t n = 0;
    for (uint32_t x = 0; x < S; ++x) {
        if (La[x] == GA_EMPTY_SITE) continue;
        for (uint32_t y = 0; y < S; ++y)
            if (Lb[y] == La[x]) {
                c[n++] = {La[x], x, y};
                break;
            }
    }
    std::sort(c, c + n, [](const Common& p, const Common& q) { return p.t < q.t; });
    const uint32_t bits = scheme->differentia_bits;
    bool have_last = false;
    uint32_t last = 0;
    for (uint32_t i = 0; i < n; ++i) {
        if (site_value(sa, c[i].ka, bits) != site_value(sb, c[i].kb, bits)) {
            *ub = c[i].t;                              // the first mismatch
            *lb = have_last ? last + 1 : 0;
            return GA_OK;
        }
        have_last = true;
        last = c[i].t;
    }
    *ub = Ta < Tb ? Ta : Tb;
    *lb = have_last ? last + 1 : 0;
    return GA_OK;
}

int hstrat_mrca_bounds_pair(uint32_t kind, uint32_t S, uint32_t Ta, const uint32_t* sa,
                            uint32_t Tb, const uint32_t* sb, uint32_t* lb, uint32_t* ub) {
    if (S != 32 && S != 64) return fail(GA_EINVAL, "S must be 32 or 64");
    const hstrat_scheme sc{kind, S, 1, 1};
    return hstrat_mrca_bounds_pair_ex(&sc, Ta, sa, Tb, sb, lb, ub);
}

}  // extern "C"
