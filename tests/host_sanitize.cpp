// Host-only parts of the library under sanitizers: the site rule's closed
// form (hstrat_layout, hstrat_sites, hstrat_mrca_bounds_pair[_ex]), the
// Newick writer (hstrat_phylo_newick), on valid, edge and invalid inputs,
// and the batched launch's dealing of tiles over the XCDs (deal_tiles,
// checked by replaying the kernel's lookup for every workgroup).
// Built by tests/test_host_sanitize.py twice: with AddressSanitizer and
// UndefinedBehaviorSanitizer (every report fatal), and with
// ThreadSanitizer, where the same calls run from eight threads at once on
// a cold table cache (the tables are built under a lock).  No GPU call is
// made.  The library's error reporting lives with the device API, so this
// file supplies its own.
#include <atomic>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

#include <hip/hip_runtime.h>

#include "../include/hsga.h"
#include "../paper_2404_10861_amd/csrc/hsga_internal.hpp"

namespace hsga_host {
static thread_local std::string g_error;
int fail(int status, const std::string& msg) {
    g_error = msg;
    return status;
}
int hip_fail(hipError_t, const char* what) {
    g_error = what;
    return GA_EDEVICE;
}
const char* last_error() { return g_error.c_str(); }
}  // namespace hsga_host

namespace {

uint64_t g_state = 0x243F6A8885A308D3ull;
thread_local uint64_t t_state = 0;
uint32_t next_word() {
    uint64_t& s = t_state ? t_state : g_state;
    s ^= s << 13;
    s ^= s >> 7;
    s ^= s << 17;
    return (uint32_t)(s >> 32);
}

std::atomic<int> g_failures{0};
void check(bool ok, const char* what, uint32_t a = 0, uint32_t b = 0) {
    if (!ok) {
        std::fprintf(stderr, "FAILED: %s (%u, %u)\n", what, a, b);
        ++g_failures;
    }
}

struct Scheme { uint32_t kind, sites, bits, interval; };

std::vector<Scheme> schemes() {
    std::vector<Scheme> out;
    for (uint32_t kind = 0; kind < 3; ++kind)
        for (uint32_t S : {2u, 3u, 4u, 6u, 8u, 16u, 32u, 48u, 64u}) {
            if (kind == 2 && (S < 4 || S % 2)) continue;
            out.push_back({kind, S, 1, 1});
        }
    out.push_back({2, 8, 8, 2});
    out.push_back({1, 4, 8, 3});
    return out;
}

// Layouts at assorted counts: on success the items are distinct, below the
// count, and fill min(count, S) sites.
void layouts(const Scheme& sc, int draws) {
    const hstrat_scheme h{sc.kind, sc.sites, sc.bits, sc.interval};
    std::vector<uint32_t> L(sc.sites);
    std::vector<uint32_t> Ts = {0, 1, 2, sc.sites - 1, sc.sites, sc.sites + 1, 1000, 65535,
                                1u << 20, 0x7FFFFFFFu, 0xFFFFFFFEu, 0xFFFFFFFFu};
    for (int i = 0; i < draws; ++i) Ts.push_back(next_word() >> (next_word() % 32));
    for (uint32_t T : Ts) {
        const int rc = hstrat_layout(&h, T, L.data());
        check(rc == GA_OK || rc == GA_EHORIZON, "layout status", sc.kind, T);
        if (rc != GA_OK) continue;
        const uint32_t tau = (uint32_t)(((uint64_t)T + sc.interval - 1) / sc.interval);
        uint32_t filled = 0;
        for (uint32_t k = 0; k < sc.sites; ++k) {
            if (L[k] == GA_EMPTY_SITE) continue;
            ++filled;
            check(L[k] / sc.interval < tau && L[k] % sc.interval == 0, "layout item", T, L[k]);
            for (uint32_t j = 0; j < k; ++j) check(L[j] != L[k], "distinct items", T, k);
        }
        check(filled == (tau < sc.sites ? tau : sc.sites), "filled sites", T, filled);
    }
    check(hstrat_layout(&h, 5, nullptr) == GA_EINVAL, "layout NULL");
}

void sites(const Scheme& sc) {
    const hstrat_scheme h{sc.kind, sc.sites, sc.bits, sc.interval};
    std::vector<uint32_t> out(4096);
    for (int i = 0; i < 6; ++i) {
        const uint32_t tau0 = i == 0 ? 0u : next_word() >> (next_word() % 32);
        const uint32_t n = 1 + next_word() % 4096;
        const int rc = hstrat_sites(&h, tau0, n, out.data());
        check(rc == GA_OK || rc == GA_EHORIZON, "sites status", tau0, n);
        if (rc == GA_OK)
            for (uint32_t k = 0; k < n; ++k) check(out[k] < sc.sites, "site range", tau0, k);
    }
    check(hstrat_sites(&h, 0, 4, nullptr) == GA_EINVAL, "sites NULL");
    check(hstrat_sites(&h, 0, 0, nullptr) == GA_OK, "sites empty");
}

void pairs(const Scheme& sc) {
    if (sc.sites * sc.bits != 32 && sc.sites * sc.bits != 64) return;
    const hstrat_scheme h{sc.kind, sc.sites, sc.bits, sc.interval};
    uint32_t a[2], b[2], lb = 0, ub = 0;
    for (int i = 0; i < 40; ++i) {
        a[0] = next_word(); a[1] = next_word();
        b[0] = i % 3 ? next_word() : a[0]; b[1] = i % 2 ? next_word() : a[1];
        const uint32_t Ta = next_word() >> (next_word() % 32);
        const uint32_t Tb = i % 4 ? next_word() >> (next_word() % 32) : Ta;
        const int rc = hstrat_mrca_bounds_pair_ex(&h, Ta, a, Tb, b, &lb, &ub);
        check(rc == GA_OK || rc == GA_EHORIZON, "pair status", Ta, Tb);
        if (rc == GA_OK) check(lb <= ub || ub == 0, "pair order", lb, ub);
    }
    check(hstrat_mrca_bounds_pair_ex(&h, 3, nullptr, 3, b, &lb, &ub) == GA_EINVAL, "pair NULL");
    const hstrat_scheme bad{7, sc.sites, sc.bits, sc.interval};
    check(hstrat_mrca_bounds_pair_ex(&bad, 3, a, 3, b, &lb, &ub) == GA_EINVAL, "pair kind");
}

// Random trees in the reconstruction's form: boundaries 0 .. n-2, a random
// subset of them nodes (the root first), each node's parent an earlier
// node, leaves hanging from nodes; times grow from the root down.
void newick_trees(int count) {
    constexpr uint32_t R = 0xffffffffu, X = 0xfffffffeu;
    std::vector<char> text;
    for (int it = 0; it < count; ++it) {
        const uint32_t n = 1 + next_word() % 200, m = n ? n - 1 : 0;
        std::vector<uint32_t> leaf(n, R), npar(m, X), ntime(m, 0), nodes;
        const uint32_t T = 1000;
        if (n > 1) {
            for (uint32_t b = 0; b < m; ++b)
                if (nodes.empty() || next_word() % 3) nodes.push_back(b);
            for (size_t i = 1; i < nodes.size(); ++i) {
                const size_t j = i - 1 - next_word() % i;   // an earlier node
                const uint32_t v = nodes[i], p = nodes[j];
                npar[v] = p;
                ntime[v] = ntime[p] + next_word() % 5;
            }
            npar[nodes[0]] = R;
            // a leaf under every node that has no child node, the rest anywhere
            std::vector<char> inner(m, 0);
            for (size_t i = 1; i < nodes.size(); ++i) inner[npar[nodes[i]]] = 1;
            uint32_t a = 0;
            for (uint32_t v : nodes)
                if (!inner[v]) leaf[a++] = v;
            for (; a < n; ++a) leaf[a] = nodes[next_word() % nodes.size()];
        }
        size_t len = 0;
        int rc = hstrat_phylo_newick(n, T, leaf.data(), npar.data(), ntime.data(), nullptr, 0,
                                     &len);
        check(rc == GA_OK && len > 0, "newick size", n, (uint32_t)rc);
        if (rc != GA_OK) continue;
        text.assign(len + 1, 'x');
        check(hstrat_phylo_newick(n, T, leaf.data(), npar.data(), ntime.data(), text.data(),
                                  len, &len) == GA_ENOMEM, "newick short buffer", n);
        rc = hstrat_phylo_newick(n, T, leaf.data(), npar.data(), ntime.data(), text.data(),
                                 len + 1, &len);
        check(rc == GA_OK && std::strlen(text.data()) == len && text[len - 1] == ';',
              "newick text", n);
        if (n < 3) continue;
        // broken variants are refused
        std::vector<uint32_t> l2 = leaf, p2 = npar, t2 = ntime;
        l2[next_word() % n] = m + next_word() % 5;                        // out of range
        check(hstrat_phylo_newick(n, T, l2.data(), npar.data(), ntime.data(), nullptr, 0,
                                  &len) == GA_EINVAL, "leaf out of range", n);
        p2[nodes[0]] = nodes.size() > 1 ? nodes[1] : X;                   // no root
        check(hstrat_phylo_newick(n, T, leaf.data(), p2.data(), ntime.data(), nullptr, 0,
                                  &len) == GA_EINVAL, "no root", n);
        if (nodes.size() > 1) {
            t2[nodes[1]] = ntime[npar[nodes[1]]] + T + 1;                  // younger than T
            check(hstrat_phylo_newick(n, T, leaf.data(), npar.data(), t2.data(), nullptr, 0,
                                      &len) == GA_EINVAL, "node time above T", n);
        }
    }
    check(hstrat_phylo_newick(0, 1, nullptr, nullptr, nullptr, nullptr, 0, nullptr) == GA_EINVAL,
          "newick NULL");
}

// Random run sets: every workgroup b of the launch, looked up as the batched
// kernel does (XCD b mod 8, its (b / 8)-th workgroup there), lands on a
// tile of a run, each tile exactly once, and each run's chunks differ in
// size by at most one.
void dealing(int count) {
    constexpr uint32_t X = hsga::kXcds;
    for (int it = 0; it < count; ++it) {
        const uint32_t n = 1 + next_word() % 70;
        std::vector<uint32_t> tiles(n);
        uint32_t T = 0;
        for (uint32_t i = 0; i < n; ++i) {
            const uint32_t kind = next_word() % 4;
            tiles[i] = kind == 0 ? next_word() % 8 : (kind == 1 ? 1 + next_word() % 40
                                                               : 1 + next_word() % 3000);
            T += tiles[i];
        }
        std::vector<uint32_t> tab(2 * X * n, 0xdeadbeefu);
        const bool ok = hsga::deal_tiles(tiles.data(), n, T, tab.data());
        check(ok, "deal status", n, T);
        if (!ok) continue;
        std::vector<uint32_t> base(n + 1, 0);
        for (uint32_t i = 0; i < n; ++i) base[i + 1] = base[i] + tiles[i];
        std::vector<char> seen(T, 0);
        for (uint32_t b = 0; b < T; ++b) {
            const uint32_t x = b % X, j = b / X;
            const uint32_t* pre = tab.data() + x * n;
            uint32_t before = 0;
            for (uint32_t i = 0; i < n; ++i) before += pre[i] <= j;
            check(before >= 1, "deal lookup", b, before);
            if (before < 1) continue;
            const uint32_t lo = before - 1;
            const uint32_t t = tab[(X + x) * n + lo] + (j - pre[lo]);
            check(t < tiles[lo], "deal tile range", lo, t);
            if (t >= tiles[lo]) continue;
            check(!seen[base[lo] + t], "deal tile twice", lo, t);
            seen[base[lo] + t] = 1;
        }
        for (uint32_t k = 0; k < T; ++k) check(seen[k], "deal tile missed", k, T);
        for (uint32_t i = 0; i < n; ++i)
            for (uint32_t x = 0; x < X; ++x) {
                const uint32_t next = i + 1 < n ? tab[x * n + i + 1] : 0xffffffffu;
                check(tab[x * n + i] <= next, "deal offsets ascending", i, x);
                const uint32_t sz = x + 1 < X ? tab[(X + x + 1) * n + i] - tab[(X + x) * n + i]
                                              : tiles[i] - tab[(X + x) * n + i];
                check(sz == tiles[i] / X || sz == tiles[i] / X + 1, "deal chunk size", i, sz);
            }
    }
    uint32_t one = 5, tab[16];
    check(!hsga::deal_tiles(&one, 1, 6, tab), "deal refuses a wrong total");
}

void workload(uint64_t seed, int scale) {
    t_state = seed;
    for (const Scheme& sc : schemes()) {
        layouts(sc, 6 * scale);
        sites(sc);
        pairs(sc);
    }
    newick_trees(20 * scale);
    dealing(30 * scale);
}

}  // namespace

int main() {
#ifdef THREADS
    std::vector<std::thread> pool;
    for (int k = 0; k < 8; ++k)
        pool.emplace_back([k] { workload(0x9E3779B97F4A7C15ull * (k + 1), 1); });
    for (auto& th : pool) th.join();
#else
    workload(0x2545F4914F6CDD1Dull, 4);
#endif
    if (g_failures) return 1;
    std::printf("ok\n");
    return 0;
}
