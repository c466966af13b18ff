/* Host sanitizer driver for the oracle (test infrastructure): calls every
 * entry point of oracle/hsga_oracle.c on small runs of each birth model,
 * annotation scheme, migration setting and asynchronous ticks, then the
 * sample, MRCA-bound and reconstruction queries on the evolved agents and
 * on ragged and degenerate inputs.  tests/test_oracle_sanitize.py builds it
 * with AddressSanitizer and UndefinedBehaviorSanitizer (every report
 * fatal) and runs it; it prints "ok" when every call returned what it
 * should. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

void orc_philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint64_t seed,
                uint32_t out[4]);
uint32_t orc_mulhi(uint32_t w, uint32_t n);
uint64_t orc_horizon(uint32_t kind, uint32_t S);
uint64_t orc_horizon_gen(uint32_t kind, uint32_t S, uint32_t interval);
int orc_place(uint32_t kind, uint32_t S, const uint32_t *L, uint32_t T);
int orc_layout(uint32_t kind, uint32_t S, uint32_t T, uint32_t *L);
int orc_site_sequence(uint32_t kind, uint32_t S, uint32_t T0, uint32_t n, int32_t *sites);
double orc_half_normal(uint32_t w_radius, uint32_t w_angle);
void *orc_create_ex(uint32_t W, uint32_t H, uint32_t N, uint32_t S, uint32_t kind,
                    uint32_t tournament, uint32_t mut_thr, int32_t mut_lo, int32_t mut_hi,
                    uint32_t migrants, uint64_t seed, uint32_t ped_gens, uint32_t bits,
                    uint32_t interval);
int orc_set_fitness(void *h, uint32_t model, uint32_t tournament, uint32_t del_thr,
                    uint32_t ben_thr, float del_sigma, float ben_sigma);
int orc_set_async(void *h, uint32_t activity);
int orc_step(void *h, uint32_t n);
uint32_t orc_generation(void *h);
uint32_t orc_num_agents(void *h);
void orc_read_agents(void *h, uint32_t *trait, uint32_t *counter, uint32_t *surf);
int orc_read_outbox(void *h, uint32_t *dir, uint32_t *trait, uint32_t *counter,
                    uint32_t *surf, uint32_t *src);
void orc_read_layout(void *h, uint32_t *L);
int orc_read_pedigree(void *h, uint32_t gen, uint32_t *parent, uint8_t *bit);
void orc_destroy(void *h);
uint32_t orc_sample(uint64_t seed, uint32_t A, uint32_t n, uint32_t T, uint32_t *idx);
int orc_mrca_pair_x(uint32_t S, uint32_t bits, uint32_t interval, uint32_t Ta,
                    const uint32_t *sa, const uint32_t *La, uint32_t Tb, const uint32_t *sb,
                    const uint32_t *Lb, uint32_t *lb, uint32_t *ub);
int orc_mrca_rows_x(uint32_t kind, uint32_t S, uint32_t bits, uint32_t interval, uint32_t n,
                    const uint32_t *counters, const uint32_t *surf, uint32_t nrows,
                    const uint32_t *rows, uint32_t *lb, uint32_t *ub);
int orc_mrca_allpairs_x(uint32_t kind, uint32_t S, uint32_t bits, uint32_t interval,
                        uint32_t n, const uint32_t *counters, const uint32_t *surf,
                        uint32_t *lb, uint32_t *ub);
int orc_phylo_metrics_x(uint32_t kind, uint32_t S, uint32_t bits, uint32_t interval,
                        uint32_t n, const uint32_t *counters, const uint32_t *surf,
                        uint64_t out[4], double *ed);
long orc_phylo_newick_x(uint32_t kind, uint32_t S, uint32_t bits, uint32_t interval,
                        uint32_t n, const uint32_t *counters, const uint32_t *surf, char *buf,
                        size_t cap);

static int failures = 0;
#define EXPECT(c)                                                          \
    do {                                                                   \
        if (!(c)) {                                                        \
            fprintf(stderr, "%s:%d: expected %s\n", __FILE__, __LINE__, #c); \
            failures++;                                                    \
        }                                                                  \
    } while (0)

static void *xmalloc(size_t n) {
    void *p = malloc(n ? n : 1);
    if (!p) {
        fprintf(stderr, "out of memory\n");
        exit(2);
    }
    return p;
}

/* The queries on n agents (counters, surfaces of W words each); tree = 1:
   the reconstruction must succeed, 0: it must be refused, -1: either. */
static void queries(uint32_t kind, uint32_t S, uint32_t bits, uint32_t interval, uint32_t n,
                    const uint32_t *cnt, const uint32_t *srf, int tree) {
    /* n x n pairs, or 3 rows of n */
    const size_t cells = (size_t)n * (n > 3 ? n : 3);
    uint32_t *lb = xmalloc(cells * 4), *ub = xmalloc(cells * 4);
    EXPECT(orc_mrca_allpairs_x(kind, S, bits, interval, n, cnt, srf, lb, ub) == 0);
    uint32_t rows[3] = {0, n / 2, n - 1};
    EXPECT(orc_mrca_rows_x(kind, S, bits, interval, n, cnt, srf, 3, rows, lb, ub) == 0);
    uint64_t out[4];
    double *ed = xmalloc((size_t)n * sizeof(double));
    int rc = orc_phylo_metrics_x(kind, S, bits, interval, n, cnt, srf, out, ed);
    if (tree >= 0) EXPECT((rc == 0) == (tree == 1));
    size_t cap = 64 * (size_t)n + 64;
    char *buf = xmalloc(cap);
    long len = orc_phylo_newick_x(kind, S, bits, interval, n, cnt, srf, buf, cap);
    if (rc == 0)
        EXPECT(len > 0 && (size_t)len < cap && buf[len - 1] == ';');
    else
        EXPECT(len < 0);
    /* a buffer too small for the shortest tree, "0;", is refused, not overrun */
    if (rc == 0) EXPECT(orc_phylo_newick_x(kind, S, bits, interval, n, cnt, srf, buf, 2) < 0);
    free(buf);
    free(ed);
    free(lb);
    free(ub);
}

struct run_case {
    uint32_t W, H, N, S, kind, tournament, migrants, bits, interval, model, activity, gens;
};

static void one_run(const struct run_case *c, uint64_t seed) {
    const uint32_t ped = c->gens;
    void *h = orc_create_ex(c->W, c->H, c->N, c->S, c->kind, c->model ? 0 : c->tournament,
                            42949672u, -8, 8, c->migrants, seed, ped, c->bits, c->interval);
    EXPECT(h != NULL);
    if (!h) return;
    if (c->model)
        EXPECT(orc_set_fitness(h, c->model, c->tournament, 1417339207u, 128849010u, 0.01f,
                               0.1f) == 0);
    if (c->activity) EXPECT(orc_set_async(h, c->activity) == 0);
    EXPECT(orc_step(h, c->gens / 2) == 0);
    EXPECT(orc_step(h, c->gens - c->gens / 2) == 0);
    EXPECT(orc_step(h, 1) != 0); /* past the recorded pedigree */
    EXPECT(orc_generation(h) == c->gens);
    const uint32_t A = orc_num_agents(h), I = c->W * c->H, SW = c->S * c->bits / 32;
    EXPECT(A == I * c->N);
    uint32_t *tr = xmalloc((size_t)A * 4), *cn = xmalloc((size_t)A * 4);
    uint32_t *sf = xmalloc((size_t)A * SW * 4);
    orc_read_agents(h, tr, cn, sf);
    uint32_t *d = xmalloc((size_t)I * 4), *ot = xmalloc((size_t)I * 4);
    uint32_t *oc = xmalloc((size_t)I * 4), *os = xmalloc((size_t)I * SW * 4);
    uint32_t *src = xmalloc((size_t)I * 4);
    EXPECT(orc_read_outbox(h, d, ot, oc, os, src) == (c->migrants ? 1 : 0));
    uint32_t L[64];
    orc_read_layout(h, L);
    uint32_t *par = xmalloc((size_t)A * 4);
    uint8_t *bit = xmalloc(A);
    for (uint32_t g = 1; g <= c->gens; g++) EXPECT(orc_read_pedigree(h, g, par, bit) == 0);
    EXPECT(orc_read_pedigree(h, 0, par, bit) != 0);
    EXPECT(orc_read_pedigree(h, c->gens + 1, par, bit) != 0);
    for (uint32_t a = 0; a < A; a++) EXPECT(par[a] < A);

    /* a stratified sample, then the queries on it */
    const uint32_t n = A < 77 ? A : 77;
    uint32_t *idx = xmalloc((size_t)n * 4);
    EXPECT(orc_sample(seed, A, n, c->gens, idx) == n);
    uint32_t *scnt = xmalloc((size_t)n * 4), *ssrf = xmalloc((size_t)n * SW * 4);
    for (uint32_t k = 0; k < n; k++) {
        EXPECT(idx[k] < A);
        scnt[k] = cn[idx[k]];
        memcpy(ssrf + (size_t)k * SW, sf + (size_t)idx[k] * SW, SW * 4);
    }
    queries(c->kind, c->S, c->bits, c->interval, n, scnt, ssrf, c->activity ? -1 : 1);
    /* one pair through the pairwise form */
    uint32_t La[64], Lb[64], plb, pub;
    if (orc_layout(c->kind, c->S, (scnt[0] + c->interval - 1) / c->interval, La) == 0 &&
        orc_layout(c->kind, c->S, (scnt[n - 1] + c->interval - 1) / c->interval, Lb) == 0)
        EXPECT(orc_mrca_pair_x(c->S, c->bits, c->interval, scnt[0], ssrf, La, scnt[n - 1],
                               ssrf + (size_t)(n - 1) * SW, Lb, &plb, &pub) == 0);
    free(idx), free(scnt), free(ssrf), free(par), free(bit), free(d), free(ot), free(oc);
    free(os), free(src), free(tr), free(cn), free(sf);
    orc_destroy(h);
}

int main(void) {
    /* Philox, mulhi, half-normal over a spread of words */
    uint32_t out[4];
    for (uint32_t k = 0; k < 1000; k++) {
        orc_philox(k, k * 7u, ~k, k >> 3, 0x123456789abcdefull, out);
        EXPECT(orc_mulhi(out[0], 17) < 17);
        double z = orc_half_normal(out[1], out[2]);
        EXPECT(z >= 0.0 && z < 10.0);
    }
    EXPECT(orc_half_normal(0u, 0u) >= 0.0);
    EXPECT(orc_half_normal(0xffffffffu, 0xffffffffu) >= 0.0);

    /* the site rule: every kind and size, around the fill phase and far out */
    const uint32_t sizes[] = {4, 8, 16, 32, 64};
    for (uint32_t kind = 0; kind < 3; kind++)
        for (int si = 0; si < 5; si++) {
            const uint32_t S = sizes[si];
            const uint64_t hz = orc_horizon(kind, S);
            EXPECT(hz > 0);
            int32_t seq[300];
            EXPECT(orc_site_sequence(kind, S, 0, 300 < hz ? 300 : (uint32_t)hz, seq) == 0);
            uint32_t L[64];
            const uint32_t Ts[] = {0, 1, S - 1, S, S + 1, 1000, 65535};
            for (int t = 0; t < 7; t++) {
                if (Ts[t] > hz) continue;
                EXPECT(orc_layout(kind, S, Ts[t], L) == 0);
                const int site = orc_place(kind, S, L, Ts[t]);
                EXPECT(site >= 0 && site < (int)S);
            }
            for (uint32_t interval = 1; interval <= 7; interval += 3)
                EXPECT(orc_horizon_gen(kind, S, interval) >= hz);
        }

    /* runs: birth models x schemes x migration x asynchronous ticks */
    const struct run_case cases[] = {
        {4, 3, 32, 64, 2, 2, 1, 1, 1, 0, 0, 90},
        {3, 5, 17, 32, 1, 0, 1, 1, 1, 0, 0, 70},
        {1, 1, 1, 32, 0, 2, 1, 1, 1, 0, 0, 40},
        {2, 1, 3, 64, 2, 2, 0, 1, 2, 0, 0, 50},
        {4, 4, 16, 8, 0, 0, 1, 8, 3, 0, 0, 60},
        {3, 3, 32, 4, 1, 0, 1, 8, 1, 0, 0, 15},
        {4, 3, 32, 64, 2, 5, 1, 1, 1, 1, 0, 80},
        {3, 3, 16, 32, 1, 0, 1, 1, 1, 2, 0, 60},
        {5, 4, 16, 64, 2, 2, 1, 1, 2, 0, 0xb3333333u, 120},
        {4, 4, 32, 32, 0, 5, 1, 1, 1, 1, 0x66666666u, 100},
        {3, 2, 8, 8, 1, 0, 0, 8, 1, 2, 0x80000000u, 90},
    };
    for (size_t k = 0; k < sizeof cases / sizeof cases[0]; k++) one_run(&cases[k], 1000 + k);

    /* ragged and degenerate query inputs: one annotation, identical ones,
       counters that differ, counters past the horizon, an invalid scheme */
    uint32_t cnt[65], srf[65 * 2];
    for (uint32_t k = 0; k < 65; k++) {
        cnt[k] = 4000;
        srf[2 * k] = k < 20 ? 0xdeadbeefu : k * 2654435761u;
        srf[2 * k + 1] = k < 20 ? 0x0badf00du : ~k;
    }
    queries(2, 64, 1, 1, 1, cnt, srf, 1);
    queries(2, 64, 1, 1, 2, cnt, srf, 1);
    queries(2, 64, 1, 1, 65, cnt, srf, 1);
    cnt[3] = 17;
    queries(2, 64, 1, 1, 65, cnt, srf, 0); /* mixed counters: bounds, no tree */
    uint64_t o4[4];
    double ed[65];
    uint32_t lb[65 * 65], ub[65 * 65];
    /* tilted, 4 byte sites: items 0 .. 14 are placeable, a counter of 16
       holds item 15 */
    for (uint32_t k = 0; k < 65; k++) cnt[k] = 15;
    EXPECT(orc_phylo_metrics_x(1, 4, 8, 1, 65, cnt, srf, o4, ed) == 0);
    EXPECT(orc_mrca_allpairs_x(1, 4, 8, 1, 65, cnt, srf, lb, ub) == 0);
    for (uint32_t k = 0; k < 65; k++) cnt[k] = k % 2 ? 16 : 0xfffffff0u;
    EXPECT(orc_phylo_metrics_x(1, 4, 8, 1, 65, cnt, srf, o4, ed) != 0);
    EXPECT(orc_mrca_allpairs_x(1, 4, 8, 1, 65, cnt, srf, lb, ub) != 0);
    EXPECT(orc_mrca_allpairs_x(0, 48, 1, 1, 2, cnt, srf, lb, ub) != 0);
    EXPECT(orc_create_ex(0, 1, 1, 32, 0, 0, 0, 0, 0, 1, 1, 0, 1, 1) == NULL);
    EXPECT(orc_create_ex(1, 1, 65, 32, 0, 0, 0, 0, 0, 1, 1, 0, 1, 1) == NULL);

    if (failures) {
        fprintf(stderr, "%d failed expectations\n", failures);
        return 1;
    }
    printf("ok\n");
    return 0;
}
