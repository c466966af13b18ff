/*
 * hsga_oracle.c -- plain, slow, single-threaded CPU oracle for the island-model
 * genetic algorithm with hereditary-stratigraphy surface annotations
 * (Moreno et al., "Trackable Agent-based Evolution Models at Wafer Scale").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls, links or
 * loads this file.  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load it.  It shares no code, header, table or
 * helper with the HIP implementation; both sides implement the Philox4x32-10
 * generator separately from its published definition.
 *
 * The integer treatments are integer arithmetic throughout.  The float
 * treatments (Results, On-hardware Trial) use a binary32 fitness and a
 * half-normal draw evaluated in binary64 by one fixed sequence of correctly
 * rounded operations (orc_half_normal), so the HIP path must agree bit for
 * bit there too.
 *
 * Where the paper is silent (it leaves the steady and tilted indexing
 * algorithms undefined, and gives no random-number mapping), this file follows
 * one fixed reading, stated at each function.  Under that reading:
 *
 *   - Philox4x32-10 is pinned by known answers from an independent library
 *     implementation.
 *   - The site rule is pinned by brute force against the retention criteria
 *     that the paper states in words (Methods, "Distributed Phylogenetic
 *     Tracking" and "Surface-based Hereditary Stratigraphy Algorithms").
 *   - The GA step has no closed form and no paper run to compare with:
 *     "parity unpinned" against the paper.  It is pinned by special cases,
 *     invariants and the pedigree.
 *   - The MRCA bounds are pinned against the true pedigree on tiny runs.
 *
 * Build:  gcc -O2 -std=c11 -ffp-contract=off -pthread -shared -fPIC -o liboracle.so
 *         hsga_oracle.c -lm
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_EMPTY 0xffffffffu

/* surface kinds (policies) */
enum { ORC_STEADY = 0, ORC_TILTED = 1, ORC_HYBRID = 2 };
/* purpose tags carried in the fourth Philox counter word */
enum { ORC_BIRTH = 0, ORC_EMIGRATE = 1, ORC_IMMIGRATE = 2, ORC_SAMPLE = 3,
       ORC_BIRTH_B = 4 /* second block of a float-treatment birth */,
       ORC_FOUNDER = 5 /* founder tags */,
       ORC_ACTIVITY = 6 /* asynchronous runs: is an island active on a tick */ };
/* fitness models */
enum { ORC_INT_TRAIT = 0, ORC_FLOAT_FITNESS = 1, ORC_FOUNDER_TAG = 2 };
/* torus directions */
enum { ORC_NORTH = 0, ORC_SOUTH = 1, ORC_WEST = 2, ORC_EAST = 3 };

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11, "Parallel random numbers:
 * as easy as 1, 2, 3").  Ten rounds; each round multiplies counter words 0
 * and 2 by the two Philox constants, then permutes and mixes in the key; the
 * key is bumped by the two Weyl constants between rounds.                    */
void orc_philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                uint64_t seed, uint32_t out[4])
{
    uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    for (int round = 0; round < 10; round++) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)p0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Map a 32-bit word onto [0, n): the high word of w * n. */
uint32_t orc_mulhi(uint32_t w, uint32_t n)
{
    return (uint32_t)(((uint64_t)w * n) >> 32);
}

static unsigned bitlen64(uint64_t x)
{
    unsigned b = 0;
    while (x) { b++; x >>= 1; }
    return b;
}

static unsigned ctz64(uint64_t x)
{
    unsigned c = 0;
    while (!(x & 1)) { c++; x >>= 1; }
    return c;
}

/* ------------------------------------------------------------------------ */
/* Retention target D(u) of one sub-surface with m sites at local time u,
 * i.e. when item u is being deposited.  Returns 1 when item t (t <= u) is
 * in D(u).
 *
 * Steady policy ("retained time points distributed evenly across history",
 * Methods, Distributed Phylogenetic Tracking): keep every multiple of the
 * spacing g(u) = 2^bitlen(floor(u / (m-1))), plus u itself.
 *
 * Tilted policy ("more recent time points are preferred", same passage): item
 * t sits on level h = ctz(t+1), i.e. t+1 = (2c+1) * 2^h.  Level h holds
 * n_h(u) = (u + 1 + 2^h) >> (h+1) items up to u.  Keep the r = floor(m / B)
 * most recent items of each level, B = bitlen(u+1) being the number of
 * levels present.                                                           */
int orc_in_D(uint32_t policy, uint32_t m, uint64_t u, uint64_t t)
{
    if (t > u)
        return 0;
    if (policy == ORC_STEADY) {
        uint64_t q = u / (m - 1);
        uint64_t spacing = (uint64_t)1 << bitlen64(q);
        return (t % spacing == 0) || (t == u);
    } else {
        unsigned B = bitlen64(u + 1);
        uint64_t r = m / B;
        unsigned h = ctz64(t + 1);
        uint64_t c = (t + 1) >> (h + 1);
        uint64_t n_h = (u + 1 + ((uint64_t)1 << h)) >> (h + 1);
        return c + r >= n_h;
    }
}

/* Which sub-surface item T goes to, its local time and its first site.
 * Steady and tilted kinds use one sub-surface of S sites with u = T.  The
 * hybrid kind gives half of the sites to each policy (same passage): sites
 * [0, S/2) take the even T with u = T/2 under the steady policy; sites
 * [S/2, S) take the odd T with u = (T-1)/2 under the tilted policy.          */
static void sub_surface(uint32_t kind, uint32_t S, uint64_t T,
                        uint32_t *policy, uint32_t *m, uint64_t *u,
                        uint32_t *offset)
{
    if (kind == ORC_HYBRID) {
        *m = S / 2;
        if (T % 2 == 0) {
            *policy = ORC_STEADY; *u = T / 2; *offset = 0;
        } else {
            *policy = ORC_TILTED; *u = (T - 1) / 2; *offset = S / 2;
        }
    } else {
        *policy = kind; *m = S; *u = T; *offset = 0;
    }
}

/* Local time of the item stored (as a global deposit time) at a site. */
static uint64_t local_time(uint32_t kind, uint32_t t_global)
{
    return kind == ORC_HYBRID ? (uint64_t)(t_global / 2) : (uint64_t)t_global;
}

/* Last deposit time T that the rule can place (inclusive).  Tilted needs
 * r >= 1, i.e. bitlen(u+1) <= m, i.e. u <= 2^m - 2; the 32-bit generation
 * counter caps every kind at T <= 2^32 - 2 (the child counter is T+1).     */
uint64_t orc_horizon(uint32_t kind, uint32_t S)
{
    uint64_t cap = 0xfffffffeull;
    uint64_t h = cap;
    if (kind == ORC_TILTED) {
        if (S < 33)
            h = ((uint64_t)1 << S) - 2;
    } else if (kind == ORC_HYBRID) {
        uint32_t m = S / 2;
        if (m < 33) {
            uint64_t umax = ((uint64_t)1 << m) - 2;   /* last tilted local time */
            h = 2 * umax + 2;                          /* next odd T is out     */
        }
    }
    return h < cap ? h : cap;
}

/* Surface placement (Methods, Surface-based Hereditary Stratigraphy
 * Algorithms): a fixed-width buffer, items stay where they are written until
 * overwritten, pruning happens by overwrite.  Reading: while the sub-surface
 * is filling (u < m) item u goes to its own site u; afterwards it goes to the
 * lowest site whose item has left D(u).  L holds global deposit times.
 * Returns the site, or -1 for an item past the horizon (the retention
 * target is not defined there) or if no site is evictable.                 */
int orc_place(uint32_t kind, uint32_t S, const uint32_t *L, uint32_t T)
{
    uint32_t policy, m, offset;
    uint64_t u;
    if ((uint64_t)T > orc_horizon(kind, S))
        return -1;
    sub_surface(kind, S, T, &policy, &m, &u, &offset);
    if (u < m)
        return (int)(offset + u);
    for (uint32_t k = 0; k < m; k++) {
        uint32_t tg = L[offset + k];
        if (tg == ORC_EMPTY)
            return (int)(offset + k);
        if (!orc_in_D(policy, m, u, local_time(kind, tg)))
            return (int)(offset + k);
    }
    return -1;
}

/* Layout after T ingests (items 0..T-1), by replaying the placements from an
 * empty surface.  Timestamps are not stored: they follow from the site index
 * and the elapsed generation count alone (Methods, Distributed Phylogenetic
 * Tracking).  Returns 0, or -1 beyond the horizon.                          */
int orc_layout(uint32_t kind, uint32_t S, uint32_t T, uint32_t *L)
{
    for (uint32_t k = 0; k < S; k++)
        L[k] = ORC_EMPTY;
    if ((uint64_t)T > orc_horizon(kind, S) + 1)   /* item T - 1 past the horizon */
        return -1;
    for (uint64_t t = 0; t < T; t++) {
        int site = orc_place(kind, S, L, (uint32_t)t);
        if (site < 0)
            return -1;
        L[site] = (uint32_t)t;
    }
    return 0;
}

/* Sites chosen for items T0 .. T0+n-1, replaying from empty. */
int orc_site_sequence(uint32_t kind, uint32_t S, uint32_t T0, uint32_t n,
                      int32_t *sites)
{
    uint32_t L[64];
    if (S > 64 || orc_layout(kind, S, T0, L) != 0)
        return -1;
    for (uint32_t j = 0; j < n; j++) {
        int site = orc_place(kind, S, L, T0 + j);
        sites[j] = site;
        if (site < 0)
            return -1;
        L[site] = T0 + j;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* ------------------------------------------------------------------------ */
/* Half-normal draw for the float treatments (Results, On-hardware Trial:
 * mutations change fitness by normally distributed amounts).  Box and
 * Muller (1958): with U1, U2 independent uniform on (0, 1),
 * Z = sqrt(-2 ln U1) cos(2 pi U2) is standard normal; its magnitude has the
 * law of sqrt(-2 ln U1) cos(pi/2 U2), which is what is evaluated here:
 *   U1 = (w_radius + 1/2) / 2^32,  U2 = (w_angle + 1/2) / 2^32.
 * The value is DEFINED as the following binary64 evaluation, written only
 * with correctly rounded operations (+, -, *, fma) and exact scalings by
 * powers of two, so that any IEEE-754 implementation of the same steps
 * returns the same bits:
 *   ln U1:  U1 = m 2^(e-33), m in [sqrt(1/2), sqrt(2)];
 *           ln m = 2 atanh(s), s = (m-1)/(m+1), the reciprocal by five
 *           Newton steps from 1/2, atanh by its series to s^21;
 *   sqrt:   y = q 4^k, q in [1, 4); 1/sqrt(q) by six Newton steps from
 *           9/8 - 3q/16, then one correction of q * (1/sqrt q);
 *   cos:    for U2 < 1/2, cos(pi/2 U2) by its series to x^18; otherwise
 *           sin(pi/2 (1 - U2)) by its series to x^19.
 * Against the exact function the relative error is below 1e-14.          */
static double orc_pow2(int k)          /* 2^k, exact, |k| < 1000 */
{
    return ldexp(1.0, k);
}

static double orc_ln_u(uint32_t w)
{
    uint64_t v = 2ull * w + 1ull;      /* U = v / 2^33, v odd */
    int e = 0;
    while ((v >> (e + 1)) != 0)
        e++;                           /* e = floor(log2 v) */
    double m = (double)v * orc_pow2(-e);
    if (m > 1.4142135623730951) {
        m = m * 0.5;
        e = e + 1;
    }
    double d = m + 1.0, r = 0.5;
    for (int k = 0; k < 5; k++) {
        double t = fma(-d, r, 1.0);
        r = fma(r, t, r);
    }
    double sv = (m - 1.0) * r;
    double z = sv * sv;
    static const double inv_odd[11] = {
        1.0, 1.0 / 3.0, 1.0 / 5.0, 1.0 / 7.0, 1.0 / 9.0, 1.0 / 11.0,
        1.0 / 13.0, 1.0 / 15.0, 1.0 / 17.0, 1.0 / 19.0, 1.0 / 21.0};
    double p = inv_odd[10];
    for (int k = 9; k >= 0; k--)
        p = fma(p, z, inv_odd[k]);
    double ln_m = (sv + sv) * p;
    return fma((double)e - 33.0, 0.6931471805599453, ln_m);
}

static double orc_sqrt_pos(double y)   /* y > 0, normal */
{
    int ex;
    (void)frexp(y, &ex);               /* y = f 2^ex, f in [1/2, 1) */
    ex -= 1;                           /* y = f' 2^ex, f' in [1, 2) */
    int k = (ex >= 0) ? ex / 2 : -((1 - ex) / 2);   /* floor(ex / 2) */
    double q = y * orc_pow2(-2 * k);   /* in [1, 4) */
    double h = 0.5 * q;
    double r = fma(-0.1875, q, 1.125);
    for (int i = 0; i < 6; i++)
        r = fma(r, fma(-h, r * r, 0.5), r);
    double sq = q * r;
    sq = fma(fma(-sq, sq, q), 0.5 * r, sq);
    return sq * orc_pow2(k);
}

static double orc_cos_quarter(uint32_t w)   /* cos(pi/2 U2) */
{
    static const double cos_c[10] = {
        1.0, -1.0 / 2.0, 1.0 / 24.0, -1.0 / 720.0, 1.0 / 40320.0,
        -1.0 / 3628800.0, 1.0 / 479001600.0, -1.0 / 87178291200.0,
        1.0 / 20922789888000.0, -1.0 / 6402373705728000.0};
    static const double sin_c[10] = {
        1.0, -1.0 / 6.0, 1.0 / 120.0, -1.0 / 5040.0, 1.0 / 362880.0,
        -1.0 / 39916800.0, 1.0 / 6227020800.0, -1.0 / 1307674368000.0,
        1.0 / 355687428096000.0, -1.0 / 121645100408832000.0};
    uint64_t v = 2ull * w + 1ull;      /* U2 = v / 2^33 */
    int use_sin = w >= 0x80000000u;
    if (use_sin)
        v = (1ull << 33) - v;          /* 1 - U2, exact */
    double x = ((double)v * orc_pow2(-33)) * 1.5707963267948966;
    double z = x * x;
    const double *c = use_sin ? sin_c : cos_c;
    double p = c[9];
    for (int k = 8; k >= 0; k--)
        p = fma(p, z, c[k]);
    return use_sin ? x * p : p;
}

double orc_half_normal(uint32_t w_radius, uint32_t w_angle)
{
    double y = -2.0 * orc_ln_u(w_radius);
    return orc_sqrt_pos(y) * orc_cos_quarter(w_angle);
}

static uint32_t f32_bits(float f)
{
    uint32_t u;
    memcpy(&u, &f, 4);
    return u;
}

static float f32_of(uint32_t u)
{
    float f;
    memcpy(&f, &u, 4);
    return f;
}

/* The island-model GA (Methods, Asynchronous Island-model Genetic Algorithm;
 * Genome Model).  Islands sit on a W x H torus, island i = y*W + x, agent
 * a = i*N + j.  An agent record is (trait, generation counter, S one-bit
 * differentia sites); site k is bit k&31 of surface word k>>5.              */
/* One island's members during a step (after immigration): N records. */
typedef struct {
    uint32_t *trait, *counter, *surf, *src;
} orc_island;

typedef struct {
    uint32_t W, H, N, S, kind, tournament, mut_thr, mut_span, migrants;
    int32_t mut_lo;
    uint64_t seed;
    /* float treatments and founder tags (orc_set_fitness) */
    uint32_t model, del_thr, ben_thr;
    float del_sigma, ben_sigma;
    /* annotation scheme: differentia width (1 or 8 bits per site) and the
     * ingest interval (one deposit every `interval` generations)          */
    uint32_t bits, interval;
    /* asynchronous runs (orc_set_async): activity threshold (0: every
     * island every step), the site of every ingest so far (tab, filled
     * entries, capacity) and the layout after them (Ltab)                 */
    uint32_t activity;
    uint32_t *tab, tab_filled, tab_cap;
    uint32_t Ltab[64];
    uint32_t I, A, SW;
    uint32_t g;                       /* generations elapsed                  */
    uint32_t *trait, *counter, *surf; /* A, A, A*SW (agent-major)             */
    uint32_t *src;                    /* pedigree: P_g index of each agent     */
    int has_outbox;                   /* O_g exists (g > 0 and migration on)   */
    uint32_t *ob_dir, *ob_trait, *ob_counter, *ob_surf, *ob_src;
    uint32_t L[64];                   /* run layout L_g (global times)         */
    /* optional pedigree: for generations 1..ped_gens, parent index in the
       previous generation and the differentia bit drawn at birth            */
    uint32_t ped_gens;
    uint32_t *ped_parent;             /* (ped_gens) * A                        */
    uint8_t *ped_bit;                 /* (ped_gens) * A                        */
    /* scratch: one island's members (q; one per thread when threaded) and
     * the next population (n_*)                                           */
    orc_island q;
    uint32_t threads;                 /* island-parallel threads (0, 1: none) */
    orc_island *tq;                   /* threads x island scratch             */
    uint32_t *n_trait, *n_counter, *n_surf, *n_src;
} orc_run;

static uint32_t neighbour(const orc_run *r, uint32_t i, uint32_t d)
{
    uint32_t x = i % r->W, y = i / r->W;
    switch (d) {
    case ORC_NORTH: y = (y + r->H - 1) % r->H; break;
    case ORC_SOUTH: y = (y + 1) % r->H; break;
    case ORC_WEST:  x = (x + r->W - 1) % r->W; break;
    default:        x = (x + 1) % r->W; break;
    }
    return y * r->W + x;
}

static uint32_t opposite(uint32_t d)
{
    return d ^ 1u;   /* north<->south, west<->east */
}

static int island_alloc(orc_island *q, uint32_t N, uint32_t SW)
{
    q->trait = calloc(N, 4); q->counter = calloc(N, 4);
    q->surf = calloc((size_t)N * SW, 4); q->src = calloc(N, 4);
    return q->trait && q->counter && q->surf && q->src;
}

static void island_free(orc_island *q)
{
    free(q->trait); free(q->counter); free(q->surf); free(q->src);
    q->trait = q->counter = q->surf = q->src = NULL;
}

void orc_destroy(void *handle)
{
    orc_run *r = (orc_run *)handle;
    if (!r)
        return;
    free(r->trait); free(r->counter); free(r->surf); free(r->src);
    free(r->ob_dir); free(r->ob_trait); free(r->ob_counter); free(r->ob_surf);
    free(r->ob_src);
    free(r->tab);
    free(r->ped_parent); free(r->ped_bit);
    island_free(&r->q);
    if (r->tq)
        for (uint32_t k = 0; k < r->threads; k++)
            island_free(&r->tq[k]);
    free(r->tq);
    free(r->n_trait); free(r->n_counter); free(r->n_surf); free(r->n_src);
    free(r);
}

/* Founders (generation 0): trait 0, counter 0, empty surface; no outboxes.
 * Founders carry no differentia: item t is deposited at the birth of the
 * generation-(t+1) individual (Distributed Phylogenetic Tracking: offspring
 * receive a new differentia on birth).  Returns NULL on an invalid config.  */
/* Annotation schemes: S sites of `bits` bits each (one-bit or byte
 * differentiae, Distributed Phylogenetic Tracking: differentia width trades
 * collisions for coverage), filling one or two 32-bit words, deposited
 * every `interval` generations (Results, Surface Algorithm Benchmark:
 * annotations may be updated only every n-th generation).                  */
static int scheme_ok(uint32_t S, uint32_t bits, uint32_t interval)
{
    if (interval == 0 || (bits != 1 && bits != 8))
        return 0;
    return S * bits == 32 || S * bits == 64;
}

/* Ingests made by an annotation with counter T: items at generations
 * 0, interval, 2 interval, ... below T.                                    */
static uint32_t ingests_of(uint32_t T, uint32_t interval)
{
    return (uint32_t)(((uint64_t)T + interval - 1) / interval);
}

/* Last generation that a run can step (inclusive): the next ingest after it
 * would be past the site rule's horizon, or the counter would overflow.   */
uint64_t orc_horizon_gen(uint32_t kind, uint32_t S, uint32_t interval)
{
    uint64_t h = orc_horizon(kind, S);
    uint64_t g = (h + 1) * (uint64_t)interval - 1;
    return g < 0xfffffffeull ? g : 0xfffffffeull;
}

void *orc_create_ex(uint32_t W, uint32_t H, uint32_t N, uint32_t S, uint32_t kind,
                    uint32_t tournament, uint32_t mut_thr, int32_t mut_lo,
                    int32_t mut_hi, uint32_t migrants, uint64_t seed,
                    uint32_t ped_gens, uint32_t bits, uint32_t interval)
{
    if (W == 0 || H == 0 || N == 0 || N > 64 || !scheme_ok(S, bits, interval) ||
        kind > ORC_HYBRID || (tournament != 0 && tournament != 2) ||
        mut_lo > mut_hi || (int64_t)mut_hi - mut_lo + 1 > 0xffffffffll ||
        migrants > 1)
        return NULL;
    orc_run *r = (orc_run *)calloc(1, sizeof(orc_run));
    r->W = W; r->H = H; r->N = N; r->S = S; r->kind = kind;
    r->bits = bits; r->interval = interval;
    r->tournament = tournament; r->mut_thr = mut_thr; r->mut_lo = mut_lo;
    r->mut_span = (uint32_t)((int64_t)mut_hi - mut_lo + 1);
    r->migrants = migrants; r->seed = seed;
    r->I = W * H; r->A = r->I * N; r->SW = S * bits / 32;
    size_t A = r->A, I = r->I, SW = r->SW;
    r->trait = calloc(A, 4); r->counter = calloc(A, 4);
    r->surf = calloc(A * SW, 4); r->src = calloc(A, 4);
    r->ob_dir = calloc(I, 4); r->ob_trait = calloc(I, 4);
    r->ob_counter = calloc(I, 4); r->ob_surf = calloc(I * SW, 4);
    r->ob_src = calloc(I, 4);
    int q_ok = island_alloc(&r->q, N, (uint32_t)SW);
    r->n_trait = calloc(A, 4); r->n_counter = calloc(A, 4);
    r->n_surf = calloc(A * SW, 4); r->n_src = calloc(A, 4);
    if (!r->trait || !r->counter || !r->surf || !r->src || !r->ob_dir ||
        !r->ob_trait || !r->ob_counter || !r->ob_surf || !r->ob_src ||
        !q_ok ||
        !r->n_trait || !r->n_counter || !r->n_surf || !r->n_src) {
        orc_destroy(r);
        return NULL;
    }
    r->ped_gens = ped_gens;
    if (ped_gens) {
        r->ped_parent = calloc((size_t)ped_gens * A, 4);
        r->ped_bit = calloc((size_t)ped_gens * A, 1);
        if (!r->ped_parent || !r->ped_bit) {
            orc_destroy(r);
            return NULL;
        }
    }
    for (uint32_t a = 0; a < r->A; a++)
        r->src[a] = a;
    for (uint32_t k = 0; k < 64; k++)
        r->L[k] = r->Ltab[k] = ORC_EMPTY;
    r->g = 0;
    r->has_outbox = 0;
    return r;
}

void *orc_create(uint32_t W, uint32_t H, uint32_t N, uint32_t S, uint32_t kind,
                 uint32_t tournament, uint32_t mut_thr, int32_t mut_lo,
                 int32_t mut_hi, uint32_t migrants, uint64_t seed,
                 uint32_t ped_gens)
{
    if (S != 32 && S != 64)
        return NULL;
    return orc_create_ex(W, H, N, S, kind, tournament, mut_thr, mut_lo, mut_hi,
                         migrants, seed, ped_gens, 1, 1);
}

/* Float treatments (Results, On-hardware Trial; Asynchronous Island-model
 * Genetic Algorithm).  model 1: the trait word is a binary32 fitness
 * (founders 0.0); selection is a tournament of `tournament` uniform draws
 * with replacement (0 or 1: one draw, neutral), the first draw of maximal
 * fitness winning, so ties go to a uniformly random tied individual; a
 * birth is deleterious with probability del_thr / 2^32 (fitness decreases
 * by del_sigma |Z|) or beneficial with probability ben_thr / 2^32 (fitness
 * increases by ben_sigma |Z|), never both; the sum and product are taken in
 * binary64 and rounded once to binary32.  Returns 0, or -1 if invalid.    */
int orc_set_fitness(void *handle, uint32_t model, uint32_t tournament,
                    uint32_t del_thr, uint32_t ben_thr, float del_sigma,
                    float ben_sigma)
{
    orc_run *r = (orc_run *)handle;
    if (model > ORC_FOUNDER_TAG || r->g != 0)
        return -1;
    if (model == ORC_FLOAT_FITNESS) {
        if (tournament > 5 || (uint64_t)del_thr + ben_thr > (1ull << 32) ||
            !(del_sigma >= 0.0f && del_sigma <= 1048576.0f) ||
            !(ben_sigma >= 0.0f && ben_sigma <= 1048576.0f))
            return -1;
    } else if (model == ORC_FOUNDER_TAG) {
        if (tournament != 0)
            return -1;
    } else if (tournament != 0 && tournament != 2) {
        return -1;
    }
    r->model = model;
    r->tournament = tournament;
    r->del_thr = del_thr;
    r->ben_thr = ben_thr;
    r->del_sigma = del_sigma;
    r->ben_sigma = ben_sigma;
    /* Founder tags (Genome Model; Results, Clade Reconstruction Trial): each
     * founder's trait word is a random 16-bit identifier, inherited without
     * mutation under neutral selection.  Tag of agent a: the low 16 bits of
     * the first word of Philox block (a, 0, 0, FOUNDER).                    */
    for (uint32_t a = 0; a < r->A; a++) {
        uint32_t w[4];
        orc_philox(a, 0, 0, ORC_FOUNDER, r->seed, w);
        r->trait[a] = model == ORC_FOUNDER_TAG ? (w[0] & 0xffffu) : 0u;
    }
    return 0;
}

/* Selection, replication and mutation of the birth into slot j of island i
 * at step g (the step index is the generation in synchronous runs and the
 * tick in asynchronous ones), reading the island's members Q: the parent's
 * index in Q, the child's trait word and the differentia drawn (the low
 * `bits` bits of the drawn word).                                          */
static void draw_birth(const orc_run *r, const orc_island *q, uint32_t i, uint32_t j,
                       uint32_t g, uint32_t *p_out, uint32_t *trait_out, uint32_t *val_out)
{
    const uint32_t N = r->N;
    uint32_t w[4], p, child_trait, bit;
    orc_philox(j, i, g, ORC_BIRTH, r->seed, w);
    if (r->model == ORC_FOUNDER_TAG) {
        /* neutral; the tag is inherited unchanged */
        p = orc_mulhi(w[0], N);
        child_trait = q->trait[p];
        bit = w[3];
    } else if (r->model == ORC_INT_TRAIT) {
        p = orc_mulhi(w[0], N);
        if (r->tournament == 2) {
            uint32_t b = orc_mulhi(w[1], N);
            if ((int32_t)q->trait[b] > (int32_t)q->trait[p])
                p = b;
        }
        uint32_t delta = 0;
        if (w[2] < r->mut_thr)
            delta = (uint32_t)((int32_t)orc_mulhi(w[3], r->mut_span) + r->mut_lo);
        child_trait = q->trait[p] + delta;
        bit = w[3];
    } else {
        /* float treatments: candidates from words w0..w3, v0; the
         * class of the mutation from v1; |Z| from v2 (radius) and
         * v3 (angle); the differentia is the low bits of v3     */
        uint32_t v[4];
        orc_philox(j, i, g, ORC_BIRTH_B, r->seed, v);
        uint32_t words[5] = {w[0], w[1], w[2], w[3], v[0]};
        uint32_t k = r->tournament < 1 ? 1 : r->tournament;
        p = orc_mulhi(words[0], N);
        for (uint32_t c = 1; c < k; c++) {
            uint32_t b = orc_mulhi(words[c], N);
            if (f32_of(q->trait[b]) > f32_of(q->trait[p]))
                p = b;
        }
        double f = (double)f32_of(q->trait[p]);
        child_trait = q->trait[p];
        if (v[1] < r->del_thr)
            child_trait = f32_bits((float)(f - (double)r->del_sigma *
                                                  orc_half_normal(v[2], v[3])));
        else if ((uint64_t)v[1] + r->ben_thr >= (1ull << 32))
            child_trait = f32_bits((float)(f + (double)r->ben_sigma *
                                                  orc_half_normal(v[2], v[3])));
        bit = v[3];
    }
    *p_out = p;
    *trait_out = child_trait;
    *val_out = bit & (r->bits == 8 ? 0xffu : 1u);
}

/* Island i of generation g: its members of P_g (and the immigrants
 * addressed to it) into the scratch q, then its N births into the next
 * population (n_*).  Reads only P_g and O_g, writes only island i's slots
 * of the next population and of the pedigree, so islands are independent
 * within a generation.  Returns 0, or -2 on a broken invariant.           */
static int breed_island(orc_run *r, orc_island *q, uint32_t i, uint32_t g, int site,
                        int ingest)
{
    const uint32_t N = r->N, SW = r->SW;
    uint32_t w[4];
    /* Q := this island's members of P_g */
    for (uint32_t j = 0; j < N; j++) {
        uint32_t a = i * N + j;
        q->trait[j] = r->trait[a];
        q->counter[j] = r->counter[a];
        for (uint32_t s = 0; s < SW; s++)
            q->surf[j * SW + s] = r->surf[(size_t)a * SW + s];
        q->src[j] = a;
    }

    /* Immigration: each neighbour's emigrant that was sent our way
     * replaces a randomly chosen member; applied north, south, west,
     * east.  Genomes are copied, not moved.                             */
    if (r->migrants && r->has_outbox) {
        orc_philox(0, i, g, ORC_IMMIGRATE, r->seed, w);
        for (uint32_t d = 0; d < 4; d++) {
            uint32_t nb = neighbour(r, i, d);
            if (r->ob_dir[nb] == opposite(d)) {
                uint32_t slot = orc_mulhi(w[d], N);
                q->trait[slot] = r->ob_trait[nb];
                q->counter[slot] = r->ob_counter[nb];
                for (uint32_t s = 0; s < SW; s++)
                    q->surf[slot * SW + s] = r->ob_surf[(size_t)nb * SW + s];
                q->src[slot] = r->ob_src[nb];
            }
        }
    }

    /* Births: each slot of the next generation gets a parent by
     * tournament selection (the higher trait of two uniform draws; a tie
     * keeps the first draw) or, when neutral, by one uniform draw; the
     * child copies the parent's record, mutates its trait with
     * probability mut_thr / 2^32 by a uniform integer in
     * [mut_lo, mut_hi], increments the generation counter, and writes a
     * fresh one-bit differentia at this generation's site.              */
    for (uint32_t j = 0; j < N; j++) {
        uint32_t a = i * N + j;
        uint32_t p, child_trait, bit;
        draw_birth(r, q, i, j, g, &p, &child_trait, &bit);
        uint32_t T = q->counter[p];
        if (T != g)
            return -2;
        r->n_trait[a] = child_trait;
        r->n_counter[a] = T + 1;
        for (uint32_t s = 0; s < SW; s++)
            r->n_surf[(size_t)a * SW + s] = q->surf[p * SW + s];
        if (ingest) {
            uint32_t per_word = 32 / r->bits;
            uint32_t shift = ((uint32_t)site % per_word) * r->bits;
            uint32_t mask = (r->bits == 8 ? 0xffu : 1u) << shift;
            uint32_t *word = &r->n_surf[(size_t)a * SW + (uint32_t)site / per_word];
            *word = (*word & ~mask) | (bit << shift);
        }
        r->n_src[a] = q->src[p];
        if (g < r->ped_gens) {
            r->ped_parent[(size_t)g * r->A + a] = q->src[p];
            r->ped_bit[(size_t)g * r->A + a] = (uint8_t)bit;
        }
    }
    return 0;
}

/* Island-parallel births, used to time the oracle on many host cores:
 * the islands are split into contiguous ranges, one per thread, each thread
 * with its own island scratch; joining the threads is the one barrier per
 * generation.  Islands are independent within a generation (breed_island),
 * so the result is the serial one.                                         */
#define ORC_MAX_THREADS 256

typedef struct {
    orc_run *r;
    orc_island *q;
    uint32_t i0, i1, g;
    int site, ingest, rc;
    int emigrate;                     /* the emigration pass instead of births */
} orc_task;

static void emigrate_island(orc_run *r, uint32_t i, uint32_t g);

static void *breed_range(void *arg)
{
    orc_task *t = (orc_task *)arg;
    for (uint32_t i = t->i0; i < t->i1 && t->rc == 0; i++) {
        if (t->emigrate)
            emigrate_island(t->r, i, t->g);
        else
            t->rc = breed_island(t->r, t->q, i, t->g, t->site, t->ingest);
    }
    return NULL;
}

static int breed_threaded(orc_run *r, uint32_t g, int site, int ingest, int emigrate)
{
    const uint32_t n = r->threads;
    pthread_t tid[ORC_MAX_THREADS];
    int started[ORC_MAX_THREADS];
    orc_task task[ORC_MAX_THREADS];
    for (uint32_t k = 0; k < n; k++) {
        task[k].r = r;
        task[k].q = &r->tq[k];
        task[k].i0 = (uint32_t)((uint64_t)r->I * k / n);
        task[k].i1 = (uint32_t)((uint64_t)r->I * (k + 1) / n);
        task[k].g = g;
        task[k].site = site;
        task[k].ingest = ingest;
        task[k].rc = 0;
        task[k].emigrate = emigrate;
        started[k] = pthread_create(&tid[k], NULL, breed_range, &task[k]) == 0;
        if (!started[k])
            breed_range(&task[k]);   /* no thread: this range in the caller */
    }
    int rc = 0;
    for (uint32_t k = 0; k < n; k++) {
        if (started[k])
            pthread_join(tid[k], NULL);
        if (rc == 0)
            rc = task[k].rc;
    }
    return rc;
}

/* Breed synchronous generations on `threads` host threads (0 or 1: one).
 * Asynchronous ticks stay serial.  Returns 0, or -1 if invalid or out of
 * memory.                                                                  */
int orc_set_threads(void *handle, uint32_t threads)
{
    orc_run *r = (orc_run *)handle;
    if (threads > ORC_MAX_THREADS)
        return -1;
    if (r->tq) {
        for (uint32_t k = 0; k < r->threads; k++)
            island_free(&r->tq[k]);
        free(r->tq);
        r->tq = NULL;
    }
    r->threads = 0;
    if (threads <= 1)
        return 0;
    r->tq = (orc_island *)calloc(threads, sizeof(orc_island));
    if (!r->tq)
        return -1;
    r->threads = threads;
    for (uint32_t k = 0; k < threads; k++) {
        if (!island_alloc(&r->tq[k], r->N, r->SW)) {
            orc_set_threads(handle, 0);
            return -1;
        }
    }
    return 0;
}

/* One generation, (P_g, O_g) -> (P_{g+1}, O_{g+1}), island by island, in the
 * paper's order: migration first, then selection, mutation and the
 * annotation update (Asynchronous Island-model Genetic Algorithm).
 * Returns 0, -1 beyond the horizon, -2 on a broken invariant.               */
static int step_one(orc_run *r)
{
    const uint32_t g = r->g;

    /* The surface site for this generation's births.  Every parent carries
     * counter g, so every birth deposits item g at the same site: the
     * placement is computed once for the whole population (Results, Surface
     * Algorithm Benchmark: synchronous generations can cache placements).   */
    /* With an ingest interval n, only generations g = n tau deposit (item
     * tau of the site rule, in ingest units); the others copy the parent's
     * annotation unchanged.                                                 */
    int site = -1;
    uint32_t tau = g / r->interval;
    int ingest = g % r->interval == 0;
    if (ingest) {
        if ((uint64_t)tau > orc_horizon(r->kind, r->S))
            return -1;
        site = orc_place(r->kind, r->S, r->L, tau);
        if (site < 0)
            return -1;
    }

    if (r->threads > 1) {
        int rc = breed_threaded(r, g, site, ingest, 0);
        if (rc)
            return rc;
    } else {
        for (uint32_t i = 0; i < r->I; i++) {
            int rc = breed_island(r, &r->q, i, g, site, ingest);
            if (rc)
                return rc;
        }
    }

    /* P_{g+1} becomes current (the buffers trade places: every slot of the
     * next population is written before it is read)                       */
    uint32_t *tmp;
    tmp = r->trait; r->trait = r->n_trait; r->n_trait = tmp;
    tmp = r->counter; r->counter = r->n_counter; r->n_counter = tmp;
    tmp = r->surf; r->surf = r->n_surf; r->n_surf = tmp;
    if (ingest)
        r->L[site] = tau;

    /* Emigration, after every island's births (the outbox the births read
     * is overwritten): islands are independent here too.                   */
    if (r->migrants) {
        if (r->threads > 1) {
            breed_threaded(r, g, site, ingest, 1);
        } else {
            for (uint32_t i = 0; i < r->I; i++)
                emigrate_island(r, i, g);
        }
        r->has_outbox = 1;
    }
    r->g = g + 1;
    return 0;
}

/* Emigration of island i at step g: a copy of a uniformly chosen member of
 * the new population goes into the island's outbox, addressed to a
 * uniformly chosen cardinal neighbour; it is read in the next generation. */
static void emigrate_island(orc_run *r, uint32_t i, uint32_t g)
{
    const uint32_t N = r->N, SW = r->SW;
    uint32_t w[4];
    orc_philox(0, i, g, ORC_EMIGRATE, r->seed, w);
    uint32_t e = orc_mulhi(w[0], N);
    uint32_t a = i * N + e;
    r->ob_dir[i] = w[1] >> 30;
    r->ob_trait[i] = r->trait[a];
    r->ob_counter[i] = r->counter[a];
    for (uint32_t s = 0; s < SW; s++)
        r->ob_surf[(size_t)i * SW + s] = r->surf[(size_t)a * SW + s];
    r->ob_src[i] = a;
}

/* ------------------------------------------------------------------------ */
/* Asynchronous runs (Methods, Asynchronous Island-model Genetic Algorithm:
 * processing elements run their own generation loops and exchange
 * migrants without synchronising, so neighbours drift apart in generation
 * count).  Reading: time advances in ticks; on tick k island i runs one
 * generation iff the first word of Philox block (0, i, k, ACTIVITY) is below
 * the activity threshold, else it stays as it is and posts no emigrant.  An
 * active island reads the emigrants its neighbours posted on tick k-1, then
 * breeds as in a synchronous generation, except that every agent carries its
 * own counter: a birth from a parent with counter T deposits item T (in
 * ingest units, when T is a multiple of the interval) at the site that the
 * rule gives the T-th ingest.  That site depends on T alone, so a table of
 * sites by ingest index makes the lookup O(1) per agent.                   */

/* Site of ingest tau, extending the table by replaying placements.  Returns
 * -1 beyond the horizon or on no memory.                                   */
static int site_of(orc_run *r, uint32_t tau)
{
    while (r->tab_filled <= tau) {
        if (r->tab_filled == r->tab_cap) {
            uint32_t cap = r->tab_cap ? 2 * r->tab_cap : 1024;
            uint32_t *t = (uint32_t *)realloc(r->tab, (size_t)cap * 4);
            if (!t)
                return -1;
            r->tab = t;
            r->tab_cap = cap;
        }
        uint32_t u = r->tab_filled;
        if ((uint64_t)u > orc_horizon(r->kind, r->S))
            return -1;
        int site = orc_place(r->kind, r->S, r->Ltab, u);
        if (site < 0)
            return -1;
        r->Ltab[site] = u;
        r->tab[u] = (uint32_t)site;
        r->tab_filled++;
    }
    return (int)r->tab[tau];
}

/* Switch a run to ticks with islands active with probability
 * activity / 2^32 (0 switches back to synchronous generations).  Only
 * before the first step.  Returns 0 or -1.                                  */
int orc_set_async(void *handle, uint32_t activity)
{
    orc_run *r = (orc_run *)handle;
    if (r->g != 0)
        return -1;
    r->activity = activity;
    return 0;
}

static int step_async(orc_run *r)
{
    const uint32_t N = r->N, SW = r->SW, k = r->g;
    orc_island *q = &r->q;
    uint32_t w[4];
    if ((uint64_t)k > orc_horizon_gen(r->kind, r->S, r->interval))
        return -1;
    uint8_t *active = (uint8_t *)malloc(r->I);
    if (!active)
        return -2;
    for (uint32_t i = 0; i < r->I; i++) {
        orc_philox(0, i, k, ORC_ACTIVITY, r->seed, w);
        active[i] = w[0] < r->activity;
    }
    for (uint32_t i = 0; i < r->I; i++) {
        if (!active[i]) {
            /* no generation: the same individuals on the next tick */
            for (uint32_t j = 0; j < N; j++) {
                uint32_t a = i * N + j;
                r->n_trait[a] = r->trait[a];
                r->n_counter[a] = r->counter[a];
                for (uint32_t s = 0; s < SW; s++)
                    r->n_surf[(size_t)a * SW + s] = r->surf[(size_t)a * SW + s];
                if (k < r->ped_gens) {
                    r->ped_parent[(size_t)k * r->A + a] = a;
                    r->ped_bit[(size_t)k * r->A + a] = 0;
                }
            }
            continue;
        }
        for (uint32_t j = 0; j < N; j++) {
            uint32_t a = i * N + j;
            q->trait[j] = r->trait[a];
            q->counter[j] = r->counter[a];
            for (uint32_t s = 0; s < SW; s++)
                q->surf[j * SW + s] = r->surf[(size_t)a * SW + s];
            q->src[j] = a;
        }
        /* immigrants posted on the previous tick toward this island */
        if (r->migrants && r->has_outbox) {
            orc_philox(0, i, k, ORC_IMMIGRATE, r->seed, w);
            for (uint32_t d = 0; d < 4; d++) {
                uint32_t nb = neighbour(r, i, d);
                if (r->ob_dir[nb] == opposite(d)) {
                    uint32_t slot = orc_mulhi(w[d], N);
                    q->trait[slot] = r->ob_trait[nb];
                    q->counter[slot] = r->ob_counter[nb];
                    for (uint32_t s = 0; s < SW; s++)
                        q->surf[slot * SW + s] = r->ob_surf[(size_t)nb * SW + s];
                    q->src[slot] = r->ob_src[nb];
                }
            }
        }
        for (uint32_t j = 0; j < N; j++) {
            uint32_t a = i * N + j;
            uint32_t p, child_trait, bit;
            draw_birth(r, q, i, j, k, &p, &child_trait, &bit);
            uint32_t T = q->counter[p];
            r->n_trait[a] = child_trait;
            r->n_counter[a] = T + 1;
            for (uint32_t s = 0; s < SW; s++)
                r->n_surf[(size_t)a * SW + s] = q->surf[p * SW + s];
            if (T % r->interval == 0) {
                int site = site_of(r, T / r->interval);
                if (site < 0) {
                    free(active);
                    return -1;
                }
                uint32_t per_word = 32 / r->bits;
                uint32_t shift = ((uint32_t)site % per_word) * r->bits;
                uint32_t mask = (r->bits == 8 ? 0xffu : 1u) << shift;
                uint32_t *word = &r->n_surf[(size_t)a * SW + (uint32_t)site / per_word];
                *word = (*word & ~mask) | (bit << shift);
            }
            if (k < r->ped_gens) {
                r->ped_parent[(size_t)k * r->A + a] = q->src[p];
                r->ped_bit[(size_t)k * r->A + a] = (uint8_t)bit;
            }
        }
    }
    memcpy(r->trait, r->n_trait, (size_t)r->A * 4);
    memcpy(r->counter, r->n_counter, (size_t)r->A * 4);
    memcpy(r->surf, r->n_surf, (size_t)r->A * SW * 4);
    /* emigration from active islands; inactive ones post nothing */
    if (r->migrants) {
        for (uint32_t i = 0; i < r->I; i++) {
            if (!active[i]) {
                r->ob_dir[i] = 4;   /* addressed to no neighbour */
                r->ob_trait[i] = r->ob_counter[i] = r->ob_src[i] = 0;
                for (uint32_t s = 0; s < SW; s++)
                    r->ob_surf[(size_t)i * SW + s] = 0;
                continue;
            }
            orc_philox(0, i, k, ORC_EMIGRATE, r->seed, w);
            uint32_t e = orc_mulhi(w[0], N);
            uint32_t a = i * N + e;
            r->ob_dir[i] = w[1] >> 30;
            r->ob_trait[i] = r->trait[a];
            r->ob_counter[i] = r->counter[a];
            for (uint32_t s = 0; s < SW; s++)
                r->ob_surf[(size_t)i * SW + s] = r->surf[(size_t)a * SW + s];
            r->ob_src[i] = a;
        }
        r->has_outbox = 1;
    }
    free(active);
    r->g = k + 1;
    return 0;
}

/* Advance n generations (the paper's main loop runs until a generation
 * count is reached).  Returns 0, -1 beyond the horizon, -2 on a broken
 * invariant, -3 if n would pass the end of the pedigree record.            */
int orc_step(void *handle, uint32_t n)
{
    orc_run *r = (orc_run *)handle;
    if (r->ped_gens && (uint64_t)r->g + n > r->ped_gens)
        return -3;
    for (uint32_t k = 0; k < n; k++) {
        int rc = r->activity ? step_async(r) : step_one(r);
        if (rc)
            return rc;
    }
    return 0;
}

uint32_t orc_generation(void *handle) { return ((orc_run *)handle)->g; }
uint32_t orc_num_agents(void *handle) { return ((orc_run *)handle)->A; }

void orc_read_agents(void *handle, uint32_t *trait, uint32_t *counter,
                     uint32_t *surf)
{
    orc_run *r = (orc_run *)handle;
    memcpy(trait, r->trait, (size_t)r->A * 4);
    memcpy(counter, r->counter, (size_t)r->A * 4);
    memcpy(surf, r->surf, (size_t)r->A * r->SW * 4);
}

/* Outbox O_g (to be read at step g).  Returns 0 when there is none.        */
int orc_read_outbox(void *handle, uint32_t *dir, uint32_t *trait,
                    uint32_t *counter, uint32_t *surf, uint32_t *src)
{
    orc_run *r = (orc_run *)handle;
    if (!r->has_outbox)
        return 0;
    memcpy(dir, r->ob_dir, (size_t)r->I * 4);
    memcpy(trait, r->ob_trait, (size_t)r->I * 4);
    memcpy(counter, r->ob_counter, (size_t)r->I * 4);
    memcpy(surf, r->ob_surf, (size_t)r->I * r->SW * 4);
    if (src)
        memcpy(src, r->ob_src, (size_t)r->I * 4);
    return 1;
}

/* The run's layout as deposit generations (ingest index times interval),
 * EMPTY for unfilled sites.                                                */
void orc_read_layout(void *handle, uint32_t *L)
{
    orc_run *r = (orc_run *)handle;
    uint32_t Lr[64];
    if (r->activity) {
        /* asynchronous: the layout of an annotation whose counter is the
         * number of ticks so far                                           */
        if (orc_layout(r->kind, r->S, ingests_of(r->g, r->interval), Lr) != 0)
            for (uint32_t k = 0; k < r->S; k++)
                Lr[k] = ORC_EMPTY;
    } else {
        memcpy(Lr, r->L, sizeof Lr);
    }
    for (uint32_t k = 0; k < r->S; k++)
        L[k] = Lr[k] == ORC_EMPTY ? ORC_EMPTY : Lr[k] * r->interval;
}

/* Pedigree of generation gen (1..ped_gens): parent index in P_{gen-1} and
 * the differentia drawn at each birth (whether or not it was deposited).   */
int orc_read_pedigree(void *handle, uint32_t gen, uint32_t *parent,
                      uint8_t *bit)
{
    orc_run *r = (orc_run *)handle;
    if (gen == 0 || gen > r->ped_gens || gen > r->g)
        return -1;
    memcpy(parent, r->ped_parent + (size_t)(gen - 1) * r->A, (size_t)r->A * 4);
    memcpy(bit, r->ped_bit + (size_t)(gen - 1) * r->A, (size_t)r->A);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* End-of-run sampling (Results, On-hardware Trial: end-state genomes are
 * sampled, then subsampled).  Reading: a stratified sample; agent k is drawn
 * uniformly from the k-th of n equal strata of the population.  When the
 * population is not larger than n, every agent is taken.  Returns the
 * number of indices written.                                                */
uint32_t orc_sample(uint64_t seed, uint32_t A, uint32_t n, uint32_t T,
                    uint32_t *idx)
{
    if (A <= n) {
        for (uint32_t k = 0; k < A; k++)
            idx[k] = k;
        return A;
    }
    uint32_t w[4];
    for (uint32_t k = 0; k < n; k++) {
        uint32_t lo = (uint32_t)((uint64_t)k * A / n);
        uint32_t hi = (uint32_t)((uint64_t)(k + 1) * A / n);
        orc_philox(k, 0, T, ORC_SAMPLE, seed, w);
        idx[k] = lo + orc_mulhi(w[0], hi - lo);
    }
    return n;
}

/* Value held at site k of a surface of `bits`-bit differentiae. */
static uint32_t site_value(const uint32_t *s, uint32_t k, uint32_t bits)
{
    uint32_t per_word = 32 / bits;
    uint32_t mask = bits == 8 ? 0xffu : 1u;
    return (s[k / per_word] >> ((k % per_word) * bits)) & mask;
}

/* MRCA-generation bounds from two annotations (Distributed Phylogenetic
 * Tracking: mismatching differentiae delimit the extent of common ancestry;
 * narrow differentiae can collide and overstate relatedness).
 *
 * Written out from the definition: C = the deposit times retained by both
 * annotations, ascending; t* = the first t in C whose differentiae differ.
 * A mismatch at t shows the two generation-(t+1) ancestors differ, so the
 * MRCA's generation is at most t*:  ub = t*, or min(Ta, Tb) if nothing
 * differs.  The last agreeing t before t* (or the last of C) gives
 * lb = t + 1, or 0 when there is none.  lb assumes no collision.  La and Lb
 * are the two layouts in ingest units (orc_layout of each annotation's
 * number of ingests); item tau was deposited at generation tau * interval.  */
int orc_mrca_pair_x(uint32_t S, uint32_t bits, uint32_t interval, uint32_t Ta,
                    const uint32_t *sa, const uint32_t *La, uint32_t Tb,
                    const uint32_t *sb, const uint32_t *Lb, uint32_t *lb, uint32_t *ub)
{
    /* common deposit times with their sites in each annotation */
    uint32_t ct[64], ka[64], kb[64];
    uint32_t nc = 0;
    for (uint32_t x = 0; x < S; x++) {
        if (La[x] == ORC_EMPTY)
            continue;
        for (uint32_t y = 0; y < S; y++) {
            if (Lb[y] == La[x]) {
                ct[nc] = La[x]; ka[nc] = x; kb[nc] = y; nc++;
                break;
            }
        }
    }
    /* ascending order of time (insertion sort: at most 64 items) */
    for (uint32_t p = 1; p < nc; p++) {
        uint32_t t = ct[p], x = ka[p], y = kb[p];
        uint32_t q = p;
        while (q > 0 && ct[q - 1] > t) {
            ct[q] = ct[q - 1]; ka[q] = ka[q - 1]; kb[q] = kb[q - 1]; q--;
        }
        ct[q] = t; ka[q] = x; kb[q] = y;
    }
    int have_last = 0;
    uint32_t last = 0;
    for (uint32_t p = 0; p < nc; p++) {
        uint32_t gen = ct[p] * interval;   /* deposit generation */
        if (site_value(sa, ka[p], bits) != site_value(sb, kb[p], bits)) {
            *ub = gen;
            *lb = have_last ? last + 1 : 0;
            return 0;
        }
        have_last = 1;
        last = gen;
    }
    *ub = Ta < Tb ? Ta : Tb;
    *lb = have_last ? last + 1 : 0;
    return 0;
}

int orc_mrca_pair(uint32_t S, uint32_t Ta, const uint32_t *sa,
                  const uint32_t *La, uint32_t Tb, const uint32_t *sb,
                  const uint32_t *Lb, uint32_t *lb, uint32_t *ub)
{
    return orc_mrca_pair_x(S, 1, 1, Ta, sa, La, Tb, sb, Lb, lb, ub);
}

/* Layouts (ingest units) of n annotations, one per counter. */
static uint32_t *layouts_of(uint32_t kind, uint32_t S, uint32_t interval, uint32_t n,
                            const uint32_t *counters)
{
    uint32_t *L = (uint32_t *)malloc((size_t)(n ? n : 1) * S * 4);
    if (!L)
        return NULL;
    for (uint32_t a = 0; a < n; a++) {
        /* reuse the previous layout when the counter repeats */
        if (a > 0 && counters[a] == counters[a - 1]) {
            memcpy(L + (size_t)a * S, L + (size_t)(a - 1) * S, (size_t)S * 4);
        } else if (orc_layout(kind, S, ingests_of(counters[a], interval),
                              L + (size_t)a * S) != 0) {
            free(L);
            return NULL;
        }
    }
    return L;
}

/* Selected rows of the all-pairs matrix: lb and ub are nrows * n, row r
 * holding annotation rows[r] against every annotation b; rows == NULL
 * means every row (nrows = n).  Surfaces are agent-major, S*bits/32 words
 * per agent.  Returns 0, or -1 beyond the horizon / bad row / no memory. */
int orc_mrca_rows_x(uint32_t kind, uint32_t S, uint32_t bits, uint32_t interval,
                    uint32_t n, const uint32_t *counters, const uint32_t *surf,
                    uint32_t nrows, const uint32_t *rows, uint32_t *lb, uint32_t *ub)
{
    if (!scheme_ok(S, bits, interval))
        return -1;
    uint32_t SW = S * bits / 32;
    uint32_t *L = layouts_of(kind, S, interval, n, counters);
    if (!L)
        return -1;
    for (uint32_t r = 0; r < nrows; r++) {
        uint32_t a = rows ? rows[r] : r;
        if (a >= n) {
            free(L);
            return -1;
        }
        for (uint32_t b = 0; b < n; b++)
            orc_mrca_pair_x(S, bits, interval, counters[a], surf + (size_t)a * SW,
                            L + (size_t)a * S, counters[b], surf + (size_t)b * SW,
                            L + (size_t)b * S, lb + (size_t)r * n + b,
                            ub + (size_t)r * n + b);
    }
    free(L);
    return 0;
}

/* All ordered pairs of n annotations: lb and ub are n*n, row-major (row a,
 * column b).                                                               */
int orc_mrca_allpairs_x(uint32_t kind, uint32_t S, uint32_t bits, uint32_t interval,
                        uint32_t n, const uint32_t *counters, const uint32_t *surf,
                        uint32_t *lb, uint32_t *ub)
{
    return orc_mrca_rows_x(kind, S, bits, interval, n, counters, surf, n, NULL, lb, ub);
}

int orc_mrca_allpairs(uint32_t kind, uint32_t S, uint32_t n,
                      const uint32_t *counters, const uint32_t *surf,
                      uint32_t *lb, uint32_t *ub)
{
    return orc_mrca_allpairs_x(kind, S, 1, 1, n, counters, surf, lb, ub);
}

int orc_mrca_rows(uint32_t kind, uint32_t S, uint32_t n, const uint32_t *counters,
                  const uint32_t *surf, uint32_t nrows, const uint32_t *rows,
                  uint32_t *lb, uint32_t *ub)
{
    return orc_mrca_rows_x(kind, S, 1, 1, n, counters, surf, nrows, rows, lb, ub);
}

/* ------------------------------------------------------------------------ */
/* Trie reconstruction and phylometrics of n annotations sharing a counter
 * T (Distributed Phylogenetic Tracking: the record of differentiae makes
 * reconstruction a trie-building procedure; Results, On-hardware Trial:
 * treatments are compared by sum branch length and mean evolutionary
 * distinctiveness).
 *
 * Reading: each annotation is read as its differentiae in ascending deposit
 * time (times t_0 < ... < t_{F-1} of the shared layout).  They are inserted
 * into a trie, one level per retained time, one child per differentia
 * value.  A trie node whose annotations split on the differentia of time
 * t_d becomes a tree node at time t_d (the MRCA upper bound of the pairs it
 * separates); annotations with identical differentiae hang from one node
 * at time T; each annotation is a leaf at time T; chains of one-child trie
 * nodes are collapsed; the root is the first branching node.
 *
 * Output: out[0] = sum of branch lengths; out[1] = sum over unordered
 * pairs of (T - time of their tree MRCA); out[2] = root time; out[3] =
 * number of internal nodes; ed[n] (may be NULL) = each leaf's evolutionary
 * distinctiveness (fair proportion: every edge's length shared equally by
 * the leaves below it), in double.  Returns 0, -1 if the counters differ
 * or are past the horizon, -2 on no memory.                                */
typedef struct {
    int first_child, next_sibling;
    uint32_t value;     /* differentia value on the edge from the parent   */
    int leaf_first;     /* first annotation index at a depth-F node, or -1 */
    int nleaves;        /* annotations below                               */
} orc_trie_node;

typedef struct {
    orc_trie_node *nodes;
    int count, cap;
} orc_trie;

static int trie_new(orc_trie *t, uint32_t value)
{
    if (t->count == t->cap) {
        int cap = t->cap ? 2 * t->cap : 1024;
        orc_trie_node *p = (orc_trie_node *)realloc(t->nodes, (size_t)cap * sizeof(*p));
        if (!p)
            return -1;
        t->nodes = p;
        t->cap = cap;
    }
    orc_trie_node *nd = &t->nodes[t->count];
    nd->first_child = nd->next_sibling = -1;
    nd->value = value;
    nd->leaf_first = -1;
    nd->nleaves = 0;
    return t->count++;
}

typedef struct {
    const uint32_t *times;   /* ascending retained deposit generations */
    uint32_t F, T;
    const orc_trie *trie;
    const int *leaf_next;    /* annotations sharing a depth-F node */
    uint64_t sbl;
    uint64_t pair_sum;
    uint32_t root_time;
    int have_root;
    uint64_t internal;
    double *ed;
} orc_phylo_ctx;

/* Walk the trie from node v at depth d, whose nearest tree ancestor sits at
 * time parent_t (or none at the very top).  acc_ed is the ED accumulated by
 * the path above v.  Adds every edge, every pair's MRCA time and every
 * leaf's ED.                                                                */
static void phylo_walk(orc_phylo_ctx *c, int v, uint32_t d, int has_parent,
                       uint32_t parent_t, double acc_ed)
{
    const orc_trie_node *nd = &c->trie->nodes[v];
    if (d == c->F) {
        /* annotations with identical differentiae */
        int k = nd->nleaves;
        uint32_t here = c->T;
        double ed_here = acc_ed;
        if (k >= 2) {
            /* a tree node at T with k leaf children (zero-length edges) */
            if (has_parent) {
                c->sbl += here - parent_t;
                ed_here += (double)(here - parent_t) / k;
            } else if (!c->have_root) {
                c->have_root = 1;
                c->root_time = here;
            }
            c->internal += 1;
            /* pairs inside: MRCA at T, contributes T - T = 0 */
        }
        for (int a = nd->leaf_first; a >= 0; a = c->leaf_next[a]) {
            double e = ed_here;
            if (k == 1 && has_parent) {
                c->sbl += c->T - parent_t;
                e += (double)(c->T - parent_t);
            }
            if (c->ed)
                c->ed[a] = e;
        }
        return;
    }
    int nchild = 0;
    for (int w = nd->first_child; w >= 0; w = c->trie->nodes[w].next_sibling)
        nchild++;
    if (nchild >= 2) {
        /* branching: a tree node at t_d */
        uint32_t here = c->times[d];
        double ed_here = acc_ed;
        if (has_parent) {
            c->sbl += here - parent_t;
            ed_here += (double)(here - parent_t) / nd->nleaves;
        } else if (!c->have_root) {
            c->have_root = 1;
            c->root_time = here;
        }
        c->internal += 1;
        /* pairs from different children meet here */
        uint64_t seen = 0;
        for (int w = nd->first_child; w >= 0; w = c->trie->nodes[w].next_sibling) {
            uint64_t k = (uint64_t)c->trie->nodes[w].nleaves;
            c->pair_sum += seen * k * (uint64_t)(c->T - here);
            seen += k;
        }
        for (int w = nd->first_child; w >= 0; w = c->trie->nodes[w].next_sibling)
            phylo_walk(c, w, d + 1, 1, here, ed_here);
    } else {
        phylo_walk(c, nd->first_child, d + 1, has_parent, parent_t, acc_ed);
    }
}

/* The trie of n annotations sharing a counter: retained deposit times in
 * ascending order (times[F]), the trie, and the annotations at each depth-F
 * node (leaf_next chains).  Returns 0, -1 if the counters differ or are past
 * the horizon, -2 on no memory.                                             */
typedef struct {
    uint32_t T, F;
    uint32_t times[64];
    orc_trie trie;
    int *leaf_next;
} orc_built_trie;

static void trie_free(orc_built_trie *b)
{
    free(b->leaf_next);
    free(b->trie.nodes);
}

static int build_trie(uint32_t kind, uint32_t S, uint32_t bits, uint32_t interval,
                      uint32_t n, const uint32_t *counters, const uint32_t *surf,
                      orc_built_trie *b)
{
    memset(b, 0, sizeof *b);
    if (!scheme_ok(S, bits, interval))
        return -1;
    uint32_t SW = S * bits / 32;
    for (uint32_t a = 1; a < n; a++)
        if (counters[a] != counters[0])
            return -1;
    uint32_t T = n ? counters[0] : 0;
    uint32_t L[64];
    if (orc_layout(kind, S, ingests_of(T, interval), L) != 0)
        return -1;
    /* retained sites in ascending deposit time */
    uint32_t sites[64], F = 0;
    for (uint32_t k = 0; k < S; k++) {
        if (L[k] == ORC_EMPTY)
            continue;
        uint32_t q = F++;
        while (q > 0 && b->times[q - 1] > L[k] * interval) {
            b->times[q] = b->times[q - 1];
            sites[q] = sites[q - 1];
            q--;
        }
        b->times[q] = L[k] * interval;
        sites[q] = k;
    }
    b->T = T;
    b->F = F;
    b->leaf_next = (int *)malloc((size_t)(n ? n : 1) * sizeof(int));
    if (!b->leaf_next || trie_new(&b->trie, 0) < 0) {
        trie_free(b);
        return -2;
    }
    orc_trie *trie = &b->trie;
    for (uint32_t a = 0; a < n; a++) {
        int v = 0;
        trie->nodes[v].nleaves++;
        for (uint32_t r = 0; r < F; r++) {
            uint32_t val = site_value(surf + (size_t)a * SW, sites[r], bits);
            int w = trie->nodes[v].first_child;
            while (w >= 0 && trie->nodes[w].value != val)
                w = trie->nodes[w].next_sibling;
            if (w < 0) {
                w = trie_new(trie, val);
                if (w < 0) {
                    trie_free(b);
                    return -2;
                }
                trie->nodes[w].next_sibling = trie->nodes[v].first_child;
                trie->nodes[v].first_child = w;
            }
            v = w;
            trie->nodes[v].nleaves++;
        }
        b->leaf_next[a] = trie->nodes[v].leaf_first;
        trie->nodes[v].leaf_first = (int)a;
    }
    return 0;
}

int orc_phylo_metrics_x(uint32_t kind, uint32_t S, uint32_t bits, uint32_t interval,
                        uint32_t n, const uint32_t *counters, const uint32_t *surf,
                        uint64_t out[4], double *ed)
{
    orc_built_trie b;
    int rc = build_trie(kind, S, bits, interval, n, counters, surf, &b);
    if (rc)
        return rc;
    orc_phylo_ctx c = {b.times, b.F, b.T, &b.trie, b.leaf_next, 0, 0, 0, 0, 0, ed};
    if (n > 0)
        phylo_walk(&c, 0, 0, 0, 0, 0.0);
    if (!c.have_root)
        c.root_time = b.T;
    out[0] = c.sbl;
    out[1] = c.pair_sum;
    out[2] = c.root_time;
    out[3] = c.internal;
    trie_free(&b);
    return 0;
}

/* The reconstructed tree as canonical Newick text: leaves are annotation
 * indices, branch lengths are generations, the children of every node are
 * listed in the order of the smallest annotation index below them (and the
 * leaves of a polytomy in ascending order), the root has no length.  A
 * single annotation is "0;".                                                */
typedef struct {
    char *buf;
    size_t cap, len;
    int overflow;
} orc_text;

static void text_put(orc_text *t, const char *s)
{
    size_t k = strlen(s);
    if (t->len + k + 1 > t->cap) {
        t->overflow = 1;
        return;
    }
    memcpy(t->buf + t->len, s, k + 1);
    t->len += k;
}

static void text_uint(orc_text *t, uint64_t v)
{
    char tmp[24];
    int k = 0;
    do {
        tmp[k++] = (char)('0' + v % 10);
        v /= 10;
    } while (v);
    char out[24];
    for (int i = 0; i < k; i++)
        out[i] = tmp[k - 1 - i];
    out[k] = 0;
    text_put(t, out);
}

/* smallest annotation index below trie node v at depth d */
static int trie_min_leaf(const orc_built_trie *b, int v, uint32_t d)
{
    const orc_trie_node *nd = &b->trie.nodes[v];
    if (d == b->F) {
        int m = -1;
        for (int a = nd->leaf_first; a >= 0; a = b->leaf_next[a])
            if (m < 0 || a < m)
                m = a;
        return m;
    }
    int m = -1;
    for (int w = nd->first_child; w >= 0; w = b->trie.nodes[w].next_sibling) {
        int x = trie_min_leaf(b, w, d + 1);
        if (m < 0 || x < m)
            m = x;
    }
    return m;
}

static int cmp_int(const void *x, const void *y)
{
    int a = *(const int *)x, c = *(const int *)y;
    return (a > c) - (a < c);
}

static int newick_walk(const orc_built_trie *b, orc_text *t, int v, uint32_t d,
                       int has_parent, uint32_t parent_t)
{
    /* collapse one-child chains */
    while (d < b->F) {
        const orc_trie_node *nd = &b->trie.nodes[v];
        if (nd->first_child >= 0 && b->trie.nodes[nd->first_child].next_sibling >= 0)
            break;
        v = nd->first_child;
        d++;
    }
    const orc_trie_node *nd = &b->trie.nodes[v];
    if (d == b->F) {
        int k = nd->nleaves;
        int *leaves = (int *)malloc((size_t)k * sizeof(int));
        if (!leaves)
            return -2;
        int i = 0;
        for (int a = nd->leaf_first; a >= 0; a = b->leaf_next[a])
            leaves[i++] = a;
        qsort(leaves, (size_t)k, sizeof(int), cmp_int);
        if (k == 1) {
            text_uint(t, (uint64_t)leaves[0]);
        } else {
            text_put(t, "(");
            for (i = 0; i < k; i++) {
                if (i)
                    text_put(t, ",");
                text_uint(t, (uint64_t)leaves[i]);
                text_put(t, ":0");
            }
            text_put(t, ")");
        }
        free(leaves);
        if (has_parent) {
            text_put(t, ":");
            text_uint(t, (uint64_t)(b->T - parent_t));
        }
        return 0;
    }
    /* a branching node at t_d: children by their smallest annotation */
    uint32_t here = b->times[d];
    int nch = 0;
    for (int w = nd->first_child; w >= 0; w = b->trie.nodes[w].next_sibling)
        nch++;
    int *ch = (int *)malloc((size_t)nch * 2 * sizeof(int));
    if (!ch)
        return -2;
    int i = 0;
    for (int w = nd->first_child; w >= 0; w = b->trie.nodes[w].next_sibling, i++) {
        ch[2 * i] = trie_min_leaf(b, w, d + 1);
        ch[2 * i + 1] = w;
    }
    /* sort pairs by smallest leaf (insertion sort: at most 256 children) */
    for (int p = 1; p < nch; p++) {
        int k0 = ch[2 * p], k1 = ch[2 * p + 1], q = p;
        while (q > 0 && ch[2 * (q - 1)] > k0) {
            ch[2 * q] = ch[2 * (q - 1)];
            ch[2 * q + 1] = ch[2 * (q - 1) + 1];
            q--;
        }
        ch[2 * q] = k0;
        ch[2 * q + 1] = k1;
    }
    text_put(t, "(");
    for (i = 0; i < nch; i++) {
        if (i)
            text_put(t, ",");
        int rc = newick_walk(b, t, ch[2 * i + 1], d + 1, 1, here);
        if (rc) {
            free(ch);
            return rc;
        }
    }
    text_put(t, ")");
    free(ch);
    if (has_parent) {
        text_put(t, ":");
        text_uint(t, (uint64_t)(here - parent_t));
    }
    return 0;
}

/* Returns the text length, -1 if the counters differ or are past the
 * horizon, -2 on no memory, -3 if cap is too small.                        */
long orc_phylo_newick_x(uint32_t kind, uint32_t S, uint32_t bits, uint32_t interval,
                        uint32_t n, const uint32_t *counters, const uint32_t *surf,
                        char *buf, size_t cap)
{
    if (n == 0 || cap == 0)
        return -3;
    orc_built_trie b;
    int rc = build_trie(kind, S, bits, interval, n, counters, surf, &b);
    if (rc)
        return rc;
    orc_text t = {buf, cap, 0, 0};
    buf[0] = 0;
    rc = newick_walk(&b, &t, 0, 0, 0, 0);
    text_put(&t, ";");
    trie_free(&b);
    if (rc)
        return rc;
    if (t.overflow)
        return -3;
    return (long)t.len;
}

int orc_phylo_metrics(uint32_t kind, uint32_t S, uint32_t n, const uint32_t *counters,
                      const uint32_t *surf, uint64_t out[4], double *ed)
{
    return orc_phylo_metrics_x(kind, S, 1, 1, n, counters, surf, out, ed);
}
