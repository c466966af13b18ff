/*
 * hsga.h -- C ABI of libhsga.so: an island-model genetic algorithm whose
 * agents carry hereditary-stratigraphy surface annotations, run on one
 * AMD Instinct MI355X (gfx950) with hand-written HIP kernels.
 *
 * The method is the one of Moreno et al., "Trackable Agent-based Evolution
 * Models at Wafer Scale":
 *   - islands of agents on a 2-D torus exchange migrants with their four
 *     cardinal neighbours; each generation does migration first, then
 *     tournament selection, mutation and the annotation update (Methods,
 *     Asynchronous Island-model Genetic Algorithm);
 *   - each birth deposits a fresh one-bit differentia into one site of a
 *     fixed-width "surface" chosen by a steady, tilted or hybrid policy
 *     (Methods, Distributed Phylogenetic Tracking; Surface-based Hereditary
 *     Stratigraphy Algorithms);
 *   - mismatching differentiae of two annotations bound the generation of
 *     their most recent common ancestor (Distributed Phylogenetic Tracking).
 *
 * Conventions shared by every call:
 *   - Memory.  The library never allocates or frees device memory.  The
 *     caller owns one device arena per run (sized by ga_footprint_bytes) and
 *     every other device buffer it passes in.  Host buffers are caller-owned.
 *   - Streams.  hip_stream is a hipStream_t borrowed from the caller (NULL
 *     means the null stream).  Device work is enqueued on it and returns
 *     without waiting, unless a call says it blocks.
 *   - Errors.  Every int-returning call returns a ga_status.  Nothing
 *     aborts or throws across the ABI.  ga_last_error() gives the text of
 *     the calling thread's last failure.
 *   - Threading.  A run handle is used by one host thread at a time.
 *   - Determinism.  Results are a function of the configuration and the
 *     seed alone.  They do not depend on launch shapes, chunking or timing.
 */
#ifndef HSGA_H
#define HSGA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    GA_OK = 0,
    GA_EINVAL = -1,    /* invalid argument or configuration                */
    GA_ENOMEM = -2,    /* caller-provided buffer or arena too small        */
    GA_EHORIZON = -3,  /* the site rule cannot place that many generations */
    GA_EDEVICE = -4,   /* a HIP call failed (text in ga_last_error)        */
    GA_EBUSY = -5      /* pool admission refused: footprint does not fit   */
} ga_status;

/* Surface site-selection policy (Distributed Phylogenetic Tracking):
 * steady spreads retained time points evenly over history, tilted prefers
 * recent ones, hybrid gives half of the sites to each.                     */
typedef enum { GA_STEADY = 0, GA_TILTED = 1, GA_HYBRID = 2 } ga_surface_kind;

/* Marker for a surface site that holds no differentia yet. */
#define GA_EMPTY_SITE 0xffffffffu

/* Fitness model.  GA_INT_TRAIT: the configured integer trait (signed
 * comparison, uniform integer mutation).  GA_FLOAT_FITNESS: the paper's
 * float treatments (Asynchronous Island-model Genetic Algorithm; Results,
 * On-hardware Trial): the trait word holds a binary32 fitness, selection is
 * a tournament of up to five, and a birth is deleterious (fitness decreases
 * by del_sigma |Z|) or beneficial (increases by ben_sigma |Z|) with the
 * configured probabilities, |Z| half-normal from a Box-Muller draw.
 * GA_FOUNDER_TAG: the clade trial's genome (Genome Model; Results, Clade
 * Reconstruction Trial): each founder's trait word is a random 16-bit tag,
 * inherited without mutation under neutral selection (tournament_size 0). */
typedef enum { GA_INT_TRAIT = 0, GA_FLOAT_FITNESS = 1, GA_FOUNDER_TAG = 2 } ga_fitness_model;

typedef struct ga_config {
    uint32_t struct_size;         /* sizeof(ga_config) = 88; 56 and 80 (the
                                     layouts ending after seed and after
                                     differentia_bits) are accepted, absent
                                     fields read as 0                         */
    uint32_t grid_w, grid_h;      /* torus of islands; island i = y*w + x      */
    uint32_t pop_per_island;      /* N agents per island, 1..64                */
    uint32_t surface_sites;       /* S sites: 32 or 64 one-bit sites, or 4 or
                                     8 byte sites (differentia_bits = 8)      */
    uint32_t surface_kind;        /* ga_surface_kind                           */
    uint32_t tournament_size;     /* GA_INT_TRAIT: 2 = tournament of two,
                                     0 = neutral.  GA_FLOAT_FITNESS: 1..5
                                     draws (0 and 1 = neutral)                 */
    uint32_t mut_threshold;       /* GA_INT_TRAIT: mutate iff a uniform 32-bit
                                     word is below this; p = 0.01 -> 42949672 */
    int32_t mut_lo, mut_hi;       /* GA_INT_TRAIT: inclusive trait-delta
                                     range, e.g. -8, 8                         */
    uint32_t migrants_per_island; /* 1, or 0 to switch migration off           */
    uint32_t ingest_interval;     /* deposit a differentia every n-th
                                     generation only (0 or 1: every one)      */
    uint64_t seed;                /* Philox4x32-10 key                         */
    /* GA_FLOAT_FITNESS only (ignored otherwise): */
    uint32_t fitness_model;       /* ga_fitness_model                          */
    uint32_t del_threshold;       /* deleterious iff the class word < this;
                                     p = 0.33 -> 1417339207                    */
    uint32_t ben_threshold;       /* beneficial iff the class word >= 2^32 -
                                     this; p = 0.003 -> 12884901; the two
                                     thresholds sum to at most 2^32            */
    float del_sigma, ben_sigma;   /* scales of |Z|, in [0, 2^20]               */
    /* any fitness model: */
    uint32_t differentia_bits;    /* 1 (0 means 1) or 8 bits per site          */
    uint32_t async_activity;      /* 0: synchronous generations.  Otherwise
                                     asynchronous ticks: on each tick an
                                     island runs a generation with
                                     probability async_activity / 2^32 and
                                     agents keep their own counters          */
    uint32_t reserved;            /* must be 0                                 */
} ga_config;

typedef struct ga_run ga_run;

/* ------------------------------------------------------------------------
 * Runs (Asynchronous Island-model Genetic Algorithm; Genome Model).
 *
 * Device state of a run, carved from the caller's arena:
 *   - two ping-pong populations, structure of arrays: trait[A], surface
 *     word planes [S/32][A] (A = w*h*N agents), and for asynchronous runs
 *     counter[A].  A synchronous run keeps no counter plane: every agent's
 *     counter is the generation count T, which the read calls report;
 *   - two ping-pong outboxes, 32 bytes reserved per island (a synchronous
 *     run's entry uses 16: direction, trait, surface words, since every
 *     emigrant's counter is the generation count);
 *   - the run's surface layout (deposit time of each site), the site
 *     rule's constant-time tables (one or two of about 25 KB, from which
 *     every deposit site and layout is looked up), and, for a synchronous
 *     run, a site schedule of max_gens_per_launch words (an asynchronous
 *     run holds a ring of the sites of its latest 4,096 ingests instead).
 * An agent record is (uint32 trait, uint32 generation counter, S one-bit
 * differentia sites); site k is bit k&31 of surface word k>>5.
 * ------------------------------------------------------------------------ */

/* Arena bytes needed by ga_create for this configuration; 0 if invalid.
 * max_gens_per_launch bounds the generations ga_step schedules at once
 * (0 selects the default of 4096; asynchronous runs ignore it).
 * Synchronous runs need no counter planes, so an asynchronous configuration
 * needs 8 bytes per agent more. */
size_t ga_footprint_bytes(const ga_config *cfg, uint32_t max_gens_per_launch);

/* Validate cfg, carve the arena (dev_arena: device pointer, 256-byte
 * aligned, arena_bytes >= ga_footprint_bytes) and enqueue the founders on
 * hip_stream: trait 0, counter 0 (stored only by asynchronous runs), all
 * sites 0, empty layout, no outboxes.
 * Founders carry no differentia; generation g's births deposit item g.
 * Errors: GA_EINVAL (struct_size not 56/80/88, S * differentia_bits not 32 or
 * 64, differentia_bits not 1/8, N = 0 or > 64, empty grid, mut_lo >
 * mut_hi, tournament not 0/2 (integer trait), above 5 (float fitness) or
 * not 0 (founder tags), migrants > 1, float thresholds summing above 2^32,
 * a scale outside [0, 2^20], reserved != 0), GA_ENOMEM
 * (arena too small), GA_EDEVICE.  *out is owned by the caller until
 * ga_destroy.                                                              */
int ga_create(const ga_config *cfg, void *dev_arena, size_t arena_bytes,
              uint32_t max_gens_per_launch, void *hip_stream, ga_run **out);

/* Enqueue n generations (the paper's main loop halts on a generation
 * count).  Each generation, island by island: immigrants from the previous
 * generation's outboxes replace random members (north, south, west, east
 * order); every slot of the next population is born from a tournament (or
 * neutral) parent, with trait mutation and one differentia written at the
 * site the surface policy picks for this generation; then a copy of a
 * random new member is posted to a random neighbour.  Returns at once.
 * Asynchronous runs (async_activity != 0; Asynchronous Island-model GA:
 * islands run their own loops and drift apart) advance n ticks instead: an
 * island active on a tick takes the emigrants its neighbours posted on the
 * previous tick and breeds, each birth depositing at the site its parent's
 * own counter selects (a constant-time lookup in the site rule's tables,
 * the same sites as hstrat_sites); an idle island keeps its members and
 * posts nothing.
 * Errors: GA_EHORIZON if generation (tick) T + n - 1 is past the site
 * rule's horizon (nothing is enqueued), GA_EINVAL if run is a pool's
 * (pools advance with ga_pool_advance), GA_EDEVICE.  After GA_EDEVICE some of the n
 * generations may be enqueued and the run's state is undefined: ga_step
 * refuses the run (GA_EDEVICE) until ga_import_state replaces its state.  */
int ga_step(ga_run *run, uint32_t n);

/* Block until all work enqueued for the run has finished. */
int ga_sync(ga_run *run);

/* Generations enqueued so far (the counter value of every agent). */
int ga_generation(const ga_run *run, uint32_t *T);

/* Blocking copy of agents [first, first + count) of the current
 * population into host buffers: trait[count], counter[count] (T for every
 * agent of a synchronous run),
 * surface_words[count * W] (agent-major, W = S * differentia_bits / 32
 * surface words per agent).  Any pointer may be NULL.
 * Errors: GA_EINVAL (range), GA_EDEVICE.                                   */
int ga_read_agents(ga_run *run, uint32_t first, uint32_t count,
                   uint32_t *trait, uint32_t *counter, uint32_t *surface_words);

/* Blocking copy of the outbox entries [first, first + count) that the next
 * generation will read: destination direction (0 north, 1 south, 2 west,
 * 3 east), and the emigrant's trait, counter and surface words (agent-
 * major).  *valid is 0 when no outbox exists yet (generation 0, or
 * migration off); the buffers are then untouched.                         */
int ga_read_outbox(ga_run *run, uint32_t first, uint32_t count,
                   uint32_t *dir, uint32_t *trait, uint32_t *counter,
                   uint32_t *surface_words, int *valid);

/* Blocking copy of the run's layout: the deposit generation held by each
 * of the S sites, GA_EMPTY_SITE if none (Distributed Phylogenetic
 * Tracking: timestamps follow from the site index and the generation
 * count); with an ingest interval n these are multiples of n.             */
int ga_read_layout(ga_run *run, uint32_t *layout);

/* Enqueue a stratified sample of the current population (Results,
 * On-hardware Trial: end-state genomes are sampled): agent k is drawn
 * uniformly from the k-th of n equal strata; if the population has at
 * most n agents, all of them are taken in order.  Writes device buffers
 * idx[n_taken], counter[n_taken], surface_words[n_taken * W]
 * (agent-major), the input layout of hstrat_mrca_bounds.  *n_taken (host)
 * is min(n, A).  Errors: GA_EINVAL (n = 0 or NULL buffers), GA_EDEVICE.    */
int ga_sample(ga_run *run, uint32_t n, uint32_t *dev_idx, uint32_t *dev_counter,
              uint32_t *dev_surface_words, uint32_t *n_taken);

/* ------------------------------------------------------------------------
 * Checkpoint and resume.  A run's state at generation (tick) T is its
 * current population and the outbox that generation T reads (Methods,
 * Asynchronous Island-model Genetic Algorithm); the layout and site table
 * follow from T and the site rule, and every random draw is a Philox block
 * of the seed and of counters the state holds.  A run resumed from an
 * exported state therefore continues exactly as the uninterrupted run.
 *
 * The state is one host blob of uint32 words (native byte order):
 *   [0] 0x53475348, [1] format version 1, [2] sizeof(ga_config), [3] T,
 *   then the run's validated ga_config (its struct_size bytes),
 *   trait[A], counter[A], the surface word planes [W][A] (plane-major),
 *   and the outbox entries [I][E] as the device holds them: E = 4 words
 *   (direction, trait, surface words, zero-padded) for a synchronous run,
 *   E = 8 (direction, trait, counter, surface words, zero-padded) for an
 *   asynchronous one; all zero when no outbox exists yet.
 * ------------------------------------------------------------------------ */

/* Bytes of the run's exported state; 0 if run is NULL. */
size_t ga_state_bytes(const ga_run *run);

/* Blocking: wait for the run's stream, then write its state at the
 * generation enqueued so far into host buffer (4-byte aligned, bytes >=
 * ga_state_bytes).  Works on runs of a pool too.
 * Errors: GA_EINVAL (NULL, short or misaligned buffer), GA_EDEVICE.        */
int ga_export_state(ga_run *run, void *host, size_t bytes);

/* Blocking: replace the state of run, which must have been created with
 * the configuration the state was exported under (compared byte for byte
 * after validation; max_gens_per_launch may differ), by the state in host.
 * The layout is rebuilt from the site rule's closed form at T (a function
 * of the scheme and T alone).  The state is checked before anything
 * is written: every counter must equal T (synchronous) or be at most T
 * (asynchronous), every outbox direction must be 0..4 and every
 * asynchronous outbox counter at most T.
 * A successful import also clears the refusal that a failed ga_step left.
 * Errors: GA_EINVAL (NULL or misaligned buffer, size, format or
 * configuration mismatch, a counter or direction outside those ranges, a
 * run of a pool),
 * GA_EHORIZON (T past the site rule's horizon + 1), GA_EDEVICE.             */
int ga_import_state(ga_run *run, const void *host, size_t bytes);

/* Release the host handle.  Does not free (or touch) the arena; work still
 * enqueued on the stream keeps using it, so sync first when reusing it.
 * A handle of a pool's run (ga_pool_run) is left alone: ga_pool_release
 * frees it; the call only records that error for ga_last_error().          */
void ga_destroy(ga_run *run);

/* Text of the calling thread's last failure ("" if none). */
const char *ga_last_error(void);

/* ------------------------------------------------------------------------
 * MRCA-generation bounds (Distributed Phylogenetic Tracking: mismatching
 * differentiae delimit the extent of common ancestry; Results, Clade
 * Reconstruction Trial: one-bit differentiae overstate relatedness).
 *
 * For annotations a, b with counters Ta, Tb: C = deposit generations
 * retained by both (ascending), t* = the first t in C where the
 * differentiae differ.
 *   ub = t*, or min(Ta, Tb) if no retained differentia differs;
 *   lb = 1 + the last t in C before t* (the last of C if no mismatch),
 *        or 0 if there is none.
 * ub never falls below the true MRCA generation; lb does only when a
 * differentia matched by chance.  An annotation against itself gives
 * (1 + its last deposit, T): (T, T) when every generation deposits.
 *
 * The plain calls take one-bit differentiae deposited every generation;
 * the _ex calls take an annotation scheme.
 * ------------------------------------------------------------------------ */

/* An annotation scheme: the surface kind, S sites of differentia_bits bits
 * each (1 with S = 32 or 64; 8 with S = 4 or 8), one deposit every
 * ingest_interval generations (the ga_config fields of the runs).          */
typedef struct hstrat_scheme {
    uint32_t kind;             /* ga_surface_kind                           */
    uint32_t sites;            /* S                                         */
    uint32_t differentia_bits; /* 1 or 8                                    */
    uint32_t ingest_interval;  /* >= 1                                      */
} hstrat_scheme;

/* Device workspace bytes hstrat_mrca_bounds needs for n annotations: the
 * flag word, ranked annotations and per-annotation layouts, then the
 * surface's site rule tables (about 51 KB), which each call uploads from
 * pinned host copies the library keeps (made on a scheme's first query)
 * and the kernels read to lay every annotation out in constant time per
 * site (Distributed Phylogenetic Tracking: deposit times follow from the
 * site index and the generation count; Surface-based Hereditary
 * Stratigraphy Algorithms: constant-time indexing).                       */
size_t hstrat_mrca_workspace_bytes(uint32_t S, uint32_t n);

/* Enqueue all n*n ordered pairs.  counter: device, n words; surface_words:
 * device, n * S/32 words, agent-major; lb, ub: device, n*n words each,
 * row-major (row a, column b); workspace: device, 256-byte aligned,
 * >= hstrat_mrca_workspace_bytes(S, n).  Annotations must share kind and S.
 * Counters may differ; when all are equal a faster route is taken on the
 * device, with identical results.  Errors: GA_EINVAL (kind, S, n = 0,
 * NULL pointers), GA_ENOMEM (workspace too small), GA_EHORIZON (a counter
 * past the horizon is reported through the flag word at the start of the
 * workspace, see hstrat_mrca_status), GA_EDEVICE.                          */
int hstrat_mrca_bounds(uint32_t kind, uint32_t S, uint32_t n,
                       const uint32_t *counter, const uint32_t *surface_words,
                       uint32_t *lb, uint32_t *ub, void *workspace,
                       size_t workspace_bytes, void *hip_stream);

/* hstrat_mrca_bounds for any annotation scheme (surface_words: n * W
 * words, W = sites * differentia_bits / 32; workspace sized by
 * hstrat_mrca_workspace_bytes(sites, n)).  Errors as hstrat_mrca_bounds,
 * plus GA_EINVAL for an invalid scheme.                                    */
int hstrat_mrca_bounds_ex(const hstrat_scheme *scheme, uint32_t n,
                          const uint32_t *counter, const uint32_t *surface_words,
                          uint32_t *lb, uint32_t *ub, void *workspace,
                          size_t workspace_bytes, void *hip_stream);

/* Host, constant time per site: the deposit generation held by each of the
 * scheme's sites in an annotation with counter T (Distributed Phylogenetic
 * Tracking: deposit times follow from the site index and the generation
 * count alone; Surface-based Hereditary Stratigraphy Algorithms: the
 * surface is indexed in constant time), GA_EMPTY_SITE for a site not
 * filled yet.  layout: host, sites words.  The same layout as replaying the
 * placements from the empty surface, computed from per-epoch tables of the
 * rule (built once per surface kind and size) in O(sites).
 * The differentia width does not enter, so any surface of 2..64 sites is
 * accepted (hybrid: an even number, at least 4).
 * Errors: GA_EINVAL (kind, sites, interval 0, NULL), GA_EHORIZON (T holds
 * an item past the horizon).                                               */
int hstrat_layout(const hstrat_scheme *scheme, uint32_t T, uint32_t *layout);

/* Host, constant time per item: the site that each of the rule's items
 * tau0 .. tau0 + n - 1 (ingest units: item tau is deposited at generation
 * tau * ingest_interval) is written to, into sites (host, n words).  The
 * same sites as placing every earlier item in turn; an asynchronous run's
 * births look sites up this way on the device.  Surfaces as for
 * hstrat_layout.  Errors: GA_EINVAL, GA_EHORIZON (an item past the
 * horizon).                                                                */
int hstrat_sites(const hstrat_scheme *scheme, uint32_t tau0, uint32_t n, uint32_t *sites);

/* Host: the MRCA-generation bounds of one pair of one-bit annotations
 * deposited every generation (Distributed Phylogenetic Tracking: two
 * annotations' mismatching differentiae delimit their common ancestry), by
 * the definition above, with the layouts of hstrat_layout.  sa, sb: host,
 * S/32 surface words each; lb, ub: host, one word each.
 * Errors: GA_EINVAL (kind, S, NULL), GA_EHORIZON.                          */
int hstrat_mrca_bounds_pair(uint32_t kind, uint32_t S, uint32_t Ta, const uint32_t *sa,
                            uint32_t Tb, const uint32_t *sb, uint32_t *lb, uint32_t *ub);

/* hstrat_mrca_bounds_pair for any annotation scheme (sa, sb: W = sites *
 * differentia_bits / 32 words each).                                       */
int hstrat_mrca_bounds_pair_ex(const hstrat_scheme *scheme, uint32_t Ta, const uint32_t *sa,
                               uint32_t Tb, const uint32_t *sb, uint32_t *lb, uint32_t *ub);

/* hstrat_mrca_bounds without a workspace, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  The workspace is a static device array
 * of 1,345,536 bytes that the library holds on every device it runs on
 * until the process ends; this call allocates nothing.  Results are those
 * of hstrat_mrca_bounds, except that a counter past the site rule's horizon
 * (which hstrat_mrca_status would report) makes every lb and ub 0xFFFFFFFF,
 * a value no bound takes.  Having no room for the site rule's tables, the
 * kernels replay each layout one placement per ingest, so counters must
 * stay at or below 2^24 ingests (above, the same 0xFFFFFFFF).
 * n <= 4096; the current device must be the one
 * hip_stream and the buffers belong to.  Every call on a device shares that
 * device's array, so calls that overlap on one device race: order them on
 * one stream or synchronise between them.
 * Errors: GA_EINVAL (kind, S, n = 0 or n > 4096, NULL pointers), GA_EDEVICE. */
int hstrat_mrca_bounds_noalloc(uint32_t kind, uint32_t S, uint32_t n,
                               const uint32_t *counter, const uint32_t *surface_words,
                               uint32_t *lb, uint32_t *ub, void *hip_stream);

/* Blocking: status of the last hstrat_mrca_bounds run on this workspace
 * (GA_OK, or GA_EHORIZON when a counter was past the horizon, in which
 * case lb/ub are unspecified).                                             */
int hstrat_mrca_status(const void *workspace, void *hip_stream);

/* ------------------------------------------------------------------------
 * Trie reconstruction and phylometrics (Distributed Phylogenetic Tracking:
 * the record of differentiae turns reconstruction into trie building;
 * Results, On-hardware Trial: treatments compared by sum branch length and
 * mean evolutionary distinctiveness).
 *
 * For n annotations sharing one counter T: each annotation is read as its
 * bits in ascending deposit time (t_0 < ... < t_{F-1}, the retained times)
 * and inserted into a binary trie.  A branching trie node whose subtrees
 * split on the bit of t_d is a tree node at time t_d (the MRCA upper bound
 * of every pair it separates); identical annotations hang from one node at
 * T; annotations are leaves at T; one-child chains are collapsed; the root
 * is the first branching node.
 * ------------------------------------------------------------------------ */

/* Device workspace bytes of hstrat_phylo_metrics for n annotations (as
 * for hstrat_mrca_workspace_bytes, the site rule tables included).       */
size_t hstrat_phylo_workspace_bytes(uint32_t S, uint32_t n);

/* Enqueue the reconstruction.  counter, surface_words: as for
 * hstrat_mrca_bounds (n <= 65535).  out: device, 8 uint64 words:
 *   [0] sum of branch lengths,
 *   [1] sum over unordered pairs of (T - the time of their tree MRCA),
 *   [2] root time, [3] internal nodes,
 *   [4] status: 0 ok, 1 counters differ (not reconstructed), 2 past the
 *       horizon, [5] n,
 *   [6] mean evolutionary distinctiveness (fair proportion: [0] / n), and
 *   [7] mean pairwise distance (2 * [1] / (n(n-1)/2); 0 when n = 1), both
 *       the bits of a binary64 value; 0 when status is not 0.
 * Errors: GA_EINVAL, GA_ENOMEM (workspace), GA_EDEVICE.                    */
int hstrat_phylo_metrics(uint32_t kind, uint32_t S, uint32_t n,
                         const uint32_t *counter, const uint32_t *surface_words,
                         uint64_t *out, void *workspace, size_t workspace_bytes,
                         void *hip_stream);

/* hstrat_phylo_metrics for any annotation scheme.  With byte differentiae
 * a trie node can split many ways (one tree node per distinct value).     */
int hstrat_phylo_metrics_ex(const hstrat_scheme *scheme, uint32_t n,
                            const uint32_t *counter, const uint32_t *surface_words,
                            uint64_t *out, void *workspace, size_t workspace_bytes,
                            void *hip_stream);

/* The reconstructed tree itself (same reconstruction and the same six
 * result words in out).  Tree nodes are named by boundary indices in
 * [0, n-1): leaf_parent (device, n words): the node each annotation hangs
 * from (0xFFFFFFFF: n = 1, the annotation is the whole tree);
 * node_parent (device, n-1 words): for a boundary naming a node, its
 * parent node (0xFFFFFFFF for the root), 0xFFFFFFFE for a boundary that
 * names no node; node_time (device, n-1 words): the time of the boundary's
 * node (the MRCA upper bound of the annotations it separates; T for a
 * polytomy of identical annotations).  Leaves sit at T.  Contents are
 * unspecified when out[4] (status) is not 0.  Errors as
 * hstrat_phylo_metrics_ex.                                                  */
int hstrat_phylo_tree_ex(const hstrat_scheme *scheme, uint32_t n,
                         const uint32_t *counter, const uint32_t *surface_words,
                         uint32_t *leaf_parent, uint32_t *node_parent, uint32_t *node_time,
                         uint64_t *out, void *workspace, size_t workspace_bytes,
                         void *hip_stream);

/* Host: the tree of hstrat_phylo_tree_ex (leaf_parent, node_parent,
 * node_time: host copies, n and n - 1 words; T: the annotations' counter)
 * as canonical Newick text: leaves named by annotation index, branch
 * lengths in generations, children ordered by the smallest annotation
 * index below them, no length on the root, "0;" when n = 1.  *length
 * receives the text's length; text (host, cap bytes, may be NULL to size
 * it) receives the text and a terminating NUL.
 * Errors: GA_EINVAL (NULL, n = 0, parents out of range or not one tree,
 * a leaf hanging from a boundary that names no node, a node time below its
 * parent's or above T),
 * GA_ENOMEM (cap too small).                                               */
int hstrat_phylo_newick(uint32_t n, uint32_t T, const uint32_t *leaf_parent,
                        const uint32_t *node_parent, const uint32_t *node_time, char *text,
                        size_t cap, size_t *length);

/* Queries on annotations taken from a run (typically its ga_sample), with
 * the run's own annotation scheme, enqueued on the run's stream.  Results
 * are those of hstrat_mrca_bounds_ex and hstrat_phylo_tree_ex.  A layout
 * is a function of the scheme and the generation count alone (Distributed
 * Phylogenetic Tracking: deposit times follow from the site index and the
 * count).  So when every counter equals the run's generation count T, the
 * run's own layout at T is used as it stands.  Otherwise (a sample taken
 * before later steps, drifted asynchronous counters) the query lays each
 * annotation out from the site rule's tables the run holds in its arena;
 * both give the same words.  The workspace is sized as for the hstrat_
 * calls (its table region is not used).  ga_phylo_tree with leaf_parent
 * NULL computes the metrics only (node_parent and node_time unused).
 * Errors as the hstrat_ calls, and GA_EINVAL for a NULL run.               */
int ga_mrca_bounds(ga_run *run, uint32_t n, const uint32_t *counter,
                   const uint32_t *surface_words, uint32_t *lb, uint32_t *ub,
                   void *workspace, size_t workspace_bytes);

int ga_phylo_tree(ga_run *run, uint32_t n, const uint32_t *counter,
                  const uint32_t *surface_words, uint32_t *leaf_parent,
                  uint32_t *node_parent, uint32_t *node_time, uint64_t *out,
                  void *workspace, size_t workspace_bytes);

/* ------------------------------------------------------------------------
 * Batched and served runs: a pool of runs of any sizes, surfaces and
 * treatments sharing one caller-owned device arena and one stream.  An
 * advance enqueues one site-schedule launch for all active runs, then per
 * generation one step launch for each of two groups of runs of about equal
 * bytes (one group when a generation reads fewer trait and surface words
 * than the split size, ga_pool_set_split); each run takes the same steps
 * as under ga_step, so its results are identical to running it alone.  A
 * launch deals every run's tiles evenly over the chip's 8 XCDs, one
 * contiguous chunk per XCD.  When both groups hold runs, the second group's launches go to a stream the pool
 * creates, forked from the pool's stream after the site schedules and
 * joined back to it at the end of the advance, so that the groups run side
 * by side.  Admission is by footprint: a run gets a first-fit range of the
 * arena or is refused.  Runs are identified by small integer ids, reused
 * after release.  All work is ordered on the pool's stream: work enqueued
 * on it after an advance sees that advance complete.
 * ------------------------------------------------------------------------ */
typedef struct ga_pool ga_pool;

/* Arena bytes the pool keeps for its own tables (max_runs <= 256). */
size_t ga_pool_overhead_bytes(uint32_t max_runs);

/* dev_arena: device, 256-byte aligned, at least ga_pool_overhead_bytes;
 * the rest holds runs.  max_gens_per_launch caps the generations of one
 * advance (0: 4096) and sizes each run's site schedule.  hip_stream must
 * be a created stream (not the null stream) for hipGraph replay.
 * Errors: GA_EINVAL, GA_ENOMEM (arena below the overhead), GA_EDEVICE.    */
int ga_pool_create(void *dev_arena, size_t arena_bytes, uint32_t max_runs,
                   uint32_t max_gens_per_launch, void *hip_stream, ga_pool **out);

/* Arena bytes a run of cfg takes in this pool (0 if cfg is invalid). */
size_t ga_pool_footprint(const ga_pool *pool, const ga_config *cfg);

/* Admit a run of cfg that stops after n_generations and enqueue its
 * founders.  Errors: GA_EINVAL (cfg, n = 0), GA_EHORIZON (n past the
 * site rule's horizon), GA_EBUSY (no free slot or no free range of its
 * footprint; nothing is changed).                                          */
int ga_pool_admit(ga_pool *pool, const ga_config *cfg, uint32_t n_generations,
                  uint32_t *id);

/* Enqueue up to max_gens generations of every admitted run that has not
 * reached its generation count; *gens_enqueued (may be NULL) receives the
 * largest number enqueued for any run (0 when none is active).  Errors:
 * GA_EINVAL (a run's tile does not fit), GA_EDEVICE (a launch failed; some
 * generations may be enqueued, and every later advance of this pool
 * returns GA_EDEVICE).                                                    */
int ga_pool_advance(ga_pool *pool, uint32_t max_gens, uint32_t *gens_enqueued);

/* Ids of runs whose last generation has been enqueued and that were not
 * reported before (at most cap).  Work enqueued later on the pool's stream
 * (ga_sample, hstrat_mrca_bounds) sees their final state; host reads
 * block until it is reached.                                              */
int ga_pool_poll(ga_pool *pool, uint32_t *ids, uint32_t cap, uint32_t *n);

/* The run handle of an admitted run, owned by the pool until release: use
 * it with ga_generation, ga_read_agents, ga_read_outbox, ga_read_layout,
 * ga_sample (not with ga_step or ga_destroy).                              */
int ga_pool_run(ga_pool *pool, uint32_t id, ga_run **run);

/* Return the run's arena range and slot.  Work already enqueued on the
 * pool's stream completes first; later runs reuse the memory after it.    */
int ga_pool_release(ga_pool *pool, uint32_t id);

/* Block until all work enqueued on the pool's stream has finished. */
int ga_pool_sync(ga_pool *pool);

/* Workgroup size of batched step launches (multiple of 64, 64..256; 0
 * keeps it) and whether an advance replays a captured hipGraph of its
 * launches when the run set's launch shape repeats (1) or launches
 * directly (0).                                                            */
int ga_pool_set_launch(ga_pool *pool, uint32_t block_threads, int use_graph);

/* Split size: an advance whose runs read at least min_words trait and
 * surface words per generation (summed over the active runs) splits them
 * into its two launch groups; smaller ones launch as one group.  Default
 * 4 Mi words (16 MiB): below it a generation's launch is short and a
 * second launch per generation costs more than it hides.  0 always splits
 * (two or more active runs).  Results do not depend on it.
 * Errors: GA_EINVAL.                                                      */
int ga_pool_set_split(ga_pool *pool, uint64_t min_words);

/* Occupancy: active runs, admitted runs, free bytes, largest free range. */
int ga_pool_info(const ga_pool *pool, uint32_t *active, uint32_t *admitted,
                 size_t *free_bytes, size_t *largest_free);

/* Wait for the work enqueued on the pool's stream, then release every run,
 * the pool's own stream and events, and its host state; the arena is
 * untouched.                                                              */
void ga_pool_destroy(ga_pool *pool);

/* ------------------------------------------------------------------------
 * Instrumentation
 * ------------------------------------------------------------------------ */

/* Enable (1) or disable (0) HIP-event timing of the step kernel launches
 * of this run.  Events bracket each batch of consecutive step launches on
 * the run's stream.                                                        */
int ga_set_kernel_timing(ga_run *run, int enable);

/* Blocking: total milliseconds and number of generations stepped by the
 * timed step-kernel launches since timing was enabled (or last reset with
 * reset = 1); a launch of the resident form counts its generations.       */
int ga_kernel_time(ga_run *run, double *ms, uint64_t *launches, int reset);

/* A plain device-to-device copy of `bytes` bytes (multiple of 16; both
 * pointers 16-byte aligned), one 16-byte load and store per thread, with
 * the non-temporal hint.  Not part of the method: it measures the attainable HBM bandwidth
 * next to the step kernel and calibrates hardware byte counters against a
 * kernel of known traffic.  Enqueued on hip_stream.  Errors: GA_EINVAL.   */
int ga_probe_copy(const void *src, void *dst, size_t bytes, void *hip_stream);

/* Launch shape of the step kernel: threads per workgroup (multiple of 64,
 * 64..1024) and agents per thread (1, 2 or 4; must divide pop_per_island;
 * 4 gives 16-byte population loads and stores).  A workgroup handles a
 * tile of block_threads * agents_per_thread / N whole islands staged in
 * LDS (at most 64 KiB).  0 keeps the current value.  Results do not depend
 * on the shape.  A run starts at 4 agents per thread when N allows, with
 * 64 threads for synchronous integer births on two-word surfaces, 128 for
 * integer births on one-word surfaces or in asynchronous ticks, and 256
 * for float births.
 * Errors: GA_EINVAL.                                                       */
int ga_set_launch_shape(ga_run *run, uint32_t block_threads,
                        uint32_t agents_per_thread);

/* The resident form of a small synchronous run (on by default): when the
 * whole torus fits one workgroup's tile (at most 4,096 agents at the run's
 * agents per thread, on the fewest multiple of 64 threads that holds them,
 * within 64 KiB of LDS), each launch batch of ga_step is one launch of one
 * workgroup that takes the run through every generation of the batch,
 * with a workgroup barrier between generations instead of a kernel
 * boundary.  Results are the same as one launch per generation, which
 * enable = 0 selects (the launch shape above then applies).  Asynchronous
 * runs and runs of a pool never step resident.  Errors: GA_EINVAL.         */
int ga_set_resident(ga_run *run, int enable);

/* *threads = the resident form's workgroup size for this run, or 0 when
 * the run steps one launch per generation.  Errors: GA_EINVAL.            */
int ga_resident_threads(const ga_run *run, uint32_t *threads);

#ifdef __cplusplus
}
#endif

#endif /* HSGA_H */
