/*
 * motifs.h -- C ABI of the MI355X Motifs-k library (libmotifs.so).
 *
 * Problem Motifs-k (arXiv 1804.09741, Section 1): given a directed graph G
 * and k, count the connected induced k-vertex subgraphs of G grouped by
 * isomorphism class; the result is the histogram H_k(G).  This library
 * solves it for k = 3..6 on one AMD Instinct MI355X (gfx950):
 *
 *   - mk_table_*   the code -> class table of Section 3.2 (isomorphism in
 *                  O(1) by precomputing the class of every adjacency matrix);
 *   - mk_count*,
 *     mk_batch_*   the histograms of one graph or a batch of graphs, by
 *                  enumeration of every connected induced k-set exactly once
 *                  (its adjacency code, the table lookup) or by Section 3's
 *                  counting from the connected (k-2)-sets (MK_METHOD_*);
 *   - mk_server_*  a continuous-batching request server over the same path;
 *   - mk_count7    H_7 (k = 7), classes reported by canonical code;
 *   - mk_randomise,
 *     mk_significance  the ensemble of random graphs and the z-score of each
 *                  class against it (Section 1's steps (a) and (c)).
 *
 * Conventions used throughout:
 *
 *   Graph input.  A simple digraph as out-adjacency CSR: vertices 0..n-1,
 *   row_ptr[n+1] (row_ptr[0] = 0, non-decreasing), col[row_ptr[n]] with the
 *   heads of the arcs leaving each vertex, in any order.  m = row_ptr[n]
 *   counts directed arcs, so a bidirected edge (u,v),(v,u) of Section 2
 *   counts twice.  Self-loops and repeated arcs are rejected (an adjacency
 *   code cannot represent them).
 *
 *   Connectivity.  Weak: delta(v) = A(v) u B(v) u C(v) ignores direction
 *   (Section 2).  This is the reading that gives the paper's class counts.
 *
 *   Adjacency code.  For an ordered k-tuple (s_0..s_{k-1}) the code has bit
 *   i*(k-1) + j - [j > i] set iff arc s_i -> s_j exists (row-major adjacency
 *   matrix without its diagonal; k(k-1) bits).
 *
 *   Class id.  0-based rank of the class's canonical code (the minimum code
 *   over all k! relabelings) among the weakly connected classes.  Id 0 is
 *   the out-star (code 2^(k-1) - 1), the last id the complete digraph.
 *   Number of classes: 13, 199, 9364, 1530843 for k = 3..6.  (Section 1
 *   prints 1,530,842 for k = 6; Burnside's lemma and the paper's own k = 7
 *   figure fix it at 1,530,843, which is what the table holds.)
 *   Codes of disconnected digraphs map to MK_INVALID_CLASS.
 *
 *   Histogram.  Dense uint64 vector of num_classes counts indexed by class
 *   id, zeros included.  Counts are exact; results do not depend on thread
 *   timing.
 *
 * Ownership.  Handles are opaque and owned by the library.  Graphs and
 * batches are freed by their *_free call; class tables belong to the
 * context that built them and live until mk_table_release or mk_destroy.
 * Caller arrays are only read during the call that receives them.
 *
 * Errors.  Every int-returning call returns MK_OK (0) or a negative MK_E*
 * status; mk_last_error() then describes the failure (per thread).
 * Calls on one context are serialised internally (thread-safe, not
 * concurrent).
 */
#ifndef MOTIFS_H
#define MOTIFS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MK_OK 0
#define MK_EINVAL (-1)    /* bad argument: NULL pointer, negative size, wrong table */
#define MK_ERANGE (-2)    /* k outside 3..6, id/code out of range, graph too large */
#define MK_EGRAPH (-3)    /* input is not a simple digraph CSR */
#define MK_ENOMEM (-4)    /* device or host allocation failed */
#define MK_EDEVICE (-5)   /* HIP runtime error or a failed device-side check */
#define MK_EBUSY (-6)     /* request can never fit the server budget / server stopped */
#define MK_ETIMEDOUT (-7) /* mk_wait timed out; the request stays pending */
#define MK_ENOTFOUND (-8) /* unknown or already collected ticket */

#define MK_INVALID_CLASS 0xFFFFFFFFu

/* Largest graph the library accepts: n <= MK_MAX_VERTICES and undirected
   degree (|delta(v)|) <= MK_MAX_DEGREE.  The paper's graphs have n <= 6175.
   Batches whose graphs all have n <= MK_LDS_MARKS_MAX_VERTICES keep each
   wave's per-vertex marks in LDS; larger ones keep them in device memory
   (MK_MARKS_GLOBAL, slower), count by enumeration only, and test arcs on the
   sorted lists (MK_ADJ_LISTS).  mk_randomise takes graphs up to
   MK_LDS_MARKS_MAX_VERTICES vertices. */
#define MK_MAX_VERTICES (1 << 20)
#define MK_MAX_DEGREE 4096
#define MK_LDS_MARKS_MAX_VERTICES 8192

typedef struct mk_ctx mk_ctx;
typedef struct mk_graph mk_graph;
typedef struct mk_table mk_table;
typedef struct mk_batch mk_batch;
typedef struct mk_server mk_server;

/* ---------------------------------------------------------------- context */

/* Open a context on HIP device `device`.  *out receives the handle. */
int mk_init(int device, mk_ctx **out);

/* Free the context, its class tables and its stream.  Graphs, batches and
   servers made from it must be freed first. */
void mk_destroy(mk_ctx *ctx);

/* Number of compute units of the context's device (for reports). */
int mk_device_info(const mk_ctx *ctx, int32_t *compute_units, int64_t *hbm_bytes);

/* ------------------------------------------------------------------ graph */

/* Validate the simple digraph (n, row_ptr, col) (see "Graph input" above)
   and copy it to device memory.  The caller keeps its arrays.  Errors:
   MK_EINVAL for NULL arrays or n < 0, MK_EGRAPH for a non-monotone row_ptr,
   ids outside [0,n), self-loops or repeated arcs, MK_ERANGE for
   n > MK_MAX_VERTICES or a vertex whose undirected degree exceeds
   MK_MAX_DEGREE. */
int mk_graph_load_csr(mk_ctx *ctx, int32_t n, const int32_t *row_ptr,
                      const int32_t *col, mk_graph **out);

/* n, m (directed arcs) and the largest undirected degree of a loaded graph;
   any output pointer may be NULL. */
int mk_graph_info(const mk_graph *g, int32_t *n, int64_t *m, int32_t *max_degree);

/* Device bytes one count of this graph needs beyond the graph itself
   (workspace, work units, histogram) for subgraph size k. */
int mk_graph_footprint(const mk_graph *g, int k, uint64_t *bytes);

void mk_graph_free(mk_graph *g);

/* Copy a graph's out-adjacency CSR back to host memory: row_ptr (n+1) and
   col (m), either may be NULL.  Blocks. */
int mk_graph_read(const mk_graph *g, int32_t *row_ptr, int32_t *col);

/* ------------------------------------------------------- random ensembles */

/* The ensemble of random graphs of Section 1 (subgraph counts of a graph are
   compared with those of random graphs; the paper does not fix the model).
   Makes `count` degree-preserving random versions of g on the device, each
   by directed switches: arcs a -> b and c -> d become a -> d and c -> b
   unless a = c, b = d, a = d, c = b or a -> d or c -> b exists.  Graph r
   draws its arc pairs from SplitMix64 (Steele, Lea and Flood, 2014) seeded
   with output r of SplitMix64(seed): attempt t uses outputs 2t and 2t+1,
   each mapped to an arc index as (high 32 bits * m) >> 32.  A graph stops
   after switches_per_arc * m accepted switches or 8 * that + 1024 attempts;
   accepted (may be NULL) receives each graph's accepted count.  Every arc
   keeps its CSR position, so out- and in-degrees are kept exactly.  out
   receives `count` new graphs (free each with mk_graph_free); on error none
   is left.  MK_ERANGE if g has more than MK_LDS_MARKS_MAX_VERTICES vertices
   or a random graph's undirected degree exceeds MK_MAX_DEGREE.  Blocks until
   the graphs are ready. */
int mk_randomise(mk_ctx *ctx, const mk_graph *g, int32_t count, uint64_t seed,
                 uint32_t switches_per_arc, mk_graph **out, uint64_t *accepted);

/* Significance of every class against an ensemble (Section 1, step (c); the
   paper names no statistic: this is the usual z-score).  d_hist: device
   array of ng x num_classes uint64 histograms, row 0 the original graph and
   rows 1..ng-1 its random graphs (ng >= 3).  d_out: device array of
   3 x num_classes float64 receiving, per class, the mean and the sample
   standard deviation (divisor ng - 2) of the random graphs' counts and
   z = (H_0 - mean) / std (0 if std = 0 and H_0 = mean, +-infinity if std = 0
   otherwise).  Enqueued on `stream` (NULL: the context's stream). */
int mk_significance(mk_ctx *ctx, const uint64_t *d_hist, int32_t ng, uint32_t num_classes,
                    double *d_out, void *stream);

/* ------------------------------------------------------------ class table */

/* The code -> class table for k (Section 3.2): 2^(k(k-1)) uint32 entries in
   device memory (k = 6: 2^30 entries, 4 GiB), built on the GPU by taking
   the minimum code over all k! vertex relabelings of every code.  Built
   once per context and k, then cached; later calls return the same handle.
   MK_ERANGE for k outside 3..6. */
int mk_table_build(mk_ctx *ctx, int k, mk_table **out);

/* Drop the cached table for k (frees its device memory).  Handles obtained
   earlier become invalid. */
int mk_table_release(mk_ctx *ctx, int k);

/* k, number of classes, number of entries (2^(k(k-1))) and the GPU build
   time in milliseconds; any output pointer may be NULL. */
int mk_table_info(const mk_table *t, int32_t *k, uint32_t *num_classes,
                  uint64_t *num_entries, double *build_ms);

/* Canonical code of class `id` (MK_ERANGE if id >= num_classes). */
int mk_table_class_code(const mk_table *t, uint32_t id, uint32_t *canon_code);

/* All canonical codes in id order (ascending) into codes[capacity];
   MK_ERANGE if capacity < num_classes. */
int mk_table_class_codes(const mk_table *t, uint32_t *codes, uint32_t capacity);

/* Class id of one code (MK_INVALID_CLASS if the digraph is disconnected);
   MK_ERANGE if code >= 2^(k(k-1)). */
int mk_table_lookup(const mk_table *t, uint32_t code, uint32_t *id);

/* Copy entries [first, first+count) of the table to host memory out[]. */
int mk_table_read(const mk_table *t, uint64_t first, uint64_t count, uint32_t *out);

/* Cores per class, classes [first, first+count) into out (host, count
   bytes).  A core of a connected k-vertex digraph is a subset of k-2 of its
   vertices that induces a weakly connected subgraph and that both other
   vertices touch (an arc either way to some vertex of the subset).  Counting
   H_k from the connected (k-2)-sets (Section 3: every pair of vertices of
   adj(X) closes a k-set with X) reaches each k-set once per core, so these
   are the divisors of that count (1..k(k-1)/2; the paper leaves them
   implicit).  MK_ERANGE if the range leaves the classes. */
int mk_table_core_mult(const mk_table *t, uint32_t first, uint32_t count, uint8_t *out);

/* ------------------------------------------------------------------ count */

/* H_k(G) for one graph (k = the table's k).  hist: host array of
   num_classes uint64 written densely; *total (may be NULL) receives the
   number of connected induced k-subgraphs (the sum of hist).  A graph with
   n < k gives all zeros.  Blocks until done. */
int mk_count(mk_ctx *ctx, const mk_graph *g, const mk_table *t, uint64_t *hist,
             uint64_t *total);

/* H_k of ng graphs in one persistent launch.  hist: host array of
   ng * num_classes uint64, graph i at hist + i*num_classes; totals (may be
   NULL): ng uint64.  Equal, graph by graph, to mk_count.  Blocks. */
int mk_count_batch(mk_ctx *ctx, const mk_graph *const *gs, int32_t ng,
                   const mk_table *t, uint64_t *hist, uint64_t *totals);

/* ----------------------------------------------------------- prepared batch */

/* Tuning knobs of a batch.  Zero fields take the library defaults. */
typedef struct mk_batch_opts {
    uint64_t split_threshold; /* floor of the estimated subgraphs per work
                                 unit (the planner raises it so that the
                                 whole batch makes about units_per_wave
                                 units per wave); 0: 512 for k = 6 by
                                 enumeration, 1024 for k = 5 by counting
                                 from (k-2)-sets and k = 4 by enumeration,
                                 else 4096 (nodes planned for sets of 3 or
                                 fewer vertices are not split) */
    int32_t waves_per_cu;     /* resident enumeration waves per compute unit */
    int32_t use_graph;        /* 1 (default): the preparation replayed as a
                                 captured hipGraph, the counting kernel
                                 launched between its timing events;
                                 2: the whole pass (preparation, counting
                                 kernel, finish) as one captured hipGraph,
                                 mk_batch_timing then gives the pass time
                                 only; -1: plain stream launches */
    int32_t units_per_grab;   /* work units a wave takes per queue atomic
                                 (0: about 1/32 of a wave's share, <= 16) */
    int32_t units_per_wave;   /* work-unit granularity: the planner splits
                                 nodes until the batch's estimated work
                                 makes about this many units per counting
                                 wave (0: 32, 128 for graphs counted on
                                 sorted lists, 16 for k = 7; 1..4096) */
    int32_t method;           /* MK_METHOD_*: how H_k is counted (0: the
                                 library's choice); results are the same */
    int32_t adjacency;        /* MK_ADJ_*: how arcs between extension
                                 vertices are tested (0: the library's
                                 choice); results are the same */
    int32_t marks;            /* MK_MARKS_*: where each wave keeps its
                                 per-vertex marks (0: the library's choice);
                                 results are the same */
} mk_batch_opts;

/* Counting methods of a batch.
   MK_METHOD_ESU: every connected k-set is enumerated once (ESU) and its
     adjacency code looked up in the class table (Section 3.2).
   MK_METHOD_CORES: Section 3's loop over the connected (k-2)-sets X: the
     vertices of adj(X) are grouped into cells by their relation to each
     member (Section 2); each pair of cells adds C(|Y|,2) or |Y||Z| k-sets
     of one class at once, each arc inside adj(X) moves one k-set to its
     true class, and the sums are divided by the cores per class
     (mk_table_core_mult). */
/* MK_METHOD_AUTO: MK_METHOD_CORES for k <= 5, MK_METHOD_ESU for k = 6 and
   for graphs with more than MK_LDS_MARKS_MAX_VERTICES vertices (which
   MK_METHOD_CORES rejects with MK_ERANGE). */
#define MK_METHOD_AUTO 0
#define MK_METHOD_ESU 1
#define MK_METHOD_CORES 2

/* Arc tests between two extension vertices w, u in the last two levels of
   the enumeration (the pair test of Section 3.1's Algorithm 2; the rest of
   the code comes from marks left by scanning the members' lists, as in its
   Algorithm 3).
   MK_ADJ_BITS: two n x n bit matrices (out- and in-arcs) per graph, built
     each pass; one bit read per test; the typed lists are built from them.
   MK_ADJ_LISTS: no bit matrix: the typed lists are built by sorting each
     vertex's out- and in-arcs, and a test is a binary search in the shorter
     of the two vertices' lists (the degree split of Algorithms 4 and 5).
   MK_ADJ_AUTO: MK_ADJ_BITS while every graph has n <=
     MK_LDS_MARKS_MAX_VERTICES, else MK_ADJ_LISTS. */
#define MK_ADJ_AUTO 0
#define MK_ADJ_BITS 1
#define MK_ADJ_LISTS 2

/* Per-vertex marks of each wave (every vertex's relation to the current
   members).
   MK_MARKS_LDS: in LDS, 2 bytes per vertex for k <= 5 and 4 for k = 6;
     needs n <= MK_LDS_MARKS_MAX_VERTICES.
   MK_MARKS_GLOBAL: a private n-entry array per wave in device memory, 4
     bytes per vertex (kept zero between work units; fewer waves when they
     would take more than 1/16 of the device memory); needs MK_ADJ_LISTS and
     MK_METHOD_ESU.
   MK_MARKS_AUTO: MK_MARKS_LDS when the graphs fit, else MK_MARKS_GLOBAL. */
#define MK_MARKS_AUTO 0
#define MK_MARKS_LDS 1
#define MK_MARKS_GLOBAL 2

/* Prepare a batch: device workspace for the typed adjacency, the work
   units and the histograms of ng graphs (counted with table t), sized by
   running the planner once.  The graphs and the table must outlive it. */
int mk_batch_create(mk_ctx *ctx, const mk_graph *const *gs, int32_t ng,
                    const mk_table *t, const mk_batch_opts *opts, mk_batch **out);

/* Enqueue one full pass of the path on `stream` (a hipStream_t; NULL = the
   context's stream): typed adjacency, work-unit plan, enumeration, codes,
   lookups and histograms.  Asynchronous.  d_hist: device array of
   ng * num_classes uint64 that receives the histograms (overwritten), or
   NULL to use the batch's own buffer.  The first run on a given d_hist
   captures the sequence as a hipGraph (see mk_batch_opts.use_graph); later
   runs replay it. */
int mk_batch_run(mk_batch *b, uint64_t *d_hist, void *stream);

/* Wait for the batch's last run, check its device-side status and copy the
   histograms (ng * num_classes) and per-graph totals to host memory (either
   pointer may be NULL). */
int mk_batch_read(mk_batch *b, uint64_t *hist, uint64_t *totals);

/* Statistics of the last plan: number of work units, of split pairs, the
   enumeration grid (workgroups of one 64-lane wave) and its LDS bytes per
   workgroup. */
typedef struct mk_batch_stats {
    uint64_t units;
    uint64_t split_pairs;
    int32_t grid;
    int32_t lds_bytes;
    int32_t k;
    int32_t ng;
    int32_t method;           /* the MK_METHOD_* the batch runs */
    int32_t adjacency;        /* the MK_ADJ_* it runs */
    int32_t marks;            /* the MK_MARKS_* it runs */
} mk_batch_stats;
int mk_batch_stats_get(const mk_batch *b, mk_batch_stats *out);

/* GPU time of the batch's last run, from HIP events recorded on the run's
   stream: the whole pass and the counting kernel alone (milliseconds; -1
   for the kernel when the whole pass is one graph, use_graph = 2).  Waits
   for the run to finish. */
int mk_batch_timing(mk_batch *b, double *pass_ms, double *enum_ms);

void mk_batch_free(mk_batch *b);

/* For callers that cannot allocate device memory (code under HIP graph
   capture, tight serving loops, harnesses that forbid hipMalloc): H_k of one
   graph by enumeration, equal to mk_count's histogram, with every buffer of
   the path other than the caller's -- counters, typed adjacency, bit
   matrices, planner slots and work units -- taken from one static device
   array of mk_static_scratch_bytes() bytes (64 MiB) that the library holds
   on each device it runs on until the process ends.  No hipMalloc, hipFree
   or allocating library call is made.  g: a loaded graph with n <=
   MK_LDS_MARKS_MAX_VERTICES whose workspace fits the array (about 8 n^2/32 +
   24 |delta| bytes plus the work units), else MK_ERANGE with a message
   giving the size needed.  t: a built table (k = 3..6).  d_hist: device
   array of t's num_classes uint64, overwritten with the histogram.  Runs on
   `stream` (NULL: the context's stream) and blocks until done, then checks
   the device-side status; work the caller queued on another stream that
   writes d_hist must be ordered before the call (else it can overwrite the
   result).  Calls through one context are serialised; calls
   from two contexts on one device at the same time share the array and
   race. */
int mk_count_static(mk_ctx *ctx, const mk_graph *g, const mk_table *t, uint64_t *d_hist,
                    void *stream);

/* Size in bytes of the static device array of mk_count_static. */
uint64_t mk_static_scratch_bytes(void);

/* H_7 of ng graphs.  Section 1 counts 880,471,142 classes of 7-vertex
   digraphs, too many for a table of all 2^42 codes, so classes are reported
   by canonical code: the minimum adjacency code over the 5040 relabelings
   (the rule behind the k <= 6 class ids).  The subgraphs are enumerated as
   for k <= 6 (graphs past MK_LDS_MARKS_MAX_VERTICES vertices with marks in
   device memory and arc tests on the sorted lists) and canonicalised on the
   device.  For graph g, n_classes[g] receives the number of distinct
   classes; the first min(n_classes[g], cap) of them, ascending, go to
   codes[g * cap + i] with their counts in counts[g * cap + i].  totals[g]
   (may be NULL) receives the number of connected 7-sets; kernel_ms (may be
   NULL) the counting kernel's time.  MK_ERANGE when a graph has more than
   cap classes (n_classes is still filled).  Blocks.  The first call on a
   context allocates a cache of 2^22 canonical codes (64 MiB) that the
   context keeps (and mk_destroy frees), so later calls skip the codes
   already canonicalised (see mk_k7_cache_info). */
int mk_count7(mk_ctx *ctx, const mk_graph *const *gs, int32_t ng, int64_t cap,
              uint64_t *codes, uint64_t *counts, int64_t *n_classes, uint64_t *totals,
              double *kernel_ms);

/* The canonical-code cache of mk_count7: its number of slots (0 before the
   context's first k = 7 count) and how many hold a code.  mk_count7 clears
   it by itself before a count once more than half of the slots are used
   (long probes, codes no longer entered). */
int mk_k7_cache_info(mk_ctx *ctx, uint64_t *slots, uint64_t *used);

/* Empty the canonical-code cache of mk_count7 (the next count starts cold).
   Blocks. */
int mk_k7_cache_clear(mk_ctx *ctx);

/* Autotuner: time the batch path on these graphs (best of `trials` runs
   each) under candidate settings -- counting method, arc tests, work-unit
   granularity (split floors 128 .. 2^18 estimated subgraphs per unit and
   4 .. 128 units per wave, two passes), units per queue grab, waves per CU,
   tried one knob at a time from the library defaults -- and return the
   fastest in *best, its whole-pass time (preparation, counting and, for
   MK_METHOD_CORES, the division) in *best_ms and the defaults' in
   *default_ms (either may be NULL).  Every candidate's histograms must
   equal the defaults' (MK_EDEVICE otherwise).  Allocates and frees its own
   batches; takes as long as about 35 runs of the batch. */
int mk_autotune(mk_ctx *ctx, const mk_graph *const *gs, int32_t ng, const mk_table *t,
                int32_t trials, mk_batch_opts *best, double *best_ms, double *default_ms);

/* ----------------------------------------------------------------- server */

/* Continuous-batching server.  Requests (graph, k) are admitted while their
   device footprint fits `hbm_budget_bytes` and fewer than `max_slots` are
   in flight; admitted requests are planned into work units and run in
   bounded slices ("ticks") of at most `tick_units` units, so requests that
   arrive while others run join the next tick and share the device with
   them.  Each request's histogram is identical to mk_count's. */
typedef struct mk_server_opts {
    uint64_t hbm_budget_bytes; /* 0: 8 GiB */
    int32_t max_slots;         /* 0: 64 */
    int32_t tick_units;        /* 0: library default */
} mk_server_opts;

/* Per-request timing, microseconds since the server started. */
typedef struct mk_request_times {
    double submit_us;
    double admit_us;
    double done_us;
} mk_request_times;

/* Start the server (a host thread and its own stream).  Class tables for
   the ks it will see are built on first use (or earlier by the caller). */
int mk_server_start(mk_ctx *ctx, const mk_server_opts *opts, mk_server **out);

/* Queue a request.  The graph must stay loaded until the request is
   collected by mk_wait.  MK_EBUSY if its footprint can never fit the
   budget or the server is stopping; MK_ERANGE for k outside 3..6. */
int mk_submit(mk_server *s, const mk_graph *g, int k, uint64_t *ticket);

/* Wait up to timeout_ms (negative: forever) for request `ticket`, then copy
   its histogram (capacity must be >= its num_classes) and timings (may be
   NULL) and forget the request.  MK_ETIMEDOUT leaves it pending. */
int mk_wait(mk_server *s, uint64_t ticket, uint64_t *hist, uint32_t capacity,
            int32_t timeout_ms, mk_request_times *times);

/* Stop accepting requests, finish the admitted and queued ones, join the
   thread and free the server.  Uncollected results are discarded. */
int mk_server_stop(mk_server *s);

/* ----------------------------------------------------------------- errors */

const char *mk_status_str(int status);
const char *mk_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* MOTIFS_H */
