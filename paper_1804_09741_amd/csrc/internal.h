// Internal declarations of libmotifs (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <mutex>
#include <string>
#include <vector>

#include "motifs.h"

namespace mk {

// ------------------------------------------------------------------ errors

int fail(int status, const char *fmt, ...);  // records the message, returns status

#define MK_HIP(call)                                                            \
    do {                                                                        \
        hipError_t mk_e_ = (call);                                              \
        if (mk_e_ != hipSuccess)                                                \
            return ::mk::fail(MK_EDEVICE, "%s: %s (%s:%d)", #call,              \
                              hipGetErrorString(mk_e_), __FILE__, __LINE__);    \
    } while (0)

// ---------------------------------------------------------- device limits

constexpr int kWave = 64;

// ------------------------------------------------------------ table object

struct Table {
    mk_ctx *ctx = nullptr;
    int k = 0;
    uint64_t entries = 0;          // 2^(k(k-1))
    uint32_t num_classes = 0;
    uint32_t *d_table = nullptr;   // entries x uint32: code -> class id
    uint32_t *d_classes = nullptr; // num_classes canonical codes, ascending
    uint8_t *d_core_mult = nullptr; // num_classes: cores per class ((k-2)-set counting)
    std::vector<uint32_t> classes; // host copy of d_classes
    double build_ms = 0.0;
};

// ----------------------------------------------------------- graph object

struct Graph {
    mk_ctx *ctx = nullptr;
    int32_t n = 0;
    int64_t m = 0;
    int64_t nnz_u = 0;        // sum of undirected degrees |delta(v)|
    int32_t max_udeg = 0;
    int32_t *d_row = nullptr; // n+1, out-adjacency CSR as given
    int32_t *d_col = nullptr; // m
};

// A pointer into device memory in the global address space.  Kernels read
// the graph arrays' addresses from the descriptors below, and the compiler
// cannot tell that such a pointer is global: loads through it would be flat
// loads, which also count against the LDS wait counter, so that every wait
// for an LDS result would wait for them too.  Kernels cast the descriptors'
// pointers to this type once.
template <class T>
using GPtr = __attribute__((address_space(1))) T *;

// Descriptor of one graph inside a batch, read by every kernel of the path.
struct DevGraph {
    int32_t n;
    int32_t words;            // 32-bit words per bit-matrix row: ceil(n/32)
    const int32_t *out_row;   // n+1
    const int32_t *out_col;   // m
    uint32_t *bits_out;       // n x words, row u bit v: arc u -> v
    uint32_t *bits_in;        // n x words, row v bit u: arc u -> v
    int32_t *urow;            // n+1 offsets of delta(v) in uadj
    uint32_t *uadj;           // (u << 2) | type; type bit0: v -> u, bit1: u -> v
    uint32_t slot_base;       // first planner slot of this graph
    uint32_t nnz_cap;         // entries reserved for uadj (host-computed sum of |delta(v)|)
    uint32_t vbase;           // index of vertex 0 in the batch's per-vertex arrays
                              // (list-built adjacency); bits_* are null then
};

// Two-bit relation of w to u read from the sorted typed lists (bit0: arc
// w -> u, bit1: arc u -> w; 0 when not adjacent): a binary search for u in
// w's list or for w in u's, whichever list is shorter.
template <class RowPtr, class AdjPtr>
__device__ __forceinline__ uint32_t list_relation(RowPtr urow, AdjPtr uadj, uint32_t w, uint32_t u)
{
    const int a0 = urow[w], a1 = urow[w + 1], b0 = urow[u], b1 = urow[u + 1];
    const bool sw = b1 - b0 < a1 - a0;
    int lo = sw ? b0 : a0;
    const int end = sw ? b1 : a1;
    const uint32_t key = sw ? w : u;
    int hi = end;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if ((uadj[mid] >> 2) < key) lo = mid + 1;
        else hi = mid;
    }
    const uint32_t t = (lo < end && (uadj[lo] >> 2) == key) ? (uadj[lo] & 3u) : 0u;
    return sw ? (((t & 1u) << 1) | (t >> 1)) : t;
}

// Work unit of the enumeration queue.
//   x: graph index in the batch, y: root vertex v,
//   z: index i of the first extension vertex in v's extension list,
//   w: kFullChild -> the whole subtree below (v, w_i);
//      else j0 | j1 << 16 -> children j0..j1-1 of the node (v, w_i).
// kHeavyBit in x marks a unit whose estimated cost is high (the core
// kernel takes such units in a first sweep of each range; every kernel
// masks the bit off the graph index).
constexpr uint32_t kFullChild = 0xFFFFFFFFu;
constexpr uint32_t kHeavyBit = 1u << 31;

// counters[] slots shared by planner and enumeration kernels
enum Counter : int {
    kSliceBegin = 0,  // first unit of the current launch (server slices; else 0)
    kNumUnits = 1,    // units written by the planner
    kErrors = 2,      // device-side consistency failures (must stay 0)
    kSplitPairs = 3,  // (root, first neighbour) pairs split at the second level
    kAdjOverflow = 4, // typed adjacency larger than reserved (must stay 0)
    kSpecSplitPairs = 5,  // kSplitPairs at the floor threshold (estimate pass)
    kEstTotal = 6,    // words 6-7: u64 estimated total cost (planner)
    kPlanThreshold = 8,  // words 8-9: u64 split threshold of the last count pass
    kQueueHeads = 16, // kQueues heads, one per XCD, kHeadStride words apart
    kHeavyHeads = 16 + 8 * 16,  // the first sweep's kQueues heads, likewise
    kNumCounters = 16 + 2 * 8 * 16,
};
constexpr int kQueues = 8;       // one queue per XCD of the MI355X
constexpr int kHeadStride = 16;  // 64 bytes: one cache line per head

// --------------------------------------------------------------- context

struct Ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    int num_cus = 0;
    int64_t hbm_bytes = 0;
    size_t max_lds = 0;
    Table *tables[7] = {};
    int k7_class_log2 = 10;  // class-table size of the last k = 7 count (grows as needed)
    // k = 7 canonical-code cache (labelled code -> canonical code; 2^22
    // slots each, made by the first count and kept: it holds no graph data)
    unsigned long long *k7_cache_key = nullptr, *k7_cache_val = nullptr;
    uint32_t *k7_cache_used = nullptr;  // device: slots claimed since the last clear
    uint64_t k7_cache_fill = 0;         // host copy, read back after every count
    std::recursive_mutex mu;
};

// ------------------------------------------------------- kernel launchers

// Exclusive prefix sum of n uint32 values (or of their popcounts when
// popcount != 0) into out; the grand total goes to *d_total.  tmp must hold
// scan_tmp_words(n) words.  Everything is on `stream`, asynchronous.
size_t scan_tmp_words(size_t n);
int scan_u32(const uint32_t *in, uint32_t *out, size_t n, int popcount, uint32_t *d_total,
             uint32_t *tmp, hipStream_t stream);

// Fill n 32-bit words with value (a kernel, so it can live in a captured
// hipGraph).
int fill_u32(void *dst, uint32_t value, size_t n, hipStream_t stream);

// Class table build for k (3..6).  Allocates and fills t->d_table,
// t->d_classes, t->num_classes.  Synchronous.
int build_table(Table *t, hipStream_t stream);

// Typed symmetric adjacency of every graph of a batch (bit matrices
// zeroed, arcs set, degrees counted and scanned, lists written).
// Typed adjacency without bit matrices: raw out/in entries per vertex,
// sorted and merged per vertex.  `lists` holds list_ws_words() words.
uint64_t list_ws_words(uint64_t total_n, uint64_t total_m);
int launch_typed_lists(const DevGraph *d_graphs, int ng, int max_n, int64_t max_m,
                       uint64_t total_n, uint64_t total_m, int max_raw, uint32_t *lists,
                       uint32_t *counters, hipStream_t stream);
int launch_typed_csr(const DevGraph *d_graphs, int ng, int max_n, int64_t max_m,
                     uint64_t bits_words_total, uint32_t *bits_base, uint32_t *counters,
                     hipStream_t stream);

// Work-unit planner: cost estimate, counts per slot, scan, emit (units ==
// nullptr: sizing only).  k = 2 plans one unit per vertex with a neighbour.
// Writes counters[kNumUnits].  The split threshold is max(split_threshold,
// estimated total / (waves * units_per_wave)); units_per_wave 0 takes the
// planner's rule (16, or 64 on sorted-list adjacency below k = 7).
// slot_l2: per slot, the extension length of its first-level node (written
// by the estimate pass, read by the count and emit passes).
// spec_threshold (0: the floor): the threshold at which the estimate pass
// also counts each slot's units; the count pass keeps those counts when the
// threshold comes out equal to it (a batch passes the one its sizing plan
// found, read from counters[kPlanThreshold]).
int launch_plan(int k, const DevGraph *d_graphs, int ng, int64_t max_nnz, uint32_t total_slots,
                uint32_t *slot_cnt, uint32_t *slot_off, uint32_t *slot_est, uint32_t *slot_vi,
                uint32_t *slot_l2, uint32_t *scan_tmp, int4 *units, uint32_t unit_cap,
                uint64_t split_threshold, uint64_t spec_threshold, uint32_t waves,
                uint32_t units_per_wave, uint32_t *counters, hipStream_t stream);

// Enumeration + code + lookup + histogram over the queued units.
// k = 7 (k7.hip): device tables of one count
struct K7Launch {
    unsigned long long *cache_key, *cache_val;  // labeled -> canonical code
    int cache_log2;                              // log2 of the cache slots
    unsigned long long *class_key, *class_cnt;  // per graph: canonical code -> count
    int class_log2;                              // log2 of the class slots per graph
    unsigned long long *totals;                  // per graph: subgraphs
    uint32_t *overflow;                          // class inserts that found no slot
    uint32_t *cache_used;                        // cache slots claimed (fill level)
    uint8_t *etag;                               // device-memory marks: tag bytes,
    size_t etag_stride;                          //   per workgroup, all zero
};
int k7_lds_bytes(int max_n, int seg_cap, int variant);
int k7_max_blocks_per_cu(int variant, int lds_bytes, int *blocks);
int launch_k7(const DevGraph *d_graphs, const int4 *units, uint32_t unit_cap, uint32_t *counters,
              const K7Launch &a, const struct EnumConfig &cfg, int grid, int lds_bytes,
              hipStream_t stream);
int launch_k7_collect(const K7Launch &a, int ng, int64_t cap, unsigned long long *out_codes,
                      unsigned long long *out_counts, unsigned long long *n_out, hipStream_t stream);
int enum_lds_bytes(int k, int max_n, int seg_cap, int variant);
int enum_max_blocks_per_cu(int k, int variant, int lds_bytes, int *blocks);
constexpr uint32_t kAllUnits = 0xFFFFFFFFu;

// Launch configuration of the enumeration kernel.
// Variants of the enumeration walk (template parameter V of its state and
// kernels):
//   kVarSearch  arc tests between extension vertices search the sorted typed
//               lists (the shorter of the two) instead of reading n x n bit
//               matrices, so no bit matrix is built;
//   kVarGlobal  every wave's marks live in a private n-entry array in global
//               memory instead of LDS, and extension segments hold u32 ids:
//               graphs with more vertices than LDS marks can hold.
//   kVarDebug   the kernel honours the kDebug* test hooks of EnumConfig
//               (the production kernels leave their checks out: about 2%
//               of the k = 6 kernel's time per hash insert).
constexpr int kVarSearch = 1;
constexpr int kVarGlobal = 2;
constexpr int kVarDebug = 4;

struct EnumConfig {
    int max_n;       // largest n of the batch (LDS marks)
    int seg_cap;     // largest undirected degree (LDS extension segments)
    uint32_t flags;  // kDebug* bits below (tests only; 0 in production)
    uint32_t chunk;  // units per queue grab; 0 = about 1/32 of a wave's share
    uint32_t *wave_scratch;  // core kernel: kParentArcCap words per workgroup
    int hash_bits;           // log2 of the per-wave hash slots (enum_/core_hash_bits)
    int variant;             // kVar* bits of the enumeration kernel (esu.h)
    void *marks;             // kVarGlobal: grid x mark_stride marks, all zero
    size_t mark_stride;      //   marks per workgroup (>= max_n)
};
int enum_hash_bits(int k);
int core_hash_bits(int k);
constexpr uint32_t kDebugNoHash = 1u;      // every code straight to the histogram
constexpr uint32_t kDebugFlushAlways = 2u; // flush the hash after every insert
constexpr uint32_t kDebugNoShare = 4u;     // core kernel: no per-parent arc lists
// Arc pairs inside adj(P) kept per parent node P by the core kernel (global
// memory, one list per workgroup); a parent with more uses the per-core scan.
constexpr uint32_t kParentArcCap = 2048;
// The units [counters[kSliceBegin], min(counters[kNumUnits], unit_cap,
// unit_end)) are cut into kQueues equal ranges; wave w starts on range
// w % kQueues (the XCD the wave runs on) and then helps the others.  Heads
// must be zero at launch.
int launch_enum(int k, const DevGraph *d_graphs, const int4 *units, uint32_t unit_cap,
                uint32_t unit_end, uint32_t *counters, const uint32_t *table, uint32_t num_classes,
                unsigned long long *hist_base, const EnumConfig &cfg, int grid, int lds_bytes,
                hipStream_t stream);

// Counting from the connected (k-2)-sets: same queues, units planned for
// (k-1)-sets (k = 3: one unit per vertex), raw sums into the histograms,
// then the division by the cores per class.
int core_lds_bytes(int k, int max_n, int seg_cap);
int core_max_blocks_per_cu(int k, int lds_bytes, int *blocks);
int launch_core(int k, const DevGraph *d_graphs, const int4 *units, uint32_t unit_cap,
                uint32_t unit_end, uint32_t *counters, const uint32_t *table, uint32_t num_classes,
                unsigned long long *hist_base, const EnumConfig &cfg, int grid, int lds_bytes,
                hipStream_t stream);
int launch_core_divide(unsigned long long *hist, int ng, uint32_t num_classes,
                       const uint8_t *mult, uint32_t *counters, hipStream_t stream);

void free_table(Table *t);

// Default split floor (estimated subgraphs per work unit) for units planned
// for sets of plan_k vertices.
uint64_t default_split_floor(int plan_k);

// Address of the static device scratch of mk_count_static on `device`
// (which must be current), looked up once per device.
int static_scratch_init(int device);

// Prepared-batch hooks used by the request server.
uint64_t batch_units(const mk_batch *b);
uint64_t batch_device_bytes(const mk_batch *b);
int batch_prepare(mk_batch *b, hipStream_t stream);
int batch_enum_slice(mk_batch *b, uint32_t begin, uint32_t end, hipStream_t stream);
int batch_collect(mk_batch *b, uint64_t *hist, hipStream_t copy_stream);

}  // namespace mk

struct mk_ctx : mk::Ctx {};
struct mk_graph : mk::Graph {};
struct mk_table : mk::Table {};
