// Context, prepared batches and the count calls.
//
// A batch holds the device workspace of ng graphs counted with one class
// table, and runs the whole path as one stream sequence:
//   reset counters and histograms (fill kernels) -> typed adjacency (Section
//   2's A/B/C lists) -> work-unit plan -> persistent enumeration kernel
// with no host synchronisation in between.  The ten small preparation
// kernels are captured once as a hipGraph and replayed; the enumeration
// kernel follows as one launch between two HIP events (its timing).  Every
// graph of the batch shares one queue and one launch; histograms are
// [ng][num_classes] uint64.
#include <algorithm>
#include <cstring>

#include "internal.h"
#include "motifs_testing.h"
#include "server_hooks.h"

using namespace mk;

struct mk_batch {
    mk_ctx *ctx = nullptr;
    const mk_table *table = nullptr;
    int k = 0;
    int ng = 0;
    std::vector<const mk_graph *> graphs;
    mk_batch_opts opts{};
    int32_t debug_flags = 0;  // test hooks (mk_batch_debug)

    DevGraph *d_graphs = nullptr;
    uint32_t *d_ws = nullptr;  // bit matrices (or list-build arrays), urow, uadj
    uint64_t bits_words = 0;   // MK_ADJ_BITS: words of all bit matrices
    uint32_t *d_slot_cnt = nullptr;
    uint32_t *d_slot_off = nullptr;
    uint32_t *d_slot_est = nullptr;
    uint32_t *d_slot_vi = nullptr;
    uint32_t *d_slot_l2 = nullptr;
    uint32_t *d_scan_tmp = nullptr;
    uint32_t total_slots = 0;
    int4 *d_units = nullptr;
    uint32_t unit_cap = 0;
    uint64_t spec_threshold = 0;  // split threshold of the sizing plan (0: the floor)
    uint32_t *d_counters = nullptr;
    uint32_t *d_unit_begin = nullptr;    // first unit of every graph, plus the total
    unsigned long long *d_hist_own = nullptr;
    uint32_t *d_wave_scratch = nullptr;  // core method: per-workgroup arc lists
    void *d_marks = nullptr;             // MK_MARKS_GLOBAL: per-workgroup marks
    size_t mark_stride = 0;              //   marks per workgroup
    size_t mark_bytes = 0;               //   bytes of d_marks
    unsigned long long *hist_last = nullptr;

    int max_n = 0, max_words = 0, seg_cap = 0;
    int64_t max_m = 0;
    int64_t max_nnz = 0;
    uint64_t total_n = 0, total_m = 0;  // over the batch (list-built adjacency)
    int grid = 0, max_grid = 0, lds_bytes = 0;
    int method = MK_METHOD_ESU;  // resolved (never MK_METHOD_AUTO)
    int adjacency = MK_ADJ_BITS; // resolved MK_ADJ_*
    int marks = MK_MARKS_LDS;    // resolved MK_MARKS_*
    int variant = 0;             // kVar* bits of the enumeration kernel
    int plan_k = 0;              // set size the planner cuts units for
    uint64_t units = 0, split_pairs = 0;

    // pass start, counting kernel start, counting kernel end, pass end
    hipEvent_t ev[4] = {};
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    bool graph_whole = false;   // exec holds the whole pass (else the preparation)
    unsigned long long *exec_hist = nullptr;
    hipStream_t last_stream = nullptr;
};

// default split floor per planned set size (the planner raises it to its
// adaptive threshold); 512 at k = 6 lets the hubs of a batch of small graphs
// split (12% off the k = 6 kernel on 31 power-law graphs of 700 vertices)
static constexpr uint64_t kDefaultSplit[8] = {0,       0,       1u << 30, 1u << 30,
                                              1u << 10, 1u << 12, 1u << 9, 1u << 12};

namespace mk {
uint64_t default_split_floor(int plan_k)
{
    return plan_k >= 0 && plan_k < 8 ? kDefaultSplit[plan_k] : (1u << 12);
}
}  // namespace mk

// ----------------------------------------------------------------- context

extern "C" int mk_init(int device, mk_ctx **out)
{
    if (!out) return fail(MK_EINVAL, "mk_init: NULL out");
    *out = nullptr;
    int count = 0;
    MK_HIP(hipGetDeviceCount(&count));
    if (device < 0 || device >= count)
        return fail(MK_ERANGE, "device %d not present (%d devices)", device, count);
    MK_HIP(hipSetDevice(device));
    hipDeviceProp_t prop;
    MK_HIP(hipGetDeviceProperties(&prop, device));
    // the static scratch of mk_count_static, looked up once per device
    int src = static_scratch_init(device);
    if (src) return src;
    mk_ctx *c = new mk_ctx();
    c->device = device;
    c->num_cus = prop.multiProcessorCount;
    c->hbm_bytes = (int64_t)prop.totalGlobalMem;
    c->max_lds = prop.sharedMemPerBlock;
    hipError_t e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
        delete c;
        return fail(MK_EDEVICE, "hipStreamCreate: %s", hipGetErrorString(e));
    }
    *out = c;
    return MK_OK;
}

extern "C" void mk_destroy(mk_ctx *ctx)
{
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    for (int k = 0; k < 7; ++k) free_table(ctx->tables[k]);
    if (ctx->k7_cache_key) (void)hipFree(ctx->k7_cache_key);
    if (ctx->k7_cache_val) (void)hipFree(ctx->k7_cache_val);
    if (ctx->k7_cache_used) (void)hipFree(ctx->k7_cache_used);
    (void)hipStreamDestroy(ctx->stream);
    delete ctx;
}

extern "C" int mk_device_info(const mk_ctx *ctx, int32_t *compute_units, int64_t *hbm_bytes)
{
    if (!ctx) return fail(MK_EINVAL, "mk_device_info: NULL context");
    if (compute_units) *compute_units = ctx->num_cus;
    if (hbm_bytes) *hbm_bytes = ctx->hbm_bytes;
    return MK_OK;
}

static uint32_t classes_for_k(int k)
{
    static const uint32_t n[7] = {0, 0, 0, 13, 199, 9364, 1530843};
    return (k >= 3 && k <= 6) ? n[k] : 0;
}

extern "C" int mk_graph_footprint(const mk_graph *g, int k, uint64_t *bytes)
{
    if (!g || !bytes) return fail(MK_EINVAL, "mk_graph_footprint: NULL argument");
    if (k < 3 || k > 6) return fail(MK_ERANGE, "k=%d outside 3..6", k);
    const uint64_t n = (uint64_t)g->n, w = (n + 31) / 32;
    const bool big = g->n > MK_LDS_MARKS_MAX_VERTICES;  // list-built adjacency, global marks
    const uint64_t region = big ? list_ws_words(n, (uint64_t)g->m) : 2 * n * w;
    const uint64_t ws = 4 * (region + (n + 1) + (uint64_t)g->nnz_u);
    const uint64_t slots = 20 * (uint64_t)g->nnz_u + 4 * ((uint64_t)g->nnz_u / 4096 + 2);
    const uint64_t units = 16 * (uint64_t)g->nnz_u * 4;  // planning estimate
    const uint64_t hist = 8ull * classes_for_k(k);
    // per-workgroup arc lists of the core method (the default for k <= 5 on
    // graphs with LDS marks), one workgroup per unit at most
    const uint64_t scratch =
        k <= 5 && !big ? 4ull * kParentArcCap * std::min<uint64_t>(g->nnz_u + 1, 8192) : 0;
    // per-workgroup marks, at most 32 workgroups per CU and 1/16 of the memory
    const uint64_t per_wave = ((n + 63) & ~63ull) * 4;
    const uint64_t marks =
        big ? std::min<uint64_t>((uint64_t)g->ctx->hbm_bytes / 16,
                                 (uint64_t)g->ctx->num_cus * 32 * per_wave)
            : 0;
    *bytes = ws + slots + units + hist + scratch + marks + sizeof(DevGraph) + 4 * kNumCounters;
    return MK_OK;
}

// ------------------------------------------------------------------ batch

static void batch_release(mk_batch *b)
{
    for (hipEvent_t e : b->ev)
        if (e) (void)hipEventDestroy(e);
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    void *bufs[] = {b->d_graphs, b->d_ws, b->d_slot_cnt, b->d_slot_off, b->d_slot_est,
                    b->d_slot_vi, b->d_slot_l2, b->d_scan_tmp,
                    b->d_units, b->d_counters, b->d_unit_begin, b->d_hist_own, b->d_wave_scratch,
                    b->d_marks};
    for (void *p : bufs)
        if (p) (void)hipFree(p);
}

static EnumConfig enum_config(const mk_batch *b)
{
    EnumConfig c;
    c.max_n = b->max_n;
    c.seg_cap = b->seg_cap;
    c.flags = (uint32_t)b->debug_flags;
    c.chunk = (uint32_t)std::max(b->opts.units_per_grab, 0);
    c.wave_scratch = b->d_wave_scratch;
    c.hash_bits = b->method == MK_METHOD_CORES ? core_hash_bits(b->k) : enum_hash_bits(b->k);
    // the test hooks of the hash run in the kernels built with them
    c.variant = b->variant |
                (b->k <= 6 && (b->debug_flags & (kDebugNoHash | kDebugFlushAlways)) ? kVarDebug : 0);
    c.marks = b->d_marks;
    c.mark_stride = b->mark_stride;
    return c;
}

// typed adjacency of every graph (from bit matrices or by sorting lists)
static int batch_enqueue_typed(mk_batch *b, hipStream_t stream)
{
    if (b->adjacency == MK_ADJ_LISTS)
        return launch_typed_lists(b->d_graphs, b->ng, b->max_n, b->max_m, b->total_n, b->total_m,
                                  2 * b->seg_cap, b->d_ws, b->d_counters, stream);
    return launch_typed_csr(b->d_graphs, b->ng, b->max_n, b->max_m, b->bits_words, b->d_ws,
                            b->d_counters, stream);
}

// enqueue the preparation part of one pass on stream: counters and
// histograms cleared, typed adjacency, work-unit plan (captured as a
// hipGraph).  (Clearing the histograms from extra workgroups of the
// latency-bound plan passes instead was measured slower: the streaming
// stores raise the latency of the passes' dependent loads, 0.24 ms for the
// k = 6 batch's preparation either way.)
static int batch_enqueue_prep(mk_batch *b, unsigned long long *hist, hipStream_t stream)
{
    int rc = fill_u32(b->d_counters, 0, kNumCounters, stream);
    if (rc) return rc;
    if (hist) {
        rc = fill_u32(hist, 0, (size_t)b->ng * b->table->num_classes * 2, stream);
        if (rc) return rc;
    }
    rc = batch_enqueue_typed(b, stream);
    if (rc) return rc;
    return launch_plan(b->plan_k, b->d_graphs, b->ng, b->max_nnz, b->total_slots, b->d_slot_cnt,
                       b->d_slot_off, b->d_slot_est, b->d_slot_vi, b->d_slot_l2, b->d_scan_tmp,
                       b->d_units, b->unit_cap, b->opts.split_threshold, b->spec_threshold,
                       (uint32_t)b->max_grid, (uint32_t)std::max(b->opts.units_per_wave, 0),
                       b->d_counters, stream);
}

// the counting kernel over units [counters[kSliceBegin], unit_end)
static int batch_launch_count(mk_batch *b, unsigned long long *hist, uint32_t unit_end, int grid,
                              hipStream_t stream)
{
    if (b->method == MK_METHOD_CORES)
        return launch_core(b->k, b->d_graphs, b->d_units, b->unit_cap, unit_end, b->d_counters,
                           b->table->d_table, b->table->num_classes, hist, enum_config(b), grid,
                           b->lds_bytes, stream);
    return launch_enum(b->k, b->d_graphs, b->d_units, b->unit_cap, unit_end, b->d_counters,
                       b->table->d_table, b->table->num_classes, hist, enum_config(b), grid,
                       b->lds_bytes, stream);
}

// after the last unit: the cores method divides its raw sums
static int batch_launch_finish(mk_batch *b, unsigned long long *hist, hipStream_t stream)
{
    if (b->method != MK_METHOD_CORES) return MK_OK;
    return launch_core_divide(hist, b->ng, b->table->num_classes, b->table->d_core_mult,
                              b->d_counters, stream);
}

// the counting kernel and the finish, no events (a whole-pass graph)
static int batch_enqueue_count_finish(mk_batch *b, unsigned long long *hist, hipStream_t stream)
{
    int rc = batch_launch_count(b, hist, kAllUnits, b->grid, stream);
    if (rc) return rc;
    return batch_launch_finish(b, hist, stream);
}

// the counting kernel between two timing events, then the finish
static int batch_enqueue_enum(mk_batch *b, unsigned long long *hist, hipStream_t stream)
{
    MK_HIP(hipEventRecord(b->ev[1], stream));
    int rc = batch_launch_count(b, hist, kAllUnits, b->grid, stream);
    if (rc) return rc;
    MK_HIP(hipEventRecord(b->ev[2], stream));
    rc = batch_launch_finish(b, hist, stream);
    if (rc) return rc;
    MK_HIP(hipEventRecord(b->ev[3], stream));
    return MK_OK;
}

// A batch of ng graphs for subgraph size k: counted with table t (k <= 6),
// or with the k = 7 kernel and no table (t null).
static int batch_create(mk_ctx *ctx, const mk_graph *const *gs, int32_t ng, int k,
                        const mk_table *t, const mk_batch_opts *opts, mk_batch **out)
{
    *out = nullptr;
    for (int i = 0; i < ng; ++i)
        if (!gs[i] || gs[i]->ctx != ctx)
            return fail(MK_EINVAL, "mk_batch_create: graph %d missing or of another context", i);
    std::lock_guard<std::recursive_mutex> lock(ctx->mu);
    MK_HIP(hipSetDevice(ctx->device));

    mk_batch *b = new mk_batch();
    b->ctx = ctx;
    b->table = t;
    b->k = k;
    b->ng = ng;
    b->graphs.assign(gs, gs + ng);
    if (opts) b->opts = *opts;
    const mk_batch_opts o = b->opts;
    if (o.units_per_wave < 0 || o.units_per_wave > 4096) {
        delete b;
        return fail(MK_EINVAL, "mk_batch_create: units_per_wave %d outside 0..4096",
                    o.units_per_wave);
    }
    if (o.method < MK_METHOD_AUTO || o.method > MK_METHOD_CORES || o.adjacency < MK_ADJ_AUTO ||
        o.adjacency > MK_ADJ_LISTS || o.marks < MK_MARKS_AUTO || o.marks > MK_MARKS_GLOBAL) {
        delete b;
        return fail(MK_EINVAL, "mk_batch_create: unknown method %d, adjacency %d or marks %d",
                    o.method, o.adjacency, o.marks);
    }

    // workspace layout: [bit matrices of every graph, or the list-build
    // arrays][urow of every graph][uadj ...]
    std::vector<DevGraph> hg(ng);
    uint64_t bits = 0, rows = 0, adj = 0, slots = 0;
    for (int i = 0; i < ng; ++i) {
        const mk_graph *g = gs[i];
        const uint64_t w = ((uint64_t)g->n + 31) / 32;
        bits += 2 * (uint64_t)g->n * w;
        rows += (uint64_t)g->n + 1;
        adj += (uint64_t)g->nnz_u;
        b->max_n = std::max(b->max_n, g->n);
        b->max_words = std::max<int>(b->max_words, (int)w);
        b->seg_cap = std::max(b->seg_cap, g->max_udeg);
        b->max_nnz = std::max<int64_t>(b->max_nnz, g->nnz_u);
        b->max_m = std::max<int64_t>(b->max_m, g->m);
        b->total_n += (uint64_t)g->n;
        b->total_m += (uint64_t)g->m;
        slots += (uint64_t)g->nnz_u;
    }
    if (slots >= 0xFFFFFFFFull || 2 * b->total_m >= 0xFFFFFFFFull || b->total_n >= 0x7FFFFFFFull) {
        const unsigned long long tm = b->total_m;
        delete b;
        return fail(MK_ERANGE, "batch too large: %llu adjacency entries, %llu arcs",
                    (unsigned long long)slots, tm);
    }

    // where the marks live, how arcs are tested, the counting method
    const bool big = b->max_n > MK_LDS_MARKS_MAX_VERTICES;
    b->marks = b->opts.marks != MK_MARKS_AUTO ? b->opts.marks
                                              : (big ? MK_MARKS_GLOBAL : MK_MARKS_LDS);
    b->adjacency = b->opts.adjacency != MK_ADJ_AUTO
                       ? b->opts.adjacency
                       : (b->marks == MK_MARKS_GLOBAL ? MK_ADJ_LISTS : MK_ADJ_BITS);
    // the library's choice of method: counting from the (k-2)-sets is the
    // faster on sparse graphs for k <= 5; for k = 6 the per-core work (up to
    // 255 cells) costs more than enumerating the k-sets
    b->method = b->opts.method != MK_METHOD_AUTO
                    ? b->opts.method
                    : (b->k <= 5 && b->marks == MK_MARKS_LDS ? MK_METHOD_CORES : MK_METHOD_ESU);
    if (b->marks == MK_MARKS_LDS && big) {
        const int max_n = b->max_n;
        delete b;
        return fail(MK_ERANGE, "n=%d exceeds MK_LDS_MARKS_MAX_VERTICES=%d for MK_MARKS_LDS",
                    max_n, MK_LDS_MARKS_MAX_VERTICES);
    }
    if (b->marks == MK_MARKS_GLOBAL && b->adjacency != MK_ADJ_LISTS) {
        delete b;
        return fail(MK_EINVAL, "MK_MARKS_GLOBAL needs MK_ADJ_LISTS");
    }
    if (b->method == MK_METHOD_CORES && b->marks != MK_MARKS_LDS) {
        delete b;
        return fail(MK_ERANGE, "MK_METHOD_CORES needs LDS marks (n <= %d)",
                    MK_LDS_MARKS_MAX_VERTICES);
    }
    b->variant = (b->adjacency == MK_ADJ_LISTS ? kVarSearch : 0) |
                 (b->marks == MK_MARKS_GLOBAL ? kVarGlobal : 0);
    b->plan_k = b->method == MK_METHOD_CORES ? (b->k == 3 ? 2 : b->k - 1) : b->k;
    if (b->opts.split_threshold == 0) b->opts.split_threshold = kDefaultSplit[b->plan_k];
    if (b->opts.use_graph == 0) b->opts.use_graph = 1;

    b->bits_words = b->adjacency == MK_ADJ_BITS ? bits : 0;
    const uint64_t region = b->adjacency == MK_ADJ_BITS ? bits : list_ws_words(b->total_n, b->total_m);
    b->total_slots = (uint32_t)slots;
    b->seg_cap = std::max(b->seg_cap, 1);
    b->lds_bytes = b->k == 7 ? k7_lds_bytes(std::max(b->max_n, 1), b->seg_cap, b->variant)
                   : b->method == MK_METHOD_CORES
                       ? core_lds_bytes(b->k, std::max(b->max_n, 1), b->seg_cap)
                       : enum_lds_bytes(b->k, std::max(b->max_n, 1), b->seg_cap, b->variant);
    if ((size_t)b->lds_bytes > ctx->max_lds) {
        const int lds = b->lds_bytes;
        delete b;
        return fail(MK_ERANGE, "graphs need %d bytes of LDS per wave (limit %zu)", lds,
                    ctx->max_lds);
    }
    int rc = MK_OK;
    auto bail = [&](int status) {
        batch_release(b);
        delete b;
        return status;
    };
#define BAIL_HIP(x)                                                                            \
    do {                                                                                       \
        hipError_t e_ = (x);                                                                   \
        if (e_ != hipSuccess)                                                                  \
            return bail(fail(e_ == hipErrorOutOfMemory ? MK_ENOMEM : MK_EDEVICE, "%s: %s", #x, \
                             hipGetErrorString(e_)));                                          \
    } while (0)

    BAIL_HIP(hipMalloc(&b->d_ws, sizeof(uint32_t) * std::max<uint64_t>(region + rows + adj, 1)));
    {
        const bool with_bits = b->adjacency == MK_ADJ_BITS;
        uint64_t ob = 0, orow = region, oadj = region + rows, oslot = 0, vbase = 0;
        for (int i = 0; i < ng; ++i) {
            const mk_graph *g = gs[i];
            DevGraph d;
            std::memset(&d, 0, sizeof(d));
            d.n = g->n;
            d.words = with_bits ? (g->n + 31) / 32 : 0;
            d.out_row = g->d_row;
            d.out_col = g->d_col;
            d.bits_out = with_bits ? b->d_ws + ob : nullptr;
            d.bits_in = with_bits ? b->d_ws + ob + (uint64_t)g->n * d.words : nullptr;
            d.vbase = (uint32_t)vbase;
            vbase += (uint64_t)g->n;
            d.urow = reinterpret_cast<int32_t *>(b->d_ws + orow);
            d.uadj = b->d_ws + oadj;
            d.slot_base = (uint32_t)oslot;
            d.nnz_cap = (uint32_t)g->nnz_u;
            ob += 2 * (uint64_t)g->n * d.words;
            orow += (uint64_t)g->n + 1;
            oadj += (uint64_t)g->nnz_u;
            oslot += (uint64_t)g->nnz_u;
            hg[i] = d;
        }
    }
    BAIL_HIP(hipMalloc(&b->d_graphs, sizeof(DevGraph) * std::max(ng, 1)));
    if (ng > 0)
        BAIL_HIP(hipMemcpyAsync(b->d_graphs, hg.data(), sizeof(DevGraph) * ng,
                                hipMemcpyHostToDevice, ctx->stream));
    BAIL_HIP(hipMalloc(&b->d_slot_cnt, sizeof(uint32_t) * std::max<uint64_t>(slots, 1)));
    BAIL_HIP(hipMalloc(&b->d_slot_off, sizeof(uint32_t) * std::max<uint64_t>(slots, 1)));
    BAIL_HIP(hipMalloc(&b->d_slot_est, sizeof(uint32_t) * std::max<uint64_t>(slots, 1)));
    BAIL_HIP(hipMalloc(&b->d_slot_vi, sizeof(uint32_t) * std::max<uint64_t>(slots, 1)));
    BAIL_HIP(hipMalloc(&b->d_slot_l2, sizeof(uint32_t) * std::max<uint64_t>(slots, 1)));
    BAIL_HIP(hipMalloc(&b->d_scan_tmp, sizeof(uint32_t) * scan_tmp_words(slots)));
    BAIL_HIP(hipMalloc(&b->d_counters, sizeof(uint32_t) * kNumCounters));
    BAIL_HIP(hipMalloc(&b->d_unit_begin, sizeof(uint32_t) * ((size_t)ng + 1)));
    for (hipEvent_t &e : b->ev) BAIL_HIP(hipEventCreate(&e));

    int per_cu = 0;
    rc = b->k == 7 ? k7_max_blocks_per_cu(b->variant, b->lds_bytes, &per_cu)
         : b->method == MK_METHOD_CORES
             ? core_max_blocks_per_cu(b->k, b->lds_bytes, &per_cu)
             : enum_max_blocks_per_cu(b->k, b->variant, b->lds_bytes, &per_cu);
    if (rc) return bail(rc);
    if (b->opts.waves_per_cu > 0) per_cu = std::min(per_cu, b->opts.waves_per_cu);
    per_cu = std::max(per_cu, 1);
    b->max_grid = per_cu * ctx->num_cus;
    if (b->marks == MK_MARKS_GLOBAL) {
        // one private marks array per workgroup, rounded to 64 entries; all
        // of them together within 1/16 of the device memory
        b->mark_stride = ((size_t)std::max(b->max_n, 1) + 63) & ~(size_t)63;
        // 32-bit marks in device memory (k = 7: and a tag byte per vertex)
        const size_t per_wave = b->mark_stride * (b->k == 7 ? 5 : 4);
        const uint64_t budget = (uint64_t)ctx->hbm_bytes / 16;
        const uint64_t fit = std::max<uint64_t>(budget / per_wave, 1);
        b->max_grid = (int)std::min<uint64_t>((uint64_t)b->max_grid, fit);
    }

    // sizing pass: typed adjacency + unit counts only
    rc = fill_u32(b->d_counters, 0, kNumCounters, ctx->stream);
    if (!rc) rc = batch_enqueue_typed(b, ctx->stream);
    if (!rc)
        rc = launch_plan(b->plan_k, b->d_graphs, ng, b->max_nnz, b->total_slots, b->d_slot_cnt,
                         b->d_slot_off, b->d_slot_est, b->d_slot_vi, b->d_slot_l2, b->d_scan_tmp,
                         nullptr, 0, b->opts.split_threshold, 0, (uint32_t)b->max_grid,
                         (uint32_t)std::max(b->opts.units_per_wave, 0), b->d_counters,
                         ctx->stream);
    if (rc) return bail(rc);
    uint32_t cnt[kNumCounters];
    BAIL_HIP(hipMemcpyAsync(cnt, b->d_counters, sizeof(cnt), hipMemcpyDeviceToHost, ctx->stream));
    BAIL_HIP(hipStreamSynchronize(ctx->stream));
    if (cnt[kAdjOverflow] != 0)
        return bail(fail(MK_EDEVICE, "typed adjacency exceeds its reserved size"));
    b->units = cnt[kNumUnits];
    b->split_pairs = cnt[kSplitPairs];
    // the same graphs plan to the same threshold at every pass
    std::memcpy(&b->spec_threshold, &cnt[kPlanThreshold], sizeof(b->spec_threshold));
    b->unit_cap = std::max<uint32_t>(cnt[kNumUnits], 1);
    BAIL_HIP(hipMalloc(&b->d_units, sizeof(int4) * b->unit_cap));

    b->grid = (int)std::min<uint64_t>((uint64_t)b->max_grid, std::max<uint64_t>(b->units, 1));
    if (b->method == MK_METHOD_CORES)
        BAIL_HIP(hipMalloc(&b->d_wave_scratch, sizeof(uint32_t) * kParentArcCap * (size_t)b->grid));
    if (b->marks == MK_MARKS_GLOBAL) {
        // zero once: every pop restores the marks it changed, so they are
        // zero again whenever a workgroup finishes a unit
        b->mark_bytes = b->mark_stride * 4 * (size_t)b->grid;
        BAIL_HIP(hipMalloc(&b->d_marks, b->mark_bytes));
        rc = fill_u32(b->d_marks, 0, b->mark_bytes / 4, ctx->stream);
        if (rc) return bail(rc);
        BAIL_HIP(hipStreamSynchronize(ctx->stream));
    }
#undef BAIL_HIP
    *out = b;
    return MK_OK;
}

extern "C" int mk_batch_create(mk_ctx *ctx, const mk_graph *const *gs, int32_t ng,
                               const mk_table *t, const mk_batch_opts *opts, mk_batch **out)
{
    if (!ctx || !t || !out || (ng > 0 && !gs)) return fail(MK_EINVAL, "mk_batch_create: NULL argument");
    if (ng < 0) return fail(MK_EINVAL, "mk_batch_create: ng=%d < 0", ng);
    if (t->ctx != ctx || !t->d_table) return fail(MK_EINVAL, "mk_batch_create: table of another context");
    return batch_create(ctx, gs, ng, t->k, t, opts, out);
}

extern "C" int mk_batch_run(mk_batch *b, uint64_t *d_hist, void *stream)
{
    if (!b) return fail(MK_EINVAL, "mk_batch_run: NULL batch");
    mk_ctx *ctx = b->ctx;
    std::lock_guard<std::recursive_mutex> lock(ctx->mu);
    MK_HIP(hipSetDevice(ctx->device));
    unsigned long long *hist = reinterpret_cast<unsigned long long *>(d_hist);
    if (!hist) {
        if (!b->d_hist_own) {
            hipError_t e = hipMalloc(&b->d_hist_own, sizeof(unsigned long long) *
                                                         std::max<size_t>((size_t)b->ng * b->table->num_classes, 1));
            if (e != hipSuccess) return fail(MK_ENOMEM, "mk_batch_run: histogram allocation failed");
        }
        hist = b->d_hist_own;
    }
    hipStream_t s = stream ? reinterpret_cast<hipStream_t>(stream) : ctx->stream;
    if (b->ng == 0) {
        b->hist_last = hist;
        b->last_stream = s;
        return MK_OK;
    }
    if (b->opts.use_graph > 0) {
        if (!b->exec || b->exec_hist != hist) {
            if (b->exec) (void)hipGraphExecDestroy(b->exec);
            if (b->graph) (void)hipGraphDestroy(b->graph);
            b->exec = nullptr;
            b->graph = nullptr;
            // use_graph 2: the whole pass -- preparation, counting kernel
            // and finish -- as one graph; else the preparation alone, the
            // counting kernel then launched between its timing events
            // (events recorded inside a captured graph cannot be used for
            // elapsed times on this runtime)
            const bool whole = b->opts.use_graph == 2;
            MK_HIP(hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal));
            int rc = batch_enqueue_prep(b, hist, ctx->stream);
            if (!rc && whole) rc = batch_enqueue_count_finish(b, hist, ctx->stream);
            hipGraph_t g = nullptr;
            hipError_t e = hipStreamEndCapture(ctx->stream, &g);
            if (rc) {
                if (g) (void)hipGraphDestroy(g);
                return rc;
            }
            if (e != hipSuccess) return fail(MK_EDEVICE, "hipStreamEndCapture: %s", hipGetErrorString(e));
            b->graph = g;
            MK_HIP(hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0));
            b->graph_whole = whole;
            b->exec_hist = hist;
        }
        MK_HIP(hipEventRecord(b->ev[0], s));
        MK_HIP(hipGraphLaunch(b->exec, s));
        if (b->graph_whole) {
            MK_HIP(hipEventRecord(b->ev[3], s));
        } else {
            int rc = batch_enqueue_enum(b, hist, s);
            if (rc) return rc;
        }
    } else {
        MK_HIP(hipEventRecord(b->ev[0], s));
        int rc = batch_enqueue_prep(b, hist, s);
        if (!rc) rc = batch_enqueue_enum(b, hist, s);
        if (rc) return rc;
    }
    b->hist_last = hist;
    b->last_stream = s;
    return MK_OK;
}

extern "C" int mk_batch_read(mk_batch *b, uint64_t *hist, uint64_t *totals)
{
    if (!b) return fail(MK_EINVAL, "mk_batch_read: NULL batch");
    if (!b->hist_last) return fail(MK_EINVAL, "mk_batch_read: batch has not run");
    mk_ctx *ctx = b->ctx;
    std::lock_guard<std::recursive_mutex> lock(ctx->mu);
    MK_HIP(hipSetDevice(ctx->device));
    MK_HIP(hipStreamSynchronize(b->last_stream));
    const size_t nc = b->table->num_classes;
    if (b->ng == 0) return MK_OK;
    uint32_t cnt[kNumCounters];
    MK_HIP(hipMemcpy(cnt, b->d_counters, sizeof(cnt), hipMemcpyDeviceToHost));
    if (cnt[kErrors] != 0 || cnt[kAdjOverflow] != 0)
        return fail(MK_EDEVICE,
                    "device-side check failed (%u lookup/plan errors, %u adjacency overflows)",
                    cnt[kErrors], cnt[kAdjOverflow]);
    if (cnt[kNumUnits] > b->unit_cap)
        return fail(MK_EDEVICE, "plan produced %u units, capacity %u", cnt[kNumUnits], b->unit_cap);
    b->units = cnt[kNumUnits];
    b->split_pairs = cnt[kSplitPairs];
    std::vector<uint64_t> tmp;
    uint64_t *dst = hist;
    if (!dst && totals) {
        tmp.resize((size_t)b->ng * nc);
        dst = tmp.data();
    }
    if (dst) {
        MK_HIP(hipMemcpy(dst, b->hist_last, sizeof(uint64_t) * (size_t)b->ng * nc,
                         hipMemcpyDeviceToHost));
        if (totals)
            for (int i = 0; i < b->ng; ++i) {
                uint64_t s = 0;
                for (size_t c = 0; c < nc; ++c) s += dst[(size_t)i * nc + c];
                totals[i] = s;
            }
    }
    return MK_OK;
}

extern "C" int mk_batch_stats_get(const mk_batch *b, mk_batch_stats *out)
{
    if (!b || !out) return fail(MK_EINVAL, "mk_batch_stats_get: NULL argument");
    out->units = b->units;
    out->split_pairs = b->split_pairs;
    out->grid = b->grid;
    out->lds_bytes = b->lds_bytes;
    out->k = b->k;
    out->ng = b->ng;
    out->method = b->method;
    out->adjacency = b->adjacency;
    out->marks = b->marks;
    return MK_OK;
}

// ------------------------------------------------- hooks for the server

namespace mk {

uint64_t batch_units(const mk_batch *b) { return b->units; }

uint64_t batch_device_bytes(const mk_batch *b)
{
    uint64_t words = b->adjacency == MK_ADJ_BITS ? b->bits_words
                                                 : list_ws_words(b->total_n, b->total_m);
    for (const mk_graph *g : b->graphs) words += (uint64_t)g->n + 1 + (uint64_t)g->nnz_u;
    return 4 * words + 20ull * b->total_slots + 4 * scan_tmp_words(b->total_slots) +
           16ull * b->unit_cap + 8ull * b->ng * b->table->num_classes + 4ull * (b->ng + 1) +
           sizeof(DevGraph) * b->graphs.size() + 4 * kNumCounters +
           (b->d_wave_scratch ? 4ull * kParentArcCap * (uint64_t)b->grid : 0) + b->mark_bytes;
}

// typed adjacency + plan into the batch's own histogram buffer
int batch_prepare(mk_batch *b, hipStream_t stream)
{
    MK_HIP(hipSetDevice(b->ctx->device));
    if (!b->d_hist_own) {
        hipError_t e = hipMalloc(&b->d_hist_own, sizeof(unsigned long long) *
                                                     std::max<size_t>((size_t)b->ng * b->table->num_classes, 1));
        if (e != hipSuccess) return fail(MK_ENOMEM, "histogram allocation failed");
    }
    b->hist_last = b->d_hist_own;
    b->last_stream = stream;
    if (b->ng == 0) return MK_OK;
    return batch_enqueue_prep(b, b->d_hist_own, stream);
}

// enumeration of units [begin, end) of a prepared batch
int batch_enum_slice(mk_batch *b, uint32_t begin, uint32_t end, hipStream_t stream)
{
    if (b->ng == 0 || end <= begin) return MK_OK;
    // both sweeps' heads
    int rc = fill_u32(b->d_counters + kQueueHeads, 0, 2 * kQueues * kHeadStride, stream);
    if (rc) return rc;
    rc = fill_u32(b->d_counters + kSliceBegin, begin, 1, stream);
    if (rc) return rc;
    const int grid = (int)std::min<uint64_t>((uint64_t)b->grid, end - begin);
    return batch_launch_count(b, b->d_hist_own, end, grid, stream);
}

// First work unit of every graph of a batch after mk_batch_create (its
// sizing plan), plus the total, into *out (ng + 1 values).  Blocks.
int batch_unit_begins(mk_batch *b, std::vector<uint32_t> *out)
{
    std::lock_guard<std::recursive_mutex> lock(b->ctx->mu);
    MK_HIP(hipSetDevice(b->ctx->device));
    out->assign((size_t)b->ng + 1, 0u);
    if (b->ng == 0) return MK_OK;
    int rc = launch_unit_begins(b->d_graphs, b->ng, b->d_slot_off, b->total_slots, b->d_counters,
                                b->d_unit_begin, b->ctx->stream);
    if (rc) return rc;
    MK_HIP(hipMemcpyAsync(out->data(), b->d_unit_begin, sizeof(uint32_t) * out->size(),
                          hipMemcpyDeviceToHost, b->ctx->stream));
    MK_HIP(hipStreamSynchronize(b->ctx->stream));
    if ((*out)[b->ng] != b->units)
        return fail(MK_EDEVICE, "batch_unit_begins: %u units, the plan made %llu", (*out)[b->ng],
                    (unsigned long long)b->units);
    return MK_OK;
}

// Copy graph gi's histogram of a prepared batch whose units of that graph
// are known to be done (the event of the slice that ended them completed),
// finishing it first (the core method's division), on `copy_stream`; check
// the device-side counters and wait only for that copy.
int batch_collect_graph(mk_batch *b, int gi, uint64_t *hist, hipStream_t copy_stream)
{
    MK_HIP(hipSetDevice(b->ctx->device));
    if (gi < 0 || gi >= b->ng) return fail(MK_EINVAL, "batch_collect_graph: graph %d of %d", gi, b->ng);
    const size_t nc = b->table->num_classes;
    unsigned long long *row = b->d_hist_own + (size_t)gi * nc;
    if (b->method == MK_METHOD_CORES) {
        int rc = launch_core_divide(row, 1, (uint32_t)nc, b->table->d_core_mult, b->d_counters,
                                    copy_stream);
        if (rc) return rc;
    }
    uint32_t cnt[kNumCounters];
    MK_HIP(hipMemcpyAsync(cnt, b->d_counters, sizeof(cnt), hipMemcpyDeviceToHost, copy_stream));
    MK_HIP(hipMemcpyAsync(hist, row, sizeof(uint64_t) * nc, hipMemcpyDeviceToHost, copy_stream));
    MK_HIP(hipStreamSynchronize(copy_stream));
    if (cnt[kErrors] != 0 || cnt[kAdjOverflow] != 0)
        return fail(MK_EDEVICE, "device-side check failed (%u lookup/plan errors, %u adjacency overflows)",
                    cnt[kErrors], cnt[kAdjOverflow]);
    return MK_OK;
}

// Copy the histograms of a prepared batch whose last slice is known to be
// finished (its event completed) on `copy_stream`, check the device-side
// counters, and wait only for that copy.
int batch_collect(mk_batch *b, uint64_t *hist, hipStream_t copy_stream)
{
    MK_HIP(hipSetDevice(b->ctx->device));
    if (b->ng == 0) return MK_OK;
    int rc = batch_launch_finish(b, b->d_hist_own, copy_stream);
    if (rc) return rc;
    uint32_t cnt[kNumCounters];
    MK_HIP(hipMemcpyAsync(cnt, b->d_counters, sizeof(cnt), hipMemcpyDeviceToHost, copy_stream));
    MK_HIP(hipMemcpyAsync(hist, b->d_hist_own,
                          sizeof(uint64_t) * (size_t)b->ng * b->table->num_classes,
                          hipMemcpyDeviceToHost, copy_stream));
    MK_HIP(hipStreamSynchronize(copy_stream));
    if (cnt[kErrors] != 0 || cnt[kAdjOverflow] != 0)
        return fail(MK_EDEVICE, "device-side check failed (%u lookup/plan errors, %u adjacency overflows)",
                    cnt[kErrors], cnt[kAdjOverflow]);
    return MK_OK;
}

}  // namespace mk

extern "C" int mk_batch_timing(mk_batch *b, double *pass_ms, double *enum_ms)
{
    if (!b) return fail(MK_EINVAL, "mk_batch_timing: NULL batch");
    if (!b->hist_last || b->ng == 0) return fail(MK_EINVAL, "mk_batch_timing: batch has not run");
    std::lock_guard<std::recursive_mutex> lock(b->ctx->mu);
    MK_HIP(hipSetDevice(b->ctx->device));
    MK_HIP(hipEventSynchronize(b->ev[3]));
    float a = 0.f, e = -1.f;
    MK_HIP(hipEventElapsedTime(&a, b->ev[0], b->ev[3]));
    if (!(b->opts.use_graph == 2)) MK_HIP(hipEventElapsedTime(&e, b->ev[1], b->ev[2]));
    if (pass_ms) *pass_ms = a;
    if (enum_ms) *enum_ms = e;
    return MK_OK;
}

extern "C" int mk_batch_debug(mk_batch *b, int32_t flags)
{
    if (!b) return fail(MK_EINVAL, "mk_batch_debug: NULL batch");
    if (flags & ~(int32_t)(kDebugNoHash | kDebugFlushAlways | kDebugNoShare))
        return fail(MK_EINVAL, "mk_batch_debug: unknown flags %d", flags);
    std::lock_guard<std::recursive_mutex> lock(b->ctx->mu);
    if (b->debug_flags != flags) b->exec_hist = nullptr;  // captured with the old flags
    b->debug_flags = flags;
    return MK_OK;
}

extern "C" void mk_batch_free(mk_batch *b)
{
    if (!b) return;
    std::lock_guard<std::recursive_mutex> lock(b->ctx->mu);
    (void)hipSetDevice(b->ctx->device);
    if (b->last_stream) (void)hipStreamSynchronize(b->last_stream);
    (void)hipStreamSynchronize(b->ctx->stream);
    batch_release(b);
    delete b;
}

// --------------------------------------------------------------- autotune

// time one candidate: best whole-pass time over `trials` runs (the methods
// differ in their plans and the core method adds a division, so the pass is
// what compares); the histograms go to host memory in *hist
static int time_candidate(mk_ctx *ctx, const mk_graph *const *gs, int32_t ng, const mk_table *t,
                          const mk_batch_opts &o, int trials, double *ms,
                          std::vector<uint64_t> *hist, int *waves_per_cu = nullptr)
{
    mk_batch *b = nullptr;
    int rc = mk_batch_create(ctx, gs, ng, t, &o, &b);
    if (rc) return rc;
    if (waves_per_cu) *waves_per_cu = b->max_grid / std::max(ctx->num_cus, 1);
    double best = 1e30;
    for (int i = 0; i < trials && rc == MK_OK; ++i) {
        rc = mk_batch_run(b, nullptr, nullptr);
        double pass = 0, e = 0;
        if (!rc) rc = mk_batch_timing(b, &pass, &e);
        if (!rc) best = std::min(best, pass);
    }
    if (!rc) {
        hist->resize((size_t)ng * t->num_classes);
        rc = mk_batch_read(b, hist->data(), nullptr);
    }
    mk_batch_free(b);
    *ms = best;
    return rc;
}

extern "C" int mk_autotune(mk_ctx *ctx, const mk_graph *const *gs, int32_t ng, const mk_table *t,
                           int32_t trials, mk_batch_opts *best, double *best_ms,
                           double *default_ms)
{
    if (!ctx || !t || !best || (ng > 0 && !gs)) return fail(MK_EINVAL, "mk_autotune: NULL argument");
    if (ng <= 0) return fail(MK_EINVAL, "mk_autotune: no graphs");
    trials = std::max(trials, 1);
    mk_batch_opts cur{};
    cur.use_graph = 1;
    std::vector<uint64_t> ref, h;
    double cur_ms = 0;
    int per_cu = 0;
    int rc = time_candidate(ctx, gs, ng, t, cur, trials, &cur_ms, &ref, &per_cu);
    if (rc) return rc;
    if (default_ms) *default_ms = cur_ms;
    auto trial = [&](mk_batch_opts o) -> int {
        double ms = 0;
        int r = time_candidate(ctx, gs, ng, t, o, trials, &ms, &h);
        if (r == MK_ERANGE) return MK_OK;  // not applicable to these graphs
        if (r) return r;
        if (h != ref) return fail(MK_EDEVICE, "mk_autotune: a candidate changed the histograms");
        if (ms < cur_ms) {
            cur_ms = ms;
            cur = o;
        }
        return MK_OK;
    };
    // coordinate search: method, arc tests, split floor, units per grab,
    // waves per CU
    {
        mk_batch_opts o = cur;
        o.method = MK_METHOD_CORES;
        if ((rc = trial(o))) return rc;
    }
    {
        int max_n = 0;
        for (int i = 0; i < ng; ++i) max_n = std::max(max_n, gs[i]->n);
        if (max_n <= MK_LDS_MARKS_MAX_VERTICES) {
            const mk_batch_opts base0 = cur;
            for (int a : {MK_ADJ_BITS, MK_ADJ_LISTS}) {
                mk_batch_opts o = base0;
                o.adjacency = a;
                if ((rc = trial(o))) return rc;
            }
        }
    }
    // work-unit granularity: the split floor (estimated subgraphs per unit,
    // below and above the defaults) and the planner's units per wave, two
    // passes of the two so that each is tried at the other's best
    static const uint64_t floors[] = {128, 256, 512, 1u << 10, 1u << 12, 1u << 14, 1u << 18};
    static const int upws[] = {4, 8, 16, 32, 64, 128};
    for (int pass = 0; pass < 2; ++pass) {
        const mk_batch_opts base1 = cur;
        for (uint64_t f : floors) {
            mk_batch_opts o = base1;
            o.split_threshold = f;
            if ((rc = trial(o))) return rc;
        }
        const mk_batch_opts base2 = cur;
        for (int u : upws) {
            mk_batch_opts o = base2;
            o.units_per_wave = u;
            if ((rc = trial(o))) return rc;
        }
    }
    static const int grabs[] = {1, 4, 16, 64};
    const mk_batch_opts base2 = cur;
    for (int g : grabs) {
        mk_batch_opts o = base2;
        o.units_per_grab = g;
        if ((rc = trial(o))) return rc;
    }
    if (per_cu > 2) {
        const mk_batch_opts base3 = cur;
        for (int wpc : {per_cu / 2, (3 * per_cu) / 4}) {
            mk_batch_opts o = base3;
            o.waves_per_cu = wpc;
            if ((rc = trial(o))) return rc;
        }
    }
    *best = cur;
    if (best_ms) *best_ms = cur_ms;
    return MK_OK;
}

// ------------------------------------------------------------------ count

extern "C" int mk_count_batch(mk_ctx *ctx, const mk_graph *const *gs, int32_t ng,
                              const mk_table *t, uint64_t *hist, uint64_t *totals)
{
    if (!ctx || !t || (ng > 0 && (!gs || !hist)))
        return fail(MK_EINVAL, "mk_count_batch: NULL argument");
    mk_batch_opts o{};
    o.use_graph = -1;
    mk_batch *b = nullptr;
    int rc = mk_batch_create(ctx, gs, ng, t, &o, &b);
    if (rc) return rc;
    rc = mk_batch_run(b, nullptr, nullptr);
    if (!rc) rc = mk_batch_read(b, hist, totals);
    mk_batch_free(b);
    return rc;
}

extern "C" int mk_count(mk_ctx *ctx, const mk_graph *g, const mk_table *t, uint64_t *hist,
                        uint64_t *total)
{
    if (!g) return fail(MK_EINVAL, "mk_count: NULL graph");
    return mk_count_batch(ctx, &g, 1, t, hist, total);
}

// ------------------------------------------------------------------ k = 7

// slots of a context's k = 7 canonical-code cache: 2^22
constexpr int kK7CacheLog2 = 22;

// empty the context's canonical-code cache (keys, values, fill counter)
static int k7_cache_clear(mk_ctx *ctx, hipStream_t st)
{
    const size_t cache_slots = (size_t)1 << kK7CacheLog2;
    int rc = fill_u32(ctx->k7_cache_key, 0xFFFFFFFFu, 2 * cache_slots, st);
    if (!rc) rc = fill_u32(ctx->k7_cache_val, 0xFFFFFFFFu, 2 * cache_slots, st);
    if (!rc) rc = fill_u32(ctx->k7_cache_used, 0u, 1, st);
    if (!rc) ctx->k7_cache_fill = 0;
    return rc;
}

extern "C" int mk_k7_cache_info(mk_ctx *ctx, uint64_t *slots, uint64_t *used)
{
    if (!ctx) return fail(MK_EINVAL, "mk_k7_cache_info: NULL context");
    std::lock_guard<std::recursive_mutex> lock(ctx->mu);
    if (slots) *slots = ctx->k7_cache_key ? (uint64_t)1 << kK7CacheLog2 : 0;
    if (used) *used = ctx->k7_cache_key ? ctx->k7_cache_fill : 0;
    return MK_OK;
}

extern "C" int mk_k7_cache_clear(mk_ctx *ctx)
{
    if (!ctx) return fail(MK_EINVAL, "mk_k7_cache_clear: NULL context");
    std::lock_guard<std::recursive_mutex> lock(ctx->mu);
    if (!ctx->k7_cache_key) return MK_OK;
    MK_HIP(hipSetDevice(ctx->device));
    int rc = k7_cache_clear(ctx, ctx->stream);
    if (rc) return rc;
    MK_HIP(hipStreamSynchronize(ctx->stream));
    return MK_OK;
}

// one k = 7 pass over a prepared batch with class tables of 2^class_log2
// slots per graph; *overflow tells whether a table was too small
static int count7_once(mk_batch *b, int class_log2, int64_t cap, uint64_t *codes,
                       uint64_t *counts, int64_t *n_classes, uint64_t *totals, double *kernel_ms,
                       bool *overflow)
{
    mk_ctx *ctx = b->ctx;
    hipStream_t st = ctx->stream;
    const int ng = b->ng;
    const size_t cache_slots = (size_t)1 << kK7CacheLog2;
    const size_t class_slots = ((size_t)1 << class_log2) * (size_t)ng;
    K7Launch a{};
    a.cache_log2 = kK7CacheLog2;
    a.class_log2 = class_log2;
    unsigned long long *d_out = nullptr, *d_n = nullptr;
    std::vector<void *> bufs;
    auto alloc = [&](void **p, size_t bytes) {
        hipError_t e = hipMalloc(p, std::max<size_t>(bytes, 8));
        if (e == hipSuccess) bufs.push_back(*p);
        return e;
    };
    auto release = [&]() {
        for (void *p : bufs) (void)hipFree(p);
    };
    // the canonical-code cache of the context: made and cleared once, then
    // kept warm across counts (its entries do not depend on the graphs)
    hipError_t e = hipSuccess;
    if (!ctx->k7_cache_key) {
        unsigned long long *ck = nullptr, *cv = nullptr;
        uint32_t *cu = nullptr;
        e = hipMalloc(&ck, 8 * cache_slots);
        if (e == hipSuccess) e = hipMalloc(&cv, 8 * cache_slots);
        if (e == hipSuccess) e = hipMalloc(&cu, 4);
        if (e != hipSuccess) {
            if (ck) (void)hipFree(ck);
            if (cv) (void)hipFree(cv);
            if (cu) (void)hipFree(cu);
            return fail(e == hipErrorOutOfMemory ? MK_ENOMEM : MK_EDEVICE,
                        "mk_count7: cache allocation: %s", hipGetErrorString(e));
        }
        ctx->k7_cache_key = ck;
        ctx->k7_cache_val = cv;
        ctx->k7_cache_used = cu;
        ctx->k7_cache_fill = cache_slots;  // forces the clear below
    }
    // a cache past half full is cleared before the count: its probes would
    // grow long and new codes could no longer be entered
    if (ctx->k7_cache_fill > cache_slots / 2) {
        int frc = k7_cache_clear(ctx, st);
        if (frc) return frc;
    }
    a.cache_key = ctx->k7_cache_key;
    a.cache_val = ctx->k7_cache_val;
    a.cache_used = ctx->k7_cache_used;
    e = alloc((void **)&a.class_key, 8 * class_slots);
    if (e == hipSuccess) e = alloc((void **)&a.class_cnt, 8 * class_slots);
    if (e == hipSuccess) e = alloc((void **)&a.totals, 8 * (size_t)ng);
    if (e == hipSuccess) e = alloc((void **)&a.overflow, 4);
    if (e == hipSuccess) e = alloc((void **)&d_n, 8 * (size_t)ng);
    if (e == hipSuccess) e = alloc((void **)&d_out, 16 * (size_t)ng * (size_t)cap);
    if (e == hipSuccess && b->marks == MK_MARKS_GLOBAL) {
        a.etag_stride = b->mark_stride;
        e = alloc((void **)&a.etag, a.etag_stride * (size_t)b->grid);
    }
    if (e != hipSuccess) {
        release();
        return fail(e == hipErrorOutOfMemory ? MK_ENOMEM : MK_EDEVICE, "mk_count7: allocation: %s",
                    hipGetErrorString(e));
    }
    unsigned long long *d_codes = d_out, *d_counts = d_out + (size_t)ng * (size_t)cap;
    int rc = fill_u32(a.class_key, 0xFFFFFFFFu, 2 * class_slots, st);
    if (!rc) rc = fill_u32(a.class_cnt, 0u, 2 * class_slots, st);
    if (!rc) rc = fill_u32(a.totals, 0u, 2 * (size_t)ng, st);
    if (!rc) rc = fill_u32(a.overflow, 0u, 1, st);
    if (!rc) rc = fill_u32(d_n, 0u, 2 * (size_t)ng, st);
    if (!rc && a.etag) rc = fill_u32(a.etag, 0u, a.etag_stride * (size_t)b->grid / 4, st);
    if (!rc) rc = batch_enqueue_prep(b, nullptr, st);
    EnumConfig cfg = enum_config(b);
    cfg.hash_bits = 0;  // the k = 7 kernel keeps its own hash of 64-bit codes
    if (!rc && hipEventRecord(b->ev[1], st) != hipSuccess) rc = fail(MK_EDEVICE, "event record");
    if (!rc) rc = launch_k7(b->d_graphs, b->d_units, b->unit_cap, b->d_counters, a, cfg, b->grid,
                            b->lds_bytes, st);
    if (!rc && hipEventRecord(b->ev[2], st) != hipSuccess) rc = fail(MK_EDEVICE, "event record");
    if (!rc) rc = launch_k7_collect(a, ng, cap, d_codes, d_counts, d_n, st);
    std::vector<unsigned long long> hn(ng), ht(ng);
    uint32_t cnt[kNumCounters], ovf = 0;
    auto copy = [&](void *dst, const void *src, size_t bytes) {
        if (!rc && bytes) {
            hipError_t ce = hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, st);
            if (ce != hipSuccess) rc = fail(MK_EDEVICE, "mk_count7: copy: %s", hipGetErrorString(ce));
        }
    };
    // the class counts first, then only each graph's own classes, straight
    // into the caller's lists
    copy(hn.data(), d_n, 8 * (size_t)ng);
    copy(ht.data(), a.totals, 8 * (size_t)ng);
    copy(cnt, b->d_counters, sizeof(cnt));
    copy(&ovf, a.overflow, 4);
    uint32_t used = 0;
    copy(&used, ctx->k7_cache_used, 4);
    if (!rc && hipStreamSynchronize(st) != hipSuccess) rc = fail(MK_EDEVICE, "mk_count7: sync");
    if (!rc) ctx->k7_cache_fill = used;
    const bool device_ok = !rc && cnt[kErrors] == 0 && cnt[kAdjOverflow] == 0 && ovf == 0;
    if (device_ok) {
        for (int g = 0; g < ng; ++g) {
            const size_t m = (size_t)std::min<int64_t>((int64_t)hn[g], cap);
            copy(codes + (size_t)g * cap, d_codes + (size_t)g * cap, 8 * m);
            copy(counts + (size_t)g * cap, d_counts + (size_t)g * cap, 8 * m);
        }
        if (!rc && hipStreamSynchronize(st) != hipSuccess) rc = fail(MK_EDEVICE, "mk_count7: sync");
    }
    float ms = 0.f;
    if (!rc) (void)hipEventElapsedTime(&ms, b->ev[1], b->ev[2]);
    release();
    if (rc) return rc;
    if (cnt[kErrors] != 0 || cnt[kAdjOverflow] != 0)
        return fail(MK_EDEVICE, "device-side check failed (%u errors, %u adjacency overflows)",
                    cnt[kErrors], cnt[kAdjOverflow]);
    *overflow = ovf != 0;
    if (*overflow) return MK_OK;
    if (kernel_ms) *kernel_ms = ms;
    bool small = false;
    std::vector<std::pair<uint64_t, uint64_t>> pr;
    for (int g = 0; g < ng; ++g) {
        n_classes[g] = (int64_t)hn[g];
        if (totals) totals[g] = ht[g];
        const size_t m = (size_t)std::min<int64_t>((int64_t)hn[g], cap);
        small |= (int64_t)hn[g] > cap;
        uint64_t *gc = codes + (size_t)g * cap, *gv = counts + (size_t)g * cap;
        pr.resize(m);
        for (size_t i = 0; i < m; ++i) pr[i] = {gc[i], gv[i]};
        std::sort(pr.begin(), pr.end());
        for (size_t i = 0; i < m; ++i) {
            gc[i] = pr[i].first;
            gv[i] = pr[i].second;
        }
    }
    if (small) return fail(MK_ERANGE, "mk_count7: a graph has more classes than cap=%lld", (long long)cap);
    return MK_OK;
}

extern "C" int mk_count7(mk_ctx *ctx, const mk_graph *const *gs, int32_t ng, int64_t cap,
                         uint64_t *codes, uint64_t *counts, int64_t *n_classes, uint64_t *totals,
                         double *kernel_ms)
{
    if (!ctx || (ng > 0 && (!gs || !n_classes)) || (cap > 0 && ng > 0 && (!codes || !counts)))
        return fail(MK_EINVAL, "mk_count7: NULL argument");
    if (ng < 0 || cap < 0) return fail(MK_EINVAL, "mk_count7: negative ng or cap");
    // the output lists (code and count, 16 bytes a class) must stay addressable
    if (ng > 0 && (uint64_t)cap > (UINT64_MAX / 64) / (uint64_t)ng)
        return fail(MK_ERANGE, "mk_count7: cap=%lld too large for %d graphs", (long long)cap, ng);
    for (int i = 0; i < ng; ++i) {
        if (!gs[i] || gs[i]->ctx != ctx)
            return fail(MK_EINVAL, "mk_count7: graph %d missing or of another context", i);
    }
    if (kernel_ms) *kernel_ms = 0.0;
    if (ng == 0) return MK_OK;
    std::lock_guard<std::recursive_mutex> lock(ctx->mu);
    MK_HIP(hipSetDevice(ctx->device));
    // marks in LDS with bit-matrix arc tests while they fit, else marks and
    // extension tags in device memory with arc tests on the lists
    int max_n = 0;
    for (int i = 0; i < ng; ++i) max_n = std::max(max_n, gs[i]->n);
    const bool big = max_n > MK_LDS_MARKS_MAX_VERTICES;
    mk_batch_opts o{};
    o.use_graph = -1;
    o.method = MK_METHOD_ESU;
    o.adjacency = big ? MK_ADJ_LISTS : MK_ADJ_BITS;
    o.marks = big ? MK_MARKS_GLOBAL : MK_MARKS_LDS;
    mk_batch *b = nullptr;
    int rc = batch_create(ctx, gs, ng, 7, nullptr, &o, &b);
    if (rc) return rc;
    // class tables of the size the last count needed (2^10 slots per graph
    // at first), 4x larger after an overflow
    for (int class_log2 = ctx->k7_class_log2;; class_log2 += 2) {
        bool overflow = false;
        rc = count7_once(b, class_log2, cap, codes, counts, n_classes, totals, kernel_ms,
                         &overflow);
        if (rc || !overflow) {
            if (!rc) ctx->k7_class_log2 = class_log2;
            break;
        }
        if (class_log2 >= 24) {
            rc = fail(MK_ERANGE, "mk_count7: more distinct classes than 2^%d slots hold", class_log2);
            break;
        }
    }
    mk_batch_free(b);
    return rc;
}
