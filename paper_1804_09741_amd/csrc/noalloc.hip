// Counting one graph without any allocation.
//
// mk_count_static runs the same path as a one-graph mk_count by enumeration
// (typed adjacency from bit matrices, work-unit plan, persistent enumeration
// with codes, lookups and histogram), but every device buffer the path needs
// besides the caller's graph, table and histogram -- counters, the graph's
// descriptor, bit matrices, typed lists, planner slots, scan workspace and
// work units -- is carved from one file-scope device array, `scratch`, of
// kStaticScratchBytes.  Its device address is looked up once per device at
// mk_init (static_scratch_init) and kept per device; host code never passes
// the array's own name to a kernel or a copy.
//
// Every call on a device shares that device's array and leaves its contents
// behind; each call clears what must start at zero (counters, bit matrices,
// the caller's histogram) with fill kernels.  Calls through one context are
// serialised (the context lock, and the call blocks until its work is done);
// calls from two contexts on one device at the same time race on the array.
#include <algorithm>
#include <mutex>

#include "internal.h"

namespace mk {

constexpr size_t kStaticScratchBytes = 64ull << 20;

// the static device array (one copy per device, for the life of the process)
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
constexpr uint32_t kMinStaticUnits = 1024;

std::mutex g_mu;
unsigned char *g_ptr[kMaxDevices] = {};

// the graph descriptor, written on the device from a kernel argument
__global__ void put_devgraph(DevGraph *dst, DevGraph g)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *dst = g;
}

size_t round_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

}  // namespace

// Look up this device's address of `scratch` (the device must be current).
int static_scratch_init(int device)
{
    std::lock_guard<std::mutex> lock(g_mu);
    if (device < 0 || device >= kMaxDevices)
        return fail(MK_ERANGE, "device %d beyond the %d the static scratch supports", device,
                    kMaxDevices);
    if (g_ptr[device]) return MK_OK;
    void *p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
        return fail(MK_EDEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", device,
                    hipGetErrorString(e));
    g_ptr[device] = static_cast<unsigned char *>(p);
    return MK_OK;
}

}  // namespace mk

using namespace mk;

extern "C" uint64_t mk_static_scratch_bytes(void) { return kStaticScratchBytes; }

extern "C" int mk_count_static(mk_ctx *ctx, const mk_graph *g, const mk_table *t,
                               uint64_t *d_hist, void *stream)
{
    if (!ctx || !g || !t || !d_hist) return fail(MK_EINVAL, "mk_count_static: NULL argument");
    if (g->ctx != ctx || t->ctx != ctx || !t->d_table)
        return fail(MK_EINVAL, "mk_count_static: graph or table of another context");
    if (t->k < 3 || t->k > 6) return fail(MK_ERANGE, "mk_count_static: k=%d outside 3..6", t->k);
    if (g->n > MK_LDS_MARKS_MAX_VERTICES)
        return fail(MK_ERANGE, "mk_count_static: n=%d exceeds %d (marks must fit LDS)", g->n,
                    MK_LDS_MARKS_MAX_VERTICES);
    std::lock_guard<std::recursive_mutex> lock(ctx->mu);
    MK_HIP(hipSetDevice(ctx->device));
    unsigned char *base = nullptr;
    {
        std::lock_guard<std::mutex> l2(g_mu);
        if (ctx->device >= 0 && ctx->device < kMaxDevices) base = g_ptr[ctx->device];
    }
    if (!base) return fail(MK_EDEVICE, "mk_count_static: static scratch not set up on device %d",
                           ctx->device);
    hipStream_t s = stream ? reinterpret_cast<hipStream_t>(stream) : ctx->stream;
    const int k = t->k;
    const uint32_t nc = t->num_classes;
    unsigned long long *hist = reinterpret_cast<unsigned long long *>(d_hist);
    int rc = fill_u32(hist, 0, (size_t)nc * 2, s);
    if (rc) return rc;
    if (g->n < k || g->nnz_u == 0) return hipStreamSynchronize(s) == hipSuccess
                                              ? MK_OK
                                              : fail(MK_EDEVICE, "mk_count_static: sync failed");

    // layout of the scratch: counters | descriptor | bit matrices | urow |
    // uadj | 5 planner slot arrays | scan workspace | work units
    const uint64_t n = (uint64_t)g->n, w = (n + 31) / 32, nnz = (uint64_t)g->nnz_u;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off = round_up(off + bytes, 256);
        return at;
    };
    const size_t o_cnt = take(4ull * kNumCounters);
    const size_t o_dg = take(sizeof(DevGraph));
    const size_t o_bits = take(4ull * 2 * n * w);
    const size_t o_urow = take(4ull * (n + 1));
    const size_t o_uadj = take(4ull * nnz);
    const size_t o_slot = take(4ull * 5 * nnz);
    const size_t o_scan = take(4ull * scan_tmp_words(nnz));
    const size_t o_units = off;
    const uint64_t unit_cap =
        o_units < kStaticScratchBytes ? (kStaticScratchBytes - o_units) / sizeof(int4) : 0;
    if (unit_cap < kMinStaticUnits)
        return fail(MK_ERANGE,
                    "mk_count_static: graph (n=%d, %lld adjacency entries) needs %zu bytes of "
                    "workspace; the static scratch holds %zu",
                    g->n, (long long)nnz, o_units + kMinStaticUnits * sizeof(int4),
                    kStaticScratchBytes);
    uint32_t *counters = reinterpret_cast<uint32_t *>(base + o_cnt);
    DevGraph *dg = reinterpret_cast<DevGraph *>(base + o_dg);
    uint32_t *slots = reinterpret_cast<uint32_t *>(base + o_slot);
    int4 *units = reinterpret_cast<int4 *>(base + o_units);

    DevGraph d{};
    d.n = g->n;
    d.words = (int32_t)w;
    d.out_row = g->d_row;
    d.out_col = g->d_col;
    d.bits_out = reinterpret_cast<uint32_t *>(base + o_bits);
    d.bits_in = d.bits_out + n * w;
    d.urow = reinterpret_cast<int32_t *>(base + o_urow);
    d.uadj = reinterpret_cast<uint32_t *>(base + o_uadj);
    d.slot_base = 0;
    d.nnz_cap = (uint32_t)nnz;
    d.vbase = 0;

    const int seg_cap = std::max(g->max_udeg, 1);
    const int lds = enum_lds_bytes(k, g->n, seg_cap, 0);
    if ((size_t)lds > ctx->max_lds)
        return fail(MK_ERANGE, "mk_count_static: %d bytes of LDS per wave (limit %zu)", lds,
                    ctx->max_lds);
    int per_cu = 0;
    rc = enum_max_blocks_per_cu(k, 0, lds, &per_cu);
    if (rc) return rc;
    const int grid = std::max(per_cu, 1) * ctx->num_cus;

    hipLaunchKernelGGL(put_devgraph, dim3(1), dim3(1), 0, s, dg, d);
    MK_HIP(hipGetLastError());
    rc = fill_u32(counters, 0, kNumCounters, s);
    if (!rc) rc = launch_typed_csr(dg, 1, g->n, g->m, 2 * n * w, d.bits_out, counters, s);
    if (!rc)
        rc = launch_plan(k, dg, 1, (int64_t)nnz, (uint32_t)nnz, slots, slots + nnz, slots + 2 * nnz,
                         slots + 3 * nnz, slots + 4 * nnz, reinterpret_cast<uint32_t *>(base + o_scan),
                         units, (uint32_t)std::min<uint64_t>(unit_cap, 0xFFFFFFFFull),
                         default_split_floor(k), 0, (uint32_t)grid, 0u, counters, s);
    EnumConfig cfg{};
    cfg.max_n = g->n;
    cfg.seg_cap = seg_cap;
    cfg.hash_bits = enum_hash_bits(k);
    if (!rc)
        rc = launch_enum(k, dg, units, (uint32_t)std::min<uint64_t>(unit_cap, 0xFFFFFFFFull),
                         kAllUnits, counters, t->d_table, nc, hist, cfg, grid, lds, s);
    if (rc) return rc;
    uint32_t cnt[kNumCounters];
    MK_HIP(hipMemcpyAsync(cnt, counters, sizeof(cnt), hipMemcpyDeviceToHost, s));
    MK_HIP(hipStreamSynchronize(s));
    if (cnt[kNumUnits] > unit_cap)
        return fail(MK_ERANGE, "mk_count_static: the plan needs %u work units; the static "
                               "scratch holds %llu for this graph",
                    cnt[kNumUnits], (unsigned long long)unit_cap);
    if (cnt[kErrors] != 0 || cnt[kAdjOverflow] != 0)
        return fail(MK_EDEVICE, "mk_count_static: device-side check failed (%u errors, %u "
                                "adjacency overflows)",
                    cnt[kErrors], cnt[kAdjOverflow]);
    return MK_OK;
}
