// Work-unit planner for the enumeration queue.
//
// The enumeration lists every connected k-set once from its smallest vertex
// v (the root) by ESU: the root's extension list is E_v = {u in delta(v) :
// u > v}; choosing its i-th vertex w_i gives the node (v, w_i), whose own
// extension list E2 is E_v[i+1:] followed by the neighbours of w_i that
// exceed v and are not in delta(v) (L2 vertices).  A work unit is a range of
// the children of such a node.  Child j (vertex x) of the node roots a
// subtree of roughly C(L2 - j - 1 + d(x) - 1, k - 3) subgraphs: its own
// extension list is the rest of E2 plus at most d(x) - 1 new neighbours.
// Children are packed greedily into ranges whose estimated sum stays under
// the split threshold, so hubs (the celebrity vertices of Section 3.1) are
// shared by many wavefronts while sparse parts stay one unit per node.
//
// Slots are the entries of the typed adjacency lists (one per (v, u) with
// u in delta(v)); a slot with u > v is a first-level node.  Pass one counts
// the units of every slot, a scan gives offsets, pass two writes the units.
// The order is graph by graph, root by root.
#include <algorithm>

#include "internal.h"
#include "server_hooks.h"

namespace mk {

constexpr int kPlanThreads = 256;

__device__ __forceinline__ uint64_t choose_small(int64_t n, int r)
{
    if (n < r) return 0;
    const uint64_t x = (uint64_t)n;
    switch (r) {
    case 0: return 1;
    case 1: return x;
    case 2: return x * (x - 1) / 2;
    case 3: return x * (x - 1) * (x - 2) / 6;
    default: return x * (x - 1) * (x - 2) / 6 * (x - 3) / 4;
    }
}

// A graph's descriptor as the planner reads it, with its arrays in the
// global address space.
struct PlanGraph {
    int32_t n;
    int32_t words;
    GPtr<const uint32_t> bits_out;
    GPtr<const uint32_t> bits_in;
    GPtr<const int32_t> urow;
    GPtr<const uint32_t> uadj;
    uint32_t slot_base;
    uint32_t nnz_cap;
};

__device__ __forceinline__ PlanGraph plan_graph(const DevGraph &d)
{
    PlanGraph g;
    g.n = d.n;
    g.words = d.words;
    g.bits_out = (GPtr<const uint32_t>)d.bits_out;
    g.bits_in = (GPtr<const uint32_t>)d.bits_in;
    g.urow = (GPtr<const int32_t>)d.urow;
    g.uadj = (GPtr<const uint32_t>)d.uadj;
    g.slot_base = d.slot_base;
    g.nnz_cap = d.nnz_cap;
    return g;
}

// vertex v with urow[v] <= e < urow[v+1]
__device__ __forceinline__ int owner_of(GPtr<const int32_t> urow, int n, int e)
{
    int lo = 0, hi = n;  // answer in [lo, hi)
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (urow[mid] <= e) lo = mid;
        else hi = mid;
    }
    return lo;
}

// first position in [r0, r1) whose vertex exceeds v (lists are sorted)
__device__ __forceinline__ int first_above(GPtr<const uint32_t> uadj, int r0, int r1, int v)
{
    int lo = r0, hi = r1;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if ((int)(uadj[mid] >> 2) > v) hi = mid;
        else lo = mid + 1;
    }
    return lo;
}

// x above v and not adjacent to v (so that it enters a node's extension
// list through another vertex): bit matrices when the batch has them, read
// without a branch so that unrolled iterations have their loads in flight
// together, else a search of the sorted lists (only for x above v)
__device__ __forceinline__ bool exclusive_above(const PlanGraph &g, int v, int x)
{
    if (!g.bits_out) return x > v && list_relation(g.urow, g.uadj, (uint32_t)v, (uint32_t)x) == 0u;
    const size_t w = (size_t)v * g.words + (x >> 5);
    return (x > v) & !(((g.bits_out[w] | g.bits_in[w]) >> (x & 31)) & 1u);
}

// Pass kinds of the planner kernel.
enum PlanPass : int { kEstimate = 0, kCount = 1, kEmit = 2 };

// Split threshold of the count and emit passes: the floor, raised so that
// the estimated total work makes about units_per_wave<K>(g) units per
// enumeration wave (large batches need little splitting, single graphs need
// more).  The defaults are the autotuner's picks on MI355X: 32 on
// bit-matrix graphs (the k = 6 batch of 31 graphs: 1.968 -> 1.929 ms per
// pass against 16; the k = 5 batch 25.58 -> 23.99 ms with the floor at
// 1,024 and one unit per grab) and 128 on graphs counted on sorted lists,
// past the bit-matrix limit -- typically one large graph whose hubs make
// the few largest units the tail of the launch (a power-law graph of 2^20
// vertices at k = 6: 197.8 -> 182.2 ms against 64).  k = 7 keeps 16: its
// units on a large graph re-push their first members' marks into device
// memory (64 cost 4% there).  A caller can set it per batch
// (mk_batch_opts.units_per_wave).
template <int K>
__device__ __forceinline__ uint64_t units_per_wave(const PlanGraph &g)
{
    return K >= 7 ? 16u : (!g.bits_out ? 128u : 32u);
}

template <int K>
__device__ __forceinline__ uint64_t effective_threshold(const PlanGraph &g,
                                                        const uint32_t *counters, uint64_t floor_t,
                                                        uint32_t waves, uint32_t upw)
{
    const uint64_t total = *reinterpret_cast<const unsigned long long *>(counters + kEstTotal);
    const uint64_t per_wave = upw ? (uint64_t)upw : units_per_wave<K>(g);
    const uint64_t adaptive = total / ((uint64_t)waves * per_wave + 1);
    return adaptive > floor_t ? adaptive : floor_t;
}

// Per-slot record of the estimate pass: (v, i) of a first-level node packed
// as v | i << 20 (n <= 2^20, degrees <= 4096), or kNoNode for a slot whose
// neighbour is not above its owner (no node has v = 2^20 - 1, i = 4095: the
// largest vertex has no neighbour above it).
constexpr int kViShift = 20;
constexpr uint32_t kViMask = (1u << kViShift) - 1u;
constexpr uint32_t kNoNode = 0xFFFFFFFFu;

// greedy ranges over the children of (v, w_i): calls put(r, j0 | j1 << 16,
// estimated cost) for every range when EMIT, returns the number of ranges
template <int K, bool EMIT, typename Put>
__device__ __forceinline__ uint32_t split_children(const PlanGraph &g, int v, int first, int r1,
                                                   int i, int y, int L2, uint64_t threshold,
                                                   uint64_t *est, Put put)
{
    uint32_t cnt = 0;
    int j = 0, j0 = 0;
    uint64_t acc = 0;
    auto child = [&](int dx) {
        const uint64_t cj = choose_small(L2 - j - 1 + dx - 1, K - 3) + 1;
        *est += cj;
        if (j > j0 && acc + cj > threshold) {
            if (EMIT) put(cnt, (uint32_t)j0 | ((uint32_t)j << 16), acc);
            ++cnt;
            j0 = j;
            acc = 0;
        }
        acc += cj;
        ++j;
    };
    // unrolled: the iterations' loads do not depend on one another
#pragma unroll 4
    for (int t = first + i + 1; t < r1; ++t) {
        const int x = (int)(g.uadj[t] >> 2);
        child(g.urow[x + 1] - g.urow[x]);
    }
    const int y0 = g.urow[y], y1 = g.urow[y + 1];
#pragma unroll 4
    for (int t = y0; t < y1; ++t) {
        const int x = (int)(g.uadj[t] >> 2);
        const int dx = g.urow[x + 1] - g.urow[x];
        if (exclusive_above(g, v, x)) child(dx);
    }
    if (L2 > j0) {
        if (EMIT) put(cnt, (uint32_t)j0 | ((uint32_t)L2 << 16), acc);
        ++cnt;
    }
    return cnt;
}

// extension length L2 of the node (v, w_i = y)
__device__ __forceinline__ int ext_len(const PlanGraph &g, int v, int ext_v, int i, int y)
{
    int fresh = 0;
    const int y0 = g.urow[y], y1 = g.urow[y + 1];
#pragma unroll 8
    for (int t = y0; t < y1; ++t) {
        const int x = (int)(g.uadj[t] >> 2);
        fresh += (int)exclusive_above(g, v, x);
    }
    return ext_v - i - 1 + fresh;
}

#ifndef MK_HEAVY_SHIFT
#define MK_HEAVY_SHIFT 1  // k = 5 core kernel 17.5 ms with 1, 17.8 with 2, 18.8 with 0
#endif

// x of a unit of graph gi with estimated cost est: kHeavyBit when est
// exceeds the split threshold >> MK_HEAVY_SHIFT (half of it)
__device__ __forceinline__ int unit_x(int gi, uint64_t est, uint64_t threshold)
{
    return (int)((uint32_t)gi | (est > (threshold >> MK_HEAVY_SHIFT) ? kHeavyBit : 0u));
}

// whether a first-level node of saturated estimate sest is cut into ranges
template <int K>
__device__ __forceinline__ bool node_split(uint32_t sest, uint64_t threshold)
{
    return K > 3 && (sest == 0xFFFFFFFFu || sest > threshold);
}

// One workgroup per (graph, 256 slots): blockIdx.y is the graph.  The
// estimate pass also counts each slot's units at the threshold spec_t (its
// walk over the children is the one the count pass would repeat); when the
// threshold comes out equal to spec_t -- the floor, or for a batch the
// threshold its sizing plan found, since a batch plans the same graphs
// every pass -- the count pass keeps those counts and returns at once.
template <int K, int PASS>
__global__ __launch_bounds__(kPlanThreads) void plan_kernel(const DevGraph *graphs,
                                                            uint32_t *slot_cnt,
                                                            const uint32_t *slot_off,
                                                            uint32_t *slot_est, uint32_t *slot_vi,
                                                            uint32_t *slot_l2,
                                                            int4 *units, uint32_t unit_cap,
                                                            uint64_t floor_t, uint64_t spec_t,
                                                            uint32_t waves,
                                                            uint32_t upw, uint32_t *counters)
{
    const int gi = blockIdx.y;
    const PlanGraph g = plan_graph(graphs[gi]);
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    uint64_t est = 0;  // kEstimate: this slot's estimated cost
    const bool live = g.n > 0 && e < min(g.urow[g.n], (int)g.nnz_cap);
    const uint64_t threshold = PASS == kEstimate ? ~0ull : effective_threshold<K>(g, counters, floor_t, waves, upw);
    if (PASS == kCount) {
        if (gi == 0 && e == 0)
            *reinterpret_cast<unsigned long long *>(counters + kPlanThreshold) = threshold;
        if (threshold == spec_t) {
            if (gi == 0 && e == 0) counters[kSplitPairs] = counters[kSpecSplitPairs];
            return;
        }
    }
    if (live) {
        const uint32_t slot = g.slot_base + (uint32_t)e;
        const int y = (int)(g.uadj[e] >> 2);
        if (PASS == kEstimate) {
            // the full walk: owner, position, extension length, child costs
            const int v = owner_of(g.urow, g.n, e);
            uint32_t vi = kNoNode, ranges = 0;
            if constexpr (K == 2) {
                // one unit per vertex, on its first list entry
                if (e == g.urow[v]) {
                    est = 1;
                    vi = (uint32_t)v;
                }
            } else if (y > v) {
                const int r1 = g.urow[v + 1];
                const int first = first_above(g.uadj, g.urow[v], r1, v);
                const int i = e - first;
                const int L2 = ext_len(g, v, r1 - first, i, y);
                slot_l2[slot] = (uint32_t)L2;
                if constexpr (K == 3) est = (uint64_t)L2 + 1;
                else ranges = split_children<K, false>(g, v, first, r1, i, y, L2, spec_t, &est,
                                                       [](uint32_t, uint32_t, uint64_t) {});
                vi = (uint32_t)v | ((uint32_t)i << kViShift);
            }
            slot_vi[slot] = vi;
            const uint32_t sest = est > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)est;
            slot_est[slot] = sest;
            uint32_t cnt = 0;  // units at the threshold spec_t
            if (vi != kNoNode) {
                cnt = node_split<K>(sest, spec_t) ? ranges : ((K > 3 && sest == 0u) ? 0u : 1u);
                if (cnt > 1) atomicAdd(&counters[kSpecSplitPairs], 1u);
            }
            slot_cnt[slot] = cnt;
        } else {
            const uint32_t vi = slot_vi[slot];
            const uint32_t sest = slot_est[slot];
            uint32_t cnt = 0;
            if (vi != kNoNode) {
                const int v = (int)(vi & kViMask), i = (int)(vi >> kViShift);
                const bool split = node_split<K>(sest, threshold);
                if (K <= 3) {
                    cnt = 1;
                } else if (sest <= 1 && !split) {
                    // no children below (v, w_i): L2 == 0 gives est 0
                    cnt = sest == 0 ? 0 : 1;
                } else if (!split) {
                    cnt = 1;
                } else if constexpr (K > 3) {
                    const int r1 = g.urow[v + 1];
                    const int first = e - i;
                    const int L2 = (int)slot_l2[slot];  // from the estimate pass
                    uint32_t base = 0;
                    if (PASS == kEmit) base = slot_off[slot];
                    auto put = [&](uint32_t r, uint32_t w, uint64_t c) {
                        const uint32_t idx = base + r;
                        if (idx < unit_cap) units[idx] = make_int4(unit_x(gi, c, threshold), v, i, (int)w);
                        else atomicOr(&counters[kErrors], 1u);
                    };
                    uint64_t dummy = 0;
                    cnt = PASS == kEmit
                              ? split_children<K, true>(g, v, first, r1, i, y, L2, threshold, &dummy, put)
                              : split_children<K, false>(g, v, first, r1, i, y, L2, threshold, &dummy, put);
                    if (PASS == kCount && cnt > 1) atomicAdd(&counters[kSplitPairs], 1u);
                }
                if (PASS == kEmit && cnt == 1 && !(K > 3 && split)) {
                    const uint32_t idx = slot_off[slot];
                    if (idx < unit_cap)
                        units[idx] = make_int4(unit_x(gi, sest, threshold), v, i, (int)kFullChild);
                    else atomicOr(&counters[kErrors], 1u);
                }
            }
            if (PASS == kCount) slot_cnt[slot] = cnt;
        }
    }
    if (PASS == kEstimate) {
        // workgroup sum, one 64-bit atomic per workgroup
        __shared__ unsigned long long part[kPlanThreads / kWave];
        unsigned long long x = est;
#pragma unroll
        for (int d = kWave / 2; d > 0; d >>= 1) x += __shfl_down(x, d, kWave);
        if (threadIdx.x % kWave == 0) part[threadIdx.x / kWave] = x;
        __syncthreads();
        if (threadIdx.x == 0) {
            unsigned long long sum = 0;
            for (int w = 0; w < kPlanThreads / kWave; ++w) sum += part[w];
            if (sum) atomicAdd(reinterpret_cast<unsigned long long *>(counters + kEstTotal), sum);
        }
    }
}

template <int K>
static int plan_k(const DevGraph *d_graphs, int ng, int64_t max_nnz, uint32_t total_slots,
                  uint32_t *slot_cnt, uint32_t *slot_off, uint32_t *slot_est, uint32_t *slot_vi,
                  uint32_t *slot_l2, uint32_t *scan_tmp, int4 *units, uint32_t unit_cap,
                  uint64_t threshold, uint64_t spec, uint32_t waves, uint32_t upw,
                  uint32_t *counters, hipStream_t stream)
{
    const dim3 grid((unsigned)std::max<int64_t>((max_nnz + kPlanThreads - 1) / kPlanThreads, 1),
                    (unsigned)ng);
    // the estimate total (counters[kEstTotal]) starts at zero: the callers
    // clear all counters before every plan
    hipLaunchKernelGGL((plan_kernel<K, kEstimate>), grid, dim3(kPlanThreads), 0, stream, d_graphs,
                       slot_cnt, slot_off, slot_est, slot_vi, slot_l2, units, unit_cap, threshold,
                       spec ? spec : threshold, waves, upw, counters);
    MK_HIP(hipGetLastError());
    hipLaunchKernelGGL((plan_kernel<K, kCount>), grid, dim3(kPlanThreads), 0, stream, d_graphs,
                       slot_cnt, slot_off, slot_est, slot_vi, slot_l2, units, unit_cap, threshold,
                       spec ? spec : threshold, waves, upw, counters);
    MK_HIP(hipGetLastError());
    int rc = scan_u32(slot_cnt, slot_off, total_slots, 0, &counters[kNumUnits], scan_tmp, stream);
    if (rc != MK_OK) return rc;
    if (!units) return MK_OK;  // sizing pass
    hipLaunchKernelGGL((plan_kernel<K, kEmit>), grid, dim3(kPlanThreads), 0, stream, d_graphs,
                       slot_cnt, slot_off, slot_est, slot_vi, slot_l2, units, unit_cap, threshold,
                       spec ? spec : threshold, waves, upw, counters);
    MK_HIP(hipGetLastError());
    return MK_OK;
}

// First work unit of every graph of a planned batch (the exclusive scan of
// the unit counts at the graph's first slot), and the total at out[ng].
// Units are emitted graph by graph, so graph gi owns [out[gi], out[gi+1]).
__global__ void unit_begins_kernel(const DevGraph *graphs, int ng, const uint32_t *slot_off,
                                   uint32_t total_slots, const uint32_t *counters, uint32_t *out)
{
    const int gi = blockIdx.x * blockDim.x + threadIdx.x;
    if (gi > ng) return;
    const uint32_t total = counters[kNumUnits];
    if (gi == ng) {
        out[gi] = total;
        return;
    }
    const uint32_t slot = graphs[gi].slot_base;
    out[gi] = slot < total_slots ? slot_off[slot] : total;
}

int launch_unit_begins(const DevGraph *d_graphs, int ng, const uint32_t *slot_off,
                       uint32_t total_slots, const uint32_t *counters, uint32_t *out,
                       hipStream_t stream)
{
    const int n = ng + 1;
    hipLaunchKernelGGL(unit_begins_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream,
                       d_graphs, ng, slot_off, total_slots, counters, out);
    MK_HIP(hipGetLastError());
    return MK_OK;
}

int launch_plan(int k, const DevGraph *d_graphs, int ng, int64_t max_nnz, uint32_t total_slots,
                uint32_t *slot_cnt, uint32_t *slot_off, uint32_t *slot_est, uint32_t *slot_vi,
                uint32_t *slot_l2, uint32_t *scan_tmp, int4 *units, uint32_t unit_cap,
                uint64_t split_threshold, uint64_t spec_threshold, uint32_t waves,
                uint32_t units_per_wave, uint32_t *counters, hipStream_t stream)
{
    if (ng <= 0) return MK_OK;
#define MK_PLAN(KK)                                                                         \
    plan_k<KK>(d_graphs, ng, max_nnz, total_slots, slot_cnt, slot_off, slot_est, slot_vi,  \
               slot_l2, scan_tmp, units, unit_cap, split_threshold, spec_threshold, waves, \
               units_per_wave, counters, stream)
    switch (k) {
    case 2: return MK_PLAN(2);
    case 3: return MK_PLAN(3);
    case 4: return MK_PLAN(4);
    case 5: return MK_PLAN(5);
    case 6: return MK_PLAN(6);
    case 7: return MK_PLAN(7);
    default: return fail(MK_ERANGE, "plan size k=%d outside 2..7", k);
    }
#undef MK_PLAN
}

}  // namespace mk
