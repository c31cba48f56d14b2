// Graph loading and the typed symmetric adjacency of Section 2.
//
// Section 2 splits the vertices around v into A(v) (bidirected neighbours),
// B(v) (out-only), C(v) (in-only) and N(v) (the rest), and works with
// delta(v) = A(v) u B(v) u C(v).  On the device every graph of a batch gets
// delta(v) as a sorted list whose entries carry the two-bit A/B/C type:
//   entry = (u << 2) | type,  type bit0 = arc v -> u,  bit1 = arc u -> v,
// so A = 3, B = 1, C = 2.
//
// Built from the out-adjacency CSR in four kernels: arcs are set in two n x n
// bit matrices (out-rows and in-rows), each vertex counts the union of its two
// rows, a per-graph scan turns counts into offsets, and each vertex writes its
// list by scanning its rows in ascending order (which sorts it for free).
// Where n x n matrices are too large (or not wanted), the lists are built
// by sorting each vertex's out- and in-arcs instead (launch_typed_lists).
#include <algorithm>

#include "internal.h"

namespace mk {

constexpr int kRowThreads = 256;

// one thread per arc u -> v (u found by binary search in the out-CSR)
__global__ void arcs_kernel(const DevGraph *graphs)
{
    const DevGraph &g = graphs[blockIdx.y];
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (g.n == 0 || e >= g.out_row[g.n]) return;
    int lo = 0, hi = g.n;  // u with out_row[u] <= e < out_row[u+1]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (g.out_row[mid] <= e) lo = mid;
        else hi = mid;
    }
    const int u = lo, v = g.out_col[e];
    const int w = g.words;
    atomicOr(&g.bits_out[(size_t)u * w + (v >> 5)], 1u << (v & 31));
    atomicOr(&g.bits_in[(size_t)v * w + (u >> 5)], 1u << (u & 31));
}

__global__ void degree_kernel(const DevGraph *graphs)
{
    const DevGraph &g = graphs[blockIdx.y];
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v > g.n) return;
    if (v == g.n) {
        g.urow[0] = 0;
        return;
    }
    const int w = g.words;
    const uint32_t *ro = g.bits_out + (size_t)v * w;
    const uint32_t *ri = g.bits_in + (size_t)v * w;
    int cnt = 0;
    for (int i = 0; i < w; ++i) cnt += __popc(ro[i] | ri[i]);
    g.urow[v + 1] = cnt;
}

// In-place inclusive scan of urow[1..n] (one workgroup per graph).
__global__ __launch_bounds__(kRowThreads) void rowscan_kernel(const DevGraph *graphs)
{
    __shared__ int wave_sums[kRowThreads / kWave];
    const DevGraph &g = graphs[blockIdx.x];
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
    int carry = 0;
    for (int base = 0; base < g.n; base += kRowThreads) {
        const int i = base + threadIdx.x;
        const int v = i < g.n ? g.urow[i + 1] : 0;
        int incl = v;
#pragma unroll
        for (int d = 1; d < kWave; d <<= 1) {
            const int o = __shfl_up(incl, d, kWave);
            if (lane >= d) incl += o;
        }
        if (lane == kWave - 1) wave_sums[wave] = incl;
        __syncthreads();
        int before = 0, all = 0;
#pragma unroll
        for (int q = 0; q < kRowThreads / kWave; ++q) {
            before += q < wave ? wave_sums[q] : 0;
            all += wave_sums[q];
        }
        if (i < g.n) g.urow[i + 1] = carry + before + incl;
        carry += all;
        __syncthreads();
    }
}

__global__ void adjfill_kernel(const DevGraph *graphs, uint32_t *counters)
{
    const DevGraph &g = graphs[blockIdx.y];
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= g.n) return;
    const int w = g.words;
    const uint32_t *ro = g.bits_out + (size_t)v * w;
    const uint32_t *ri = g.bits_in + (size_t)v * w;
    int pos = g.urow[v];
    for (int i = 0; i < w; ++i) {
        const uint32_t a = ro[i], b = ri[i];
        uint32_t m = a | b;
        while (m) {
            const int bit = __ffs(m) - 1;
            const uint32_t type = ((a >> bit) & 1u) | (((b >> bit) & 1u) << 1);
            if ((uint32_t)pos < g.nnz_cap) g.uadj[pos] = ((uint32_t)(i * 32 + bit) << 2) | type;
            else atomicAdd(&counters[kAdjOverflow], 1u);
            ++pos;
            m &= m - 1;
        }
    }
}

int launch_typed_csr(const DevGraph *d_graphs, int ng, int max_n, int64_t max_m,
                     uint64_t bits_words_total, uint32_t *bits_base, uint32_t *counters,
                     hipStream_t stream)
{
    if (ng <= 0) return MK_OK;
    int rc = fill_u32(bits_base, 0, bits_words_total, stream);
    if (rc != MK_OK) return rc;
    const dim3 grid((unsigned)((max_n + 1 + kRowThreads - 1) / kRowThreads), (unsigned)ng);
    const dim3 agrid((unsigned)std::max<int64_t>((max_m + kRowThreads - 1) / kRowThreads, 1),
                     (unsigned)ng);
    hipLaunchKernelGGL(arcs_kernel, agrid, dim3(kRowThreads), 0, stream, d_graphs);
    MK_HIP(hipGetLastError());
    hipLaunchKernelGGL(degree_kernel, grid, dim3(kRowThreads), 0, stream, d_graphs);
    MK_HIP(hipGetLastError());
    hipLaunchKernelGGL(rowscan_kernel, dim3((unsigned)ng), dim3(kRowThreads), 0, stream,
                       d_graphs);
    MK_HIP(hipGetLastError());
    hipLaunchKernelGGL(adjfill_kernel, grid, dim3(kRowThreads), 0, stream, d_graphs, counters);
    MK_HIP(hipGetLastError());
    return MK_OK;
}

// ------------------------------------------------ typed lists, no matrices
//
// For graphs whose n x n bit matrices would be too large (and as a variant
// for any graph): every arc u -> v gives a raw entry (v << 2 | 1) to u and
// (u << 2 | 2) to v; each vertex's raw entries are sorted (then the two
// entries of a bidirected pair are adjacent) and merged into one typed entry
// per neighbour.  Per-vertex arrays of the whole batch are indexed by
// vbase + v:
//   cnt[N]      raw counts, then merged degrees
//   roff[N+1]   exclusive scan of the raw counts
//   raw[2M]     raw entries, merged lists at the front of each vertex's range
//   uoff[N+1]   exclusive scan of the merged degrees
//   tmp         scan workspace

static uint64_t list_tmp_words(uint64_t total_n) { return scan_tmp_words(total_n + 1); }

uint64_t list_ws_words(uint64_t total_n, uint64_t total_m)
{
    return total_n + 2 * (total_n + 1) + 2 * total_m + list_tmp_words(total_n);
}

// arc e of the out-CSR: tail by binary search
__device__ __forceinline__ int arc_tail(const DevGraph &g, int e)
{
    int lo = 0, hi = g.n;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (g.out_row[mid] <= e) lo = mid;
        else hi = mid;
    }
    return lo;
}

__global__ void rawcount_kernel(const DevGraph *graphs, uint32_t *cnt)
{
    const DevGraph &g = graphs[blockIdx.y];
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (g.n == 0 || e >= g.out_row[g.n]) return;
    const int u = arc_tail(g, e), v = g.out_col[e];
    atomicAdd(&cnt[g.vbase + u], 1u);
    atomicAdd(&cnt[g.vbase + v], 1u);
}

// each end takes a slot counting down from the end of its range; cnt ends at 0
__global__ void rawfill_kernel(const DevGraph *graphs, uint32_t *cnt, const uint32_t *roff,
                               uint32_t *raw)
{
    const DevGraph &g = graphs[blockIdx.y];
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (g.n == 0 || e >= g.out_row[g.n]) return;
    const int u = arc_tail(g, e), v = g.out_col[e];
    const uint32_t xu = g.vbase + (uint32_t)u, xv = g.vbase + (uint32_t)v;
    raw[roff[xu] + atomicSub(&cnt[xu], 1u) - 1u] = ((uint32_t)v << 2) | 1u;
    raw[roff[xv] + atomicSub(&cnt[xv], 1u) - 1u] = ((uint32_t)u << 2) | 2u;
}

// One wave per vertex: bitonic sort of its raw entries in LDS (padded to a
// power of two with all-ones), then one typed entry per neighbour written
// to the front of its raw range; cnt receives the merged degree.
__global__ __launch_bounds__(kWave) void merge_kernel(const DevGraph *graphs, uint32_t *cnt,
                                                      const uint32_t *roff, uint32_t *raw)
{
    extern __shared__ uint32_t buf[];
    const DevGraph &g = graphs[blockIdx.y];
    const int v = blockIdx.x;
    if (v >= g.n) return;
    const int lane = threadIdx.x;
    const uint32_t x = g.vbase + (uint32_t)v;
    const uint32_t r0 = roff[x];
    const int len = (int)(roff[x + 1] - r0);
    int p = kWave;
    while (p < len) p <<= 1;
    for (int i = lane; i < p; i += kWave) buf[i] = i < len ? raw[r0 + i] : 0xFFFFFFFFu;
    __syncthreads();
    for (int size = 2; size <= p; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int t = lane; t < p / 2; t += kWave) {
                const int i = 2 * t - (t & (stride - 1));
                const int j = i + stride;
                const uint32_t a = buf[i], b = buf[j];
                const bool up = (i & size) == 0;
                if ((a > b) == up) {
                    buf[i] = b;
                    buf[j] = a;
                }
            }
            __syncthreads();
        }
    }
    int out = 0;
    for (int base = 0; base < len; base += kWave) {
        const int i = base + lane;
        uint32_t key = 0, t = 0;
        bool head = false;
        if (i < len) {
            key = buf[i];
            head = i == 0 || (buf[i - 1] >> 2) != (key >> 2);
            t = key & 3u;
            if (head && i + 1 < len && (buf[i + 1] >> 2) == (key >> 2)) t |= buf[i + 1] & 3u;
        }
        const unsigned long long bal = __ballot(head);
        if (head)
            raw[r0 + out + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32),
                                                         __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u))] =
                (key & ~3u) | t;
        out += __popcll(bal);
    }
    if (lane == 0) cnt[x] = (uint32_t)out;
}

// One wave per vertex: its merged list to the graph's uadj, its offset to
// urow (positions from the batch-wide scan, less the graph's first).
__global__ __launch_bounds__(kWave) void place_kernel(const DevGraph *graphs, const uint32_t *cnt,
                                                      const uint32_t *roff, const uint32_t *uoff,
                                                      const uint32_t *raw, uint32_t *counters)
{
    const DevGraph &g = graphs[blockIdx.y];
    const int v = blockIdx.x;
    const int lane = threadIdx.x;
    if (g.n == 0) {
        if (v == 0 && lane == 0) g.urow[0] = 0;
        return;
    }
    if (v >= g.n) return;
    const uint32_t x = g.vbase + (uint32_t)v;
    const uint32_t d = cnt[x];
    const uint32_t pos = uoff[x] - uoff[g.vbase];
    if ((uint64_t)pos + d > g.nnz_cap) {
        if (lane == 0) atomicAdd(&counters[kAdjOverflow], 1u);
        return;
    }
    for (uint32_t i = lane; i < d; i += kWave) g.uadj[pos + i] = raw[roff[x] + i];
    if (lane == 0) {
        g.urow[v] = (int32_t)pos;
        if (v == g.n - 1) g.urow[g.n] = (int32_t)(pos + d);
    }
}

int launch_typed_lists(const DevGraph *d_graphs, int ng, int max_n, int64_t max_m,
                       uint64_t total_n, uint64_t total_m, int max_raw, uint32_t *lists,
                       uint32_t *counters, hipStream_t stream)
{
    if (ng <= 0) return MK_OK;
    uint32_t *cnt = lists;
    uint32_t *roff = cnt + total_n;
    uint32_t *raw = roff + total_n + 1;
    uint32_t *uoff = raw + 2 * total_m;
    uint32_t *tmp = uoff + total_n + 1;
    int rc = fill_u32(cnt, 0, std::max<uint64_t>(total_n, 1), stream);
    if (rc != MK_OK) return rc;
    const dim3 agrid((unsigned)std::max<int64_t>((max_m + kRowThreads - 1) / kRowThreads, 1),
                     (unsigned)ng);
    hipLaunchKernelGGL(rawcount_kernel, agrid, dim3(kRowThreads), 0, stream, d_graphs, cnt);
    MK_HIP(hipGetLastError());
    rc = scan_u32(cnt, roff, total_n, 0, roff + total_n, tmp, stream);
    if (rc != MK_OK) return rc;
    hipLaunchKernelGGL(rawfill_kernel, agrid, dim3(kRowThreads), 0, stream, d_graphs, cnt, roff,
                       raw);
    MK_HIP(hipGetLastError());
    int p = kWave;
    while (p < max_raw) p <<= 1;
    const dim3 vgrid((unsigned)std::max(max_n, 1), (unsigned)ng);
    hipLaunchKernelGGL(merge_kernel, vgrid, dim3(kWave), sizeof(uint32_t) * (size_t)p, stream,
                       d_graphs, cnt, roff, raw);
    MK_HIP(hipGetLastError());
    rc = scan_u32(cnt, uoff, total_n, 0, uoff + total_n, tmp, stream);
    if (rc != MK_OK) return rc;
    hipLaunchKernelGGL(place_kernel, vgrid, dim3(kWave), 0, stream, d_graphs, cnt, roff, uoff,
                       raw, counters);
    MK_HIP(hipGetLastError());
    return MK_OK;
}

}  // namespace mk

using namespace mk;

extern "C" int mk_graph_load_csr(mk_ctx *ctx, int32_t n, const int32_t *row_ptr,
                                 const int32_t *col, mk_graph **out)
{
    if (!ctx || !out || !row_ptr) return fail(MK_EINVAL, "mk_graph_load_csr: NULL argument");
    *out = nullptr;
    if (n < 0) return fail(MK_EINVAL, "mk_graph_load_csr: n=%d < 0", n);
    if (n > MK_MAX_VERTICES)
        return fail(MK_ERANGE, "n=%d exceeds MK_MAX_VERTICES=%d", n, MK_MAX_VERTICES);
    if (row_ptr[0] != 0) return fail(MK_EGRAPH, "row_ptr[0]=%d, expected 0", row_ptr[0]);
    for (int v = 0; v < n; ++v)
        if (row_ptr[v + 1] < row_ptr[v])
            return fail(MK_EGRAPH, "row_ptr decreases at vertex %d", v);
    const int64_t m = row_ptr[n];
    if (m > 0 && !col) return fail(MK_EINVAL, "mk_graph_load_csr: col is NULL");

    // loops, range, repeated arcs: one marker per head vertex
    std::vector<int32_t> mark(n, -1), indeg(n, 0);
    for (int u = 0; u < n; ++u)
        for (int32_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
            const int32_t v = col[e];
            if (v < 0 || v >= n) return fail(MK_EGRAPH, "arc %d -> %d: head out of range", u, v);
            if (v == u) return fail(MK_EGRAPH, "self-loop at vertex %d", u);
            if (mark[v] == u) return fail(MK_EGRAPH, "repeated arc %d -> %d", u, v);
            mark[v] = u;
            indeg[v]++;
        }
    // undirected degree |out(v) u in(v)| for workspace sizing
    std::vector<int32_t> in_ptr(n + 1, 0), in_col(m > 0 ? m : 1);
    for (int v = 0; v < n; ++v) in_ptr[v + 1] = in_ptr[v] + indeg[v];
    std::vector<int32_t> fill(in_ptr.begin(), in_ptr.end() - (n > 0 ? 1 : 0));
    for (int u = 0; u < n; ++u)
        for (int32_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) in_col[fill[col[e]]++] = u;
    std::fill(mark.begin(), mark.end(), -1);
    int64_t nnz_u = 0;
    int32_t max_udeg = 0;
    for (int v = 0; v < n; ++v) {
        int32_t d = row_ptr[v + 1] - row_ptr[v];
        for (int32_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) mark[col[e]] = v;
        for (int32_t e = in_ptr[v]; e < in_ptr[v + 1]; ++e)
            if (mark[in_col[e]] != v) ++d;
        nnz_u += d;
        max_udeg = std::max(max_udeg, d);
    }
    if (max_udeg > MK_MAX_DEGREE)
        return fail(MK_ERANGE, "undirected degree %d exceeds MK_MAX_DEGREE=%d", max_udeg,
                    MK_MAX_DEGREE);

    std::lock_guard<std::recursive_mutex> lock(ctx->mu);
    MK_HIP(hipSetDevice(ctx->device));
    mk_graph *g = new mk_graph();
    g->ctx = ctx;
    g->n = n;
    g->m = m;
    g->nnz_u = nnz_u;
    g->max_udeg = max_udeg;
    hipError_t e1 = hipMalloc(&g->d_row, sizeof(int32_t) * ((size_t)n + 1));
    hipError_t e2 = hipMalloc(&g->d_col, sizeof(int32_t) * (size_t)std::max<int64_t>(m, 1));
    if (e1 != hipSuccess || e2 != hipSuccess) {
        if (g->d_row) (void)hipFree(g->d_row);
        if (g->d_col) (void)hipFree(g->d_col);
        delete g;
        return fail(MK_ENOMEM, "mk_graph_load_csr: device allocation failed");
    }
    hipError_t e3 = hipMemcpyAsync(g->d_row, row_ptr, sizeof(int32_t) * ((size_t)n + 1),
                                   hipMemcpyHostToDevice, ctx->stream);
    hipError_t e4 = m > 0 ? hipMemcpyAsync(g->d_col, col, sizeof(int32_t) * (size_t)m,
                                           hipMemcpyHostToDevice, ctx->stream)
                          : hipSuccess;
    hipError_t e5 = hipStreamSynchronize(ctx->stream);
    if (e3 != hipSuccess || e4 != hipSuccess || e5 != hipSuccess) {
        (void)hipFree(g->d_row);
        (void)hipFree(g->d_col);
        delete g;
        return fail(MK_EDEVICE, "mk_graph_load_csr: upload failed");
    }
    *out = g;
    return MK_OK;
}

extern "C" int mk_graph_info(const mk_graph *g, int32_t *n, int64_t *m, int32_t *max_degree)
{
    if (!g) return fail(MK_EINVAL, "mk_graph_info: NULL graph");
    if (n) *n = g->n;
    if (m) *m = g->m;
    if (max_degree) *max_degree = g->max_udeg;
    return MK_OK;
}

extern "C" void mk_graph_free(mk_graph *g)
{
    if (!g) return;
    (void)hipSetDevice(g->ctx->device);
    (void)hipStreamSynchronize(g->ctx->stream);
    if (g->d_row) (void)hipFree(g->d_row);
    if (g->d_col) (void)hipFree(g->d_col);
    delete g;
}
