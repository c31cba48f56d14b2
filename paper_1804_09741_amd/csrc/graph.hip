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
