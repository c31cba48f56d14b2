// The ensemble of random graphs and the significance of each class
// (Section 1: the subgraphs of a graph are counted in the graph and in a set
// of random graphs, and each class's frequency is compared with theirs).
//
// Random graphs: degree-preserving directed switches.  Graph r of an
// ensemble with seed s draws from SplitMix64 (Steele, Lea and Flood, 2014)
// seeded with output r of SplitMix64(s); attempt t takes outputs 2t and
// 2t+1, each mapped to an arc index in [0, m) by its high 32 bits times m.
// With arcs a -> b and c -> d the attempt is rejected when a = c or b = d
// (nothing would change), a = d or c = b (a loop), or a -> d or c -> b
// exists (a duplicate); otherwise the heads are swapped: a -> d, c -> b.
// Every arc keeps its CSR position, so the row offsets (out-degrees) and the
// in-degrees stay; attempts go on until the target number of switches is
// accepted or the attempt cap is reached.
//
// One workgroup per random graph, the paper's parallelism over the graphs of
// an ensemble: its 64 lanes copy the arcs and set an n x n arc bit matrix,
// run the chain 64 attempts at a time (tested together, committed in order
// in registers, re-tested where an earlier commit of the round touched them,
// written together), then count reciprocal arcs for the sizes of delta(v).  The output graphs are
// ordinary device-resident graphs, ready for a batch.
//
// Significance: per class, over the random graphs 1..R of a batch's
// histograms, the mean, the sample standard deviation (divisor R - 1) and
// z = (H_0 - mean) / std (0 where std = 0 and H_0 = mean, an infinity of
// the sign of H_0 - mean where std = 0 otherwise), in float64.
#include <algorithm>
#include <cmath>

#include "internal.h"

namespace mk {

__device__ __forceinline__ uint64_t splitmix(uint64_t seed, uint64_t i)
{
    uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ uint32_t draw_arc(uint64_t r, uint32_t m)
{
    return (uint32_t)(((r >> 32) * (uint64_t)m) >> 32);
}

// tail of every arc of the out-CSR, and the in-degrees
__global__ void tails_kernel(const int32_t *row, const int32_t *col, int n, int32_t *src,
                             int32_t *indeg)
{
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    for (int t = row[v]; t < row[v + 1]; ++t) {
        src[t] = v;
        atomicAdd(&indeg[col[t]], 1);
    }
}

struct ChainArgs {
    const int32_t *row, *col0, *src, *indeg;
    int n, words;
    uint32_t m;
    uint64_t seed, first, target, max_attempts;
    int32_t *const *cols;         // output heads, one array per graph of this launch
    uint32_t *bits;               // per graph of this launch: n x words
    int32_t *recip;               // per graph of this launch: n
    unsigned long long *stats;    // per graph of the ensemble: accepted, nnz_u, max |delta|
};

__global__ __launch_bounds__(kWave) void switch_kernel(ChainArgs a)
{
    const int lane = threadIdx.x;
    const uint64_t r = a.first + blockIdx.x;
    int32_t *col = a.cols[blockIdx.x];
    uint32_t *bits = a.bits + (size_t)blockIdx.x * a.n * a.words;
    int32_t *recip = a.recip + (size_t)blockIdx.x * a.n;
    for (size_t i = lane; i < (size_t)a.n * a.words; i += kWave) bits[i] = 0u;
    for (int v = lane; v < a.n; v += kWave) recip[v] = 0;
    __syncthreads();
    for (uint32_t t = lane; t < a.m; t += kWave) {
        const int u = a.src[t], v = a.col0[t];
        col[t] = v;
        atomicOr(&bits[(size_t)u * a.words + (v >> 5)], 1u << (v & 31));
    }
    __syncthreads();
    // The chain, 64 attempts per round: every lane draws and tests one
    // attempt against the state at the start of the round (one round trip
    // for all), then the attempts are committed in order without touching
    // memory.  An attempt whose arc slots, or whose tested arcs, an earlier
    // accepted attempt of the round has touched is decided again on the
    // current state: a slot's head is the one the latest accepted attempt
    // wrote there, an arc's presence is the stored bit flipped once per
    // accepted attempt that removed or added it.  So the result is that of
    // taking the attempts one by one.  The round's switches are then written
    // together: bits by XOR (order-free), each slot by its last writer.
    {
        const uint64_t stream = splitmix(a.seed, r);
        auto stored = [&](int u, int v) {
            return (bits[(size_t)u * a.words + (v >> 5)] >> (v & 31)) & 1u;
        };
        auto same = [](int u1, int v1, int u2, int v2) { return u1 == u2 && v1 == v2; };
        uint64_t accepted = 0, t0 = 0;
        while (a.m >= 2 && accepted < a.target && t0 < a.max_attempts) {
            const uint64_t t = t0 + (uint64_t)lane;
            uint32_t i = 0, j = 0;
            int ta = -1, hb = -1, tc = -1, hd = -1;
            bool ok = false;
            if (t < a.max_attempts) {
                i = draw_arc(splitmix(stream, 2 * t), a.m);
                j = draw_arc(splitmix(stream, 2 * t + 1), a.m);
                ta = a.src[i];
                hb = col[i];
                tc = a.src[j];
                hd = col[j];
                ok = ta != tc && hb != hd && ta != hd && tc != hb && !stored(ta, hd) &&
                     !stored(tc, hb);
            }
            // acc: this lane's attempt was accepted, with heads hb, hd as they
            // were then; sup_i / sup_j: a later accepted attempt rewrote slot i / j
            bool acc = false, sup_i = false, sup_j = false;
            // does an accepted attempt of this round flip arc (u, v)?  (its
            // removed arcs ta->hb, tc->hd and added ta->hd, tc->hb)
            auto flips = [&](int u, int v) {
                return acc && (same(ta, hb, u, v) || same(tc, hd, u, v) || same(ta, hd, u, v) ||
                               same(tc, hb, u, v));
            };
            int l = 0;
            for (; l < kWave; ++l) {
                if (accepted >= a.target || t0 + (uint64_t)l >= a.max_attempts) break;
                const uint32_t il = (uint32_t)__builtin_amdgcn_readlane((int)i, l);
                const uint32_t jl = (uint32_t)__builtin_amdgcn_readlane((int)j, l);
                const int al = __builtin_amdgcn_readlane(ta, l);
                const int cl = __builtin_amdgcn_readlane(tc, l);
                int bl = __builtin_amdgcn_readlane(hb, l);
                int dl = __builtin_amdgcn_readlane(hd, l);
                bool okl = __builtin_amdgcn_readlane((int)ok, l) != 0;
                const unsigned long long at_i = __ballot(acc && (i == il || j == il));
                const unsigned long long at_j = __ballot(acc && (i == jl || j == jl));
                const bool hit = (at_i | at_j) != 0ull ||
                                 __ballot(flips(al, dl) || flips(cl, bl)) != 0ull;
                if (hit) {
                    // current heads of slots il, jl: the latest writer's
                    if (at_i) {
                        const int k = 63 - __builtin_clzll(at_i);
                        bl = __builtin_amdgcn_readlane(i == il ? hd : hb, k);
                    }
                    if (at_j) {
                        const int k = 63 - __builtin_clzll(at_j);
                        dl = __builtin_amdgcn_readlane(i == jl ? hd : hb, k);
                    }
                    bool fine = al != cl && bl != dl && al != dl && cl != bl;
                    if (fine) {
                        // current presence of al->dl and cl->bl
                        const uint32_t p1 = (uint32_t)__popcll(__ballot(flips(al, dl))) & 1u;
                        const uint32_t p2 = (uint32_t)__popcll(__ballot(flips(cl, bl))) & 1u;
                        fine = (stored(al, dl) ^ p1) == 0u && (stored(cl, bl) ^ p2) == 0u;
                    }
                    okl = fine;
                }
                if (okl) {
                    if (acc && (i == il || i == jl)) sup_i = true;
                    if (acc && (j == il || j == jl)) sup_j = true;
                    if (lane == l) {
                        acc = true;
                        hb = bl;
                        hd = dl;
                    }
                    ++accepted;
                }
            }
            t0 += (uint64_t)l;
            if (acc) {
                atomicXor(&bits[(size_t)ta * a.words + (hb >> 5)], 1u << (hb & 31));
                atomicXor(&bits[(size_t)tc * a.words + (hd >> 5)], 1u << (hd & 31));
                atomicXor(&bits[(size_t)ta * a.words + (hd >> 5)], 1u << (hd & 31));
                atomicXor(&bits[(size_t)tc * a.words + (hb >> 5)], 1u << (hb & 31));
                if (!sup_i) col[i] = hd;
                if (!sup_j) col[j] = hb;
            }
            __syncthreads();
        }
        if (lane == 0) a.stats[3 * r] = accepted;
    }
    // reciprocal arcs: u -> v with v -> u
    for (uint32_t t = lane; t < a.m; t += kWave) {
        const int u = a.src[t], v = col[t];
        if ((bits[(size_t)v * a.words + (u >> 5)] >> (u & 31)) & 1u) atomicAdd(&recip[u], 1);
    }
    __syncthreads();
    // |delta(v)| = out + in - reciprocal
    unsigned long long sum = 0;
    int mx = 0;
    for (int v = lane; v < a.n; v += kWave) {
        const int d = (a.row[v + 1] - a.row[v]) + a.indeg[v] - recip[v];
        sum += (unsigned long long)d;
        mx = d > mx ? d : mx;
    }
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) {
        sum += __shfl_down(sum, o, kWave);
        const int other = __shfl_down(mx, o, kWave);
        mx = other > mx ? other : mx;
    }
    if (lane == 0) {
        a.stats[3 * r + 1] = sum;
        a.stats[3 * r + 2] = (unsigned long long)mx;
    }
}

__global__ void significance_kernel(const unsigned long long *hist, int ng, uint32_t nc,
                                    double *out)
{
    const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nc) return;
    const int R = ng - 1;
    double sum = 0.0;
    for (int r = 1; r <= R; ++r) sum += (double)hist[(size_t)r * nc + c];
    const double mean = sum / R;
    double ss = 0.0;
    for (int r = 1; r <= R; ++r) {
        const double d = (double)hist[(size_t)r * nc + c] - mean;
        ss += d * d;
    }
    const double sd = sqrt(ss / (R - 1));
    const double diff = (double)hist[c] - mean;
    double z = 0.0;
    if (sd > 0.0) z = diff / sd;
    else if (diff > 0.0) z = INFINITY;
    else if (diff < 0.0) z = -INFINITY;
    out[c] = mean;
    out[(size_t)nc + c] = sd;
    out[2 * (size_t)nc + c] = z;
}

}  // namespace mk

using namespace mk;

// bytes of bit matrix per launch of the chain kernel
static constexpr uint64_t kChainScratchBytes = 512ull << 20;

extern "C" int mk_randomise(mk_ctx *ctx, const mk_graph *g, int32_t count, uint64_t seed,
                            uint32_t switches_per_arc, mk_graph **out, uint64_t *accepted)
{
    if (!ctx || !g || (count > 0 && !out)) return fail(MK_EINVAL, "mk_randomise: NULL argument");
    if (count < 0) return fail(MK_EINVAL, "mk_randomise: count=%d < 0", count);
    if (g->ctx != ctx) return fail(MK_EINVAL, "mk_randomise: graph of another context");
    for (int i = 0; i < count; ++i) out[i] = nullptr;
    if (count == 0) return MK_OK;
    std::lock_guard<std::recursive_mutex> lock(ctx->mu);
    MK_HIP(hipSetDevice(ctx->device));
    const int n = g->n;
    const uint32_t m = (uint32_t)g->m;
    const int words = (n + 31) / 32;
    const uint64_t target = (uint64_t)switches_per_arc * m;
    const uint64_t max_attempts = 8 * target + 1024;
    hipStream_t st = ctx->stream;

    std::vector<mk_graph *> made;
    int32_t *src = nullptr, *indeg = nullptr, *recip = nullptr;
    uint32_t *bits = nullptr;
    int32_t **d_cols = nullptr;
    unsigned long long *stats = nullptr;
    int rc = MK_OK;
    auto cleanup = [&](bool drop_graphs) {
        for (void *p : {(void *)src, (void *)indeg, (void *)recip, (void *)bits, (void *)d_cols,
                        (void *)stats})
            if (p) (void)hipFree(p);
        if (drop_graphs)
            for (mk_graph *h : made) mk_graph_free(h);
    };
#define ENS_HIP(x)                                                                             \
    do {                                                                                       \
        hipError_t e_ = (x);                                                                   \
        if (e_ != hipSuccess) {                                                                \
            cleanup(true);                                                                     \
            return fail(e_ == hipErrorOutOfMemory ? MK_ENOMEM : MK_EDEVICE, "%s: %s", #x,      \
                        hipGetErrorString(e_));                                                \
        }                                                                                      \
    } while (0)

    std::vector<int32_t *> cols(count);
    for (int r = 0; r < count; ++r) {
        mk_graph *h = new mk_graph();
        h->ctx = ctx;
        h->n = n;
        h->m = g->m;
        made.push_back(h);
        ENS_HIP(hipMalloc(&h->d_row, sizeof(int32_t) * ((size_t)n + 1)));
        ENS_HIP(hipMalloc(&h->d_col, sizeof(int32_t) * std::max<size_t>(m, 1)));
        ENS_HIP(hipMemcpyAsync(h->d_row, g->d_row, sizeof(int32_t) * ((size_t)n + 1),
                               hipMemcpyDeviceToDevice, st));
        cols[r] = h->d_col;
    }
    const uint64_t per_graph = 4ull * (uint64_t)n * words + 4ull * n;
    const int chunk = (int)std::max<uint64_t>(1, std::min<uint64_t>(count, kChainScratchBytes /
                                                                            std::max<uint64_t>(per_graph, 1)));
    ENS_HIP(hipMalloc(&src, sizeof(int32_t) * std::max<size_t>(m, 1)));
    ENS_HIP(hipMalloc(&indeg, sizeof(int32_t) * std::max(n, 1)));
    ENS_HIP(hipMalloc(&bits, sizeof(uint32_t) * std::max<size_t>((size_t)chunk * n * words, 1)));
    ENS_HIP(hipMalloc(&recip, sizeof(int32_t) * std::max<size_t>((size_t)chunk * n, 1)));
    ENS_HIP(hipMalloc(&d_cols, sizeof(int32_t *) * count));
    ENS_HIP(hipMalloc(&stats, sizeof(unsigned long long) * 3 * count));
    ENS_HIP(hipMemcpyAsync(d_cols, cols.data(), sizeof(int32_t *) * count, hipMemcpyHostToDevice, st));
    rc = fill_u32(indeg, 0, (size_t)std::max(n, 1), st);
    if (rc) {
        cleanup(true);
        return rc;
    }
    if (n > 0) {
        hipLaunchKernelGGL(tails_kernel, dim3((n + 255) / 256), dim3(256), 0, st, g->d_row,
                           g->d_col, n, src, indeg);
        ENS_HIP(hipGetLastError());
    }
    for (int first = 0; first < count; first += chunk) {
        const int cnt = std::min(chunk, count - first);
        ChainArgs a;
        a.row = g->d_row;
        a.col0 = g->d_col;
        a.src = src;
        a.indeg = indeg;
        a.n = n;
        a.words = words;
        a.m = m;
        a.seed = seed;
        a.first = (uint64_t)first;
        a.target = target;
        a.max_attempts = max_attempts;
        a.cols = d_cols + first;
        a.bits = bits;
        a.recip = recip;
        a.stats = stats;
        hipLaunchKernelGGL(switch_kernel, dim3(cnt), dim3(kWave), 0, st, a);
        ENS_HIP(hipGetLastError());
    }
    std::vector<unsigned long long> hs(3 * (size_t)count);
    ENS_HIP(hipMemcpyAsync(hs.data(), stats, sizeof(unsigned long long) * 3 * count,
                           hipMemcpyDeviceToHost, st));
    ENS_HIP(hipStreamSynchronize(st));
    for (int r = 0; r < count; ++r) {
        made[r]->nnz_u = (int64_t)hs[3 * r + 1];
        made[r]->max_udeg = (int32_t)hs[3 * r + 2];
        if (made[r]->max_udeg > MK_MAX_DEGREE) {
            cleanup(true);
            return fail(MK_ERANGE, "random graph %d has undirected degree %d > MK_MAX_DEGREE=%d", r,
                        (int)hs[3 * r + 2], MK_MAX_DEGREE);
        }
        if (accepted) accepted[r] = hs[3 * r];
    }
#undef ENS_HIP
    cleanup(false);
    for (int r = 0; r < count; ++r) out[r] = made[r];
    return MK_OK;
}

extern "C" int mk_significance(mk_ctx *ctx, const uint64_t *d_hist, int32_t ng,
                               uint32_t num_classes, double *d_out, void *stream)
{
    if (!ctx || (num_classes > 0 && (!d_hist || !d_out)))
        return fail(MK_EINVAL, "mk_significance: NULL argument");
    if (ng < 3) return fail(MK_EINVAL, "mk_significance: need the original and >= 2 random graphs (ng=%d)", ng);
    if (num_classes == 0) return MK_OK;
    std::lock_guard<std::recursive_mutex> lock(ctx->mu);
    MK_HIP(hipSetDevice(ctx->device));
    hipStream_t st = stream ? reinterpret_cast<hipStream_t>(stream) : ctx->stream;
    hipLaunchKernelGGL(significance_kernel, dim3((num_classes + 255) / 256), dim3(256), 0, st,
                       reinterpret_cast<const unsigned long long *>(d_hist), ng, num_classes, d_out);
    MK_HIP(hipGetLastError());
    return MK_OK;
}

extern "C" int mk_graph_read(const mk_graph *g, int32_t *row_ptr, int32_t *col)
{
    if (!g || (!row_ptr && !col)) return fail(MK_EINVAL, "mk_graph_read: NULL argument");
    mk_ctx *ctx = g->ctx;
    std::lock_guard<std::recursive_mutex> lock(ctx->mu);
    MK_HIP(hipSetDevice(ctx->device));
    if (row_ptr)
        MK_HIP(hipMemcpyAsync(row_ptr, g->d_row, sizeof(int32_t) * ((size_t)g->n + 1),
                              hipMemcpyDeviceToHost, ctx->stream));
    if (col && g->m > 0)
        MK_HIP(hipMemcpyAsync(col, g->d_col, sizeof(int32_t) * (size_t)g->m, hipMemcpyDeviceToHost,
                              ctx->stream));
    MK_HIP(hipStreamSynchronize(ctx->stream));
    return MK_OK;
}
