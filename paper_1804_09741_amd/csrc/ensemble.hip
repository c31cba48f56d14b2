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
// run the chain 64 attempts at a time (tested together; only the attempts
// that depend on an earlier one of the round are decided again, in order, in
// registers; written together), then count reciprocal arcs for the sizes of
// delta(v).  The output graphs are
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

// round-stamped LDS tables of the chain's dependence test (slots, arcs)
constexpr int kChainTableBits = 12;

__global__ __launch_bounds__(kWave) void switch_kernel(ChainArgs a)
{
    __shared__ uint32_t slot_tab[1 << kChainTableBits];
    __shared__ uint32_t arc_tab[1 << kChainTableBits];
    const int lane = threadIdx.x;
    for (int x = lane; x < (1 << kChainTableBits); x += kWave) {
        slot_tab[x] = 0u;
        arc_tab[x] = 0u;
    }
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
    // The chain, 64 attempts per round.  Every lane draws and tests one
    // attempt against the state at the start of the round (one round trip
    // for all).  An attempt's outcome can differ from that test only if an
    // earlier accepted attempt of the round rewrote one of its two arc slots
    // or flipped one of the two arcs it tests.  So: (1) each lane registers
    // its slots and its four switch arcs (as drawn) in round-stamped LDS
    // tables and finds whether an earlier attempt registered one of its
    // slots or tested arcs -- a dependence (hash collisions only add
    // dependences); (2) attempts without one keep their test, the others are
    // decided in order on the current state -- a slot's head from its latest
    // accepted writer, an arc's presence from the stored bit and the parity
    // of the round's accepted flips; an accepted attempt whose heads differ
    // from its draw marks the later attempts it touches as dependent too;
    // (3) the round's switches are written together (bits by XOR,
    // order-free; each slot by its last writer).  The result is that of
    // taking the attempts one by one.
    {
        const uint64_t stream = splitmix(a.seed, r);
        auto stored = [&](int u, int v) {
            return (bits[(size_t)u * a.words + (v >> 5)] >> (v & 31)) & 1u;
        };
        auto same = [](int u1, int v1, int u2, int v2) { return u1 == u2 && v1 == v2; };
        auto slot_hash = [](uint32_t x) { return (x * 2654435761u) >> (32 - kChainTableBits); };
        auto arc_hash = [](int u, int v) {
            return (((uint32_t)u * 8192u + (uint32_t)v) * 2654435761u) >> (32 - kChainTableBits);
        };
        uint64_t accepted = 0, t0 = 0;
        uint32_t round = 0;
        while (a.m >= 2 && accepted < a.target && t0 < a.max_attempts) {
            if (++round == (1u << 26)) {
                // stamps would wrap: start the tables afresh
                for (int x = lane; x < (1 << kChainTableBits); x += kWave) {
                    slot_tab[x] = 0u;
                    arc_tab[x] = 0u;
                }
                round = 1;
                __syncthreads();
            }
            const uint64_t t = t0 + (uint64_t)lane;
            const bool live = t < a.max_attempts;
            uint32_t i = 0, j = 0;
            int ta = -1, hb = -1, tc = -1, hd = -1;
            bool ok = false;
            uint32_t s1 = 1, s2 = 1;  // stored bits of the tested arcs ta->hd, tc->hb
            if (live) {
                i = draw_arc(splitmix(stream, 2 * t), a.m);
                j = draw_arc(splitmix(stream, 2 * t + 1), a.m);
                ta = a.src[i];
                hb = col[i];
                tc = a.src[j];
                hd = col[j];
                s1 = stored(ta, hd);
                s2 = stored(tc, hb);
                ok = ta != tc && hb != hd && ta != hd && tc != hb && !s1 && !s2;
            }
            // (1) dependences: the lowest lane of this round holding a bucket wins
            const uint32_t stamp = (round << 6) | (uint32_t)(63 - lane);
            if (live) {
                atomicMax(&slot_tab[slot_hash(i)], stamp);
                atomicMax(&slot_tab[slot_hash(j)], stamp);
                atomicMax(&arc_tab[arc_hash(ta, hb)], stamp);
                atomicMax(&arc_tab[arc_hash(tc, hd)], stamp);
                atomicMax(&arc_tab[arc_hash(ta, hd)], stamp);
                atomicMax(&arc_tab[arc_hash(tc, hb)], stamp);
            }
            __syncthreads();
            auto earlier = [&](uint32_t e) {
                return (e >> 6) == round && (int)(63u - (e & 63u)) < lane;
            };
            const bool dep = live && (earlier(slot_tab[slot_hash(i)]) || earlier(slot_tab[slot_hash(j)]) ||
                                      earlier(arc_tab[arc_hash(ta, hd)]) ||
                                      earlier(arc_tab[arc_hash(tc, hb)]));
            // (2) decisions: independent attempts keep their test
            bool acc = live && ok && !dep;
            unsigned long long pending = __ballot(dep);
            unsigned long long redone = 0ull;
            while (pending) {
                const int l = __builtin_ctzll(pending);
                pending &= pending - 1ull;
                redone |= 1ull << l;
                const uint32_t il = (uint32_t)__builtin_amdgcn_readlane((int)i, l);
                const uint32_t jl = (uint32_t)__builtin_amdgcn_readlane((int)j, l);
                const int al = __builtin_amdgcn_readlane(ta, l);
                const int cl = __builtin_amdgcn_readlane(tc, l);
                const int bl0 = __builtin_amdgcn_readlane(hb, l);
                const int dl0 = __builtin_amdgcn_readlane(hd, l);
                // the round's accepted attempts before l, with their applied heads
                const bool prior = acc && lane < l;
                const unsigned long long at_i = __ballot(prior && (i == il || j == il));
                const unsigned long long at_j = __ballot(prior && (i == jl || j == jl));
                int bl = bl0, dl = dl0;
                if (at_i) {
                    const int k = 63 - __builtin_clzll(at_i);
                    bl = __builtin_amdgcn_readlane(i == il ? hd : hb, k);
                }
                if (at_j) {
                    const int k = 63 - __builtin_clzll(at_j);
                    dl = __builtin_amdgcn_readlane(i == jl ? hd : hb, k);
                }
                auto flips = [&](int u, int v) {
                    return prior && (same(ta, hb, u, v) || same(tc, hd, u, v) ||
                                     same(ta, hd, u, v) || same(tc, hb, u, v));
                };
                bool fine = al != cl && bl != dl && al != dl && cl != bl;
                if (fine) {
                    // stored bits: those read at the draw while the heads are as drawn
                    const bool drawn = bl == bl0 && dl == dl0;
                    const uint32_t b1 = drawn ? (uint32_t)__builtin_amdgcn_readlane((int)s1, l)
                                              : stored(al, dl);
                    const uint32_t b2 = drawn ? (uint32_t)__builtin_amdgcn_readlane((int)s2, l)
                                              : stored(cl, bl);
                    const uint32_t p1 = (uint32_t)__popcll(__ballot(flips(al, dl))) & 1u;
                    const uint32_t p2 = (uint32_t)__popcll(__ballot(flips(cl, bl))) & 1u;
                    fine = (b1 ^ p1) == 0u && (b2 ^ p2) == 0u;
                }
                if (lane == l) {
                    acc = fine;
                    hb = bl;
                    hd = dl;
                }
                if (fine && (bl != bl0 || dl != dl0)) {
                    // heads other than drawn: later attempts whose tested
                    // arcs these switch arcs meet now depend on l
                    const bool touched =
                        lane > l && live &&
                        (same(al, bl, ta, hd) || same(cl, dl, ta, hd) || same(al, dl, ta, hd) ||
                         same(cl, bl, ta, hd) || same(al, bl, tc, hb) || same(cl, dl, tc, hb) ||
                         same(al, dl, tc, hb) || same(cl, bl, tc, hb));
                    pending |= __ballot(touched) & ~redone;
                }
            }
            // the target cut: attempts after the one that reaches it do not happen
            const unsigned long long accm = __ballot(acc);
            int cut = kWave;
            const uint64_t room = a.target - accepted;
            if ((uint64_t)__popcll(accm) >= room) {
                unsigned long long mm = accm;
                for (uint64_t q = 1; q < room; ++q) mm &= mm - 1ull;
                cut = __builtin_ctzll(mm) + 1;
            }
            if (t0 + (uint64_t)cut > a.max_attempts) cut = (int)(a.max_attempts - t0);
            acc = acc && lane < cut;
            accepted += (uint64_t)__popcll(__ballot(acc));
            // (3) write: each slot by its last accepted writer (a later writer
            // of a slot shares it with an earlier attempt, so it was redone),
            // bits by XOR
            bool sup_i = false, sup_j = false;
            unsigned long long later = __ballot(acc) & redone;
            while (later) {
                const int mlane = __builtin_ctzll(later);
                later &= later - 1ull;
                const uint32_t im = (uint32_t)__builtin_amdgcn_readlane((int)i, mlane);
                const uint32_t jm = (uint32_t)__builtin_amdgcn_readlane((int)j, mlane);
                sup_i |= lane < mlane && (i == im || i == jm);
                sup_j |= lane < mlane && (j == im || j == jm);
            }
            if (acc) {
                atomicXor(&bits[(size_t)ta * a.words + (hb >> 5)], 1u << (hb & 31));
                atomicXor(&bits[(size_t)tc * a.words + (hd >> 5)], 1u << (hd & 31));
                atomicXor(&bits[(size_t)ta * a.words + (hd >> 5)], 1u << (hd & 31));
                atomicXor(&bits[(size_t)tc * a.words + (hb >> 5)], 1u << (hb & 31));
                if (!sup_i) col[i] = hd;
                if (!sup_j) col[j] = hb;
            }
            t0 += (uint64_t)cut;
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
    // each chain keeps an n x n arc bit matrix
    if (g->n > MK_LDS_MARKS_MAX_VERTICES)
        return fail(MK_ERANGE, "mk_randomise: n=%d exceeds %d", g->n, MK_LDS_MARKS_MAX_VERTICES);
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
