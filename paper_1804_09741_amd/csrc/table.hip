// Code -> class table (Section 3.2 of arXiv 1804.09741: isomorphism in O(1)
// through a precomputed table keyed by the adjacency matrix).
//
// For every k(k-1)-bit adjacency code c the table holds the class id of the
// digraph c, or MK_INVALID_CLASS when c is not weakly connected.  The class
// of c is represented by its canonical code, the minimum over all k! vertex
// relabelings of c; ids are the ranks of the canonical codes of connected
// classes.
//
// Build, all on the GPU:
//   1. canon pass: every lane owns 32 codes, spaced one wavefront apart so
//      that stores coalesce, and walks all k! relabelings of them with one
//      adjacent transposition per step (Steinhaus-Johnson-Trotter order).
//      Swapping vertices a and a+1 of a code is two delta swaps: rows a and
//      a+1 trade places as whole (k-1)-bit fields, and in every other row the
//      two neighbouring column bits for a and a+1 trade places.  The running
//      minimum is the canonical code.  A wavefront ballot marks the codes
//      that are their own canonical form and connected ("representatives").
//   2. rank: exclusive prefix sum of the popcounts of the representative
//      bitmap.
//   3. class list (representatives in rank order) and final pass: entry c
//      becomes rank(canonical(c)) or MK_INVALID_CLASS.
//
// The pass is plain integer ALU work: k = 6 is 2^30 codes x 719 steps of
// about nine VALU operations each.
#include <algorithm>
#include <numeric>
#include <set>

#include "internal.h"

namespace mk {

struct SwapMasks {
    uint32_t row;  // bits of row a (its lower field of the row swap)
    uint32_t col;  // lower bit of each (a, a+1) column pair outside rows a, a+1
};

constexpr int kMaxSteps = 719;  // 6! - 1
__constant__ SwapMasks c_swaps[kMaxSteps];

static int bit_pos(int k, int i, int j) { return i * (k - 1) + j - (j > i ? 1 : 0); }

// Positions a (swap a, a+1) of the Steinhaus-Johnson-Trotter order of S_k.
static std::vector<int> sjt_positions(int k)
{
    std::vector<int> perm(k), dir(k, -1), out;
    std::iota(perm.begin(), perm.end(), 0);
    for (;;) {
        int best = -1, pos = -1;
        for (int i = 0; i < k; ++i) {
            int j = i + dir[perm[i]];
            if (j >= 0 && j < k && perm[j] < perm[i] && perm[i] > best) {
                best = perm[i];
                pos = i;
            }
        }
        if (best < 0) break;
        int j = pos + dir[best];
        std::swap(perm[pos], perm[j]);
        out.push_back(std::min(pos, j));
        for (int v = best + 1; v < k; ++v) dir[v] = -dir[v];
    }
    return out;
}

static std::vector<SwapMasks> swap_masks(int k, const std::vector<int> &seq)
{
    std::vector<SwapMasks> out;
    for (int a : seq) {
        SwapMasks m;
        m.row = ((1u << (k - 1)) - 1) << (a * (k - 1));
        m.col = 0;
        for (int r = 0; r < k; ++r)
            if (r != a && r != a + 1) m.col |= 1u << bit_pos(k, r, a);
        out.push_back(m);
    }
    return out;
}

// Check on the host that the step sequence visits every relabeling once.
static bool sequence_covers_group(int k, const std::vector<int> &seq)
{
    std::vector<int> perm(k);
    std::iota(perm.begin(), perm.end(), 0);
    std::set<std::vector<int>> seen{perm};
    for (int a : seq) {
        std::swap(perm[a], perm[a + 1]);
        seen.insert(perm);
    }
    size_t fact = 1;
    for (int i = 2; i <= k; ++i) fact *= i;
    return seen.size() == fact && seq.size() == fact - 1;
}

template <int K>
__device__ __forceinline__ bool code_connected(uint32_t c)
{
    uint32_t und[K];
#pragma unroll
    for (int i = 0; i < K; ++i) und[i] = 0;
#pragma unroll
    for (int i = 0; i < K; ++i)
#pragma unroll
        for (int j = 0; j < K; ++j)
            if (i != j) {
                const int b = i * (K - 1) + j - (j > i ? 1 : 0);
                const uint32_t on = (c >> b) & 1u;
                und[i] |= on << j;
                und[j] |= on << i;
            }
    uint32_t reach = 1;
#pragma unroll
    for (int r = 0; r < K - 1; ++r) {
        uint32_t nr = reach;
#pragma unroll
        for (int i = 0; i < K; ++i) nr |= ((reach >> i) & 1u) ? und[i] : 0u;
        reach = nr;
    }
    return reach == (1u << K) - 1;
}

template <int K, int NJ>
__global__ __launch_bounds__(256) void canon_kernel(uint32_t *table, uint32_t *repbits,
                                                    uint64_t ncodes, int steps)
{
    const int lane = threadIdx.x % kWave;
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const uint64_t base = wave * (uint64_t)(kWave * NJ);
    if (base >= ncodes) return;
    uint32_t x[NJ], best[NJ];
#pragma unroll
    for (int j = 0; j < NJ; ++j) x[j] = best[j] = (uint32_t)(base + j * kWave + lane);
    for (int s = 0; s < steps; ++s) {
        const uint32_t rm = c_swaps[s].row;
        const uint32_t cm = c_swaps[s].col;
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
            uint32_t v = x[j];
            uint32_t t = ((v >> (K - 1)) ^ v) & rm;
            v ^= t | (t << (K - 1));
            t = ((v >> 1) ^ v) & cm;
            v ^= t | (t << 1);
            x[j] = v;
            best[j] = min(best[j], v);
        }
    }
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
        const uint32_t c = (uint32_t)(base + j * kWave + lane);
        const bool conn = code_connected<K>(c);
        table[c] = conn ? best[j] : (best[j] | 0x80000000u);
        const unsigned long long rep = __ballot(conn && best[j] == c);
        if (lane == 0)
            reinterpret_cast<unsigned long long *>(repbits)[(base + j * kWave) / kWave] = rep;
    }
}

__global__ void classlist_kernel(const uint32_t *repbits, const uint32_t *rankbase,
                                 uint64_t nwords, uint32_t *classes)
{
    uint64_t w = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= nwords) return;
    uint32_t bits = repbits[w];
    uint32_t r = rankbase[w];
    while (bits) {
        const int b = __ffs(bits) - 1;
        classes[r++] = (uint32_t)(w * 32 + b);
        bits &= bits - 1;
    }
}

__global__ void assign_kernel(uint32_t *table, const uint32_t *repbits, const uint32_t *rankbase,
                              uint64_t ncodes)
{
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (; i < ncodes; i += stride) {
        const uint32_t x = table[i];
        if (x & 0x80000000u) {
            table[i] = MK_INVALID_CLASS;
        } else {
            const uint32_t w = x >> 5;
            table[i] = rankbase[w] + (uint32_t)__popc(repbits[w] & ((1u << (x & 31)) - 1u));
        }
    }
}

template <int K, int NJ>
static int launch_canon(uint32_t *table, uint32_t *repbits, uint64_t ncodes, int steps,
                        hipStream_t stream)
{
    const uint64_t waves = ncodes / (kWave * NJ);
    const uint64_t blocks = (waves * kWave + 255) / 256;
    hipLaunchKernelGGL((canon_kernel<K, NJ>), dim3((unsigned)blocks), dim3(256), 0, stream, table,
                       repbits, ncodes, steps);
    MK_HIP(hipGetLastError());
    return MK_OK;
}

// Cores of every class (the divisor of the (k-2)-set counting): subsets X
// of k-2 vertices whose induced subgraph is weakly connected and which both
// other vertices touch.  One thread per class, on bitmasks: nb[i] = vertices
// joined to i by an arc either way; X's connectivity by growing the set
// reached from its lowest vertex.
template <int K>
__global__ void core_mult_kernel(const uint32_t *classes, uint32_t n, uint8_t *mult)
{
    const uint32_t id = blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= n) return;
    const uint32_t code = classes[id];
    uint32_t nb[K];
#pragma unroll
    for (int i = 0; i < K; ++i) nb[i] = 0;
#pragma unroll
    for (int i = 0; i < K; ++i)
#pragma unroll
        for (int j = 0; j < K; ++j)
            if (i != j && ((code >> (i * (K - 1) + j - (j > i ? 1 : 0))) & 1u)) {
                nb[i] |= 1u << j;
                nb[j] |= 1u << i;
            }
    const uint32_t all = (1u << K) - 1u;
    uint32_t cores = 0;
#pragma unroll
    for (int y = 0; y < K; ++y)
#pragma unroll
        for (int z = y + 1; z < K; ++z) {
            const uint32_t x = all & ~(1u << y) & ~(1u << z);
            if (!(nb[y] & x) || !(nb[z] & x)) continue;
            uint32_t reach = x & (0u - x);
#pragma unroll
            for (int it = 0; it < K - 3; ++it) {
                uint32_t grow = 0;
#pragma unroll
                for (int i = 0; i < K; ++i)
                    if ((reach >> i) & 1u) grow |= nb[i];
                reach |= grow & x;
            }
            cores += reach == x ? 1u : 0u;
        }
    mult[id] = (uint8_t)cores;
}

static int launch_core_mult(int k, const uint32_t *classes, uint32_t n, uint8_t *mult,
                            hipStream_t stream)
{
    const dim3 grid((n + 255) / 256), block(256);
    switch (k) {
    case 3: hipLaunchKernelGGL(core_mult_kernel<3>, grid, block, 0, stream, classes, n, mult); break;
    case 4: hipLaunchKernelGGL(core_mult_kernel<4>, grid, block, 0, stream, classes, n, mult); break;
    case 5: hipLaunchKernelGGL(core_mult_kernel<5>, grid, block, 0, stream, classes, n, mult); break;
    case 6: hipLaunchKernelGGL(core_mult_kernel<6>, grid, block, 0, stream, classes, n, mult); break;
    default: return fail(MK_ERANGE, "k=%d outside 3..6", k);
    }
    MK_HIP(hipGetLastError());
    return MK_OK;
}

int build_table(Table *t, hipStream_t stream)
{
    const int k = t->k;
    const uint64_t ncodes = 1ull << (k * (k - 1));
    const uint64_t nwords = ncodes / 32;
    std::vector<int> seq = sjt_positions(k);
    if (!sequence_covers_group(k, seq))
        return fail(MK_EDEVICE, "relabeling sequence for k=%d is incomplete", k);
    std::vector<SwapMasks> masks = swap_masks(k, seq);
    MK_HIP(hipMemcpyToSymbolAsync(HIP_SYMBOL(c_swaps), masks.data(),
                                  masks.size() * sizeof(SwapMasks), 0, hipMemcpyHostToDevice,
                                  stream));

    uint32_t *repbits = nullptr, *rankbase = nullptr, *tmp = nullptr, *d_total = nullptr;
    int rc = MK_OK;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    auto cleanup = [&]() {
        if (repbits) (void)hipFree(repbits);
        if (rankbase) (void)hipFree(rankbase);
        if (tmp) (void)hipFree(tmp);
        if (d_total) (void)hipFree(d_total);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
    };
#define TRY(x)                                                                                \
    do {                                                                                      \
        rc = (x);                                                                             \
        if (rc != MK_OK) {                                                                    \
            cleanup();                                                                        \
            return rc;                                                                        \
        }                                                                                     \
    } while (0)
#define TRYHIP(x)                                                                             \
    do {                                                                                      \
        hipError_t e_ = (x);                                                                  \
        if (e_ != hipSuccess) {                                                               \
            cleanup();                                                                        \
            return fail(e_ == hipErrorOutOfMemory ? MK_ENOMEM : MK_EDEVICE, "%s: %s", #x,     \
                        hipGetErrorString(e_));                                               \
        }                                                                                     \
    } while (0)

    TRYHIP(hipMalloc(&t->d_table, ncodes * sizeof(uint32_t)));
    TRYHIP(hipMalloc(&repbits, nwords * sizeof(uint32_t)));
    TRYHIP(hipMalloc(&rankbase, nwords * sizeof(uint32_t)));
    TRYHIP(hipMalloc(&tmp, scan_tmp_words(nwords) * sizeof(uint32_t)));
    TRYHIP(hipMalloc(&d_total, sizeof(uint32_t)));
    TRYHIP(hipEventCreate(&e0));
    TRYHIP(hipEventCreate(&e1));
    TRYHIP(hipEventRecord(e0, stream));

    const int steps = (int)seq.size();
    switch (k) {
    case 3: TRY((launch_canon<3, 1>(t->d_table, repbits, ncodes, steps, stream))); break;
    case 4: TRY((launch_canon<4, 32>(t->d_table, repbits, ncodes, steps, stream))); break;
    case 5: TRY((launch_canon<5, 32>(t->d_table, repbits, ncodes, steps, stream))); break;
    case 6: TRY((launch_canon<6, 32>(t->d_table, repbits, ncodes, steps, stream))); break;
    default: cleanup(); return fail(MK_ERANGE, "k=%d outside 3..6", k);
    }
    TRY(scan_u32(repbits, rankbase, nwords, 1, d_total, tmp, stream));
    uint32_t num = 0;
    TRYHIP(hipMemcpyAsync(&num, d_total, sizeof(uint32_t), hipMemcpyDeviceToHost, stream));
    TRYHIP(hipStreamSynchronize(stream));
    if (num == 0) {
        cleanup();
        return fail(MK_EDEVICE, "class table for k=%d has no classes", k);
    }
    t->num_classes = num;
    TRYHIP(hipMalloc(&t->d_classes, (size_t)num * sizeof(uint32_t)));
    hipLaunchKernelGGL(classlist_kernel, dim3((unsigned)((nwords + 255) / 256)), dim3(256), 0,
                       stream, repbits, rankbase, nwords, t->d_classes);
    TRYHIP(hipGetLastError());
    const uint64_t ablocks = std::min<uint64_t>((ncodes + 255) / 256, 1u << 20);
    hipLaunchKernelGGL(assign_kernel, dim3((unsigned)ablocks), dim3(256), 0, stream, t->d_table,
                       repbits, rankbase, ncodes);
    TRYHIP(hipGetLastError());
    TRYHIP(hipMalloc(&t->d_core_mult, (size_t)num));
    TRY(launch_core_mult(k, t->d_classes, num, t->d_core_mult, stream));
    TRYHIP(hipEventRecord(e1, stream));
    t->classes.resize(num);
    TRYHIP(hipMemcpyAsync(t->classes.data(), t->d_classes, (size_t)num * sizeof(uint32_t),
                          hipMemcpyDeviceToHost, stream));
    TRYHIP(hipStreamSynchronize(stream));
    float ms = 0.f;
    TRYHIP(hipEventElapsedTime(&ms, e0, e1));
    t->build_ms = ms;
    t->entries = ncodes;
    cleanup();
#undef TRY
#undef TRYHIP
    return MK_OK;
}

}  // namespace mk

using namespace mk;

static bool table_ok(const mk_table *t) { return t && t->d_table && t->k >= 3 && t->k <= 6; }

extern "C" int mk_table_build(mk_ctx *ctx, int k, mk_table **out)
{
    if (!ctx || !out) return fail(MK_EINVAL, "mk_table_build: NULL argument");
    if (k < 3 || k > 6) return fail(MK_ERANGE, "mk_table_build: k=%d outside 3..6", k);
    std::lock_guard<std::recursive_mutex> lock(ctx->mu);
    if (ctx->tables[k]) {
        *out = static_cast<mk_table *>(ctx->tables[k]);
        return MK_OK;
    }
    MK_HIP(hipSetDevice(ctx->device));
    mk_table *t = new mk_table();
    t->ctx = ctx;
    t->k = k;
    int rc = build_table(t, ctx->stream);
    if (rc != MK_OK) {
        if (t->d_table) (void)hipFree(t->d_table);
        if (t->d_classes) (void)hipFree(t->d_classes);
        if (t->d_core_mult) (void)hipFree(t->d_core_mult);
        delete t;
        return rc;
    }
    ctx->tables[k] = t;
    *out = t;
    return MK_OK;
}

namespace mk {
void free_table(Table *t)
{
    if (!t) return;
    if (t->d_table) (void)hipFree(t->d_table);
    if (t->d_classes) (void)hipFree(t->d_classes);
    if (t->d_core_mult) (void)hipFree(t->d_core_mult);
    delete static_cast<mk_table *>(t);
}
}  // namespace mk

extern "C" int mk_table_release(mk_ctx *ctx, int k)
{
    if (!ctx) return fail(MK_EINVAL, "mk_table_release: NULL context");
    if (k < 3 || k > 6) return fail(MK_ERANGE, "mk_table_release: k=%d outside 3..6", k);
    std::lock_guard<std::recursive_mutex> lock(ctx->mu);
    MK_HIP(hipSetDevice(ctx->device));
    MK_HIP(hipStreamSynchronize(ctx->stream));
    free_table(ctx->tables[k]);
    ctx->tables[k] = nullptr;
    return MK_OK;
}

extern "C" int mk_table_info(const mk_table *t, int32_t *k, uint32_t *num_classes,
                             uint64_t *num_entries, double *build_ms)
{
    if (!table_ok(t)) return fail(MK_EINVAL, "mk_table_info: bad table");
    if (k) *k = t->k;
    if (num_classes) *num_classes = t->num_classes;
    if (num_entries) *num_entries = t->entries;
    if (build_ms) *build_ms = t->build_ms;
    return MK_OK;
}

extern "C" int mk_table_class_code(const mk_table *t, uint32_t id, uint32_t *canon_code)
{
    if (!table_ok(t) || !canon_code) return fail(MK_EINVAL, "mk_table_class_code: bad argument");
    if (id >= t->num_classes)
        return fail(MK_ERANGE, "class id %u >= %u classes", id, t->num_classes);
    *canon_code = t->classes[id];
    return MK_OK;
}

extern "C" int mk_table_class_codes(const mk_table *t, uint32_t *codes, uint32_t capacity)
{
    if (!table_ok(t) || !codes) return fail(MK_EINVAL, "mk_table_class_codes: bad argument");
    if (capacity < t->num_classes)
        return fail(MK_ERANGE, "capacity %u < %u classes", capacity, t->num_classes);
    std::copy(t->classes.begin(), t->classes.end(), codes);
    return MK_OK;
}

extern "C" int mk_table_read(const mk_table *t, uint64_t first, uint64_t count, uint32_t *out)
{
    if (!table_ok(t) || (!out && count)) return fail(MK_EINVAL, "mk_table_read: bad argument");
    if (first > t->entries || count > t->entries - first)
        return fail(MK_ERANGE, "entries [%llu, +%llu) outside the table",
                    (unsigned long long)first, (unsigned long long)count);
    if (count == 0) return MK_OK;
    std::lock_guard<std::recursive_mutex> lock(t->ctx->mu);
    MK_HIP(hipSetDevice(t->ctx->device));
    MK_HIP(hipMemcpyAsync(out, t->d_table + first, count * sizeof(uint32_t),
                          hipMemcpyDeviceToHost, t->ctx->stream));
    MK_HIP(hipStreamSynchronize(t->ctx->stream));
    return MK_OK;
}

extern "C" int mk_table_lookup(const mk_table *t, uint32_t code, uint32_t *id)
{
    if (!table_ok(t) || !id) return fail(MK_EINVAL, "mk_table_lookup: bad argument");
    if (code >= t->entries) return fail(MK_ERANGE, "code %u >= 2^(k(k-1))", code);
    return mk_table_read(t, code, 1, id);
}

extern "C" int mk_table_core_mult(const mk_table *t, uint32_t first, uint32_t count, uint8_t *out)
{
    if (!table_ok(t) || (!out && count)) return fail(MK_EINVAL, "mk_table_core_mult: bad argument");
    if (first > t->num_classes || count > t->num_classes - first)
        return fail(MK_ERANGE, "classes [%u, +%u) outside the %u classes", first, count,
                    t->num_classes);
    if (count == 0) return MK_OK;
    std::lock_guard<std::recursive_mutex> lock(t->ctx->mu);
    MK_HIP(hipSetDevice(t->ctx->device));
    MK_HIP(hipMemcpyAsync(out, t->d_core_mult + first, count, hipMemcpyDeviceToHost,
                          t->ctx->stream));
    MK_HIP(hipStreamSynchronize(t->ctx->stream));
    return MK_OK;
}
