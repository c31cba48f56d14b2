// Error strings, fill and prefix-sum kernels shared by the rest of the
// library.
#include <cstdio>

#include "internal.h"

namespace mk {

static thread_local std::string g_last_error;

int fail(int status, const char *fmt, ...)
{
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return status;
}

// ------------------------------------------------------------------ fill

__global__ void fill_kernel(uint32_t *dst, uint32_t value, size_t n)
{
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) dst[i] = value;
}

// 16-byte non-temporal (streaming) vector stores for a 16-byte aligned dst;
// the last n % 4 words by the first threads.  Clearing a 380 MB histogram
// this way with up to 65,536 workgroups takes 20 us less on MI355X than
// cached stores from 8,192.
typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));
__global__ void fill4_kernel(uint32_t *dst, uint32_t value, size_t n)
{
    const size_t n4 = n >> 2;
    u32x4_t *d4 = reinterpret_cast<u32x4_t *>(dst);
    const u32x4_t v = {value, value, value, value};
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = t; i < n4; i += stride) __builtin_nontemporal_store(v, d4 + i);
    if (t < (n & 3)) dst[(n4 << 2) + t] = value;
}

int fill_u32(void *dst, uint32_t value, size_t n, hipStream_t stream)
{
    if (n == 0) return MK_OK;
    if (((uintptr_t)dst & 15) == 0 && n >= 4096) {
        size_t blocks = (n / 4 + 255) / 256;
        if (blocks > 65536) blocks = 65536;
        hipLaunchKernelGGL(fill4_kernel, dim3((unsigned)blocks), dim3(256), 0, stream,
                           (uint32_t *)dst, value, n);
    } else {
        size_t blocks = (n + 255) / 256;
        if (blocks > 16384) blocks = 16384;
        hipLaunchKernelGGL(fill_kernel, dim3((unsigned)blocks), dim3(256), 0, stream,
                           (uint32_t *)dst, value, n);
    }
    MK_HIP(hipGetLastError());
    return MK_OK;
}

// ------------------------------------------------------------------ scan
//
// Three passes: per-block sums, a single-block scan of those sums, and a
// rescan that adds each block's offset.  A block covers kScanItems items
// per thread x kScanThreads threads.

constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanTile = kScanThreads * kScanItems;

__device__ __forceinline__ uint32_t load_item(const uint32_t *in, size_t i, size_t n, int popcount)
{
    if (i >= n) return 0;
    uint32_t v = in[i];
    return popcount ? (uint32_t)__popc(v) : v;
}

// exclusive scan of one value per thread over the block; returns the
// block total in *total
__device__ uint32_t block_exclusive(uint32_t v, uint32_t *total)
{
    __shared__ uint32_t wave_sums[kScanThreads / kWave];
    const int lane = threadIdx.x % kWave;
    const int wave = threadIdx.x / kWave;
    uint32_t incl = v;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        uint32_t o = __shfl_up(incl, d, kWave);
        if (lane >= d) incl += o;
    }
    if (lane == kWave - 1) wave_sums[wave] = incl;
    __syncthreads();
    uint32_t before = 0, all = 0;
#pragma unroll
    for (int w = 0; w < kScanThreads / kWave; ++w) {
        uint32_t s = wave_sums[w];
        if (w < wave) before += s;
        all += s;
    }
    __syncthreads();
    *total = all;
    return before + incl - v;
}

__global__ __launch_bounds__(kScanThreads) void scan_block_sums(const uint32_t *in, size_t n,
                                                                int popcount, uint32_t *sums)
{
    size_t base = (size_t)blockIdx.x * kScanTile + (size_t)threadIdx.x * kScanItems;
    uint32_t s = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) s += load_item(in, base + j, n, popcount);
    uint32_t total;
    block_exclusive(s, &total);
    if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

__global__ __launch_bounds__(kScanThreads) void scan_sums(uint32_t *sums, size_t nb,
                                                          uint32_t *d_total)
{
    uint32_t carry = 0;
    for (size_t base = 0; base < nb; base += kScanThreads) {
        size_t i = base + threadIdx.x;
        uint32_t v = i < nb ? sums[i] : 0;
        uint32_t total;
        uint32_t ex = block_exclusive(v, &total);
        if (i < nb) sums[i] = carry + ex;
        carry += total;
    }
    if (threadIdx.x == 0 && d_total) *d_total = carry;
}

__global__ __launch_bounds__(kScanThreads) void scan_apply(const uint32_t *in, uint32_t *out,
                                                           size_t n, int popcount,
                                                           const uint32_t *sums)
{
    size_t base = (size_t)blockIdx.x * kScanTile + (size_t)threadIdx.x * kScanItems;
    uint32_t vals[kScanItems];
    uint32_t s = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        vals[j] = load_item(in, base + j, n, popcount);
        s += vals[j];
    }
    uint32_t total;
    uint32_t run = block_exclusive(s, &total) + sums[blockIdx.x];
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        if (base + j < n) out[base + j] = run;
        run += vals[j];
    }
}

size_t scan_tmp_words(size_t n) { return (n + kScanTile - 1) / kScanTile + 1; }

int scan_u32(const uint32_t *in, uint32_t *out, size_t n, int popcount, uint32_t *d_total,
             uint32_t *tmp, hipStream_t stream)
{
    size_t nb = (n + kScanTile - 1) / kScanTile;
    if (nb == 0) {
        if (d_total) return fill_u32(d_total, 0, 1, stream);
        return MK_OK;
    }
    if (nb > 0x7FFFFFFFull) return fail(MK_ERANGE, "scan too large (%zu items)", n);
    hipLaunchKernelGGL(scan_block_sums, dim3((unsigned)nb), dim3(kScanThreads), 0, stream, in, n,
                       popcount, tmp);
    MK_HIP(hipGetLastError());
    hipLaunchKernelGGL(scan_sums, dim3(1), dim3(kScanThreads), 0, stream, tmp, nb, d_total);
    MK_HIP(hipGetLastError());
    hipLaunchKernelGGL(scan_apply, dim3((unsigned)nb), dim3(kScanThreads), 0, stream, in, out, n,
                       popcount, tmp);
    MK_HIP(hipGetLastError());
    return MK_OK;
}

}  // namespace mk

extern "C" const char *mk_last_error(void) { return mk::g_last_error.c_str(); }

extern "C" const char *mk_status_str(int status)
{
    switch (status) {
    case MK_OK: return "ok";
    case MK_EINVAL: return "invalid argument";
    case MK_ERANGE: return "out of range";
    case MK_EGRAPH: return "not a simple digraph CSR";
    case MK_ENOMEM: return "out of memory";
    case MK_EDEVICE: return "device error";
    case MK_EBUSY: return "busy";
    case MK_ETIMEDOUT: return "timed out";
    case MK_ENOTFOUND: return "not found";
    default: return "unknown status";
    }
}
