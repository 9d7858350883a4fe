// Error reporting, allocation and a device-wide prefix sum.
#include <cstdarg>
#include <cstdio>
#include <cstdlib>

#include "fea_internal.h"

namespace fea {

static thread_local std::string g_error;

int set_error(int code, const char *fmt, ...)
{
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_error = buf;
    return code;
}

void clear_error() { g_error.clear(); }

// Allocation-failure injection for tests of the error path: when the
// environment variable FEA_FAIL_ALLOC_AT=n is set, the n-th device
// allocation of the process (1-based) fails.
static long g_alloc_count = 0;

int dalloc(void **p, size_t bytes)
{
    *p = nullptr;
    static const char *fail_at = getenv("FEA_FAIL_ALLOC_AT");
    ++g_alloc_count;
    if (fail_at && atol(fail_at) == g_alloc_count)
        return set_error(FEA_ENOMEM, "device allocation of %zu bytes failed (injected)", bytes);
    if (bytes == 0) bytes = 8;
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return set_error(FEA_ENOMEM, "device allocation of %zu bytes failed: %s", bytes,
                         hipGetErrorString(e));
    }
    return FEA_OK;
}

void dfree(void *p)
{
    if (p) (void)hipFree(p);
}

// ------------------------------------------------------------------ scan
// Three passes: per-tile sums, a single-workgroup scan of the tile sums,
// then per-tile rescans with the tile offset. 256 threads x 8 items.
constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;

int64_t scan_tmp_elems(int64_t n) { return (n + kScanTile - 1) / kScanTile + 1; }

__device__ inline int64_t block_exclusive_scan(int64_t v, int64_t *total)
{
    __shared__ int64_t s[kScanThreads];
    int t = threadIdx.x;
    s[t] = v;
    __syncthreads();
    for (int off = 1; off < kScanThreads; off <<= 1) {
        int64_t add = (t >= off) ? s[t - off] : 0;
        __syncthreads();
        s[t] += add;
        __syncthreads();
    }
    int64_t incl = s[t];
    *total = s[kScanThreads - 1];
    __syncthreads();
    return incl - v;
}

template <typename T>
__global__ void __launch_bounds__(kScanThreads) k_scan_partials(const T *in, int64_t n, int64_t *part)
{
    int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int64_t sum = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i)
        if (base + i < n) sum += (int64_t)in[base + i];
    int64_t total;
    block_exclusive_scan(sum, &total);
    if (threadIdx.x == 0) part[blockIdx.x] = total;
}

__global__ void __launch_bounds__(kScanThreads) k_scan_tiles(int64_t *part, int64_t ntiles)
{
    int64_t carry = 0;
    for (int64_t b = 0; b < ntiles; b += kScanThreads) {
        int64_t i = b + threadIdx.x;
        int64_t v = (i < ntiles) ? part[i] : 0;
        int64_t total;
        int64_t ex = block_exclusive_scan(v, &total);
        if (i < ntiles) part[i] = carry + ex;
        carry += total;
        __syncthreads();
    }
}

template <typename T>
__global__ void __launch_bounds__(kScanThreads) k_scan_final(const T *in, int64_t n, const int64_t *part,
                                                            int64_t *ptr)
{
    int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int64_t v[kScanItems];
    int64_t sum = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        v[i] = (base + i < n) ? (int64_t)in[base + i] : 0;
        sum += v[i];
    }
    int64_t total;
    int64_t run = block_exclusive_scan(sum, &total) + part[blockIdx.x];
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        run += v[i];
        if (base + i < n) ptr[base + i + 1] = run;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) ptr[0] = 0;
}

template <typename T>
static int scan_impl(const T *in, int64_t n, int64_t *ptr, int64_t *tmp, hipStream_t s)
{
    if (n <= 0) {
        FEA_HIP(hipMemsetAsync(ptr, 0, sizeof(int64_t), s));
        return FEA_OK;
    }
    int64_t ntiles = (n + kScanTile - 1) / kScanTile;
    k_scan_partials<T><<<(unsigned)ntiles, kScanThreads, 0, s>>>(in, n, tmp);
    k_scan_tiles<<<1, kScanThreads, 0, s>>>(tmp, ntiles);
    k_scan_final<T><<<(unsigned)ntiles, kScanThreads, 0, s>>>(in, n, tmp, ptr);
    FEA_HIP(hipGetLastError());
    return FEA_OK;
}

int scan_to_ptr_u8(const uint8_t *in, int64_t n, int64_t *ptr, int64_t *tmp, hipStream_t s)
{
    return scan_impl(in, n, ptr, tmp, s);
}
int scan_to_ptr_i32(const int32_t *in, int64_t n, int64_t *ptr, int64_t *tmp, hipStream_t s)
{
    return scan_impl(in, n, ptr, tmp, s);
}
int scan_to_ptr_i64(const int64_t *in, int64_t n, int64_t *ptr, int64_t *tmp, hipStream_t s)
{
    return scan_impl(in, n, ptr, tmp, s);
}

}  // namespace fea

extern "C" const char *fea_last_error(void) { return fea::g_error.c_str(); }

extern "C" const char *fea_version(void) { return "fea-gfx950 0.1"; }
