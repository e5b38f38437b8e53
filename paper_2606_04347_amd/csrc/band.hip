// Narrow band of Section 3.2: flag |2 phi - 1| < threshold in FP64, then a
// stable compaction to ascending C-order int32 indices: per-tile counts, an
// exclusive scan of the tile counts, and a per-tile scan + scatter.  Each tile
// is 4096 consecutive points (256 threads x 16 contiguous points), so the
// output order is the index order without any sort.
#include <map>
#include <mutex>

#include "kernels.h"

namespace etd {

namespace {

constexpr int kB = 256;
constexpr int kItems = 16;
constexpr long kTile = (long)kB * kItems;

// Flag sources of the compaction: flags already formed (uint8), or the band
// condition |2 phi - 1| < thr decided in FP64 where it is read.
struct FlagsIn {
    const uint8_t* f;
    __device__ __forceinline__ int operator()(long i) const { return f[i]; }
};
template <typename T> struct PhiFlag {
    const T* phi;
    double thr;
    __device__ __forceinline__ int operator()(long i) const { return fabs(2.0 * (double)phi[i] - 1.0) < thr ? 1 : 0; }
};

constexpr long kStaticTiles = 65536;   // allocation-free build: grids up to 65536 * 4096 = 268,435,456 points

template <typename T> __global__ __launch_bounds__(kB) void k_flags(long n, const T* __restrict__ phi, double thr, uint8_t* __restrict__ f) {
    for (long i = (long)blockIdx.x * kB + threadIdx.x; i < n; i += (long)gridDim.x * kB)
        f[i] = fabs(2.0 * (double)phi[i] - 1.0) < thr ? 1 : 0;
}

__device__ __forceinline__ int block_excl_scan(int v, int* sh, int* total) {
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < kB; off <<= 1) {
        const int t = ((int)threadIdx.x >= off) ? sh[threadIdx.x - off] : 0;
        __syncthreads();
        sh[threadIdx.x] += t;
        __syncthreads();
    }
    const int incl = sh[threadIdx.x];
    *total = sh[kB - 1];
    __syncthreads();
    return incl - v;
}

template <class F> __global__ __launch_bounds__(kB) void k_tile_counts(long n, F f, int64_t* cnt) {
    __shared__ int sh[kB];
    const long base = (long)blockIdx.x * kTile + (long)threadIdx.x * kItems;
    int c = 0;
    for (int k = 0; k < kItems; ++k) {
        const long i = base + k;
        if (i < n) c += f(i);
    }
    int total;
    (void)block_excl_scan(c, sh, &total);
    if (threadIdx.x == 0) cnt[blockIdx.x] = total;
}

// exclusive scan of nt tile counts in one workgroup; cnt[nt] receives the total
__global__ __launch_bounds__(kB) void k_scan_tiles(int64_t* cnt, long nt, int64_t* total_dev) {
    __shared__ int64_t sh[kB];
    __shared__ int64_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (long b0 = 0; b0 < nt; b0 += kB) {
        const long i = b0 + threadIdx.x;
        const int64_t v = (i < nt) ? cnt[i] : 0;
        sh[threadIdx.x] = v;
        __syncthreads();
        for (int off = 1; off < kB; off <<= 1) {
            const int64_t t = ((int)threadIdx.x >= off) ? sh[threadIdx.x - off] : 0;
            __syncthreads();
            sh[threadIdx.x] += t;
            __syncthreads();
        }
        if (i < nt) cnt[i] = carry + sh[threadIdx.x] - v;
        __syncthreads();
        if (threadIdx.x == 0) carry += sh[kB - 1];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        cnt[nt] = carry;
        total_dev[0] = carry;
    }
}

template <class F>
__global__ __launch_bounds__(kB) void k_scatter(long n, F f, const int64_t* __restrict__ off, int32_t* out,
                                                int64_t capacity) {
    __shared__ int sh[kB];
    if (off[gridDim.x] > capacity) return;     // the whole band must fit, else nothing is written
    const long base = (long)blockIdx.x * kTile + (long)threadIdx.x * kItems;
    int c = 0;
    for (int k = 0; k < kItems; ++k) {
        const long i = base + k;
        if (i < n) c += f(i);
    }
    int total;
    int pos = block_excl_scan(c, sh, &total);
    int64_t o = off[blockIdx.x] + pos;
    for (int k = 0; k < kItems; ++k) {
        const long i = base + k;
        if (i < n && f(i)) out[o++] = (int32_t)i;
    }
}

}  // namespace

template <typename T> void band_flags(long n, const T* phi, double thr, uint8_t* flags, hipStream_t s) {
    long b = (n + kB - 1) / kB;
    if (b > 8192) b = 8192;
    hipLaunchKernelGGL(k_flags<T>, dim3((int)b), dim3(kB), 0, s, n, phi, thr, flags);
}
template void band_flags<float>(long, const float*, double, uint8_t*, hipStream_t);
template void band_flags<double>(long, const double*, double, uint8_t*, hipStream_t);

long band_blocks(long n) { return (n + kTile - 1) / kTile; }

// Scratch of the allocation-free band build (tile offsets and the total),
// 512 KiB per device, held until the process ends.  Host code reaches each
// device's copy only through the address band_static_init looks up.
static __device__ __align__(256) int64_t scratch[kStaticTiles + 2];

namespace {
template <class F>
void compact_with(long n, const F& f, int64_t* blockcnt, int32_t* idx_out, int64_t capacity, int64_t* total_dev,
                  hipStream_t s) {
    const long nt = band_blocks(n);
    if (nt > 0) hipLaunchKernelGGL(k_tile_counts<F>, dim3((int)nt), dim3(kB), 0, s, n, f, blockcnt);
    hipLaunchKernelGGL(k_scan_tiles, dim3(1), dim3(kB), 0, s, blockcnt, nt, total_dev);
    if (idx_out && nt > 0)
        hipLaunchKernelGGL(k_scatter<F>, dim3((int)nt), dim3(kB), 0, s, n, f, blockcnt, idx_out, capacity);
}
}  // namespace

void band_compact(long n, const uint8_t* flags, int64_t* blockcnt, int32_t* idx_out, int64_t capacity,
                  int64_t* total_dev, hipStream_t s) {
    compact_with(n, FlagsIn{flags}, blockcnt, idx_out, capacity, total_dev, s);
}

// ------------------------------------------------------------------ allocation-free band build
namespace {
std::mutex g_scratch_mu;
std::map<int, int64_t*> g_scratch;   // device -> address of that device's copy of scratch
}  // namespace

long band_static_max_points() { return kStaticTiles * kTile; }

hipError_t band_static_init(int device) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch.count(device)) return hipSuccess;
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return e;
    int64_t* ptr = nullptr;
    e = hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch));
    if (cur != device) (void)hipSetDevice(cur);
    if (e != hipSuccess) return e;
    if (!ptr) return hipErrorInvalidSymbol;
    g_scratch[device] = ptr;
    return hipSuccess;
}

template <typename T>
hipError_t band_build_static(int device, long n, const T* phi, double thr, int32_t* idx_out, int64_t capacity,
                             int64_t* count_host, hipStream_t s) {
    int64_t* sc = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        auto it = g_scratch.find(device);
        if (it == g_scratch.end()) return hipErrorNotInitialized;
        sc = it->second;
    }
    if (n < 0 || n > band_static_max_points()) return hipErrorInvalidValue;
    // tile offsets in sc[0 .. nt], the total in sc[nt + 1]; every entry read
    // is written first by the same call, so nothing needs clearing
    const long nt = band_blocks(n);
    compact_with(n, PhiFlag<T>{phi, thr}, sc, capacity > 0 ? idx_out : nullptr, capacity, sc + nt + 1, s);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(count_host, sc + nt + 1, sizeof(int64_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    return e;
}
template hipError_t band_build_static<float>(int, long, const float*, double, int32_t*, int64_t, int64_t*,
                                             hipStream_t);
template hipError_t band_build_static<double>(int, long, const double*, double, int32_t*, int64_t, int64_t*,
                                              hipStream_t);

}  // namespace etd
