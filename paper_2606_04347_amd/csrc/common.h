// Shared device/host definitions of the ETD library (gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace etd {

template <typename T> struct V2;
template <> struct V2<float> { using t = float2; };
template <> struct V2<double> { using t = double2; };
template <typename T> using c2 = typename V2<T>::t;

template <typename T> __host__ __device__ __forceinline__ c2<T> mk(T x, T y) {
    c2<T> r;
    r.x = x;
    r.y = y;
    return r;
}
// complex helpers on float2 / double2 (V deduced directly)
template <typename V> __device__ __forceinline__ V cadd(V a, V b) {
    V r;
    r.x = a.x + b.x;
    r.y = a.y + b.y;
    return r;
}
template <typename V> __device__ __forceinline__ V csub(V a, V b) {
    V r;
    r.x = a.x - b.x;
    r.y = a.y - b.y;
    return r;
}
template <typename V> __device__ __forceinline__ V cmul(V a, V b) {
    V r;
    r.x = a.x * b.x - a.y * b.y;
    r.y = a.x * b.y + a.y * b.x;
    return r;
}
template <typename V, typename S> __device__ __forceinline__ V cscale(V a, S s) {
    V r;
    r.x = a.x * s;
    r.y = a.y * s;
    return r;
}
template <typename V> __device__ __forceinline__ V cconj(V a) {
    V r;
    r.x = a.x;
    r.y = -a.y;
    return r;
}

// Grid description used by every kernel.  A 2D grid is stored as nx = 1.
struct GridK {
    int nx, ny, nz;      // real extents (C order, z contiguous)
    int nzh;             // nz / 2 + 1 (half spectrum along z)
    double h[3];         // mesh widths (h[0] unused when nx == 1)
    double X[3];         // half lengths
    double cell;         // product of the active mesh widths
    int dim;
    __host__ __device__ long nreal() const { return (long)nx * ny * nz; }
    __host__ __device__ long nspec() const { return (long)nx * ny * nzh; }
};

// Integer wavenumber helpers (Section 3.2).  lam: Laplacian index
// (i for i <= N/2, N - i above); der: first-derivative index (i below N/2,
// 0 at the Nyquist bin, i - N above).
__host__ __device__ __forceinline__ int lam_index(int i, int N) { return i <= N / 2 ? i : N - i; }
__host__ __device__ __forceinline__ int der_index(int i, int N) {
    return i < N / 2 ? i : (i == N / 2 ? 0 : i - N);
}

constexpr double kPi = 3.14159265358979323846264338327950288;

// Round-robin dispatch puts block b on XCD b % 8 (eight XCDs, each with its
// own L2); renumber so that each XCD works on one contiguous range of tiles
// (neighbouring tiles then share L2 lines).
__device__ __forceinline__ int xcd_remap(int b, int nb) {
    const int q = nb >> 3, r = nb & 7, x = b & 7, k = b >> 3;
    return x * q + min(x, r) + k;
}

}  // namespace etd
