// Batched 1D FFT passes (Stockham engine in stockham.h) and the 3D real
// transforms built from them.
//
// Passes over a 3D array (real [nx][ny][nz] <-> half spectrum [nx][ny][nzh]):
//   z  : contiguous rows; r2c packs x_{2n} + i x_{2n+1} into a length-nz/2
//        complex transform and splits it with w_nz^k; c2r inverts that.
//   y,x: strided lines.  A workgroup takes L consecutive kz columns of one
//        line family so that every global access is a run of L contiguous
//        complex values (L = 16: 128 B in FP32, 256 B in FP64).
#include "fft.h"

#include <cmath>

#include "launch.h"
#include "zrows.h"

namespace etd {

using namespace stk;

namespace {

// ---------------------------------------------------------------- strided lines
template <typename T, int N> constexpr int strided_lines() { return lines_per_block<T, N, 1>(); }

// Plain transform of lines: element e of line l at sbase[l] + e * estride
// (sbase[l] < 0: the line is past the end).  In place is safe: every read of a
// tile happens in the first stage, every write in the last, with barriers in
// between, and tiles are disjoint.
template <typename T> struct PlainLinesOp {
    static constexpr int NS = 1;
    const c2<T>* in;
    c2<T>* out;
    const long* sbase;
    long estride;
    __device__ __forceinline__ void load(int l, int e, c2<T>* v) const {
        const long b = sbase[l];
        v[0] = b >= 0 ? in[b + (long)e * estride] : mk<T>(0, 0);
    }
    __device__ __forceinline__ void store(int l, int, int e, c2<T> v) const {
        const long b = sbase[l];
        if (b >= 0) out[b + (long)e * estride] = v;
    }
};

// Lines are numbered j = o * C + c (o the outer index, c the contiguous column
// index, C columns); line j starts at o * ostride + c and its elements are
// estride apart.  A workgroup takes L consecutive line numbers, so no tile is
// ragged and (for the x pass, where o * ostride + c == j) every tile row is one
// aligned run of L complex values.
template <typename T, int N, int DIR>
__device__ __forceinline__ void fft_lines(const c2<T>* in, c2<T>* out, const c2<T>* __restrict__ tw, int C,
                                          int nlines, long ostride, long estride) {
    constexpr int L = strided_lines<T, N>();
    constexpr int LS = line_stride<N>();
    extern __shared__ unsigned char smem_raw[];
    __shared__ long sbase[L];
    c2<T>* lds = reinterpret_cast<c2<T>*>(smem_raw);
    c2<T>* stw = lds + L * LS;
    load_table<T>(stw, tw, N);
    const int tile = xcd_remap(blockIdx.x, gridDim.x);
    if (threadIdx.x < L) {
        const int j = tile * L + threadIdx.x;
        sbase[threadIdx.x] = j < nlines ? (long)(j / C) * ostride + (j % C) : -1;
    }
    __syncthreads();
    lines_fft<T, N, L, DIR, true>(lds, stw, PlainLinesOp<T>{in, out, sbase, estride});
}

// The y- and x-line passes share the body; separate symbols keep them apart in traces.
template <typename T, int N, int DIR>
struct k_fft_ylines_body {
    static __device__ __forceinline__ void run(const c2<T>* in, c2<T>* out, const c2<T>* __restrict__ tw,
                                                         int C, int nlines, long ostride, long estride) {
        fft_lines<T, N, DIR>(in, out, tw, C, nlines, ostride, estride);
    }
};
template <typename T, int N, int DIR>
__global__ __launch_bounds__(kThreads) void k_fft_ylines(const c2<T>* in, c2<T>* out, const c2<T>* __restrict__ tw,
                                                         int C, int nlines, long ostride, long estride) {
    k_fft_ylines_body<T, N, DIR>::run(in, out, tw, C, nlines, ostride, estride);
}
template <typename T, int N, int DIR>
struct k_fft_xlines_body {
    static __device__ __forceinline__ void run(const c2<T>* in, c2<T>* out, const c2<T>* __restrict__ tw,
                                                         int C, int nlines, long ostride, long estride) {
        fft_lines<T, N, DIR>(in, out, tw, C, nlines, ostride, estride);
    }
};
template <typename T, int N, int DIR>
__global__ __launch_bounds__(kThreads) void k_fft_xlines(const c2<T>* in, c2<T>* out, const c2<T>* __restrict__ tw,
                                                         int C, int nlines, long ostride, long estride) {
    k_fft_xlines_body<T, N, DIR>::run(in, out, tw, C, nlines, ostride, estride);
}

// ---------------------------------------------------------------- z rows (r2c / c2r)
template <typename T, int NR>
struct k_fft_z_r2c_body {
    static __device__ __forceinline__ void run(const T* __restrict__ in, c2<T>* __restrict__ out,
                                                        const c2<T>* __restrict__ twh,
                                                        const c2<T>* __restrict__ twf, long nrows) {
        constexpr int L = z_rows<T, NR>();
        extern __shared__ unsigned char smem_raw[];
        c2<T>* lds = reinterpret_cast<c2<T>*>(smem_raw);
        c2<T>* stw = lds + L * z_row_stride<NR>();
        load_table<T>(stw, twh, NR / 2);
        const long row0 = (long)blockIdx.x * L;
        const int nl = (int)min((long)L, nrows - row0);
        zrow_forward<T, NR>(lds, stw, twf, in + row0 * NR, out + row0 * (NR / 2 + 1), nl);
    }
};
template <typename T, int NR>
__global__ __launch_bounds__(kThreads) void k_fft_z_r2c(const T* __restrict__ in, c2<T>* __restrict__ out,
                                                        const c2<T>* __restrict__ twh,
                                                        const c2<T>* __restrict__ twf, long nrows) {
    k_fft_z_r2c_body<T, NR>::run(in, out, twh, twf, nrows);
}

template <typename T, int NR>
struct k_fft_z_c2r_body {
    static __device__ __forceinline__ void run(const c2<T>* __restrict__ in, T* __restrict__ out,
                                                        const c2<T>* __restrict__ twh,
                                                        const c2<T>* __restrict__ twf, long nrows,
                                                        T scale) {
        constexpr int L = z_rows<T, NR>();
        extern __shared__ unsigned char smem_raw[];
        c2<T>* lds = reinterpret_cast<c2<T>*>(smem_raw);
        c2<T>* stw = lds + L * z_row_stride<NR>();
        load_table<T>(stw, twh, NR / 2);
        const long row0 = (long)blockIdx.x * L;
        const int nl = (int)min((long)L, nrows - row0);
        zrow_inverse<T, NR, false>(lds, stw, twf, in + row0 * (NR / 2 + 1), out + row0 * NR, nl, scale, 0.0);
    }
};
template <typename T, int NR>
__global__ __launch_bounds__(kThreads) void k_fft_z_c2r(const c2<T>* __restrict__ in, T* __restrict__ out,
                                                        const c2<T>* __restrict__ twh,
                                                        const c2<T>* __restrict__ twf, long nrows,
                                                        T scale) {
    k_fft_z_c2r_body<T, NR>::run(in, out, twh, twf, nrows, scale);
}

// ---------------------------------------------------------------- launch helpers
template <typename T, int N, int DIR, bool XLINES>
hipError_t launch_strided(const c2<T>* in, c2<T>* out, const c2<T>* tw, int C, int nouter, long ostride,
                          long estride, hipStream_t s) {
    constexpr int L = strided_lines<T, N>();
    const size_t smem = lines_smem<T, N, L, 1>();
    static_assert(lines_smem<T, N, L, 1>() <= kLdsBytes, "LDS tile larger than a workgroup can hold");
    const long nlines = (long)C * nouter;
    const int ntiles = (int)((nlines + L - 1) / L);
    if constexpr (XLINES) {
        static std::once_flag flag;
        set_smem_limit(k_fft_xlines<T, N, DIR>, smem, flag);
        launch_k<k_fft_xlines_body<T, N, DIR>>(k_fft_xlines<T, N, DIR>, dim3(ntiles), dim3(kThreads), smem, s, in,
                                               out, tw, C, (int)nlines, ostride, estride);
    } else {
        static std::once_flag flag;
        set_smem_limit(k_fft_ylines<T, N, DIR>, smem, flag);
        launch_k<k_fft_ylines_body<T, N, DIR>>(k_fft_ylines<T, N, DIR>, dim3(ntiles), dim3(kThreads), smem, s, in,
                                               out, tw, C, (int)nlines, ostride, estride);
    }
    return hipGetLastError();
}

template <typename T, int NR>
hipError_t launch_z(bool forward, const void* in, void* out, const c2<T>* twh, const c2<T>* twf, long nrows,
                    T scale, hipStream_t s) {
    constexpr int L = z_rows<T, NR>();
    const size_t smem = z_smem<T, NR>();
    static_assert(z_smem<T, NR>() <= kLdsBytes, "LDS tile larger than a workgroup can hold");
    const int nblk = (int)((nrows + L - 1) / L);
    if (forward) {
        auto kern = k_fft_z_r2c<T, NR>;
        static std::once_flag flag_f;
        set_smem_limit(kern, smem, flag_f);
        launch_k<k_fft_z_r2c_body<T, NR>>(kern, dim3(nblk), dim3(kThreads), smem, s, (const T*)in, (c2<T>*)out,
                                          twh, twf, nrows);
    } else {
        auto kern = k_fft_z_c2r<T, NR>;
        static std::once_flag flag_i;
        set_smem_limit(kern, smem, flag_i);
        launch_k<k_fft_z_c2r_body<T, NR>>(kern, dim3(nblk), dim3(kThreads), smem, s, (const c2<T>*)in, (T*)out,
                                          twh, twf, nrows, scale);
    }
    return hipGetLastError();
}


template <typename T, int DIR, bool XLINES>
hipError_t dispatch_strided(int N, const c2<T>* in, c2<T>* out, const c2<T>* tw, int C, int nouter,
                            long ostride, long estride, hipStream_t s) {
    switch (N) {
#define CASE(n) \
    case n: return launch_strided<T, n, DIR, XLINES>(in, out, tw, C, nouter, ostride, estride, s);
        ETD_FFT_SIZES(CASE)
#undef CASE
        default: return hipErrorInvalidValue;
    }
}

template <typename T>
hipError_t dispatch_z(int NR, bool forward, const void* in, void* out, const c2<T>* twh, const c2<T>* twf,
                      long nrows, T scale, hipStream_t s) {
    switch (NR) {
#define CASE(n) \
    case n: return launch_z<T, n>(forward, in, out, twh, twf, nrows, scale, s);
        ETD_FFT_SIZES(CASE)
#undef CASE
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

bool fft_length_supported(int n) {
    switch (n) {
#define CASE(v) case v:
        ETD_FFT_SIZES(CASE)
#undef CASE
        return true;
        default: return false;
    }
}

void fft_twiddles_host(int n, double* re_im) {
    // exp(-2 pi i k / n) from the exact integer k, evaluated in long double and
    // rounded once; the quarter points are set exactly.
    const long double twopi = 6.283185307179586476925286766559005768L;
    for (int k = 0; k < n; ++k) {
        const long double a = twopi * (long double)k / (long double)n;
        re_im[2 * k] = (double)cosl(a);
        re_im[2 * k + 1] = (double)(-sinl(a));
    }
    // exact values at the quarter points
    for (int k = 0; k < n; ++k) {
        if ((4L * k) % n == 0) {
            const int q = (int)((4L * k) / n);
            const double c[4] = {1, 0, -1, 0}, sn[4] = {0, -1, 0, 1};
            re_im[2 * k] = c[q];
            re_im[2 * k + 1] = sn[q];
        }
    }
}

PassHook* g_pass_hook = nullptr;

void fft_set_pass_hook(PassHook* h) { g_pass_hook = h; }

template <typename T>
hipError_t fft_pass_z(const GridK& g, const FFTTables<T>& t, bool forward, const void* in, void* out, T scale,
                      hipStream_t s) {
    const double bytes = 2.0 * sizeof(T) * (double)g.nspec() + sizeof(T) * (double)g.nreal();
    return timed_pass(forward ? PASS_Z_R2C : PASS_Z_C2R, bytes, s, [&] {
        return dispatch_z<T>(g.nz, forward, in, out, t.tzh, t.tzf, (long)g.nx * g.ny, scale, s);
    });
}

template <typename T>
hipError_t fft_pass_y(const GridK& g, const FFTTables<T>& t, int dir, const c2<T>* in, c2<T>* out, hipStream_t s) {
    const double cb = 2.0 * sizeof(T) * (double)g.nspec();
    return timed_pass(PASS_Y, 2.0 * cb, s, [&] {
        return dir < 0 ? dispatch_strided<T, -1, false>(g.ny, in, out, t.ty, g.nzh, g.nx, (long)g.ny * g.nzh, g.nzh, s)
                       : dispatch_strided<T, +1, false>(g.ny, in, out, t.ty, g.nzh, g.nx, (long)g.ny * g.nzh, g.nzh, s);
    });
}

template <typename T>
hipError_t fft_pass_x(const GridK& g, const FFTTables<T>& t, int dir, const c2<T>* in, c2<T>* out, hipStream_t s) {
    const double cb = 2.0 * sizeof(T) * (double)g.nspec();
    return timed_pass(PASS_X, 2.0 * cb, s, [&] {
        return dir < 0 ? dispatch_strided<T, -1, true>(g.nx, in, out, t.tx, g.nzh, g.ny, g.nzh, (long)g.ny * g.nzh, s)
                       : dispatch_strided<T, +1, true>(g.nx, in, out, t.tx, g.nzh, g.ny, g.nzh, (long)g.ny * g.nzh, s);
    });
}

template <typename T>
hipError_t fft_r2c_3d(const GridK& g, const FFTTables<T>& t, const T* in, c2<T>* out, hipStream_t s) {
    hipError_t e = fft_pass_z<T>(g, t, true, in, out, (T)1, s);
    if (e != hipSuccess) return e;
    if (g.ny > 1 && (e = fft_pass_y<T>(g, t, -1, out, out, s)) != hipSuccess) return e;
    if (g.nx > 1) e = fft_pass_x<T>(g, t, -1, out, out, s);
    return e;
}

template <typename T>
hipError_t fft_c2r_3d(const GridK& g, const FFTTables<T>& t, const c2<T>* in, c2<T>* tmp, T* out,
                      hipStream_t s) {
    const c2<T>* cur = in;
    hipError_t e = hipSuccess;
    if (g.nx > 1) {
        if ((e = fft_pass_x<T>(g, t, +1, cur, tmp, s)) != hipSuccess) return e;
        cur = tmp;
    }
    if (g.ny > 1) {
        if ((e = fft_pass_y<T>(g, t, +1, cur, tmp, s)) != hipSuccess) return e;
        cur = tmp;
    }
    const T scale = (T)(1.0 / ((double)g.nx * g.ny * g.nz));
    return fft_pass_z<T>(g, t, false, cur, out, scale, s);
}

template hipError_t fft_r2c_3d<float>(const GridK&, const FFTTables<float>&, const float*, float2*, hipStream_t);
template hipError_t fft_r2c_3d<double>(const GridK&, const FFTTables<double>&, const double*, double2*,
                                       hipStream_t);
template hipError_t fft_c2r_3d<float>(const GridK&, const FFTTables<float>&, const float2*, float2*, float*,
                                      hipStream_t);
template hipError_t fft_c2r_3d<double>(const GridK&, const FFTTables<double>&, const double2*, double2*,
                                       double*, hipStream_t);
#define INST_PASS(T)                                                                                            \
    template hipError_t fft_pass_z<T>(const GridK&, const FFTTables<T>&, bool, const void*, void*, T,          \
                                      hipStream_t);                                                            \
    template hipError_t fft_pass_y<T>(const GridK&, const FFTTables<T>&, int, const c2<T>*, c2<T>*, hipStream_t); \
    template hipError_t fft_pass_x<T>(const GridK&, const FFTTables<T>&, int, const c2<T>*, c2<T>*, hipStream_t);
INST_PASS(float)
INST_PASS(double)
#undef INST_PASS

}  // namespace etd
