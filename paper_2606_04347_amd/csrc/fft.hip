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
#include <mutex>

#include "lines.h"

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
__global__ __launch_bounds__(kThreads) void k_fft_ylines(const c2<T>* in, c2<T>* out, const c2<T>* __restrict__ tw,
                                                         int C, int nlines, long ostride, long estride) {
    fft_lines<T, N, DIR>(in, out, tw, C, nlines, ostride, estride);
}
template <typename T, int N, int DIR>
__global__ __launch_bounds__(kThreads) void k_fft_xlines(const c2<T>* in, c2<T>* out, const c2<T>* __restrict__ tw,
                                                         int C, int nlines, long ostride, long estride) {
    fft_lines<T, N, DIR>(in, out, tw, C, nlines, ostride, estride);
}

// ---------------------------------------------------------------- z rows (r2c / c2r)
template <int NR> constexpr int z_rows() { return NR >= 512 ? 8 : (NR >= 256 ? 16 : (4096 / NR)); }

// Row l of a z tile viewed as M complex pairs (x_{2n}, x_{2n+1}); rows past the end read 0.
template <typename T, int M> struct RowPairLoad {
    static constexpr int NS = 1;
    const c2<T>* src;   // first row of the tile
    int nl;
    __device__ __forceinline__ void load(int l, int e, c2<T>* v) const {
        v[0] = l < nl ? src[(long)l * M + e] : mk<T>(0, 0);
    }
    __device__ __forceinline__ void store(int, int, int, c2<T>) const {}
};

template <typename T, int M> struct RowPairStore {
    static constexpr int NS = 1;
    c2<T>* dst;         // first row of the tile, as pairs
    int nl;
    T scale;
    __device__ __forceinline__ void load(int, int, c2<T>*) const {}
    __device__ __forceinline__ void store(int l, int, int e, c2<T> v) const {
        if (l < nl) dst[(long)l * M + e] = cscale(v, scale);
    }
};

template <typename T, int NR>
__global__ __launch_bounds__(kThreads) void k_fft_z_r2c(const T* __restrict__ in, c2<T>* __restrict__ out,
                                                        const c2<T>* __restrict__ twh,
                                                        const c2<T>* __restrict__ twf, long nrows) {
    constexpr int M = NR / 2;
    constexpr int L = z_rows<NR>();
    constexpr int LS = line_stride<M + 1>();
    extern __shared__ unsigned char smem_raw[];
    c2<T>* lds = reinterpret_cast<c2<T>*>(smem_raw);
    c2<T>* stw = lds + L * LS;
    load_table<T>(stw, twh, M);
    const long row0 = (long)blockIdx.x * L;
    const int nl = (int)min((long)L, nrows - row0);
    const c2<T>* src = reinterpret_cast<const c2<T>*>(in + row0 * NR);
    if constexpr (NextRadix<M>::v == M) {   // single stage: load to LDS, transform there
        for (int idx = threadIdx.x; idx < L * M; idx += kThreads) {
            const int r = idx / M, n = idx % M;
            lds[r * LS + sk(n)] = (r < nl) ? src[idx] : mk<T>(0, 0);
        }
        __syncthreads();
        stockham<T, M, L, LS, 1, -1>(lds, stw);
    } else {
        // z_n = x_{2n} + i x_{2n+1}: first stage straight from the real rows
        lines_fft_to_lds<T, M, L, LS, 1, -1, false>(lds, stw, RowPairLoad<T, M>{src, nl});
    }
    c2<T>* dst = out + row0 * (M + 1);
    const T half = (T)0.5;
    for (int idx = threadIdx.x; idx < L * (M + 1); idx += kThreads) {
        const int r = idx / (M + 1), k = idx % (M + 1);
        if (r < nl) {
            const c2<T> zk = lds[r * LS + sk(k == M ? 0 : k)];
            const c2<T> zc = cconj(lds[r * LS + sk(k == 0 ? 0 : M - k)]);
            const c2<T> ev = cadd(zk, zc);                  // 2 E_k
            const c2<T> od = csub(zk, zc);                  // 2 i O_k
            const c2<T> w = twf[k];
            // X_k = E_k + w^k O_k = (ev - i w od) / 2
            const c2<T> wod = cmul(w, od);
            dst[idx] = mk<T>(half * (ev.x + wod.y), half * (ev.y - wod.x));
        }
    }
}

template <typename T, int NR>
__global__ __launch_bounds__(kThreads) void k_fft_z_c2r(const c2<T>* __restrict__ in, T* __restrict__ out,
                                                        const c2<T>* __restrict__ twh,
                                                        const c2<T>* __restrict__ twf, long nrows,
                                                        T scale) {
    constexpr int M = NR / 2;
    constexpr int L = z_rows<NR>();
    constexpr int LS = line_stride<M + 1>();
    extern __shared__ unsigned char smem_raw[];
    c2<T>* lds = reinterpret_cast<c2<T>*>(smem_raw);
    c2<T>* stw = lds + L * LS;
    load_table<T>(stw, twh, M);
    const long row0 = (long)blockIdx.x * L;
    const int nl = (int)min((long)L, nrows - row0);
    const c2<T>* src = in + row0 * (M + 1);
    for (int idx = threadIdx.x; idx < L * (M + 1); idx += kThreads) {
        const int r = idx / (M + 1), k = idx % (M + 1);
        lds[r * LS + sk(k)] = (r < nl) ? src[idx] : mk<T>(0, 0);
    }
    __syncthreads();
    // Z_k = (X_k + conj X_{M-k}) + i (X_k - conj X_{M-k}) e^{+2 pi i k / NR}; each thread
    // owns the pair (k, M - k), so the update is in place without a barrier.
    constexpr int HP = M / 2 + 1;
    for (int idx = threadIdx.x; idx < L * HP; idx += kThreads) {
        const int r = idx / HP, k = idx % HP;
        c2<T>* row = lds + r * LS;
        c2<T> a = row[sk(k)], b = row[sk(M - k)];
        if (k == 0) {
            a.y = 0;
            b.y = 0;
        }
        {
            const c2<T> s = cadd(a, cconj(b));
            const c2<T> d = cmul(csub(a, cconj(b)), cconj(twf[k]));
            row[sk(k)] = mk<T>(s.x - d.y, s.y + d.x);
        }
        if (k != 0 && 2 * k != M) {
            const c2<T> s = cadd(b, cconj(a));
            const c2<T> d = cmul(csub(b, cconj(a)), cconj(twf[M - k]));
            row[sk(M - k)] = mk<T>(s.x - d.y, s.y + d.x);
        }
    }
    __syncthreads();
    c2<T>* dst = reinterpret_cast<c2<T>*>(out + row0 * NR);
    if constexpr (NextRadix<M>::v == M) {
        stockham<T, M, L, LS, 1, +1>(lds, stw);
        for (int idx = threadIdx.x; idx < L * M; idx += kThreads) {
            const int r = idx / M, n = idx % M;
            if (r < nl) dst[idx] = cscale(lds[r * LS + sk(n)], scale);
        }
    } else {
        // the last stage writes the real pairs (x_{2n}, x_{2n+1}) = z_n straight to the rows
        lines_fft_from_lds<T, M, L, LS, +1, false>(lds, stw, RowPairStore<T, M>{dst, nl, scale});
    }
}

// ---------------------------------------------------------------- launch helpers
// Raises the dynamic-LDS limit of one kernel instantiation once (each call
// site below is its own template instantiation, hence its own flag).
template <typename K> void set_smem_limit(K kernel, size_t bytes, std::once_flag& flag) {
    std::call_once(flag, [&] {
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    });
}

template <typename T, int N, int DIR, bool XLINES>
hipError_t launch_strided(const c2<T>* in, c2<T>* out, const c2<T>* tw, int C, int nouter, long ostride,
                          long estride, hipStream_t s) {
    constexpr int L = strided_lines<T, N>();
    const size_t smem = lines_smem<T, N, L, 1>();
    auto kern = XLINES ? k_fft_xlines<T, N, DIR> : k_fft_ylines<T, N, DIR>;
    static std::once_flag flag;
    set_smem_limit(kern, smem, flag);
    const long nlines = (long)C * nouter;
    const int ntiles = (int)((nlines + L - 1) / L);
    hipLaunchKernelGGL(kern, dim3(ntiles), dim3(kThreads), smem, s, in, out, tw, C, (int)nlines, ostride,
                       estride);
    return hipGetLastError();
}

template <typename T, int NR>
hipError_t launch_z(bool forward, const void* in, void* out, const c2<T>* twh, const c2<T>* twf, long nrows,
                    T scale, hipStream_t s) {
    constexpr int L = z_rows<NR>();
    const size_t smem = sizeof(c2<T>) * (size_t)(L * line_stride<NR / 2 + 1>() + NR / 2);
    const int nblk = (int)((nrows + L - 1) / L);
    if (forward) {
        auto kern = k_fft_z_r2c<T, NR>;
        static std::once_flag flag_f;
        set_smem_limit(kern, smem, flag_f);
        hipLaunchKernelGGL(kern, dim3(nblk), dim3(kThreads), smem, s, (const T*)in, (c2<T>*)out, twh, twf,
                           nrows);
    } else {
        auto kern = k_fft_z_c2r<T, NR>;
        static std::once_flag flag_i;
        set_smem_limit(kern, smem, flag_i);
        hipLaunchKernelGGL(kern, dim3(nblk), dim3(kThreads), smem, s, (const c2<T>*)in, (T*)out, twh, twf,
                           nrows, scale);
    }
    return hipGetLastError();
}

#define ETD_FFT_SIZES(X) X(8) X(16) X(32) X(64) X(128) X(256) X(512) X(12) X(24) X(48) X(96) X(192) X(384)

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

PassHook* g_hook = nullptr;

void fft_set_pass_hook(PassHook* h) { g_hook = h; }

// Run one pass launch under the optional timing hook.
template <typename F> hipError_t timed_pass(int kind, double bytes, hipStream_t s, F&& launch) {
    if (g_hook) g_hook->begin(kind, s);
    hipError_t e = launch();
    if (g_hook) g_hook->end(kind, bytes, s);
    return e;
}

template <typename T>
hipError_t fft_r2c_3d(const GridK& g, const FFTTables<T>& t, const T* in, c2<T>* out, hipStream_t s) {
    const long rows = (long)g.nx * g.ny;
    const double cb = 2.0 * sizeof(T) * (double)g.nspec();     // one complex half spectrum
    hipError_t e = timed_pass(0, cb + sizeof(T) * (double)g.nreal(), s, [&] {
        return dispatch_z<T>(g.nz, true, in, out, t.tzh, t.tzf, rows, (T)1, s);
    });
    if (e != hipSuccess) return e;
    if (g.ny > 1) {   // y lines: outer x, stride nzh
        e = timed_pass(2, 2.0 * cb, s, [&] {
            return dispatch_strided<T, -1, false>(g.ny, out, out, t.ty, g.nzh, g.nx, (long)g.ny * g.nzh, g.nzh, s);
        });
        if (e != hipSuccess) return e;
    }
    if (g.nx > 1) {   // x lines: outer y, stride ny * nzh
        e = timed_pass(3, 2.0 * cb, s, [&] {
            return dispatch_strided<T, -1, true>(g.nx, out, out, t.tx, g.nzh, g.ny, g.nzh, (long)g.ny * g.nzh, s);
        });
    }
    return e;
}

template <typename T>
hipError_t fft_c2r_3d(const GridK& g, const FFTTables<T>& t, const c2<T>* in, c2<T>* tmp, T* out,
                      hipStream_t s) {
    const c2<T>* cur = in;
    hipError_t e = hipSuccess;
    const double cb = 2.0 * sizeof(T) * (double)g.nspec();
    if (g.nx > 1) {
        e = timed_pass(3, 2.0 * cb, s, [&] {
            return dispatch_strided<T, +1, true>(g.nx, cur, tmp, t.tx, g.nzh, g.ny, g.nzh, (long)g.ny * g.nzh, s);
        });
        if (e != hipSuccess) return e;
        cur = tmp;
    }
    if (g.ny > 1) {
        e = timed_pass(2, 2.0 * cb, s, [&] {
            return dispatch_strided<T, +1, false>(g.ny, cur, tmp, t.ty, g.nzh, g.nx, (long)g.ny * g.nzh, g.nzh, s);
        });
        if (e != hipSuccess) return e;
        cur = tmp;
    }
    const T scale = (T)(1.0 / ((double)g.nx * g.ny * g.nz));
    return timed_pass(1, cb + sizeof(T) * (double)g.nreal(), s, [&] {
        return dispatch_z<T>(g.nz, false, cur, out, t.tzh, t.tzf, (long)g.nx * g.ny, scale, s);
    });
}

template hipError_t fft_r2c_3d<float>(const GridK&, const FFTTables<float>&, const float*, float2*, hipStream_t);
template hipError_t fft_r2c_3d<double>(const GridK&, const FFTTables<double>&, const double*, double2*,
                                       hipStream_t);
template hipError_t fft_c2r_3d<float>(const GridK&, const FFTTables<float>&, const float2*, float2*, float*,
                                      hipStream_t);
template hipError_t fft_c2r_3d<double>(const GridK&, const FFTTables<double>&, const double2*, double2*,
                                       double*, hipStream_t);

}  // namespace etd
