// Stockham autosort engine shared by the FFT pass kernels (device code).
//
// A workgroup of kThreads threads (four 64-wide wavefronts) holds a set of
// independent lines of length N in LDS.  A radix-R stage reads the R inputs of
// each butterfly into registers, applies the twiddles w_N^(r k N/(Ns R)) with k
// the position inside the current span Ns, does the R-point DFT and writes the
// outputs to their autosorted positions (span Ns -> Ns R), so the final order
// is natural and no bit-reversal pass exists.  Radices: 3 (once, first), then
// 8 and 4 (2 only for N = 2 * 8^a), all with constant internal twiddles.
#pragma once

#include "common.h"

namespace etd {
namespace stk {

constexpr int kThreads = 256;

template <int M> struct Ilog2 { static constexpr int v = 1 + Ilog2<M / 2>::v; };
template <> struct Ilog2<1> { static constexpr int v = 0; };

// Radix of the next stage for the remaining length M.
template <int M> struct NextRadix {
    static constexpr int k = Ilog2<M>::v;
    static constexpr int v = (M % 3 == 0) ? 3 : (k == 1 ? 2 : ((k % 3 == 1 || k == 2) ? 4 : 8));
};

// multiply by DIR * i  (the quarter-turn of the transform's sign)
template <typename T, int DIR> __device__ __forceinline__ c2<T> qturn(c2<T> a) {
    return DIR > 0 ? mk<T>(-a.y, a.x) : mk<T>(a.y, -a.x);
}

template <typename T, int DIR> __device__ __forceinline__ void dft2(c2<T>* v) {
    c2<T> a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
}

template <typename T, int DIR> __device__ __forceinline__ void dft4(c2<T>* v) {
    c2<T> t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
    c2<T> t2 = cadd(v[1], v[3]), t3 = qturn<T, DIR>(csub(v[1], v[3]));
    v[0] = cadd(t0, t2);
    v[2] = csub(t0, t2);
    v[1] = cadd(t1, t3);
    v[3] = csub(t1, t3);
}

template <typename T, int DIR> __device__ __forceinline__ void dft8(c2<T>* v) {
    const T r = (T)0.70710678118654752440084436210484903;
    c2<T> b[4], c[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        b[j] = cadd(v[j], v[j + 4]);
        c[j] = csub(v[j], v[j + 4]);
    }
    // c_j *= w_8^j with w_8 = (1 + DIR i) / sqrt(2)
    c[1] = cscale(cadd(c[1], qturn<T, DIR>(c[1])), r);
    c[2] = qturn<T, DIR>(c[2]);
    c[3] = cscale(csub(qturn<T, DIR>(c[3]), c[3]), r);
    dft4<T, DIR>(b);
    dft4<T, DIR>(c);
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        v[2 * m] = b[m];
        v[2 * m + 1] = c[m];
    }
}

template <typename T, int DIR> __device__ __forceinline__ void dft3(c2<T>* v) {
    const T s3 = (T)0.86602540378443864676372317075293618;
    c2<T> t = cadd(v[1], v[2]);
    c2<T> s = cscale(qturn<T, DIR>(csub(v[1], v[2])), s3);
    c2<T> m = csub(v[0], cscale(t, (T)0.5));
    v[0] = cadd(v[0], t);
    v[1] = cadd(m, s);
    v[2] = csub(m, s);
}

template <typename T, int R, int DIR> __device__ __forceinline__ void dftR(c2<T>* v) {
    if constexpr (R == 2) dft2<T, DIR>(v);
    else if constexpr (R == 3) dft3<T, DIR>(v);
    else if constexpr (R == 4) dft4<T, DIR>(v);
    else dft8<T, DIR>(v);
}

// LDS layout of one line: element e sits at slot e + (e >> 4), one pad slot per
// 16 elements, which spreads the strided writes of the early Stockham stages
// (stride R Ns) over the LDS banks.
__host__ __device__ __forceinline__ constexpr int sk(int e) { return e + (e >> 4); }
template <int N> constexpr int line_stride() { return N + (N >> 4) + 1; }

// sk(a + c) = sk(a) + sk(c) whenever (a mod 16) + (c mod 16) < 16 (no carry
// into the pad count), so the slot of a + c is a constant offset from that of
// a and the LDS access takes it as an immediate.  NC = true only where the
// caller's (a, c) satisfy that for every c it passes.
template <bool NC> __device__ __forceinline__ int sk_add(int a, int ska, int c) {
    if constexpr (NC) return ska + sk(c);
    else return sk(a + c);
}
constexpr bool pow2(int x) { return x > 0 && (x & (x - 1)) == 0; }

// One radix-R Stockham stage on L lines of length N in LDS (line stride LS).
template <typename T, int N, int L, int LS, int R, int NS, int DIR>
__device__ __forceinline__ void stage(c2<T>* lds, const c2<T>* tw) {
    constexpr int NR = N / R;
    constexpr int NB = L * NR;
    constexpr int BPT = (NB + kThreads - 1) / kThreads;
    c2<T> v[BPT][R];
    const int tid = threadIdx.x;
#pragma unroll
    for (int i = 0; i < BPT; ++i) {
        const int b = tid + i * kThreads;
        if ((NB % kThreads == 0) || b < NB) {
            const int l = b / NR, j = b % NR;
            const c2<T>* src = lds + l * LS;
            const int skj = sk(j);
#pragma unroll
            for (int r = 0; r < R; ++r) v[i][r] = src[sk_add<NR % 16 == 0>(j, skj, r * NR)];
            if constexpr (NS > 1) {
                const int k = j % NS;
#pragma unroll
                for (int r = 1; r < R; ++r) {
                    c2<T> w = tw[r * k * (N / (NS * R))];
                    if constexpr (DIR > 0) w.y = -w.y;
                    v[i][r] = cmul(v[i][r], w);
                }
            }
            dftR<T, R, DIR>(v[i]);
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < BPT; ++i) {
        const int b = tid + i * kThreads;
        if ((NB % kThreads == 0) || b < NB) {
            const int l = b / NR, j = b % NR;
            const int k = j % NS;
            c2<T>* dst = lds + l * LS;
            const int o = (j / NS) * NS * R + k;
            const int sko = sk(o);
            // o mod 16 + (r NS) mod 16 < 16 when NS and R are powers of two
#pragma unroll
            for (int r = 0; r < R; ++r) dst[sk_add<pow2(NS) && pow2(R)>(o, sko, r * NS)] = v[i][r];
        }
    }
    __syncthreads();
}

template <typename T, int N, int L, int LS, int NS, int DIR>
__device__ __forceinline__ void stockham(c2<T>* lds, const c2<T>* tw) {
    if constexpr (NS < N) {
        constexpr int R = NextRadix<N / NS>::v;
        stage<T, N, L, LS, R, NS, DIR>(lds, tw);
        stockham<T, N, L, LS, NS * R, DIR>(lds, tw);
    }
}

template <typename T> __device__ __forceinline__ void load_table(c2<T>* dst, const c2<T>* src, int n) {
    for (int i = threadIdx.x; i < n; i += kThreads) dst[i] = src[i];
}

}  // namespace stk
}  // namespace etd
