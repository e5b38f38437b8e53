// Real <-> half-spectrum transforms of contiguous z rows (device code).
//
// A row of NR reals is viewed as M = NR / 2 complex pairs z_n = x_{2n} +
// i x_{2n+1}; the half spectrum X_k, k = 0..M, follows from the M-point
// transform Z of z by X_k = E_k + w^k O_k with 2 E_k = Z_k + conj Z_{M-k},
// 2 i O_k = Z_k - conj Z_{M-k}, w = exp(-2 pi i / NR).  The inverse packs
// Z_k = (X_k + conj X_{M-k}) + i (X_k - conj X_{M-k}) w^{-k} and transforms back.
// A workgroup handles L rows; its LDS holds L rows of stride LS plus the M
// twiddles of the half-length transform.
#pragma once

#include "lines.h"

namespace etd {
namespace stk {

template <int NR> constexpr int z_rows() { return NR >= 512 ? 8 : (NR >= 256 ? 16 : (4096 / NR)); }
template <int NR> constexpr int z_row_stride() { return line_stride<NR / 2 + 1>(); }
template <typename T, int NR> constexpr size_t z_smem() {
    return sizeof(c2<T>) * (size_t)(z_rows<NR>() * z_row_stride<NR>() + NR / 2);
}

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

// Forward: real rows src (nl <= L of them) -> half-spectrum rows dst (stride
// M + 1).  stw: the M twiddles in LDS.  On entry the LDS rows are free; on
// exit they still hold Z (callers barrier before reusing them).
template <typename T, int NR>
__device__ __forceinline__ void zrow_forward(c2<T>* lds, const c2<T>* stw, const c2<T>* __restrict__ twf,
                                             const T* src_rows, c2<T>* dst, int nl) {
    constexpr int M = NR / 2;
    constexpr int L = z_rows<NR>();
    constexpr int LS = z_row_stride<NR>();
    const c2<T>* src = reinterpret_cast<const c2<T>*>(src_rows);
    if constexpr (NextRadix<M>::v == M) {   // single stage: load to LDS, transform there
        for (int idx = threadIdx.x; idx < L * M; idx += kThreads) {
            const int r = idx / M, n = idx % M;
            lds[r * LS + sk(n)] = (r < nl) ? src[idx] : mk<T>(0, 0);
        }
        __syncthreads();
        stockham<T, M, L, LS, 1, -1>(lds, stw);
    } else {
        // first stage straight from the real rows
        lines_fft_to_lds<T, M, L, LS, 1, -1, false>(lds, stw, RowPairLoad<T, M>{src, nl});
    }
    const T half = (T)0.5;
    for (int idx = threadIdx.x; idx < L * (M + 1); idx += kThreads) {
        const int r = idx / (M + 1), k = idx % (M + 1);
        if (r < nl) {
            const c2<T> zk = lds[r * LS + sk(k == M ? 0 : k)];
            const c2<T> zc = cconj(lds[r * LS + sk(k == 0 ? 0 : M - k)]);
            const c2<T> ev = cadd(zk, zc);                  // 2 E_k
            const c2<T> od = csub(zk, zc);                  // 2 i O_k
            const c2<T> wod = cmul(twf[k], od);
            // X_k = (ev - i w^k od) / 2
            dst[idx] = mk<T>(half * (ev.x + wod.y), half * (ev.y - wod.x));
        }
    }
}

// Inverse: half-spectrum rows src -> real rows dst, times scale.  DZ: take
// i kz X_k instead of X_k (kz = az * derivative index of k, Nyquist bin 0).
// The imaginary parts of the k = 0 and k = M bins are ignored.  On entry the
// LDS rows are free.
template <typename T, int NR, bool DZ>
__device__ __forceinline__ void zrow_inverse(c2<T>* lds, const c2<T>* stw, const c2<T>* __restrict__ twf,
                                             const c2<T>* src, T* dst_rows, int nl, T scale, double az) {
    constexpr int M = NR / 2;
    constexpr int L = z_rows<NR>();
    constexpr int LS = z_row_stride<NR>();
    for (int idx = threadIdx.x; idx < L * (M + 1); idx += kThreads) {
        const int r = idx / (M + 1), k = idx % (M + 1);
        c2<T> v = (r < nl) ? src[idx] : mk<T>(0, 0);
        if constexpr (DZ) {
            const T kz = (T)(az * (double)der_index(k, NR));
            v = mk<T>(-kz * v.y, kz * v.x);
        }
        lds[r * LS + sk(k)] = v;
    }
    __syncthreads();
    // each thread owns the pair (k, M - k), so the update is in place without a barrier
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
    c2<T>* dst = reinterpret_cast<c2<T>*>(dst_rows);
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

}  // namespace stk
}  // namespace etd
