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

// Rows per workgroup of the z passes: 8 at lengths >= 512 and in FP64 at 256
// (measured faster), 16 in FP32 at 256 and below (4096 / NR for the shortest
// rows): at 64^3 the 64-row tiles of 4096 / NR left 64 workgroups per pass,
// and 16 rows took the FP32 step from 0.246 to 0.199 ms (96^3: 0.344 to
// 0.292).  The two-field forward (z_rows_pair) takes 8 in FP32 at 256 too:
// its LDS holds both fields.
template <typename T, int NR> constexpr int z_rows() {
    return NR >= 512 ? 8 : (NR >= 256 ? (sizeof(T) == 8 ? 8 : 16) : (4096 / NR > 16 ? 16 : 4096 / NR));
}
template <typename T, int NR> constexpr int z_rows_pair() { return NR >= 256 ? 8 : z_rows<T, NR>(); }
template <int NR> constexpr int z_row_stride() { return line_stride<NR / 2 + 1>(); }
template <typename T, int NR> constexpr size_t z_smem() {
    return sizeof(c2<T>) * (size_t)(z_rows<T, NR>() * z_row_stride<NR>() + NR / 2);
}

// Row l of a z tile viewed as M complex pairs (x_{2n}, x_{2n+1}); rows past the end read 0.
template <typename T, int M> struct RowPairLoad {
    static constexpr int NS = 1;
    const c2<T>* src;   // first row of the tile
    int nl;
    __device__ __forceinline__ void load(int l, int e, c2<T>* v) const {
        const c2<T> x = src[(long)(l < nl ? l : 0) * M + e];   // unconditional: row 0 read for rows past the end
        v[0] = l < nl ? x : mk<T>(0, 0);
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
// Forward of one field whose pairs come from Op::load(l, e, v) (NS == 1; 0
// for rows l >= nl): a field read from memory (RowPairLoad) or formed in the
// load.
template <typename T, int NR, class Op>
__device__ __forceinline__ void zrow_forward_op(c2<T>* lds, const c2<T>* stw, const c2<T>* __restrict__ twf,
                                                const Op& op, c2<T>* dst, int nl) {
    constexpr int M = NR / 2;
    constexpr int L = z_rows<T, NR>();
    constexpr int LS = z_row_stride<NR>();
    if constexpr (NextRadix<M>::v == M) {   // single stage: load to LDS, transform there
        for (int idx = threadIdx.x; idx < L * M; idx += kThreads) {
            const int r = idx / M, n = idx % M;
            c2<T> v[1];
            op.load(r, n, v);
            lds[r * LS + sk(n)] = v[0];
        }
        __syncthreads();
        stockham<T, M, L, LS, 1, -1>(lds, stw);
    } else {
        // first stage straight from the loads
        lines_fft_to_lds<T, M, L, LS, 1, -1, false>(lds, stw, op);
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

template <typename T, int NR>
__device__ __forceinline__ void zrow_forward(c2<T>* lds, const c2<T>* stw, const c2<T>* __restrict__ twf,
                                             const T* src_rows, c2<T>* dst, int nl) {
    zrow_forward_op<T, NR>(lds, stw, twf, RowPairLoad<T, NR / 2>{reinterpret_cast<const c2<T>*>(src_rows), nl}, dst,
                           nl);
}

// Forward of two fields at once: Op::NS == 2 and Op::load(l, e, v[2]) gives
// the pairs (x_{2e}, x_{2e+1}) of both fields in row l (0 for rows l >= nl),
// so one read of the sources feeds both transforms; field s goes through LDS
// rows s * L + l; dst0 / dst1 receive the half-spectrum rows.
template <typename T, int NR> constexpr size_t z_smem2() {
    return sizeof(c2<T>) * (size_t)(2 * z_rows_pair<T, NR>() * z_row_stride<NR>() + NR / 2);
}
template <typename T, int NR, class Op>
__device__ __forceinline__ void zrow_forward2(c2<T>* lds, const c2<T>* stw, const c2<T>* __restrict__ twf,
                                              const Op& op, c2<T>* dst0, c2<T>* dst1, int nl) {
    constexpr int M = NR / 2;
    constexpr int L = z_rows_pair<T, NR>();
    constexpr int LS = z_row_stride<NR>();
    if constexpr (NextRadix<M>::v == M) {   // single stage: load to LDS, transform there
        for (int idx = threadIdx.x; idx < L * M; idx += kThreads) {
            const int r = idx / M, n = idx % M;
            c2<T> v[2];
            op.load(r, n, v);
            lds[r * LS + sk(n)] = v[0];
            lds[(L + r) * LS + sk(n)] = v[1];
        }
        __syncthreads();
        stockham<T, M, 2 * L, LS, 1, -1>(lds, stw);
    } else {
        // The first stage issues the producer's loads (the stencils of R1 and
        // P2), at the radix first_radix picks: one butterfly per thread.
        lines_fft_to_lds<T, M, L, LS, 2, -1, false>(lds, stw, op);
    }
    const T half = (T)0.5;
    for (int idx = threadIdx.x; idx < 2 * L * (M + 1); idx += kThreads) {
        const int rr = idx / (M + 1), k = idx % (M + 1);
        const int r = rr % L;
        if (r < nl) {
            const c2<T>* row = lds + rr * LS;
            const c2<T> zk = row[sk(k == M ? 0 : k)];
            const c2<T> zc = cconj(row[sk(k == 0 ? 0 : M - k)]);
            const c2<T> ev = cadd(zk, zc);
            const c2<T> od = csub(zk, zc);
            const c2<T> wod = cmul(twf[k], od);
            (rr < L ? dst0 : dst1)[r * (M + 1) + k] = mk<T>(half * (ev.x + wod.y), half * (ev.y - wod.x));
        }
    }
}

// ---- inverse, in three steps so that a kernel with several outputs can fetch
// the next input while the current one is transformed.  L: rows of the tile
// (z_rows by default; the two-field passes take z_rows_pair).
template <typename T, int NR, int L = z_rows<T, NR>()> constexpr int z_fetch_count() {
    return (L * (NR / 2 + 1) + kThreads - 1) / kThreads;
}
template <typename T, int NR, int L = z_rows<T, NR>()>
using ZPre = c2<T>[z_fetch_count<T, NR, L>()];   // the fetched tile of a thread

// Half-spectrum rows of a tile (nl <= L rows of M + 1 values) into registers;
// element idx = threadIdx.x + p * kThreads of the row-major tile.
template <typename T, int NR, int L = z_rows<T, NR>()>
__device__ __forceinline__ void zrow_fetch(ZPre<T, NR, L>& pre, const c2<T>* src, int nl) {
    constexpr int MS = NR / 2 + 1;
    constexpr int TOT = L * MS;
#pragma unroll
    for (int p = 0; p < z_fetch_count<T, NR, L>(); ++p) {
        const int idx = threadIdx.x + p * kThreads;
        pre[p] = (idx < TOT && idx / MS < nl) ? src[idx] : mk<T>(0, 0);
    }
}

// Registers -> LDS rows, times i kz (kz = az * derivative index of k, Nyquist
// bin 0) if DZ.  The LDS rows must be free (callers barrier first).
template <typename T, int NR, bool DZ, int L = z_rows<T, NR>()>
__device__ __forceinline__ void zrow_put(c2<T>* lds, const ZPre<T, NR, L>& pre, double az) {
    constexpr int MS = NR / 2 + 1;
    constexpr int TOT = L * MS;
    constexpr int LS = z_row_stride<NR>();
#pragma unroll
    for (int p = 0; p < z_fetch_count<T, NR, L>(); ++p) {
        const int idx = threadIdx.x + p * kThreads;
        if (idx < TOT) {
            const int r = idx / MS, k = idx % MS;
            c2<T> v = pre[p];
            if constexpr (DZ) {
                const T kz = (T)(az * (double)der_index(k, NR));
                v = mk<T>(-kz * v.y, kz * v.x);
            }
            lds[r * LS + sk(k)] = v;
        }
    }
}

// LDS rows of X (written by zrow_put, not yet behind a barrier) -> pack ->
// inverse half-length transform -> Op::store(row, 0, n, z_n) with z_n the
// unscaled pair (x_{2n}, x_{2n+1}).  The imaginary parts of the k = 0 and
// k = M bins are ignored.
template <typename T, int NR, class Op, int L = z_rows<T, NR>()>
__device__ __forceinline__ void zrow_inverse_lds(c2<T>* lds, const c2<T>* stw, const c2<T>* __restrict__ twf,
                                                 const Op& op) {
    constexpr int M = NR / 2;
    constexpr int LS = z_row_stride<NR>();
    __syncthreads();
    // Z_k = (X_k + conj X_{M-k}) + i (X_k - conj X_{M-k}) w^{-k}; each thread owns
    // the pair (k, M - k), so the update is in place without a barrier
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
    if constexpr (NextRadix<M>::v == M) {
        stockham<T, M, L, LS, 1, +1>(lds, stw);
        if constexpr (IndexedOf<Op>::v) {
            constexpr int P = (L * M + kThreads - 1) / kThreads;
#pragma unroll
            for (int p = 0; p < P; ++p) {
                const int idx = threadIdx.x + p * kThreads;
                if (idx < L * M) {
                    const c2<T> v = lds[(idx / M) * LS + sk(idx % M)];
                    if constexpr (PrefetchOf<Op>::v) {
                        typename Op::Pre pre;
                        op.prefetch(idx / M, idx % M, pre);
                        op.store_at(p, idx / M, idx % M, v, pre);
                    } else {
                        op.store_at(p, idx / M, idx % M, v);
                    }
                }
            }
        } else {
            for (int idx = threadIdx.x; idx < L * M; idx += kThreads) {
                const int r = idx / M, n = idx % M;
                if constexpr (PrefetchOf<Op>::v) {
                    typename Op::Pre pre;
                    op.prefetch(r, 0, n, pre);
                    op.store(r, 0, n, lds[r * LS + sk(n)], pre);
                } else {
                    op.store(r, 0, n, lds[r * LS + sk(n)]);
                }
            }
        }
    } else {
        lines_fft_from_lds<T, M, L, LS, +1, false>(lds, stw, op);
    }
}

// Outputs per thread of zrow_inverse_lds: the slots an indexed store op
// (lines.h, IndexedOf) is given, 0 .. z_out_slots - 1.
template <typename T, int NR> constexpr int z_out_slots() {
    constexpr int M = NR / 2, L = z_rows<T, NR>();
    if constexpr (NextRadix<M>::v == M) {
        return (L * M + kThreads - 1) / kThreads;
    } else {
        constexpr int R = last_radix(M);
        return ((L * (M / R) + kThreads - 1) / kThreads) * R;
    }
}

// Inverse: half-spectrum rows src -> real rows dst, times scale.  On entry the
// LDS rows are free.
template <typename T, int NR, bool DZ>
__device__ __forceinline__ void zrow_inverse(c2<T>* lds, const c2<T>* stw, const c2<T>* __restrict__ twf,
                                             const c2<T>* src, T* dst_rows, int nl, T scale, double az) {
    c2<T> pre[z_fetch_count<T, NR>()];
    zrow_fetch<T, NR>(pre, src, nl);
    zrow_put<T, NR, DZ>(lds, pre, az);
    zrow_inverse_lds<T, NR>(lds, stw, twf, RowPairStore<T, NR / 2>{reinterpret_cast<c2<T>*>(dst_rows), nl, scale});
}

}  // namespace stk
}  // namespace etd
