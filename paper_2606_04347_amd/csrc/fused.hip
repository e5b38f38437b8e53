// Fused spectral pipelines (fused.h): several transforms, spectral
// multipliers and the ETD combine share one pass over memory.
//
// Strided line passes number their lines j = o * C + c (o the outer index, c
// the kz column, C = nzh columns); a workgroup takes L consecutive j, so each
// row of its tile is a contiguous run of L complex values.  On an x line the
// wavenumbers ky (from o) and kz (from c) are constants of the line; on a y
// line (x already in real space) kz is.
#include "fused.h"

#include "blocksum.h"
#include "launch.h"
#include "remainders.h"
#include "zrows.h"

namespace etd {

using namespace stk;

namespace {

template <int L> struct LineTile {
    long base[L];   // offset of element 0 of line l (< 0: past the end)
    int o[L];       // outer index
    int c[L];       // kz column
};

template <int L>
__device__ __forceinline__ void tile_setup(LineTile<L>& t, int tile, int C, int nlines, long ostride) {
    if (threadIdx.x < L) {
        const int j = tile * L + threadIdx.x;
        const bool ok = j < nlines;
        const int o = ok ? j / C : 0, c = ok ? j % C : 0;
        t.base[threadIdx.x] = ok ? (long)o * ostride + c : -1;
        t.o[threadIdx.x] = o;
        t.c[threadIdx.x] = c;
    }
}

template <typename T> __device__ __forceinline__ c2<T> times_ik(T k, c2<T> v) { return mk<T>(-k * v.y, k * v.x); }

// ------------------------------------------------------------------ derivative pipeline
// Inverse x lines at fixed (ky, kz):  A = X^-1 S,  B = X^-1 (i kx S),  C = X^-1 (-kx^2 S).
// LSRC > 0: S is read from the LDS (line l at l * LSRC, natural order, left
// there by an earlier phase of the kernel) instead of global memory.
template <typename T, int L, int LSRC = 0> struct DerivXOp {
    static constexpr int NT = 3;
    struct In {
        c2<T> s;
    };
    const LineTile<L>* t;
    const c2<T>* S;
    c2<T>* A;
    c2<T>* B;
    c2<T>* C;
    long es;
    int n;
    double a;   // pi / X_x
    __device__ __forceinline__ void load(int l, int e, In& in) const {
        if constexpr (LSRC > 0) {
            in.s = S[l * LSRC + sk(e)];
        } else {
            const long b = t->base[l];
            in.s = b >= 0 ? S[b + (long)e * es] : mk<T>(0, 0);
        }
    }
    template <int K> __device__ __forceinline__ c2<T> input(int, int e, const In& in) const {
        if constexpr (K == 0) {
            return in.s;
        } else if constexpr (K == 1) {
            return times_ik((T)(a * der_index(e, n)), in.s);
        } else {
            const double lx = a * lam_index(e, n);
            return cscale(in.s, (T)(-(lx * lx)));
        }
    }
    template <int K> __device__ __forceinline__ void store(int l, int e, c2<T> v) const {
        const long b = t->base[l];
        if (b < 0) return;
        c2<T>* dst = K == 0 ? A : (K == 1 ? B : C);
        dst[b + (long)e * es] = v;
    }
};

// Plain inverse x lines of a spectrum left in the LDS by an earlier phase.
template <typename T, int L, int LSRC> struct InvXFromLds {
    static constexpr int NT = 1;
    struct In {
        c2<T> s;
    };
    const LineTile<L>* t;
    const c2<T>* S;   // LDS
    c2<T>* W;
    long es;
    __device__ __forceinline__ void load(int l, int e, In& in) const { in.s = S[l * LSRC + sk(e)]; }
    template <int K> __device__ __forceinline__ c2<T> input(int, int, const In& in) const { return in.s; }
    template <int K> __device__ __forceinline__ void store(int l, int e, c2<T> v) const {
        const long b = t->base[l];
        if (b >= 0) W[b + (long)e * es] = v;
    }
};

// Inverse y lines at fixed (x, kz) over the x-pass outputs A, B, C:
//   Y^-1 B -> B,  Y^-1 (C - (ky^2 + kz^2) A) -> C,  Y^-1 A -> A,  Y^-1 (i ky A) -> D.
// A is fetched up front into registers; B and C are read by the transform
// that overwrites them (fetching all three up front measured slower: the
// extra registers cost more occupancy than the early loads gain).
template <typename T, int L> struct DerivYOp {
    static constexpr int NT = 4;
    static constexpr bool kFetchAll = false;   // the loop of the first stage (measured faster)
    struct In {
        c2<T> a;
    };
    const LineTile<L>* t;
    c2<T>* A;
    c2<T>* B;
    c2<T>* C;
    c2<T>* D;
    long es;
    int n;
    double ay, az;
    __device__ __forceinline__ void load(int l, int e, In& in) const {
        const long b = t->base[l];
        in.a = b >= 0 ? A[b + (long)e * es] : mk<T>(0, 0);
    }
    template <int K> __device__ __forceinline__ c2<T> input(int l, int e, const In& in) const {
        const long b = t->base[l];
        if constexpr (K == 0) {
            return b >= 0 ? B[b + (long)e * es] : mk<T>(0, 0);
        } else if constexpr (K == 1) {
            const double ly = ay * lam_index(e, n), lz = az * t->c[l];
            const T m = (T)(-(ly * ly + lz * lz));
            const c2<T> c = b >= 0 ? C[b + (long)e * es] : mk<T>(0, 0);
            return mk<T>(c.x + m * in.a.x, c.y + m * in.a.y);
        } else if constexpr (K == 2) {
            return in.a;
        } else {
            return times_ik((T)(ay * der_index(e, n)), in.a);
        }
    }
    template <int K> __device__ __forceinline__ void store(int l, int e, c2<T> v) const {
        const long b = t->base[l];
        if (b < 0) return;
        c2<T>* dst = K == 0 ? B : (K == 1 ? C : (K == 2 ? A : D));
        dst[b + (long)e * es] = v;
    }
};

template <typename T, int N>
struct k_deriv_x_body {
    static __device__ __forceinline__ void run(GridK g, const c2<T>* S, c2<T>* A, c2<T>* B, c2<T>* C,
                                                      const c2<T>* __restrict__ tw) {
        constexpr int L = lines_per_block<T, N, 1>();
        constexpr int LS = line_stride<N>();
        extern __shared__ unsigned char smem_raw[];
        __shared__ LineTile<L> tile;
        c2<T>* lds = reinterpret_cast<c2<T>*>(smem_raw);
        c2<T>* stw = lds + L * LS;
        load_table<T>(stw, tw, N);
        tile_setup<L>(tile, xcd_remap(blockIdx.x, gridDim.x), g.nzh, g.ny * g.nzh, (long)g.nzh);
        __syncthreads();
        lines_fft_seq<T, N, L, +1, true>(
            lds, stw, DerivXOp<T, L>{&tile, S, A, B, C, (long)g.ny * g.nzh, g.nx, kPi / g.X[0]});
    }
};
template <typename T, int N>
__global__ __launch_bounds__(kThreads) void k_deriv_x(GridK g, const c2<T>* S, c2<T>* A, c2<T>* B, c2<T>* C,
                                                      const c2<T>* __restrict__ tw) {
    k_deriv_x_body<T, N>::run(g, S, A, B, C, tw);
}

template <typename T, int N>
struct k_deriv_y_body {
    static __device__ __forceinline__ void run(GridK g, c2<T>* A, c2<T>* B, c2<T>* C, c2<T>* D,
                                                      const c2<T>* __restrict__ tw) {
        constexpr int L = lines_per_block<T, N, 1>();
        constexpr int LS = line_stride<N>();
        extern __shared__ unsigned char smem_raw[];
        __shared__ LineTile<L> tile;
        c2<T>* lds = reinterpret_cast<c2<T>*>(smem_raw);
        c2<T>* stw = lds + L * LS;
        load_table<T>(stw, tw, N);
        tile_setup<L>(tile, xcd_remap(blockIdx.x, gridDim.x), g.nzh, g.nx * g.nzh, (long)g.ny * g.nzh);
        __syncthreads();
        lines_fft_seq<T, N, L, +1, true>(
            lds, stw, DerivYOp<T, L>{&tile, A, B, C, D, (long)g.nzh, g.ny, kPi / g.X[1], kPi / g.X[2]});
    }
};
template <typename T, int N>
__global__ __launch_bounds__(kThreads) void k_deriv_y(GridK g, c2<T>* A, c2<T>* B, c2<T>* C, c2<T>* D,
                                                      const c2<T>* __restrict__ tw) {
    k_deriv_y_body<T, N>::run(g, A, B, C, D, tw);
}

// RowPairStore that also accumulates the stored values (FP64, compensated).
template <typename T, int M> struct SumRowPairStore {
    static constexpr int NS = 1;
    c2<T>* dst;
    int nl;
    T scale;
    Neu& acc;
    __device__ __forceinline__ void load(int, int, c2<T>*) const {}
    __device__ __forceinline__ void store(int l, int, int e, c2<T> v) const {
        if (l < nl) {
            const c2<T> w = cscale(v, scale);
            dst[(long)l * M + e] = w;
            acc.add((double)w.x);
            acc.add((double)w.y);
        }
    }
};

// z rows c2r of the y-pass outputs: phi = Z^-1 A, gz = Z^-1 (i kz A), gx = Z^-1 B,
// gy = Z^-1 D, lap = Z^-1 C.  Of the gradient only its norm gn = |grad phi|
// leaves the pass (R1 sees the gradient through its norm alone); with the
// velocity also g+ and v.
template <typename T> struct DerivZArgs {
    const c2<T>* A;
    const c2<T>* B;
    const c2<T>* C;
    const c2<T>* D;
    T* phi;
    T* gn;
    T* lap;
    const double* halt;   // nullable: once set, the pass writes nothing, except that
                          // with the velocity it copies phi^n into phi (the buffer
                          // that becomes the state)
};

// Keeps, slot by slot in registers (lines.h, IndexedOf), either the gradient
// component of this thread's outputs (KEEP, needed for the velocity) or the
// running sum of squares of the components.
template <typename T, int K, bool KEEP> struct GradStash {
    static constexpr int NS = 1;
    static constexpr bool kIndexed = true;
    c2<T> (&st)[K];
    bool first;         // this transform starts the sums
    T scale;
    __device__ __forceinline__ void load(int, int, c2<T>*) const {}
    __device__ __forceinline__ void store_at(int slot, int, int, c2<T> v) const {
        const c2<T> w = cscale(v, scale);
        if constexpr (KEEP) {
            st[slot] = w;
        } else {
            const c2<T> w2 = mk<T>(w.x * w.x, w.y * w.y);
            st[slot] = first ? w2 : mk<T>(st[slot].x + w2.x, st[slot].y + w2.y);
        }
    }
};

// The last gradient component gy: gn = |grad phi| is stored, from the sum of
// squares so far (sq) or, with VEL, from the kept gz and gx, with which it
// also forms g+ and the velocity of the u equation (velocity_point) from
// phi (stored by this thread in the first transform of the tile and read
// back) and phi^n.
template <typename T, int M, int K, bool VEL> struct GradNormStore {
    static constexpr int NS = 1;
    static constexpr bool kIndexed = true;
    const c2<T> (&sq)[K];   // !VEL
    const c2<T> (&kz)[K];   // VEL
    const c2<T> (&kx)[K];   // VEL
    c2<T>* gn;              // each: first row of the tile, as pairs
    const c2<T>* phi;
    const c2<T>* po;
    c2<T>* G;
    c2<T>* vx;
    c2<T>* vy;
    c2<T>* vz;
    int nl;
    T scale, itau;
    double thr;   // support threshold, compared in FP64
    // with VEL, phi and phi^n at the output, fetched before the butterfly
    // that makes it (rows past the tile's end read row 0, unused); FP32 only
    // (in FP64 the registers they hold cost more than the overlap gains)
    static constexpr bool kPrefetch = VEL && sizeof(T) == 4;
    struct Pre {
        c2<T> p, o;
    };
    __device__ __forceinline__ void prefetch(int l, int e, Pre& pr) const {
        if constexpr (kPrefetch) {
            const long i = (long)(l < nl ? l : 0) * M + e;
            pr.p = phi[i];
            pr.o = po[i];
        }
    }
    __device__ __forceinline__ void load(int, int, c2<T>*) const {}
    __device__ __forceinline__ void store_at(int slot, int l, int e, c2<T> v) const {
        Pre pr{};
        if constexpr (VEL) {
            if (l < nl) {
                pr.p = phi[(long)l * M + e];
                pr.o = po[(long)l * M + e];
            }
        }
        store_at(slot, l, e, v, pr);
    }
    __device__ __forceinline__ void store_at(int slot, int l, int e, c2<T> v, const Pre& pr) const {
        if (l >= nl) return;
        const long i = (long)l * M + e;
        const c2<T> b = cscale(v, scale);
        if constexpr (VEL) {
            const c2<T> p = pr.p, o = pr.o, a = kx[slot], c = kz[slot];
            gn[i] = mk<T>(sqrt(c.x * c.x + a.x * a.x + b.x * b.x), sqrt(c.y * c.y + a.y * a.y + b.y * b.y));
            c2<T> g, x, y, w;
            velocity_point(itau, thr, p.x, o.x, a.x, b.x, c.x, &g.x, &x.x, &y.x, &w.x);
            velocity_point(itau, thr, p.y, o.y, a.y, b.y, c.y, &g.y, &x.y, &y.y, &w.y);
            G[i] = g;
            vx[i] = x;
            vy[i] = y;
            vz[i] = w;
        } else {
            gn[i] = mk<T>(sqrt(sq[slot].x + b.x * b.x), sqrt(sq[slot].y + b.y * b.y));
        }
    }
};

template <typename T, int NR, bool VEL>
struct k_deriv_z_body {
    static __device__ __forceinline__ void run(DerivZArgs<T> z, VelocityArgs<T> va,
                                                      const c2<T>* __restrict__ twh, const c2<T>* __restrict__ twf,
                                                      long nrows, T scale, double az, double* part) {
        constexpr int L = z_rows<T, NR>();
        constexpr int MS = NR / 2 + 1;
        constexpr int M = NR / 2;
        constexpr int K = z_out_slots<T, NR>();
        if (halted(z.halt)) {
            if constexpr (VEL) {
                const long r0 = (long)blockIdx.x * L * NR, r1 = min(r0 + (long)L * NR, nrows * NR);
                for (long i = r0 + threadIdx.x; i < r1; i += kThreads) z.phi[i] = va.po[i];
            }
            return;
        }
        extern __shared__ unsigned char smem_raw[];
        c2<T>* lds = reinterpret_cast<c2<T>*>(smem_raw);
        c2<T>* stw = lds + L * z_row_stride<NR>();
        load_table<T>(stw, twh, M);
        const long row0 = (long)blockIdx.x * L;
        const int nl = (int)min((long)L, nrows - row0);
        const long si = row0 * MS, ro = row0 * NR;
        auto pr = [&](const T* f) { return reinterpret_cast<const c2<T>*>(f + ro); };
        auto pw = [&](T* f) { return reinterpret_cast<c2<T>*>(f + ro); };
        // each input is fetched into registers while the previous output is transformed
        c2<T> pre[z_fetch_count<T, NR>()];
        zrow_fetch<T, NR>(pre, z.A + si, nl);
        zrow_put<T, NR, false>(lds, pre, az);
        Neu acc;   // this thread's share of sum phi over the tile
        zrow_inverse_lds<T, NR>(lds, stw, twf, SumRowPairStore<T, M>{pw(z.phi), nl, scale, acc});
        // gradient components in registers: gz and gx with VEL, else their sum of squares
        c2<T> kz[K], kx[K];
        __syncthreads();
        zrow_put<T, NR, true>(lds, pre, az);
        zrow_fetch<T, NR>(pre, z.B + si, nl);
        zrow_inverse_lds<T, NR>(lds, stw, twf, GradStash<T, K, VEL>{kz, true, scale});
        __syncthreads();
        zrow_put<T, NR, false>(lds, pre, az);
        zrow_fetch<T, NR>(pre, z.D + si, nl);
        zrow_inverse_lds<T, NR>(lds, stw, twf, GradStash<T, K, VEL>{VEL ? kx : kz, false, scale});
        __syncthreads();
        zrow_put<T, NR, false>(lds, pre, az);
        zrow_fetch<T, NR>(pre, z.C + si, nl);
        zrow_inverse_lds<T, NR>(
            lds, stw, twf,
            GradNormStore<T, M, K, VEL>{kz, kz, kx, pw(z.gn), pr(z.phi), VEL ? pr(va.po) : nullptr,
                                        VEL ? pw(va.G) : nullptr, VEL ? pw(va.vx) : nullptr, VEL ? pw(va.vy) : nullptr,
                                        VEL ? pw(va.vz) : nullptr, nl, scale, (T)(VEL ? 1.0 / va.tau : 0.0),
                                        va.thr});
        __syncthreads();
        zrow_put<T, NR, false>(lds, pre, az);
        zrow_inverse_lds<T, NR>(lds, stw, twf, RowPairStore<T, M>{pw(z.lap), nl, scale});
        if (part) {
            // block partial of sum phi over this tile, for the integral of phi the
            // next R1 evaluation needs
            __syncthreads();
            const double tot = block_sum_256(acc.val(), reinterpret_cast<double*>(lds));
            if (threadIdx.x == 0) part[blockIdx.x] = tot;
        }
    }
};
template <typename T, int NR, bool VEL>
__global__ __launch_bounds__(kThreads) void k_deriv_z(DerivZArgs<T> z, VelocityArgs<T> va,
                                                      const c2<T>* __restrict__ twh, const c2<T>* __restrict__ twf,
                                                      long nrows, T scale, double az, double* part) {
    k_deriv_z_body<T, NR, VEL>::run(z, va, twh, twf, nrows, scale, az, part);
}

// z rows c2r of an increment spectrum D with the recovery of U in the store
// (Section 3.3 after Algorithm 1): d = Z^-1 D, out = u_old + d / G where
// G > thr, G u_old + d elsewhere (out may alias u_old).
template <typename T, int M> struct RecoverStore {
    static constexpr int NS = 1;
    const c2<T>* uo;    // first row of the tile, as pairs
    const c2<T>* G;
    c2<T>* out;
    int nl;
    T scale;
    double thr;   // the recovery threshold, compared in FP64 on both paths
    // u_old and G at the output, fetched before the butterfly that makes it
    // (rows past the tile's end read row 0, unused)
    static constexpr bool kPrefetch = true;
    struct Pre {
        c2<T> u, g;
    };
    __device__ __forceinline__ void prefetch(int l, int, int e, Pre& p) const {
        const long i = (long)(l < nl ? l : 0) * M + e;
        p.u = uo[i];
        p.g = G[i];
    }
    __device__ __forceinline__ void load(int, int, c2<T>*) const {}
    __device__ __forceinline__ void store(int l, int, int e, c2<T> v, const Pre& p) const {
        if (l >= nl) return;
        const long i = (long)l * M + e;
        const c2<T> u = p.u, g = p.g;
        const T d0 = v.x * scale, d1 = v.y * scale;
        c2<T> r;
        r.x = ((double)g.x > thr) ? u.x + d0 / g.x : g.x * u.x + d0;
        r.y = ((double)g.y > thr) ? u.y + d1 / g.y : g.y * u.y + d1;
        out[i] = r;
    }
};

template <typename T, int NR>
struct k_z_c2r_recover_body {
    static __device__ __forceinline__ void run(const c2<T>* D, const T* uo, const T* G, T* out,
                                                            const c2<T>* __restrict__ twh,
                                                            const c2<T>* __restrict__ twf, long nrows, T scale,
                                                            double thr, const double* halt) {
        constexpr int L = z_rows<T, NR>();
        constexpr int M = NR / 2;
        if (halted(halt)) {   // U keeps its value: out = u_old
            if (out != uo) {
                const long r0 = (long)blockIdx.x * L * NR, r1 = min(r0 + (long)L * NR, nrows * NR);
                for (long i = r0 + threadIdx.x; i < r1; i += kThreads) out[i] = uo[i];
            }
            return;
        }
        extern __shared__ unsigned char smem_raw[];
        c2<T>* lds = reinterpret_cast<c2<T>*>(smem_raw);
        c2<T>* stw = lds + L * z_row_stride<NR>();
        load_table<T>(stw, twh, M);
        const long row0 = (long)blockIdx.x * L;
        const int nl = (int)min((long)L, nrows - row0);
        const long ro = row0 * NR;
        c2<T> pre[z_fetch_count<T, NR>()];
        zrow_fetch<T, NR>(pre, D + row0 * (M + 1), nl);
        zrow_put<T, NR, false>(lds, pre, 0.0);
        zrow_inverse_lds<T, NR>(lds, stw, twf,
                                RecoverStore<T, M>{reinterpret_cast<const c2<T>*>(uo + ro),
                                                   reinterpret_cast<const c2<T>*>(G + ro),
                                                   reinterpret_cast<c2<T>*>(out + ro), nl, scale, thr});
    }
};
template <typename T, int NR>
__global__ __launch_bounds__(kThreads) void k_z_c2r_recover(const c2<T>* D, const T* uo, const T* G, T* out,
                                                            const c2<T>* __restrict__ twh,
                                                            const c2<T>* __restrict__ twf, long nrows, T scale,
                                                            double thr, const double* halt) {
    k_z_c2r_recover_body<T, NR>::run(D, uo, G, out, twh, twf, nrows, scale, thr, halt);
}

// ------------------------------------------------------------------ forward pair + ETD
template <typename T, int NR>
struct k_z_r2c_pair_body {
    static __device__ __forceinline__ void run(const T* P, const T* Q, c2<T>* WP, c2<T>* WQ,
                                                         const c2<T>* __restrict__ twh,
                                                         const c2<T>* __restrict__ twf, long nrows) {
        constexpr int L = z_rows<T, NR>();
        constexpr int MS = NR / 2 + 1;
        extern __shared__ unsigned char smem_raw[];
        c2<T>* lds = reinterpret_cast<c2<T>*>(smem_raw);
        c2<T>* stw = lds + L * z_row_stride<NR>();
        load_table<T>(stw, twh, NR / 2);
        const long row0 = (long)blockIdx.x * L;
        const int nl = (int)min((long)L, nrows - row0);
        __syncthreads();
        zrow_forward<T, NR>(lds, stw, twf, P + row0 * NR, WP + row0 * MS, nl);
        __syncthreads();
        zrow_forward<T, NR>(lds, stw, twf, Q + row0 * NR, WQ + row0 * MS, nl);
    }
};
template <typename T, int NR>
__global__ __launch_bounds__(kThreads) void k_z_r2c_pair(const T* P, const T* Q, c2<T>* WP, c2<T>* WQ,
                                                         const c2<T>* __restrict__ twh,
                                                         const c2<T>* __restrict__ twf, long nrows) {
    k_z_r2c_pair_body<T, NR>::run(P, Q, WP, WQ, twh, twf, nrows);
}

// ------------------------------------------------------------------ z r2c with R1 / P2 producers
// Row geometry of a z tile (rows row0 .. row0 + L - 1): first point of each
// row and of its x and y neighbour rows (periodic).
template <int L> struct RowTile {
    long c[L], xm[L], xp[L], ym[L], yp[L];
};
// Every row of the tile (L can exceed the workgroup: 512 rows of Nz = 8).
template <int L> __device__ __forceinline__ void row_tile_setup(RowTile<L>& t, const GridK& g, long row0) {
    for (int l = threadIdx.x; l < L; l += kThreads) {
        const long r = min(row0 + (long)l, (long)g.nx * g.ny - 1);
        const int ix = (int)(r / g.ny), iy = (int)(r % g.ny);
        const long sx = (long)g.ny * g.nz, sy = g.nz;
        const long c = r * g.nz;
        t.c[l] = c;
        t.xp[l] = c + ((ix + 1 < g.nx) ? sx : -(long)(g.nx - 1) * sx);
        t.xm[l] = c + ((ix > 0) ? -sx : (long)(g.nx - 1) * sx);
        t.yp[l] = c + ((iy + 1 < g.ny) ? sy : -(long)(g.ny - 1) * sy);
        t.ym[l] = c + ((iy > 0) ? -sy : (long)(g.ny - 1) * sy);
    }
}
template <typename T> __device__ __forceinline__ c2<T> ld2(const T* p) { return *reinterpret_cast<const c2<T>*>(p); }

// (P1, W'(phi) - A1 phi) at the point pair (2e, 2e + 1) of row l: the R1
// remainder formed where the z transform loads it.
template <typename T, int L, bool BAND> struct R1PairLoad {
    static constexpr int NS = 2;
    const RowTile<L>* rt;
    int nl, nz;
    const T *phi, *lap, *gn, *u;
    const uint8_t* mask;
    const T* surf;   // with the band: the surface part of P1, formed on the band list
    R1Const<T> k;
    __device__ __forceinline__ void load(int l, int e, c2<T>* v) const {
        if (l >= nl) {
            v[0] = v[1] = mk<T>(0, 0);
            return;
        }
        const long c = rt->c[l], o = 2 * (long)e;
        if constexpr (BAND) {
            // P1 = the local part from phi and its Laplacian, plus on the band
            // the surface part (every lane runs the same loads: no stencil
            // here, so the band costs a wave no divergent gathers)
            const c2<T> p = ld2(phi + c + o), L2 = ld2(lap + c + o);
            const unsigned short mb = *reinterpret_cast<const unsigned short*>(mask + c + o);
            T P0, Q0, P1, Q1;
            r1_core(k, p.x, L2.x, &P0, &Q0);
            r1_core(k, p.y, L2.y, &P1, &Q1);
            if (mb != 0) {
                const c2<T> sf = ld2(surf + c + o);
                P0 = P0 + ((mb & 0xff) ? sf.x : (T)0);
                P1 = P1 + ((mb >> 8) ? sf.y : (T)0);
            }
            v[0] = mk<T>(P0, P1);
            v[1] = mk<T>(Q0, Q1);
            return;
        }
        const c2<T> p = ld2(phi + c + o), L2 = ld2(lap + c + o), gg = ld2(gn + c + o), uu = ld2(u + c + o);
        const c2<T> pxm = ld2(phi + rt->xm[l] + o), pxp = ld2(phi + rt->xp[l] + o), pym = ld2(phi + rt->ym[l] + o),
                    pyp = ld2(phi + rt->yp[l] + o);
        const c2<T> uxm = ld2(u + rt->xm[l] + o), uxp = ld2(u + rt->xp[l] + o), uym = ld2(u + rt->ym[l] + o),
                    uyp = ld2(u + rt->yp[l] + o);
        const long zm = c + (o > 0 ? o - 1 : nz - 1), zp = c + (o + 2 < nz ? o + 2 : 0);
        const T pzm = phi[zm], pzp = phi[zp], uzm = u[zm], uzp = u[zp];
        T P0, Q0, P1, Q1;
        {
            const T un[6] = {uxm.x, uxp.x, uym.x, uyp.x, uzm, uu.y};
            const T pn[6] = {pxm.x, pxp.x, pym.x, pyp.x, pzm, p.y};
            r1_point(k, p.x, L2.x, gg.x, uu.x, un, pn, true, &P0, &Q0);
        }
        {
            const T un[6] = {uxm.y, uxp.y, uym.y, uyp.y, uu.x, uzp};
            const T pn[6] = {pxm.y, pxp.y, pym.y, pyp.y, p.x, pzp};
            r1_point(k, p.y, L2.y, gg.y, uu.y, un, pn, true, &P1, &Q1);
        }
        v[0] = mk<T>(P0, P1);
        v[1] = mk<T>(Q0, Q1);
    }
    __device__ __forceinline__ void store(int, int, int, c2<T>) const {}
};

// (P2, g+ u) at the point pair (2e, 2e + 1) of row l; psi from memory, or
// with psl != null from the pairs of the tile's rows in the LDS (row l at
// l * NR / 2).
template <typename T, int L, bool BAND> struct P2PairLoad {
    static constexpr int NS = 2;
    const RowTile<L>* rt;
    int nl, nz;
    const T *u, *G, *vx, *vy, *vz, *psi;
    const uint8_t* mask;
    const T* surf;   // with the band: P2 without its nonlocal term, formed on the band list
    P2Const<T> k;
    const c2<T>* psl;
    __device__ __forceinline__ void load(int l, int e, c2<T>* v) const {
        if (l >= nl) {
            v[0] = v[1] = mk<T>(0, 0);
            return;
        }
        const long c = rt->c[l], o = 2 * (long)e;
        if constexpr (BAND) {
            // g+ u everywhere; P2 (0 off the band) from its stencil part formed on
            // the band list and the nonlocal term - gamma g+ psi
            const c2<T> uu = ld2(u + c + o), GG = ld2(G + c + o);
            const unsigned short mb = *reinterpret_cast<const unsigned short*>(mask + c + o);
            T P0 = (T)0, P1 = (T)0;
            if (mb != 0) {
                const c2<T> sf = ld2(surf + c + o);
                const c2<T> ps = psl ? psl[l * (nz / 2) + e] : ld2(psi + c + o);
                if (mb & 0xff) P0 = p2_from_local(k, sf.x, GG.x, ps.x);
                if (mb >> 8) P1 = p2_from_local(k, sf.y, GG.y, ps.y);
            }
            v[0] = mk<T>(P0, P1);
            v[1] = mk<T>(GG.x * uu.x, GG.y * uu.y);
            return;
        }
        const c2<T> uu = ld2(u + c + o), GG = ld2(G + c + o), wz = ld2(vz + c + o);
        const c2<T> ps = psl ? psl[l * (nz / 2) + e] : ld2(psi + c + o);
        const c2<T> uxm = ld2(u + rt->xm[l] + o), uxp = ld2(u + rt->xp[l] + o), uym = ld2(u + rt->ym[l] + o),
                    uyp = ld2(u + rt->yp[l] + o);
        const c2<T> Gxm = ld2(G + rt->xm[l] + o), Gxp = ld2(G + rt->xp[l] + o), Gym = ld2(G + rt->ym[l] + o),
                    Gyp = ld2(G + rt->yp[l] + o);
        const c2<T> vxm = ld2(vx + rt->xm[l] + o), vxp = ld2(vx + rt->xp[l] + o), vym = ld2(vy + rt->ym[l] + o),
                    vyp = ld2(vy + rt->yp[l] + o);
        const long zm = c + (o > 0 ? o - 1 : nz - 1), zp = c + (o + 2 < nz ? o + 2 : 0);
        const T uzm = u[zm], uzp = u[zp], Gzm = G[zm], Gzp = G[zp], vzm = vz[zm], vzp = vz[zp];
        T P0, P1;
        {
            const T un[6] = {uxm.x, uxp.x, uym.x, uyp.x, uzm, uu.y};
            const T Gn[6] = {Gxm.x, Gxp.x, Gym.x, Gyp.x, Gzm, GG.y};
            const T vn[6] = {vxm.x, vxp.x, vym.x, vyp.x, vzm, wz.y};
            P0 = p2_point(k, uu.x, GG.x, ps.x, un, Gn, vn, true);
        }
        {
            const T un[6] = {uxm.y, uxp.y, uym.y, uyp.y, uu.x, uzp};
            const T Gn[6] = {Gxm.y, Gxp.y, Gym.y, Gyp.y, GG.x, Gzp};
            const T vn[6] = {vxm.y, vxp.y, vym.y, vyp.y, wz.x, vzp};
            P1 = p2_point(k, uu.y, GG.y, ps.y, un, Gn, vn, true);
        }
        v[0] = mk<T>(P0, P1);
        v[1] = mk<T>(GG.x * uu.x, GG.y * uu.y);
    }
    __device__ __forceinline__ void store(int, int, int, c2<T>) const {}
};

// q = g+ (u - ubar) on the band (Section 3.1, the nonlocal argument) at the
// point pair (2e, 2e + 1) of row l, accumulated into this thread's share of
// the mass sum.
template <typename T, int M, bool BAND> struct QPairLoad {
    static constexpr int NS = 1;
    // the loop of the first stage: fetching every butterfly first kept the
    // FP64 mass partials of all of them live (158 VGPRs, 3 waves per SIMD)
    static constexpr bool kFetchAll = false;
    const T* u;      // first row of the tile
    const T* G;
    const uint8_t* mask;
    int nl;
    T ubar;
    Neu& acc;
    __device__ __forceinline__ void load(int l, int e, c2<T>* v) const {
        // rows past the tile's end read row 0 and give 0: every load is unconditional
        const bool ok = l < nl;
        const long i = (long)(ok ? l : 0) * 2 * M + 2 * e;
        const c2<T> uu = ld2(u + i), GG = ld2(G + i);
        T q0 = GG.x * (uu.x - ubar), q1 = GG.y * (uu.y - ubar);
        if constexpr (BAND) {
            q0 = mask[i] ? q0 : (T)0;
            q1 = mask[i + 1] ? q1 : (T)0;
        }
        if (!ok) q0 = q1 = (T)0;
        acc.add((double)q0);
        acc.add((double)q1);
        v[0] = mk<T>(q0, q1);
    }
    __device__ __forceinline__ void store(int, int, int, c2<T>) const {}
};

template <typename T, int NR>
struct k_z_r2c_q_body {
    static __device__ __forceinline__ void run(const T* u, const T* G, const uint8_t* mask, T ubar, c2<T>* W,
                                                      const c2<T>* __restrict__ twh, const c2<T>* __restrict__ twf,
                                                      long nrows, double* part) {
        constexpr int L = z_rows<T, NR>();
        extern __shared__ unsigned char smem_raw[];
        c2<T>* lds = reinterpret_cast<c2<T>*>(smem_raw);
        c2<T>* stw = lds + L * z_row_stride<NR>();
        load_table<T>(stw, twh, NR / 2);
        const long row0 = (long)blockIdx.x * L;
        const int nl = (int)min((long)L, nrows - row0);
        const long ro = row0 * NR;
        Neu acc;
        if (mask)
            zrow_forward_op<T, NR>(lds, stw, twf, QPairLoad<T, NR / 2, true>{u + ro, G + ro, mask + ro, nl, ubar, acc},
                                   W + row0 * (NR / 2 + 1), nl);
        else
            zrow_forward_op<T, NR>(lds, stw, twf, QPairLoad<T, NR / 2, false>{u + ro, G + ro, nullptr, nl, ubar, acc},
                                   W + row0 * (NR / 2 + 1), nl);
        __syncthreads();
        const double tot = block_sum_256(acc.val(), reinterpret_cast<double*>(lds));
        if (threadIdx.x == 0) part[blockIdx.x] = tot;
    }
};
template <typename T, int NR>
__global__ __launch_bounds__(kThreads) void k_z_r2c_q(const T* u, const T* G, const uint8_t* mask, T ubar, c2<T>* W,
                                                      const c2<T>* __restrict__ twh, const c2<T>* __restrict__ twf,
                                                      long nrows, double* part) {
    k_z_r2c_q_body<T, NR>::run(u, G, mask, ubar, W, twh, twf, nrows, part);
}

template <typename T, int NR, bool BAND>
struct k_z_r2c_r1_body {
    static __device__ __forceinline__ void run(GridK g, CoupledK K, const T* phi, const T* lap, const T* gn,
                                                       const T* u, const uint8_t* mask, const T* surf,
                                                       const double* int_phi, double A0, c2<T>* WP, c2<T>* WQ,
                                                       const c2<T>* __restrict__ twh,
                                                       const c2<T>* __restrict__ twf, long nrows) {
        constexpr int L = z_rows_pair<T, NR>();
        constexpr int MS = NR / 2 + 1;
        extern __shared__ unsigned char smem_raw[];
        __shared__ RowTile<L> rt;
        c2<T>* lds = reinterpret_cast<c2<T>*>(smem_raw);
        c2<T>* stw = lds + 2 * L * z_row_stride<NR>();
        load_table<T>(stw, twh, NR / 2);
        const long row0 = (long)blockIdx.x * L;
        const int nl = (int)min((long)L, nrows - row0);
        row_tile_setup<L>(rt, g, row0);
        __syncthreads();
        const R1PairLoad<T, L, BAND> op{&rt, nl, g.nz, phi, lap, gn, u, mask, surf, R1Const<T>(g, K, int_phi[0], A0)};
        zrow_forward2<T, NR>(lds, stw, twf, op, WP + row0 * MS, WQ + row0 * MS, nl);
    }
};
template <typename T, int NR, bool BAND>
__global__ __launch_bounds__(kThreads) void k_z_r2c_r1(GridK g, CoupledK K, const T* phi, const T* lap, const T* gn,
                                                       const T* u, const uint8_t* mask, const T* surf,
                                                       const double* int_phi, double A0, c2<T>* WP, c2<T>* WQ,
                                                       const c2<T>* __restrict__ twh,
                                                       const c2<T>* __restrict__ twf, long nrows) {
    k_z_r2c_r1_body<T, NR, BAND>::run(g, K, phi, lap, gn, u, mask, surf, int_phi, A0, WP, WQ, twh, twf, nrows);
}

// The pairs of an inverse z transform kept in the LDS (row l at l * M).
template <typename T, int M> struct LdsPairStore {
    static constexpr int NS = 1;
    c2<T>* dst;
    T scale;
    __device__ __forceinline__ void load(int, int, c2<T>*) const {}
    __device__ __forceinline__ void store(int l, int, int e, c2<T> v) const { dst[l * M + e] = cscale(v, scale); }
};

// Dynamic LDS of the P2 z pass: the two-field forward, and with psi from its
// spectrum (PSI_HAT) the tile's psi pairs after it.
template <typename T, int NR, bool PSI_HAT> constexpr size_t z_smem_p2() {
    return z_smem2<T, NR>() + (PSI_HAT ? sizeof(c2<T>) * (size_t)z_rows_pair<T, NR>() * (NR / 2) : 0);
}

template <typename T, int NR, bool PSI_HAT, bool BAND>
struct k_z_r2c_p2_body {
    static __device__ __forceinline__ void run(GridK g, CoupledK K, const T* u, const T* G, const T* vx,
                                                       const T* vy, const T* vz, const T* psi,
                                                       const c2<T>* psi_hat, T psi_scale, const double* m,
                                                       const uint8_t* mask, const T* surf, c2<T>* WP, c2<T>* WQ,
                                                       const c2<T>* __restrict__ twh,
                                                       const c2<T>* __restrict__ twf, long nrows) {
        constexpr int L = z_rows_pair<T, NR>();
        constexpr int MS = NR / 2 + 1;
        constexpr int M = NR / 2;
        extern __shared__ unsigned char smem_raw[];
        __shared__ RowTile<L> rt;
        c2<T>* lds = reinterpret_cast<c2<T>*>(smem_raw);
        c2<T>* stw = lds + 2 * L * z_row_stride<NR>();
        c2<T>* psl = PSI_HAT ? stw + M : nullptr;   // the tile's psi pairs
        load_table<T>(stw, twh, M);
        const long row0 = (long)blockIdx.x * L;
        const int nl = (int)min((long)L, nrows - row0);
        row_tile_setup<L>(rt, g, row0);
        if constexpr (PSI_HAT) {
            // psi of the tile's rows: inverse z transform of its spectrum into the LDS
            c2<T> pre[z_fetch_count<T, NR, L>()];
            zrow_fetch<T, NR, L>(pre, psi_hat + row0 * MS, nl);
            zrow_put<T, NR, false, L>(lds, pre, 0.0);
            zrow_inverse_lds<T, NR, LdsPairStore<T, M>, L>(lds, stw, twf, LdsPairStore<T, M>{psl, psi_scale});
        }
        __syncthreads();
        const P2PairLoad<T, L, BAND> op{&rt, nl, g.nz, u, G, vx, vy, vz, psi, mask, surf, P2Const<T>(g, K, m[0]), psl};
        zrow_forward2<T, NR>(lds, stw, twf, op, WP + row0 * MS, WQ + row0 * MS, nl);
    }
};
template <typename T, int NR, bool PSI_HAT, bool BAND>
__global__ __launch_bounds__(kThreads) void k_z_r2c_p2(GridK g, CoupledK K, const T* u, const T* G, const T* vx,
                                                       const T* vy, const T* vz, const T* psi,
                                                       const c2<T>* psi_hat, T psi_scale, const double* m,
                                                       const uint8_t* mask, const T* surf, c2<T>* WP, c2<T>* WQ,
                                                       const c2<T>* __restrict__ twh,
                                                       const c2<T>* __restrict__ twf, long nrows) {
    k_z_r2c_p2_body<T, NR, PSI_HAT, BAND>::run(g, K, u, G, vx, vy, vz, psi, psi_hat, psi_scale, m, mask, surf, WP, WQ, twh,
                                             twf, nrows);
}

// two spectra through the same plain line transform, one after the other
// (each read by its own transform)
template <typename T, int L> struct PairOp {
    static constexpr int NT = 2;
    struct In {};
    const LineTile<L>* t;
    c2<T>* X0;
    c2<T>* X1;
    long es;
    __device__ __forceinline__ void load(int, int, In&) const {}
    template <int K> __device__ __forceinline__ c2<T> input(int l, int e, const In&) const {
        const long b = t->base[l];
        return b >= 0 ? (K == 0 ? X0 : X1)[b + (long)e * es] : mk<T>(0, 0);
    }
    template <int K> __device__ __forceinline__ void store(int l, int e, c2<T> v) const {
        const long b = t->base[l];
        if (b >= 0) (K == 0 ? X0 : X1)[b + (long)e * es] = v;
    }
};

template <typename T, int N>
struct k_y_pair_body {
    static __device__ __forceinline__ void run(GridK g, c2<T>* X0, c2<T>* X1, const c2<T>* __restrict__ tw) {
        constexpr int L = lines_per_block<T, N, 1>();
        constexpr int LS = line_stride<N>();
        extern __shared__ unsigned char smem_raw[];
        __shared__ LineTile<L> tile;
        c2<T>* lds = reinterpret_cast<c2<T>*>(smem_raw);
        c2<T>* stw = lds + L * LS;
        load_table<T>(stw, tw, N);
        tile_setup<L>(tile, xcd_remap(blockIdx.x, gridDim.x), g.nzh, g.nx * g.nzh, (long)g.ny * g.nzh);
        __syncthreads();
        lines_fft_seq<T, N, L, -1, true>(lds, stw, PairOp<T, L>{&tile, X0, X1, (long)g.nzh});
    }
};
template <typename T, int N>
__global__ __launch_bounds__(kThreads) void k_y_pair(GridK g, c2<T>* X0, c2<T>* X1, const c2<T>* __restrict__ tw) {
    k_y_pair_body<T, N>::run(g, X0, X1, tw);
}

// forward x lines of P and Q (both fetched up front, transformed one after
// the other); the epilogue forms k^2 in FP64 (same association as the
// standalone combine), applies the ETD combine, stores the stage output if
// asked and leaves it in the LDS (each last-stage thread writes back exactly
// the LDS entries it has read, so no barrier is needed before the write).
template <int ST, typename T, int L, int LS, bool PF> struct EtdXOp {
    static constexpr int NT = 2;
    // FP64 fetches P and Q up front (measured faster); FP32 reads each in its
    // own transform (fewer registers, higher occupancy)
    static constexpr bool kCache = sizeof(T) == 8;
    struct In {
        c2<T> p, q;
    };
    const LineTile<L>* t;
    const c2<T>* P;
    const c2<T>* Q;
    long es;
    int nx, ny;
    double ax, ay, az;
    const CoupledK* K;
    EtdArgs<T> a;
    c2<T>* lds;
    const double* kyz;   // ly^2 + lz^2 of each line of the tile
    int store_out;
    __device__ __forceinline__ void load(int l, int e, In& in) const {
        if constexpr (kCache) {
            const long b = t->base[l];
            in.p = b >= 0 ? P[b + (long)e * es] : mk<T>(0, 0);
            in.q = b >= 0 ? Q[b + (long)e * es] : mk<T>(0, 0);
        }
    }
    template <int K> __device__ __forceinline__ c2<T> input(int l, int e, const In& in) const {
        if constexpr (kCache) return K == 0 ? in.p : in.q;
        const long b = t->base[l];
        return b >= 0 ? (K == 0 ? P : Q)[b + (long)e * es] : mk<T>(0, 0);
    }
    // PF: the spectra the combine reads at (l, e) are fetched by the last
    // stage before its transform (Pre), so a thread's fetches overlap; off
    // at length 512, where the registers they take cost occupancy
    static constexpr bool kPrefetch = PF;
    using Pre = CombineIn<T>;
    __device__ __forceinline__ void prefetch(int l, int e, Pre& pre) const {
        // a line past the tile's end (base < 0) reads line 0 instead, in
        // bounds, and discards it: the loads stay unconditional
        const long b = t->base[l];
        pre = combine_load<ST, T>(a, (b >= 0 ? b : 0) + (long)e * es);
    }
    __device__ __forceinline__ void store_joint(int l, int e, const c2<T>* v) const {
        const long b = t->base[l];
        Pre pre{};
        if (b >= 0) pre = combine_load<ST, T>(a, b + (long)e * es);
        store_joint(l, e, v, pre);
    }
    __device__ __forceinline__ void store_joint(int l, int e, const c2<T>* v, const Pre& pre) const {
        const long b = t->base[l];
        c2<T> r = mk<T>(0, 0);
        if (b >= 0) {
            const double lx = ax * lam_index(e, nx);
            const double k2 = lx * lx + kyz[l];
            r = etd_combine<ST, T>(*K, k2, b + (long)e * es, v[0], v[1], a, pre);
            if (store_out) a.out[b + (long)e * es] = r;
        }
        lds[l * LS + sk(e)] = r;
    }
};

// Lines per workgroup of the ETD x pass: 16 in FP32 (runs of 128 contiguous
// bytes per x element; measured faster than 8 despite the lower occupancy),
// 8 in FP64 (the register stash of the joint transforms).  The nonlocal line
// pass measured faster with 8 in both precisions.
template <typename T, int N> constexpr int xline_tile() {
    return sizeof(T) == 4 ? lines_per_block<T, N, 1>() : lines_per_block_8<T, N, 1>();
}

// Forward x pass of the remainder pair with the ETD combine, then, on the
// combined spectrum still in the LDS, the inverse x transforms the next
// passes need: the derivative triple (S, i kx S, -kx^2 S) -> (X0, X1, X2)
// after a phi stage, the plain inverse -> X0 after a u stage.
template <int ST, typename T, int N, int L>
struct k_x_etd_body {
    static __device__ __forceinline__ void run(GridK g, CoupledK K, const c2<T>* P, const c2<T>* Q,
                                                    EtdArgs<T> a, int store_out, c2<T>* X0, c2<T>* X1, c2<T>* X2,
                                                    const c2<T>* __restrict__ tw) {
        if (halted(a.halt)) return;   // the state spectrum keeps its value
        constexpr int LS = line_stride<N>();
        extern __shared__ unsigned char smem_raw[];
        __shared__ LineTile<L> tile;
        __shared__ double kyz[L];
        c2<T>* lds = reinterpret_cast<c2<T>*>(smem_raw);
        c2<T>* stw = lds + L * LS;
        load_table<T>(stw, tw, N);
        tile_setup<L>(tile, xcd_remap(blockIdx.x, gridDim.x), g.nzh, g.ny * g.nzh, (long)g.nzh);
        if (threadIdx.x < L) {   // the entries tile_setup wrote in this thread
            const double ly = (kPi / g.X[1]) * lam_index(tile.o[threadIdx.x], g.ny);
            const double lz = (kPi / g.X[2]) * tile.c[threadIdx.x];
            kyz[threadIdx.x] = ly * ly + lz * lz;
        }
        __syncthreads();
        const long es = (long)g.ny * g.nzh;
        lines_fft_seq_joint<T, N, L, -1, true>(
            lds, stw,
            EtdXOp<ST, T, L, LS, (N <= 256)>{&tile, P, Q, es, g.nx, g.ny, kPi / g.X[0], kPi / g.X[1], kPi / g.X[2], &K,
                                             a, lds, kyz, store_out});
        __syncthreads();
        if constexpr (ST == ETD_STAGE_PHI1 || ST == ETD_STAGE_PHI2) {
            lines_fft_seq<T, N, L, +1, true, DerivXOp<T, L, LS>, true>(
                lds, stw, DerivXOp<T, L, LS>{&tile, lds, X0, X1, X2, es, g.nx, kPi / g.X[0]});
        } else {
            lines_fft_seq<T, N, L, +1, true, InvXFromLds<T, L, LS>, true>(lds, stw,
                                                                           InvXFromLds<T, L, LS>{&tile, lds, X0, es});
        }
    }
};
template <int ST, typename T, int N, int L>
__global__ __launch_bounds__(kThreads) void k_x_etd(GridK g, CoupledK K, const c2<T>* P, const c2<T>* Q,
                                                    EtdArgs<T> a, int store_out, c2<T>* X0, c2<T>* X1, c2<T>* X2,
                                                    const c2<T>* __restrict__ tw) {
    k_x_etd_body<ST, T, N, L>::run(g, K, P, Q, a, store_out, X0, X1, X2, tw);
}

// ------------------------------------------------------------------ (-Delta_h)^{-1}
template <typename T, int L> struct TileLoad {
    static constexpr int NS = 1;
    const LineTile<L>* t;
    const c2<T>* X;
    long es;
    __device__ __forceinline__ void load(int l, int e, c2<T>* v) const {
        const long b = t->base[l];
        v[0] = b >= 0 ? X[b + (long)e * es] : mk<T>(0, 0);
    }
    __device__ __forceinline__ void store(int, int, int, c2<T>) const {}
};
template <typename T, int L> struct TileStore {
    static constexpr int NS = 1;
    const LineTile<L>* t;
    c2<T>* X;
    long es;
    __device__ __forceinline__ void load(int, int, c2<T>*) const {}
    __device__ __forceinline__ void store(int l, int, int e, c2<T> v) const {
        const long b = t->base[l];
        if (b >= 0) X[b + (long)e * es] = v;
    }
};

// Lines along the last forward axis: forward transform, times 1/mu with
// mu = fde[e] + fdo[o] + fdc[c] (0 where mu = 0), inverse transform, in place.
template <typename T, int N>
struct k_lapinv_lines_body {
    static __device__ __forceinline__ void run(c2<T>* X, const c2<T>* __restrict__ tw, int C,
                                                           int nlines, long ostride, long es,
                                                           const double* __restrict__ fde,
                                                           const double* __restrict__ fdo,
                                                           const double* __restrict__ fdc) {
        constexpr int L = lines_per_block_8<T, N, 1>();
        constexpr int LS = line_stride<N>();
        extern __shared__ unsigned char smem_raw[];
        __shared__ LineTile<L> tile;
        c2<T>* lds = reinterpret_cast<c2<T>*>(smem_raw);
        c2<T>* stw = lds + L * LS;
        load_table<T>(stw, tw, N);
        tile_setup<L>(tile, xcd_remap(blockIdx.x, gridDim.x), C, nlines, ostride);
        __syncthreads();
        lines_fft_to_lds<T, N, L, LS, 1, -1, true>(lds, stw, TileLoad<T, L>{&tile, X, es});
        for (int idx = threadIdx.x; idx < L * N; idx += kThreads) {
            const int l = idx % L, e = idx / L;
            const double mu = fde[e] + fdo[tile.o[l]] + fdc[tile.c[l]];
            const T m = (T)(mu > 0.0 ? 1.0 / mu : 0.0);
            c2<T>& v = lds[l * LS + sk(e)];
            v = cscale(v, m);
        }
        __syncthreads();
        lines_fft_from_lds<T, N, L, LS, +1, true>(lds, stw, TileStore<T, L>{&tile, X, es});
    }
};
template <typename T, int N>
__global__ __launch_bounds__(kThreads) void k_lapinv_lines(c2<T>* X, const c2<T>* __restrict__ tw, int C,
                                                           int nlines, long ostride, long es,
                                                           const double* __restrict__ fde,
                                                           const double* __restrict__ fdo,
                                                           const double* __restrict__ fdc) {
    k_lapinv_lines_body<T, N>::run(X, tw, C, nlines, ostride, es, fde, fdo, fdc);
}

// ------------------------------------------------------------------ launchers
template <typename T, int N> hipError_t launch_deriv_x(const GridK& g, const c2<T>* S, c2<T>* A, c2<T>* B, c2<T>* C,
                                                       const c2<T>* tw, hipStream_t s) {
    constexpr int L = lines_per_block<T, N, 1>();
    const size_t smem = lines_smem<T, N, L, 1>();
    static_assert(lines_smem<T, N, L, 1>() <= kLdsBytes, "LDS tile larger than a workgroup can hold");
    static std::once_flag flag;
    set_smem_limit(k_deriv_x<T, N>, smem, flag);
    const int ntiles = (g.ny * g.nzh + L - 1) / L;
    launch_k<k_deriv_x_body<T, N>>(k_deriv_x<T, N>, dim3(ntiles), dim3(kThreads), smem, s, g, S, A, B, C, tw);
    return hipGetLastError();
}
template <typename T, int N> hipError_t launch_deriv_y(const GridK& g, c2<T>* A, c2<T>* B, c2<T>* C, c2<T>* D,
                                                       const c2<T>* tw, hipStream_t s) {
    constexpr int L = lines_per_block<T, N, 1>();
    const size_t smem = lines_smem<T, N, L, 1>();
    static_assert(lines_smem<T, N, L, 1>() <= kLdsBytes, "LDS tile larger than a workgroup can hold");
    static std::once_flag flag;
    set_smem_limit(k_deriv_y<T, N>, smem, flag);
    const int ntiles = (g.nx * g.nzh + L - 1) / L;
    launch_k<k_deriv_y_body<T, N>>(k_deriv_y<T, N>, dim3(ntiles), dim3(kThreads), smem, s, g, A, B, C, D, tw);
    return hipGetLastError();
}
template <typename T, int NR, bool VEL>
void launch_deriv_z_k(int nb, size_t smem, const DerivZArgs<T>& z, const VelocityArgs<T>& va, const c2<T>* twh,
                      const c2<T>* twf, long nrows, T scale, double az, double* part, hipStream_t s) {
    static std::once_flag flag;
    set_smem_limit(k_deriv_z<T, NR, VEL>, smem, flag);
    launch_k<k_deriv_z_body<T, NR, VEL>>(k_deriv_z<T, NR, VEL>, dim3(nb), dim3(kThreads), smem, s, z, va, twh, twf, nrows, scale,
                       az, part);
}
template <typename T, int NR> hipError_t launch_deriv_z(const GridK& g, const DerivZArgs<T>& z,
                                                        const VelocityArgs<T>* vel, const c2<T>* twh,
                                                        const c2<T>* twf, const GridSum* isum, hipStream_t s) {
    constexpr int L = z_rows<T, NR>();
    const size_t smem = z_smem<T, NR>();
    static_assert(z_smem<T, NR>() <= kLdsBytes, "LDS tile larger than a workgroup can hold");
    const long nrows = (long)g.nx * g.ny;
    const T scale = (T)(1.0 / ((double)g.nx * g.ny * g.nz));
    const int nb = (int)((nrows + L - 1) / L);
    double* part = isum ? isum->part : nullptr;
    if (vel)
        launch_deriv_z_k<T, NR, true>(nb, smem, z, *vel, twh, twf, nrows, scale, kPi / g.X[2], part, s);
    else
        launch_deriv_z_k<T, NR, false>(nb, smem, z, VelocityArgs<T>{}, twh, twf, nrows, scale, kPi / g.X[2], part,
                                       s);
    if (isum) reduce_final_sum(isum->part, nb, isum->scale, isum->out, s, isum->halt);
    return hipGetLastError();
}
template <typename T, int NR>
hipError_t launch_z_recover(const GridK& g, const c2<T>* D, const T* uo, const T* G, T* out, double thr,
                            const double* halt, const c2<T>* twh, const c2<T>* twf, hipStream_t s) {
    constexpr int L = z_rows<T, NR>();
    const size_t smem = z_smem<T, NR>();
    static_assert(z_smem<T, NR>() <= kLdsBytes, "LDS tile larger than a workgroup can hold");
    static std::once_flag flag;
    set_smem_limit(k_z_c2r_recover<T, NR>, smem, flag);
    const long nrows = (long)g.nx * g.ny;
    const T scale = (T)(1.0 / ((double)g.nx * g.ny * g.nz));
    launch_k<k_z_c2r_recover_body<T, NR>>(k_z_c2r_recover<T, NR>, dim3((int)((nrows + L - 1) / L)), dim3(kThreads), smem, s, D, uo, G,
                       out, twh, twf, nrows, scale, thr, halt);
    return hipGetLastError();
}
template <typename T, int NR>
hipError_t launch_z_q(const GridK& g, const T* u, const T* G, const uint8_t* mask, T ubar, c2<T>* W, const c2<T>* twh,
                      const c2<T>* twf, const GridSum& msum, hipStream_t s) {
    constexpr int L = z_rows<T, NR>();
    const size_t smem = z_smem<T, NR>();
    static_assert(z_smem<T, NR>() <= kLdsBytes, "LDS tile larger than a workgroup can hold");
    static std::once_flag flag;
    set_smem_limit(k_z_r2c_q<T, NR>, smem, flag);
    const long nrows = (long)g.nx * g.ny;
    const int nb = (int)((nrows + L - 1) / L);
    launch_k<k_z_r2c_q_body<T, NR>>(k_z_r2c_q<T, NR>, dim3(nb), dim3(kThreads), smem, s, u, G, mask, ubar, W, twh, twf, nrows,
                       msum.part);
    reduce_final_sum(msum.part, nb, msum.scale, msum.out, s, msum.halt);
    return hipGetLastError();
}

template <typename T, int NR, bool BAND>
void launch_z_r1_k(const GridK& g, const CoupledK& K, const R1Fields<T>& f, c2<T>* WP, c2<T>* WQ, const c2<T>* twh,
                   const c2<T>* twf, hipStream_t s) {
    constexpr int L = z_rows_pair<T, NR>();
    const size_t smem = z_smem2<T, NR>();
    static std::once_flag flag;
    set_smem_limit(k_z_r2c_r1<T, NR, BAND>, smem, flag);
    const long nrows = (long)g.nx * g.ny;
    launch_k<k_z_r2c_r1_body<T, NR, BAND>>(k_z_r2c_r1<T, NR, BAND>, dim3((int)((nrows + L - 1) / L)), dim3(kThreads),
                                           smem, s, g, K, f.phi, f.lap, f.gn, f.u, f.mask, f.surf, f.int_phi, f.A0, WP,
                                           WQ, twh, twf, nrows);
}
// The band form (mask set) is its own instantiation, so the full-grid pass
// carries none of its code.
template <typename T, int NR>
hipError_t launch_z_r1(const GridK& g, const CoupledK& K, const R1Fields<T>& f, c2<T>* WP, c2<T>* WQ,
                       const c2<T>* twh, const c2<T>* twf, hipStream_t s) {
    static_assert(z_smem2<T, NR>() <= kLdsBytes, "LDS tile larger than a workgroup can hold");
    if (f.mask) launch_z_r1_k<T, NR, true>(g, K, f, WP, WQ, twh, twf, s);
    else launch_z_r1_k<T, NR, false>(g, K, f, WP, WQ, twh, twf, s);
    return hipGetLastError();
}
template <typename T, int NR, bool PSI_HAT, bool BAND>
void launch_z_p2_k(const GridK& g, const CoupledK& K, const P2Fields<T>& f, c2<T>* WP, c2<T>* WQ, const c2<T>* twh,
                   const c2<T>* twf, hipStream_t s) {
    constexpr int L = z_rows_pair<T, NR>();
    const long nrows = (long)g.nx * g.ny;
    const dim3 grid((int)((nrows + L - 1) / L));
    const T scale = (T)(1.0 / ((double)g.nx * g.ny * g.nz));
    const size_t smem = z_smem_p2<T, NR, PSI_HAT>();
    static_assert(z_smem_p2<T, NR, PSI_HAT>() <= kLdsBytes, "LDS tile larger than a workgroup can hold");
    static std::once_flag flag;
    set_smem_limit(k_z_r2c_p2<T, NR, PSI_HAT, BAND>, smem, flag);
    launch_k<k_z_r2c_p2_body<T, NR, PSI_HAT, BAND>>(k_z_r2c_p2<T, NR, PSI_HAT, BAND>, grid, dim3(kThreads), smem, s, g,
                                                    K, f.u, f.G, f.vx, f.vy, f.vz, f.psi, f.psi_hat, scale, f.m,
                                                    f.mask, f.surf, WP, WQ, twh, twf, nrows);
}
// Forms: psi from its spectrum (the full-grid FFT path), psi from memory (the
// band solve without a band list in the pass), and the band form (psi from
// memory at band points).
template <typename T, int NR>
hipError_t launch_z_p2(const GridK& g, const CoupledK& K, const P2Fields<T>& f, c2<T>* WP, c2<T>* WQ,
                       const c2<T>* twh, const c2<T>* twf, hipStream_t s) {
    if (f.mask) {
        if (f.psi_hat) return hipErrorInvalidValue;   // the band form reads psi from memory
        launch_z_p2_k<T, NR, false, true>(g, K, f, WP, WQ, twh, twf, s);
    } else if (f.psi_hat) {
        launch_z_p2_k<T, NR, true, false>(g, K, f, WP, WQ, twh, twf, s);
    } else {
        launch_z_p2_k<T, NR, false, false>(g, K, f, WP, WQ, twh, twf, s);
    }
    return hipGetLastError();
}
template <typename T, int NR> hipError_t launch_z_pair(const GridK& g, const T* P, const T* Q, c2<T>* WP, c2<T>* WQ,
                                                       const c2<T>* twh, const c2<T>* twf, hipStream_t s) {
    constexpr int L = z_rows<T, NR>();
    const size_t smem = z_smem<T, NR>();
    static_assert(z_smem<T, NR>() <= kLdsBytes, "LDS tile larger than a workgroup can hold");
    static std::once_flag flag;
    set_smem_limit(k_z_r2c_pair<T, NR>, smem, flag);
    const long nrows = (long)g.nx * g.ny;
    launch_k<k_z_r2c_pair_body<T, NR>>(k_z_r2c_pair<T, NR>, dim3((int)((nrows + L - 1) / L)), dim3(kThreads), smem, s, P, Q, WP, WQ,
                       twh, twf, nrows);
    return hipGetLastError();
}
template <typename T, int N> hipError_t launch_y_pair(const GridK& g, c2<T>* X0, c2<T>* X1, const c2<T>* tw,
                                                      hipStream_t s) {
    constexpr int L = lines_per_block<T, N, 1>();
    const size_t smem = lines_smem<T, N, L, 1>();
    static_assert(lines_smem<T, N, L, 1>() <= kLdsBytes, "LDS tile larger than a workgroup can hold");
    static std::once_flag flag;
    set_smem_limit(k_y_pair<T, N>, smem, flag);
    const int ntiles = (g.nx * g.nzh + L - 1) / L;
    launch_k<k_y_pair_body<T, N>>(k_y_pair<T, N>, dim3(ntiles), dim3(kThreads), smem, s, g, X0, X1, tw);
    return hipGetLastError();
}
template <int ST, typename T, int N, int L>
hipError_t launch_x_etd(const GridK& g, const CoupledK& K, const c2<T>* P, const c2<T>* Q, const EtdArgs<T>& a,
                        int store_out, c2<T>* X0, c2<T>* X1, c2<T>* X2, const c2<T>* tw, hipStream_t s) {
    const size_t smem = lines_smem<T, N, L, 1>();
    static_assert(lines_smem<T, N, L, 1>() <= kLdsBytes, "LDS tile larger than a workgroup can hold");
    static std::once_flag flag;
    set_smem_limit(k_x_etd<ST, T, N, L>, smem, flag);
    const int ntiles = (g.ny * g.nzh + L - 1) / L;
    launch_k<k_x_etd_body<ST, T, N, L>>(k_x_etd<ST, T, N, L>, dim3(ntiles), dim3(kThreads), smem, s, g, K, P, Q, a, store_out, X0,
                       X1, X2, tw);
    return hipGetLastError();
}
// The tile of the ETD x pass at length N: xline_tile, or 8 lines where the
// FP32 default is 16 and the schedule asks for 8 (a.lines, autotuned).
template <int ST, typename T, int N>
hipError_t launch_x_etd_tiled(const GridK& g, const CoupledK& K, const c2<T>* P, const c2<T>* Q, const EtdArgs<T>& a,
                              int store_out, c2<T>* X0, c2<T>* X1, c2<T>* X2, const c2<T>* tw, hipStream_t s) {
    constexpr int L = xline_tile<T, N>();
    if constexpr (sizeof(T) == 4 && L == 16) {
        if (a.lines == 8) return launch_x_etd<ST, T, N, 8>(g, K, P, Q, a, store_out, X0, X1, X2, tw, s);
    }
    return launch_x_etd<ST, T, N, L>(g, K, P, Q, a, store_out, X0, X1, X2, tw, s);
}
template <typename T, int N>
hipError_t launch_lapinv(c2<T>* X, const c2<T>* tw, int C, int nouter, long ostride, long es, const double* fde,
                         const double* fdo, const double* fdc, hipStream_t s) {
    constexpr int L = lines_per_block_8<T, N, 1>();
    const size_t smem = lines_smem<T, N, L, 1>();
    static_assert(lines_smem<T, N, L, 1>() <= kLdsBytes, "LDS tile larger than a workgroup can hold");
    static std::once_flag flag;
    set_smem_limit(k_lapinv_lines<T, N>, smem, flag);
    const int nlines = C * nouter;
    const int ntiles = (nlines + L - 1) / L;
    launch_k<k_lapinv_lines_body<T, N>>(k_lapinv_lines<T, N>, dim3(ntiles), dim3(kThreads), smem, s, X, tw, C, nlines, ostride, es,
                       fde, fdo, fdc);
    return hipGetLastError();
}

template <int ST, typename T>
hipError_t dispatch_x_etd(const GridK& g, const CoupledK& K, const c2<T>* P, const c2<T>* Q, const EtdArgs<T>& a,
                          int store_out, c2<T>* X0, c2<T>* X1, c2<T>* X2, const c2<T>* tw, hipStream_t s) {
    switch (g.nx) {
#define CASE(n) \
    case n: return launch_x_etd_tiled<ST, T, n>(g, K, P, Q, a, store_out, X0, X1, X2, tw, s);
        ETD_FFT_SIZES(CASE)
#undef CASE
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

template <typename T>
hipError_t derivs_fused_yz(const GridK& g, const FFTTables<T>& t, c2<T>* W0, c2<T>* W1, c2<T>* W2, c2<T>* W3, T* phi,
                           T* gn, T* lap, const GridSum* isum, hipStream_t s, const VelocityArgs<T>* vel) {
    if (g.nx < 2) return hipErrorInvalidValue;
    const double cb = 2.0 * sizeof(T) * (double)g.nspec();
    const double rb = sizeof(T) * (double)g.nreal();
    hipError_t e = timed_pass(PASS_Y_DERIV, 7.0 * cb, s, [&]() -> hipError_t {
        switch (g.ny) {
#define CASE(n) \
    case n: return launch_deriv_y<T, n>(g, W0, W1, W2, W3, t.ty, s);
            ETD_FFT_SIZES(CASE)
#undef CASE
            default: return hipErrorInvalidValue;
        }
    });
    if (e != hipSuccess) return e;
    const DerivZArgs<T> z{W0, W1, W2, W3, phi, gn, lap, isum ? isum->halt : nullptr};
    // phi, |grad phi| and lap written; with the velocity also phi^n read and
    // g+ and v written (the read-back of phi is served by the cache)
    return timed_pass(PASS_Z_DERIV, 4.0 * cb + (vel ? 8.0 : 3.0) * rb, s, [&]() -> hipError_t {
        switch (g.nz) {
#define CASE(n) \
    case n: return launch_deriv_z<T, n>(g, z, vel, t.tzh, t.tzf, isum, s);
            ETD_FFT_SIZES(CASE)
#undef CASE
            default: return hipErrorInvalidValue;
        }
    });
}

template <typename T>
hipError_t derivs_fused(const GridK& g, const FFTTables<T>& t, const c2<T>* S, c2<T>* W0, c2<T>* W1, c2<T>* W2,
                        c2<T>* W3, T* phi, T* gn, T* lap, const GridSum* isum, hipStream_t s) {
    if (g.nx < 2) return hipErrorInvalidValue;
    const double cb = 2.0 * sizeof(T) * (double)g.nspec();
    hipError_t e = timed_pass(PASS_X_DERIV, 4.0 * cb, s, [&]() -> hipError_t {
        switch (g.nx) {
#define CASE(n) \
    case n: return launch_deriv_x<T, n>(g, S, W0, W1, W2, t.tx, s);
            ETD_FFT_SIZES(CASE)
#undef CASE
            default: return hipErrorInvalidValue;
        }
    });
    if (e != hipSuccess) return e;
    return derivs_fused_yz<T>(g, t, W0, W1, W2, W3, phi, gn, lap, isum, s, nullptr);
}

namespace {

// forward y pass of both spectra, then the x pass with the ETD combine and
// the inverse x transforms (fused.h, fwd_pair_etd)
template <typename T>
hipError_t pair_yx_etd(const GridK& g, const FFTTables<T>& t, const CoupledK& K, EtdStage stage, c2<T>* WP,
                       c2<T>* WQ, const EtdArgs<T>& a, bool store_out, c2<T>* X0, c2<T>* X1, c2<T>* X2,
                       hipStream_t s) {
    const double cb = 2.0 * sizeof(T) * (double)g.nspec();
    hipError_t e = timed_pass(PASS_Y_PAIR, 4.0 * cb, s, [&]() -> hipError_t {
        switch (g.ny) {
#define CASE(n) \
    case n: return launch_y_pair<T, n>(g, WP, WQ, t.ty, s);
            ETD_FFT_SIZES(CASE)
#undef CASE
            default: return hipErrorInvalidValue;
        }
    });
    if (e != hipSuccess) return e;
    // spectra read and written besides the two inputs: the combine's own
    // (prev, ra, out as the stage uses them) and the inverse x outputs
    const bool phi = stage == ETD_STAGE_PHI1 || stage == ETD_STAGE_PHI2;
    double extra = phi ? 3.0 : 1.0;
    if (stage == ETD_STAGE_PHI1) extra += 1.0 + (store_out ? 1.0 : 0.0);       // prev, ra, out
    else if (stage == ETD_STAGE_PHI2) extra += 2.0 + (store_out ? 1.0 : 0.0);  // prev, ra, out
    else if (stage == ETD_STAGE_U1) extra += 1.0 + (store_out ? 1.0 : 0.0);    // ra, out
    else extra += 2.0 + (store_out ? 1.0 : 0.0);                               // out (read), ra, out
    const int so = store_out ? 1 : 0;
    return timed_pass(PASS_X_ETD, (2.0 + extra) * cb, s, [&]() -> hipError_t {
        switch (stage) {
            case ETD_STAGE_PHI1: return dispatch_x_etd<ETD_STAGE_PHI1, T>(g, K, WP, WQ, a, so, X0, X1, X2, t.tx, s);
            case ETD_STAGE_PHI2: return dispatch_x_etd<ETD_STAGE_PHI2, T>(g, K, WP, WQ, a, so, X0, X1, X2, t.tx, s);
            case ETD_STAGE_U1: return dispatch_x_etd<ETD_STAGE_U1, T>(g, K, WP, WQ, a, so, X0, X1, X2, t.tx, s);
            case ETD_STAGE_U2: return dispatch_x_etd<ETD_STAGE_U2, T>(g, K, WP, WQ, a, so, X0, X1, X2, t.tx, s);
        }
        return hipErrorInvalidValue;
    });
}

}  // namespace

template <typename T>
hipError_t fwd_pair_etd(const GridK& g, const FFTTables<T>& t, const CoupledK& K, EtdStage stage, const T* P,
                        const T* Q, c2<T>* WP, c2<T>* WQ, const EtdArgs<T>& a, bool store_out, c2<T>* X0,
                        c2<T>* X1, c2<T>* X2, hipStream_t s) {
    if (g.nx < 2) return hipErrorInvalidValue;
    const double cb = 2.0 * sizeof(T) * (double)g.nspec();
    const double rb = sizeof(T) * (double)g.nreal();
    hipError_t e = timed_pass(PASS_Z_R2C_PAIR, 2.0 * (cb + rb), s, [&]() -> hipError_t {
        switch (g.nz) {
#define CASE(n) \
    case n: return launch_z_pair<T, n>(g, P, Q, WP, WQ, t.tzh, t.tzf, s);
            ETD_FFT_SIZES(CASE)
#undef CASE
            default: return hipErrorInvalidValue;
        }
    });
    if (e != hipSuccess) return e;
    return pair_yx_etd<T>(g, t, K, stage, WP, WQ, a, store_out, X0, X1, X2, s);
}

template <typename T>
hipError_t r1_etd(const GridK& g, const FFTTables<T>& t, const CoupledK& K, const R1Fields<T>& f, EtdStage stage,
                  c2<T>* WP, c2<T>* WQ, const EtdArgs<T>& a, bool store_out, c2<T>* X0, c2<T>* X1, c2<T>* X2,
                  hipStream_t s) {
    if (g.nx < 2) return hipErrorInvalidValue;
    const double cb = 2.0 * sizeof(T) * (double)g.nspec();
    const double rb = sizeof(T) * (double)g.nreal();
    // with the band: phi, its Laplacian and the mask (the surface part is
    // read on the band alone); else phi, lap, |grad phi| and u
    const double in = f.mask ? 2.0 * rb + (double)g.nreal() : 4.0 * rb;
    hipError_t e = timed_pass(PASS_Z_R2C_R1, in + 2.0 * cb, s, [&]() -> hipError_t {
        switch (g.nz) {
#define CASE(n) \
    case n: return launch_z_r1<T, n>(g, K, f, WP, WQ, t.tzh, t.tzf, s);
            ETD_FFT_SIZES(CASE)
#undef CASE
            default: return hipErrorInvalidValue;
        }
    });
    if (e != hipSuccess) return e;
    return pair_yx_etd<T>(g, t, K, stage, WP, WQ, a, store_out, X0, X1, X2, s);
}

template <typename T>
hipError_t p2_etd(const GridK& g, const FFTTables<T>& t, const CoupledK& K, const P2Fields<T>& f, EtdStage stage,
                  c2<T>* WP, c2<T>* WQ, const EtdArgs<T>& a, bool store_out, c2<T>* X0, hipStream_t s) {
    if (g.nx < 2) return hipErrorInvalidValue;
    const double cb = 2.0 * sizeof(T) * (double)g.nspec();
    const double rb = sizeof(T) * (double)g.nreal();
    // with psi from its spectrum the pass reads that spectrum in place of psi;
    // with the band: u, g+ and the mask (the stencil part, and psi from
    // memory, are read on the band alone); else u, g+, v and psi
    const double in = f.mask ? 2.0 * rb + (double)g.nreal() + (f.psi_hat ? cb : 0.0)
                             : (f.psi_hat ? 5.0 * rb + cb : 6.0 * rb);
    hipError_t e = timed_pass(PASS_Z_R2C_P2, in + 2.0 * cb, s,
                              [&]() -> hipError_t {
        switch (g.nz) {
#define CASE(n) \
    case n: return launch_z_p2<T, n>(g, K, f, WP, WQ, t.tzh, t.tzf, s);
            ETD_FFT_SIZES(CASE)
#undef CASE
            default: return hipErrorInvalidValue;
        }
    });
    if (e != hipSuccess) return e;
    return pair_yx_etd<T>(g, t, K, stage, WP, WQ, a, store_out, X0, nullptr, nullptr, s);
}

namespace {

// the passes of (-Delta_h)^{-1} after the forward z pass: W holds the z
// transform of q; psi receives the result
template <typename T>
hipError_t lapinv_after_z(const GridK& g, const FFTTables<T>& t, const double* fd, c2<T>* W, T* psi, hipStream_t s) {
    const double cb = 2.0 * sizeof(T) * (double)g.nspec();
    hipError_t e = hipSuccess;
    const double* fdx = fd;
    const double* fdy = fd + g.nx;
    const double* fdz = fd + g.nx + g.ny;
    if (g.nx > 1) {
        if ((e = fft_pass_y<T>(g, t, -1, W, W, s)) != hipSuccess) return e;
        // x lines: outer y (stride nzh), elements ny * nzh apart
        e = timed_pass(PASS_LAPINV, 2.0 * cb, s, [&]() -> hipError_t {
            switch (g.nx) {
#define CASE(n) \
    case n: return launch_lapinv<T, n>(W, t.tx, g.nzh, g.ny, (long)g.nzh, (long)g.ny * g.nzh, fdx, fdy, fdz, s);
                ETD_FFT_SIZES(CASE)
#undef CASE
                default: return hipErrorInvalidValue;
            }
        });
        if (e != hipSuccess) return e;
        if ((e = fft_pass_y<T>(g, t, +1, W, W, s)) != hipSuccess) return e;
    } else {
        // y lines of a two-dimensional grid: outer x (one), elements nzh apart
        e = timed_pass(PASS_LAPINV, 2.0 * cb, s, [&]() -> hipError_t {
            switch (g.ny) {
#define CASE(n) \
    case n: return launch_lapinv<T, n>(W, t.ty, g.nzh, g.nx, (long)g.ny * g.nzh, (long)g.nzh, fdy, fdx, fdz, s);
                ETD_FFT_SIZES(CASE)
#undef CASE
                default: return hipErrorInvalidValue;
            }
        });
        if (e != hipSuccess) return e;
    }
    // psi == null (three-dimensional grids): the z pass is left to the P2 pass
    if (!psi) return g.nx > 1 ? hipSuccess : hipErrorInvalidValue;
    const T scale = (T)(1.0 / ((double)g.nx * g.ny * g.nz));
    return fft_pass_z<T>(g, t, false, W, psi, scale, s);
}

}  // namespace

template <typename T>
hipError_t lapinv_fused(const GridK& g, const FFTTables<T>& t, const double* fd, const T* q, c2<T>* W, T* psi,
                        hipStream_t s) {
    hipError_t e = fft_pass_z<T>(g, t, true, q, W, (T)1, s);
    if (e != hipSuccess) return e;
    return lapinv_after_z<T>(g, t, fd, W, psi, s);
}

template <typename T>
hipError_t lapinv_q_fused(const GridK& g, const FFTTables<T>& t, const double* fd, double ubar, const T* u,
                          const T* G, const uint8_t* mask, c2<T>* W, T* psi, const GridSum& msum,
                          hipStream_t s) {
    const double cb = 2.0 * sizeof(T) * (double)g.nspec();
    const double rb = sizeof(T) * (double)g.nreal();
    const double mb = mask ? (double)g.nreal() : 0.0;
    hipError_t e = timed_pass(PASS_Z_R2C_Q, 2.0 * rb + mb + cb, s, [&]() -> hipError_t {
        switch (g.nz) {
#define CASE(n) \
    case n: return launch_z_q<T, n>(g, u, G, mask, (T)ubar, W, t.tzh, t.tzf, msum, s);
            ETD_FFT_SIZES(CASE)
#undef CASE
            default: return hipErrorInvalidValue;
        }
    });
    if (e != hipSuccess) return e;
    return lapinv_after_z<T>(g, t, fd, W, psi, s);
}

template <typename T>
hipError_t c2r_recover_yz(const GridK& g, const FFTTables<T>& t, c2<T>* W, const T* u_old, const T* G, T* out,
                          double thr, const double* halt, hipStream_t s) {
    hipError_t e = fft_pass_y<T>(g, t, +1, W, W, s);
    if (e != hipSuccess) return e;
    const double cb = 2.0 * sizeof(T) * (double)g.nspec();
    const double rb = sizeof(T) * (double)g.nreal();
    return timed_pass(PASS_Z_RECOVER, cb + 3.0 * rb, s, [&]() -> hipError_t {
        switch (g.nz) {
#define CASE(n) \
    case n: return launch_z_recover<T, n>(g, W, u_old, G, out, thr, halt, t.tzh, t.tzf, s);
            ETD_FFT_SIZES(CASE)
#undef CASE
            default: return hipErrorInvalidValue;
        }
    });
}

template <typename T>
hipError_t c2r_recover(const GridK& g, const FFTTables<T>& t, const c2<T>* D, c2<T>* W, const T* u_old, const T* G,
                       T* out, double thr, const double* halt, hipStream_t s) {
    const c2<T>* cur = D;
    hipError_t e = hipSuccess;
    if (g.nx > 1) {
        if ((e = fft_pass_x<T>(g, t, +1, cur, W, s)) != hipSuccess) return e;
    } else {
        // two-dimensional grid: the y pass reads D and writes W
        if ((e = fft_pass_y<T>(g, t, +1, cur, W, s)) != hipSuccess) return e;
        const double cb = 2.0 * sizeof(T) * (double)g.nspec();
        const double rb = sizeof(T) * (double)g.nreal();
        return timed_pass(PASS_Z_RECOVER, cb + 3.0 * rb, s, [&]() -> hipError_t {
            switch (g.nz) {
#define CASE(n) \
    case n: return launch_z_recover<T, n>(g, W, u_old, G, out, thr, halt, t.tzh, t.tzf, s);
                ETD_FFT_SIZES(CASE)
#undef CASE
                default: return hipErrorInvalidValue;
            }
        });
    }
    return c2r_recover_yz<T>(g, t, W, u_old, G, out, thr, halt, s);
}

// The instantiations are spread over several compilations of this file, so
// that they build in parallel: ETD_FUSED_PART = 2 * pipeline + precision,
// pipelines 0 (R1 and the plain pair), 1 (P2), 2 (derivatives), 3
// (recovery and the nonlocal inverse); undefined: all of them.
#ifndef ETD_FUSED_PART
#define ETD_FUSED_PART -1
#endif
#define ETD_PART(k) (ETD_FUSED_PART < 0 || ETD_FUSED_PART == (k))
#define INST_R1(T)                                                                                                \
    template hipError_t r1_etd<T>(const GridK&, const FFTTables<T>&, const CoupledK&, const R1Fields<T>&,         \
                                  EtdStage, c2<T>*, c2<T>*, const EtdArgs<T>&, bool, c2<T>*, c2<T>*, c2<T>*,      \
                                  hipStream_t);                                                                   \
    template hipError_t fwd_pair_etd<T>(const GridK&, const FFTTables<T>&, const CoupledK&, EtdStage, const T*,   \
                                        const T*, c2<T>*, c2<T>*, const EtdArgs<T>&, bool, c2<T>*, c2<T>*,        \
                                        c2<T>*, hipStream_t);
#define INST_P2(T)                                                                                                \
    template hipError_t p2_etd<T>(const GridK&, const FFTTables<T>&, const CoupledK&, const P2Fields<T>&,         \
                                  EtdStage, c2<T>*, c2<T>*, const EtdArgs<T>&, bool, c2<T>*, hipStream_t);
#define INST_DERIVS(T)                                                                                            \
    template hipError_t derivs_fused<T>(const GridK&, const FFTTables<T>&, const c2<T>*, c2<T>*, c2<T>*, c2<T>*,  \
                                        c2<T>*, T*, T*, T*, const GridSum*, hipStream_t);                         \
    template hipError_t derivs_fused_yz<T>(const GridK&, const FFTTables<T>&, c2<T>*, c2<T>*, c2<T>*, c2<T>*, T*, \
                                           T*, T*, const GridSum*, hipStream_t,                                   \
                                           const VelocityArgs<T>*);
#define INST_REST(T)                                                                                              \
    template hipError_t c2r_recover<T>(const GridK&, const FFTTables<T>&, const c2<T>*, c2<T>*, const T*,         \
                                       const T*, T*, double, const double*, hipStream_t);                         \
    template hipError_t c2r_recover_yz<T>(const GridK&, const FFTTables<T>&, c2<T>*, const T*, const T*, T*,      \
                                          double, const double*, hipStream_t);                                    \
    template hipError_t lapinv_fused<T>(const GridK&, const FFTTables<T>&, const double*, const T*, c2<T>*, T*,   \
                                        hipStream_t);                                                             \
    template hipError_t lapinv_q_fused<T>(const GridK&, const FFTTables<T>&, const double*, double, const T*,     \
                                          const T*, const uint8_t*, c2<T>*, T*, const GridSum&, hipStream_t);
#if ETD_PART(0)
INST_R1(float)
#endif
#if ETD_PART(1)
INST_R1(double)
#endif
#if ETD_PART(2)
INST_P2(float)
#endif
#if ETD_PART(3)
INST_P2(double)
#endif
#if ETD_PART(4)
INST_DERIVS(float)
#endif
#if ETD_PART(5)
INST_DERIVS(double)
#endif
#if ETD_PART(6)
INST_REST(float)
#endif
#if ETD_PART(7)
INST_REST(double)
#endif
#undef INST_R1
#undef INST_P2
#undef INST_DERIVS
#undef INST_REST
#undef ETD_PART

}  // namespace etd
