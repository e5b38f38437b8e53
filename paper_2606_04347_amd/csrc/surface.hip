// (-Delta_S,h)^{-1} on a narrow band by preconditioned conjugate gradients
// (Section 2.1 operator:diff and the pseudo-inverse on mean-zero functions;
// Section 3.2 narrow band).  FP64 iteration; the preconditioner's vectors
// are stored in the precision of the fields (ChebStart).
//
// Unknowns: the band nodes (mask != 0), listed in idx[0 .. *total).  Row i of
// the band matrix A is sum_{j band neighbour} w_ij (psi_i - psi_j) with
// w_ij = (g_i + g_j) / (2 h_d^2); faces to nodes off the band carry no flux.
// Right-hand side f_i - mean_band(f); A is symmetric positive semidefinite
// with the constants of a connected band as its null space, so CG from
// psi = 0 converges on the mean-zero part; the band mean of the iterate is
// removed at the end and psi = 0 off the band.
//
// Preconditioner: M^-1 = p(D^-1 A) D^-1 with D the diagonal of A and p the
// polynomial of kChebTerms terms of Chebyshev acceleration (Saad, Iterative
// Methods for Sparse Linear Systems, the Chebyshev iteration) for
// D^-1 A z = D^-1 r from z = 0 on [b / kChebRatio, b], b = 2.  D^-1 A =
// I - D^-1 W with D^-1 W row-stochastic, so its spectrum lies in [0, 2];
// there 1 - lambda p(lambda) is a scaled Chebyshev polynomial of modulus
// < 1 on (0, 2], so p > 0 and M is symmetric positive definite
// (p(D^-1 A) D^-1 = D^-1/2 p(D^-1/2 A D^-1/2) D^-1/2).  With one term it is
// Jacobi.  The polynomial lowers the condition number about kChebTerms^2
// times, so CG takes about kChebTerms times fewer iterations, each with
// kChebTerms - 1 extra stencil launches and no extra reduction.
//
// The iteration is the single-reduction (Chronopoulos-Gear) form of PCG:
// one vector-update launch, one launch for the product w = A u with all
// three dot products, and a one-workgroup launch that closes the partial
// sums (taken per workgroup in a fixed order, so results do not depend on
// scheduling) and forms the step scalars.  The scalars (alpha, beta, the
// residual norms, a done flag) live in device memory, and every kernel
// returns at once when the flag is set.
#include <algorithm>
#include <cmath>

#include "blocksum.h"
#include "kernels.h"

namespace etd {
namespace {

constexpr int kSbThreads = 256;
constexpr int kSbBlocks = 4096;
// Chebyshev preconditioner: terms and interval ratio.  Measured at 256^3
// (1.22e6 band nodes, relative residual 1e-9): Jacobi 1,061 iterations in
// 62.7 ms; 8 terms on [2/300, 2] 139 in 34.1 ms; 16 on [2/1000, 2] 71 in
// 32.5 ms (the stencil applications then dominate).
constexpr int kChebTerms = 16;
constexpr double kChebRatio = 1000.0;

enum SbSlot {
    SB_GAMMA = 0, SB_RR, SB_RR0, SB_ALPHA, SB_BETA, SB_DONE, SB_ITER, SB_MEAN, SB_XMEAN, SB_BB, SB_COUNT
};
enum SbFinal { FIN_MEAN = 0, FIN_BNORM, FIN_START, FIN_STEP, FIN_XMEAN };

struct BandGeom {
    int nx, ny, nz;
    double ihx2, ihy2, ihz2;   // 1 / h_d^2
};

BandGeom band_geom(const GridK& g) {
    return BandGeom{g.nx, g.ny, g.nz, g.nx > 1 ? 1.0 / (g.h[0] * g.h[0]) : 0.0, 1.0 / (g.h[1] * g.h[1]),
                    1.0 / (g.h[2] * g.h[2])};
}

// Calls f(j, 1/h^2) for the periodic axis neighbours j of node i (x only on
// three-dimensional grids).
template <class F> __device__ __forceinline__ void for_neighbours(const BandGeom& b, long i, F f) {
    const long sy = b.nz, sx = (long)b.ny * b.nz;
    const int z = (int)(i % b.nz);
    const long t = i / b.nz;
    const int y = (int)(t % b.ny);
    const int x = (int)(t / b.ny);
    f(z + 1 < b.nz ? i + 1 : i + 1 - b.nz, b.ihz2);
    f(z > 0 ? i - 1 : i - 1 + b.nz, b.ihz2);
    f(y + 1 < b.ny ? i + sy : i + sy - (long)b.ny * sy, b.ihy2);
    f(y > 0 ? i - sy : i - sy + (long)b.ny * sy, b.ihy2);
    if (b.nx > 1) {
        f(x + 1 < b.nx ? i + sx : i + sx - (long)b.nx * sx, b.ihx2);
        f(x > 0 ? i - sx : i - sx + (long)b.nx * sx, b.ihx2);
    }
}

// Calls f(k) for the band positions k < nb of this workgroup.  The band is
// cut into eight contiguous ranges of 256-position chunks, one per XCD
// (workgroup b is dispatched to XCD b % 8), whose workgroups take the chunks
// of their range in turn: the band neighbours of a node along y and x lie a
// few chunks away in band order, so they are mostly read through the L2 of
// the same XCD, in this launch and the next.
template <class F> __device__ __forceinline__ void band_for(long nb, F f) {
    static_assert(kSbBlocks % 8 == 0, "whole workgroups per XCD");
    const long chunks = (nb + kSbThreads - 1) / kSbThreads;
    const int x = (int)(blockIdx.x & 7u), per = (int)(gridDim.x >> 3);
    const long c1 = (x + 1) * chunks / 8;
    for (long c = x * chunks / 8 + (long)(blockIdx.x >> 3); c < c1; c += per) {
        const long k = c * kSbThreads + threadIdx.x;
        if (k < nb) f(k);
    }
}

// Three block partials per workgroup: part[3 blockIdx.x + c].
__device__ __forceinline__ void store_partials(double a, double b, double c, double* part) {
    __shared__ double sh[kSbThreads];
    const double ta = block_sum_256(a, sh);
    const double tb = block_sum_256(b, sh);
    const double tc = block_sum_256(c, sh);
    if (threadIdx.x == 0) {
        part[3 * blockIdx.x] = ta;
        part[3 * blockIdx.x + 1] = tb;
        part[3 * blockIdx.x + 2] = tc;
    }
}

__device__ __forceinline__ bool sb_done(const double* S) { return S[SB_DONE] != 0.0; }

// Jacobi diagonal (its inverse) and the band sum of f.
// gm = g on the band, -1 off it (g >= 0 everywhere): one gather per
// neighbour tells both whether the face enters and its coefficient.
template <typename T>
__global__ __launch_bounds__(kSbThreads) void k_sb_gm(long n, const T* __restrict__ G,
                                                      const uint8_t* __restrict__ mask, T* __restrict__ gm) {
    for (long i = (long)blockIdx.x * kSbThreads + threadIdx.x; i < n; i += (long)gridDim.x * kSbThreads)
        gm[i] = mask[i] ? G[i] : (T)-1;
}

template <typename T>
__global__ __launch_bounds__(kSbThreads) void k_sb_setup(BandGeom b, const T* __restrict__ gm,
                                                         const T* __restrict__ f,
                                                         const int32_t* __restrict__ idx,
                                                         const int64_t* __restrict__ total, T* dinv,
                                                         double* part) {
    const long nb = *total;
    Neu acc;
    band_for(nb, [&](long k) {
        const long i = idx[k];
        const double gi = (double)gm[i];
        double d = 0.0;
        for_neighbours(b, i, [&](long j, double ih2) {
            const T gj = gm[j];
            if (gj >= (T)0) d += 0.5 * (gi + (double)gj) * ih2;
        });
        dinv[k] = (T)(d > 0.0 ? 1.0 / d : 0.0);
        acc.add((double)f[i]);
    });
    store_partials(acc.val(), 0.0, 0.0, part);
}

// First term of the preconditioner for node k (band order), i = idx[k]:
// residual c = D^-1 r, direction d0 = c / theta (grid layout), z = d0; with
// a one-term polynomial z is the preconditioned residual u itself.
// The preconditioner's vectors (D^-1, the Chebyshev residual, sum and
// directions) are stored in P: FP32 for FP32 fields, where the solve takes
// a residual of 1e-9 at most, FP64 otherwise; their arithmetic is FP64 and
// u, the preconditioned residual handed to the iteration, is FP64.  A
// preconditioner only steers the search directions (the residual the
// iteration stops on is updated in FP64), so its rounding changes the
// iteration count, not the residual reached.
template <typename P> struct ChebStart {
    double inv_theta;
    int single;
    P* cres;
    P* cz;
    P* d0;
    double* u;
    __device__ __forceinline__ void operator()(long k, long i, double rk, double dk) const {
        const double c = rk * dk;
        const double d = c * inv_theta;
        cres[k] = (P)c;
        cz[k] = (P)d;
        d0[i] = (P)d;
        if (single) u[i] = d;
    }
};

// b = f - mean; cold start: x = 0, r = b; warm start: x as the last solve
// left it (its result on its band, 0 elsewhere), r = b - A x.  p = s = 0
// (band nodes), the preconditioner's first term; partials of (b, b); clears
// the done flag of an earlier solve.
template <typename T>
__global__ __launch_bounds__(kSbThreads) void k_sb_init(BandGeom bg, const T* __restrict__ gm, const T* __restrict__ f,
                                                        const int32_t* __restrict__ idx,
                                                        const int64_t* __restrict__ total,
                                                        const T* __restrict__ dinv, double* S, double* x,
                                                        double* r, double* p, double* sv, ChebStart<T> cs, int warm,
                                                        double* part) {
    const long nb = *total;
    const double mean = S[SB_MEAN];
    Neu bb;
    band_for(nb, [&](long k) {
        const long i = idx[k];
        const double bk = (double)f[i] - mean;
        double rk = bk;
        if (warm) {
            const double gi = (double)gm[i], xi = x[i];
            double a = 0.0;
            for_neighbours(bg, i, [&](long j, double ih2) {
                const T gj = gm[j];
                if (gj >= (T)0) a += 0.5 * (gi + (double)gj) * ih2 * (xi - x[j]);
            });
            rk = bk - a;
        } else {
            x[i] = 0.0;
        }
        bb.add(bk * bk);
        r[k] = rk;
        cs(k, i, rk, (double)dinv[k]);
        p[k] = 0.0;
        sv[k] = 0.0;
    });
    store_partials(bb.val(), 0.0, 0.0, part);
    if (blockIdx.x == 0 && threadIdx.x == 0) S[SB_DONE] = 0.0;
}

// One further term of the preconditioner: c -= D^-1 A d_prev (d_prev read at
// the band neighbours, grid layout), d = c1 d_prev + c2 c into the other
// direction buffer, z += d; the last term writes z to u (grid layout).
template <typename T>
__global__ __launch_bounds__(kSbThreads) void k_sb_cheb(BandGeom b, const T* __restrict__ gm,
                                                        const int32_t* __restrict__ idx,
                                                        const int64_t* __restrict__ total, const double* S,
                                                        const T* __restrict__ dinv, const T* __restrict__ dprev,
                                                        T* dnext, T* cres, T* cz, double c1, double c2, int last,
                                                        double* u) {
    if (sb_done(S)) return;
    const long nb = *total;
    band_for(nb, [&](long k) {
        const long i = idx[k];
        const double gi = (double)gm[i], di = (double)dprev[i];
        double a = 0.0;
        for_neighbours(b, i, [&](long j, double ih2) {
            const T gj = gm[j];
            if (gj >= (T)0) a += 0.5 * (gi + (double)gj) * ih2 * (di - (double)dprev[j]);
        });
        const double c = (double)cres[k] - (double)dinv[k] * a;
        cres[k] = (T)c;
        const double d = c1 * di + c2 * c;
        dnext[i] = (T)d;
        const double z = (double)cz[k] + d;
        cz[k] = (T)z;
        if (last) u[i] = z;
    });
}

// w = A u on the band; partials (r, u), (w, u), (r, r).
template <typename T>
__global__ __launch_bounds__(kSbThreads) void k_sb_matvec(BandGeom b, const T* __restrict__ gm,
                                                          const int32_t* __restrict__ idx,
                                                          const int64_t* __restrict__ total, const double* S,
                                                          const double* __restrict__ u, const double* __restrict__ r,
                                                          double* w, double* part) {
    if (sb_done(S)) return;
    const long nb = *total;
    Neu ru, wu, rr;
    band_for(nb, [&](long k) {
        const long i = idx[k];
        const double gi = (double)gm[i], ui = u[i];
        double a = 0.0;
        for_neighbours(b, i, [&](long j, double ih2) {
            const T gj = gm[j];
            if (gj >= (T)0) a += 0.5 * (gi + (double)gj) * ih2 * (ui - u[j]);
        });
        w[k] = a;
        const double rk = r[k];
        ru.add(rk * ui);
        wu.add(a * ui);
        rr.add(rk * rk);
    });
    store_partials(ru.val(), wu.val(), rr.val(), part);
}

// p = u + beta p, s = w + beta s, x += alpha p, r -= alpha s, the
// preconditioner's first term of the new r.
template <typename T>
__global__ __launch_bounds__(kSbThreads) void k_sb_vectors(const int32_t* __restrict__ idx,
                                                           const int64_t* __restrict__ total,
                                                           const T* __restrict__ dinv, const double* S,
                                                           double* x, const double* u, double* r, double* p,
                                                           double* sv, const double* __restrict__ w, ChebStart<T> cs) {
    if (sb_done(S)) return;
    const long nb = *total;
    const double alpha = S[SB_ALPHA], beta = S[SB_BETA];
    band_for(nb, [&](long k) {
        const long i = idx[k];
        const double pk = u[i] + beta * p[k];
        const double sk = w[k] + beta * sv[k];
        p[k] = pk;
        sv[k] = sk;
        x[i] += alpha * pk;
        const double rk = r[k] - alpha * sk;
        r[k] = rk;
        cs(k, i, rk, (double)dinv[k]);
    });
}

// band sum of x
__global__ __launch_bounds__(kSbThreads) void k_sb_xsum(const int32_t* __restrict__ idx,
                                                        const int64_t* __restrict__ total,
                                                        const double* __restrict__ x, double* part) {
    const long nb = *total;
    Neu acc;
    band_for(nb, [&](long k) { acc.add(x[idx[k]]); });
    store_partials(acc.val(), 0.0, 0.0, part);
}

// psi = x - mean_band(x) on the band, 0 elsewhere; x keeps the same values
// (in FP64), the start of a warm-started next solve.
template <typename T>
__global__ __launch_bounds__(kSbThreads) void k_sb_out(long n, const uint8_t* __restrict__ mask, double* x,
                                                       const double* S, T* psi) {
    const double m = S[SB_XMEAN];
    const bool zero = !(S[SB_BB] > 0.0);   // b = 0: the solution is 0 whatever x started from
    for (long i = (long)blockIdx.x * kSbThreads + threadIdx.x; i < n; i += (long)gridDim.x * kSbThreads) {
        const double v = (mask[i] && !zero) ? x[i] - m : 0.0;
        x[i] = v;
        psi[i] = (T)v;
    }
}

// Closes the partial sums of one kernel (fixed order) and updates the step
// scalars of the single-reduction (Chronopoulos-Gear) form of PCG:
//   gamma = (r, u), delta = (w, u), beta = gamma / gamma_old,
//   alpha = gamma / (delta - beta gamma / alpha_old).
__global__ __launch_bounds__(kSbThreads) void k_sb_final(int mode, const double* __restrict__ part,
                                                         const int64_t* __restrict__ total, double tol2, double* S) {
    if ((mode == FIN_START || mode == FIN_STEP) && sb_done(S)) return;
    __shared__ double sh[kSbThreads];
    Neu a, b, c;
    for (int k = threadIdx.x; k < kSbBlocks; k += kSbThreads) {
        a.add(part[3 * k]);
        b.add(part[3 * k + 1]);
        c.add(part[3 * k + 2]);
    }
    const double sa = block_sum_256(a.val(), sh);
    const double sb = block_sum_256(b.val(), sh);
    const double sc = block_sum_256(c.val(), sh);
    if (threadIdx.x != 0) return;
    const double nb = (double)*total;
    switch (mode) {
        case FIN_MEAN:
            S[SB_MEAN] = nb > 0 ? sa / nb : 0.0;
            break;
        case FIN_BNORM:
            S[SB_BB] = sa;
            break;
        case FIN_START:
            // the tolerance is relative to |b|, so a warm start stops where a
            // cold one would
            S[SB_GAMMA] = sa;
            S[SB_RR] = sc;
            S[SB_RR0] = S[SB_BB];
            S[SB_ITER] = 0.0;
            S[SB_BETA] = 0.0;
            if (S[SB_BB] > 0.0 && sc > tol2 * S[SB_BB] && sb > 0.0) S[SB_ALPHA] = sa / sb;
            else S[SB_DONE] = 1.0;
            break;
        case FIN_STEP: {
            S[SB_ITER] += 1.0;
            S[SB_RR] = sc;
            const double beta = S[SB_GAMMA] > 0.0 ? sa / S[SB_GAMMA] : 0.0;
            const double denom = sb - beta * sa / S[SB_ALPHA];
            if (sc <= tol2 * S[SB_RR0] || !(denom > 0.0)) {
                S[SB_DONE] = 1.0;
                break;
            }
            S[SB_BETA] = beta;
            S[SB_ALPHA] = sa / denom;
            S[SB_GAMMA] = sa;
            break;
        }
        case FIN_XMEAN:
            S[SB_XMEAN] = nb > 0 ? sa / nb : 0.0;
            break;
    }
}

template <typename T>
__global__ __launch_bounds__(kSbThreads) void k_band_ge(long n, const T* __restrict__ G, double delta,
                                                        uint8_t* mask) {
    for (long i = (long)blockIdx.x * kSbThreads + threadIdx.x; i < n; i += (long)gridDim.x * kSbThreads)
        mask[i] = (double)G[i] >= delta ? 1 : 0;
}

}  // namespace

template <typename T> void band_ge(long n, const T* G, double delta, uint8_t* mask, hipStream_t s) {
    const int nb = (int)std::min<long>(4096, (n + kSbThreads - 1) / kSbThreads);
    hipLaunchKernelGGL(k_band_ge<T>, dim3(nb), dim3(kSbThreads), 0, s, n, G, delta, mask);
}
template void band_ge<double>(long, const double*, double, uint8_t*, hipStream_t);

// Lays the workspace out from base (256-byte aligned pieces) and returns the
// bytes it spans; with base == nullptr only the size is computed.
static size_t surface_layout(long n, char* base, SurfaceWork* w) {
    size_t off = 0;
    auto take = [&](size_t bytes) -> void* {
        void* p = base ? base + off : nullptr;
        off += (bytes + 255) & ~(size_t)255;
        return p;
    };
    SurfaceWork t;
    t.x = (double*)take(n * sizeof(double));
    t.u = (double*)take(n * sizeof(double));
    t.r = (double*)take(n * sizeof(double));
    t.p = (double*)take(n * sizeof(double));
    t.s = (double*)take(n * sizeof(double));
    t.w = (double*)take(n * sizeof(double));
    t.dinv = (double*)take(n * sizeof(double));
    t.cres = (double*)take(n * sizeof(double));
    t.cz = (double*)take(n * sizeof(double));
    t.dA = (double*)take(n * sizeof(double));
    t.dB = (double*)take(n * sizeof(double));
    t.gm = (double*)take(n * sizeof(double));
    t.idx = (int32_t*)take(n * sizeof(int32_t));
    t.cnt = (int64_t*)take((band_blocks(n) + 2) * sizeof(int64_t));
    t.total = (int64_t*)take(sizeof(int64_t));
    t.part = (double*)take(3 * kSbBlocks * sizeof(double));
    t.S = (double*)take(16 * sizeof(double));
    if (w) *w = t;
    return off;
}

size_t surface_work_bytes(long n) { return surface_layout(n, nullptr, nullptr); }

void surface_work_carve(long n, void* base, SurfaceWork& w) { surface_layout(n, static_cast<char*>(base), &w); }

template <typename T>
hipError_t surface_lapinv(const GridK& g, const T* G, const T* f, const uint8_t* mask, const int32_t* idx,
                          const int64_t* total, T* psi, const SurfaceWork& w, double tol, int max_iter,
                          bool warm, SurfaceResult* res, hipStream_t s) {
    const BandGeom b = band_geom(g);
    const double tol2 = tol * tol;
    const dim3 grid(kSbBlocks), blk(kSbThreads);
    // Chebyshev acceleration on [lo, hi]: theta, delta, sigma1 = theta / delta,
    // rho_0 = 1 / sigma1, rho_j = 1 / (2 sigma1 - rho_{j-1}); term j >= 1 takes
    // d_j = rho_j rho_{j-1} d_{j-1} + (2 rho_j / delta) c_j.
    constexpr int terms = kChebTerms;
    const double hi = 2.0, lo = hi / kChebRatio;
    const double theta = 0.5 * (hi + lo), delta = 0.5 * (hi - lo), sigma1 = theta / delta;
    double c1[kChebTerms], c2[kChebTerms];
    double rho = 1.0 / sigma1;
    for (int j = 1; j < terms; ++j) {
        const double rn = 1.0 / (2.0 * sigma1 - rho);
        c1[j] = rn * rho;
        c2[j] = 2.0 * rn / delta;
        rho = rn;
    }
    // n values of T in slots of n doubles: g on the band and the preconditioner's vectors
    T* gm = reinterpret_cast<T*>(w.gm);
    T* dinv = reinterpret_cast<T*>(w.dinv);
    T* cres = reinterpret_cast<T*>(w.cres);
    T* cz = reinterpret_cast<T*>(w.cz);
    T* dA = reinterpret_cast<T*>(w.dA);
    T* dB = reinterpret_cast<T*>(w.dB);
    const ChebStart<T> cs{1.0 / theta, terms == 1 ? 1 : 0, cres, cz, dA, w.u};
    auto precond = [&]() {   // terms 1 .. terms - 1 (term 0 is formed with r)
        for (int j = 1; j < terms; ++j) {
            T* dp = (j % 2 == 1) ? dA : dB;
            T* dn = (j % 2 == 1) ? dB : dA;
            hipLaunchKernelGGL(k_sb_cheb<T>, grid, blk, 0, s, b, gm, idx, total, w.S, dinv, dp, dn, cres, cz, c1[j],
                               c2[j], j == terms - 1 ? 1 : 0, w.u);
        }
    };
    auto fin = [&](int mode) {
        hipLaunchKernelGGL(k_sb_final, dim3(1), blk, 0, s, mode, w.part, total, tol2, w.S);
    };
    auto matvec = [&]() {
        hipLaunchKernelGGL(k_sb_matvec<T>, grid, blk, 0, s, b, gm, idx, total, w.S, w.u, w.r, w.w, w.part);
    };
    const long n = g.nreal();
    const int nbo = (int)std::min<long>(4096, (n + kSbThreads - 1) / kSbThreads);
    hipLaunchKernelGGL(k_sb_gm<T>, dim3(nbo), blk, 0, s, n, G, mask, gm);
    hipLaunchKernelGGL(k_sb_setup<T>, grid, blk, 0, s, b, gm, f, idx, total, dinv, w.part);
    fin(FIN_MEAN);
    hipLaunchKernelGGL(k_sb_init<T>, grid, blk, 0, s, b, gm, f, idx, total, dinv, w.S, w.x, w.r, w.p, w.s, cs,
                       warm ? 1 : 0, w.part);
    fin(FIN_BNORM);
    precond();
    matvec();
    fin(FIN_START);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // 3 + kChebTerms - 1 launches per iteration; the host reads the done flag
    // every 25 iterations
    constexpr int kChunk = 25;
    double done = 0.0;
    for (int it = 0; it < max_iter && done == 0.0; it += kChunk) {
        for (int j = 0; j < kChunk && it + j < max_iter; ++j) {
            hipLaunchKernelGGL(k_sb_vectors<T>, grid, blk, 0, s, idx, total, dinv, w.S, w.x, w.u, w.r, w.p, w.s,
                               w.w, cs);
            precond();
            matvec();
            fin(FIN_STEP);
        }
        if ((e = hipMemcpyAsync(&done, w.S + SB_DONE, sizeof(double), hipMemcpyDeviceToHost, s)) != hipSuccess)
            return e;
        if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_sb_xsum, grid, blk, 0, s, idx, total, w.x, w.part);
    fin(FIN_XMEAN);
    hipLaunchKernelGGL(k_sb_out<T>, dim3(nbo), blk, 0, s, n, mask, w.x, w.S, psi);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (res) {
        double sc[SB_COUNT];
        if ((e = hipMemcpyAsync(sc, w.S, sizeof sc, hipMemcpyDeviceToHost, s)) != hipSuccess) return e;
        if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
        res->iters = (int)sc[SB_ITER];
        res->relres = sc[SB_RR0] > 0.0 ? std::sqrt(sc[SB_RR] / sc[SB_RR0]) : 0.0;
        res->converged = sc[SB_RR0] == 0.0 || sc[SB_RR] <= tol2 * sc[SB_RR0];
    }
    return hipSuccess;
}

template hipError_t surface_lapinv<float>(const GridK&, const float*, const float*, const uint8_t*, const int32_t*,
                                          const int64_t*, float*, const SurfaceWork&, double, int, bool,
                                          SurfaceResult*, hipStream_t);
template hipError_t surface_lapinv<double>(const GridK&, const double*, const double*, const uint8_t*,
                                           const int32_t*, const int64_t*, double*, const SurfaceWork&, double, int,
                                           bool, SurfaceResult*, hipStream_t);

}  // namespace etd
