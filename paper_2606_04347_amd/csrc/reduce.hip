// Deterministic FP64 reductions.  Stage 1: a fixed grid of kRedBlocks
// workgroups; each thread walks a grid-stride range accumulating sums with
// Neumaier compensation (and maxima), the workgroup combines its 256 threads
// in a fixed tree.  Stage 2: one workgroup combines the kRedBlocks partials in
// the same fixed order.  Same inputs and sizes therefore give bitwise-equal
// results run to run; the totals stay on the device for later kernels.
#include "blocksum.h"
#include "kernels.h"
#include "launch.h"

namespace etd {

namespace {

constexpr int kB = 256;


// F: __device__ void operator()(long i, double* sums, double* maxes) const (accumulates in place:
// sums are plain per-element values to add, maxes are per-element values to max)
template <int NS, int NM, class F>
__global__ __launch_bounds__(kB) void k_reduce(F f, long n, double* part) {
    // U interleaved accumulator sets per thread (element i + u * stride goes to
    // set u), so U independent loads and compensated adds are in flight; the
    // sets are combined in a fixed order
    constexpr int U = (NS + NM <= 2) ? 4 : 1;
    Neu acc[U][NS > 0 ? NS : 1];
    double mx[U][NM > 0 ? NM : 1];
#pragma unroll
    for (int u = 0; u < U; ++u)
        for (int j = 0; j < NM; ++j) mx[u][j] = -INFINITY;
    const long stride = (long)gridDim.x * kB;
    for (long i0 = (long)blockIdx.x * kB + threadIdx.x; i0 < n; i0 += U * stride) {
        double s[U][NS > 0 ? NS : 1], m[U][NM > 0 ? NM : 1];
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (i0 + u * stride < n) f(i0 + u * stride, s[u], m[u]);
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (i0 + u * stride < n) {
                for (int j = 0; j < NS; ++j) acc[u][j].add(s[u][j]);
                for (int j = 0; j < NM; ++j) mx[u][j] = fmax(mx[u][j], m[u][j]);
            }
    }
#pragma unroll
    for (int u = 1; u < U; ++u) {
        for (int j = 0; j < NS; ++j) {
            acc[0][j].add(acc[u][j].s);
            acc[0][j].add(acc[u][j].c);
        }
        for (int j = 0; j < NM; ++j) mx[0][j] = fmax(mx[0][j], mx[u][j]);
    }
    __shared__ double sh[4];
    for (int j = 0; j < NS + NM; ++j) {
        const double r = (j < NS) ? block_sum_256(acc[0][j].val(), sh) : block_max_256(mx[0][j - NS], sh);
        if (threadIdx.x == 0) part[(long)blockIdx.x * (NS + NM) + j] = r;
    }
}

template <int NS, int NM>
struct k_reduce_final_body {
    static __device__ __forceinline__ void run(const double* part, int nb, double* out, double scale,
                                                   double* halt) {
        __shared__ double sh[4];
        for (int j = 0; j < NS + NM; ++j) {
            Neu acc;
            double mx = -INFINITY;
            for (int b = threadIdx.x; b < nb; b += kB) {
                const double v = part[(long)b * (NS + NM) + j];
                if (j < NS) acc.add(v);
                else mx = fmax(mx, v);
            }
            const double r = (j < NS) ? block_sum_256(acc.val(), sh) : block_max_256(mx, sh);
            if (threadIdx.x == 0) {
                out[j] = (j < NS) ? scale * r : r;
                if (halt && j < NS && !isfinite(r)) *halt = 1.0;
            }
        }
    }
};
template <int NS, int NM>
__global__ __launch_bounds__(kB) void k_reduce_final(const double* part, int nb, double* out, double scale,
                                                   double* halt) {
    k_reduce_final_body<NS, NM>::run(part, nb, out, scale, halt);
}

template <int NS, int NM, class F>
void run_reduce(const F& f, long n, double scale, double* part, double* out, hipStream_t s,
                double* halt = nullptr) {
    hipLaunchKernelGGL((k_reduce<NS, NM, F>), dim3(kRedBlocks), dim3(kB), 0, s, f, n, part);
    hipLaunchKernelGGL((k_reduce_final<NS, NM>), dim3(1), dim3(kB), 0, s, part, kRedBlocks, out, scale, halt);
}

struct AbsSumF {
    const double* x;
    __device__ void operator()(long i, double* s, double*) const { s[0] = fabs(x[i]); }
};

template <typename T> struct SumF {
    const T* x;
    __device__ void operator()(long i, double* s, double*) const { s[0] = (double)x[i]; }
};

__device__ __forceinline__ double gloc_d(double p) {
    const double a = p * p - p;
    return 18.0 * a * a;
}
__device__ __forceinline__ double W_d(double s) {
    const double a = s * s - s;
    return 18.0 * a * a;
}
__device__ __forceinline__ double Wp_d(double s) { return 36.0 * (s * s - s) * (2.0 * s - 1.0); }
__device__ __forceinline__ double f_d(double s) { return 3.0 * s * s - 2.0 * s * s * s; }

// 3 sums + 4 maxima
template <typename T> struct DiagF {
    const T* phi;
    const double* gfix;
    const T* u;
    double ubar;
    int fixed_model;
    __device__ void operator()(long i, double* s, double* m) const {
        const double uu = (double)u[i];
        double G, p = 0.0;
        if (phi) {
            p = (double)phi[i];
            G = gloc_d(p);
        } else {
            G = gfix[i];
        }
        s[0] = p;
        s[1] = fixed_model ? G * (f_d(uu) - ubar) : G * (uu - ubar);
        s[2] = G * uu;
        m[0] = -uu;
        m[1] = uu;
        m[2] = fabs(2.0 * uu - 1.0);
        m[3] = (isfinite(uu) && isfinite(p)) ? 0.0 : 1.0;
    }
};

struct Idx3 {
    long xp, yp, zp;
};
__device__ __forceinline__ Idx3 plus_neighbours(const GridK& g, long i) {
    const unsigned u = (unsigned)i;
    const unsigned t = u / (unsigned)g.nz;
    const int iz = (int)(u - t * (unsigned)g.nz);
    const unsigned ix_ = t / (unsigned)g.ny;
    const int iy = (int)(t - ix_ * (unsigned)g.ny);
    const int ix = (int)ix_;
    const long sx = (long)g.ny * g.nz, sy = g.nz;
    Idx3 r;
    r.xp = i + ((ix + 1 < g.nx) ? sx : -(long)(g.nx - 1) * sx);
    r.yp = i + ((iy + 1 < g.ny) ? sy : -(long)(g.ny - 1) * sy);
    r.zp = i + ((iz + 1 < g.nz) ? 1 : -(long)(g.nz - 1));
    return r;
}

// sum over the edges (i, i + e_d) of g_{i+1/2} (D+ u)^2, g from phi (coupled) or gfix
template <typename T, typename TG>
__device__ __forceinline__ double edge_energy(const GridK& g, long i, const T* u, const TG* G, bool from_phi) {
    const Idx3 nb = plus_neighbours(g, i);
    const double uc = (double)u[i];
    const double gc = from_phi ? gloc_d((double)G[i]) : (double)G[i];
    double e = 0.0;
    const long nbs[3] = {nb.xp, nb.yp, nb.zp};
    for (int d = 0; d < 3; ++d) {
        if (d == 0 && g.nx == 1) continue;
        const long j = nbs[d];
        const double gj = from_phi ? gloc_d((double)G[j]) : (double)G[j];
        if (!from_phi && (gc < 0.0 || gj < 0.0)) continue;   // a face leaving the band of a restricted step
        const double du = ((double)u[j] - uc) / g.h[d];
        e += 0.5 * (gc + gj) * du * du;
    }
    return e;
}

template <typename T> struct EnergyCoupledF {
    GridK g;
    double e2, ieps;
    const T *phi, *lap, *gx, *gy, *gz, *u, *psi, *q;
    __device__ void operator()(long i, double* s, double*) const {
        const double p = (double)phi[i];
        // gy == nullptr: gx holds |grad phi|
        const double a = (double)gx[i], b = gy ? (double)gy[i] : 0.0, c = gz ? (double)gz[i] : 0.0;
        s[0] = 0.5 * (a * a + b * b + c * c) + W_d(p) / e2;
        const double w = (double)lap[i] - Wp_d(p) / e2;
        s[1] = w * w;
        s[2] = p;
        s[3] = edge_energy(g, i, u, phi, true);
        s[4] = gloc_d(p) * W_d((double)u[i]);
        s[5] = (double)psi[i] * (double)q[i];
        s[6] = (double)q[i];
    }
};

struct EnergyFixedF {
    GridK g;
    double ubar;
    const double *G, *U, *psi, *q;
    __device__ void operator()(long i, double* s, double*) const {
        const double uu = U[i];
        s[0] = edge_energy(g, i, U, G, false);
        s[1] = G[i] >= 0.0 ? G[i] * W_d(uu) : 0.0;   // G < 0: off the band of a restricted step
        s[2] = psi[i] * q[i];
        s[3] = G[i] >= 0.0 ? G[i] * (f_d(uu) - ubar) : 0.0;
    }
};

template <typename T> struct MassF {
    const T *G, *U;
    double thr;
    __device__ void operator()(long i, double* s, double*) const {
        const double Gc = (double)G[i];
        s[0] = Gc * (double)U[i];
        s[1] = (Gc > thr) ? Gc : 0.0;
    }
};

template <typename T>
__global__ __launch_bounds__(kB) void k_mass_apply(long n, const T* __restrict__ G, T* U, double thr, double cell, const double* Q0,
                             const double* sums, const double* halt) {
    if (halted(halt)) return;
    const double den = cell * sums[1];
    const double c = den > 0.0 ? (Q0[0] - cell * sums[0]) / den : 0.0;
    for (long i = (long)blockIdx.x * kB + threadIdx.x; i < n; i += (long)gridDim.x * kB) {
        if ((double)G[i] > thr) U[i] = (T)((double)U[i] + c);
    }
}

// H row bound: H_ii + sum_{j != i} |H_ij| with H = -g^{-1/2} Delta_{S,h} g^{-1/2}:
// H_ii = isg_i^2 sum_d (g_{i+1/2} + g_{i-1/2}) / h_d^2, H_ij = -isg_i isg_j g_edge / h_d^2.
struct GershF {
    GridK g;
    const double *G, *isg;
    __device__ void operator()(long i, double*, double* m) const {
        const int iz = (int)(i % g.nz);
        const long t = i / g.nz;
        const int iy = (int)(t % g.ny);
        const int ix = (int)(t / g.ny);
        const long sx = (long)g.ny * g.nz, sy = g.nz;
        long nb[3][2];
        nb[0][1] = i + ((ix + 1 < g.nx) ? sx : -(long)(g.nx - 1) * sx);
        nb[0][0] = i + ((ix > 0) ? -sx : (long)(g.nx - 1) * sx);
        nb[1][1] = i + ((iy + 1 < g.ny) ? sy : -(long)(g.ny - 1) * sy);
        nb[1][0] = i + ((iy > 0) ? -sy : (long)(g.ny - 1) * sy);
        nb[2][1] = i + ((iz + 1 < g.nz) ? 1 : -(long)(g.nz - 1));
        nb[2][0] = i + ((iz > 0) ? -1 : (long)(g.nz - 1));
        const double gc = G[i], ic = isg[i];
        double diag = 0.0, off = 0.0;
        for (int d = 0; d < 3; ++d) {
            if (d == 0 && g.nx == 1) continue;
            const double ih2 = 1.0 / (g.h[d] * g.h[d]);
            for (int sgn = 0; sgn < 2; ++sgn) {
                const long j = nb[d][sgn];
                if (gc < 0.0 || G[j] < 0.0) continue;   // a face leaving the band of a restricted step
                const double ge = 0.5 * (gc + G[j]);
                diag += ic * ic * ge * ih2;
                off += ic * isg[j] * ge * ih2;
            }
        }
        m[0] = diag + off;
    }
};

}  // namespace

namespace {
__global__ void k_diag_ring_push(const double* __restrict__ diag, const double* halt, const int64_t* band_total,
                                 double* ring, int cap, int64_t* meta) {
    if (threadIdx.x != 0) return;
    const int64_t c = meta[0];
    double* e = ring + (long)(c % cap) * kDiagRingFields;
    e[0] = (double)(meta[1] + c + 1);
    e[1] = diag[0];
    e[2] = diag[1];
    e[3] = diag[2];
    e[4] = -diag[3];
    e[5] = diag[4];
    e[6] = diag[5];
    e[7] = band_total ? (double)band_total[0] : 0.0;
    e[8] = (diag[6] > 0.0 || (halt && halt[0] != 0.0)) ? 1.0 : 0.0;
    meta[0] = c + 1;
}
}  // namespace

void diag_ring_push(const double* diag, const double* halt, const int64_t* band_total, double* ring, int cap,
                    int64_t* meta, hipStream_t s) {
    hipLaunchKernelGGL(k_diag_ring_push, dim3(1), dim3(64), 0, s, diag, halt, band_total, ring, cap, meta);
}

void reduce_final_sum(const double* part, int nb, double scale, double* out, hipStream_t s, double* halt) {
    launch_k<k_reduce_final_body<1, 0>>(k_reduce_final<1, 0>, dim3(1), dim3(kB), 0, s, part, nb, out, scale, halt);
}

template <typename T>
void reduce_sum(long n, const T* x, double scale, double* part, double* out, hipStream_t s, double* halt) {
    run_reduce<1, 0>(SumF<T>{x}, n, scale, part, out, s, halt);
}

void reduce_abs_sum(long n, const double* x, double* part, double* out, hipStream_t s) {
    run_reduce<1, 0>(AbsSumF{x}, n, 1.0, part, out, s);
}

template <typename T>
void reduce_diag(const GridK& g, const T* phi, const double* gfix, const T* u, double ubar, bool fixed_model,
                 double* part, double* out, hipStream_t s) {
    run_reduce<3, 4>(DiagF<T>{phi, gfix, u, ubar, fixed_model ? 1 : 0}, g.nreal(), g.cell, part, out, s);
}

template <typename T>
void reduce_energy_coupled(const GridK& g, const CoupledK& K, const T* phi, const T* lap, const T* gx, const T* gy,
                           const T* gz, const T* u, const T* psi, const T* q, double* part, double* out,
                           hipStream_t s) {
    EnergyCoupledF<T> f{g, K.eps_phi * K.eps_phi, 1.0 / K.eps_u, phi, lap, gx, gy, gz, u, psi, q};
    run_reduce<7, 0>(f, g.nreal(), 1.0, part, out, s);
}

void reduce_energy_fixed(const GridK& g, const FixedK& K, const double* G, const double* U, const double* psi,
                         const double* q, double* part, double* out, hipStream_t s) {
    run_reduce<4, 0>(EnergyFixedF{g, K.ubar, G, U, psi, q}, g.nreal(), 1.0, part, out, s);
}

void fixed_gershgorin(const GridK& g, const double* G, const double* isg, double* part, double* out,
                      hipStream_t s) {
    run_reduce<0, 1>(GershF{g, G, isg}, g.nreal(), 1.0, part, out, s);
}

template <typename T>
void mass_project_sums(long n, const T* G, const T* U, double thr, double* part, double* out, hipStream_t s) {
    run_reduce<2, 0>(MassF<T>{G, U, thr}, n, 1.0, part, out, s);
}

template <typename T>
void mass_project_apply(long n, const T* G, T* U, double thr, double cell, const double* Q0, const double* sums,
                        const double* halt, hipStream_t s) {
    long b = (n + kB - 1) / kB;
    if (b > 8192) b = 8192;
    hipLaunchKernelGGL(k_mass_apply<T>, dim3((int)b), dim3(kB), 0, s, n, G, U, thr, cell, Q0, sums, halt);
}

#define INST(T)                                                                                                 \
    template void reduce_sum<T>(long, const T*, double, double*, double*, hipStream_t, double*);               \
    template void reduce_diag<T>(const GridK&, const T*, const double*, const T*, double, bool, double*,        \
                                 double*, hipStream_t);                                                         \
    template void reduce_energy_coupled<T>(const GridK&, const CoupledK&, const T*, const T*, const T*,         \
                                           const T*, const T*, const T*, const T*, const T*, double*, double*,  \
                                           hipStream_t);                                                        \
    template void mass_project_sums<T>(long, const T*, const T*, double, double*, double*, hipStream_t);       \
    template void mass_project_apply<T>(long, const T*, T*, double, double, const double*, const double*,      \
                                        const double*, hipStream_t);
INST(float)
INST(double)
#undef INST

}  // namespace etd
