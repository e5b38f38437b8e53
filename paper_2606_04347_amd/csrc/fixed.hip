// Fixed-membrane kernels (Section 2.2), FP64: the localization split
// L = B + eps_u H, H = -g^{-1/2} Delta_{S,h} g^{-1/2}, its Chebyshev recurrence,
// and the nonlinear remainder R_phi.
#include "kernels.h"

namespace etd {

namespace {

constexpr int kB = 256;

int grid_for(long n) {
    long b = (n + kB - 1) / kB;
    if (b > 8192) b = 8192;
    return (int)(b < 1 ? 1 : b);
}

__global__ __launch_bounds__(kB) void k_prep(long n, const double* __restrict__ G, double* __restrict__ sg, double* __restrict__ isg) {
    for (long i = (long)blockIdx.x * kB + threadIdx.x; i < n; i += (long)gridDim.x * kB) {
        const double s = sqrt(G[i]);
        sg[i] = s;
        isg[i] = 1.0 / s;
    }
}

__device__ __forceinline__ double f_ind(double s) { return 3.0 * s * s - 2.0 * s * s * s; }
__device__ __forceinline__ double fp_ind(double s) { return 6.0 * s * (1.0 - s); }
__device__ __forceinline__ double Wp(double s) { return 36.0 * (s * s - s) * (2.0 * s - 1.0); }

// gf (nullable): the band of a restricted step, g on it and -1 off it;
// off the band the nonlocal argument and the mass summand are 0
__global__ __launch_bounds__(kB) void k_nonlocal_arg(long n, FixedK K, const double* __restrict__ G, const double* __restrict__ U,
                               double* __restrict__ q, double* __restrict__ mq, const double* __restrict__ gf) {
    for (long i = (long)blockIdx.x * kB + threadIdx.x; i < n; i += (long)gridDim.x * kB) {
        if (gf && gf[i] < 0.0) {
            q[i] = 0.0;
            mq[i] = 0.0;
            continue;
        }
        const double f = f_ind(U[i]);
        const double gq = G[i] * (f - K.ubar);
        q[i] = K.with_ubar ? gq : G[i] * f;
        mq[i] = gq;
    }
}

// Off the band of a restricted step (gf[i] < 0) only the stabilizer term
// remains, formed as B (sqrt(g) U), the association of L w with w = sqrt(g) U,
// so that R - L w is exactly 0 there.
template <typename TP>
__global__ __launch_bounds__(kB) void k_remainder(long n, FixedK K, const double* __restrict__ sg, const double* __restrict__ U,
                            const TP* __restrict__ psi, const double* __restrict__ m, double* __restrict__ R,
                            const double* __restrict__ gf) {
    const double Mm = K.M * m[0];
    const double ieu = 1.0 / K.eps_u;
    for (long i = (long)blockIdx.x * kB + threadIdx.x; i < n; i += (long)gridDim.x * kB) {
        const double u = U[i], s = sg[i];
        if (gf && gf[i] < 0.0) {
            R[i] = K.B * (s * u);
            continue;
        }
        const double fp = fp_ind(u);
        R[i] = K.B * s * u - s * Wp(u) * ieu - K.gamma * s * (double)psi[i] * fp - Mm * s * fp;
    }
}

__global__ __launch_bounds__(kB) void k_band_field(long n, const double* __restrict__ G, double delta,
                                                   double* __restrict__ gf) {
    for (long i = (long)blockIdx.x * kB + threadIdx.x; i < n; i += (long)gridDim.x * kB)
        gf[i] = G[i] >= delta ? G[i] : -1.0;
}

// (H x)_i with H = -isg_i sum_d D^-(g_{i+1/2} D^+(isg x)).  G holds g, or for
// a restricted step g on the band and -1 off it: a face carries flux only
// when both of its nodes are on the band (g >= 0), so rows off the band are 0.
__device__ __forceinline__ double H_apply(const GridK& g, long i, const double* G, const double* isg,
                                          const double* x) {
    const unsigned u = (unsigned)i;
    const unsigned t = u / (unsigned)g.nz;
    const int iz = (int)(u - t * (unsigned)g.nz);
    const unsigned ix_ = t / (unsigned)g.ny;
    const int iy = (int)(t - ix_ * (unsigned)g.ny);
    const int ix = (int)ix_;
    const long sx = (long)g.ny * g.nz, sy = g.nz;
    const double gc = G[i];
    const double zc = isg[i] * x[i];
    double acc = 0.0;
    long m[3], p[3];
    p[0] = i + ((ix + 1 < g.nx) ? sx : -(long)(g.nx - 1) * sx);
    m[0] = i + ((ix > 0) ? -sx : (long)(g.nx - 1) * sx);
    p[1] = i + ((iy + 1 < g.ny) ? sy : -(long)(g.ny - 1) * sy);
    m[1] = i + ((iy > 0) ? -sy : (long)(g.ny - 1) * sy);
    p[2] = i + ((iz + 1 < g.nz) ? 1 : -(long)(g.nz - 1));
    m[2] = i + ((iz > 0) ? -1 : (long)(g.nz - 1));
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        if (d == 0 && g.nx == 1) continue;
        const double ih2 = 1.0 / (g.h[d] * g.h[d]);
        const double zp = isg[p[d]] * x[p[d]], zm = isg[m[d]] * x[m[d]];
        const double gp = G[p[d]], gm = G[m[d]];
        const double ghp = (gc >= 0.0 && gp >= 0.0) ? 0.5 * (gc + gp) : 0.0;
        const double ghm = (gc >= 0.0 && gm >= 0.0) ? 0.5 * (gm + gc) : 0.0;
        acc += (ghp * (zp - zc) - ghm * (zc - zm)) * ih2;
    }
    return -isg[i] * acc;
}

__global__ __launch_bounds__(kB) void k_cheb(GridK g, FixedK K, const double* __restrict__ G, const double* __restrict__ isg, double a,
                       double b, double alpha, double beta, const double* __restrict__ x, const double* xprev,
                       double* y, double* acc, double c, double c0, int first) {
    const long n = g.nreal();
    const double s2 = 2.0 / (b - a), sh = (b + a) / (b - a);
    // workgroups renumbered so each XCD walks a contiguous range of rows: the
    // y and x neighbours of a point are then mostly read through the same L2
    for (long i = (long)xcd_remap(blockIdx.x, gridDim.x) * kB + threadIdx.x; i < n; i += (long)gridDim.x * kB) {
        const double xi = x[i];
        const double Lx = K.B * xi + K.eps_u * H_apply(g, i, G, isg, x);
        double yi = alpha * (s2 * Lx - sh * xi);
        if (beta != 0.0) yi -= beta * xprev[i];
        y[i] = yi;
        acc[i] = first ? (c0 * xi + c * yi) : (acc[i] + c * yi);
    }
}

__global__ __launch_bounds__(kB) void k_L(GridK g, FixedK K, const double* __restrict__ G, const double* __restrict__ isg,
                    const double* __restrict__ x, double* __restrict__ out) {
    const long n = g.nreal();
    for (long i = (long)xcd_remap(blockIdx.x, gridDim.x) * kB + threadIdx.x; i < n; i += (long)gridDim.x * kB)
        out[i] = K.B * x[i] + K.eps_u * H_apply(g, i, G, isg, x);
}

__global__ __launch_bounds__(kB) void k_axpby(long n, double a, const double* x, double b, const double* y, double* out) {
    for (long i = (long)blockIdx.x * kB + threadIdx.x; i < n; i += (long)gridDim.x * kB) out[i] = a * x[i] + b * y[i];
}

__global__ __launch_bounds__(kB) void k_mul(long n, const double* x, const double* y, double* out,
                                          const double* halt, const double* gf) {
    if (halted(halt)) return;
    for (long i = (long)blockIdx.x * kB + threadIdx.x; i < n; i += (long)gridDim.x * kB)
        if (!gf || gf[i] >= 0.0) out[i] = x[i] * y[i];
}

}  // namespace

void fixed_prep(const GridK& g, const double* G, double* sg, double* isg, hipStream_t s) {
    hipLaunchKernelGGL(k_prep, dim3(grid_for(g.nreal())), dim3(kB), 0, s, g.nreal(), G, sg, isg);
}
void fixed_nonlocal_arg(long n, const FixedK& K, const double* G, const double* U, double* q, double* mq,
                        const double* gf, hipStream_t s) {
    hipLaunchKernelGGL(k_nonlocal_arg, dim3(grid_for(n)), dim3(kB), 0, s, n, K, G, U, q, mq, gf);
}
template <typename TP>
void fixed_remainder(long n, const FixedK& K, const double* sg, const double* U, const TP* psi, const double* m,
                     double* R, const double* gf, hipStream_t s) {
    hipLaunchKernelGGL(k_remainder<TP>, dim3(grid_for(n)), dim3(kB), 0, s, n, K, sg, U, psi, m, R, gf);
}
template void fixed_remainder<double>(long, const FixedK&, const double*, const double*, const double*,
                                      const double*, double*, const double*, hipStream_t);
template void fixed_remainder<float>(long, const FixedK&, const double*, const double*, const float*,
                                     const double*, double*, const double*, hipStream_t);
void fixed_band_field(long n, const double* G, double delta, double* gf, hipStream_t s) {
    hipLaunchKernelGGL(k_band_field, dim3(grid_for(n)), dim3(kB), 0, s, n, G, delta, gf);
}
void fixed_cheb_step(const GridK& g, const FixedK& K, const double* G, const double* isg, double a, double b,
                     double alpha, double beta, const double* x, const double* xprev, double* y, double* acc,
                     double c, double c0, int first, hipStream_t s) {
    hipLaunchKernelGGL(k_cheb, dim3(grid_for(g.nreal())), dim3(kB), 0, s, g, K, G, isg, a, b, alpha, beta, x, xprev,
                       y, acc, c, c0, first);
}
void fixed_L_apply(const GridK& g, const FixedK& K, const double* G, const double* isg, const double* x,
                   double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_L, dim3(grid_for(g.nreal())), dim3(kB), 0, s, g, K, G, isg, x, out);
}
void axpby(long n, double a, const double* x, double b, const double* y, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_axpby, dim3(grid_for(n)), dim3(kB), 0, s, n, a, x, b, y, out);
}
void mul(long n, const double* x, const double* y, double* out, hipStream_t s, const double* halt,
         const double* gf) {
    hipLaunchKernelGGL(k_mul, dim3(grid_for(n)), dim3(kB), 0, s, n, x, y, out, halt, gf);
}

}  // namespace etd
