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
                            const double* __restrict__ gf, const double* __restrict__ Rprev) {
    const double Mm = K.M * m[0];
    const double ieu = 1.0 / K.eps_u;
    for (long i = (long)blockIdx.x * kB + threadIdx.x; i < n; i += (long)gridDim.x * kB) {
        const double u = U[i], s = sg[i];
        double r;
        if (gf && gf[i] < 0.0) {
            r = K.B * (s * u);
        } else {
            const double fp = fp_ind(u);
            r = K.B * s * u - s * Wp(u) * ieu - K.gamma * s * (double)psi[i] * fp - Mm * s * fp;
        }
        R[i] = Rprev ? r - Rprev[i] : r;
    }
}

__global__ __launch_bounds__(kB) void k_band_field(long n, const double* __restrict__ G, double delta,
                                                   double* __restrict__ gf) {
    for (long i = (long)blockIdx.x * kB + threadIdx.x; i < n; i += (long)gridDim.x * kB)
        gf[i] = G[i] >= delta ? G[i] : -1.0;
}

// One axis of the flux sum of H (z = isg x): the faces to the + and -
// neighbours.  G holds g, or for a restricted step g on the band and -1 off
// it: a face carries flux only when both of its nodes are on the band (g >= 0),
// so rows off the band are 0.
__device__ __forceinline__ double h_axis(double gc, double zc, double gp, double zp, double gm, double zm,
                                         double ih2) {
    const double ghp = (gc >= 0.0 && gp >= 0.0) ? 0.5 * (gc + gp) : 0.0;
    const double ghm = (gc >= 0.0 && gm >= 0.0) ? 0.5 * (gm + gc) : 0.0;
    return (ghp * (zp - zc) - ghm * (zc - zm)) * ih2;
}

// One Chebyshev term at a node: y = alpha (s2 L x - sh x) - beta xprev with
// L x = B x + eps_u H x and (H x)_i = -isg_i * flux (flux: the axis sums).
__device__ __forceinline__ double cheb_y(const FixedK& K, double xi, double isgi, double flux, double alpha,
                                         double s2, double sh, double beta, double xprev) {
    const double Lx = K.B * xi + K.eps_u * (-isgi * flux);
    double yi = alpha * (s2 * Lx - sh * xi);
    if (beta != 0.0) yi -= beta * xprev;
    return yi;
}

// Flux sum of (H x)_i = -isg_i sum_d D^-(g_{i+1/2} D^+(isg x)).
__device__ __forceinline__ double H_flux(const GridK& g, long i, const double* G, const double* isg,
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
        acc += h_axis(gc, zc, G[p[d]], isg[p[d]] * x[p[d]], G[m[d]], isg[m[d]] * x[m[d]], ih2);
    }
    return acc;
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
        const double yi = cheb_y(K, xi, isg[i], H_flux(g, i, G, isg, x), alpha, s2, sh, beta,
                                 beta != 0.0 ? xprev[i] : 0.0);
        y[i] = yi;
        acc[i] = first ? (c0 * xi + c * yi) : (acc[i] + c * yi);
    }
}

// Two consecutive terms of the recurrence in one pass over the grid (3D):
//   y1 = alpha (s2 L x - sh x) - beta xprev,   y2 = alpha (s2 L y1 - sh y1) - beta x,
//   acc += c1 y1, then acc += c2 y2,
// each node's arithmetic exactly as one term of k_cheb takes it.  A workgroup
// owns a tile of kPY x kPZ nodes in (y, z) (one thread per node) and kPX
// consecutive x planes, and
// walks along x with rolling LDS planes: z = isg x and G over the tile with a
// two-node halo, z1 = isg y1 over the tile with a one-node halo (y1 is formed
// there too, so a tile needs no y1 of its neighbours).  Per node one pass
// reads x, xprev, acc, G and isg and writes y1, y2 and acc, instead of two
// passes that read five fields and write two each.  The global reads of the
// next plane are issued before the current plane is worked on, and the
// barriers order LDS only, so those reads stay in flight across them.
constexpr int kPY = 16, kPZ = 32, kPX = 8;
constexpr int kH2Y = kPY + 4, kH2Z = kPZ + 4, kH2 = kH2Y * kH2Z;   // tile + 2-node halo
constexpr int kH1Y = kPY + 2, kH1Z = kPZ + 2, kH1 = kH1Y * kH1Z;   // tile + 1-node halo
constexpr int kBP = 512;   // threads of a workgroup: one per node of the tile
constexpr int kSlots2 = (kH2 + kBP - 1) / kBP;
constexpr int kSlots1 = (kH1 + kBP - 1) / kBP;

// v mod n in [0, n) (tiles wider than the grid wrap more than once)
__device__ __forceinline__ int wrap(int v, int n) {
    const int r = v % n;
    return r < 0 ? r + n : r;
}

// Workgroup barrier for LDS traffic alone: global loads in flight are not
// waited for (no thread reads another's global writes within the pass).
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

__global__ __launch_bounds__(kBP) void k_cheb_pair(GridK g, FixedK K, const double* __restrict__ G,
                                                  const double* __restrict__ isg, double a, double b, double alpha,
                                                  double beta, const double* __restrict__ x,
                                                  const double* __restrict__ xprev, double* __restrict__ y1out,
                                                  double* __restrict__ y2out, double* __restrict__ acc, double c1,
                                                  double c2) {
    __shared__ double zb[3][kH2];    // isg x on planes p mod 3
    __shared__ double gb[4][kH2];    // G on planes p mod 4
    __shared__ double z1b[3][kH1];   // isg y1 on planes q mod 3
    const int nty = (g.ny + kPY - 1) / kPY, ntz = (g.nz + kPZ - 1) / kPZ;
    const int t = xcd_remap(blockIdx.x, gridDim.x);
    const int tz = t % ntz, ty = (t / ntz) % nty, seg = t / (ntz * nty);
    const int y0 = ty * kPY, z0 = tz * kPZ, xs = seg * kPX, xe = min(xs + kPX, g.nx);
    const long sx = (long)g.ny * g.nz;
    const double s2 = 2.0 / (b - a), sh = (b + a) / (b - a);
    const double ihx = 1.0 / (g.h[0] * g.h[0]), ihy = 1.0 / (g.h[1] * g.h[1]), ihz = 1.0 / (g.h[2] * g.h[2]);
    auto plane = [&](int p) { return (long)wrap(p, g.nx) * sx; };
    // this thread's nodes of the two-halo region (plane offsets)
    long off2[kSlots2];
#pragma unroll
    for (int k = 0; k < kSlots2; ++k) {
        const int j = threadIdx.x + k * kBP;
        const int jy = j / kH2Z, jz = j - jy * kH2Z;
        off2[k] = (long)wrap(y0 - 2 + jy, g.ny) * g.nz + wrap(z0 - 2 + jz, g.nz);
    }
    // ... of the one-halo region: plane offset, index into the two-halo plane,
    // and whether the tile owns the node
    long off1[kSlots1];
    int c2i[kSlots1];
    bool own[kSlots1];
    double y1keep[kSlots1], y1now[kSlots1];
#pragma unroll
    for (int k = 0; k < kSlots1; ++k) {
        const int j = threadIdx.x + k * kBP;
        const int jy = j / kH1Z, jz = j - jy * kH1Z;
        const int yy = y0 - 1 + jy, zz = z0 - 1 + jz;
        off1[k] = (long)wrap(yy, g.ny) * g.nz + wrap(zz, g.nz);
        c2i[k] = (jy + 1) * kH2Z + (jz + 1);
        own[k] = j < kH1 && jy >= 1 && jy <= kPY && jz >= 1 && jz <= kPZ && yy < g.ny && zz < g.nz;
        y1keep[k] = 0.0;
        y1now[k] = 0.0;
    }
    // register stages of the global reads: x, isg, G of the plane to load;
    // x, isg, xprev of the next y1 plane; x, isg, acc of the next y2 plane
    double lx[kSlots2], li[kSlots2], lg[kSlots2];
    double ax[kSlots1], ai[kSlots1], ap[kSlots1];
    double bx[kSlots1], bi[kSlots1], ba[kSlots1];
    auto fetch_plane = [&](int p) {
        const long base = plane(p);
#pragma unroll
        for (int k = 0; k < kSlots2; ++k) {
            if (threadIdx.x + k * kBP >= kH2) continue;
            const long i = base + off2[k];
            lx[k] = x[i];
            li[k] = isg[i];
            lg[k] = G[i];
        }
    };
    auto fetch_y1 = [&](int q, int k) {
        const long i = plane(q) + off1[k];
        ax[k] = x[i];
        ai[k] = isg[i];
        ap[k] = xprev[i];
    };
    auto fetch_y2 = [&](int r, int k) {
        const long i = plane(r) + off1[k];
        bx[k] = x[i];
        bi[k] = isg[i];
        ba[k] = acc[i];
    };
    fetch_plane(xs - 2);
#pragma unroll
    for (int k = 0; k < kSlots1; ++k) {
        if (threadIdx.x + k * kBP < kH1) fetch_y1(xs - 1, k);
        if (own[k]) fetch_y2(xs, k);
    }
    for (int p = xs - 2; p <= xe + 1; ++p) {
        {   // plane p of isg x and G over the two-halo region, then the reads of plane p + 1
            double* zp = zb[(p + 3) % 3];
            double* gp = gb[(p + 4) % 4];
#pragma unroll
            for (int k = 0; k < kSlots2; ++k) {
                const int j = threadIdx.x + k * kBP;
                if (j >= kH2) continue;
                zp[j] = li[k] * lx[k];
                gp[j] = lg[k];
            }
            if (p + 1 <= xe + 1) fetch_plane(p + 1);
        }
        lds_barrier();
        const int q = p - 1;   // y1 on plane q (one-halo region)
        if (q >= xs - 1) {
            const double* zm = zb[(q - 1 + 3) % 3];
            const double* zc = zb[(q + 3) % 3];
            const double* zpl = zb[(q + 1 + 3) % 3];
            const double* gm = gb[(q - 1 + 4) % 4];
            const double* gc = gb[(q + 4) % 4];
            const double* gpl = gb[(q + 1 + 4) % 4];
            double* z1 = z1b[(q + 3) % 3];
            const long base = plane(q);
#pragma unroll
            for (int k = 0; k < kSlots1; ++k) {
                const int j = threadIdx.x + k * kBP;
                if (j >= kH1) continue;
                const int c = c2i[k];
                const double gci = gc[c], zci = zc[c];
                double flux = 0.0;
                flux += h_axis(gci, zci, gpl[c], zpl[c], gm[c], zm[c], ihx);
                flux += h_axis(gci, zci, gc[c + kH2Z], zc[c + kH2Z], gc[c - kH2Z], zc[c - kH2Z], ihy);
                flux += h_axis(gci, zci, gc[c + 1], zc[c + 1], gc[c - 1], zc[c - 1], ihz);
                const double v = cheb_y(K, ax[k], ai[k], flux, alpha, s2, sh, beta, ap[k]);
                z1[j] = ai[k] * v;
                y1now[k] = v;
                if (own[k] && q >= xs && q < xe) y1out[base + off1[k]] = v;
                if (q + 1 <= xe) fetch_y1(q + 1, k);
            }
        }
        lds_barrier();
        const int r = p - 2;   // y2 and acc on plane r (the tile)
        if (r >= xs) {
            const double* zm = z1b[(r - 1 + 3) % 3];
            const double* zc = z1b[(r + 3) % 3];
            const double* zpl = z1b[(r + 1 + 3) % 3];
            const double* gm = gb[(r - 1 + 4) % 4];
            const double* gc = gb[(r + 4) % 4];
            const double* gpl = gb[(r + 1 + 4) % 4];
            const long base = plane(r);
#pragma unroll
            for (int k = 0; k < kSlots1; ++k) {
                if (!own[k]) continue;
                const int j = threadIdx.x + k * kBP;
                const int c = c2i[k];
                const long i = base + off1[k];
                const double gci = gc[c], zci = zc[j];
                double flux = 0.0;
                flux += h_axis(gci, zci, gpl[c], zpl[j], gm[c], zm[j], ihx);
                flux += h_axis(gci, zci, gc[c + kH2Z], zc[j + kH1Z], gc[c - kH2Z], zc[j - kH1Z], ihy);
                flux += h_axis(gci, zci, gc[c + 1], zc[j + 1], gc[c - 1], zc[j - 1], ihz);
                const double v1 = y1keep[k];
                const double v2 = cheb_y(K, v1, bi[k], flux, alpha, s2, sh, beta, bx[k]);
                y2out[i] = v2;
                double s_ = ba[k] + c1 * v1;
                s_ = s_ + c2 * v2;
                acc[i] = s_;
                if (r + 1 < xe) fetch_y2(r + 1, k);
            }
        }
#pragma unroll
        for (int k = 0; k < kSlots1; ++k) y1keep[k] = y1now[k];
        lds_barrier();
    }
}

__global__ __launch_bounds__(kB) void k_L(GridK g, FixedK K, const double* __restrict__ G, const double* __restrict__ isg,
                    const double* __restrict__ x, const double* __restrict__ r, double* __restrict__ out) {
    const long n = g.nreal();
    for (long i = (long)xcd_remap(blockIdx.x, gridDim.x) * kB + threadIdx.x; i < n; i += (long)gridDim.x * kB) {
        const double Lx = K.B * x[i] + K.eps_u * (-isg[i] * H_flux(g, i, G, isg, x));
        out[i] = r ? r[i] - Lx : Lx;
    }
}

// w = w + tau acc, then U = isg w (where gf >= 0, when gf is given); once the
// instance is halted neither is written
__global__ __launch_bounds__(kB) void k_advance(long n, double tau, const double* __restrict__ acc,
                                                double* __restrict__ w, const double* __restrict__ isg,
                                                double* __restrict__ U, const double* halt,
                                                const double* __restrict__ gf) {
    if (halted(halt)) return;
    for (long i = (long)blockIdx.x * kB + threadIdx.x; i < n; i += (long)gridDim.x * kB) {
        const double wn = w[i] + tau * acc[i];
        w[i] = wn;
        if (!gf || gf[i] >= 0.0) U[i] = isg[i] * wn;
    }
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
                     double* R, const double* gf, hipStream_t s, const double* Rprev) {
    hipLaunchKernelGGL(k_remainder<TP>, dim3(grid_for(n)), dim3(kB), 0, s, n, K, sg, U, psi, m, R, gf, Rprev);
}
template void fixed_remainder<double>(long, const FixedK&, const double*, const double*, const double*,
                                      const double*, double*, const double*, hipStream_t, const double*);
template void fixed_remainder<float>(long, const FixedK&, const double*, const double*, const float*,
                                     const double*, double*, const double*, hipStream_t, const double*);
void fixed_band_field(long n, const double* G, double delta, double* gf, hipStream_t s) {
    hipLaunchKernelGGL(k_band_field, dim3(grid_for(n)), dim3(kB), 0, s, n, G, delta, gf);
}
void fixed_cheb_step(const GridK& g, const FixedK& K, const double* G, const double* isg, double a, double b,
                     double alpha, double beta, const double* x, const double* xprev, double* y, double* acc,
                     double c, double c0, int first, hipStream_t s) {
    hipLaunchKernelGGL(k_cheb, dim3(grid_for(g.nreal())), dim3(kB), 0, s, g, K, G, isg, a, b, alpha, beta, x, xprev,
                       y, acc, c, c0, first);
}
bool fixed_cheb_pair_supported(const GridK& g) { return g.nx > 1; }
void fixed_cheb_pair(const GridK& g, const FixedK& K, const double* G, const double* isg, double a, double b,
                     double alpha, double beta, const double* x, const double* xprev, double* y1, double* y2,
                     double* acc, double c1, double c2, hipStream_t s) {
    const int nb = ((g.nx + kPX - 1) / kPX) * ((g.ny + kPY - 1) / kPY) * ((g.nz + kPZ - 1) / kPZ);
    hipLaunchKernelGGL(k_cheb_pair, dim3(nb), dim3(kBP), 0, s, g, K, G, isg, a, b, alpha, beta, x, xprev, y1, y2, acc,
                       c1, c2);
}
void fixed_L_apply(const GridK& g, const FixedK& K, const double* G, const double* isg, const double* x,
                   double* out, hipStream_t s, const double* r) {
    hipLaunchKernelGGL(k_L, dim3(grid_for(g.nreal())), dim3(kB), 0, s, g, K, G, isg, x, r, out);
}
void fixed_advance(long n, double tau, const double* acc, double* w, const double* isg, double* U,
                   const double* halt, const double* gf, hipStream_t s) {
    hipLaunchKernelGGL(k_advance, dim3(grid_for(n)), dim3(kB), 0, s, n, tau, acc, w, isg, U, halt, gf);
}
void mul(long n, const double* x, const double* y, double* out, hipStream_t s, const double* halt,
         const double* gf) {
    hipLaunchKernelGGL(k_mul, dim3(grid_for(n)), dim3(kB), 0, s, n, x, y, out, halt, gf);
}

}  // namespace etd
