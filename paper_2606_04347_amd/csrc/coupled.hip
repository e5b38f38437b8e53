// Coupled-model kernels: spectral multipliers and ETD combines (Section 3.2,
// Section 3.3) and the real-space remainders R1, R2 (Section 3.1) with the
// second-order FD operators of Section 2.1.
#include "blocksum.h"
#include "etd_point.h"
#include "remainders.h"

namespace etd {

namespace {

constexpr int kBlock = 256;

// wavenumbers of half-spectrum entry idx (layout [nx][ny][nzh])
struct Wave {
    double k2;      // sum_d lambda_d^2
    double kd[3];   // first-derivative wavenumbers (Nyquist zeroed)
    double mu;      // FD symbol sum_d (4/h_d^2) sin^2(pi i_d / N_d)
};

__device__ __forceinline__ Wave wave(const GridK& g, long idx, const double* fd) {
    // the half spectrum has fewer than 2^32 entries: 32-bit decode (64-bit
    // division is a long software sequence on the GPU)
    const unsigned u = (unsigned)idx;
    const unsigned t = u / (unsigned)g.nzh;
    const int iz = (int)(u - t * (unsigned)g.nzh);
    const unsigned ix_ = t / (unsigned)g.ny;
    const int iy = (int)(t - ix_ * (unsigned)g.ny);
    const int ix = (int)ix_;
    const double ax = kPi / g.X[0], ay = kPi / g.X[1], az = kPi / g.X[2];
    const double lx = ax * lam_index(ix, g.nx), ly = ay * lam_index(iy, g.ny), lz = az * iz;
    Wave w;
    w.k2 = lx * lx + ly * ly + lz * lz;
    w.kd[0] = ax * der_index(ix, g.nx);
    w.kd[1] = ay * der_index(iy, g.ny);
    w.kd[2] = az * der_index(iz, g.nz);
    // FD symbol from the per-axis tables fd = [4/h_x^2 sin^2(pi i/N_x) | ... y | ... z]
    w.mu = fd ? fd[ix] + fd[g.nx + iy] + fd[g.nx + g.ny + iz] : 0.0;
    return w;
}


template <typename T>
__global__ __launch_bounds__(kBlock) void k_spec_apply(GridK g, int op, const c2<T>* in, c2<T>* out, const double* __restrict__ fd) {
    const long n = g.nspec();
    for (long i = (long)blockIdx.x * kBlock + threadIdx.x; i < n; i += (long)gridDim.x * kBlock) {
        const Wave w = wave(g, i, op == SPEC_INV_FD ? fd : nullptr);
        const c2<T> a = in[i];
        c2<T> r;
        if (op == SPEC_NEG_K2) {
            const T m = (T)(-w.k2);
            r = mk<T>(m * a.x, m * a.y);
        } else if (op == SPEC_INV_FD) {
            const T m = (T)(w.mu > 0.0 ? 1.0 / w.mu : 0.0);
            r = mk<T>(m * a.x, m * a.y);
        } else {
            const T k = (T)(op == SPEC_IKX ? w.kd[0] : (op == SPEC_IKY ? w.kd[1] : w.kd[2]));   // i k a = (-k a.y, k a.x)
            r = mk<T>(-k * a.y, k * a.x);
        }
        out[i] = r;
    }
}

// One ETD combine (etd_point.h) per half-spectrum entry: p = P[i], q = Q[i].
template <int ST, typename T>
__global__ __launch_bounds__(kBlock) void k_etd(GridK g, CoupledK K, const c2<T>* __restrict__ P, const c2<T>* __restrict__ Q, EtdArgs<T> a) {
    if (halted(a.halt)) return;
    const long n = g.nspec();
    for (long i = (long)blockIdx.x * kBlock + threadIdx.x; i < n; i += (long)gridDim.x * kBlock) {
        const Wave w = wave(g, i, nullptr);
        a.out[i] = etd_combine<ST, T>(K, w.k2, i, P[i], Q[i], a);
    }
}

// ----------------------------------------------------------------- real space
// The stencil kernels give each thread four consecutive z points (every
// supported Nz is a multiple of 4): one vector load per field and neighbour
// row serves four points, and the index decode is paid once per quad.
template <typename T> struct Q4 {
    T v[4];
};
template <typename T> __device__ __forceinline__ Q4<T> ld4(const T* p) {
    Q4<T> r;
    if constexpr (sizeof(T) == 4) {
        const float4 a = *reinterpret_cast<const float4*>(p);
        r.v[0] = a.x;
        r.v[1] = a.y;
        r.v[2] = a.z;
        r.v[3] = a.w;
    } else {
        const double2 a = reinterpret_cast<const double2*>(p)[0], b = reinterpret_cast<const double2*>(p)[1];
        r.v[0] = a.x;
        r.v[1] = a.y;
        r.v[2] = b.x;
        r.v[3] = b.y;
    }
    return r;
}
template <typename T> __device__ __forceinline__ void st4(T* p, const Q4<T>& r) {
    if constexpr (sizeof(T) == 4) {
        *reinterpret_cast<float4*>(p) = make_float4(r.v[0], r.v[1], r.v[2], r.v[3]);
    } else {
        reinterpret_cast<double2*>(p)[0] = make_double2(r.v[0], r.v[1]);
        reinterpret_cast<double2*>(p)[1] = make_double2(r.v[2], r.v[3]);
    }
}

// Quad q (points 4q .. 4q+3, one z row): its first point c, the first points
// of the x and y neighbour quads, and the z neighbours before and after it
// (all periodic).
struct QuadNbr {
    long c, xm, xp, ym, yp, zm, zp;
};
__device__ __forceinline__ QuadNbr quad_neighbours(const GridK& g, long q) {
    const unsigned nz4 = (unsigned)g.nz >> 2;
    const unsigned uq = (unsigned)q;   // grids hold fewer than 2^31 points
    const unsigned row = uq / nz4;
    const int iz = (int)(uq - row * nz4) * 4;
    const unsigned ix_ = row / (unsigned)g.ny;
    const int iy = (int)(row - ix_ * (unsigned)g.ny);
    const int ix = (int)ix_;
    const long sx = (long)g.ny * g.nz, sy = g.nz, r0 = (long)row * g.nz;
    QuadNbr n;
    n.c = r0 + iz;
    n.xp = n.c + ((ix + 1 < g.nx) ? sx : -(long)(g.nx - 1) * sx);
    n.xm = n.c + ((ix > 0) ? -sx : (long)(g.nx - 1) * sx);
    n.yp = n.c + ((iy + 1 < g.ny) ? sy : -(long)(g.ny - 1) * sy);
    n.ym = n.c + ((iy > 0) ? -sy : (long)(g.ny - 1) * sy);
    n.zm = r0 + (iz > 0 ? iz - 1 : g.nz - 1);
    n.zp = r0 + (iz + 4 < g.nz ? iz + 4 : 0);
    return n;
}

// mask bytes of a quad (4-byte aligned: the quad's first point is a multiple of 4)
__device__ __forceinline__ unsigned ld_mask4(const uint8_t* mask, long c) {
    return *reinterpret_cast<const unsigned*>(mask + c);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_R1_point(GridK g, CoupledK K, const T* __restrict__ phi,
                                                     const T* __restrict__ lap, const T* __restrict__ gx,
                                                     const T* __restrict__ gy, const T* __restrict__ gz,
                                                     const T* __restrict__ u, const uint8_t* __restrict__ mask,
                                                     const double* __restrict__ int_phi, double A0,
                                                     T* __restrict__ P, T* __restrict__ Q, int tpb) {
    const long nq = g.nreal() / 4;
    const R1Const<T> kc(g, K, int_phi[0], A0);
    // a block takes tpb consecutive tiles of kBlock quads, blocks in XCD-contiguous
    // order, so that the y and x neighbour rows of a tile are read through the same L2
    const long t0 = (long)xcd_remap(blockIdx.x, gridDim.x) * tpb;
    for (int it = 0; it < tpb; ++it) {
        const long q = (t0 + it) * kBlock + threadIdx.x;
        if (q >= nq) return;
        const QuadNbr nb = quad_neighbours(g, q);
        const Q4<T> p = ld4(phi + nb.c), L = ld4(lap + nb.c), a = ld4(gx + nb.c), b = ld4(gy + nb.c),
                    c = ld4(gz + nb.c), uu = ld4(u + nb.c);
        const Q4<T> pxm = ld4(phi + nb.xm), pxp = ld4(phi + nb.xp), pym = ld4(phi + nb.ym), pyp = ld4(phi + nb.yp);
        const Q4<T> uxm = ld4(u + nb.xm), uxp = ld4(u + nb.xp), uym = ld4(u + nb.ym), uyp = ld4(u + nb.yp);
        const T pzm = phi[nb.zm], pzp = phi[nb.zp], uzm = u[nb.zm], uzp = u[nb.zp];
        const unsigned mk = mask ? ld_mask4(mask, nb.c) : 0xffffffffu;
        Q4<T> oP, oQ;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const T un[6] = {uxm.v[k], uxp.v[k], uym.v[k], uyp.v[k], k > 0 ? uu.v[k - 1] : uzm,
                             k < 3 ? uu.v[k + 1] : uzp};
            const T pn[6] = {pxm.v[k], pxp.v[k], pym.v[k], pyp.v[k], k > 0 ? p.v[k - 1] : pzm,
                             k < 3 ? p.v[k + 1] : pzp};
            const T gn = sqrt(a.v[k] * a.v[k] + b.v[k] * b.v[k] + c.v[k] * c.v[k]);
            r1_point(kc, p.v[k], L.v[k], gn, uu.v[k], un, pn, ((mk >> (8 * k)) & 0xffu) != 0,
                     &oP.v[k], &oQ.v[k]);
        }
        st4(P + nb.c, oP);
        st4(Q + nb.c, oQ);
    }
}

// Neighbour indices of grid point i on a periodic 3D grid (x-, x+, y-, y+, z-, z+).
struct PointNbr {
    long xm, xp, ym, yp, zm, zp;
};
__device__ __forceinline__ PointNbr point_neighbours(const GridK& g, long i) {
    const long nyz = (long)g.ny * g.nz;
    const int ix = (int)(i / nyz);
    const long r = i - (long)ix * nyz;
    const int iy = (int)(r / g.nz), iz = (int)(r - (long)iy * g.nz);
    PointNbr n;
    n.xm = i + (ix > 0 ? -nyz : (long)(g.nx - 1) * nyz);
    n.xp = i + (ix + 1 < g.nx ? nyz : -(long)(g.nx - 1) * nyz);
    n.ym = i + (iy > 0 ? -(long)g.nz : (long)(g.ny - 1) * g.nz);
    n.yp = i + (iy + 1 < g.ny ? (long)g.nz : -(long)(g.ny - 1) * g.nz);
    n.zm = i + (iz > 0 ? -1 : g.nz - 1);
    n.zp = i + (iz + 1 < g.nz ? 1 : -(g.nz - 1));
    return n;
}

// The surface part of P1 (r1_surf) at every point of the band list.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_r1_surf_band(GridK g, CoupledK K, const T* __restrict__ phi,
                                                         const T* __restrict__ lap, const T* __restrict__ gn,
                                                         const T* __restrict__ u, const int32_t* __restrict__ idx,
                                                         const int64_t* __restrict__ total,
                                                         const double* __restrict__ int_phi, double A0,
                                                         T* __restrict__ surf) {
    const long nb = total[0];
    const R1Const<T> kc(g, K, int_phi[0], A0);
    for (long b = (long)blockIdx.x * kBlock + threadIdx.x; b < nb; b += (long)gridDim.x * kBlock) {
        const long i = idx[b];
        const PointNbr n = point_neighbours(g, i);
        const T un[6] = {u[n.xm], u[n.xp], u[n.ym], u[n.yp], u[n.zm], u[n.zp]};
        const T pn[6] = {phi[n.xm], phi[n.xp], phi[n.ym], phi[n.yp], phi[n.zm], phi[n.zp]};
        surf[i] = r1_surf(kc, phi[i], lap[i], gn[i], u[i], un, pn);
    }
}

// P2 without its nonlocal term (p2_local) at every point of the band list.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_p2_local_band(GridK g, CoupledK K, const T* __restrict__ u,
                                                          const T* __restrict__ G, const T* __restrict__ vx,
                                                          const T* __restrict__ vy, const T* __restrict__ vz,
                                                          const int32_t* __restrict__ idx,
                                                          const int64_t* __restrict__ total,
                                                          const double* __restrict__ m, T* __restrict__ surf) {
    const long nb = total[0];
    const P2Const<T> kc(g, K, m[0]);
    for (long b = (long)blockIdx.x * kBlock + threadIdx.x; b < nb; b += (long)gridDim.x * kBlock) {
        const long i = idx[b];
        const PointNbr n = point_neighbours(g, i);
        const T un[6] = {u[n.xm], u[n.xp], u[n.ym], u[n.yp], u[n.zm], u[n.zp]};
        const T Gn[6] = {G[n.xm], G[n.xp], G[n.ym], G[n.yp], G[n.zm], G[n.zp]};
        const T vn[6] = {vx[n.xm], vx[n.xp], vy[n.ym], vy[n.yp], vz[n.zm], vz[n.zp]};
        surf[i] = p2_local(kc, u[i], G[i], un, Gn, vn);
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_velocity(GridK g, CoupledK K, const T* __restrict__ po, const T* __restrict__ pn,
                           const T* __restrict__ gx, const T* __restrict__ gy, const T* __restrict__ gz,
                           T* __restrict__ gp, T* __restrict__ vx, T* __restrict__ vy, T* __restrict__ vz,
                           const double* halt) {
    if (halted(halt)) return;
    const long n = g.nreal();
    const T itau = (T)(1.0 / K.tau);
    const double thr = K.thr;
    for (long i = (long)blockIdx.x * kBlock + threadIdx.x; i < n; i += (long)gridDim.x * kBlock)
        velocity_point(itau, thr, pn[i], po[i], gx[i], gy[i], gz[i], &gp[i], &vx[i], &vy[i], &vz[i]);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_q_gu(long n, T ubar, const T* __restrict__ u, const T* __restrict__ G,
                       const uint8_t* __restrict__ mask, T* __restrict__ q, T* __restrict__ gu, double* part) {
    Neu acc;
    for (long i = (long)blockIdx.x * kBlock + threadIdx.x; i < n; i += (long)gridDim.x * kBlock) {
        const T uc = u[i], Gc = G[i];
        T qq = Gc * (uc - ubar);
        if (mask) qq = mask[i] ? qq : (T)0;
        q[i] = qq;
        if (gu) gu[i] = Gc * uc;
        acc.add((double)qq);
    }
    if (part) {
        __shared__ double sh[kBlock];
        const double tot = block_sum_256(acc.val(), sh);
        if (threadIdx.x == 0) part[blockIdx.x] = tot;
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_P2_point(GridK g, CoupledK K, const T* __restrict__ u,
                                                     const T* __restrict__ G, const T* __restrict__ vx,
                                                     const T* __restrict__ vy, const T* __restrict__ vz,
                                                     const T* __restrict__ psi, const double* __restrict__ m,
                                                     const uint8_t* __restrict__ mask, T* __restrict__ P, int tpb) {
    const long nq = g.nreal() / 4;
    const P2Const<T> kc(g, K, m[0]);
    const long t0 = (long)xcd_remap(blockIdx.x, gridDim.x) * tpb;
    for (int it = 0; it < tpb; ++it) {
        const long q = (t0 + it) * kBlock + threadIdx.x;
        if (q >= nq) return;
        const QuadNbr nb = quad_neighbours(g, q);
        const Q4<T> uu = ld4(u + nb.c), GG = ld4(G + nb.c), ps = ld4(psi + nb.c), wz = ld4(vz + nb.c);
        const Q4<T> uxm = ld4(u + nb.xm), uxp = ld4(u + nb.xp), uym = ld4(u + nb.ym), uyp = ld4(u + nb.yp);
        const Q4<T> Gxm = ld4(G + nb.xm), Gxp = ld4(G + nb.xp), Gym = ld4(G + nb.ym), Gyp = ld4(G + nb.yp);
        const Q4<T> vxm = ld4(vx + nb.xm), vxp = ld4(vx + nb.xp), vym = ld4(vy + nb.ym), vyp = ld4(vy + nb.yp);
        const T uzm = u[nb.zm], uzp = u[nb.zp], Gzm = G[nb.zm], Gzp = G[nb.zp], vzm = vz[nb.zm], vzp = vz[nb.zp];
        const unsigned mk = mask ? ld_mask4(mask, nb.c) : 0xffffffffu;
        Q4<T> oP;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const T un[6] = {uxm.v[k], uxp.v[k], uym.v[k], uyp.v[k], k > 0 ? uu.v[k - 1] : uzm,
                             k < 3 ? uu.v[k + 1] : uzp};
            const T Gn[6] = {Gxm.v[k], Gxp.v[k], Gym.v[k], Gyp.v[k], k > 0 ? GG.v[k - 1] : Gzm,
                             k < 3 ? GG.v[k + 1] : Gzp};
            const T vn[6] = {vxm.v[k], vxp.v[k], vym.v[k], vyp.v[k], k > 0 ? wz.v[k - 1] : vzm,
                             k < 3 ? wz.v[k + 1] : vzp};
            oP.v[k] = p2_point(kc, uu.v[k], GG.v[k], ps.v[k], un, Gn, vn, ((mk >> (8 * k)) & 0xffu) != 0);
        }
        st4(P + nb.c, oP);
    }
}

template <typename TI, typename TO> __global__ __launch_bounds__(kBlock) void k_convert(long n, const TI* __restrict__ in, TO* __restrict__ out) {
    for (long i = (long)blockIdx.x * kBlock + threadIdx.x; i < n; i += (long)gridDim.x * kBlock) out[i] = (TO)in[i];
}

template <typename T> __global__ __launch_bounds__(kBlock) void k_gloc(long n, const T* __restrict__ phi, T* __restrict__ G) {
    for (long i = (long)blockIdx.x * kBlock + threadIdx.x; i < n; i += (long)gridDim.x * kBlock) G[i] = gloc(phi[i]);
}

__global__ __launch_bounds__(kBlock) void k_delta(long n, double* x) {
    for (long i = (long)blockIdx.x * kBlock + threadIdx.x; i < n; i += (long)gridDim.x * kBlock) x[i] = (i == 0) ? 1.0 : 0.0;
}

// Stencil launches: tiles of kBlock points, tpb consecutive tiles per block,
// at most 8192 blocks (grids hold fewer than 2^31 points).
struct TileGrid {
    int blocks, tpb;
};
TileGrid tiles_for(long n) {
    const long tiles = (n + kBlock - 1) / kBlock;
    const int tpb = (int)((tiles + 8191) / 8192);
    return {(int)((tiles + tpb - 1) / tpb), tpb};
}

int grid_for(long n) {
    long b = (n + kBlock - 1) / kBlock;
    if (b > 8192) b = 8192;
    return (int)(b < 1 ? 1 : b);
}

}  // namespace

template <typename T>
void spec_apply(const GridK& g, SpecOp op, const c2<T>* in, c2<T>* out, const double* fd, hipStream_t s) {
    hipLaunchKernelGGL(k_spec_apply<T>, dim3(grid_for(g.nspec())), dim3(kBlock), 0, s, g, (int)op, in, out, fd);
}
template <typename T>
void spec_etd_phi1(const GridK& g, const CoupledK& K, const c2<T>* P, const c2<T>* Q, const c2<T>* ph, c2<T>* RA,
                   c2<T>* out, const double* halt, hipStream_t s) {
    hipLaunchKernelGGL((k_etd<ETD_STAGE_PHI1, T>), dim3(grid_for(g.nspec())), dim3(kBlock), 0, s, g, K, P, Q,
                       EtdArgs<T>{ph, RA, out, halt});
}
template <typename T>
void spec_etd_phi2(const GridK& g, const CoupledK& K, const c2<T>* P, const c2<T>* Q, const c2<T>* pt,
                   const c2<T>* RA, c2<T>* out, const double* halt, hipStream_t s) {
    hipLaunchKernelGGL((k_etd<ETD_STAGE_PHI2, T>), dim3(grid_for(g.nspec())), dim3(kBlock), 0, s, g, K, P, Q,
                       EtdArgs<T>{pt, const_cast<c2<T>*>(RA), out, halt});
}
template <typename T>
void spec_etd_u1(const GridK& g, const CoupledK& K, const c2<T>* P, const c2<T>* GU0, c2<T>* D, c2<T>* RA,
                 const double* halt, hipStream_t s) {
    hipLaunchKernelGGL((k_etd<ETD_STAGE_U1, T>), dim3(grid_for(g.nspec())), dim3(kBlock), 0, s, g, K, P, GU0,
                       EtdArgs<T>{nullptr, RA, D, halt});
}
template <typename T>
void spec_etd_u2(const GridK& g, const CoupledK& K, const c2<T>* P, const c2<T>* GB, c2<T>* D, const c2<T>* RA,
                 const double* halt, hipStream_t s) {
    hipLaunchKernelGGL((k_etd<ETD_STAGE_U2, T>), dim3(grid_for(g.nspec())), dim3(kBlock), 0, s, g, K, P, GB,
                       EtdArgs<T>{nullptr, const_cast<c2<T>*>(RA), D, halt});
}
template <typename T>
void coupled_R1_point(const GridK& g, const CoupledK& K, const T* phi, const T* lap, const T* gx, const T* gy,
                      const T* gz, const T* u, const uint8_t* mask, const double* int_phi, double A0, T* P, T* Q,
                      hipStream_t s) {
    const TileGrid tg = tiles_for(g.nreal() / 4);   // one thread per quad of z points
    hipLaunchKernelGGL(k_R1_point<T>, dim3(tg.blocks), dim3(kBlock), 0, s, g, K, phi, lap, gx, gy, gz, u, mask, int_phi,
                       A0, P, Q, tg.tpb);
}
template <typename T>
void r1_surface_band(const GridK& g, const CoupledK& K, const T* phi, const T* lap, const T* gn, const T* u,
                     const int32_t* idx, const int64_t* total, long capacity, const double* int_phi, double A0,
                     T* surf, hipStream_t s) {
    hipLaunchKernelGGL(k_r1_surf_band<T>, dim3(grid_for(capacity)), dim3(kBlock), 0, s, g, K, phi, lap, gn, u, idx,
                       total, int_phi, A0, surf);
}
template <typename T>
void p2_local_band(const GridK& g, const CoupledK& K, const T* u, const T* G, const T* vx, const T* vy,
                   const T* vz, const int32_t* idx, const int64_t* total, long capacity, const double* m, T* surf,
                   hipStream_t s) {
    hipLaunchKernelGGL(k_p2_local_band<T>, dim3(grid_for(capacity)), dim3(kBlock), 0, s, g, K, u, G, vx, vy, vz, idx,
                       total, m, surf);
}
template <typename T>
void coupled_velocity(const GridK& g, const CoupledK& K, const T* po, const T* pn, const T* gx, const T* gy,
                      const T* gz, T* gp, T* vx, T* vy, T* vz, const double* halt, hipStream_t s) {
    hipLaunchKernelGGL(k_velocity<T>, dim3(grid_for(g.nreal())), dim3(kBlock), 0, s, g, K, po, pn, gx, gy, gz, gp, vx,
                       vy, vz, halt);
}
template <typename T>
void coupled_q_gu(const GridK& g, const CoupledK& K, const T* u, const T* G, const uint8_t* mask, T* q, T* gu,
                  double* part, double* mass_out, double* halt, hipStream_t s) {
    const int nb = grid_for(g.nreal());
    hipLaunchKernelGGL(k_q_gu<T>, dim3(nb), dim3(kBlock), 0, s, g.nreal(), (T)K.ubar, u, G, mask, q, gu, part);
    if (part) reduce_final_sum(part, nb, g.cell, mass_out, s, halt);
}
template <typename T>
void coupled_P2_point(const GridK& g, const CoupledK& K, const T* u, const T* G, const T* vx, const T* vy,
                      const T* vz, const T* psi, const double* m, const uint8_t* mask, T* P, hipStream_t s) {
    const TileGrid tg = tiles_for(g.nreal() / 4);   // one thread per quad of z points
    hipLaunchKernelGGL(k_P2_point<T>, dim3(tg.blocks), dim3(kBlock), 0, s, g, K, u, G, vx, vy, vz, psi, m, mask, P,
                       tg.tpb);
}
template <typename TI, typename TO> void convert(long n, const TI* in, TO* out, hipStream_t s) {
    hipLaunchKernelGGL((k_convert<TI, TO>), dim3(grid_for(n)), dim3(kBlock), 0, s, n, in, out);
}

template <typename T> void gloc_field(long n, const T* phi, T* G, hipStream_t s) {
    hipLaunchKernelGGL(k_gloc<T>, dim3(grid_for(n)), dim3(kBlock), 0, s, n, phi, G);
}
void set_delta(long n, double* x, hipStream_t s) {
    hipLaunchKernelGGL(k_delta, dim3(grid_for(n)), dim3(kBlock), 0, s, n, x);
}

#define INST(T)                                                                                                   \
    template void gloc_field<T>(long, const T*, T*, hipStream_t);                                                 \
    template void spec_apply<T>(const GridK&, SpecOp, const c2<T>*, c2<T>*, const double*, hipStream_t);         \
    template void spec_etd_phi1<T>(const GridK&, const CoupledK&, const c2<T>*, const c2<T>*, const c2<T>*,       \
                                   c2<T>*, c2<T>*, const double*, hipStream_t);                                   \
    template void spec_etd_phi2<T>(const GridK&, const CoupledK&, const c2<T>*, const c2<T>*, const c2<T>*,       \
                                   const c2<T>*, c2<T>*, const double*, hipStream_t);                             \
    template void spec_etd_u1<T>(const GridK&, const CoupledK&, const c2<T>*, const c2<T>*, c2<T>*, c2<T>*,       \
                                 const double*, hipStream_t);                                                     \
    template void spec_etd_u2<T>(const GridK&, const CoupledK&, const c2<T>*, const c2<T>*, c2<T>*,               \
                                 const c2<T>*, const double*, hipStream_t);                                       \
    template void coupled_R1_point<T>(const GridK&, const CoupledK&, const T*, const T*, const T*, const T*,      \
                                      const T*, const T*, const uint8_t*, const double*, double, T*, T*,          \
                                      hipStream_t);                                                               \
    template void r1_surface_band<T>(const GridK&, const CoupledK&, const T*, const T*, const T*, const T*,       \
                                     const int32_t*, const int64_t*, long, const double*, double, T*,             \
                                     hipStream_t);                                                                \
    template void p2_local_band<T>(const GridK&, const CoupledK&, const T*, const T*, const T*, const T*,         \
                                   const T*, const int32_t*, const int64_t*, long, const double*, T*,             \
                                   hipStream_t);                                                                  \
    template void coupled_velocity<T>(const GridK&, const CoupledK&, const T*, const T*, const T*, const T*,      \
                                      const T*, T*, T*, T*, T*, const double*, hipStream_t);                      \
    template void coupled_q_gu<T>(const GridK&, const CoupledK&, const T*, const T*, const uint8_t*, T*, T*,      \
                                  double*, double*, double*, hipStream_t);                                        \
    template void coupled_P2_point<T>(const GridK&, const CoupledK&, const T*, const T*, const T*, const T*,      \
                                      const T*, const T*, const double*, const uint8_t*, T*, hipStream_t);
INST(float)
INST(double)
#undef INST
template void convert<float, double>(long, const float*, double*, hipStream_t);
template void convert<double, float>(long, const double*, float*, hipStream_t);
template void convert<double, double>(long, const double*, double*, hipStream_t);
template void convert<float, float>(long, const float*, float*, hipStream_t);

}  // namespace etd
