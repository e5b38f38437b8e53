// Pointwise arithmetic of the coupled model's real-space remainders (device
// code): P1 and W'(phi) - A1 phi of R1 (Section 3.1, eqn:linear_force split),
// P2 of R2 (Section 3.1, eqn:linear_OK split), with the second-order FD
// operators of Section 2.1.  Shared by the standalone stencil kernels and the
// producers fused into the forward z pass.
#pragma once

#include "kernels.h"

namespace etd {

template <typename T> __device__ __forceinline__ T gloc(T p) {
    const T a = p * p - p;
    return (T)18 * a * a;
}
template <typename T> __device__ __forceinline__ T Wp(T s) { return (T)36 * (s * s - s) * ((T)2 * s - (T)1); }
template <typename T> __device__ __forceinline__ T Wpp(T s) { return (T)36 * ((T)6 * s * s - (T)6 * s + (T)1); }

// D^-(g_{i+1/2} D^+ u) along one axis, g at the three points given
template <typename T>
__device__ __forceinline__ T lapS_axis(T um, T uc, T up, T gm, T gc, T gp, T ih2) {
    const T ghp = (T)0.5 * (gc + gp), ghm = (T)0.5 * (gm + gc);
    return (ghp * (up - uc) - ghm * (uc - um)) * ih2;
}

// Constants of P1 in the working precision (area term from the device scalar int phi).
template <typename T> struct R1Const {
    T e2, c1, A1, A2, cW, cs, cl, ca, area, eu, ieu, ep, iep, u0, ihx, ihy, ihz;
    __device__ __forceinline__ R1Const(const GridK& g, const CoupledK& K, double int_phi, double A0) {
        e2 = (T)(K.eps_phi * K.eps_phi);
        c1 = (T)K.c1;
        A1 = (T)K.A1;
        A2 = (T)K.A2;
        cW = (T)(K.kappa / (K.mu * K.eps_phi * K.eps_phi * K.eps_phi * K.eps_phi));
        cs = (T)(K.lambda_surf / (K.mu * K.eps_phi * K.eps_phi));
        cl = (T)(K.lambda_line / K.mu);
        ca = (T)(K.alpha / K.mu);
        area = (T)((K.M_area / K.mu) * (int_phi - A0));
        eu = (T)K.eps_u;
        ieu = (T)(1.0 / K.eps_u);
        ep = (T)K.eps_phi;
        iep = (T)(1.0 / K.eps_phi);
        u0 = (T)K.u0;
        ihx = (T)(g.nx > 1 ? 1.0 / (g.h[0] * g.h[0]) : 0.0);
        ihy = (T)(1.0 / (g.h[1] * g.h[1]));
        ihz = (T)(1.0 / (g.h[2] * g.h[2]));
    }
};

// P1 (into *P) and W'(phi) - A1 phi (into *Q) at one point: centre values
// (phi, its spectral Laplacian L, the norm gn = |grad phi| of its spectral
// gradient, u), the six neighbours of u and phi (x-, x+, y-, y+, z-, z+), and
// the band flag.  P1 sees the gradient only through its norm.
// The part of P1 and Q that does not involve u or |grad phi| (a point off the band).
template <typename T> __device__ __forceinline__ void r1_core(const R1Const<T>& k, T pc, T L, T* P, T* Q) {
    const T wp = Wp(pc), wpp = Wpp(pc);
    const T q1 = wp - k.A1 * pc;
    *P = k.c1 * (wpp - k.A2) * (L - k.A1 * pc / k.e2) - (k.cW * wpp + k.cs) * q1;
    *Q = q1;
}

// The |grad phi|-weighted (surface) part of P1 at one point from its
// ingredients: gc = g(phi), the weighted Laplacian S of u, wp = W'(phi).
template <typename T>
__device__ __forceinline__ T r1_surf_terms(const R1Const<T>& k, T L, T gn, T uc, T gc, T S, T wp) {
    return k.cl * (k.eu * S - gc * Wp(uc) * k.ieu) * gn - k.area * gn + k.ca * (uc + k.u0) * gn * (k.ep * L - wp * k.iep);
}
// S = the g(phi)-weighted Laplacian of u at one point (six neighbours of u and phi).
template <typename T>
__device__ __forceinline__ T r1_stencil(const R1Const<T>& k, T uc, T gc, const T (&un)[6], const T (&pn)[6]) {
    T S = lapS_axis(un[0], uc, un[1], gloc(pn[0]), gc, gloc(pn[1]), k.ihx);
    S += lapS_axis(un[2], uc, un[3], gloc(pn[2]), gc, gloc(pn[3]), k.ihy);
    S += lapS_axis(un[4], uc, un[5], gloc(pn[4]), gc, gloc(pn[5]), k.ihz);
    return S;
}
// The surface part of P1 at one point (zero off the band).
template <typename T>
__device__ __forceinline__ T r1_surf(const R1Const<T>& k, T pc, T L, T gn, T uc, const T (&un)[6],
                                     const T (&pn)[6]) {
    const T gc = gloc(pc);
    return r1_surf_terms(k, L, gn, uc, gc, r1_stencil(k, uc, gc, un, pn), Wp(pc));
}

template <typename T>
__device__ __forceinline__ void r1_point(const R1Const<T>& k, T pc, T L, T gn, T uc, const T (&un)[6],
                                         const T (&pn)[6], bool band, T* P, T* Q) {
    const T gc = gloc(pc);
    const T S = r1_stencil(k, uc, gc, un, pn);
    const T wp = Wp(pc), wpp = Wpp(pc);
    const T q1 = wp - k.A1 * pc;
    const T p1 = k.c1 * (wpp - k.A2) * (L - k.A1 * pc / k.e2) - (k.cW * wpp + k.cs) * q1;
    const T surf = band ? r1_surf_terms(k, L, gn, uc, gc, S, wp) : (T)0;
    *P = p1 + surf;
    *Q = q1;
}

// Constants of P2 in the working precision (mass term from the device scalar m).
template <typename T> struct P2Const {
    T eu, ieu, B2, gam, Mm, ihx, ihy, ihz, i2hx, i2hy, i2hz;
    __device__ __forceinline__ P2Const(const GridK& g, const CoupledK& K, double m) {
        eu = (T)K.eps_u;
        ieu = (T)(1.0 / K.eps_u);
        B2 = (T)K.B2;
        gam = (T)K.gamma;
        Mm = (T)(K.M * m);
        ihx = (T)(g.nx > 1 ? 1.0 / (g.h[0] * g.h[0]) : 0.0);
        ihy = (T)(1.0 / (g.h[1] * g.h[1]));
        ihz = (T)(1.0 / (g.h[2] * g.h[2]));
        i2hx = (T)(g.nx > 1 ? 0.5 / g.h[0] : 0.0);
        i2hy = (T)(0.5 / g.h[1]);
        i2hz = (T)(0.5 / g.h[2]);
    }
};

// P2 at one point: centre u, G, psi; the six neighbours of u and G; the
// velocity component along each neighbour's axis (vx at x-+, vy at y-+,
// vz at z-+); the band flag.
// P2 at one point without its nonlocal term - gamma G psi (the stencil part,
// formed on the band list when the band is in use).
template <typename T>
__device__ __forceinline__ T p2_local(const P2Const<T>& k, T uc, T Gc, const T (&un)[6], const T (&Gn)[6],
                                      const T (&vn)[6]) {
    T S = lapS_axis(un[0], uc, un[1], Gn[0], Gc, Gn[1], k.ihx);
    S += lapS_axis(un[2], uc, un[3], Gn[2], Gc, Gn[3], k.ihy);
    S += lapS_axis(un[4], uc, un[5], Gn[4], Gc, Gn[5], k.ihz);
    const T div = (Gn[1] * un[1] * vn[1] - Gn[0] * un[0] * vn[0]) * k.i2hx +
                  (Gn[3] * un[3] * vn[3] - Gn[2] * un[2] * vn[2]) * k.i2hy +
                  (Gn[5] * un[5] * vn[5] - Gn[4] * un[4] * vn[4]) * k.i2hz;
    return k.eu * S + k.B2 * Gc * uc - Gc * Wp(uc) * k.ieu - k.Mm * Gc - div;
}
template <typename T> __device__ __forceinline__ T p2_from_local(const P2Const<T>& k, T local, T Gc, T ps) {
    return local - k.gam * Gc * ps;
}

template <typename T>
__device__ __forceinline__ T p2_point(const P2Const<T>& k, T uc, T Gc, T ps, const T (&un)[6], const T (&Gn)[6],
                                      const T (&vn)[6], bool band) {
    return band ? p2_from_local(k, p2_local(k, uc, Gc, un, Gn, vn), Gc, ps) : (T)0;
}

// g+ = g(phi^{n+1}) and the velocity v = -phi_t grad phi / |grad phi|^2
// (phi_t = (phi^{n+1} - phi^n) / tau) on {g+ > thr, |grad phi| > 0}, 0
// elsewhere (Section 3.1, the advection velocity of the u equation).
template <typename T>
__device__ __forceinline__ void velocity_point(T itau, double thr, T p, T po, T a, T b, T c, T* G, T* vx, T* vy, T* vz) {
    const T g = gloc(p);
    const T gn2 = a * a + b * b + c * c;
    const bool sel = ((double)g > thr) && (gn2 > (T)0);   // threshold decided in FP64
    const T dt = (p - po) * itau;
    const T w = sel ? -dt / gn2 : (T)0;   // one division for the three components
    *G = g;
    *vx = sel ? w * a : (T)0;
    *vy = sel ? w * b : (T)0;
    *vz = sel ? w * c : (T)0;
}

}  // namespace etd
