// Pointwise ETD combines of the coupled scheme in Fourier space (Section 3.3,
// Algorithm 1), shared by the standalone spectral kernels and the epilogue of
// the fused forward x pass.  The arguments z = tau l(k^2) and the
// phi-function values are formed in FP64 on both paths (a series branch for
// small z); the FP32 path rounds the finished multipliers to FP32.
#pragma once

#include "kernels.h"

namespace etd {

// phi1(z) = (1 - e^{-z})/z, phi2(z) = (e^{-z} - 1 + z)/z^2; for |z| < 0.1 the
// series sum_j (-z)^j / (j + k)! (14 terms, truncation < 1e-25) avoids the
// cancellation of the closed forms.
__device__ __forceinline__ double phi_taylor(double z, int k) {
    double f = 1.0;
    for (int j = 1; j <= k; ++j) f *= j;
    double fact[14];
    fact[0] = 1.0 / f;
    for (int j = 1; j < 14; ++j) fact[j] = fact[j - 1] / (double)(j + k);
    double out = 0.0;
    for (int j = 13; j >= 0; --j) out = out * (-z) + fact[j];
    return out;
}
__device__ __forceinline__ double phi1d(double z) { return fabs(z) < 0.1 ? phi_taylor(z, 1) : -expm1(-z) / z; }
__device__ __forceinline__ double phi2d(double z) {
    return fabs(z) < 0.1 ? phi_taylor(z, 2) : (expm1(-z) + z) / (z * z);
}

// The FP32 path forms the same values in FP64 from a single exponential
// e = e^{-z}: phi1 = (1 - e)/z and phi2 = (z - 1 + e)/z^2 for z >= 0.1, the
// series below.  The cancellation there costs at most a factor ~1/(1 - e^{-0.1})
// = 10.5 (phi1) or ~2/0.1^2 = 200 (phi2) of FP64 precision, below 1e-13
// relative: far under the FP32 rounding of the result.
struct PhiE {
    double e0, p1, p2;
};
template <int K> __device__ __forceinline__ PhiE phi_one_exp(double z) {
    PhiE r;
    r.e0 = exp(-z);
    if (fabs(z) < 0.1) {
        if constexpr (K & 1) r.p1 = phi_taylor(z, 1);
        if constexpr (K & 2) r.p2 = phi_taylor(z, 2);
    } else {
        const double iz = 1.0 / z;
        if constexpr (K & 1) r.p1 = (1.0 - r.e0) * iz;
        if constexpr (K & 2) r.p2 = ((z - 1.0) + r.e0) * (iz * iz);
    }
    return r;
}

// linear symbols (eqn:linear_force and the u equation)
__device__ __forceinline__ double lphi(const CoupledK& K, double k2) { return (K.lp4 * k2 + K.lp2) * k2 + K.lp0; }
__device__ __forceinline__ double lu(const CoupledK& K, double k2) { return K.B2 + K.eps_u * K.B1 * k2; }

// The four combines.  p = FFT of the first remainder field, q = FFT of the
// second (W'(phi) - A1 phi for phi, g+ u for u); index i addresses the other
// spectra of the stage.
enum EtdStage { ETD_STAGE_PHI1 = 0, ETD_STAGE_PHI2 = 1, ETD_STAGE_U1 = 2, ETD_STAGE_U2 = 3 };

template <typename T> struct EtdArgs {
    const c2<T>* prev;   // PHI1: phi^n hat;  PHI2: phi~ hat
    c2<T>* ra;           // stage-1 remainder R(.)^ (written by *1, read by *2)
    c2<T>* out;          // PHI*: new phi hat;  U*: increment D (U2 reads and updates it)
    const double* halt = nullptr;   // the instance's halt flag: the combine is skipped once it is set
    int lines = 0;                  // FP32 ETD x pass: lines per workgroup (0 or 16: 16, 8: 8)
};

// The values a combine reads at its index besides p and q: PHI1 phi^n hat;
// PHI2 phi~ hat and R; U2 D and R (U1 none).  Loaded apart from the combine
// so a caller can issue the loads of several indices before the first of
// their stores.
template <typename T> struct CombineIn {
    c2<T> a, b;
};
template <int ST, typename T> __device__ __forceinline__ CombineIn<T> combine_load(const EtdArgs<T>& a, long i) {
    CombineIn<T> c;
    if constexpr (ST == ETD_STAGE_PHI1) {
        c.a = a.prev[i];
    } else if constexpr (ST == ETD_STAGE_PHI2) {
        c.a = a.prev[i];
        c.b = a.ra[i];
    } else if constexpr (ST == ETD_STAGE_U2) {
        c.a = a.out[i];
        c.b = a.ra[i];
    }
    return c;
}

// Returns the stage's output value at i (PHI*: the new phi hat, U*: the
// increment D) from the values combine_load read at i; the stage-1
// remainder is stored into a.ra here, the output is left to the caller.
template <int ST, typename T>
__device__ __forceinline__ c2<T> etd_combine(const CoupledK& K, double k2, long i, c2<T> p, c2<T> q,
                                             const EtdArgs<T>& a, const CombineIn<T>& in) {
    if constexpr (ST == ETD_STAGE_PHI1) {
        // R = P - c1 k^2 Q;  phi~ = e^{-tau l} phi^n + tau phi1(tau l) R
        const double z = K.tau * lphi(K, k2);
        T e0, te1;
        if constexpr (sizeof(T) == 4) {
            const PhiE f = phi_one_exp<1>(z);
            e0 = (T)f.e0;
            te1 = (T)(K.tau * f.p1);
        } else {
            e0 = exp(-z);
            te1 = K.tau * phi1d(z);
        }
        const T ck = (T)(K.c1 * k2);
        const c2<T> f = in.a;
        const c2<T> R = mk<T>(p.x - ck * q.x, p.y - ck * q.y);
        a.ra[i] = R;
        return mk<T>(e0 * f.x + te1 * R.x, e0 * f.y + te1 * R.y);
    } else if constexpr (ST == ETD_STAGE_PHI2) {
        // phi^{n+1} = phi~ + tau phi2(tau l) (R~ - R)
        const double z = K.tau * lphi(K, k2);
        const T te2 = (T)(K.tau * (sizeof(T) == 4 ? phi_one_exp<2>(z).p2 : phi2d(z)));
        const T ck = (T)(K.c1 * k2);
        const c2<T> t = in.a, ra = in.b;
        const T dx = (p.x - ck * q.x) - ra.x, dy = (p.y - ck * q.y) - ra.y;
        return mk<T>(t.x + te2 * dx, t.y + te2 * dy);
    } else if constexpr (ST == ETD_STAGE_U1) {
        // R = P + eps_u B1 k^2 GU;  D = tau phi1(tau l_u) (R - l_u GU)  (GU~ - GU^n)
        const double l = lu(K, k2);
        const double z = K.tau * l;
        const T te1 = (T)(K.tau * (sizeof(T) == 4 ? phi_one_exp<1>(z).p1 : phi1d(z)));
        const T ck = (T)(K.eps_u * K.B1 * k2), lt = (T)l;
        const c2<T> R = mk<T>(p.x + ck * q.x, p.y + ck * q.y);
        a.ra[i] = R;
        return mk<T>(te1 * (R.x - lt * q.x), te1 * (R.y - lt * q.y));
    } else {
        // D <- D + tau phi2(tau l_u) (R~ - R)
        const double z = K.tau * lu(K, k2);
        const T te2 = (T)(K.tau * (sizeof(T) == 4 ? phi_one_exp<2>(z).p2 : phi2d(z)));
        const T ck = (T)(K.eps_u * K.B1 * k2);
        const c2<T> d = in.a, ra = in.b;
        const T dx = (p.x + ck * q.x) - ra.x, dy = (p.y + ck * q.y) - ra.y;
        return mk<T>(d.x + te2 * dx, d.y + te2 * dy);
    }
}
template <int ST, typename T>
__device__ __forceinline__ c2<T> etd_combine(const CoupledK& K, double k2, long i, c2<T> p, c2<T> q,
                                             const EtdArgs<T>& a) {
    return etd_combine<ST, T>(K, k2, i, p, q, a, combine_load<ST, T>(a, i));
}

}  // namespace etd
