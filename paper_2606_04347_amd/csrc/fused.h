// Fused spectral pipelines built on the line-FFT engine (three-dimensional
// grids, nx > 1; lapinv_fused also takes two-dimensional grids).
#pragma once

#include "etd_point.h"
#include "fft.h"

namespace etd {

// From the half spectrum S of phi: phi, the norm gn = |grad phi| of its
// spectral gradient and its spectral Laplacian lap (Section 3.2), in three
// passes: inverse x lines (S -> S, i kx S, -kx^2 S), inverse y lines (3 -> 4
// spectra), z rows c2r (4 spectra -> phi, the three gradient components kept
// in registers and reduced to gn, lap).  W0..W3: complex work arrays (nspec
// each); S is preserved.  With isum != null the z pass also forms the
// integral h^3 sum phi into isum->out (block partials in isum->part,
// nx * ny / 8 doubles at most, then a fixed-order final sum).
template <typename T>
hipError_t derivs_fused(const GridK& g, const FFTTables<T>& t, const c2<T>* S, c2<T>* W0, c2<T>* W1, c2<T>* W2,
                        c2<T>* W3, T* phi, T* gn, T* lap, const GridSum* isum, hipStream_t s);

// g+ and the velocity of the u equation (Section 3.1) from phi^{n+1} (the
// field being formed), phi^n = po and the step tau; thr the support threshold.
template <typename T> struct VelocityArgs {
    const T* po;
    T* G;
    T* vx;
    T* vy;
    T* vz;
    double tau, thr;
};

// The y and z passes of derivs_fused, for spectra already through the
// inverse x pass (W0 = X^-1 S, W1 = X^-1 i kx S, W2 = X^-1 (-kx^2) S); W3 work.
// With vel != null the z pass also writes g+ and the velocity at the new phi.
template <typename T>
hipError_t derivs_fused_yz(const GridK& g, const FFTTables<T>& t, c2<T>* W0, c2<T>* W1, c2<T>* W2, c2<T>* W3, T* phi,
                           T* gn, T* lap, const GridSum* isum, hipStream_t s, const VelocityArgs<T>* vel = nullptr);

// Forward transforms of two real fields P, Q (into the work spectra WP, WQ)
// and, in the last (x) pass, the ETD combine of the given stage (etd_point.h)
// with p = FFT P, q = FFT Q; its output goes to a.out if store_out.  The same
// pass then runs the inverse x transforms of that output the next passes
// need: after a phi stage (S, i kx S, -kx^2 S) -> (X0, X1, X2) (continue
// with derivs_fused_yz), after a u stage the plain inverse -> X0 (continue
// with c2r_recover_yz).  X0..X2 may alias WP / WQ.
template <typename T>
hipError_t fwd_pair_etd(const GridK& g, const FFTTables<T>& t, const CoupledK& K, EtdStage stage, const T* P,
                        const T* Q, c2<T>* WP, c2<T>* WQ, const EtdArgs<T>& a, bool store_out, c2<T>* X0,
                        c2<T>* X1, c2<T>* X2, hipStream_t s);

// Sources of R1 (Section 3.1) at phi and u: phi, its spectral Laplacian and
// gradient norm, u, the band mask (nullable), the device scalar h^3 sum phi
// and A0.
template <typename T> struct R1Fields {
    const T *phi, *lap, *gn, *u;   // gn = |grad phi|
    const uint8_t* mask;
    const double* int_phi;
    double A0;
    // with mask: the surface part of P1 on the band (r1_surface_band), read
    // where the mask is set; the z pass then forms no stencils
    const T* surf = nullptr;
};
// Sources of P2 (Section 3.1): u, G = g+, the velocity, psi = the nonlocal
// inverse of q ((-Delta_h)^{-1} by FFT, or the band solve), the band mask
// (nullable) and the device scalar m = h^3 sum q.  With psi_hat != null,
// psi is taken from that spectrum instead (psi's half spectrum after the
// inverse x and y passes, the output of lapinv_q_fused with psi == null):
// the z pass of P2 runs psi's inverse z transform into its LDS first.
template <typename T> struct P2Fields {
    const T *u, *G, *vx, *vy, *vz, *psi;
    const uint8_t* mask;
    const double* m;
    const c2<T>* psi_hat = nullptr;
    // with mask: P2 without its nonlocal term on the band (p2_local_band),
    // read where the mask is set
    const T* surf = nullptr;
};

// fwd_pair_etd with the pair (P1, W'(phi) - A1 phi) formed from its sources
// in the load of the z pass (no R1 fields written or read back).
template <typename T>
hipError_t r1_etd(const GridK& g, const FFTTables<T>& t, const CoupledK& K, const R1Fields<T>& f, EtdStage stage,
                  c2<T>* WP, c2<T>* WQ, const EtdArgs<T>& a, bool store_out, c2<T>* X0, c2<T>* X1, c2<T>* X2,
                  hipStream_t s);
// fwd_pair_etd with the pair (P2, g+ u) formed in the load of the z pass
// (u stages: X0 receives the inverse x transform of the increment).
template <typename T>
hipError_t p2_etd(const GridK& g, const FFTTables<T>& t, const CoupledK& K, const P2Fields<T>& f, EtdStage stage,
                  c2<T>* WP, c2<T>* WQ, const EtdArgs<T>& a, bool store_out, c2<T>* X0, hipStream_t s);

// psi = (-Delta_h)^{-1} q through the FD symbol mu (zero mean mode): forward
// transform, then the last forward axis is multiplied by 1/mu and inverted in
// the same pass.  fd: per-axis symbol tables [x (nx) | y (ny) | z (nzh)].
// W: complex work array.  q and psi may alias.
template <typename T>
hipError_t lapinv_fused(const GridK& g, const FFTTables<T>& t, const double* fd, const T* q, c2<T>* W, T* psi,
                        hipStream_t s);
// The same for q = G (u - ubar) on the band (mask nullable) formed in the load
// of the z pass, which also forms the mass h^d sum q into msum.out (block
// partials in msum.part, at most nx * ny / 8 doubles, then a fixed-order
// final sum).  With psi == null (three-dimensional grids) the last (z) pass
// is left out: W holds psi's half spectrum after the inverse x and y passes,
// for P2Fields::psi_hat.
template <typename T>
hipError_t lapinv_q_fused(const GridK& g, const FFTTables<T>& t, const double* fd, double ubar, const T* u,
                          const T* G, const uint8_t* mask, c2<T>* W, T* psi, const GridSum& msum, hipStream_t s);

// U from an increment spectrum D of G U (Section 3.3 after Algorithm 1):
// d = F^-1 D, out = u_old + d / G where G > thr, G u_old + d elsewhere; the
// recovery runs in the store of the z c2r pass.  W: complex work array (D is
// preserved); out may alias u_old.  Once *halt != 0 (halt nullable) the pass
// writes out = u_old instead.
template <typename T>
hipError_t c2r_recover(const GridK& g, const FFTTables<T>& t, const c2<T>* D, c2<T>* W, const T* u_old, const T* G,
                       T* out, double thr, const double* halt, hipStream_t s);
// The y and z passes of c2r_recover for W = X^-1 D (W is overwritten).
template <typename T>
hipError_t c2r_recover_yz(const GridK& g, const FFTTables<T>& t, c2<T>* W, const T* u_old, const T* G, T* out,
                          double thr, const double* halt, hipStream_t s);

}  // namespace etd
