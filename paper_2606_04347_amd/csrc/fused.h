// Fused spectral pipelines built on the line-FFT engine (three-dimensional
// grids, nx > 1; lapinv_fused also takes two-dimensional grids).
#pragma once

#include "etd_point.h"
#include "fft.h"

namespace etd {

// From the half spectrum S of phi: phi, its spectral gradient (gx, gy, gz)
// and spectral Laplacian lap (Section 3.2), in three passes: inverse x lines
// (S -> S, i kx S, -kx^2 S), inverse y lines (3 -> 4 spectra), z rows c2r
// (4 spectra -> 5 real fields).  W0..W3: complex work arrays (nspec each); S
// is preserved.
template <typename T>
hipError_t derivs_fused(const GridK& g, const FFTTables<T>& t, const c2<T>* S, c2<T>* W0, c2<T>* W1, c2<T>* W2,
                        c2<T>* W3, T* phi, T* gx, T* gy, T* gz, T* lap, hipStream_t s);

// Forward transforms of two real fields P, Q (into the work spectra WP, WQ)
// and, in the epilogue of the last (x) pass, the ETD combine of the given
// stage (etd_point.h) with p = FFT P, q = FFT Q.
template <typename T>
hipError_t fwd_pair_etd(const GridK& g, const FFTTables<T>& t, const CoupledK& K, EtdStage stage, const T* P,
                        const T* Q, c2<T>* WP, c2<T>* WQ, const EtdArgs<T>& a, hipStream_t s);

// psi = (-Delta_h)^{-1} q through the FD symbol mu (zero mean mode): forward
// transform, then the last forward axis is multiplied by 1/mu and inverted in
// the same pass.  fd: per-axis symbol tables [x (nx) | y (ny) | z (nzh)].
// W: complex work array.  q and psi may alias.
template <typename T>
hipError_t lapinv_fused(const GridK& g, const FFTTables<T>& t, const double* fd, const T* q, c2<T>* W, T* psi,
                        hipStream_t s);

// U from an increment spectrum D of G U (Section 3.3 after Algorithm 1):
// d = F^-1 D, out = u_old + d / G where G > thr, G u_old + d elsewhere; the
// recovery runs in the store of the z c2r pass.  W: complex work array (D is
// preserved); out may alias u_old.
template <typename T>
hipError_t c2r_recover(const GridK& g, const FFTTables<T>& t, const c2<T>* D, c2<T>* W, const T* u_old, const T* G,
                       T* out, double thr, hipStream_t s);

}  // namespace etd
