// Launchers of the pointwise, stencil, spectral and reduction kernels.
#pragma once

#include "common.h"

namespace etd {

// Constants of the coupled model as the kernels use them (Section 3.1).
struct CoupledK {
    double mu, lambda_surf, kappa, lambda_line, M_area, alpha, u0;
    double eps_phi, eps_u, gamma, ubar, M, A1, A2, B1, B2;
    double tau;
    double c1;                 // kappa / (mu eps_phi^2)
    double lp4, lp2, lp0;      // l_phi(k^2) = lp4 k^4 + lp2 k^2 + lp0  (eqn:linear_force)
    double thr;                // recovery threshold on g
};

// A grid-wide FP64 sum formed by a fused kernel: its workgroups leave block
// partials in part, a fixed-order final sum writes scale * total to *out.
struct GridSum {
    double* part;
    double* out;
    double scale;
    double* halt = nullptr;   // set to 1 when the total is not finite (nullable)
};

// Kernels that write a step's state take the instance's halt flag (a device
// scalar, nullable): once it is non-zero they leave the state as it is, so
// the steps after a non-finite value was detected are no-ops, also inside a
// captured graph.
__device__ __forceinline__ bool halted(const double* halt) { return halt && *halt != 0.0; }

// ------------------------------------------------------------------ spectral
enum SpecOp { SPEC_NEG_K2 = 0, SPEC_IKX = 1, SPEC_IKY = 2, SPEC_IKZ = 3, SPEC_INV_FD = 4 };

// out = m(k) in for one of the SpecOp multipliers (FP64-formed, rounded to T).
// fd: per-axis FD symbol tables [4/h_x^2 sin^2(pi i/N_x), i < N_x | y | z] (SPEC_INV_FD).
template <typename T>
void spec_apply(const GridK& g, SpecOp op, const c2<T>* in, c2<T>* out, const double* fd, hipStream_t s);

// phi stage 1: R = P - c1 k^2 Q  -> RA;  out = E0 phi_hat + tau E1 R.
// Each combine is a no-op once *halt != 0 (nullable).
template <typename T>
void spec_etd_phi1(const GridK& g, const CoupledK& K, const c2<T>* P, const c2<T>* Q, const c2<T>* phi_hat,
                   c2<T>* RA, c2<T>* out, const double* halt, hipStream_t s);
// phi stage 2: out = phit + tau E2 ((P - c1 k^2 Q) - RA).
template <typename T>
void spec_etd_phi2(const GridK& g, const CoupledK& K, const c2<T>* P, const c2<T>* Q, const c2<T>* phit,
                   const c2<T>* RA, c2<T>* out, const double* halt, hipStream_t s);
// u stage 1: RA = P + eps_u B1 k^2 GU0;  D = GU~^ - GU0 = tau phi1(tau l_u) (RA - l_u GU0).
template <typename T>
void spec_etd_u1(const GridK& g, const CoupledK& K, const c2<T>* P, const c2<T>* GU0, c2<T>* D, c2<T>* RA,
                 const double* halt, hipStream_t s);
// u stage 2: D <- D + tau E2u ((P + eps_u B1 k^2 GB) - RA).
template <typename T>
void spec_etd_u2(const GridK& g, const CoupledK& K, const c2<T>* P, const c2<T>* GB, c2<T>* D,
                 const c2<T>* RA, const double* halt, hipStream_t s);

// ------------------------------------------------------------------ real space, coupled
template <typename T>
void coupled_R1_point(const GridK& g, const CoupledK& K, const T* phi, const T* lap, const T* gx, const T* gy,
                      const T* gz, const T* u, const uint8_t* mask, const double* int_phi, double A0, T* P,
                      T* Q, hipStream_t s);
// On a 3D grid with the band: the surface part of P1 (the |grad phi|-weighted
// terms, stencils of u and g(phi)) and P2 without its nonlocal term (the
// stencils of u, g+ and v) at the points of the band list idx (total[0]
// entries on the device, at most capacity), written to surf at those points
// only; the z passes add them where the band mask is set.
template <typename T>
void r1_surface_band(const GridK& g, const CoupledK& K, const T* phi, const T* lap, const T* gn, const T* u,
                     const int32_t* idx, const int64_t* total, long capacity, const double* int_phi, double A0,
                     T* surf, hipStream_t s);
template <typename T>
void p2_local_band(const GridK& g, const CoupledK& K, const T* u, const T* gplus, const T* vx, const T* vy,
                   const T* vz, const int32_t* idx, const int64_t* total, long capacity, const double* m, T* surf,
                   hipStream_t s);
template <typename T>
void coupled_velocity(const GridK& g, const CoupledK& K, const T* phi_old, const T* phi_new, const T* gx,
                      const T* gy, const T* gz, T* gplus, T* vx, T* vy, T* vz, const double* halt, hipStream_t s);
// q = g+ (u - ubar) (masked), gu = g+ u (gu may be null); with part != null also the mass
// mass_out[0] = cell * sum q (block partials in part, then a fixed-order final
// sum; part holds at least kRedBlocks * 4 doubles); a mass that is not finite
// sets *halt (nullable).
template <typename T>
void coupled_q_gu(const GridK& g, const CoupledK& K, const T* u, const T* gplus, const uint8_t* mask, T* q,
                  T* gu, double* part, double* mass_out, double* halt, hipStream_t s);
template <typename T>
void coupled_P2_point(const GridK& g, const CoupledK& K, const T* u, const T* gplus, const T* vx, const T* vy,
                      const T* vz, const T* psi, const double* m, const uint8_t* mask, T* P, hipStream_t s);

// ------------------------------------------------------------------ reductions (FP64, deterministic)
constexpr int kRedBlocks = 2048;

// out[0] = scale * sum of part[0..nb) (Neumaier-compensated, fixed order); a
// total that is not finite sets *halt to 1 (halt nullable).
void reduce_final_sum(const double* part, int nb, double scale, double* out, hipStream_t s, double* halt = nullptr);

// out[0] = scale * sum_i x_i  (Neumaier-compensated, fixed order).  part: kRedBlocks doubles.
template <typename T>
void reduce_sum(long n, const T* x, double scale, double* part, double* out, hipStream_t s, double* halt = nullptr);

// Diagnostics of a state: out = [h^d sum phi, h^d sum g (u - ubar), h^d sum g u, min u, max u,
// max |2u - 1|, nonfinite count].  phi may be null (then g is taken from gfix, the fixed membrane).
// For the fixed model the second entry is h^d sum g (f(u) - ubar).
template <typename T>
void reduce_diag(const GridK& g, const T* phi, const double* gfix, const T* u, double ubar, bool fixed_model,
                 double* part, double* out, hipStream_t s);

// Coupled energy sums: out = [sum(|grad phi|^2/2 + W(phi)/eps^2), sum (lap - W'(phi)/eps^2)^2,
// sum phi, sum g_half (D+ u)^2 (edges), sum g W(u), sum psi q, sum q]  (unscaled).
// gy = gz = nullptr: gx holds |grad phi|.
template <typename T>
void reduce_energy_coupled(const GridK& g, const CoupledK& K, const T* phi, const T* lap, const T* gx,
                           const T* gy, const T* gz, const T* u, const T* psi, const T* q, double* part,
                           double* out, hipStream_t s);

// ------------------------------------------------------------------ conversions / small helpers
template <typename TI, typename TO> void convert(long n, const TI* in, TO* out, hipStream_t s);
// G = g(phi) = 18 (phi^2 - phi)^2
template <typename T> void gloc_field(long n, const T* phi, T* G, hipStream_t s);
// x = unit impulse at index 0
void set_delta(long n, double* x, hipStream_t s);
// out[0] = sum |x_i|
void reduce_abs_sum(long n, const double* x, double* part, double* out, hipStream_t s);

// ------------------------------------------------------------------ fixed membrane (FP64)
struct FixedK {
    double eps_u, gamma, ubar, M, B;
    int with_ubar;
};
void fixed_prep(const GridK& g, const double* gg, double* sg, double* isg, hipStream_t s);
// H row bound: out[i] = H_ii + sum_j |H_ij|; reduced with max.
void fixed_gershgorin(const GridK& g, const double* gg, const double* isg, double* part, double* out,
                      hipStream_t s);
// The band of a step restricted to {g >= delta} (the narrow-band fixed-membrane
// step), as the operator kernels take it: gf = g on the band, -1 off it.
void fixed_band_field(long n, const double* G, double delta, double* gf, hipStream_t s);
// q = g f(U) (or g (f(U) - ubar)); mq = g (f(U) - ubar) (for the mass integral);
// gf (nullable): both 0 off the band of a restricted step
void fixed_nonlocal_arg(long n, const FixedK& K, const double* gg, const double* U, double* q, double* mq,
                        const double* gf, hipStream_t s);
// R = B sg U - sg W'(U)/eps_u - gamma sg psi f'(U) - M m sg f'(U); gf (nullable):
// off the band of a restricted step R = B (sg U).  With Rprev (nullable) R
// receives that value minus Rprev (the difference the second ETDRK2 stage uses).
template <typename TP>
void fixed_remainder(long n, const FixedK& K, const double* sg, const double* U, const TP* psi,
                     const double* m, double* R, const double* gf, hipStream_t s, const double* Rprev = nullptr);
// y = alpha * Atil x - beta * xprev  (Atil = (2 L - (a + b)) / (b - a), L = B + eps_u H),
// acc (+)= c * y.  xprev may be null when beta == 0.  first != 0: acc = c0 * x + c * y.
void fixed_cheb_step(const GridK& g, const FixedK& K, const double* gg, const double* isg, double a, double b,
                     double alpha, double beta, const double* x, const double* xprev, double* y, double* acc,
                     double c, double c0, int first, hipStream_t s);
// Two terms at once (3D grids, fixed_cheb_pair_supported): y1 = alpha Atil x -
// beta xprev, y2 = alpha Atil y1 - beta x, acc += c1 y1, then acc += c2 y2.
// y1, y2 must not alias x, xprev or each other.
bool fixed_cheb_pair_supported(const GridK& g);
void fixed_cheb_pair(const GridK& g, const FixedK& K, const double* gg, const double* isg, double a, double b,
                     double alpha, double beta, const double* x, const double* xprev, double* y1, double* y2,
                     double* acc, double c1, double c2, hipStream_t s);
// out = L x, or with r (nullable) out = r - L x
void fixed_L_apply(const GridK& g, const FixedK& K, const double* gg, const double* isg, const double* x,
                   double* out, hipStream_t s, const double* r = nullptr);
// w = w + tau acc, then U = isg w (on the band only when gf is given); a no-op
// once *halt != 0
void fixed_advance(long n, double tau, const double* acc, double* w, const double* isg, double* U,
                   const double* halt, const double* gf, hipStream_t s);
// elementwise helpers
// out = x * y; a no-op once *halt != 0 (halt nullable); with gf (nullable) only
// on the band of a restricted step (gf >= 0)
void mul(long n, const double* x, const double* y, double* out, hipStream_t s, const double* halt = nullptr,
         const double* gf = nullptr);
// Fixed energy sums: out = [sum g_half (D+U)^2 (edges), sum g W(U), sum psi q, sum g (f(U) - ubar)] (unscaled)
void reduce_energy_fixed(const GridK& g, const FixedK& K, const double* gg, const double* U, const double* psi,
                         const double* q, double* part, double* out, hipStream_t s);
// Mass projection: U += c on {g > thr}, c = (Q0 - h^d sum g U) / (h^d sum_{g > thr} g), read from sums[0..1].
template <typename T>
void mass_project_sums(long n, const T* G, const T* U, double thr, double* part, double* out, hipStream_t s);
template <typename T>
void mass_project_apply(long n, const T* G, T* U, double thr, double cell, const double* Q0,
                        const double* sums, const double* halt, hipStream_t s);

// ------------------------------------------------------------------ narrow band
// flags[i] = |2 phi_i - 1| < thr (FP64); counts per block, exclusive scan, stable scatter.
template <typename T>
void band_flags(long n, const T* phi, double thr, uint8_t* flags, hipStream_t s);
// (-Delta_S,h)^{-1} on a narrow band (surface.hip): FP64 conjugate gradients
// (single-reduction form) with a Chebyshev polynomial preconditioner over the
// band list
// idx[0 .. *total) of mask.  Workspace
// carved from one device allocation of surface_work_bytes(n) bytes (its own
// band list buffers idx / cnt / total serve callers without one).
struct SurfaceWork {
    double *x = nullptr, *u = nullptr;                                                // grid layout
    double *r = nullptr, *p = nullptr, *s = nullptr, *w = nullptr, *dinv = nullptr;   // band order
    double *cres = nullptr, *cz = nullptr;   // preconditioner residual and sum (band order)
    double *dA = nullptr, *dB = nullptr;     // preconditioner directions (grid layout)
    double* gm = nullptr;                    // g on the band, -1 off it (grid layout, element type of g)
    int32_t* idx = nullptr;
    int64_t *cnt = nullptr, *total = nullptr;
    double *part = nullptr, *S = nullptr;
};
struct SurfaceResult {
    int iters = 0;
    double relres = 0.0;
    bool converged = false;
};
// mask[i] = G[i] >= delta (the band {g >= delta} of Section 3.2).
template <typename T> void band_ge(long n, const T* G, double delta, uint8_t* mask, hipStream_t s);
size_t surface_work_bytes(long n);
void surface_work_carve(long n, void* base, SurfaceWork& w);
// psi = (-Delta_S,h)^{-1} f on the band (0 off it); stops when the residual
// relative to f - mean_band(f) reaches tol or after max_iter iterations.
// warm: start from w.x as the previous solve left it (its result on its band,
// 0 elsewhere; all 0 before the first solve), else from 0.  Synchronizes the
// stream every 25 iterations (convergence check); res (nullable) gets the
// outcome.
template <typename T>
hipError_t surface_lapinv(const GridK& g, const T* G, const T* f, const uint8_t* mask, const int32_t* idx,
                          const int64_t* total, T* psi, const SurfaceWork& w, double tol, int max_iter, bool warm,
                          SurfaceResult* res, hipStream_t s);

// Per-step diagnostics ring: one entry (kDiagRingFields doubles: step, the
// seven diagnostics sums of reduce_diag with the minimum's sign restored,
// band count, non-finite flag) pushed into slot meta[0] mod cap, meta[0]
// then incremented; the step is meta[1] + meta[0] + 1.  One thread.
constexpr int kDiagRingFields = 9;
void diag_ring_push(const double* diag, const double* halt, const int64_t* band_total, double* ring, int cap,
                    int64_t* meta, hipStream_t s);

// Compact flagged indices in ascending order.  blockcnt: scratch of band_blocks(n) + 1 int64.
long band_blocks(long n);
void band_compact(long n, const uint8_t* flags, int64_t* blockcnt, int32_t* idx_out, int64_t capacity,
                  int64_t* total_dev, hipStream_t s);
// The same list for |2 phi - 1| < thr with no device memory of its own beyond a
// static per-device scratch array (band.hip): band_static_init(device) looks up
// that device's copy once (the device is made current for the lookup);
// band_build_static then runs the flag, count, scan and scatter kernels on s
// with the flags formed where they are read, copies the count to *count_host
// and synchronizes s.  At most band_static_max_points() points.  Calls on one
// device share the array: calls that overlap in time race.
long band_static_max_points();
hipError_t band_static_init(int device);
template <typename T>
hipError_t band_build_static(int device, long n, const T* phi, double thr, int32_t* idx_out, int64_t capacity,
                             int64_t* count_host, hipStream_t s);

}  // namespace etd
