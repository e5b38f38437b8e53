// Host runtime of the C ABI: validation, plan/workspace management, the step
// schedules of both models, Chebyshev set-up, energies and diagnostics.
#include <hip/hip_runtime.h>

#include <rocprofiler-sdk-roctx/roctx.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "fused.h"
#include "plan.h"

using namespace etd;

namespace etd {

std::string g_last_error = "";

namespace {
int env_int(const char* name, int dflt) {
    const char* v = std::getenv(name);
    return (v && *v) ? std::atoi(v) : dflt;
}
}  // namespace

int log_level() {
    static const int level = std::min(2, std::max(0, env_int("ETD_LOG", 0)));
    return level;
}

void log_msg(int level, const char* fmt, ...) {
    if (level > log_level()) return;
    std::fprintf(stderr, "[etd] ");
    va_list ap;
    va_start(ap, fmt);
    std::vfprintf(stderr, fmt, ap);
    va_end(ap);
    std::fputc('\n', stderr);
}

etd_status fail(std::string* sink, etd_status st, const std::string& msg) {
    g_last_error = msg;
    if (sink) *sink = msg;
    log_msg(1, "error %d: %s", (int)st, msg.c_str());
    return st;
}

StageRange::StageRange(const char* name) {
    static const bool enabled = env_int("ETD_ROCTX", 1) != 0;
    on_ = enabled;
    if (on_) roctxRangePushA(name);
}

StageRange::~StageRange() {
    if (on_) roctxRangePop();
}

}  // namespace etd

namespace {

bool finite_pos(double x) { return std::isfinite(x) && x > 0.0; }

// Launch a non-FFT kernel under the pass-timing hook (kind: PassKind; bytes:
// algorithmic bytes it moves).
template <typename F> void timed_kernel(int kind, double bytes, hipStream_t s, F&& launch) {
    (void)timed_pass(kind, bytes, s, [&] {
        launch();
        return hipSuccess;
    });
}

etd_status validate(const etd_instance_desc& d, std::string& msg) {
    if (d.model != ETD_COUPLED && d.model != ETD_FIXED_MEMBRANE) { msg = "unknown model"; return ETD_E_ARG; }
    if (d.scheme != ETD_ETD1 && d.scheme != ETD_ETDRK2) { msg = "unknown scheme"; return ETD_E_ARG; }
    if (d.precision != ETD_FP64 && d.precision != ETD_FP32) { msg = "unknown precision"; return ETD_E_ARG; }
    if (d.grid.dim != 2 && d.grid.dim != 3) { msg = "grid.dim must be 2 or 3"; return ETD_E_ARG; }
    for (int k = 0; k < d.grid.dim; ++k) {
        const int n = d.grid.n[k];
        if (n < 8 || n > 512 || (n % 2) != 0) { msg = "grid.n must be even and in [8, 512]"; return ETD_E_SIZE; }
        if (!fft_length_supported(n)) { msg = "grid.n must be 2^a or 3*2^a"; return ETD_E_SIZE; }
        if (!finite_pos(d.grid.half_len[k])) { msg = "grid.half_len must be finite and > 0"; return ETD_E_ARG; }
    }
    if (!finite_pos(d.tau)) { msg = "tau must be finite and > 0"; return ETD_E_ARG; }
    if (!std::isfinite(d.recover_threshold) || d.recover_threshold < 0.0) {
        msg = "recover_threshold must be finite and >= 0"; return ETD_E_ARG;
    }
    if (!std::isfinite(d.band_threshold) || d.band_threshold < 0.0) {
        msg = "band_threshold must be finite and >= 0"; return ETD_E_ARG;
    }
    if (d.band_threshold > 0.0 && d.band_rebuild_every < 1) { msg = "band_rebuild_every must be >= 1"; return ETD_E_ARG; }
    if (d.flags & ~(ETD_F_MASS_PROJECT | ETD_F_FROZEN_MEMBRANE | ETD_F_SURFACE_NONLOCAL | ETD_F_BAND_STEP)) {
        msg = "unknown flag bits"; return ETD_E_ARG;
    }
    if ((d.flags & ETD_F_SURFACE_NONLOCAL) && !(d.band_threshold > 0.0)) {
        msg = "ETD_F_SURFACE_NONLOCAL needs a band (band_threshold > 0)"; return ETD_E_ARG;
    }
    if ((d.flags & ETD_F_FROZEN_MEMBRANE) && d.model != ETD_COUPLED) {
        msg = "ETD_F_FROZEN_MEMBRANE applies to the coupled model only"; return ETD_E_ARG;
    }
    if ((d.flags & ETD_F_BAND_STEP) && (d.model != ETD_FIXED_MEMBRANE || !(d.band_threshold > 0.0))) {
        msg = "ETD_F_BAND_STEP applies to the fixed model and needs band_threshold > 0"; return ETD_E_ARG;
    }
    long total = 1;
    for (int k = 0; k < d.grid.dim; ++k) total *= d.grid.n[k];
    if (total >= (1L << 31)) { msg = "grid too large for int32 band indices"; return ETD_E_SIZE; }
    if (d.model == ETD_COUPLED) {
        if (!d.coupled) { msg = "coupled parameters missing"; return ETD_E_ARG; }
        const etd_coupled_params& p = *d.coupled;
        const double all[] = {p.mu, p.lambda_surf, p.kappa, p.lambda_line, p.M_area, p.alpha, p.u0, p.eps_phi,
                              p.eps_u, p.gamma, p.ubar, p.M, p.A1, p.A2, p.B1, p.B2, p.A0};
        for (double v : all)
            if (!std::isfinite(v)) { msg = "non-finite coupled parameter"; return ETD_E_ARG; }
        if (!(p.mu > 0 && p.eps_phi > 0 && p.eps_u > 0)) { msg = "mu, eps_phi, eps_u must be > 0"; return ETD_E_ARG; }
        if (p.B2 < 0 || p.B1 < 0 || p.A1 < 0 || p.A2 < 0) { msg = "stabilizers must be >= 0"; return ETD_E_ARG; }
    } else {
        if (!d.fixed) { msg = "fixed-membrane parameters missing"; return ETD_E_ARG; }
        const etd_fixed_params& p = *d.fixed;
        const double all[] = {p.eps_u, p.gamma, p.ubar, p.M, p.B};
        for (double v : all)
            if (!std::isfinite(v)) { msg = "non-finite fixed parameter"; return ETD_E_ARG; }
        if (!(p.eps_u > 0)) { msg = "eps_u must be > 0"; return ETD_E_ARG; }
        if (p.gamma < 0 || p.M < 0) { msg = "gamma and M must be >= 0"; return ETD_E_ARG; }
    }
    return ETD_OK;
}

GridK make_grid(const etd_grid& gr) {
    GridK g{};
    g.dim = gr.dim;
    if (gr.dim == 2) {
        g.nx = 1;
        g.ny = gr.n[0];
        g.nz = gr.n[1];
        g.X[0] = 1.0;
        g.X[1] = gr.half_len[0];
        g.X[2] = gr.half_len[1];
    } else {
        g.nx = gr.n[0];
        g.ny = gr.n[1];
        g.nz = gr.n[2];
        g.X[0] = gr.half_len[0];
        g.X[1] = gr.half_len[1];
        g.X[2] = gr.half_len[2];
    }
    g.nzh = g.nz / 2 + 1;
    g.h[0] = g.nx > 1 ? 2.0 * g.X[0] / g.nx : 1.0;
    g.h[1] = 2.0 * g.X[1] / g.ny;
    g.h[2] = 2.0 * g.X[2] / g.nz;
    g.cell = (g.nx > 1 ? g.h[0] : 1.0) * g.h[1] * g.h[2];
    return g;
}

double domain_volume(const GridK& g) {
    return (g.nx > 1 ? 2.0 * g.X[0] : 1.0) * 2.0 * g.X[1] * 2.0 * g.X[2];
}

etd_status dalloc(etd_plan* P, Instance& I, size_t bytes, void** out) {
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
        return fail(&P->err, ETD_E_NOMEM, "hipMalloc(" + std::to_string(bytes) + "): " + hipGetErrorString(e));
    }
    I.allocs.push_back(p);
    I.bytes += bytes;
    *out = p;
    return ETD_OK;
}

#define ALLOC(ptr, bytes)                                                 \
    do {                                                                  \
        void* tmp_ = nullptr;                                             \
        etd_status st_ = dalloc(P, I, (bytes), &tmp_);                    \
        if (st_ != ETD_OK) return st_;                                    \
        ptr = reinterpret_cast<decltype(ptr)>(tmp_);                      \
    } while (0)

// Workspace of the band solve, allocated once per instance; its iterate
// starts at 0 (the first warm-started solve starts cold).
etd_status ensure_surface(etd_plan* P, Instance& I) {
    if (I.surf) return ETD_OK;
    const long n = I.g.nreal();
    ALLOC(I.surf, surface_work_bytes(n));
    surface_work_carve(n, I.surf, I.sw);
    HIPCHK(P, hipMemsetAsync(I.sw.x, 0, sizeof(double) * (size_t)n, P->stream));
    return ETD_OK;
}

template <typename T> etd_status upload_table(etd_plan* P, Instance& I, int n, const c2<T>** out) {
    std::vector<double> h(2 * (size_t)n);
    fft_twiddles_host(n, h.data());
    std::vector<T> hv(2 * (size_t)n);
    for (size_t k = 0; k < h.size(); ++k) hv[k] = (T)h[k];
    c2<T>* d = nullptr;
    ALLOC(d, sizeof(c2<T>) * (size_t)n);
    HIPCHK(P, hipMemcpy(d, hv.data(), sizeof(c2<T>) * (size_t)n, hipMemcpyHostToDevice));
    *out = d;
    return ETD_OK;
}

template <typename T> etd_status make_tables(etd_plan* P, Instance& I, FFTTables<T>& t) {
    etd_status st;
    if (I.g.nx > 1 && (st = upload_table<T>(P, I, I.g.nx, &t.tx)) != ETD_OK) return st;
    if ((st = upload_table<T>(P, I, I.g.ny, &t.ty)) != ETD_OK) return st;
    if ((st = upload_table<T>(P, I, I.g.nz / 2, &t.tzh)) != ETD_OK) return st;
    if ((st = upload_table<T>(P, I, I.g.nz, &t.tzf)) != ETD_OK) return st;
    return ETD_OK;
}

// ------------------------------------------------------------------ Chebyshev (host, FP64)
double phi1_host(double z) { return std::fabs(z) < 1e-5 ? 1.0 - z / 2.0 + z * z / 6.0 : -std::expm1(-z) / z; }
double phi2_host(double z) {
    if (std::fabs(z) < 0.1) {
        double out = 0.0, fact = 1.0;
        double c[20];
        fact = 0.5;
        c[0] = fact;
        for (int j = 1; j < 16; ++j) c[j] = c[j - 1] / (double)(j + 2);
        for (int j = 15; j >= 0; --j) out = out * (-z) + c[j];
        return out;
    }
    return (std::expm1(-z) + z) / (z * z);
}

// Chebyshev coefficients of x -> f(tau x) on [a, b]: f ~ c_0/2 + sum_k c_k T_k(t),
// t = (2x - a - b)/(b - a), from M samples at the Chebyshev points (a DCT in
// long double).  The series is kept up to the last coefficient above
// 2e-16 max|f| plus two more (the DCT's own rounding leaves |c_k| ~ 1e-17
// max|f| in the tail); M doubles from 512 until that index lies in the first
// half of the M computed coefficients (so aliasing has not folded the tail
// back), up to 8192.  Returns an empty vector when even 8192 samples do not
// resolve the series (an operator spectrum too wide for the expansion).
std::vector<double> cheb_coeffs(double (*f)(double), double tau, double a, double b) {
    for (int M = 512; M <= 8192; M *= 2) {
        std::vector<double> F(M), c(M);
        double fmax = 0.0;
        for (int j = 0; j < M; ++j) {
            const double th = kPi * (j + 0.5) / M;
            const double x = 0.5 * (a + b) + 0.5 * (b - a) * std::cos(th);
            F[j] = f(tau * x);
            fmax = std::fmax(fmax, std::fabs(F[j]));
        }
        for (int k = 0; k < M; ++k) {
            long double s = 0.0L;
            for (int j = 0; j < M; ++j) s += (long double)F[j] * cosl((long double)kPi * k * (j + 0.5L) / M);
            c[k] = (double)(2.0L * s / M);
        }
        int K = 1;
        for (int k = 0; k < M; ++k)
            if (std::fabs(c[k]) > 2e-16 * fmax) K = k;
        if (K + 2 < M / 2) {
            c.resize(K + 3);
            return c;
        }
    }
    return {};
}

// ------------------------------------------------------------------ instance set-up
etd_status setup_coupled(etd_plan* P, Instance& I) {
    const GridK& g = I.g;
    const size_t nr = (size_t)g.nreal(), ns = (size_t)g.nspec();
    const size_t es = I.f32 ? sizeof(float) : sizeof(double);
    const size_t cs = 2 * es;
    void** reals[] = {&I.phiA, &I.phiB, &I.u, &I.ut, &I.lap, &I.gx, &I.P, &I.Q, &I.gp, &I.vx, &I.vy, &I.vz,
                      &I.psi};
    for (void** r : reals) ALLOC(*r, nr * es);
    if (I.g.nx == 1) {   // two-dimensional grids keep all gradient components
        ALLOC(I.gy, nr * es);
        ALLOC(I.gz, nr * es);
    }
    void** specs[] = {&I.Sphi, &I.St, &I.Sra, &I.Sa, &I.Sb, &I.Sgu, &I.Stmp};
    for (void** r : specs) ALLOC(*r, ns * cs);
    ALLOC(I.mask, nr);
    ALLOC(I.band_idx, nr * sizeof(int32_t));
    ALLOC(I.band_cnt, (band_blocks((long)nr) + 2) * sizeof(int64_t));
    ALLOC(I.band_total, sizeof(int64_t));
    etd_status st = I.f32 ? make_tables<float>(P, I, I.tf) : make_tables<double>(P, I, I.td);
    if (st != ETD_OK) return st;
    const etd_coupled_params& p = I.cp;
    CoupledK& K = I.K;
    K.mu = p.mu; K.lambda_surf = p.lambda_surf; K.kappa = p.kappa; K.lambda_line = p.lambda_line;
    K.M_area = p.M_area; K.alpha = p.alpha; K.u0 = p.u0; K.eps_phi = p.eps_phi; K.eps_u = p.eps_u;
    K.gamma = p.gamma; K.ubar = p.ubar; K.M = p.M; K.A1 = p.A1; K.A2 = p.A2; K.B1 = p.B1; K.B2 = p.B2;
    K.tau = I.d.tau;
    const double e2 = p.eps_phi * p.eps_phi;
    K.c1 = p.kappa / (p.mu * e2);
    K.lp4 = p.kappa / p.mu;
    K.lp2 = (p.kappa * (p.A1 + p.A2) + p.lambda_surf * e2) / (p.mu * e2);
    K.lp0 = (p.kappa * p.A1 * p.A2 + p.lambda_surf * p.A1 * e2) / (p.mu * e2 * e2);
    K.thr = I.d.recover_threshold;
    if (I.d.flags & ETD_F_SURFACE_NONLOCAL) return ensure_surface(P, I);
    return ETD_OK;
}

etd_status setup_fixed(etd_plan* P, Instance& I) {
    const GridK& g = I.g;
    const size_t nr = (size_t)g.nreal(), ns = (size_t)g.nspec();
    double** reals[] = {&I.G, &I.sg, &I.isg, &I.U, &I.w, &I.R0, &I.vv, &I.t1, &I.t2, &I.acc, &I.q, &I.mq,
                        &I.psid};
    for (double** r : reals) ALLOC(*r, nr * sizeof(double));
    if (fixed_cheb_pair_supported(g)) {
        ALLOC(I.t3, nr * sizeof(double));
        ALLOC(I.t4, nr * sizeof(double));
    }
    if (I.d.flags & ETD_F_BAND_STEP) ALLOC(I.gf, nr * sizeof(double));
    else I.gf = I.G;
    ALLOC(I.Sa, ns * sizeof(double2));
    ALLOC(I.Stmp, ns * sizeof(double2));
    etd_status st = make_tables<double>(P, I, I.td);
    if (st != ETD_OK) return st;
    if (I.f32) {
        ALLOC(I.qf, nr * sizeof(float));
        ALLOC(I.psif, nr * sizeof(float));
        ALLOC(I.Sb, ns * sizeof(float2));
        ALLOC(I.Sgu, ns * sizeof(float2));
        if ((st = make_tables<float>(P, I, I.tf)) != ETD_OK) return st;
    }
    if (I.d.flags & ETD_F_SURFACE_NONLOCAL) {   // band {g >= band_threshold}, listed at set_state
        ALLOC(I.mask, nr);
        ALLOC(I.band_idx, nr * sizeof(int32_t));
        ALLOC(I.band_cnt, (band_blocks((long)nr) + 2) * sizeof(int64_t));
        ALLOC(I.band_total, sizeof(int64_t));
        if ((st = ensure_surface(P, I)) != ETD_OK) return st;
    }
    const etd_fixed_params& p = I.fp;
    I.FK.eps_u = p.eps_u; I.FK.gamma = p.gamma; I.FK.ubar = p.ubar; I.FK.M = p.M;
    I.FK.with_ubar = p.nonlocal_with_ubar ? 1 : 0;
    // C = sum_j |a_j| with a = IDFT(1/mu) (zero mode removed): the column of the
    // pseudo-inverse at index 0, i.e. (-Delta_h)^{-1} of a unit impulse.
    hipStream_t s = P->stream;
    set_delta(g.nreal(), I.q, s);
    HIPCHK(P, fft_r2c_3d<double>(g, I.td, I.q, (double2*)I.Sa, s));
    spec_apply<double>(g, SPEC_INV_FD, (const double2*)I.Sa, (double2*)I.Sa, I.fd, s);
    HIPCHK(P, fft_c2r_3d<double>(g, I.td, (const double2*)I.Sa, (double2*)I.Stmp, I.psid, s));
    reduce_abs_sum(g.nreal(), I.psid, I.part, I.scal + S_ABS, s);
    HIPCHK(P, hipGetLastError());
    double C = 0.0;
    HIPCHK(P, hipMemcpyAsync(&C, I.scal + S_ABS, sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(P, hipStreamSynchronize(s));
    I.C = C;
    const double vol = domain_volume(g);
    const double LW2 = 36.0, LF2 = 6.0, LF1 = 1.5, LG = 9.0 / 8.0;
    I.Bmbp = LW2 / p.eps_u + p.gamma * C * LF2 * LG + p.M * vol * LF2 * LG;
    I.Bes = LW2 / p.eps_u + (0.5 * p.gamma * C + 0.5 * p.M * vol) * (LF2 + LF1 * LF1) * LG;
    I.FK.B = p.B > 0.0 ? p.B : I.Bmbp;
    return ETD_OK;
}

etd_status setup_common(etd_plan* P, Instance& I) {
    ALLOC(I.scal, S_COUNT * sizeof(double));
    // reduction partials: the fixed reduction grid, or one per z-row tile of the fused z pass
    ALLOC(I.part, std::max((size_t)kRedBlocks * 8, (size_t)I.g.nx * I.g.ny) * sizeof(double));
    HIPCHK(P, hipMemset(I.scal, 0, S_COUNT * sizeof(double)));
    // eigenvalues of the periodic second difference per axis, mu_d(i) = (4/h^2) sin^2(pi i / N)
    const GridK& g = I.g;
    const int ns[3] = {g.nx, g.ny, g.nz};
    std::vector<double> fd;
    for (int d = 0; d < 3; ++d)
        for (int i = 0; i < ns[d]; ++i) {
            if (ns[d] == 1) {
                fd.push_back(0.0);
                continue;
            }
            const long double sn = sinl(3.141592653589793238462643383279502884L * i / ns[d]);
            fd.push_back((double)(4.0L / ((long double)g.h[d] * g.h[d]) * sn * sn));
        }
    ALLOC(I.fd, fd.size() * sizeof(double));
    HIPCHK(P, hipMemcpy(I.fd, fd.data(), fd.size() * sizeof(double), hipMemcpyHostToDevice));
    return ETD_OK;
}

etd_status check_instance(etd_plan* plan, int instance) {
    if (!plan) return fail(nullptr, ETD_E_ARG, "null plan");
    if (instance < 0 || instance >= (int)plan->inst.size())
        return fail(&plan->err, ETD_E_ARG, "instance out of range");
    return ETD_OK;
}

// ------------------------------------------------------------------ coupled step
// Three-dimensional grids keep only |grad phi| (gn, in the gx buffer): the
// fused derivative pass reduces the gradient to its norm, the only form R1
// and the energy use; two-dimensional grids keep the components gx, gy, gz.
template <typename T> struct CoupledView {
    T *phiA, *phiB, *u, *ut, *lap, *gx, *gy, *gz, *gn, *P, *Q, *gp, *vx, *vy, *vz, *psi;
    c2<T> *Sphi, *St, *Sra, *Sa, *Sb, *Sgu, *Stmp;
    explicit CoupledView(Instance& I) {
        phiA = (T*)I.phiA; phiB = (T*)I.phiB; u = (T*)I.u; ut = (T*)I.ut; lap = (T*)I.lap; gx = (T*)I.gx;
        gn = (T*)I.gx;
        gy = (T*)I.gy; gz = (T*)I.gz; P = (T*)I.P; Q = (T*)I.Q; gp = (T*)I.gp; vx = (T*)I.vx; vy = (T*)I.vy;
        vz = (T*)I.vz; psi = (T*)I.psi;
        Sphi = (c2<T>*)I.Sphi; St = (c2<T>*)I.St; Sra = (c2<T>*)I.Sra; Sa = (c2<T>*)I.Sa; Sb = (c2<T>*)I.Sb;
        Sgu = (c2<T>*)I.Sgu; Stmp = (c2<T>*)I.Stmp;
    }
};

// Grid sum of cell-weighted values into a device scalar slot.
GridSum grid_sum(const Instance& I, int slot) { return GridSum{I.part, I.scal + slot, I.g.cell, I.scal + S_HALT}; }
double* halt_flag(const Instance& I) { return I.scal + S_HALT; }

template <typename T> const FFTTables<T>& tables(const Instance& I);
template <> const FFTTables<float>& tables<float>(const Instance& I) { return I.tf; }
template <> const FFTTables<double>& tables<double>(const Instance& I) { return I.td; }

// phi and its spectral derivatives from a spectrum: out phi, lap and the
// gradient (its norm in the gx buffer on three-dimensional grids, the
// components gx, gy, gz on two-dimensional ones).
// Three-dimensional grids take the fused three-pass pipeline with the work
// spectra Sa, Sb, Sgu, Stmp (S must be none of them); two-dimensional grids
// take one c2r per field.
template <typename T>
hipError_t phi_and_derivs(const Instance& I, CoupledView<T>& v, const c2<T>* S, T* phi, hipStream_t s) {
    const GridK& g = I.g;
    const FFTTables<T>& t = tables<T>(I);
    if (g.nx > 1) {
        const GridSum isum = grid_sum(I, S_INTPHI);
        return derivs_fused<T>(g, t, S, v.Sa, v.Sb, v.Sgu, v.Stmp, phi, v.gn, v.lap, &isum, s);
    }
    hipError_t e = fft_c2r_3d<T>(g, t, S, v.Stmp, phi, s);
    if (e != hipSuccess) return e;
    const SpecOp ops[4] = {SPEC_NEG_K2, SPEC_IKX, SPEC_IKY, SPEC_IKZ};
    T* outs[4] = {v.lap, v.gx, v.gy, v.gz};
    for (int k = 0; k < 4; ++k) {
        spec_apply<T>(g, ops[k], S, v.Sa, I.fd, s);
        if ((e = fft_c2r_3d<T>(g, t, v.Sa, v.Stmp, outs[k], s)) != hipSuccess) return e;
    }
    return hipGetLastError();
}

// Two-dimensional grids: forward transforms of the remainder pair (P, Q)
// and the ETD combine of the stage as a separate spectral kernel.
template <typename T>
hipError_t remainder_etd_2d(const Instance& I, CoupledView<T>& v, EtdStage st, const EtdArgs<T>& a, hipStream_t s) {
    const GridK& g = I.g;
    const FFTTables<T>& t = tables<T>(I);
    hipError_t e = fft_r2c_3d<T>(g, t, v.P, v.Sa, s);
    if (e != hipSuccess) return e;
    if ((e = fft_r2c_3d<T>(g, t, v.Q, v.Sb, s)) != hipSuccess) return e;
    switch (st) {
        case ETD_STAGE_PHI1: spec_etd_phi1<T>(g, I.K, v.Sa, v.Sb, a.prev, a.ra, a.out, a.halt, s); break;
        case ETD_STAGE_PHI2: spec_etd_phi2<T>(g, I.K, v.Sa, v.Sb, a.prev, a.ra, a.out, a.halt, s); break;
        case ETD_STAGE_U1: spec_etd_u1<T>(g, I.K, v.Sa, v.Sb, a.out, a.ra, a.halt, s); break;
        case ETD_STAGE_U2: spec_etd_u2<T>(g, I.K, v.Sa, v.Sb, a.out, a.ra, a.halt, s); break;
    }
    return hipGetLastError();
}

// One phi stage: R1 at (phi_in, its derivatives, u^n), the ETD combine into
// the spectrum a.out and, in real space, phi_out with its derivatives (lap
// and the gradient, its norm only on three-dimensional grids, where the
// integral of phi_out is formed too).  On
// three-dimensional grids R1 is formed in the load of the z pass and the x
// pass of the pair also runs the inverse x transforms of the derivatives.
// With vel (three-dimensional grids, the last stage of a step) the final
// derivative pass also writes g+ and the velocity at phi_out.
template <typename T>
hipError_t phi_stage(const Instance& I, CoupledView<T>& v, const T* phi_in, const uint8_t* mask, EtdStage st,
                     const EtdArgs<T>& a, T* phi_out, hipStream_t s, const VelocityArgs<T>* vel = nullptr) {
    const GridK& g = I.g;
    const FFTTables<T>& t = tables<T>(I);
    if (g.nx > 1) {
        R1Fields<T> f{phi_in, v.lap, v.gn, v.u, mask, I.scal + S_INTPHI, I.A0};
        if (mask) {   // the surface part of P1 on the band list (into the P buffer, free in 3D)
            timed_kernel(PASS_R1, 0.0, s, [&] {
                r1_surface_band<T>(g, I.K, phi_in, v.lap, v.gn, v.u, I.band_idx, I.band_total, g.nreal(),
                                   I.scal + S_INTPHI, I.A0, v.P, s);
            });
            f.surf = v.P;
        }
        hipError_t e = r1_etd<T>(g, t, I.K, f, st, v.Sa, v.Sb, a, true, v.Sa, v.Sb, v.Sgu, s);
        if (e != hipSuccess) return e;
        const GridSum isum = grid_sum(I, S_INTPHI);
        return derivs_fused_yz<T>(g, t, v.Sa, v.Sb, v.Sgu, v.Stmp, phi_out, v.gn, v.lap, &isum, s, vel);
    }
    const long n = g.nreal();
    const double fb = (double)sizeof(T) * n, mb = mask ? (double)n : 0.0;
    timed_kernel(PASS_REDUCE, fb, s, [&] {
        reduce_sum<T>(n, phi_in, g.cell, I.part, I.scal + S_INTPHI, s, halt_flag(I));
    });
    timed_kernel(PASS_R1, 8.0 * fb + mb, s, [&] {
        coupled_R1_point<T>(g, I.K, phi_in, v.lap, v.gx, v.gy, v.gz, v.u, mask, I.scal + S_INTPHI, I.A0, v.P, v.Q,
                            s);
    });
    hipError_t e = remainder_etd_2d<T>(I, v, st, a, s);
    if (e != hipSuccess) return e;
    return phi_and_derivs<T>(I, v, a.out, phi_out, s);
}

// One u stage: q = g (u - ubar) (masked) -> P; m = h^3 sum q;
// psi = (-Delta_h)^{-1} q; P2(u) and g+ u; their transforms, the combine into
// the increment D (Sgu; stored if store_D) and Sra, and the recovery
// out = rec(g+ u^n + F^-1 D).  On three-dimensional grids P2 and g+ u are
// formed in the load of the z pass.
template <typename T>
hipError_t u_stage(Instance& I, CoupledView<T>& v, const T* uu, const uint8_t* mask, EtdStage st, bool store_D,
                   T* out, hipStream_t s) {
    const GridK& g = I.g;
    const FFTTables<T>& t = tables<T>(I);
    const long n = g.nreal();
    const double fb = (double)sizeof(T) * n, mb = mask ? (double)n : 0.0;
    const EtdArgs<T> a{nullptr, v.Sra, v.Sgu, halt_flag(I), I.xlines};
    hipError_t e = hipSuccess;
    const bool surface = (I.d.flags & ETD_F_SURFACE_NONLOCAL) != 0;
    // band solve of the nonlocal term: q and m pointwise, psi = (-Delta_S,h)^{-1} q on the band
    auto surface_psi = [&]() -> hipError_t {
        StageRange r("etd.band_solve");
        timed_kernel(PASS_POINT, 3.0 * fb + mb, s, [&] {
            coupled_q_gu<T>(g, I.K, uu, v.gp, mask, v.P, nullptr, I.part, I.scal + S_MASS, halt_flag(I), s);
        });
        const double tol = I.f32 ? 1e-9 : 1e-12;
        return surface_lapinv<T>(g, v.gp, v.P, mask, I.band_idx, I.band_total, v.psi, I.sw, tol, 20000, true,
                                 &I.surf_last, s);
    };
    if (g.nx > 1) {
        // q formed in the load of the nonlocal transform (with m), whose last (z)
        // pass runs inside the P2 pass; P2 and g+ u in the load of the pair
        // with the band, P2 reads psi at band points only: psi's inverse z
        // transform runs as its own plain pass instead of inside every P2 tile
        e = surface ? surface_psi()
                    : lapinv_q_fused<T>(g, t, I.fd, I.K.ubar, uu, v.gp, mask, v.Stmp, mask ? v.psi : nullptr,
                                        grid_sum(I, S_MASS), s);
        if (e != hipSuccess) return e;
        P2Fields<T> f{uu, v.gp, v.vx, v.vy, v.vz, v.psi, mask, I.scal + S_MASS, (surface || mask) ? nullptr : v.Stmp};
        if (mask) {   // P2 without its nonlocal term on the band list (into the Q buffer, free in 3D)
            timed_kernel(PASS_P2, 0.0, s, [&] {
                p2_local_band<T>(g, I.K, uu, v.gp, v.vx, v.vy, v.vz, I.band_idx, I.band_total, g.nreal(),
                                 I.scal + S_MASS, v.Q, s);
            });
            f.surf = v.Q;
        }
        e = p2_etd<T>(g, t, I.K, f, st, v.Sa, v.Sb, a, store_D, v.Sa, s);
        if (e != hipSuccess) return e;
        return c2r_recover_yz<T>(g, t, v.Sa, v.u, v.gp, out, I.K.thr, halt_flag(I), s);
    }
    timed_kernel(PASS_POINT, 4.0 * fb + mb, s, [&] {
        coupled_q_gu<T>(g, I.K, uu, v.gp, mask, v.P, v.Q, I.part, I.scal + S_MASS, halt_flag(I), s);
    });
    if ((e = lapinv_fused<T>(g, t, I.fd, v.P, v.Sa, v.psi, s)) != hipSuccess) return e;
    timed_kernel(PASS_P2, 7.0 * fb + mb, s, [&] {
        coupled_P2_point<T>(g, I.K, uu, v.gp, v.vx, v.vy, v.vz, v.psi, I.scal + S_MASS, mask, v.P, s);
    });
    if ((e = remainder_etd_2d<T>(I, v, st, a, s)) != hipSuccess) return e;
    return c2r_recover<T>(g, t, v.Sgu, v.Stmp, v.u, v.gp, out, I.K.thr, halt_flag(I), s);
}

template <typename T> etd_status step_coupled(etd_plan* plan, Instance& I, hipStream_t s) {
    const GridK& g = I.g;
    const FFTTables<T>& t = tables<T>(I);
    CoupledView<T> v(I);
    const long n = g.nreal();
    const bool rk2 = I.d.scheme == ETD_ETDRK2;
    const uint8_t* mask = nullptr;
    if (I.d.band_threshold > 0.0) {
        if (I.step % I.d.band_rebuild_every == 0) {
            StageRange r("etd.band_rebuild");
            timed_kernel(PASS_BAND, (sizeof(T) + 2.0) * n, s, [&] {
                band_flags<T>(n, v.phiA, I.d.band_threshold, I.mask, s);
                band_compact(n, I.mask, I.band_cnt, I.band_idx, n, I.band_total, s);
            });
        }
        mask = I.mask;
    }
    // ---- phi stages (u frozen at u^n); phiA holds phi^n, lap/gx/gy/gz its derivatives
    // and (three-dimensional grids) the device scalar the integral of phi^n
    const double fb = (double)sizeof(T) * n;   // one real field
    // frozen membrane: phi, g+ = g(phi) and v = 0 stay as set_state left them
    const bool frozen = (I.d.flags & ETD_F_FROZEN_MEMBRANE) != 0;
    // g+ and the velocity at phi^{n+1}: on three-dimensional grids in the last
    // derivative pass, else a pointwise kernel after it
    const VelocityArgs<T> va{v.phiA, v.gp, v.vx, v.vy, v.vz, I.K.tau, I.K.thr};
    const VelocityArgs<T>* vel = g.nx > 1 ? &va : nullptr;
    const double* halt = halt_flag(I);
    if (!frozen && !rk2) {
        StageRange r("etd.phi (S1 S4)");
        HIPCHK(plan, phi_stage<T>(I, v, v.phiA, mask, ETD_STAGE_PHI1, EtdArgs<T>{v.Sphi, v.Sra, v.Sphi, halt, I.xlines}, v.phiB,
                                  s, vel));
    } else if (!frozen) {
        {
            StageRange r("etd.phi1 (S1 S2)");
            HIPCHK(plan, phi_stage<T>(I, v, v.phiA, mask, ETD_STAGE_PHI1, EtdArgs<T>{v.Sphi, v.Sra, v.St, halt, I.xlines},
                                      v.phiB, s));
        }
        StageRange r("etd.phi2 (S3 S4)");
        HIPCHK(plan, phi_stage<T>(I, v, v.phiB, mask, ETD_STAGE_PHI2, EtdArgs<T>{v.St, v.Sra, v.Sphi, halt, I.xlines}, v.phiB,
                                  s, vel));
    }
    // phi^{n+1} and its derivatives are kept for the next step
    if (!vel && !frozen) {
        timed_kernel(PASS_POINT, 9.0 * fb, s, [&] {
            coupled_velocity<T>(g, I.K, v.phiA, v.phiB, v.gx, v.gy, v.gz, v.gp, v.vx, v.vy, v.vz, halt, s);
        });
    }
    // ---- g u stages with g = g(phi^{n+1})
    // The spectral g u values are kept as increments D over FFT(g+ u^n), so the
    // inverse transforms carry only the per-step change; g+ u^n is added back in
    // real space inside the recovery (same scheme, smaller rounding in FP32).
    if (!rk2) {
        StageRange r("etd.u1 (S5 S6)");
        HIPCHK(plan, u_stage<T>(I, v, v.u, mask, ETD_STAGE_U1, false, v.ut, s));     // U^{n+1}
        std::swap(I.u, I.ut);
    } else {
        {
            StageRange r("etd.u1 (S5 S6)");
            HIPCHK(plan, u_stage<T>(I, v, v.u, mask, ETD_STAGE_U1, true, v.ut, s));      // U~
        }
        StageRange r("etd.u2 (S7 S8)");
        HIPCHK(plan, u_stage<T>(I, v, v.ut, mask, ETD_STAGE_U2, false, v.u, s));     // U^{n+1}
    }
    if (I.d.flags & ETD_F_MASS_PROJECT) {
        StageRange r("etd.mass_project");
        timed_kernel(PASS_POINT, 5.0 * fb, s, [&] {
            mass_project_sums<T>(n, v.gp, (T*)I.u, I.K.thr, I.part, I.scal + S_MPS, s);
            mass_project_apply<T>(n, v.gp, (T*)I.u, I.K.thr, g.cell, I.scal + S_Q0, I.scal + S_MPS, halt, s);
        });
    }
    if (!frozen) std::swap(I.phiA, I.phiB);
    HIPCHK(plan, hipGetLastError());
    return ETD_OK;
}

// ------------------------------------------------------------------ fixed step
// psi = (-Delta_h)^{-1} q  (FP64, or FP32 transforms on the FP32-FFT path)
// With ETD_F_SURFACE_NONLOCAL: psi = (-Delta_S,h)^{-1} q on the band {g >= delta}
// (FP64 band solve on both paths).
etd_status fixed_nonlocal(etd_plan* plan, Instance& I, const double* q, hipStream_t s) {
    const GridK& g = I.g;
    if (I.d.flags & ETD_F_SURFACE_NONLOCAL) {
        StageRange r("etd.band_solve");
        HIPCHK(plan, surface_lapinv<double>(g, I.G, q, I.mask, I.band_idx, I.band_total, I.psid, I.sw, 1e-12, 20000,
                                            true, &I.surf_last, s));
    } else if (!I.f32) {
        HIPCHK(plan, lapinv_fused<double>(g, I.td, I.fd, q, (double2*)I.Sa, I.psid, s));
    } else {
        convert<double, float>(g.nreal(), q, I.qf, s);
        HIPCHK(plan, lapinv_fused<float>(g, I.tf, I.fd, I.qf, (float2*)I.Sb, I.psif, s));
    }
    return ETD_OK;
}

// R = R(U); with Rprev (nullable) R receives R(U) - Rprev instead.
etd_status fixed_R(etd_plan* plan, Instance& I, const double* U, double* R, hipStream_t s,
                   const double* Rprev = nullptr) {
    const GridK& g = I.g;
    const long n = g.nreal();
    const double fb = 8.0 * n;
    const double* band = (I.d.flags & ETD_F_BAND_STEP) ? I.gf : nullptr;
    timed_kernel(PASS_FIXED_POINT, 4.0 * fb, s, [&] { fixed_nonlocal_arg(n, I.FK, I.G, U, I.q, I.mq, band, s); });
    timed_kernel(PASS_REDUCE, fb, s, [&] {
        reduce_sum<double>(n, I.mq, g.cell, I.part, I.scal + S_MASS, s, halt_flag(I));
    });
    etd_status st = fixed_nonlocal(plan, I, I.q, s);
    if (st != ETD_OK) return st;
    timed_kernel(PASS_FIXED_POINT, (Rprev ? 4.0 : 3.0) * fb + (I.f32 ? 4.0 : 8.0) * n, s, [&] {
        if (!I.f32 || (I.d.flags & ETD_F_SURFACE_NONLOCAL))
            fixed_remainder<double>(n, I.FK, I.sg, U, I.psid, I.scal + S_MASS, R, band, s, Rprev);
        else
            fixed_remainder<float>(n, I.FK, I.sg, U, I.psif, I.scal + S_MASS, R, band, s, Rprev);
    });
    return ETD_OK;
}

// acc = f(tau L) v by the Chebyshev recurrence (coefficients c); v is only read
void cheb_apply(Instance& I, const std::vector<double>& c, const double* v, double* acc, hipStream_t s) {
    const GridK& g = I.g;
    // first: T_1 v = Atil v; acc = c0/2 v + c1 T_1 v
    const double fb = 8.0 * g.nreal();
    timed_kernel(PASS_FIXED_STENCIL, 5.0 * fb, s, [&] {
        fixed_cheb_step(g, I.FK, I.gf, I.isg, I.a, I.b, 1.0, 0.0, v, nullptr, I.t1, acc, c.size() > 1 ? c[1] : 0.0,
                        0.5 * c[0], 1, s);
    });
    // T_k = 2 Atil T_{k-1} - T_{k-2}, acc += c_k T_k
    const double* prev = v;   // T_{k-2}
    double* cur = I.t1;       // T_{k-1}
    size_t k = 2;
    if (I.t3) {   // two terms per pass, into two buffers that hold neither input
        double* const pool[4] = {I.t1, I.t2, I.t3, I.t4};
        for (; k + 1 < c.size(); k += 2) {
            double* o[2] = {nullptr, nullptr};
            int m = 0;
            for (double* b : pool)
                if (b != cur && b != prev && m < 2) o[m++] = b;
            timed_kernel(PASS_FIXED_STENCIL, 8.0 * fb, s, [&] {
                fixed_cheb_pair(g, I.FK, I.gf, I.isg, I.a, I.b, 2.0, 1.0, cur, prev, o[0], o[1], acc, c[k], c[k + 1],
                                s);
            });
            prev = o[0];
            cur = o[1];
        }
    }
    for (; k < c.size(); ++k) {
        // one term, written over the T_{k-2} buffer (never over v)
        double* out = (prev == v) ? (cur == I.t1 ? I.t2 : I.t1) : const_cast<double*>(prev);
        timed_kernel(PASS_FIXED_STENCIL, 7.0 * fb, s, [&] {
            fixed_cheb_step(g, I.FK, I.gf, I.isg, I.a, I.b, 2.0, 1.0, cur, prev, out, acc, c[k], 0.0, 0, s);
        });
        prev = cur;
        cur = out;
    }
}

etd_status step_fixed(etd_plan* plan, Instance& I, hipStream_t s) {
    const GridK& g = I.g;
    const long n = g.nreal();
    etd_status st;
    // w = sg U;  v = R(U) - L w;  w~ = w + tau phi1(tau L) v
    const double fb = 8.0 * n;
    StageRange r1("etd.fixed.stage1");
    timed_kernel(PASS_FIXED_POINT, 3.0 * fb, s, [&] { mul(n, I.sg, I.U, I.w, s); });
    if ((st = fixed_R(plan, I, I.U, I.R0, s)) != ETD_OK) return st;
    // v = R0 - L w in the operator pass
    timed_kernel(PASS_FIXED_STENCIL, 5.0 * fb, s, [&] { fixed_L_apply(g, I.FK, I.gf, I.isg, I.w, I.vv, s, I.R0); });
    const double* band = (I.d.flags & ETD_F_BAND_STEP) ? I.gf : nullptr;   // U changes on the band only
    cheb_apply(I, I.ch1, I.vv, I.acc, s);
    // w = w~ = w + tau acc, U = w~ / sg (the ETD1 result / the predictor)
    timed_kernel(PASS_FIXED_POINT, 5.0 * fb, s, [&] { fixed_advance(n, I.d.tau, I.acc, I.w, I.isg, I.U, halt_flag(I), band, s); });
    if (I.d.scheme == ETD_ETDRK2) {
        StageRange r2("etd.fixed.stage2");
        // v = R(U~) - R0, formed where R(U~) is
        if ((st = fixed_R(plan, I, I.U, I.vv, s, I.R0)) != ETD_OK) return st;
        cheb_apply(I, I.ch2, I.vv, I.acc, s);
        timed_kernel(PASS_FIXED_POINT, 5.0 * fb, s, [&] { fixed_advance(n, I.d.tau, I.acc, I.w, I.isg, I.U, halt_flag(I), band, s); });
    }
    if (I.d.flags & ETD_F_MASS_PROJECT) {
        timed_kernel(PASS_FIXED_POINT, 5.0 * fb, s, [&] {
            mass_project_sums<double>(n, I.G, I.U, I.d.recover_threshold, I.part, I.scal + S_MPS, s);
            mass_project_apply<double>(n, I.G, I.U, I.d.recover_threshold, g.cell, I.scal + S_Q0, I.scal + S_MPS,
                                       halt_flag(I), s);
        });
    }
    HIPCHK(plan, hipGetLastError());
    return ETD_OK;
}

template <typename TI, typename TO> void copy_conv(long n, const void* in, void* out, hipStream_t s) {
    convert<TI, TO>(n, (const TI*)in, (TO*)out, s);
}

// state element type T (float/double) <-> ABI dtype
template <typename T> void load_field(long n, const void* src, etd_dtype dt, T* dst, hipStream_t s) {
    if (dt == ETD_F64) copy_conv<double, T>(n, src, dst, s);
    else copy_conv<float, T>(n, src, dst, s);
}
template <typename T> void store_field(long n, const T* src, etd_dtype dt, void* dst, hipStream_t s) {
    if (dt == ETD_F64) copy_conv<T, double>(n, src, dst, s);
    else copy_conv<T, float>(n, src, dst, s);
}

template <typename T> etd_status set_state_coupled(etd_plan* plan, Instance& I, const void* a, const void* u,
                                                   etd_dtype dt) {
    hipStream_t s = plan->stream;
    const GridK& g = I.g;
    const long n = g.nreal();
    CoupledView<T> v(I);
    HIPCHK(plan, hipMemsetAsync(halt_flag(I), 0, sizeof(double), s));   // a new state: steps run again
    load_field<T>(n, a, dt, v.phiA, s);
    load_field<T>(n, u, dt, v.u, s);
    HIPCHK(plan, fft_r2c_3d<T>(g, tables<T>(I), v.phiA, v.Sphi, s));
    // phi^0 from its spectrum (as every later phi^n is), with its derivatives
    HIPCHK(plan, phi_and_derivs<T>(I, v, v.Sphi, v.phiA, s));   // 3D: also the integral of phi
    if (g.nx == 1) reduce_sum<T>(n, v.phiA, g.cell, I.part, I.scal + S_INTPHI, s);
    gloc_field<T>(n, v.phiA, v.gp, s);
    if (I.d.flags & ETD_F_FROZEN_MEMBRANE) {   // v = 0 for every step
        for (T* f : {v.vx, v.vy, v.vz}) HIPCHK(plan, hipMemsetAsync(f, 0, n * sizeof(T), s));
    }
    mass_project_sums<T>(n, v.gp, v.u, I.K.thr, I.part, I.scal + S_MPS, s);
    double host[3] = {0, 0, 0};
    HIPCHK(plan, hipMemcpyAsync(host, I.scal + S_INTPHI, sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(plan, hipMemcpyAsync(host + 1, I.scal + S_MPS, sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(plan, hipStreamSynchronize(s));
    I.A0 = I.cp.A0_from_initial ? host[0] : I.cp.A0;
    const double Q0 = host[1] * g.cell;
    HIPCHK(plan, hipMemcpy(I.scal + S_Q0, &Q0, sizeof(double), hipMemcpyHostToDevice));
    // a NaN or Inf anywhere in phi or u reaches the integral of phi or <g u, 1>
    // (phi through its transform): such a state is kept, and every step is a no-op
    if (!std::isfinite(host[0]) || !std::isfinite(host[1])) {
        const double one = 1.0;
        HIPCHK(plan, hipMemcpy(halt_flag(I), &one, sizeof(double), hipMemcpyHostToDevice));
    }
    return ETD_OK;
}

etd_status set_state_fixed(etd_plan* plan, Instance& I, const void* a, const void* u, etd_dtype dt) {
    hipStream_t s = plan->stream;
    const GridK& g = I.g;
    const long n = g.nreal();
    HIPCHK(plan, hipMemsetAsync(halt_flag(I), 0, sizeof(double), s));   // a new state: steps run again
    load_field<double>(n, a, dt, I.G, s);
    load_field<double>(n, u, dt, I.U, s);
    fixed_prep(g, I.G, I.sg, I.isg, s);
    if (I.d.flags & ETD_F_BAND_STEP) fixed_band_field(n, I.G, I.d.band_threshold, I.gf, s);
    fixed_gershgorin(g, I.gf, I.isg, I.part, I.scal + S_GERSH, s);
    mass_project_sums<double>(n, I.G, I.U, I.d.recover_threshold, I.part, I.scal + S_MPS, s);
    // min g and a non-finite count, through the diagnostics reduction with g in the u slot
    reduce_diag<double>(g, nullptr, I.G, I.G, I.fp.ubar, true, I.part, I.scal + S_DIAG, s);
    double host[3], dg[7];
    HIPCHK(plan, hipMemcpyAsync(host, I.scal + S_GERSH, sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(plan, hipMemcpyAsync(host + 1, I.scal + S_MPS, sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(plan, hipMemcpyAsync(dg, I.scal + S_DIAG, 7 * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(plan, hipStreamSynchronize(s));
    const double gmin = -dg[3];
    if (!(gmin > 0.0) || dg[6] > 0.0 || !std::isfinite(host[0]))
        return fail(&plan->err, ETD_E_ARG, "g must be finite and strictly positive");
    if (I.d.flags & ETD_F_SURFACE_NONLOCAL) {
        band_ge<double>(n, I.G, I.d.band_threshold, I.mask, s);
        band_compact(n, I.mask, I.band_cnt, I.band_idx, n, I.band_total, s);
        HIPCHK(plan, hipGetLastError());
    }
    I.rho = host[0];
    I.a = I.FK.B;
    I.b = I.FK.B + I.FK.eps_u * I.rho;
    if (!(I.b > I.a)) I.b = I.a * (1.0 + 1e-12) + 1e-300;
    I.ch1 = cheb_coeffs(phi1_host, I.d.tau, I.a, I.b);
    I.ch2 = cheb_coeffs(phi2_host, I.d.tau, I.a, I.b);
    if (I.ch1.empty() || I.ch2.empty())
        return fail(&plan->err, ETD_E_ARG,
                    "the spectrum of tau L, [" + std::to_string(I.d.tau * I.a) + ", " + std::to_string(I.d.tau * I.b) +
                        "], is too wide for the Chebyshev expansion (more than 4096 terms): g varies too fast "
                        "between neighbours where it is tiny; ETD_F_BAND_STEP restricts the step to {g >= delta}");
    const double Q0 = host[1] * g.cell;
    HIPCHK(plan, hipMemcpy(I.scal + S_Q0, &Q0, sizeof(double), hipMemcpyHostToDevice));
    if (!std::isfinite(host[1])) {   // U not finite (g is checked above): keep it, steps are no-ops
        const double one = 1.0;
        HIPCHK(plan, hipMemcpy(halt_flag(I), &one, sizeof(double), hipMemcpyHostToDevice));
    }
    return ETD_OK;
}

}  // namespace

// =================================================================== C ABI
namespace {
// The instance's diagnostics sums of its current state into S_DIAG.
void diag_sums(Instance& I, hipStream_t s) {
    const GridK& g = I.g;
    if (I.d.model == ETD_COUPLED) {
        if (I.f32) reduce_diag<float>(g, (const float*)I.phiA, nullptr, (const float*)I.u, I.cp.ubar, false, I.part,
                                      I.scal + S_DIAG, s);
        else reduce_diag<double>(g, (const double*)I.phiA, nullptr, (const double*)I.u, I.cp.ubar, false, I.part,
                                 I.scal + S_DIAG, s);
    } else {
        reduce_diag<double>(g, nullptr, I.G, I.U, I.fp.ubar, true, I.part, I.scal + S_DIAG, s);
    }
}
}  // namespace

etd_status etd::step_instance(etd_plan* plan, Instance& I, hipStream_t s) {
    StageRange r("etd.step");
    etd_status st = I.d.model == ETD_COUPLED ? (I.f32 ? step_coupled<float>(plan, I, s)
                                                       : step_coupled<double>(plan, I, s))
                                             : step_fixed(plan, I, s);
    if (st != ETD_OK || !I.ring) return st;
    // the ring entry of this step, on the step's stream (so also inside a captured graph)
    diag_sums(I, s);
    const bool band = I.d.model == ETD_COUPLED && I.d.band_threshold > 0.0 && I.band_total;
    diag_ring_push(I.scal + S_DIAG, halt_flag(I), band ? I.band_total : nullptr, I.ring, I.ring_cap, I.ring_meta, s);
    HIPCHK(plan, hipGetLastError());
    return ETD_OK;
}

extern "C" {

const char* etd_status_string(etd_status s) {
    switch (s) {
        case ETD_OK: return "ok";
        case ETD_E_ARG: return "invalid argument";
        case ETD_E_SIZE: return "unsupported size";
        case ETD_E_STATE: return "invalid state (call order)";
        case ETD_E_HIP: return "HIP runtime error";
        case ETD_E_NOMEM: return "device out of memory";
        case ETD_E_NONFINITE: return "non-finite state";
        case ETD_E_CAPACITY: return "capacity too small";
    }
    return "unknown status";
}

const char* etd_last_error(etd_plan_t plan) {
    if (plan) return plan->err.c_str();
    return g_last_error.c_str();
}

etd_status etd_plan_create(const etd_instance_desc* inst, int n_instances, void* hip_stream, etd_plan_t* out) {
    if (!out) return fail(nullptr, ETD_E_ARG, "out is null");
    *out = nullptr;
    if (!inst || n_instances < 1) return fail(nullptr, ETD_E_ARG, "need at least one instance descriptor");
    for (int i = 0; i < n_instances; ++i) {
        std::string msg;
        etd_status st = validate(inst[i], msg);
        if (st != ETD_OK) return fail(nullptr, st, "instance " + std::to_string(i) + ": " + msg);
    }
    etd_plan* P = new etd_plan();
    P->stream = (hipStream_t)hip_stream;
    if (hipGetDevice(&P->device) != hipSuccess) {
        delete P;
        return fail(nullptr, ETD_E_HIP, "no HIP device");
    }
    // the device's copy of the allocation-free band build's scratch (once per device)
    if (hipError_t e = band_static_init(P->device); e != hipSuccess) {
        delete P;
        return fail(nullptr, ETD_E_HIP, std::string("scratch lookup: ") + hipGetErrorString(e));
    }
    P->inst.resize(n_instances);
    for (int i = 0; i < n_instances; ++i) {
        Instance& I = P->inst[i];
        I.d = inst[i];
        if (inst[i].model == ETD_COUPLED) I.cp = *inst[i].coupled;
        else I.fp = *inst[i].fixed;
        I.d.coupled = nullptr;
        I.d.fixed = nullptr;
        I.g = make_grid(inst[i].grid);
        I.f32 = inst[i].precision == ETD_FP32;
        etd_status st = setup_common(P, I);
        if (st == ETD_OK) st = (I.d.model == ETD_COUPLED) ? setup_coupled(P, I) : setup_fixed(P, I);
        if (st != ETD_OK) {
            g_last_error = P->err;
            etd_plan_destroy(P);
            return st;
        }
    }
    *out = P;
    if (log_level() >= 2) {
        size_t bytes = 0;
        for (const Instance& I : P->inst) bytes += I.bytes;
        log_msg(2, "plan %p: %d instance(s), %.1f MiB of device memory", (void*)P, n_instances,
                bytes / 1048576.0);
        for (int i = 0; i < n_instances; ++i) {
            const Instance& I = P->inst[i];
            log_msg(2, "  instance %d: %s %s %s %dx%dx%d tau %g band %g", i,
                    I.d.model == ETD_COUPLED ? "coupled" : "fixed", I.d.scheme == ETD_ETDRK2 ? "ETDRK2" : "ETD1",
                    I.f32 ? "fp32" : "fp64", I.g.nx, I.g.ny, I.g.nz, I.d.tau, I.d.band_threshold);
        }
    }
    return ETD_OK;
}

etd_status etd_plan_destroy(etd_plan_t plan) {
    if (!plan) return ETD_OK;
    if (plan->timing) fft_set_pass_hook(nullptr);
    (void)hipStreamSynchronize(plan->stream);
    release_schedule(plan);
    for (Instance& I : plan->inst)
        for (void* p : I.allocs) (void)hipFree(p);
    delete plan;
    return ETD_OK;
}

etd_status etd_set_state(etd_plan_t plan, int instance, const void* a, const void* u, etd_dtype dtype) {
    etd_status st = check_instance(plan, instance);
    if (st != ETD_OK) return st;
    if (!a || !u) return fail(&plan->err, ETD_E_ARG, "state pointers must not be null");
    if (dtype != ETD_F64 && dtype != ETD_F32) return fail(&plan->err, ETD_E_ARG, "bad dtype");
    Instance& I = plan->inst[instance];
    if (I.d.model == ETD_COUPLED)
        st = I.f32 ? set_state_coupled<float>(plan, I, a, u, dtype) : set_state_coupled<double>(plan, I, a, u, dtype);
    else
        st = set_state_fixed(plan, I, a, u, dtype);
    if (st != ETD_OK) return st;
    // the band solves of a new state start cold, so a run depends on its state alone
    if (I.surf) HIPCHK(plan, hipMemsetAsync(I.sw.x, 0, sizeof(double) * (size_t)I.g.nreal(), plan->stream));
    // the diagnostics ring records the steps of the new state
    if (I.ring_meta) HIPCHK(plan, hipMemsetAsync(I.ring_meta, 0, 2 * sizeof(int64_t), plan->stream));
    I.step = 0;
    I.has_state = true;
    drop_graphs(plan);   // captured kernel arguments (A0, Chebyshev coefficients) may have changed
    return ETD_OK;
}

etd_status etd_set_tau(etd_plan_t plan, int instance, double tau) {
    etd_status st = check_instance(plan, instance);
    if (st != ETD_OK) return st;
    if (!(std::isfinite(tau) && tau > 0.0)) return fail(&plan->err, ETD_E_ARG, "tau must be finite and > 0");
    Instance& I = plan->inst[instance];
    if (I.d.model == ETD_FIXED_MEMBRANE && I.has_state) {
        std::vector<double> c1 = cheb_coeffs(phi1_host, tau, I.a, I.b), c2 = cheb_coeffs(phi2_host, tau, I.a, I.b);
        if (c1.empty() || c2.empty())   // the instance keeps its step
            return fail(&plan->err, ETD_E_ARG, "the spectrum of tau L is too wide for the Chebyshev expansion");
        I.ch1 = std::move(c1);
        I.ch2 = std::move(c2);
    }
    I.d.tau = tau;
    I.K.tau = tau;
    drop_graphs(plan);
    return ETD_OK;
}

etd_status etd_get_state(etd_plan_t plan, int instance, void* a, void* u, etd_dtype dtype) {
    etd_status st = check_instance(plan, instance);
    if (st != ETD_OK) return st;
    Instance& I = plan->inst[instance];
    if (!I.has_state) return fail(&plan->err, ETD_E_STATE, "get_state before set_state");
    if (!u || (I.d.model == ETD_COUPLED && !a)) return fail(&plan->err, ETD_E_ARG, "null output pointer");
    if (dtype != ETD_F64 && dtype != ETD_F32) return fail(&plan->err, ETD_E_ARG, "bad dtype");
    hipStream_t s = plan->stream;
    const long n = I.g.nreal();
    if (I.d.model == ETD_COUPLED) {
        if (I.f32) {
            store_field<float>(n, (const float*)I.phiA, dtype, a, s);
            store_field<float>(n, (const float*)I.u, dtype, u, s);
        } else {
            store_field<double>(n, (const double*)I.phiA, dtype, a, s);
            store_field<double>(n, (const double*)I.u, dtype, u, s);
        }
    } else {
        if (a) store_field<double>(n, I.G, dtype, a, s);
        store_field<double>(n, I.U, dtype, u, s);
    }
    double halt = 0.0;
    HIPCHK(plan, hipGetLastError());
    HIPCHK(plan, hipMemcpyAsync(&halt, halt_flag(I), sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(plan, hipStreamSynchronize(s));
    if (halt != 0.0)
        return fail(&plan->err, ETD_E_NONFINITE,
                    "non-finite state: the steps since it was detected left the state as it was");
    return ETD_OK;
}

// ------------------------------------------------------------------ checkpoints
namespace {

constexpr char kCkptMagic[8] = {'E', 'T', 'D', 'C', 'K', 'P', 'T', '1'};
constexpr int kCkptMaxParts = 24;

struct CkptHeader {
    char magic[8];
    int32_t model, scheme, precision, nx, ny, nz;
    uint32_t flags;
    int32_t nparts;
    double band_threshold, recover_threshold;
    int32_t band_rebuild_every, pad;
    int64_t step;
    double A0;
    uint64_t part_bytes[kCkptMaxParts];
};

// carried_state, plus g for the fixed model (its derived fields are
// recomputed from it by the load)
std::vector<std::pair<void*, size_t>> ckpt_parts(const Instance& I) {
    std::vector<std::pair<void*, size_t>> parts = carried_state(I);
    if (I.d.model == ETD_FIXED_MEMBRANE) parts.push_back({I.G, (size_t)I.g.nreal() * sizeof(double)});
    return parts;
}

size_t ckpt_bytes(const std::vector<std::pair<void*, size_t>>& parts) {
    size_t b = sizeof(CkptHeader);
    for (const auto& p : parts) b += p.second;
    return b;
}

CkptHeader ckpt_header(const Instance& I, const std::vector<std::pair<void*, size_t>>& parts) {
    CkptHeader h{};
    std::memcpy(h.magic, kCkptMagic, sizeof h.magic);
    h.model = I.d.model;
    h.scheme = I.d.scheme;
    h.precision = I.d.precision;
    h.nx = I.g.nx;
    h.ny = I.g.ny;
    h.nz = I.g.nz;
    h.flags = I.d.flags;
    h.nparts = (int32_t)parts.size();
    h.band_threshold = I.d.band_threshold;
    h.recover_threshold = I.d.recover_threshold;
    h.band_rebuild_every = I.d.band_rebuild_every;
    h.step = I.step;
    h.A0 = I.A0;
    for (size_t k = 0; k < parts.size() && k < (size_t)kCkptMaxParts; ++k) h.part_bytes[k] = parts[k].second;
    return h;
}

etd_status ckpt_copy_in(etd_plan* plan, const std::vector<std::pair<void*, size_t>>& parts, const char* src) {
    src += sizeof(CkptHeader);
    for (const auto& p : parts) {
        HIPCHK(plan, hipMemcpyAsync(p.first, src, p.second, hipMemcpyHostToDevice, plan->stream));
        src += p.second;
    }
    HIPCHK(plan, hipStreamSynchronize(plan->stream));
    return ETD_OK;
}

}  // namespace

etd_status etd_checkpoint_size(etd_plan_t plan, int instance, size_t* bytes) {
    etd_status st = check_instance(plan, instance);
    if (st != ETD_OK) return st;
    if (!bytes) return fail(&plan->err, ETD_E_ARG, "null output");
    *bytes = ckpt_bytes(ckpt_parts(plan->inst[instance]));
    return ETD_OK;
}

etd_status etd_checkpoint_save(etd_plan_t plan, int instance, void* host, size_t bytes) {
    etd_status st = check_instance(plan, instance);
    if (st != ETD_OK) return st;
    if (!host) return fail(&plan->err, ETD_E_ARG, "null host buffer");
    const Instance& I = plan->inst[instance];
    if (!I.has_state) return fail(&plan->err, ETD_E_STATE, "checkpoint before set_state");
    const auto parts = ckpt_parts(I);
    if (parts.size() > (size_t)kCkptMaxParts) return fail(&plan->err, ETD_E_ARG, "checkpoint: too many buffers");
    if (bytes < ckpt_bytes(parts)) return fail(&plan->err, ETD_E_CAPACITY, "checkpoint buffer too small");
    const CkptHeader h = ckpt_header(I, parts);
    char* dst = static_cast<char*>(host);
    std::memcpy(dst, &h, sizeof h);
    dst += sizeof h;
    for (const auto& p : parts) {
        HIPCHK(plan, hipMemcpyAsync(dst, p.first, p.second, hipMemcpyDeviceToHost, plan->stream));
        dst += p.second;
    }
    HIPCHK(plan, hipStreamSynchronize(plan->stream));
    return ETD_OK;
}

etd_status etd_checkpoint_load(etd_plan_t plan, int instance, const void* host, size_t bytes) {
    etd_status st = check_instance(plan, instance);
    if (st != ETD_OK) return st;
    if (!host) return fail(&plan->err, ETD_E_ARG, "null host buffer");
    Instance& I = plan->inst[instance];
    if (bytes < sizeof(CkptHeader)) return fail(&plan->err, ETD_E_ARG, "checkpoint image too small");
    CkptHeader h;
    std::memcpy(&h, host, sizeof h);
    // the instance's buffers before any state is set: the same list as after
    const auto parts = ckpt_parts(I);
    CkptHeader want = ckpt_header(I, parts);
    if (std::memcmp(h.magic, kCkptMagic, sizeof h.magic) != 0)
        return fail(&plan->err, ETD_E_ARG, "not a checkpoint image of this library");
    bool same = h.model == want.model && h.scheme == want.scheme && h.precision == want.precision &&
                h.nx == want.nx && h.ny == want.ny && h.nz == want.nz && h.flags == want.flags &&
                h.nparts == want.nparts && h.band_threshold == want.band_threshold &&
                h.recover_threshold == want.recover_threshold && h.band_rebuild_every == want.band_rebuild_every;
    for (int k = 0; same && k < h.nparts && k < kCkptMaxParts; ++k) same = h.part_bytes[k] == want.part_bytes[k];
    if (!same) return fail(&plan->err, ETD_E_ARG, "checkpoint of a different instance configuration");
    if (bytes < ckpt_bytes(parts)) return fail(&plan->err, ETD_E_ARG, "checkpoint image truncated");
    const char* src = static_cast<const char*>(host);
    // the saved buffers in place, then set_state from the saved state (the
    // fields it derives from phi or g, the schedule reset), then the saved
    // buffers again over everything set_state recomputed
    if ((st = ckpt_copy_in(plan, parts, src)) != ETD_OK) return st;
    if (I.d.model == ETD_COUPLED)
        st = I.f32 ? set_state_coupled<float>(plan, I, I.phiA, I.u, ETD_F32)
                   : set_state_coupled<double>(plan, I, I.phiA, I.u, ETD_F64);
    else
        st = set_state_fixed(plan, I, I.G, I.U, ETD_F64);
    if (st != ETD_OK) return st;
    if ((st = ckpt_copy_in(plan, parts, src)) != ETD_OK) return st;
    I.step = h.step;
    I.A0 = h.A0;
    if (I.ring_meta) {   // the diagnostics ring records the resumed steps
        const int64_t meta[2] = {0, h.step};
        HIPCHK(plan, hipMemcpy(I.ring_meta, meta, sizeof meta, hipMemcpyHostToDevice));
    }
    I.has_state = true;
    drop_graphs(plan);
    return ETD_OK;
}

etd_status etd_step(etd_plan_t plan, int nsteps) {
    if (!plan) return fail(nullptr, ETD_E_ARG, "null plan");
    if (nsteps < 0) return fail(&plan->err, ETD_E_ARG, "nsteps must be >= 0");
    for (Instance& I : plan->inst)
        if (!I.has_state) return fail(&plan->err, ETD_E_STATE, "step before set_state");
    return run_steps(plan, nsteps);
}

etd_status etd_energy(etd_plan_t plan, int instance, double* host_out, int n_out) {
    etd_status st = check_instance(plan, instance);
    if (st != ETD_OK) return st;
    Instance& I = plan->inst[instance];
    if (!I.has_state) return fail(&plan->err, ETD_E_STATE, "energy before set_state");
    if (!host_out) return fail(&plan->err, ETD_E_ARG, "null output");
    hipStream_t s = plan->stream;
    const GridK& g = I.g;
    const long n = g.nreal();
    double sums[7] = {0};
    if (I.d.model == ETD_FIXED_MEMBRANE) {
        if (n_out < 5) return fail(&plan->err, ETD_E_ARG, "fixed energy needs n_out >= 5");
        fixed_nonlocal_arg(n, I.FK, I.G, I.U, I.q, I.mq, (I.d.flags & ETD_F_BAND_STEP) ? I.gf : nullptr, s);
        HIPCHK(plan, fft_r2c_3d<double>(g, I.td, I.q, (double2*)I.Sa, s));
        spec_apply<double>(g, SPEC_INV_FD, (const double2*)I.Sa, (double2*)I.Sa, I.fd, s);
        HIPCHK(plan, fft_c2r_3d<double>(g, I.td, (const double2*)I.Sa, (double2*)I.Stmp, I.psid, s));
        reduce_energy_fixed(g, I.FK, I.gf, I.U, I.psid, I.q, I.part, I.scal + S_ENERGY, s);
        HIPCHK(plan, hipMemcpyAsync(sums, I.scal + S_ENERGY, 4 * sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHK(plan, hipStreamSynchronize(s));
        const double c = g.cell;
        const double eg = 0.5 * I.FK.eps_u * c * sums[0], ew = c * sums[1] / I.FK.eps_u,
                     en = 0.5 * I.FK.gamma * c * sums[2], mf = c * sums[3], em = 0.5 * I.FK.M * mf * mf;
        host_out[0] = eg + ew + en + em;
        host_out[1] = eg;
        host_out[2] = ew;
        host_out[3] = en;
        host_out[4] = em;
    } else {
        if (n_out < 6) return fail(&plan->err, ETD_E_ARG, "coupled energy needs n_out >= 6");
        auto run = [&](auto tag) -> etd_status {
            using T = decltype(tag);
            CoupledView<T> v(I);
            const FFTTables<T>& t = tables<T>(I);
            gloc_field<T>(n, v.phiA, v.gp, s);
            coupled_q_gu<T>(g, I.K, v.u, v.gp, nullptr, v.P, v.Q, nullptr, nullptr, nullptr, s);
            HIPCHK(plan, fft_r2c_3d<T>(g, t, v.P, v.Sa, s));
            spec_apply<T>(g, SPEC_INV_FD, v.Sa, v.Sa, I.fd, s);
            HIPCHK(plan, fft_c2r_3d<T>(g, t, v.Sa, v.Stmp, v.psi, s));
            const bool norm_only = g.nx > 1;   // gx holds |grad phi|
            reduce_energy_coupled<T>(g, I.K, v.phiA, v.lap, v.gx, norm_only ? nullptr : v.gy,
                                     norm_only ? nullptr : v.gz, v.u, v.psi, v.P, I.part, I.scal + S_ENERGY, s);
            return ETD_OK;
        };
        st = I.f32 ? run(0.0f) : run(0.0);
        if (st != ETD_OK) return st;
        HIPCHK(plan, hipMemcpyAsync(sums, I.scal + S_ENERGY, 7 * sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHK(plan, hipStreamSynchronize(s));
        const double c = g.cell;
        const etd_coupled_params& p = I.cp;
        const double area = c * sums[2] - I.A0;
        const double mq = c * sums[6];
        host_out[0] = p.lambda_surf * c * sums[0];
        host_out[1] = 0.5 * p.kappa * c * sums[1];
        host_out[2] = 0.5 * p.M_area * area * area;
        host_out[3] = 0.5 * p.eps_u * c * sums[3] + c * sums[4] / p.eps_u;
        host_out[4] = 0.5 * p.gamma * c * sums[5];
        host_out[5] = 0.5 * p.M * mq * mq;
    }
    for (int k = 0; k < (I.d.model == ETD_COUPLED ? 6 : 5); ++k)
        if (!std::isfinite(host_out[k])) return fail(&plan->err, ETD_E_NONFINITE, "non-finite energy");
    return ETD_OK;
}

etd_status etd_diag_ring_enable(etd_plan_t plan, int instance, int capacity) {
    etd_status st = check_instance(plan, instance);
    if (st != ETD_OK) return st;
    if (capacity < 0 || capacity > (1 << 24)) return fail(&plan->err, ETD_E_ARG, "capacity must be in 0 .. 2^24");
    Instance& I = plan->inst[instance];
    HIPCHK(plan, hipStreamSynchronize(plan->stream));
    for (void* p : {(void*)I.ring, (void*)I.ring_meta}) {
        if (!p) continue;
        (void)hipFree(p);
        I.allocs.erase(std::remove(I.allocs.begin(), I.allocs.end(), p), I.allocs.end());
    }
    I.ring = nullptr;
    I.ring_meta = nullptr;
    I.ring_cap = 0;
    drop_graphs(plan);   // captured steps include the push, or not
    if (capacity == 0) return ETD_OK;
    etd_plan* P = plan;
    ALLOC(I.ring, (size_t)capacity * kDiagRingFields * sizeof(double));
    ALLOC(I.ring_meta, 2 * sizeof(int64_t));
    I.ring_cap = capacity;
    const int64_t meta[2] = {0, I.step};
    HIPCHK(plan, hipMemcpy(I.ring_meta, meta, sizeof meta, hipMemcpyHostToDevice));
    return ETD_OK;
}

etd_status etd_diag_ring_read(etd_plan_t plan, int instance, etd_diag* host_out, int max_entries,
                              int64_t* recorded) {
    etd_status st = check_instance(plan, instance);
    if (st != ETD_OK) return st;
    if (!recorded || (max_entries > 0 && !host_out) || max_entries < 0)
        return fail(&plan->err, ETD_E_ARG, "null output or negative max_entries");
    const Instance& I = plan->inst[instance];
    if (!I.ring) return fail(&plan->err, ETD_E_STATE, "diagnostics ring not enabled");
    hipStream_t s = plan->stream;
    int64_t meta[2] = {0, 0};
    std::vector<double> ring((size_t)I.ring_cap * kDiagRingFields);
    HIPCHK(plan, hipMemcpyAsync(meta, I.ring_meta, sizeof meta, hipMemcpyDeviceToHost, s));
    HIPCHK(plan, hipMemcpyAsync(ring.data(), I.ring, ring.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(plan, hipStreamSynchronize(s));
    *recorded = meta[0];
    const int64_t n = std::min<int64_t>({meta[0], (int64_t)I.ring_cap, (int64_t)max_entries});
    for (int64_t k = 0; k < n; ++k) {   // the last n entries, oldest first
        const double* e = ring.data() + (size_t)((meta[0] - n + k) % I.ring_cap) * kDiagRingFields;
        etd_diag& o = host_out[k];
        o.step = (int64_t)e[0];
        o.int_phi = I.d.model == ETD_COUPLED ? e[1] : 0.0;
        o.mass = e[2];
        o.Q = e[3];
        o.umin = e[4];
        o.umax = e[5];
        o.bound = e[6];
        o.band_count = (int64_t)e[7];
        o.nonfinite = e[8] != 0.0 ? 1 : 0;
        o.b_warning = (I.d.model == ETD_FIXED_MEMBRANE && I.FK.B < I.Bmbp) ? 1 : 0;
    }
    return ETD_OK;
}

etd_status etd_diagnostics(etd_plan_t plan, int instance, etd_diag* out) {
    etd_status st = check_instance(plan, instance);
    if (st != ETD_OK) return st;
    Instance& I = plan->inst[instance];
    if (!I.has_state) return fail(&plan->err, ETD_E_STATE, "diagnostics before set_state");
    if (!out) return fail(&plan->err, ETD_E_ARG, "null output");
    hipStream_t s = plan->stream;
    diag_sums(I, s);
    double d[7], halt = 0.0;
    int64_t bc = 0;
    HIPCHK(plan, hipMemcpyAsync(d, I.scal + S_DIAG, 7 * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(plan, hipMemcpyAsync(&halt, halt_flag(I), sizeof(double), hipMemcpyDeviceToHost, s));
    if (I.d.model == ETD_COUPLED && I.d.band_threshold > 0.0 && I.band_total)
        HIPCHK(plan, hipMemcpyAsync(&bc, I.band_total, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    HIPCHK(plan, hipStreamSynchronize(s));
    out->step = I.step;
    out->int_phi = I.d.model == ETD_COUPLED ? d[0] : 0.0;
    out->mass = d[1];
    out->Q = d[2];
    out->umin = -d[3];
    out->umax = d[4];
    out->bound = d[5];
    out->band_count = bc;
    out->nonfinite = (d[6] > 0.0 || halt != 0.0) ? 1 : 0;
    out->b_warning = (I.d.model == ETD_FIXED_MEMBRANE && I.FK.B < I.Bmbp) ? 1 : 0;
    if (out->nonfinite) return fail(&plan->err, ETD_E_NONFINITE, "non-finite state");
    return ETD_OK;
}

etd_status etd_narrowband_build(etd_plan_t plan, int instance, const void* phi, etd_dtype dtype, double threshold,
                                int32_t* dev_idx_out, int64_t capacity, int64_t* count_out) {
    etd_status st = check_instance(plan, instance);
    if (st != ETD_OK) return st;
    if (!phi || !count_out) return fail(&plan->err, ETD_E_ARG, "null pointer");
    if (!std::isfinite(threshold) || threshold <= 0.0) return fail(&plan->err, ETD_E_ARG, "threshold must be > 0");
    if (capacity < 0) return fail(&plan->err, ETD_E_ARG, "capacity must be >= 0");
    if (capacity > 0 && !dev_idx_out) return fail(&plan->err, ETD_E_ARG, "null index buffer");
    if (dtype != ETD_F64 && dtype != ETD_F32) return fail(&plan->err, ETD_E_ARG, "bad dtype");
    Instance& I = plan->inst[instance];
    hipStream_t s = plan->stream;
    const long n = I.g.nreal();
    // scratch: the instance's mask and tile counters (coupled) or a temporary (fixed)
    uint8_t* flags = I.mask;
    int64_t* cnt = I.band_cnt;
    int64_t* total = I.band_total;
    std::vector<void*> tmp;
    if (!flags) {
        void* p1 = nullptr;
        void* p2 = nullptr;
        HIPCHK(plan, hipMalloc(&p1, (size_t)n));
        if (hipMalloc(&p2, (band_blocks(n) + 3) * sizeof(int64_t)) != hipSuccess) {
            (void)hipFree(p1);
            return fail(&plan->err, ETD_E_NOMEM, "band scratch");
        }
        tmp = {p1, p2};
        flags = (uint8_t*)p1;
        cnt = (int64_t*)p2;
        total = cnt + band_blocks(n) + 2;
    }
    if (dtype == ETD_F64) band_flags<double>(n, (const double*)phi, threshold, flags, s);
    else band_flags<float>(n, (const float*)phi, threshold, flags, s);
    band_compact(n, flags, cnt, capacity > 0 ? dev_idx_out : nullptr, capacity, total, s);
    int64_t c = 0;
    hipError_t e = hipMemcpyAsync(&c, total, sizeof(int64_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    for (void* p : tmp) (void)hipFree(p);
    if (e != hipSuccess) return fail(&plan->err, ETD_E_HIP, std::string("band: ") + hipGetErrorString(e));
    *count_out = c;
    if (c > capacity) return fail(&plan->err, ETD_E_CAPACITY, "band larger than capacity");
    return ETD_OK;
}

etd_status etd_narrowband_build_noalloc(etd_plan_t plan, const void* phi, etd_dtype dtype, int64_t n,
                                        double threshold, int32_t* dev_idx_out, int64_t capacity,
                                        int64_t* count_out) {
    if (!plan) return fail(nullptr, ETD_E_ARG, "null plan");
    if (!count_out) return fail(&plan->err, ETD_E_ARG, "null count_out");
    if (n < 0) return fail(&plan->err, ETD_E_ARG, "n must be >= 0");
    if (n > 0 && !phi) return fail(&plan->err, ETD_E_ARG, "null phi");
    if (!std::isfinite(threshold) || threshold <= 0.0) return fail(&plan->err, ETD_E_ARG, "threshold must be > 0");
    if (capacity < 0) return fail(&plan->err, ETD_E_ARG, "capacity must be >= 0");
    if (capacity > 0 && !dev_idx_out) return fail(&plan->err, ETD_E_ARG, "null index buffer");
    if (dtype != ETD_F64 && dtype != ETD_F32) return fail(&plan->err, ETD_E_ARG, "bad dtype");
    if (n > band_static_max_points())
        return fail(&plan->err, ETD_E_SIZE,
                    "n = " + std::to_string(n) + " exceeds the static scratch's limit of " +
                        std::to_string(band_static_max_points()) + " points");
    int64_t c = 0;
    const hipError_t e =
        dtype == ETD_F64
            ? band_build_static<double>(plan->device, (long)n, (const double*)phi, threshold, dev_idx_out, capacity, &c,
                                        plan->stream)
            : band_build_static<float>(plan->device, (long)n, (const float*)phi, threshold, dev_idx_out, capacity, &c,
                                       plan->stream);
    if (e != hipSuccess) return fail(&plan->err, ETD_E_HIP, std::string("band (static scratch): ") + hipGetErrorString(e));
    *count_out = c;
    if (c > capacity) return fail(&plan->err, ETD_E_CAPACITY, "band larger than capacity");
    return ETD_OK;
}

etd_status etd_spectral_apply(etd_plan_t plan, int instance, etd_spectral_op op, const void* in, void* out,
                              etd_dtype dtype) {
    etd_status st = check_instance(plan, instance);
    if (st != ETD_OK) return st;
    if (!in || !out) return fail(&plan->err, ETD_E_ARG, "null pointer");
    if (dtype != ETD_F64 && dtype != ETD_F32) return fail(&plan->err, ETD_E_ARG, "bad dtype");
    Instance& I = plan->inst[instance];
    const bool two_d = I.g.nx == 1;
    SpecOp sop;
    bool ident = false;
    switch (op) {
        case ETD_OP_IDENTITY: ident = true; sop = SPEC_NEG_K2; break;
        case ETD_OP_LAPLACE: sop = SPEC_NEG_K2; break;
        case ETD_OP_DX: sop = two_d ? SPEC_IKY : SPEC_IKX; break;
        case ETD_OP_DY: sop = two_d ? SPEC_IKZ : SPEC_IKY; break;
        case ETD_OP_DZ:
            if (two_d) return fail(&plan->err, ETD_E_ARG, "DZ on a 2D grid");
            sop = SPEC_IKZ;
            break;
        case ETD_OP_LAPINV: sop = SPEC_INV_FD; break;
        default: return fail(&plan->err, ETD_E_ARG, "unknown spectral op");
    }
    hipStream_t s = plan->stream;
    const GridK& g = I.g;
    const long n = g.nreal();
    auto run = [&](auto tag, void* rbuf, void* sa, void* sb, void* stmp, const FFTTables<decltype(tag)>& t) {
        using T = decltype(tag);
        load_field<T>(n, in, dtype, (T*)rbuf, s);
        hipError_t e = fft_r2c_3d<T>(g, t, (const T*)rbuf, (c2<T>*)sa, s);
        if (e != hipSuccess) return e;
        const c2<T>* src = (const c2<T>*)sa;
        if (!ident) {
            spec_apply<T>(g, sop, (const c2<T>*)sa, (c2<T>*)sb, I.fd, s);
            src = (const c2<T>*)sb;
        }
        if ((e = fft_c2r_3d<T>(g, t, src, (c2<T>*)stmp, (T*)rbuf, s)) != hipSuccess) return e;
        store_field<T>(n, (const T*)rbuf, dtype, out, s);
        return hipGetLastError();
    };
    hipError_t e;
    if (I.d.model == ETD_COUPLED) {
        e = I.f32 ? run(0.0f, I.P, I.Sa, I.Sb, I.Stmp, I.tf) : run(0.0, I.P, I.Sa, I.Sb, I.Stmp, I.td);
    } else {
        e = I.f32 ? run(0.0f, I.qf, I.Sb, I.Sb, I.Sgu, I.tf) : run(0.0, I.q, I.Sa, I.Sa, I.Stmp, I.td);
    }
    if (e != hipSuccess) return fail(&plan->err, ETD_E_HIP, std::string("spectral_apply: ") + hipGetErrorString(e));
    return ETD_OK;
}

etd_status etd_pass_timing(etd_plan_t plan, int enable, etd_pass_times* out) {
    if (!plan) return fail(nullptr, ETD_E_ARG, "null plan");
    if (enable) {
        plan->hook.reset();
        plan->timing = true;
        fft_set_pass_hook(&plan->hook);
        return ETD_OK;
    }
    fft_set_pass_hook(nullptr);
    plan->timing = false;
    HIPCHK(plan, hipStreamSynchronize(plan->stream));
    etd_pass_times t{};
    for (const auto& r : plan->hook.recs) {
        float ms = 0.f;
        HIPCHK(plan, hipEventElapsedTime(&ms, r.e0, r.e1));
        if (r.kind < 0 || r.kind >= ETD_PASS_KINDS) continue;
        t.launches[r.kind] += 1;
        t.total_ms[r.kind] += ms;
        t.bytes[r.kind] += r.bytes;
    }
    plan->hook.reset();
    if (out) *out = t;
    return ETD_OK;
}

etd_status etd_surface_lapinv(etd_plan_t plan, int instance, const void* g, const void* f, const uint8_t* mask,
                              void* psi, etd_dtype dtype, double tol, int max_iter, int* iters_out,
                              double* relres_out) {
    etd_status st = check_instance(plan, instance);
    if (st != ETD_OK) return st;
    if (!g || !f || !mask || !psi) return fail(&plan->err, ETD_E_ARG, "null pointer");
    if (dtype != ETD_F64 && dtype != ETD_F32) return fail(&plan->err, ETD_E_ARG, "bad dtype");
    if (!(std::isfinite(tol) && tol > 0.0)) return fail(&plan->err, ETD_E_ARG, "tol must be finite and > 0");
    if (max_iter < 1) return fail(&plan->err, ETD_E_ARG, "max_iter must be >= 1");
    Instance& I = plan->inst[instance];
    if ((st = ensure_surface(plan, I)) != ETD_OK) return st;
    hipStream_t s = plan->stream;
    const long n = I.g.nreal();
    const SurfaceWork& w = I.sw;
    band_compact(n, mask, w.cnt, w.idx, n, w.total, s);
    SurfaceResult r;
    hipError_t e = dtype == ETD_F64
                       ? surface_lapinv<double>(I.g, (const double*)g, (const double*)f, mask, w.idx, w.total,
                                                (double*)psi, w, tol, max_iter, false, &r, s)
                       : surface_lapinv<float>(I.g, (const float*)g, (const float*)f, mask, w.idx, w.total,
                                               (float*)psi, w, tol, max_iter, false, &r, s);
    HIPCHK(plan, e);
    if (iters_out) *iters_out = r.iters;
    if (relres_out) *relres_out = r.relres;
    return ETD_OK;
}

etd_status etd_plan_query(etd_plan_t plan, int instance, etd_query what, double* out) {
    etd_status st = check_instance(plan, instance);
    if (st != ETD_OK) return st;
    if (!out) return fail(&plan->err, ETD_E_ARG, "null output");
    const Instance& I = plan->inst[instance];
    switch (what) {
        case ETD_Q_B: *out = I.FK.B; break;
        case ETD_Q_B_MBP: *out = I.Bmbp; break;
        case ETD_Q_B_ES: *out = I.Bes; break;
        case ETD_Q_C: *out = I.C; break;
        case ETD_Q_RHO: *out = I.rho; break;
        case ETD_Q_CHEB_DEG: *out = (double)std::max(I.ch1.size(), I.ch2.size()); break;
        case ETD_Q_A0: *out = I.A0; break;
        case ETD_Q_WORKSPACE: *out = (double)I.bytes; break;
        case ETD_Q_SURF_ITERS: *out = (double)I.surf_last.iters; break;
        case ETD_Q_SURF_RELRES: *out = I.surf_last.relres; break;
        default: return fail(&plan->err, ETD_E_ARG, "unknown query");
    }
    return ETD_OK;
}

}  // extern "C"
