// Batched Stockham FFTs and the 3D real transforms built from them.
#pragma once

#include <mutex>

#include "common.h"

namespace etd {

// Twiddle tables w_N^k = exp(-2 pi i k / N), k = 0..N-1, one per transform
// length, formed on the host in extended precision from the exact integer
// index and rounded to T.
template <typename T> struct FFTTables {
    const c2<T>* tx = nullptr;      // length nx (unused when nx == 1)
    const c2<T>* ty = nullptr;      // length ny
    const c2<T>* tzh = nullptr;     // length nz / 2 (the complex half-length transform)
    const c2<T>* tzf = nullptr;     // length nz (r2c / c2r post- and pre-twiddles)
};

// True if a 1D transform of this length is compiled in (8..512, 2^a or 3 * 2^a).
bool fft_length_supported(int n);
#define ETD_FFT_SIZES(X) X(8) X(16) X(32) X(64) X(128) X(256) X(512) X(12) X(24) X(48) X(96) X(192) X(384)

// Raises the dynamic-LDS limit of one kernel instantiation once (each launcher
// instantiation owns its flag).
// LDS of one gfx950 workgroup; every dynamic tile is checked against it at
// compile time (the static tile tables of a kernel come on top; a launch
// asking for more than the device holds fails rather than overrunning).
constexpr size_t kLdsBytes = 160 * 1024;

template <typename K> void set_smem_limit(K kernel, size_t bytes, std::once_flag& flag) {
    std::call_once(flag, [&] {
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    });
}

// Optional per-launch timing of the FFT passes: when set, every pass launch is
// bracketed by begin(kind) / end(kind) on its stream (kinds: PassKind).
// bytes: algorithmic bytes the launch must move (each input element read
// once, each output element written once).
enum PassKind {
    PASS_Z_R2C = 0,        // z rows, real -> half spectrum
    PASS_Z_C2R = 1,        // z rows, half spectrum -> real
    PASS_Y = 2,            // y lines
    PASS_X = 3,            // x lines
    PASS_X_DERIV = 4,      // inverse x lines, S -> (S, i kx S, -kx^2 S)
    PASS_Y_DERIV = 5,      // inverse y lines, 3 -> 4 spectra
    PASS_Z_DERIV = 6,      // z rows c2r, 4 spectra -> phi, grad phi, lap phi
    PASS_Z_R2C_PAIR = 7,   // z rows r2c of two fields
    PASS_Y_PAIR = 8,       // forward y lines of two spectra
    PASS_X_ETD = 9,        // forward x lines of two spectra + ETD combine
    PASS_LAPINV = 10,      // last forward axis, times 1/mu, inverse along the same axis
    PASS_Z_RECOVER = 11,   // z rows c2r of an increment with the recovery of U
    // kernels other than FFT passes (timed through the same hook)
    PASS_BAND = 12,        // narrow-band flags and compaction
    PASS_R1 = 13,          // R1 remainder (stencil of u and g(phi))
    PASS_P2 = 14,          // R2 remainder P2 (stencil of u, g, v)
    PASS_POINT = 15,       // coupled pointwise kernels (velocity, q and g u, mass projection)
    PASS_REDUCE = 16,      // FP64 reductions
    PASS_FIXED_STENCIL = 17,   // fixed model: Chebyshev recurrence and L apply (stencils)
    PASS_FIXED_POINT = 18,     // fixed model: pointwise kernels
    PASS_Z_R2C_R1 = 19,    // z rows r2c of (P1, W'(phi) - A1 phi) formed in the load (R1 fused)
    PASS_Z_R2C_P2 = 20,    // z rows r2c of (P2, g u) formed in the load (P2 fused)
    PASS_Z_R2C_Q = 21,     // z rows r2c of q = g (u - ubar) formed in the load, with its sum
    PASS_KIND_COUNT = 24
};
struct PassHook {
    virtual void begin(int kind, hipStream_t s) = 0;
    virtual void end(int kind, double bytes, hipStream_t s) = 0;
    virtual ~PassHook() = default;
};
void fft_set_pass_hook(PassHook* h);
extern PassHook* g_pass_hook;

// Run one pass launch under the optional timing hook.
template <typename F> hipError_t timed_pass(int kind, double bytes, hipStream_t s, F&& launch) {
    if (g_pass_hook) g_pass_hook->begin(kind, s);
    hipError_t e = launch();
    if (g_pass_hook) g_pass_hook->end(kind, bytes, s);
    return e;
}

// Host-side table of exp(-2 pi i k / n), k < n, in double (extended-precision trig).
void fft_twiddles_host(int n, double* re_im /* 2n values */);

// real [nx][ny][nz] -> half spectrum [nx][ny][nz/2+1], forward, unnormalized.
template <typename T>
hipError_t fft_r2c_3d(const GridK& g, const FFTTables<T>& t, const T* in, c2<T>* out, hipStream_t s);

// half spectrum -> real, inverse with the 1/(nx ny nz) normalization.  The
// input is preserved; tmp must hold nspec complex values.  The imaginary parts
// of the kz = 0 and kz = nz/2 bins are ignored, i.e. the Hermitian part of the
// spectrum is transformed.
template <typename T>
hipError_t fft_c2r_3d(const GridK& g, const FFTTables<T>& t, const c2<T>* in, c2<T>* tmp, T* out,
                      hipStream_t s);

// Single passes (timed like the 3D transforms).  z: real rows <-> half-spectrum
// rows (forward = r2c); y / x: in-place-capable complex line passes over the
// half spectrum, dir -1 forward, +1 inverse (unnormalized; the z c2r pass
// applies scale).
template <typename T>
hipError_t fft_pass_z(const GridK& g, const FFTTables<T>& t, bool forward, const void* in, void* out, T scale,
                      hipStream_t s);
template <typename T>
hipError_t fft_pass_y(const GridK& g, const FFTTables<T>& t, int dir, const c2<T>* in, c2<T>* out, hipStream_t s);
template <typename T>
hipError_t fft_pass_x(const GridK& g, const FFTTables<T>& t, int dir, const c2<T>* in, c2<T>* out, hipStream_t s);

}  // namespace etd
