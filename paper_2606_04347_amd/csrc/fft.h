// Batched Stockham FFTs and the 3D real transforms built from them.
#pragma once

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

// Optional per-launch timing of the FFT passes: when set, every pass launch is
// bracketed by begin(kind) / end(kind) on its stream.  kind: 0 z-r2c, 1 z-c2r,
// 2 y lines, 3 x lines.  bytes: algorithmic bytes the launch must move (each
// input element read once, each output element written once).
struct PassHook {
    virtual void begin(int kind, hipStream_t s) = 0;
    virtual void end(int kind, double bytes, hipStream_t s) = 0;
    virtual ~PassHook() = default;
};
void fft_set_pass_hook(PassHook* h);

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

}  // namespace etd
