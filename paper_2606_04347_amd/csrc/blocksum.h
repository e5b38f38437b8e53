// Deterministic FP64 block sums (device code).
#pragma once

#include "common.h"

namespace etd {

// Neumaier-compensated FP64 accumulator.
struct Neu {
    double s = 0.0, c = 0.0;
    __device__ __forceinline__ void add(double x) {
        const double t = s + x;
        if (fabs(s) >= fabs(x)) c += (s - t) + x;
        else c += (x - t) + s;
        s = t;
    }
    __device__ __forceinline__ double val() const { return s + c; }
};

// Sum of v over the 256 threads of a workgroup in a fixed order; every
// thread returns the total.  Each 64-wide wavefront folds its values with a
// butterfly of lane exchanges (xor distances 32 ... 1, so every lane holds
// the wavefront sum), the four wavefront sums meet in LDS and are added in
// wavefront order.  sh: at least 4 doubles of LDS, free on entry; ends
// behind a barrier.
__device__ __forceinline__ double block_sum_256(double v, double* sh) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) sh[wave] = v;
    __syncthreads();
    const double r = (sh[0] + sh[1]) + (sh[2] + sh[3]);
    __syncthreads();
    return r;
}

// Largest v over the 256 threads (same pattern); every thread returns it.
__device__ __forceinline__ double block_max_256(double v, double* sh) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) sh[wave] = v;
    __syncthreads();
    const double r = fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3]));
    __syncthreads();
    return r;
}

}  // namespace etd
