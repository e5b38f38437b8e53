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

// Sum of v over the 256 threads of a workgroup in a fixed tree order; every
// thread returns the total.  sh: 256 doubles of LDS, free on entry; ends
// behind a barrier.
__device__ __forceinline__ double block_sum_256(double v, double* sh) {
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

}  // namespace etd
