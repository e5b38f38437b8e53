// Kernel launches that the grouped step schedule can merge across instances.
//
// A kernel on the coupled step path is written as a body struct B with a
// static device function B::run(params...) and a thin __global__ wrapper that
// calls it.  Its launcher calls launch_k<B>(wrapper, grid, block, smem, s,
// args...).  Normally that is a plain launch of the wrapper.  While a
// LaunchRecorder is installed (the grouped schedule records the steps of its
// instances), the launch is recorded instead: the grouped twin k_grouped<B>
// and the arguments packed into one trivially copyable struct.  Instances
// whose recorded launches agree in kernel, grid, block and LDS (instances of
// one shape and configuration) then run each pass as ONE launch of the twin
// over a grid of gridDim.x tiles by as many rows as instances: blockIdx.y
// selects the instance, whose arguments the twin reads from a device table.
#pragma once

#include <hip/hip_runtime.h>

#include <cstring>
#include <vector>

#include "common.h"
#include "stockham.h"

namespace etd {

// A flat, trivially copyable argument record (same layout on host and device).
template <typename... P> struct Pack;
template <> struct Pack<> {};
template <typename H, typename... R> struct Pack<H, R...> {
    H h;
    Pack<R...> r;
};

template <typename... P> struct PackMaker;
template <> struct PackMaker<> {
    static Pack<> make() { return Pack<>{}; }
};
template <typename H, typename... R> struct PackMaker<H, R...> {
    static Pack<H, R...> make(H h, R... r) {
        Pack<H, R...> p;
        p.h = h;
        p.r = PackMaker<R...>::make(r...);
        return p;
    }
};

template <typename B, typename... D> __device__ __forceinline__ void apply_pack(const Pack<>&, D... d) {
    B::run(d...);
}
template <typename B, typename H, typename... R, typename... D>
__device__ __forceinline__ void apply_pack(const Pack<H, R...>& p, D... d) {
    apply_pack<B>(p.r, d..., p.h);
}

// The grouped twin of a kernel: row blockIdx.y of the grid runs instance
// blockIdx.y with the arguments tab[blockIdx.y].
template <typename B, typename... P>
__global__ __launch_bounds__(stk::kThreads) void k_grouped(const Pack<P...>* __restrict__ tab) {
    const Pack<P...> a = tab[blockIdx.y];
    apply_pack<B>(a);
}

struct LaunchRecord {
    const void* fn;   // k_grouped<B, P...>
    dim3 grid, block;
    size_t smem;
    std::vector<unsigned char> args;   // Pack<P...>
};

struct LaunchRecorder {
    std::vector<LaunchRecord> ops;
};

// The recorder of the grouped schedule while it records a step (host thread).
extern thread_local LaunchRecorder* g_launch_recorder;

template <typename X> struct ident {
    using type = X;
};

// The launch of kernel (or its record).  Like hipLaunchKernelGGL it returns
// nothing: a launch error is left for the caller's hipGetLastError.
template <typename B, typename... P>
void launch_k(void (*kernel)(P...), dim3 grid, dim3 block, size_t smem, hipStream_t s,
                    typename ident<P>::type... a) {
    if (LaunchRecorder* r = g_launch_recorder) {
        const Pack<P...> p = PackMaker<P...>::make(a...);
        LaunchRecord rec{reinterpret_cast<const void*>(&k_grouped<B, P...>), grid, block, smem, {}};
        rec.args.resize(sizeof p);
        std::memcpy(rec.args.data(), &p, sizeof p);
        r->ops.push_back(std::move(rec));
        return;
    }
    hipLaunchKernelGGL(kernel, grid, block, smem, s, a...);
}

}  // namespace etd
