// Line-FFT driver with register-resident first and last stages (device code).
//
// A workgroup transforms L lines of length N, each carrying NS "slots"
// (independent transforms formed from the same loaded elements, e.g. S,
// i k S and -k^2 S).  Stage 1 reads its R inputs per butterfly straight from
// global memory (Op::load), does the DFT in registers for every slot and
// writes the autosorted results to LDS; the middle stages run in LDS
// (stockham.h); the last stage reads LDS, applies its twiddles and hands each
// output straight to Op::store.  A transform of R1 * R2 * R3 points therefore
// makes two LDS round trips instead of four, and a single-stage transform none.
//
// LF selects the thread mapping of the global accesses: true (strided line
// passes) puts consecutive lines on consecutive threads, so a wavefront reads
// runs of contiguous line starts; false (contiguous rows) puts consecutive
// elements of a line on consecutive threads.
//
// Op concept (T the real type):
//   static constexpr int NS;                                   // slots per line
//   __device__ void load(int l, int e, c2<T>* v) const;        // v[0..NS) at element e of line l
//   __device__ void store(int l, int s, int e, c2<T> v) const; // output of slot s at element e
#pragma once

#include <type_traits>

#include "stockham.h"

namespace etd {
namespace stk {

// Radix of the first stage for L lines of length N: the plan's own, unless a
// radix-8 first stage leaves threads of the workgroup without a butterfly
// (lengths 32 and 64 at 16 lines); then 4 or 2, so every thread holds one
// (one LDS stage more).  The first stage issues the pass's global loads.
template <int N, int L> constexpr int first_radix() {
    constexpr int R = NextRadix<N>::v;
    if constexpr (R != 8 || L * (N / 8) >= kThreads) return R;
    else return L * (N / 4) >= kThreads ? 4 : 2;
}

// First stage (span 1, radix R): global -> registers -> DFT -> LDS.
// When the values of all of a thread's butterflies fit in 32 registers, every
// load is issued before the first transform, so one memory latency covers
// them all (a loop over butterflies waits for each one's loads in turn).
// Larger sets (FP64, length 512, two fields) keep the loop: there the extra
// registers cost more occupancy than the overlap gains (measured).
// An Op may declare kFetchAll = false to keep the first stage's loop
// (a register-heavy Op whose occupancy the early loads would lower).
template <class Op, class = void> struct FetchAllOf {
    static constexpr bool v = true;
};
template <class Op> struct FetchAllOf<Op, std::enable_if_t<!Op::kFetchAll>> {
    static constexpr bool v = false;
};

template <typename T, int N, int L, int LS, int R, int DIR, bool LF, class Op>
__device__ __forceinline__ void first_stage(c2<T>* lds, const Op& op) {
    constexpr int NS = Op::NS;
    constexpr int NR = N / R;
    constexpr int NB = L * NR;
    constexpr int IT = (NB + kThreads - 1) / kThreads;
    if constexpr (FetchAllOf<Op>::v && IT * NS * R * sizeof(c2<T>) <= 32 * 4) {
        c2<T> v[IT][NS][R];
#pragma unroll
        for (int it = 0; it < IT; ++it) {
            const int b = threadIdx.x + it * kThreads;
            if ((NB % kThreads == 0) || b < NB) {
                const int l = LF ? b % L : b / NR, j = LF ? b / L : b % NR;
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    c2<T> x[NS];
                    op.load(l, j + r * NR, x);
#pragma unroll
                    for (int s = 0; s < NS; ++s) v[it][s][r] = x[s];
                }
            }
        }
#pragma unroll
        for (int it = 0; it < IT; ++it) {
            const int b = threadIdx.x + it * kThreads;
            if ((NB % kThreads == 0) || b < NB) {
                const int l = LF ? b % L : b / NR, j = LF ? b / L : b % NR;
#pragma unroll
                for (int s = 0; s < NS; ++s) {
                    dftR<T, R, DIR>(v[it][s]);
                    c2<T>* dst = lds + (s * L + l) * LS;
#pragma unroll
                    for (int r = 0; r < R; ++r) dst[sk_add<16 % R == 0>(j * R, sk(j * R), r)] = v[it][s][r];
                }
            }
        }
        __syncthreads();
        return;
    }
    for (int b = threadIdx.x; b < NB; b += kThreads) {
        const int l = LF ? b % L : b / NR, j = LF ? b / L : b % NR;
        c2<T> v[NS][R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            c2<T> x[NS];
            op.load(l, j + r * NR, x);
#pragma unroll
            for (int s = 0; s < NS; ++s) v[s][r] = x[s];
        }
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            dftR<T, R, DIR>(v[s]);
            c2<T>* dst = lds + (s * L + l) * LS;
#pragma unroll
            for (int r = 0; r < R; ++r) dst[sk_add<16 % R == 0>(j * R, sk(j * R), r)] = v[s][r];
        }
    }
    __syncthreads();
}

// The epilogue's own global reads: a store Op may declare a type Pre, a
// prefetch and kPrefetch (true to use them); the last stage of a transform then issues the prefetches of a
// butterfly's R outputs before the butterfly and hands each output its Pre
// (last_stage: prefetch(l, s, e, Pre&), store(l, s, e, v, pre);
// last_stage_indexed: prefetch(l, e, Pre&), store_at(slot, l, e, v, pre);
// joint transforms: prefetch(l, e, Pre&), store_joint(l, e, v, pre)), so
// a thread's fetches overlap instead of each waiting in turn.
template <class Op, class = void> struct PrefetchOf {
    static constexpr bool v = false;
    struct Pre {};
};
template <class Op> struct PrefetchOf<Op, std::void_t<typename Op::Pre>> {
    static constexpr bool v = Op::kPrefetch;
    using Pre = typename Op::Pre;
};

// Last stage (span SP = N / R): LDS -> twiddles -> DFT -> Op::store.
template <typename T, int N, int L, int LS, int R, int DIR, bool LF, class Op>
__device__ __forceinline__ void last_stage(const c2<T>* lds, const c2<T>* tw, const Op& op) {
    constexpr int NS = Op::NS;
    constexpr int SP = N / R;
    constexpr int LL = L * NS;
    constexpr int NB = LL * SP;
    constexpr int IT = (NB + kThreads - 1) / kThreads;
    if constexpr (!PrefetchOf<Op>::v) {   // a loop: fewer registers than the unrolled form
        for (int b = threadIdx.x; b < NB; b += kThreads) {
            const int ll = LF ? b % LL : b / SP, j = LF ? b / LL : b % SP;
            const int s = ll / L, l = ll % L;
            const c2<T>* src = lds + ll * LS;
            c2<T> v[R];
#pragma unroll
            for (int r = 0; r < R; ++r) v[r] = src[sk_add<SP % 16 == 0>(j, sk(j), r * SP)];
#pragma unroll
            for (int r = 1; r < R; ++r) {
                c2<T> w = tw[r * j];
                if constexpr (DIR > 0) w.y = -w.y;
                v[r] = cmul(v[r], w);
            }
            dftR<T, R, DIR>(v);
#pragma unroll
            for (int r = 0; r < R; ++r) op.store(l, s, j + r * SP, v[r]);
        }
        return;
    }
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        const int b = threadIdx.x + it * kThreads;
        if ((NB % kThreads == 0) || b < NB) {
            const int ll = LF ? b % LL : b / SP, j = LF ? b / LL : b % SP;
            const int s = ll / L, l = ll % L;
            typename PrefetchOf<Op>::Pre pre[R];
            if constexpr (PrefetchOf<Op>::v) {
#pragma unroll
                for (int r = 0; r < R; ++r) op.prefetch(l, s, j + r * SP, pre[r]);
            }
            const c2<T>* src = lds + ll * LS;
            c2<T> v[R];
#pragma unroll
            for (int r = 0; r < R; ++r) v[r] = src[sk_add<SP % 16 == 0>(j, sk(j), r * SP)];
#pragma unroll
            for (int r = 1; r < R; ++r) {
                c2<T> w = tw[r * j];
                if constexpr (DIR > 0) w.y = -w.y;
                v[r] = cmul(v[r], w);
            }
            dftR<T, R, DIR>(v);
#pragma unroll
            for (int r = 0; r < R; ++r) {
                if constexpr (PrefetchOf<Op>::v) op.store(l, s, j + r * SP, v[r], pre[r]);
                else op.store(l, s, j + r * SP, v[r]);
            }
        }
    }
}

// Ops with kIndexed (NS == 1) take each last-stage output through
// store_at(slot, l, e, v), slot = it R + r its compile-time position among the
// outputs of this thread.  Every transform of one line set maps outputs to
// threads the same way, so such an Op can carry per-point values in
// registers from one transform of the set to the next.
template <class Op, class = void> struct IndexedOf {
    static constexpr bool v = false;
};
template <class Op> struct IndexedOf<Op, std::enable_if_t<Op::kIndexed>> {
    static constexpr bool v = true;
};

template <typename T, int N, int L, int LS, int R, int DIR, bool LF, class Op>
__device__ __forceinline__ void last_stage_indexed(const c2<T>* lds, const c2<T>* tw, const Op& op) {
    constexpr int SP = N / R;
    constexpr int NB = L * SP;
    constexpr int IT = (NB + kThreads - 1) / kThreads;
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        const int b = threadIdx.x + it * kThreads;
        if ((NB % kThreads == 0) || b < NB) {
            const int l = LF ? b % L : b / SP, j = LF ? b / L : b % SP;
            typename PrefetchOf<Op>::Pre pre[R];
            if constexpr (PrefetchOf<Op>::v) {
#pragma unroll
                for (int r = 0; r < R; ++r) op.prefetch(l, j + r * SP, pre[r]);
            }
            const c2<T>* src = lds + l * LS;
            c2<T> v[R];
#pragma unroll
            for (int r = 0; r < R; ++r) v[r] = src[sk_add<SP % 16 == 0>(j, sk(j), r * SP)];
#pragma unroll
            for (int r = 1; r < R; ++r) {
                c2<T> w = tw[r * j];
                if constexpr (DIR > 0) w.y = -w.y;
                v[r] = cmul(v[r], w);
            }
            dftR<T, R, DIR>(v);
#pragma unroll
            for (int r = 0; r < R; ++r) {
                if constexpr (PrefetchOf<Op>::v) op.store_at(it * R + r, l, j + r * SP, v[r], pre[r]);
                else op.store_at(it * R + r, l, j + r * SP, v[r]);
            }
        }
    }
}

// Stages from span NSP on; the last one goes to Op::store (Op::store_at for
// an indexed Op).
template <typename T, int N, int LL, int LS, int NSP, int DIR, bool LF, class Op>
__device__ __forceinline__ void middle_and_last(c2<T>* lds, const c2<T>* tw, const Op& op) {
    constexpr int R = NextRadix<N / NSP>::v;
    if constexpr (NSP * R == N) {
        if constexpr (IndexedOf<Op>::v) last_stage_indexed<T, N, LL, LS, R, DIR, LF, Op>(lds, tw, op);
        else last_stage<T, N, LL / Op::NS, LS, R, DIR, LF, Op>(lds, tw, op);
    } else {
        stage<T, N, LL, LS, R, NSP, DIR>(lds, tw);
        middle_and_last<T, N, LL, LS, NSP * R, DIR, LF, Op>(lds, tw, op);
    }
}

// Single-stage transform (N is one radix): global -> registers -> global.
template <typename T, int N, int L, int DIR, class Op>
__device__ __forceinline__ void single_stage(const Op& op) {
    constexpr int NS = Op::NS;
    for (int l = threadIdx.x; l < L; l += kThreads) {
        c2<T> v[NS][N];
#pragma unroll
        for (int e = 0; e < N; ++e) {
            c2<T> x[NS];
            op.load(l, e, x);
#pragma unroll
            for (int s = 0; s < NS; ++s) v[s][e] = x[s];
        }
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            dftR<T, N, DIR>(v[s]);
#pragma unroll
            for (int e = 0; e < N; ++e) op.store(l, s, e, v[s][e]);
        }
    }
}

// Global -> global: L lines x NS slots of length N; lds holds L * NS * LS
// elements, tw the N twiddles (already in LDS).
template <typename T, int N, int L, int DIR, bool LF, class Op>
__device__ __forceinline__ void lines_fft(c2<T>* lds, const c2<T>* tw, const Op& op) {
    constexpr int LS = line_stride<N>();
    constexpr int R0 = first_radix<N, L>();
    if constexpr (R0 == N) {
        single_stage<T, N, L, DIR, Op>(op);
    } else {
        first_stage<T, N, L, LS, R0, DIR, LF, Op>(lds, op);
        middle_and_last<T, N, L * Op::NS, LS, R0, DIR, LF, Op>(lds, tw, op);
    }
}

// LDS -> global: the L * NS lines (line stride LS) are already in LDS in
// natural order (after a barrier); every stage runs from LDS, the last one
// stores through Op.
template <typename T, int N, int L, int LS, int DIR, bool LF, class Op>
__device__ __forceinline__ void lines_fft_from_lds(c2<T>* lds, const c2<T>* tw, const Op& op) {
    middle_and_last<T, N, L * Op::NS, LS, 1, DIR, LF, Op>(lds, tw, op);
}

// Global -> LDS: first stage from Op::load, every later stage in LDS; the
// result is left in LDS in natural order, after a barrier.
// FIRST: the radix of the first stage (0: first_radix).
template <typename T, int N, int L, int LS, int NSLOT, int DIR, bool LF, int FIRST = 0, class Op>
__device__ __forceinline__ void lines_fft_to_lds(c2<T>* lds, const c2<T>* tw, const Op& op) {
    constexpr int R0 = FIRST > 0 ? FIRST : first_radix<N, L>();
    static_assert(N % R0 == 0, "the first radix must divide the length");
    first_stage<T, N, L, LS, R0, DIR, LF, Op>(lds, op);
    stockham<T, N, L * NSLOT, LS, R0, DIR>(lds, tw);
}

// ---------------------------------------------------------------- sequential transforms
// NT transforms per line, run one after another through the LDS of a single
// transform.  Their inputs are formed from per-element values loaded once by
// the first stage and kept in registers (Op::In), so one read of a line family
// feeds several outputs (e.g. S -> F^-1 S, F^-1 i k S, F^-1 (-k^2) S).
//
// SeqOp concept (T the real type):
//   static constexpr int NT;
//   struct In;                                                    // per-element register cache
//   void load(int l, int e, In& in) const;
//   template <int S> c2<T> input(int l, int e, const In& in) const;
//   template <int S> void store(int l, int e, c2<T> v) const;
// input<S> may also read global memory; an array read there must not be
// written by a transform S' < S of the same line (writes of transform S' are
// issued before transform S starts).

template <typename T, class Op, int S> struct SlotStore {
    static constexpr int NS = 1;
    const Op& op;
    __device__ __forceinline__ void store(int l, int, int e, c2<T> v) const { op.template store<S>(l, e, v); }
};

// First stage of transform S of a sequential Op: the inputs of the thread's
// IT butterflies (all of them fetched before the first transform when they
// fit in 32 registers, as in first_stage), radix R0, into the LDS.
template <typename T, int N, int L, int LS, int R0, int IT, bool LF, int S, int DIR, class Op>
__device__ __forceinline__ void first_stage_inputs(c2<T>* lds, const Op& op, const typename Op::In (&in)[IT][R0]) {
    constexpr int NR = N / R0;
    constexpr int NB = L * NR;
    constexpr bool kAll = FetchAllOf<Op>::v && IT * R0 * sizeof(c2<T>) <= 32 * 4;
    c2<T> v[kAll ? IT : 1][R0];
    if constexpr (kAll) {
#pragma unroll
        for (int it = 0; it < IT; ++it) {
            const int b = threadIdx.x + it * kThreads;
            if ((NB % kThreads == 0) || b < NB) {
                const int l = LF ? b % L : b / NR, j = LF ? b / L : b % NR;
#pragma unroll
                for (int r = 0; r < R0; ++r) v[it][r] = op.template input<S>(l, j + r * NR, in[it][r]);
            }
        }
    }
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        const int b = threadIdx.x + it * kThreads;
        if ((kAll && NB % kThreads == 0) || b < NB) {
            const int l = LF ? b % L : b / NR, j = LF ? b / L : b % NR;
            c2<T>* w = v[kAll ? it : 0];
            if constexpr (!kAll) {
#pragma unroll
                for (int r = 0; r < R0; ++r) w[r] = op.template input<S>(l, j + r * NR, in[it][r]);
            }
            dftR<T, R0, DIR>(w);
            c2<T>* dst = lds + l * LS;
#pragma unroll
            for (int r = 0; r < R0; ++r) dst[sk_add<16 % R0 == 0>(j * R0, sk(j * R0), r)] = w[r];
        }
    }
}

template <typename T, int N, int L, int LS, int R0, int IT, int DIR, bool LF, class Op, int S>
__device__ __forceinline__ void seq_transforms(c2<T>* lds, const c2<T>* tw, const Op& op,
                                               const typename Op::In (&in)[IT][R0]) {
    constexpr int NR = N / R0;
    constexpr int NB = L * NR;
    if constexpr (R0 == N) {
#pragma unroll
        for (int it = 0; it < IT; ++it) {
            const int l = threadIdx.x + it * kThreads;
            if (l < NB) {
                c2<T> v[R0];
#pragma unroll
                for (int r = 0; r < R0; ++r) v[r] = op.template input<S>(l, r, in[it][r]);
                dftR<T, R0, DIR>(v);
#pragma unroll
                for (int r = 0; r < R0; ++r) op.template store<S>(l, r, v[r]);
            }
        }
    } else {
        if constexpr (S > 0) __syncthreads();   // the previous transform's last stage has read the LDS
        first_stage_inputs<T, N, L, LS, R0, IT, LF, S, DIR>(lds, op, in);
        __syncthreads();
        middle_and_last<T, N, L, LS, R0, DIR, LF>(lds, tw, SlotStore<T, Op, S>{op});
    }
    if constexpr (S + 1 < Op::NT) seq_transforms<T, N, L, LS, R0, IT, DIR, LF, Op, S + 1>(lds, tw, op, in);
}

// SYNC: barrier between the loads and the first LDS writes, for an Op whose
// load() reads the LDS (a transform of data left there by an earlier phase).
template <typename T, int N, int L, int DIR, bool LF, class Op, bool SYNC = false>
__device__ __forceinline__ void lines_fft_seq(c2<T>* lds, const c2<T>* tw, const Op& op) {
    constexpr int LS = line_stride<N>();
    constexpr int R0 = first_radix<N, L>();
    constexpr int NR = N / R0;
    constexpr int NB = L * NR;
    constexpr int IT = (NB + kThreads - 1) / kThreads;
    typename Op::In in[IT][R0];
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        const int b = threadIdx.x + it * kThreads;
        if (b < NB) {
            const int l = (R0 == N) ? b : (LF ? b % L : b / NR), j = (R0 == N) ? 0 : (LF ? b / L : b % NR);
#pragma unroll
            for (int r = 0; r < R0; ++r) op.load(l, j + r * NR, in[it][r]);
        }
    }
    if constexpr (SYNC) __syncthreads();
    seq_transforms<T, N, L, LS, R0, IT, DIR, LF, Op, 0>(lds, tw, op, in);
}

// ---------------------------------------------------------------- sequential transforms, joint store
// As lines_fft_seq, but the outputs of the NT transforms are combined per
// element: the last stage maps elements to threads identically for every
// transform, so transforms 0..NT-2 leave their results in registers and the
// last one hands all NT values of element (l, e) to Op::store_joint(l, e, v).
// LDS use is that of a single transform.

constexpr int ilog2c(int m) {
    int k = 0;
    while (m > 1) {
        m /= 2;
        ++k;
    }
    return k;
}
// same rule as NextRadix
constexpr int next_radix(int m) {
    const int k = ilog2c(m);
    return (m % 3 == 0) ? 3 : (k == 1 ? 2 : ((k % 3 == 1 || k == 2) ? 4 : 8));
}
constexpr int last_radix(int n) {
    int sp = 1;
    for (;;) {
        const int r = next_radix(n / sp);
        if (sp * r == n) return r;
        sp *= r;
    }
}

template <typename T, class Op, class P>
__device__ __forceinline__ void store_joint_with(const Op& op, int l, int e, const c2<T>* o, const P& pre) {
    if constexpr (PrefetchOf<Op>::v) op.store_joint(l, e, o, pre);
    else op.store_joint(l, e, o);
}

template <typename T, int N, int L, int LS, int R, int DIR, bool LF, int NT, int IT, int S, class Op>
__device__ __forceinline__ void last_stage_stash(const c2<T>* lds, const c2<T>* tw, const Op& op,
                                                 c2<T> (&stash)[NT][IT][R]) {
    constexpr int SP = N / R;
    constexpr int NB = L * SP;
    constexpr bool kPre = (S + 1 == NT) && PrefetchOf<Op>::v;
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        const int b = threadIdx.x + it * kThreads;
        if ((NB % kThreads == 0) || b < NB) {
            const int l = LF ? b % L : b / SP, j = LF ? b / L : b % SP;
            typename PrefetchOf<Op>::Pre pre[R];
            if constexpr (kPre) {
#pragma unroll
                for (int r = 0; r < R; ++r) op.prefetch(l, j + r * SP, pre[r]);
            }
            const c2<T>* src = lds + l * LS;
            c2<T> v[R];
#pragma unroll
            for (int r = 0; r < R; ++r) v[r] = src[sk_add<SP % 16 == 0>(j, sk(j), r * SP)];
#pragma unroll
            for (int r = 1; r < R; ++r) {
                c2<T> w = tw[r * j];
                if constexpr (DIR > 0) w.y = -w.y;
                v[r] = cmul(v[r], w);
            }
            dftR<T, R, DIR>(v);
#pragma unroll
            for (int r = 0; r < R; ++r) {
                if constexpr (S + 1 < NT) {
                    stash[S][it][r] = v[r];
                } else {
                    c2<T> o[NT];
#pragma unroll
                    for (int s = 0; s + 1 < NT; ++s) o[s] = stash[s][it][r];
                    o[NT - 1] = v[r];
                    store_joint_with<T>(op, l, j + r * SP, o, pre[r]);
                }
            }
        }
    }
}

template <typename T, int N, int L, int LS, int NSP, int DIR, bool LF, int NT, int IT, int RL, int S, class Op>
__device__ __forceinline__ void middle_and_last_stash(c2<T>* lds, const c2<T>* tw, const Op& op,
                                                      c2<T> (&stash)[NT][IT][RL]) {
    constexpr int R = NextRadix<N / NSP>::v;
    if constexpr (NSP * R == N) {
        last_stage_stash<T, N, L, LS, R, DIR, LF, NT, IT, S, Op>(lds, tw, op, stash);
    } else {
        stage<T, N, L, LS, R, NSP, DIR>(lds, tw);
        middle_and_last_stash<T, N, L, LS, NSP * R, DIR, LF, NT, IT, RL, S, Op>(lds, tw, op, stash);
    }
}

template <typename T, int N, int L, int LS, int R0, int ITI, int DIR, bool LF, class Op, int S, int ITL, int RL>
__device__ __forceinline__ void seq_joint_transforms(c2<T>* lds, const c2<T>* tw, const Op& op,
                                                     const typename Op::In (&in)[ITI][R0],
                                                     c2<T> (&stash)[Op::NT][ITL][RL]) {
    constexpr int NT = Op::NT;
    constexpr int NR = N / R0;
    constexpr int NB = L * NR;
    if constexpr (R0 == N) {
        // single stage: a thread owns whole lines (ITL == ITI, RL == N)
#pragma unroll
        for (int it = 0; it < ITI; ++it) {
            const int l = threadIdx.x + it * kThreads;
            if (l < L) {
                c2<T> v[R0];
#pragma unroll
                for (int r = 0; r < R0; ++r) v[r] = op.template input<S>(l, r, in[it][r]);
                dftR<T, R0, DIR>(v);
#pragma unroll
                for (int r = 0; r < R0; ++r) {
                    if constexpr (S + 1 < NT) {
                        stash[S][it][r] = v[r];
                    } else {
                        c2<T> o[NT];
#pragma unroll
                        for (int s = 0; s + 1 < NT; ++s) o[s] = stash[s][it][r];
                        o[NT - 1] = v[r];
                        typename PrefetchOf<Op>::Pre pre{};
                        if constexpr (PrefetchOf<Op>::v) op.prefetch(l, r, pre);
                        store_joint_with<T>(op, l, r, o, pre);
                    }
                }
            }
        }
    } else {
        if constexpr (S > 0) __syncthreads();
        first_stage_inputs<T, N, L, LS, R0, ITI, LF, S, DIR>(lds, op, in);
        __syncthreads();
        middle_and_last_stash<T, N, L, LS, R0, DIR, LF, NT, ITL, RL, S, Op>(lds, tw, op, stash);
    }
    if constexpr (S + 1 < NT)
        seq_joint_transforms<T, N, L, LS, R0, ITI, DIR, LF, Op, S + 1, ITL, RL>(lds, tw, op, in, stash);
}

// SeqJointOp concept: NT, In, load, input<S> as for lines_fft_seq, and
// store_joint(int l, int e, const c2<T>* v /* NT values */).
template <typename T, int N, int L, int DIR, bool LF, class Op>
__device__ __forceinline__ void lines_fft_seq_joint(c2<T>* lds, const c2<T>* tw, const Op& op) {
    constexpr int LS = line_stride<N>();
    constexpr int R0 = NextRadix<N>::v;
    constexpr int NR = N / R0;
    constexpr int NB = L * NR;
    constexpr int ITI = (NB + kThreads - 1) / kThreads;
    constexpr int RL = (R0 == N) ? N : last_radix(N);
    constexpr int ITL = (R0 == N) ? ITI : (L * (N / RL) + kThreads - 1) / kThreads;
    typename Op::In in[ITI][R0];
#pragma unroll
    for (int it = 0; it < ITI; ++it) {
        const int b = threadIdx.x + it * kThreads;
        if (b < NB) {
            const int l = (R0 == N) ? b : (LF ? b % L : b / NR), j = (R0 == N) ? 0 : (LF ? b / L : b % NR);
#pragma unroll
            for (int r = 0; r < R0; ++r) op.load(l, j + r * NR, in[it][r]);
        }
    }
    c2<T> stash[Op::NT][ITL][RL];
    seq_joint_transforms<T, N, L, LS, R0, ITI, DIR, LF, Op, 0, ITL, RL>(lds, tw, op, in, stash);
}

// ---------------------------------------------------------------- joint transforms
// NS transforms per line held together in LDS (slot s of line l at row
// s * L + l); the last stage finishes element (l, e) of every slot in one
// thread and hands the NS results to Op::store_joint(l, e, v[NS]), so an
// epilogue can combine the slots (e.g. R = F P - c k^2 F Q).

template <typename T, int N, int L, int LS, int R, int DIR, bool LF, class Op>
__device__ __forceinline__ void last_stage_joint(const c2<T>* lds, const c2<T>* tw, const Op& op) {
    constexpr int NS = Op::NS;
    constexpr int SP = N / R;
    constexpr int NB = L * SP;
    for (int b = threadIdx.x; b < NB; b += kThreads) {
        const int l = LF ? b % L : b / SP, j = LF ? b / L : b % SP;
        c2<T> v[NS][R];
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const c2<T>* src = lds + (s * L + l) * LS;
#pragma unroll
            for (int r = 0; r < R; ++r) v[s][r] = src[sk_add<SP % 16 == 0>(j, sk(j), r * SP)];
#pragma unroll
            for (int r = 1; r < R; ++r) {
                c2<T> w = tw[r * j];
                if constexpr (DIR > 0) w.y = -w.y;
                v[s][r] = cmul(v[s][r], w);
            }
            dftR<T, R, DIR>(v[s]);
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            c2<T> o[NS];
#pragma unroll
            for (int s = 0; s < NS; ++s) o[s] = v[s][r];
            op.store_joint(l, j + r * SP, o);
        }
    }
}

template <typename T, int N, int L, int LS, int NSP, int DIR, bool LF, class Op>
__device__ __forceinline__ void middle_and_last_joint(c2<T>* lds, const c2<T>* tw, const Op& op) {
    constexpr int R = NextRadix<N / NSP>::v;
    if constexpr (NSP * R == N) {
        last_stage_joint<T, N, L, LS, R, DIR, LF, Op>(lds, tw, op);
    } else {
        stage<T, N, L * Op::NS, LS, R, NSP, DIR>(lds, tw);
        middle_and_last_joint<T, N, L, LS, NSP * R, DIR, LF, Op>(lds, tw, op);
    }
}

// JointOp concept: NS, load(l, e, v[NS]) as for lines_fft, and
// store_joint(int l, int e, const c2<T>* v /* NS values */).
template <typename T, int N, int L, int DIR, bool LF, class Op>
__device__ __forceinline__ void lines_fft_joint(c2<T>* lds, const c2<T>* tw, const Op& op) {
    constexpr int NS = Op::NS;
    constexpr int LS = line_stride<N>();
    constexpr int R0 = NextRadix<N>::v;
    if constexpr (R0 == N) {
        for (int l = threadIdx.x; l < L; l += kThreads) {
            c2<T> v[NS][N];
#pragma unroll
            for (int e = 0; e < N; ++e) {
                c2<T> x[NS];
                op.load(l, e, x);
#pragma unroll
                for (int s = 0; s < NS; ++s) v[s][e] = x[s];
            }
#pragma unroll
            for (int s = 0; s < NS; ++s) dftR<T, N, DIR>(v[s]);
#pragma unroll
            for (int e = 0; e < N; ++e) {
                c2<T> o[NS];
#pragma unroll
                for (int s = 0; s < NS; ++s) o[s] = v[s][e];
                op.store_joint(l, e, o);
            }
        }
    } else {
        first_stage<T, N, L, LS, R0, DIR, LF, Op>(lds, op);
        middle_and_last_joint<T, N, L, LS, R0, DIR, LF, Op>(lds, tw, op);
    }
}

// LDS elements needed by lines_fft plus the twiddle table.
template <typename T, int N, int L, int NS> constexpr size_t lines_smem() {
    return sizeof(c2<T>) * (size_t)(L * NS * line_stride<N>() + N);
}

// Lines per workgroup: coalescing wants >= 8 consecutive lines; keep the LDS
// of one workgroup near 64 KiB so several fit in a CU.  lines_per_block_8
// caps the tile at 8 lines, for register-heavy kernels (more resident
// workgroups per CU outweigh the shorter contiguous runs there; measured).
template <typename T, int N, int NS> constexpr int lines_per_block() {
    constexpr size_t per_line = sizeof(c2<T>) * NS * line_stride<N>();
    return per_line * 16 <= 72 * 1024 ? 16 : (per_line * 8 <= 80 * 1024 ? 8 : 4);
}
template <typename T, int N, int NS> constexpr int lines_per_block_8() {
    constexpr int L = lines_per_block<T, N, NS>();
    return L > 8 ? 8 : L;
}

}  // namespace stk
}  // namespace etd
