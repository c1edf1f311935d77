// step_common.h -- helpers shared by the per-step kernels (dynamics and
// steepest descent): kernel arguments, pair/species constant selection,
// wavefront reductions and the double-single periodic wrap.
#pragma once

#include "internal.h"

namespace ljmd {

struct StepArgs {
    State st;
    Geom g;
    BoxC box;
    PairC pc;
    DynC dyn;
    int cur;
    int forced;
    int mode;
    int slot;
    int64_t step;
};

template <int NS, class T>
__device__ inline T by_t(int t, const T (&a)[3]) {
    if constexpr (NS == 1) {
        return a[0];
    } else {
        return t == 0 ? a[0] : (t == 1 ? a[1] : a[2]);
    }
}

// A per-pair-type table held in registers: selecting among loaded values,
// never indexing the kernel-argument copy (which would place it in scratch).
template <class T>
struct Tri {
    T v0, v1, v2;
    __device__ explicit Tri(const T (&a)[3]) : v0(a[0]), v1(a[1]), v2(a[2]) {}
    __device__ T operator()(int t) const { return t == 0 ? v0 : (t == 1 ? v1 : v2); }
};

template <class T>
__device__ inline T by_s(int s, const T (&a)[2]) {
    return s == 0 ? a[0] : a[1];
}

template <class T>
__device__ inline T wave_sum(T v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

__device__ inline uint32_t wave_max_u(uint32_t v) {
    for (int o = 32; o > 0; o >>= 1) {
        uint32_t y = __shfl_xor(v, o);
        v = y > v ? y : v;
    }
    return v;
}


// Double-single wrap into [0, L) with image bookkeeping.
__device__ inline void wrap_ds(dsf &x, float Lhi, float Llo, int &im) {
    if (x.hi < 0.0f || (x.hi == 0.0f && x.lo < 0.0f)) {
        x = ds_add(x, dsf{Lhi, Llo});
        im -= 1;
    } else if (x.hi > Lhi || (x.hi == Lhi && x.lo >= Llo)) {
        x = ds_add(x, dsf{-Lhi, -Llo});
        im += 1;
    }
}


}  // namespace ljmd
