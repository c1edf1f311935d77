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
        return (t & 2) ? a[2] : ((t & 1) ? a[1] : a[0]);  // t in {0, 1, 2}
    }
}

// The per-pair-type values (types 0: AA, 1: AB, 2: BB) seen from a particle
// of species si: partner species 0 gives type si, partner species 1 type
// si + 1. Picked once per particle, so a pair costs one select on the
// partner's species (a three-way choice per pair can be compiled into a
// table lookup in scratch or LDS).
template <class T>
struct PairRow {
    T c0, c1;
    __device__ PairRow(const T (&a)[3], int si) : c0(si ? a[1] : a[0]), c1(si ? a[2] : a[1]) {}
    __device__ T operator()(int sj) const { return sj ? c1 : c0; }
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
