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


// Philox4x32-10, the counter-based generator of Salmon, Moraes, Dror and
// Shaw (SC'11): ten rounds of two 32x32->64-bit products (multipliers
// 0xD2511F53, 0xCD9E8D57) that mix the four counter words with the two key
// words, the key advancing by the Weyl constants 0x9E3779B9, 0xBB67AE85.
__device__ inline uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
        c = make_uint4((uint32_t)(p1 >> 32) ^ c.y ^ k0, (uint32_t)p1, (uint32_t)(p0 >> 32) ^ c.w ^ k1,
                       (uint32_t)p0);
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

// The thermostat's draws for particle `id` (original id) at step `step`:
// counters (id, step_lo, step_hi, 0) and (id, step_lo, step_hi, 1) under the
// key (seed_lo, seed_hi). The particle collides when the first word is below
// the threshold; its three standard normal deviates come from the
// Box-Muller transform sqrt(-2 ln a) (cos 2 pi b, sin 2 pi b) of the word
// pairs (w1, w2) and (w3, w4), a word u read as the uniform (u + 1/2) 2^-32.
__device__ inline double u01(uint32_t u) { return ((double)u + 0.5) * (1.0 / 4294967296.0); }
__device__ inline bool thermo_draw(const DynC &d, uint32_t id, int64_t step, double z[3]) {
    const uint32_t slo = (uint32_t)(uint64_t)step, shi = (uint32_t)((uint64_t)step >> 32);
    const uint4 a = philox4x32_10(make_uint4(id, slo, shi, 0u), d.seed_lo, d.seed_hi);
    if (a.x >= d.thermo_thr) return false;
    const uint4 b = philox4x32_10(make_uint4(id, slo, shi, 1u), d.seed_lo, d.seed_hi);
    const double two_pi = 6.283185307179586476925286766559;
    const double r1 = sqrt(-2.0 * log(u01(a.y))), t1 = two_pi * u01(a.z);
    const double r2 = sqrt(-2.0 * log(u01(a.w))), t2 = two_pi * u01(b.x);
    z[0] = r1 * cos(t1);
    z[1] = r1 * sin(t1);
    z[2] = r2 * cos(t2);
    return true;
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
