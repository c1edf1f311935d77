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

// Data-parallel-primitive (DPP) moves within a row of 16 lanes, no LDS
// round trip: CTRL is the move (quad permutations 0x00-0xff, row mirrors
// 0x140 / 0x141, row broadcasts 0x142 / 0x143), ROWM the rows written; other
// lanes read 0. Every lane of the wavefront must be active.
template <int CTRL, int ROWM = 0xf>
__device__ inline uint32_t dpp_u(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROWM, 0xf, false);
}
template <int CTRL, int ROWM = 0xf>
__device__ inline float dpp_f(float v) {
    return __uint_as_float(dpp_u<CTRL, ROWM>(__float_as_uint(v)));
}
template <int CTRL, int ROWM = 0xf>
__device__ inline double dpp_d(double v) {
    const uint64_t b = (uint64_t)__double_as_longlong(v);
    const uint64_t lo = dpp_u<CTRL, ROWM>((uint32_t)b), hi = dpp_u<CTRL, ROWM>((uint32_t)(b >> 32));
    return __longlong_as_double((long long)((hi << 32) | lo));
}
constexpr int kDppXor1 = 0xb1, kDppXor2 = 0x4e;  // quad permutations [1,0,3,2], [2,3,0,1]

// Sum (max) over the wavefront, complete in lane 63: lane pairs and quads,
// half-row and row mirrors (after each step every lane of a quad, half row,
// row holds the same value), then row 0 into row 1 and row 2 into row 3,
// and row 1 into rows 2 and 3. A fixed order, so the result is
// reproducible.
__device__ inline double wave_sum_last(double v) {
    v += dpp_d<kDppXor1>(v);
    v += dpp_d<kDppXor2>(v);
    v += dpp_d<0x141>(v);
    v += dpp_d<0x140>(v);
    v += dpp_d<0x142, 0xa>(v);
    v += dpp_d<0x143, 0xc>(v);
    return v;
}
__device__ inline uint32_t wave_max_last(uint32_t v) {
    v = max(v, dpp_u<kDppXor1>(v));
    v = max(v, dpp_u<kDppXor2>(v));
    v = max(v, dpp_u<0x141>(v));
    v = max(v, dpp_u<0x140>(v));
    v = max(v, dpp_u<0x142, 0xa>(v));
    v = max(v, dpp_u<0x143, 0xc>(v));
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

// Block-level deterministic reduction of the six observable partials and the
// displacement maximum; one row of partials per block.
// Without OBS only the displacement maximum is reduced.
template <bool OBS = true, int BS = kBlock>
__device__ inline void block_finish(const StepArgs &a, Ctl *ctl, int blk, double u, double w, double k,
                                    double px, double py, double pz, uint32_t dmax) {
    constexpr int WPB = BS / kWave;
    __shared__ double red[WPB][6];
    __shared__ uint32_t redm[WPB];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    double v6[6] = {u, w, k, px, py, pz};
    if constexpr (OBS) {
#pragma unroll
        for (int q = 0; q < 6; ++q) v6[q] = wave_sum_last(v6[q]);
    }
    dmax = wave_max_last(dmax);
    if (lane == kWave - 1) {
        if constexpr (OBS) {
#pragma unroll
            for (int q = 0; q < 6; ++q) red[wv][q] = v6[q];
        }
        redm[wv] = dmax;
    }
    __syncthreads();
    if (OBS && threadIdx.x < kNP) {
        double s = 0.0;
        if (threadIdx.x < 6)
            for (int q = 0; q < WPB; ++q) s += red[q][threadIdx.x];
        a.st.partials[((size_t)a.slot * a.g.max_blocks + blk) * kNP + threadIdx.x] = s;
    }
    if (threadIdx.x == 0 && (a.mode & kIntegrate)) {
        uint32_t m = 0;
        for (int q = 0; q < WPB; ++q) m = redm[q] > m ? redm[q] : m;
        // Only "exceeded or not" decides the rebuild, so blocks below the
        // threshold skip the same-address atomic entirely.
        if (m > __float_as_uint(a.dyn.thr2)) atomicMax(&ctl->maxd[(a.step + 1) & 1], m);
        if (m > 0x7f800000u) atomicOr(&ctl->flags, kErrNaN);
    }
}

// The tail of a step for slot i of the single-precision paths, after its
// forces (fx, fy, fz) and pair-energy and virial sums (e, w: both halves of
// its pairs) are known: "finalize" of step s (v_s = v' + dt/(2m) F), the
// thermostat (TH), the particle's observable terms (OBS: K_i, m v_i, e/2,
// w/2) and "integrate" of step s+1 (v' = v_s + dt/(2m) F, x_{s+1} =
// x_s + dt v', wrapped into the box with image bookkeeping, the new
// fixed-point record, the squared displacement from the list reference in
// dm against the list reference xr). ds_in is the slot's state as read by
// the caller. Double-single arithmetic, or with PLAIN single floats (the lo
// parts stay zero).
template <bool OBS, bool TH, bool PLAIN = false>
__device__ inline void finish_ds(const StepArgs &a, const BoxC &box, int64_t i, int si, const int4 &xr,
                                 const DsState &ds_in, float fx, float fy, float fz, double e, double w, double &pu,
                                 double &pw, double &pk, double &ppx, double &ppy, double &ppz, uint32_t &dm) {
    const State &st = a.st;
    const float chi = by_s(si, a.dyn.hdt_m_hi), clo = by_s(si, a.dyn.hdt_m_lo);
    const float mass = by_s(si, a.dyn.massf);
    DsState ds = ds_in;
    dsf vx = ds.vx, vy = ds.vy, vz = ds.vz;
    // v += dt/(2m) F: double-single, or one float product and one float sum.
    auto kick = [&](dsf &v, float f) {
        if constexpr (PLAIN)
            v = dsf{v.hi + chi * f, 0.0f};
        else
            v = ds_add(v, ds_mul_f(chi, clo, f));
    };
    if (a.mode & kFinalize) {
        kick(vx, fx);
        kick(vy, fy);
        kick(vz, fz);
        if constexpr (TH) {
            double z[3];
            if (thermo_draw(a.dyn, (uint32_t)st.id[i], a.step, z)) {
                const double sd = by_s(si, a.dyn.thermo_sd);
                if (a.g.dim == 2) z[2] = 0.0;  // motion in the x-y plane
                if constexpr (PLAIN) {
                    vx = dsf{(float)(sd * z[0]), 0.0f};
                    vy = dsf{(float)(sd * z[1]), 0.0f};
                    vz = dsf{(float)(sd * z[2]), 0.0f};
                } else {
                    vx = ds_of(sd * z[0]);
                    vy = ds_of(sd * z[1]);
                    vz = ds_of(sd * z[2]);
                }
            }
        }
    }
    const float ux = vx.hi + vx.lo, uy = vy.hi + vy.lo, uz = vz.hi + vz.lo;
    if constexpr (OBS) {
        pk = 0.5 * (double)(mass * fmaf(uz, uz, fmaf(uy, uy, ux * ux)));
        ppx = (double)(mass * ux);
        ppy = (double)(mass * uy);
        ppz = (double)(mass * uz);
        pu = 0.5 * e;
        pw = 0.5 * w;
    }
    if (a.mode & kIntegrate) {
        kick(vx, fx);
        kick(vy, fy);
        kick(vz, fz);
        dsf x = ds.x, y = ds.y, z = ds.z;
        int ix = 0, iy = 0, iz = 0;
        if constexpr (PLAIN) {
            // x += dt v in floats; wrap by one box edge (as a float).
            const float dtf = a.dyn.dt_hi;
            auto drift = [&](dsf &q, float v, float L, int &im) {
                float t = q.hi + dtf * v;
                if (t < 0.0f) {
                    t += L;
                    im -= 1;
                } else if (t >= L) {
                    t -= L;
                    im += 1;
                }
                if (t >= L) t -= L;
                q = dsf{t, 0.0f};
            };
            drift(x, vx.hi, box.Lhi[0], ix);
            drift(y, vy.hi, box.Lhi[1], iy);
            drift(z, vz.hi, box.Lhi[2], iz);
        } else {
            x = ds_add(x, ds_mul(vx, a.dyn.dt_hi, a.dyn.dt_lo));
            y = ds_add(y, ds_mul(vy, a.dyn.dt_hi, a.dyn.dt_lo));
            z = ds_add(z, ds_mul(vz, a.dyn.dt_hi, a.dyn.dt_lo));
            wrap_ds(x, box.Lhi[0], box.Llo[0], ix);
            wrap_ds(y, box.Lhi[1], box.Llo[1], iy);
            wrap_ds(z, box.Lhi[2], box.Llo[2], iz);
        }
        if (ix | iy | iz) {
            int4 im = st.img[i];
            st.img[i] = make_int4(im.x + ix, im.y + iy, im.z + iz, 0);
        }
        const uint32_t qx = q_from_ds(x.hi, x.lo, box.S_hi[0], box.S_lo[0]);
        const uint32_t qy = q_from_ds(y.hi, y.lo, box.S_hi[1], box.S_lo[1]);
        const uint32_t qz = q_from_ds(z.hi, z.lo, box.S_hi[2], box.S_lo[2]);
        st.recq[a.cur ^ 1][i] = make_int4((int)qx, (int)qy, (int)qz, si);
        ds.x = x;
        ds.y = y;
        ds.z = z;
        const float ddx = disp_q(qx, (uint32_t)xr.x, box.qs_hi[0], box.qs_lo[0]);
        const float ddy = disp_q(qy, (uint32_t)xr.y, box.qs_hi[1], box.qs_lo[1]);
        const float ddz = disp_q(qz, (uint32_t)xr.z, box.qs_hi[2], box.qs_lo[2]);
        const float d2 = fmaf(ddz, ddz, fmaf(ddy, ddy, ddx * ddx));
        // A non-finite position has no fixed-point image: report it as NaN.
        const bool fin = __builtin_isfinite(x.hi) && __builtin_isfinite(y.hi) && __builtin_isfinite(z.hi);
        dm = (fin && d2 == d2) ? __float_as_uint(d2) : 0x7fc00000u;
    }
    ds.vx = vx;
    ds.vy = vy;
    ds.vz = vz;
    ds_store(st.dsw, i, ds);
    if (a.mode & kStoreForce) st.frc32[i] = make_float4(fx, fy, fz, 0.f);
}

// The same tail for the FP64 path (record ri: position and species of slot i).
template <bool TH>
__device__ inline void finish_fp64(const StepArgs &a, const BoxC &box, int64_t i, const double4 &ri, double fx,
                                   double fy, double fz, double e, double w, double &pu, double &pw, double &pk,
                                   double &ppx, double &ppy, double &ppz, uint32_t &dm) {
    const State &st = a.st;
    const int si = (int)ri.w;
    const double c = by_s(si, a.dyn.hdt_m);
    const double mass = by_s(si, a.dyn.mass);
    double4 v = st.vel64[i];
    if (a.mode & kFinalize) {
        v.x += c * fx;
        v.y += c * fy;
        v.z += c * fz;
        if constexpr (TH) {
            double z[3];
            if (thermo_draw(a.dyn, (uint32_t)st.id[i], a.step, z)) {
                const double sd = by_s(si, a.dyn.thermo_sd);
                v.x = sd * z[0];
                v.y = sd * z[1];
                v.z = a.g.dim == 2 ? 0.0 : sd * z[2];
            }
        }
    }
    pk = 0.5 * mass * fma(v.z, v.z, fma(v.y, v.y, v.x * v.x));
    ppx = mass * v.x;
    ppy = mass * v.y;
    ppz = mass * v.z;
    pu = 0.5 * e;
    pw = 0.5 * w;
    if (a.mode & kIntegrate) {
        v.x += c * fx;
        v.y += c * fy;
        v.z += c * fz;
        double x[3] = {ri.x + a.dyn.dt * v.x, ri.y + a.dyn.dt * v.y, ri.z + a.dyn.dt * v.z};
        int d[3] = {0, 0, 0};
        for (int k = 0; k < 3; ++k) {
            if (x[k] < 0.0) {
                x[k] += box.L[k];
                d[k] = -1;
            } else if (x[k] >= box.L[k]) {
                x[k] -= box.L[k];
                d[k] = 1;
            }
            if (x[k] >= box.L[k]) x[k] -= box.L[k];
        }
        if (d[0] | d[1] | d[2]) {
            int4 im = st.img[i];
            st.img[i] = make_int4(im.x + d[0], im.y + d[1], im.z + d[2], 0);
        }
        st.rec64[a.cur ^ 1][i] = make_double4(x[0], x[1], x[2], ri.w);
        const int4 xr = st.xref[i];
        const float ddx = disp_q(q_from_d(x[0], box.S[0]), (uint32_t)xr.x, box.qs_hi[0], box.qs_lo[0]);
        const float ddy = disp_q(q_from_d(x[1], box.S[1]), (uint32_t)xr.y, box.qs_hi[1], box.qs_lo[1]);
        const float ddz = disp_q(q_from_d(x[2], box.S[2]), (uint32_t)xr.z, box.qs_hi[2], box.qs_lo[2]);
        const float d2 = fmaf(ddz, ddz, fmaf(ddy, ddy, ddx * ddx));
        dm = (d2 == d2 && __builtin_isfinite(x[0]) && __builtin_isfinite(x[1]) && __builtin_isfinite(x[2]))
                 ? __float_as_uint(d2)
                 : 0x7fc00000u;
    }
    st.vel64[i] = v;
    if (a.mode & kStoreForce) st.frc64[i] = make_double4(fx, fy, fz, 0.0);
}

}  // namespace ljmd
