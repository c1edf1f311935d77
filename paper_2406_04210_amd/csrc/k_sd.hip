// k_sd.hip -- steepest descent on gfx950, used to relax random starting
// positions before dynamics (overlapping particles would otherwise give
// unbounded forces). Per iteration:
//   F_i   = sum_j fs(max(r_ij, c sigma_ab)) r_ij over list partners with
//           r_ij < r_c  (pair distance clamped from below, this mode only)
//   F_max = max_i |F_i|
//   x_i  <- x_i + delta F_i / F_max   (no particle moves more than delta)
// with the same list and half-skin rebuild machinery as the dynamics.
#include "step_common.h"

namespace ljmd {

struct SdArgs {
    StepArgs s;
    double clamp2[3];   // (c sigma_t)^2 per pair type
    float clamp2f[3];
    double delta;
    double *fmax_out;   // device, one value per iteration (nullable)
    int iter;
};

// Block maximum of |F| (non-negative doubles order like their bit patterns).
__device__ inline void block_max_u64(unsigned long long v, unsigned long long *dst) {
    __shared__ unsigned long long red[kBlock / kWave];
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long y = __shfl_xor(v, o);
        v = y > v ? y : v;
    }
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int q = 0; q < (int)(blockDim.x >> 6); ++q) v = red[q] > v ? red[q] : v;
        if (v > 0ull) atomicMax(dst, v);
    }
}

template <int PREC, int NS>
__global__ __launch_bounds__(kBlock) void k_sd_force(SdArgs sa) {
    const StepArgs &a = sa.s;
    const State &st = a.st;
    const int lanes = a.g.lanes;
    const int lg = lanes >= 16 ? 4 : (lanes >= 8 ? 3 : (lanes >= 4 ? 2 : (lanes >= 2 ? 1 : 0)));
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t chunk = (int64_t)blockIdx.x * (kBlock / kWave) + wv;
    const int l = lane & (lanes - 1);
    const int64_t i = (chunk << (6 - lg)) + (lane >> lg);
    const bool valid = i < a.g.n;
    if (halted_record(st.ctl, a.step, blockIdx.x == 0)) return;
    // After a rebuild, clear the cell counters for the next binning.
    if (rebuild_due(st.ctl, a.step, a.forced, a.dyn.thr2)) {
        const int64_t nthr = (int64_t)gridDim.x * blockDim.x;
        for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < a.box.ncell; c += nthr)
            st.cell_count[c] = 0;
    }
    int cnt = valid ? st.nbr_cnt[i] : 0;
    cnt = cnt < a.g.cap ? cnt : a.g.cap;
    const int32_t *__restrict__ nb = st.nbr + ((chunk * (int64_t)a.g.cap) << (6 - lg)) + 4 * lane;
    const int iters = cnt > l ? (cnt - l + lanes - 1) >> lg : 0;
    double fxd = 0, fyd = 0, fzd = 0;
    float fxf = 0, fyf = 0, fzf = 0;
    if constexpr (PREC == LJMD_FP64) {
        const double4 *__restrict__ rec = st.rec64[a.cur];
        const double4 ri = valid ? rec[i] : make_double4(0, 0, 0, 0);
        const int si = (int)ri.w;
        for (int m = 0; m < iters; ++m) {
            const int j = nb_entry(nb, m);
            const double4 rj = rec[j];
            const double dx = disp_d(ri.x, rj.x, a.box.L[0], a.box.invL[0]);
            const double dy = disp_d(ri.y, rj.y, a.box.L[1], a.box.invL[1]);
            const double dz = disp_d(ri.z, rj.z, a.box.L[2], a.box.invL[2]);
            const double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
            const int t = NS == 1 ? 0 : si + (int)rj.w;
            if (r2 < by_t<NS>(t, a.pc.rc2)) {
                const double c2 = by_t<NS>(t, sa.clamp2);
                const double re2 = r2 < c2 ? c2 : r2;
                const double ir2 = 1.0 / re2;
                const double s2 = by_t<NS>(t, a.pc.sig2) * ir2;
                const double s6 = s2 * s2 * s2;
                const double fs = by_t<NS>(t, a.pc.eps24) * s6 * fma(2.0, s6, -1.0) * ir2;
                fxd = fma(fs, dx, fxd);
                fyd = fma(fs, dy, fyd);
                fzd = fma(fs, dz, fzd);
            }
        }
        for (int o = lanes >> 1; o > 0; o >>= 1) {
            fxd += __shfl_xor(fxd, o);
            fyd += __shfl_xor(fyd, o);
            fzd += __shfl_xor(fzd, o);
        }
    } else {
        const int4 *__restrict__ rec = st.recq[a.cur];
        const int4 ri = valid ? rec[i] : make_int4(0, 0, 0, 0);
        for (int m = 0; m < iters; ++m) {
            const int j = nb_entry(nb, m);
            const int4 rj = rec[j];
            const float dx = disp_q((uint32_t)ri.x, (uint32_t)rj.x, a.box.qs_hi[0], a.box.qs_lo[0]);
            const float dy = disp_q((uint32_t)ri.y, (uint32_t)rj.y, a.box.qs_hi[1], a.box.qs_lo[1]);
            const float dz = disp_q((uint32_t)ri.z, (uint32_t)rj.z, a.box.qs_hi[2], a.box.qs_lo[2]);
            const float r2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
            const int t = NS == 1 ? 0 : ri.w + rj.w;
            if (r2 < by_t<NS>(t, a.pc.rc2f)) {
                const float c2 = by_t<NS>(t, sa.clamp2f);
                const float re2 = r2 < c2 ? c2 : r2;
                const float ir2 = __builtin_amdgcn_rcpf(re2);
                const float s2 = by_t<NS>(t, a.pc.sig2f) * ir2;
                const float s6 = s2 * s2 * s2;
                const float fs = by_t<NS>(t, a.pc.eps24f) * ((s6 * ir2) * fmaf(2.0f, s6, -1.0f));
                fxf = fmaf(fs, dx, fxf);
                fyf = fmaf(fs, dy, fyf);
                fzf = fmaf(fs, dz, fzf);
            }
        }
        for (int o = lanes >> 1; o > 0; o >>= 1) {
            fxf += __shfl_xor(fxf, o);
            fyf += __shfl_xor(fyf, o);
            fzf += __shfl_xor(fzf, o);
        }
        fxd = fxf;
        fyd = fyf;
        fzd = fzf;
    }
    unsigned long long fm = 0ull;
    if (valid && l == 0) {
        if constexpr (PREC == LJMD_FP64)
            st.frc64[i] = make_double4(fxd, fyd, fzd, 0.0);
        else
            st.frc32[i] = make_float4(fxf, fyf, fzf, 0.f);
        const double a2 = sqrt(fma(fzd, fzd, fma(fyd, fyd, fxd * fxd)));
        fm = a2 == a2 ? (unsigned long long)__double_as_longlong(a2) : 0x7ff8000000000000ull;
    }
    block_max_u64(fm, &st.ctl->fmax[a.step & 1]);
}

// PLAIN (single-precision state): x += delta F / F_max in one float sum.
template <int PREC, bool PLAIN = false>
__global__ __launch_bounds__(kBlock) void k_sd_move(SdArgs sa) {
    const StepArgs &a = sa.s;
    const State &st = a.st;
    if (halted(st.ctl)) return;
    const unsigned long long fbits = st.ctl->fmax[a.step & 1];
    const double fmax = __longlong_as_double((long long)fbits);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st.ctl->fmax[(a.step + 1) & 1] = 0ull;
        if (sa.fmax_out) sa.fmax_out[sa.iter] = fmax;
    }
    const bool go = fmax > 0.0 && fbits < 0x7ff0000000000000ull;
    const double scale = go ? sa.delta / fmax : 0.0;
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    uint32_t dm = 0u;
    if (i < a.g.n && go) {
        uint32_t q[3];
        int d[3] = {0, 0, 0};
        if constexpr (PREC == LJMD_FP64) {
            const double4 f = st.frc64[i];
            const double4 r = st.rec64[a.cur][i];
            double x[3] = {fma(scale, f.x, r.x), fma(scale, f.y, r.y), fma(scale, f.z, r.z)};
            for (int k = 0; k < 3; ++k) {
                if (x[k] < 0.0) {
                    x[k] += a.box.L[k];
                    d[k] = -1;
                } else if (x[k] >= a.box.L[k]) {
                    x[k] -= a.box.L[k];
                    d[k] = 1;
                }
                if (x[k] >= a.box.L[k]) x[k] -= a.box.L[k];
                q[k] = q_from_d(x[k], a.box.S[k]);
            }
            st.rec64[a.cur][i] = make_double4(x[0], x[1], x[2], r.w);
        } else {
            const float4 f = st.frc32[i];
            const float sc = (float)scale;
            DsState ds = ds_load(st.dsw, i);
            dsf x = ds.x, y = ds.y, z = ds.z;
            if constexpr (PLAIN) {
                dsf *c3[3] = {&x, &y, &z};
                const float fc[3] = {f.x, f.y, f.z};
                for (int k = 0; k < 3; ++k) {
                    float t = c3[k]->hi + sc * fc[k];
                    if (t < 0.0f) {
                        t += a.box.Lhi[k];
                        d[k] = -1;
                    } else if (t >= a.box.Lhi[k]) {
                        t -= a.box.Lhi[k];
                        d[k] = 1;
                    }
                    if (t >= a.box.Lhi[k]) t -= a.box.Lhi[k];
                    *c3[k] = dsf{t, 0.0f};
                }
            } else {
                x = ds_add(x, dsf{sc * f.x, 0.f});
                y = ds_add(y, dsf{sc * f.y, 0.f});
                z = ds_add(z, dsf{sc * f.z, 0.f});
                wrap_ds(x, a.box.Lhi[0], a.box.Llo[0], d[0]);
                wrap_ds(y, a.box.Lhi[1], a.box.Llo[1], d[1]);
                wrap_ds(z, a.box.Lhi[2], a.box.Llo[2], d[2]);
            }
            q[0] = q_from_ds(x.hi, x.lo, a.box.S_hi[0], a.box.S_lo[0]);
            q[1] = q_from_ds(y.hi, y.lo, a.box.S_hi[1], a.box.S_lo[1]);
            q[2] = q_from_ds(z.hi, z.lo, a.box.S_hi[2], a.box.S_lo[2]);
            const int sp = st.recq[a.cur][i].w;
            st.recq[a.cur][i] = make_int4((int)q[0], (int)q[1], (int)q[2], sp);
            ds.x = x;
            ds.y = y;
            ds.z = z;
            ds_store(st.dsw, i, ds);
        }
        if (d[0] | d[1] | d[2]) {
            const int4 im = st.img[i];
            st.img[i] = make_int4(im.x + d[0], im.y + d[1], im.z + d[2], 0);
        }
        const int4 xr = st.xref[i];
        const float ddx = disp_q(q[0], (uint32_t)xr.x, a.box.qs_hi[0], a.box.qs_lo[0]);
        const float ddy = disp_q(q[1], (uint32_t)xr.y, a.box.qs_hi[1], a.box.qs_lo[1]);
        const float ddz = disp_q(q[2], (uint32_t)xr.z, a.box.qs_hi[2], a.box.qs_lo[2]);
        const float d2 = fmaf(ddz, ddz, fmaf(ddy, ddy, ddx * ddx));
        dm = d2 == d2 ? __float_as_uint(d2) : 0x7fc00000u;
    }
    dm = wave_max_u(dm);
    if ((threadIdx.x & 63) == 0 && dm > __float_as_uint(a.dyn.thr2)) {
        atomicMax(&st.ctl->maxd[(a.step + 1) & 1], dm);
        if (dm > 0x7f800000u) atomicOr(&st.ctl->flags, kErrNaN);
    }
}

hipError_t launch_sd(const Launch &L, int64_t step, int forced, int iter, double delta,
                     double clamp, double *fmax_out) {
    SdArgs sa;
    sa.s.st = *L.st;
    sa.s.g = *L.g;
    sa.s.box = *L.box;
    sa.s.pc = *L.pc;
    sa.s.dyn = *L.dyn;
    sa.s.cur = L.cur;
    sa.s.forced = forced;
    sa.s.mode = 0;
    sa.s.slot = (int)(step % kRing);
    sa.s.step = step;
    for (int t = 0; t < 3; ++t) {
        const double c2 = clamp * clamp * L.pc->sig2[t];
        sa.clamp2[t] = c2;
        sa.clamp2f[t] = (float)c2;
    }
    sa.delta = delta;
    sa.fmax_out = fmax_out;
    sa.iter = iter;
    const int per_block = (kBlock / kWave) * (kWave / L.g->lanes);
    const dim3 gf((unsigned)((L.g->n + per_block - 1) / per_block)), b(kBlock);
    const dim3 gm((unsigned)((L.g->n + kBlock - 1) / kBlock));
    const bool two = L.g->nspecies == 2;
    if (L.g->prec == LJMD_FP64) {
        if (two)
            hipLaunchKernelGGL((k_sd_force<LJMD_FP64, 2>), gf, b, 0, L.stream, sa);
        else
            hipLaunchKernelGGL((k_sd_force<LJMD_FP64, 1>), gf, b, 0, L.stream, sa);
        hipLaunchKernelGGL(k_sd_move<LJMD_FP64>, gm, b, 0, L.stream, sa);
    } else {
        if (two)
            hipLaunchKernelGGL((k_sd_force<LJMD_FP32_DS, 2>), gf, b, 0, L.stream, sa);
        else
            hipLaunchKernelGGL((k_sd_force<LJMD_FP32_DS, 1>), gf, b, 0, L.stream, sa);
        if (L.g->prec == LJMD_FP32)
            hipLaunchKernelGGL((k_sd_move<LJMD_FP32_DS, true>), gm, b, 0, L.stream, sa);
        else
            hipLaunchKernelGGL((k_sd_move<LJMD_FP32_DS, false>), gm, b, 0, L.stream, sa);
    }
    return hipGetLastError();
}

}  // namespace ljmd
