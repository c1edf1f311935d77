// k_step.hip -- the per-step hot kernel on gfx950: truncated LJ pair forces
// gathered over the Verlet list, fused with both velocity-Verlet half steps
// and the reductions that follow them (paper Sec. 3 "Code structure" and
// Fig. 1: force, finalize and integrate; Sec. 5: truncated pair forces).
//
// One launch per step s does, for every particle i:
//   F_i(x_s)      = sum_j fs(r_ij) r_ij over list partners with r_ij < r_c
//   finalize      v_s   = v' + dt/(2m) F_i              (completes step s)
//   observables   e_i, w_i (half of every pair), K_i, m v_i -> FP64 block partials
//   integrate     v'    = v_s + dt/(2m) F_i ; x_{s+1} = x_s + dt v'  (starts step s+1)
//   displacement  |x_{s+1} - x_ref|^2 -> max -> rebuild decision of step s+1
// Positions are read from one record buffer and written to the other, so no
// wave ever sees a partner that has already moved.
//
// Gather geometry: LANES lanes per particle, 64/LANES particles per
// wavefront; in the interleaved list layout a lane's entries come in groups
// of four, so every list load of a wave is one 1 KiB contiguous read. Each
// XCD gets a contiguous eighth of the particles.
#include "batch.h"
#include "step_common.h"

namespace ljmd {

// Housekeeping shared by both precisions: the rebuilt marker of this step and,
// after a rebuild, clearing the cell counters for the next binning.
// Cells [c_lo, c_hi) belong to this system; block bj of its nbj blocks
// clears every nbj-th stretch of them. rebuilt (may be NULL) receives the marker.
__device__ inline void step_housekeeping(const StepArgs &a, const Ctl *ctl, int64_t c_lo, int64_t c_hi,
                                         int bj, int nbj, int32_t *rebuilt) {
    const bool rb = rebuild_due(ctl, a.step, a.forced, a.dyn.thr2);
    if (rebuilt && bj == 0 && threadIdx.x == 0) *rebuilt = rb ? 1 : 0;
    if (rb) {
        const int64_t nthr = (int64_t)nbj * blockDim.x;
        for (int64_t c = c_lo + (int64_t)bj * blockDim.x + threadIdx.x; c < c_hi; c += nthr)
            a.st.cell_count[c] = 0;
    }
}

// ---------------------------------------------------------------- FP32 ---
// Q: a cubic box. Then the pair loop works in quanta: the raw wrapped
// fixed-point differences are the displacements, r_c^2 and sigma^2 are
// pre-divided by the squared quantum (exactly, in FP64, before one
// rounding), and the quantum goes into the force factor 24 eps / quantum
// (once per particle with one species, per pair with two). The energy and
// virial terms are summed per lane in FP32 over the lane's few dozen pairs
// before the FP64 reductions. The lists are padded and every slot holds a valid index,
// so the entries the unrolled loop reads past a list are loaded unclamped
// and skipped.
//
// OBS: accumulate the pair energy and virial terms and reduce the
// observable partials; steps whose observables nobody reads skip them.
// Records are addressed by 32-bit byte offsets (fewer than 2^28 slots).
//
// The body serves one block of one system: box holds its constants, ctl its
// control words, particles below i_end are real (the rest of the block is
// padding), and the block is number bj of the nbj blocks that share the
// clearing of its cells [c_lo, c_hi).
// TH: the thermostat resamples colliding particles' velocities after
// "finalize" (a separate instantiation, so that the plain NVE kernel keeps
// its register budget).
template <int NS, int LANES, bool Q, bool OBS, bool TH = false, bool PLAIN = false>
__device__ inline void step_ds_body(const StepArgs &a, const BoxC &box, Ctl *ctl, int blk, int64_t i_end,
                                    int64_t c_lo, int64_t c_hi, int bj, int nbj, int32_t *rebuilt) {
    constexpr int P = kWave / LANES;
    constexpr int WPB = kBlock / kWave;
    const State &st = a.st;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t chunk = (int64_t)blk * WPB + wv;
    const int l = lane % LANES;
    const int64_t i = chunk * P + lane / LANES;
    const bool valid = i < i_end;
    if (halted_record(ctl, a.step, bj == 0)) return;
    step_housekeeping(a, ctl, c_lo, c_hi, bj, nbj, rebuilt);

    // Own record (position and species). The double-single state and the
    // list reference are read once, by the step tail after the pair loop:
    // reading the state here as well and again there costs a second fetch,
    // because the list stream of the loop evicts it from L2. (Staging the
    // tail's operands in LDS with asynchronous loads issued here measured
    // 0.7 us slower per launch at N = 256,000.)
    const int4 *__restrict__ rec = st.recq[a.cur];
    const int4 ri = valid ? rec[i] : make_int4(0, 0, 0, 0);
    int cnt = valid ? st.nbr_cnt[i] : 0;
    cnt = cnt < a.g.cap ? cnt : a.g.cap;
    const int32_t *__restrict__ nb = st.nbr + chunk * (int64_t)(P * a.g.cap) + 4 * lane;
    const int iters = cnt > l ? (cnt - l + LANES - 1) / LANES : 0;
    const float qsx = box.qs_hi[0], qsy = box.qs_hi[1], qsz = box.qs_hi[2];
    const float qlx = box.qs_lo[0], qly = box.qs_lo[1], qlz = box.qs_lo[2];
    // Pair arithmetic: d = (q_i - q_j) * quantum (wrapping difference, i.e.
    // the minimum image), u = sigma^2 / r^2, s6 = u^3. With one species the
    // per-pair constants are factored out: the lanes accumulate
    //   f' = sum s6 (2 s6 - 1) / r^2 * d,  a12 = sum s6^2,  a6 = sum s6,  an = #pairs,
    // and F = 24 eps f', sum phi_s = 4 eps (a12 - a6) - an phi(r_c),
    // sum fs r^2 = 24 eps (2 a12 - a6). With two species every pair carries
    // its own constants. Forces are accumulated in FP32; outside the quanta
    // loop the energy and virial terms are summed in FP64.
    float fx = 0.f, fy = 0.f, fz = 0.f;
    double e = 0.0, w = 0.0, a12 = 0.0, a6 = 0.0;
    int an = 0;
    const float rc2_1 = a.pc.rc2f[0], sig2_1 = a.pc.sig2f[0];
    const PairRow<float> t_rc2(a.pc.rc2f, ri.w), t_sig2(a.pc.sig2f, ri.w), t_eps24(a.pc.eps24f, ri.w),
        t_eps4(a.pc.eps4f, ri.w), t_shift(a.pc.shiftf, ri.w);
    const float c2x = box.r2c[0], c2y = box.r2c[1], c2z = box.r2c[2];
    // Outside the quanta loop: four list entries per trip (one group load),
    // all record gathers in flight before the arithmetic of the first one.
    constexpr int U = 4;
    if constexpr (Q) {
        const float rc2q = box.rc2q[0], sig2q = box.sig2q[0];
        const PairRow<float> q_rc2(box.rc2q, ri.w), q_sig2(box.sig2q, ri.w), q_f(box.fq, ri.w);
        const char *__restrict__ recb = reinterpret_cast<const char *>(rec);
        // Per lane over a few dozen pairs, in FP32: one species, sum s6^2 and
        // sum s6; two species, the pair energies and virials themselves.
        float sa = 0.f, sb = 0.f;
        // Eight entries per trip (two 16-byte group loads per lane) keep more
        // of the list stream in flight; groups past a list end read padding
        // or other lists (valid indices) and are skipped. (Masking the loads
        // of entries past a lane's list end instead, per entry, serialised
        // them: 38.5 us against 30.3 us per launch at N = 256,000.)
        constexpr int UQ = 8;
        static_assert((size_t)4 * kWave <= kListPad, "list padding below the unroll depth");
        for (int m = 0; m < iters; m += UQ) {
            const int4 g0 = *reinterpret_cast<const int4 *>(nb + ((int64_t)(m >> 2) << 8));
            const int4 g1 = *reinterpret_cast<const int4 *>(nb + ((int64_t)((m >> 2) + 1) << 8));
            const int jj[UQ] = {g0.x, g0.y, g0.z, g0.w, g1.x, g1.y, g1.z, g1.w};
            int4 rr[UQ];
#pragma unroll
            for (int u = 0; u < UQ; ++u) rr[u] = *reinterpret_cast<const int4 *>(recb + ((uint32_t)jj[u] << 4));
#pragma unroll
            for (int u = 0; u < UQ; ++u) {
                const float dx = (float)(int32_t)((uint32_t)ri.x - (uint32_t)rr[u].x);
                const float dy = (float)(int32_t)((uint32_t)ri.y - (uint32_t)rr[u].y);
                const float dz = (float)(int32_t)((uint32_t)ri.z - (uint32_t)rr[u].z);
                const float r2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
                const int sj = rr[u].w;
                if (m + u < iters && r2 < (NS == 1 ? rc2q : q_rc2(sj))) {
                    const float ir2 = __builtin_amdgcn_rcpf(r2);
                    const float s2 = (NS == 1 ? sig2q : q_sig2(sj)) * ir2;
                    const float s6 = s2 * s2 * s2;
                    float t = (s6 * ir2) * fmaf(2.0f, s6, -1.0f);
                    if constexpr (NS == 2) t *= q_f(sj);
                    fx = fmaf(t, dx, fx);
                    fy = fmaf(t, dy, fy);
                    fz = fmaf(t, dz, fz);
                    if constexpr (OBS) {
                        if constexpr (NS == 1) {
                            sa = fmaf(s6, s6, sa);
                            sb += s6;
                            an += 1;
                        } else {
                            const float s12 = s6 * s6;
                            sa += fmaf(t_eps4(sj), s12 - s6, -t_shift(sj));
                            sb += t_eps24(sj) * fmaf(2.0f, s12, -s6);
                        }
                    }
                }
            }
        }
        if constexpr (NS == 1) {
            a12 = (double)sa;
            a6 = (double)sb;
        } else {
            e = (double)sa;
            w = (double)sb;
        }
    } else {
    for (int m = 0; m < iters; m += U) {
        // One 16-byte group load per lane: its four entries m .. m+3 (entries
        // past the list end are valid indices and are skipped).
        static_assert(U == 4, "one entry group per trip");
        const int4 grp = *reinterpret_cast<const int4 *>(nb + ((int64_t)(m >> 2) << 8));
        const int jj[U] = {grp.x, grp.y, grp.z, grp.w};
        int4 rr[U];
#pragma unroll
        for (int u = 0; u < U; ++u) rr[u] = rec[jj[u]];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (m + u >= iters) continue;
            const int4 rj = rr[u];
            const float dx = (float)(int32_t)((uint32_t)ri.x - (uint32_t)rj.x) * qsx;
            const float dy = (float)(int32_t)((uint32_t)ri.y - (uint32_t)rj.y) * qsy;
            const float dz = (float)(int32_t)((uint32_t)ri.z - (uint32_t)rj.z) * qsz;
            // d carries the single-float quantum's relative rounding (a few
            // 1e-8, the same for every pair); r^2 takes it out exactly per axis.
            const float r2 = fmaf(dz * c2z, dz, fmaf(dy * c2y, dy, (dx * c2x) * dx));
            if constexpr (NS == 1) {
                if (r2 < rc2_1) {
                    const float ir2 = __builtin_amdgcn_rcpf(r2);
                    const float s2 = sig2_1 * ir2;
                    const float s6 = s2 * s2 * s2;
                    const float t = (s6 * ir2) * fmaf(2.0f, s6, -1.0f);
                    fx = fmaf(t, dx, fx);
                    fy = fmaf(t, dy, fy);
                    fz = fmaf(t, dz, fz);
                    a12 += (double)(s6 * s6);
                    a6 += (double)s6;
                    an += 1;
                }
            } else {
                const int sj = rj.w;
                if (r2 < t_rc2(sj)) {
                    const float ir2 = __builtin_amdgcn_rcpf(r2);
                    const float s2 = t_sig2(sj) * ir2;
                    const float s6 = s2 * s2 * s2;
                    const float s12 = s6 * s6;
                    const float c24 = t_eps24(sj);
                    const float fs = c24 * ((s6 * ir2) * fmaf(2.0f, s6, -1.0f));
                    fx = fmaf(fs, dx, fx);
                    fy = fmaf(fs, dy, fy);
                    fz = fmaf(fs, dz, fz);
                    e += (double)fmaf(t_eps4(sj), s12 - s6, -t_shift(sj));
                    w += (double)(c24 * fmaf(2.0f, s12, -s6));
                }
            }
        }
    }
    }
    if constexpr (LANES > 1) {
        // The particle's lanes exchange their sums: within a quad by DPP
        // moves (no LDS round trip), wider by shuffles.
        auto xsum = [](auto &v, int o) {
            using V = std::remove_reference_t<decltype(v)>;
            if (o == 1 || o == 2) {
                if constexpr (std::is_same_v<V, double>) v += o == 1 ? dpp_d<kDppXor1>(v) : dpp_d<kDppXor2>(v);
                else if constexpr (std::is_same_v<V, float>) v += o == 1 ? dpp_f<kDppXor1>(v) : dpp_f<kDppXor2>(v);
                else v += (V)(o == 1 ? dpp_u<kDppXor1>((uint32_t)v) : dpp_u<kDppXor2>((uint32_t)v));
            } else {
                v += __shfl_xor(v, o);
            }
        };
#pragma unroll
        for (int o = LANES / 2; o > 0; o >>= 1) {
            xsum(fx, o);
            xsum(fy, o);
            xsum(fz, o);
            if constexpr (NS == 1) {
                if constexpr (OBS) {
                    xsum(a12, o);
                    xsum(a6, o);
                    xsum(an, o);
                }
            } else {
                xsum(e, o);
                xsum(w, o);
            }
        }
    }
    if constexpr (NS == 1) {
        const float c24 = Q ? box.fq[0] : a.pc.eps24f[0];
        fx *= c24;
        fy *= c24;
        fz *= c24;
        e = a.pc.eps4[0] * (a12 - a6) - (double)an * a.pc.shift[0];
        w = a.pc.eps24[0] * (2.0 * a12 - a6);
    }
    double pu = 0.0, pw = 0.0, pk = 0.0, ppx = 0.0, ppy = 0.0, ppz = 0.0;
    uint32_t dm = 0u;
    if (valid && l == 0)
        finish_ds<OBS, TH, PLAIN>(a, box, i, ri.w, st.xref[i], ds_load(st.dsw, i), fx, fy, fz, e, w, pu, pw, pk, ppx,
                                  ppy, ppz, dm);
    block_finish<OBS>(a, ctl, blk, pu, pw, pk, ppx, ppy, ppz, dm);
}

// PLAIN: the single-precision state (positions and velocities as single
// floats) instead of double-single.
template <int NS, int LANES, bool Q, bool OBS, bool TH, bool PLAIN>
__global__ __launch_bounds__(kBlock) void k_step_ds(StepArgs a) {
    static_assert(OBS || Q, "observables are skipped on the quanta path only");
    step_ds_body<NS, LANES, Q, OBS, TH, PLAIN>(a, a.box, a.st.ctl, xcd_remap(blockIdx.x, gridDim.x), a.g.n, 0,
                                               a.box.ncell, blockIdx.x, gridDim.x, a.st.rebuilt + a.slot);
}
// Two species, NVE: held to 64 VGPRs, eight waves per SIMD (unbounded it
// takes 65-66 and drops to seven; the 4M mixture's step kernel measured
// 727 -> 683 us). The thermostat's form would spill under that bound.
template <int LANES, bool Q, bool OBS, bool PLAIN>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(8))) void k_step_ds_mix(StepArgs a) {
    static_assert(OBS || Q, "observables are skipped on the quanta path only");
    step_ds_body<2, LANES, Q, OBS, false, PLAIN>(a, a.box, a.st.ctl, xcd_remap(blockIdx.x, gridDim.x), a.g.n, 0,
                                                 a.box.ncell, blockIdx.x, gridDim.x, a.st.rebuilt + a.slot);
}
template <int NS, int LANES, bool Q, bool OBS, bool TH, bool PLAIN>
constexpr void (*step_ds_kernel())(StepArgs) {
    if constexpr (NS == 2 && !TH)
        return k_step_ds_mix<LANES, Q, OBS, PLAIN>;
    else
        return k_step_ds<NS, LANES, Q, OBS, TH, PLAIN>;
}

// A batch of independent one-species cubic systems, each over its own run of
// blocks (particle ranges padded to whole blocks): the block finds its
// system, then runs the same body with that system's box and control words.
template <int LANES, bool OBS>
__global__ __launch_bounds__(kBlock) void k_batch_step(StepArgs a, const SysC *sys, const int32_t *sys_of_g16) {
    const int blk = xcd_remap(blockIdx.x, gridDim.x);
    const int64_t first = (int64_t)blk * (kBlock / LANES);
    const SysC &y = sys[sys_of_g16[first >> 4]];
    step_ds_body<1, LANES, true, OBS>(a, y.box, a.st.ctl + y.id, blk, y.p_off + y.n, y.c_off, y.c_off + y.box.ncell,
                                 blk - y.b_off, y.nb, nullptr);
}

// ---------------------------------------------------------------- FP64 ---
template <int NS, int LANES, bool TH>
__global__ __launch_bounds__(kBlockF64) void k_step_fp64(StepArgs a) {
    constexpr int P = kWave / LANES;
    constexpr int WPB = kBlockF64 / kWave;
    const State &st = a.st;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int blk = xcd_remap(blockIdx.x, gridDim.x);
    const int64_t chunk = (int64_t)blk * WPB + wv;
    const int l = lane % LANES;
    const int64_t i = chunk * P + lane / LANES;
    const bool valid = i < a.g.n;
    if (halted_record(a.st.ctl, a.step, blockIdx.x == 0)) return;
    step_housekeeping(a, a.st.ctl, 0, a.box.ncell, blockIdx.x, gridDim.x, a.st.rebuilt + a.slot);

    const double4 *__restrict__ rec = st.rec64[a.cur];
    double4 ri = valid ? rec[i] : make_double4(0, 0, 0, 0);
    const int si = (int)ri.w;
    int cnt = valid ? st.nbr_cnt[i] : 0;
    cnt = cnt < a.g.cap ? cnt : a.g.cap;
    const int32_t *__restrict__ nb = st.nbr + chunk * (int64_t)(P * a.g.cap) + 4 * lane;
    const int iters = cnt > l ? (cnt - l + LANES - 1) / LANES : 0;
    double fx = 0, fy = 0, fz = 0, e = 0, w = 0;
    const PairRow<double> t_rc2(a.pc.rc2, si), t_sig2(a.pc.sig2, si), t_eps24(a.pc.eps24, si),
        t_eps4(a.pc.eps4, si), t_shift(a.pc.shift, si);
    constexpr int U = 4;
    for (int m = 0; m < iters; m += U) {
        // One 16-byte group load per lane: its four entries m .. m+3 (entries
        // past the list end are valid indices and are skipped).
        static_assert(U == 4, "one entry group per trip");
        const int4 grp = *reinterpret_cast<const int4 *>(nb + ((int64_t)(m >> 2) << 8));
        const int jj[U] = {grp.x, grp.y, grp.z, grp.w};
        double4 rr[U];
#pragma unroll
        for (int u = 0; u < U; ++u) rr[u] = rec[jj[u]];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (m + u >= iters) continue;
            const double4 rj = rr[u];
            const double dx = disp_d(ri.x, rj.x, a.box.L[0], a.box.invL[0]);
            const double dy = disp_d(ri.y, rj.y, a.box.L[1], a.box.invL[1]);
            const double dz = disp_d(ri.z, rj.z, a.box.L[2], a.box.invL[2]);
            const double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
            const int sj = (int)rj.w;
            if (r2 < (NS == 1 ? a.pc.rc2[0] : t_rc2(sj))) {
                // Reciprocal: hardware estimate refined by two Newton steps.
                double ir2 = __builtin_amdgcn_rcp(r2);
                ir2 = fma(ir2, fma(-r2, ir2, 1.0), ir2);
                ir2 = fma(ir2, fma(-r2, ir2, 1.0), ir2);
                const double s2 = (NS == 1 ? a.pc.sig2[0] : t_sig2(sj)) * ir2;
                const double s6 = s2 * s2 * s2;
                const double fs = (NS == 1 ? a.pc.eps24[0] : t_eps24(sj)) * s6 * fma(2.0, s6, -1.0) * ir2;
                fx = fma(fs, dx, fx);
                fy = fma(fs, dy, fy);
                fz = fma(fs, dz, fz);
                e += fma((NS == 1 ? a.pc.eps4[0] : t_eps4(sj)) * s6, s6 - 1.0,
                         -(NS == 1 ? a.pc.shift[0] : t_shift(sj)));
                w = fma(fs, r2, w);
            }
        }
    }
    if constexpr (LANES > 1) {
#pragma unroll
        for (int o = LANES / 2; o > 0; o >>= 1) {
            fx += __shfl_xor(fx, o);
            fy += __shfl_xor(fy, o);
            fz += __shfl_xor(fz, o);
            e += __shfl_xor(e, o);
            w += __shfl_xor(w, o);
        }
    }
    double pu = 0.0, pw = 0.0, pk = 0.0, ppx = 0.0, ppy = 0.0, ppz = 0.0;
    uint32_t dm = 0u;
    if (valid && l == 0)
        finish_fp64<TH>(a, a.box, i, ri, fx, fy, fz, e, w, pu, pw, pk, ppx, ppy, ppz, dm);
    block_finish<true, kBlockF64>(a, a.st.ctl, blk, pu, pw, pk, ppx, ppy, ppz, dm);
}

// Start of a run: "integrate" from the stored forces of the current step
// (the tail of a step with only its integrate half: a.mode is kIntegrate).
template <int PREC>
__device__ inline void integrate_body(const StepArgs &a, const BoxC &box, Ctl *ctl, int64_t i_end) {
    const State &st = a.st;
    if (halted(ctl)) return;
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    uint32_t dm = 0u;
    double pu, pw, pk, ppx, ppy, ppz;
    if (i < i_end) {
        if constexpr (PREC == LJMD_FP64) {
            const double4 f = st.frc64[i];
            finish_fp64<false>(a, box, i, st.rec64[a.cur][i], f.x, f.y, f.z, 0.0, 0.0, pu, pw, pk, ppx, ppy, ppz, dm);
        } else {
            const float4 f = st.frc32[i];
            finish_ds<false, false, PREC == LJMD_FP32>(a, box, i, st.recq[a.cur][i].w, st.xref[i],
                                                       ds_load(st.dsw, i), f.x, f.y, f.z, 0.0,
                                                       0.0, pu,
                                                       pw, pk, ppx, ppy, ppz, dm);
        }
    }
    dm = wave_max_u(dm);
    if ((threadIdx.x & 63) == 0 && dm > __float_as_uint(a.dyn.thr2)) {
        atomicMax(&ctl->maxd[(a.step + 1) & 1], dm);
        if (dm > 0x7f800000u) atomicOr(&ctl->flags, kErrNaN);
    }
}

template <int PREC>
__global__ __launch_bounds__(kBlock) void k_integrate(StepArgs a) {
    integrate_body<PREC>(a, a.box, a.st.ctl, a.g.n);
}

// Batch form: systems are padded to whole step-kernel blocks (at least 64
// slots), so the 64 slots of a wave lie inside one system.
__global__ __launch_bounds__(kBlock) void k_batch_integrate(StepArgs a, const SysC *sys, const int32_t *sys_of_g16,
                                                            int64_t nslots) {
    const int64_t w0 = (int64_t)blockIdx.x * kBlock + (threadIdx.x & ~(kWave - 1));
    if (w0 >= nslots) return;
    const SysC &y = sys[sys_of_g16[w0 >> 4]];
    integrate_body<LJMD_FP32_DS>(a, y.box, a.st.ctl + y.id, y.p_off + y.n);
}

// ------------------------------------------------------------------------
int step_blocks(const Geom &g) {
    const int per_block = (step_block_threads(g.prec) / kWave) * (kWave / g.lanes);
    return (int)((g.n + per_block - 1) / per_block);
}

static StepArgs make_args(const Launch &L, int64_t step, int forced, int mode, int slot) {
    StepArgs a;
    a.st = *L.st;
    a.g = *L.g;
    a.box = *L.box;
    a.pc = *L.pc;
    a.dyn = *L.dyn;
    a.cur = L.cur;
    a.forced = forced;
    a.mode = mode;
    a.slot = slot;
    a.step = step;
    return a;
}

hipError_t launch_step(const Launch &L, int64_t step, int forced, int mode, int slot) {
    if (L.g->all_pairs) return launch_allpairs_step(L, step, mode, slot);
    StepArgs a = make_args(L, step, forced, mode, slot);
    dim3 grid(step_blocks(*L.g)), block(step_block_threads(L.g->prec));
    const bool ds = L.g->prec != LJMD_FP64;
    const bool plain = L.g->prec == LJMD_FP32;
    const bool two = L.g->nspecies == 2;
    const bool quanta = ds && L.box->cubic && L.g->n < kQuantaMaxSlots;
    const bool obs = (mode & kObserve) != 0;
    // The thermostat acts on "finalize" only.
    const bool th = L.dyn->thermo_on && (mode & kFinalize);
#define STEP_DS(NS, LN, TH, PL)                                                                         \
    do {                                                                                                \
        if (quanta && obs)                                                                              \
            launch_k(L, step_ds_kernel<NS, LN, true, true, TH, PL>(), grid, block, a);                   \
        else if (quanta)                                                                                \
            launch_k(L, step_ds_kernel<NS, LN, true, false, TH, PL>(), grid, block, a);                  \
        else                                                                                            \
            launch_k(L, step_ds_kernel<NS, LN, false, true, TH, PL>(), grid, block, a);                  \
    } while (0)
#define STEP_TH(NS, LN, TH)                                                              \
    do {                                                                                 \
        if (ds && plain)                                                                 \
            STEP_DS(NS, LN, TH, true);                                                   \
        else if (ds)                                                                     \
            STEP_DS(NS, LN, TH, false);                                                  \
        else                                                                             \
            launch_k(L, k_step_fp64<NS, LN, TH>, grid, block, a);                     \
    } while (0)
#define STEP(NS, LN)              \
    do {                          \
        if (th)                   \
            STEP_TH(NS, LN, true);  \
        else                      \
            STEP_TH(NS, LN, false); \
    } while (0)
#define BY_LANES(NS)                          \
    switch (L.g->lanes) {                     \
        case 1: STEP(NS, 1); break;           \
        case 2: STEP(NS, 2); break;           \
        case 4: STEP(NS, 4); break;           \
        case 8: STEP(NS, 8); break;           \
        default: STEP(NS, 16); break;         \
    }
    if (two) {
        BY_LANES(2);
    } else {
        BY_LANES(1);
    }
#undef BY_LANES
#undef STEP
#undef STEP_TH
#undef STEP_DS
    return hipGetLastError();
}

hipError_t launch_integrate(const Launch &L, int64_t step) {
    StepArgs a = make_args(L, step, 0, kIntegrate, 0);
    dim3 grid((unsigned)((L.g->n + kBlock - 1) / kBlock)), block(kBlock);
    if (L.g->prec == LJMD_FP64)
        hipLaunchKernelGGL(k_integrate<LJMD_FP64>, grid, block, 0, L.stream, a);
    else if (L.g->prec == LJMD_FP32)
        hipLaunchKernelGGL(k_integrate<LJMD_FP32>, grid, block, 0, L.stream, a);
    else
        hipLaunchKernelGGL(k_integrate<LJMD_FP32_DS>, grid, block, 0, L.stream, a);
    return hipGetLastError();
}


hipError_t launch_batch_step(const Launch &L, const SysC *sys, const int32_t *sys_of_g16, int nblocks,
                             int64_t step, int forced, int mode, int slot) {
    StepArgs a = make_args(L, step, forced, mode, slot);
    const dim3 grid((unsigned)nblocks), block(kBlock);
#define BSTEP(LN)                                                                                        \
    do {                                                                                                 \
        if (mode & kObserve)                                                                             \
            hipLaunchKernelGGL((k_batch_step<LN, true>), grid, block, 0, L.stream, a, sys, sys_of_g16);  \
        else                                                                                             \
            hipLaunchKernelGGL((k_batch_step<LN, false>), grid, block, 0, L.stream, a, sys, sys_of_g16); \
    } while (0)
    switch (L.g->lanes) {
        case 1: BSTEP(1); break;
        case 2: BSTEP(2); break;
        case 4: BSTEP(4); break;
        case 8: BSTEP(8); break;
        default: BSTEP(16); break;
    }
#undef BSTEP
    return hipGetLastError();
}

hipError_t launch_batch_integrate(const Launch &L, const SysC *sys, const int32_t *sys_of_g16, int64_t nslots,
                                  int64_t step) {
    StepArgs a = make_args(L, step, 0, kIntegrate, 0);
    const dim3 grid((unsigned)((nslots + kBlock - 1) / kBlock)), block(kBlock);
    hipLaunchKernelGGL(k_batch_integrate, grid, block, 0, L.stream, a, sys, sys_of_g16, nslots);
    return hipGetLastError();
}

}  // namespace ljmd
