// k_adjoint.hip -- hand-written adjoint of the truncated LJ forces and of
// velocity Verlet on gfx950: the differentiable form of the force pass
// (Sec. 5 pair forces; the gradient itself is not in the paper).
//
// Force vector-Jacobian product at positions x for a cotangent g:
//   gx_i = sum_j [ fs D + c (d.D) d ],  D = g_i - g_j,  d = x_i - x_j (minimum image),
//   fs = 24 eps (2 s12 - s6) / r^2,  c = 2 dfs/d(r^2) = -(96 eps / r^4)(7 s12 - 2 s6),
// which is (dF/dx)^T g (dF/dx is minus the Hessian of U, a symmetric matrix).
// Parameter gradient of g.F for the symmetric pair type t (AA, AB, BB):
//   d/d eps_t   = sum_{i<j} (D.d) fs / eps_t,
//   d/d sigma_t = sum_{i<j} (D.d) (144 eps_t / sigma_t)(4 s12 - s6) / r^2.
// Energy gradient (the cutoff r_c is a fixed length; the shift moves with
// eps and sigma):
//   dU/d eps_t   = sum_{i<j} phi_s / eps_t,
//   dU/d sigma_t = sum_{i<j} (4 eps_t / sigma_t) [(12 s12 - 6 s6) - (12 s12 - 6 s6) at r_c].
// Lists are full, so every unordered pair is met from both ends and each
// visit adds half of the parameter terms. Only pairs inside the cutoff
// contribute: the truncated force is differentiated where it is smooth.
//
// Geometry and pair arithmetic follow the step kernel of the same precision:
// FP64 repeats its displacement, r^2 and cutoff test. FP32 takes the cutoff
// decision exactly as the force pass of the same box does -- in a cubic box
// r^2 in squared quanta from the raw fixed-point differences against r_c^2
// in quanta, otherwise the general form below -- so a pair within rounding
// of r_c is inside for both or for neither, and the gradient is that of the
// forces the step computed. The pair terms use the general form
// (fixed-point difference times the single-float quantum, r^2 corrected per
// axis for the quantum's rounding). The FP32 path accumulates gx in FP32
// like the forces; parameter sums are FP64 everywhere, reduced per block and
// then over blocks in a fixed order.
#include "adjoint.h"
#include "step_common.h"

namespace ljmd {

// Squared displacement of slot i (record buffer cur) from its list
// reference, as the bits of a non-negative float (NaN as a quiet NaN).
template <int PREC>
__device__ inline uint32_t frame_d2_rec(const void *recs, const int4 *xref, const BoxC &box, int64_t i) {
    uint32_t q[3];
    if constexpr (PREC == LJMD_FP64) {
        const double4 r = ((const double4 *)recs)[i];
        q[0] = q_from_d(r.x, box.S[0]);
        q[1] = q_from_d(r.y, box.S[1]);
        q[2] = q_from_d(r.z, box.S[2]);
    } else {
        const int4 r = ((const int4 *)recs)[i];
        q[0] = (uint32_t)r.x;
        q[1] = (uint32_t)r.y;
        q[2] = (uint32_t)r.z;
    }
    const int4 xr = xref[i];
    const float dx = disp_q(q[0], (uint32_t)xr.x, box.qs_hi[0], box.qs_lo[0]);
    const float dy = disp_q(q[1], (uint32_t)xr.y, box.qs_hi[1], box.qs_lo[1]);
    const float dz = disp_q(q[2], (uint32_t)xr.z, box.qs_hi[2], box.qs_lo[2]);
    const float d2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
    return d2 == d2 ? __float_as_uint(d2) : 0x7fc00000u;
}
template <int PREC>
__device__ inline uint32_t frame_d2_bits(const State &st, const BoxC &box, int cur, int64_t i) {
    const void *recs = PREC == LJMD_FP64 ? (const void *)st.rec64[cur] : (const void *)st.recq[cur];
    return frame_d2_rec<PREC>(recs, st.xref, box, i);
}

// Every wave folds the largest of its lanes' values into the rebuild word of
// `step` (only values past the threshold matter).
__device__ inline void fold_disp(Ctl *ctl, int64_t step, float thr2, uint32_t dm) {
    dm = wave_max_u(dm);
    if ((threadIdx.x & 63) == 0 && dm > __float_as_uint(thr2)) {
        atomicMax(&ctl->maxd[step & 1], dm);
        if (dm > 0x7f800000u) atomicOr(&ctl->flags, kErrNaN);
    }
}

struct AdjArgs {
    State st;
    Geom g;
    BoxC box;
    PairC pc;
    int cur;
    const void *gvec;  // per-slot cotangent: double4 (FP64) or float4 (FP32)
    double4 *gx;       // per-slot output, += weight * VJP
    double weight;
    double c12[3], c6[3];  // (sigma/r_c)^12, (sigma/r_c)^6 per pair type
    double inv_eps[3], inv_sig[3];
    int shifted;
    // Block partial rows: row = (init ? 0 : row) + rows_weight * block sums.
    double *rows;
    double rows_weight;
    int rows_init;
    // Cell counters cleared here if the lists were rebuilt for `step`.
    int clear_cells;
    int forced;
    int64_t step;
    float thr2;
    // Reverse sweep (next set): once a slot's gx is final, the drift and
    // cotangent of the next (earlier) frame for that slot -- lv += next_scale
    // * gx (skipped when next_scale == 0), gv_next = lv / m -- and that
    // frame's displacement (records next_rec) folded into the rebuild word of
    // next_step.
    int next;
    double4 *lv;
    void *gv_next;
    double next_scale;
    int64_t next_step;
    const void *next_rec;
    double mass[2];
};

// Six FP64 sums of one block into row `blk` of the partials (stride kNP):
// row = (init ? 0 : row) + weight * sums.
__device__ inline void block_rows6(const double (&v)[6], double *row, double weight, int init) {
    constexpr int WPB = kBlock / kWave;
    __shared__ double red[WPB][6];
    double s[6];
#pragma unroll
    for (int q = 0; q < 6; ++q) s[q] = wave_sum_last(v[q]);
    if ((threadIdx.x & 63) == kWave - 1) {
#pragma unroll
        for (int q = 0; q < 6; ++q) red[threadIdx.x >> 6][q] = s[q];
    }
    __syncthreads();
    if (threadIdx.x < 6) {
        double acc = 0.0;
        for (int w = 0; w < WPB; ++w) acc += red[w][threadIdx.x];
        row[threadIdx.x] = (init ? 0.0 : row[threadIdx.x]) + weight * acc;
    }
}

// Per-lane parameter sums, one named register per type: an indexed array
// would be placed in scratch memory.
struct Theta {
    double e0 = 0, e1 = 0, e2 = 0, s0 = 0, s1 = 0, s2 = 0;
};

template <int NS>
__device__ inline void add_theta(Theta &th, int t, double ge, double gs) {
    if constexpr (NS == 1) {
        th.e0 += ge;
        th.s0 += gs;
    } else {
        th.e0 += t == 0 ? ge : 0.0;
        th.e1 += t == 1 ? ge : 0.0;
        th.e2 += t == 2 ? ge : 0.0;
        th.s0 += t == 0 ? gs : 0.0;
        th.s1 += t == 1 ? gs : 0.0;
        th.s2 += t == 2 ? gs : 0.0;
    }
}

template <int PREC, int NS, int MODE>
__global__ __launch_bounds__(kBlock) void k_adjoint_pairs(AdjArgs a) {
    constexpr int WPB = kBlock / kWave;
    const State &st = a.st;
    const int lanes = a.g.lanes;
    const int lg = lanes >= 16 ? 4 : (lanes >= 8 ? 3 : (lanes >= 4 ? 2 : (lanes >= 2 ? 1 : 0)));
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int blk = xcd_remap(blockIdx.x, gridDim.x);
    const int64_t chunk = (int64_t)blk * WPB + wv;
    const int l = lane & (lanes - 1);
    const int64_t i = (chunk << (6 - lg)) + (lane >> lg);
    const bool valid = i < a.g.n;
    if (a.clear_cells && rebuild_due(st.ctl, a.step, a.forced, a.thr2)) {
        const int64_t nthr = (int64_t)gridDim.x * blockDim.x;
        for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < a.box.ncell; c += nthr)
            st.cell_count[c] = 0;
    }
    int cnt = valid ? st.nbr_cnt[i] : 0;
    cnt = cnt < a.g.cap ? cnt : a.g.cap;
    const int32_t *__restrict__ nb = st.nbr + ((chunk * (int64_t)a.g.cap) << (6 - lg)) + 4 * lane;
    const int iters = cnt > l ? (cnt - l + lanes - 1) >> lg : 0;
    Theta th;
    double ox = 0, oy = 0, oz = 0;
    constexpr int U = 4;
    if constexpr (PREC == LJMD_FP64) {
        const double4 *__restrict__ rec = st.rec64[a.cur];
        const double4 *__restrict__ gv = (const double4 *)a.gvec;
        const double4 ri = valid ? rec[i] : make_double4(0, 0, 0, 0);
        const double4 gi = (MODE == kAdjVjp && valid) ? gv[i] : make_double4(0, 0, 0, 0);
        const int si = (int)ri.w;
        for (int m = 0; m < iters; m += U) {
            // One 16-byte group load per lane: its four entries m .. m+3
            // (entries past the list end are valid indices and are skipped).
            static_assert(U == 4, "one entry group per trip");
            const int4 grp = *reinterpret_cast<const int4 *>(nb + ((int64_t)(m >> 2) << 8));
            const int jj[U] = {grp.x, grp.y, grp.z, grp.w};
            double4 rr[U], gg[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                rr[u] = rec[jj[u]];
                if constexpr (MODE == kAdjVjp) gg[u] = gv[jj[u]];
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (m + u >= iters) continue;
                const double4 rj = rr[u];
                const double dx = disp_d(ri.x, rj.x, a.box.L[0], a.box.invL[0]);
                const double dy = disp_d(ri.y, rj.y, a.box.L[1], a.box.invL[1]);
                const double dz = disp_d(ri.z, rj.z, a.box.L[2], a.box.invL[2]);
                const double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
                const int t = NS == 1 ? 0 : si + (int)rj.w;
                if (!(r2 < by_t<NS>(t, a.pc.rc2))) continue;
                double ir2 = __builtin_amdgcn_rcp(r2);
                ir2 = fma(ir2, fma(-r2, ir2, 1.0), ir2);
                ir2 = fma(ir2, fma(-r2, ir2, 1.0), ir2);
                const double s2 = by_t<NS>(t, a.pc.sig2) * ir2;
                const double s6 = s2 * s2 * s2, s12 = s6 * s6;
                const double eps24 = by_t<NS>(t, a.pc.eps24);
                if constexpr (MODE == kAdjVjp) {
                    const double4 gj = gg[u];
                    const double Dx = gi.x - gj.x, Dy = gi.y - gj.y, Dz = gi.z - gj.z;
                    const double dD = fma(dz, Dz, fma(dy, Dy, dx * Dx));
                    const double fs = eps24 * (2.0 * s12 - s6) * ir2;
                    const double c = -4.0 * eps24 * (7.0 * s12 - 2.0 * s6) * (ir2 * ir2) * dD;
                    ox = fma(fs, Dx, fma(c, dx, ox));
                    oy = fma(fs, Dy, fma(c, dy, oy));
                    oz = fma(fs, Dz, fma(c, dz, oz));
                    const double h = 0.5 * dD;
                    add_theta<NS>(th, t, h * fs * by_t<NS>(t, a.inv_eps),
                                  h * 6.0 * eps24 * by_t<NS>(t, a.inv_sig) * (4.0 * s12 - s6) * ir2);
                } else {
                    const double c12 = by_t<NS>(t, a.c12), c6 = by_t<NS>(t, a.c6);
                    const double ue = 4.0 * (s12 - s6) - (a.shifted ? 4.0 * (c12 - c6) : 0.0);
                    const double us = (12.0 * s12 - 6.0 * s6) - (a.shifted ? 12.0 * c12 - 6.0 * c6 : 0.0);
                    add_theta<NS>(th, t, 0.5 * ue, 0.5 * by_t<NS>(t, a.pc.eps4) * by_t<NS>(t, a.inv_sig) * us);
                }
            }
        }
    } else {
        const int4 *__restrict__ rec = st.recq[a.cur];
        const float4 *__restrict__ gv = (const float4 *)a.gvec;
        const int4 ri = valid ? rec[i] : make_int4(0, 0, 0, 0);
        const float4 gi = (MODE == kAdjVjp && valid) ? gv[i] : make_float4(0, 0, 0, 0);
        const float qsx = a.box.qs_hi[0], qsy = a.box.qs_hi[1], qsz = a.box.qs_hi[2];
        const float c2x = a.box.r2c[0], c2y = a.box.r2c[1], c2z = a.box.r2c[2];
        // The force pass's cutoff test (see above).
        const bool quanta = a.box.cubic && a.g.n < kQuantaMaxSlots;
        float fx = 0.f, fy = 0.f, fz = 0.f;
        for (int m = 0; m < iters; m += U) {
            const int4 grp = *reinterpret_cast<const int4 *>(nb + ((int64_t)(m >> 2) << 8));
            const int jj[U] = {grp.x, grp.y, grp.z, grp.w};
            int4 rr[U];
            float4 gg[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                rr[u] = rec[jj[u]];
                if constexpr (MODE == kAdjVjp) gg[u] = gv[jj[u]];
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (m + u >= iters) continue;
                const int4 rj = rr[u];
                const float ax = (float)(int32_t)((uint32_t)ri.x - (uint32_t)rj.x);
                const float ay = (float)(int32_t)((uint32_t)ri.y - (uint32_t)rj.y);
                const float az = (float)(int32_t)((uint32_t)ri.z - (uint32_t)rj.z);
                const float dx = ax * qsx, dy = ay * qsy, dz = az * qsz;
                const float r2 = fmaf(dz * c2z, dz, fmaf(dy * c2y, dy, (dx * c2x) * dx));
                const int t = NS == 1 ? 0 : ri.w + rj.w;
                const bool inside = quanta ? fmaf(az, az, fmaf(ay, ay, ax * ax)) < by_t<NS>(t, a.box.rc2q)
                                           : r2 < by_t<NS>(t, a.pc.rc2f);
                if (!inside) continue;
                const float ir2 = __builtin_amdgcn_rcpf(r2);
                const float s2 = by_t<NS>(t, a.pc.sig2f) * ir2;
                const float s6 = s2 * s2 * s2;
                const float s12 = s6 * s6;
                const float eps24 = by_t<NS>(t, a.pc.eps24f);
                if constexpr (MODE == kAdjVjp) {
                    const float4 gj = gg[u];
                    const float Dx = gi.x - gj.x, Dy = gi.y - gj.y, Dz = gi.z - gj.z;
                    const float dD = fmaf(dz, Dz, fmaf(dy, Dy, dx * Dx));
                    const float fs = eps24 * ((s6 * ir2) * fmaf(2.0f, s6, -1.0f));
                    const float c = (-4.0f * eps24) * (fmaf(7.0f, s12, -2.0f * s6) * (ir2 * ir2)) * dD;
                    fx = fmaf(fs, Dx, fmaf(c, dx, fx));
                    fy = fmaf(fs, Dy, fmaf(c, dy, fy));
                    fz = fmaf(fs, Dz, fmaf(c, dz, fz));
                    const double h = 0.5 * (double)dD;
                    add_theta<NS>(th, t, h * (double)fs * by_t<NS>(t, a.inv_eps),
                                  h * (double)(eps24 * fmaf(4.0f, s12, -s6) * ir2) * 6.0 *
                                      by_t<NS>(t, a.inv_sig));
                } else {
                    const double c12 = by_t<NS>(t, a.c12), c6 = by_t<NS>(t, a.c6);
                    const double ds12 = (double)s12, ds6 = (double)s6;
                    const double ue = 4.0 * (ds12 - ds6) - (a.shifted ? 4.0 * (c12 - c6) : 0.0);
                    const double us = (12.0 * ds12 - 6.0 * ds6) - (a.shifted ? 12.0 * c12 - 6.0 * c6 : 0.0);
                    add_theta<NS>(th, t, 0.5 * ue, 0.5 * by_t<NS>(t, a.pc.eps4) * by_t<NS>(t, a.inv_sig) * us);
                }
            }
        }
        ox = fx;
        oy = fy;
        oz = fz;
    }
    if constexpr (MODE == kAdjVjp) {
        // Within a quad by DPP moves (FP64, both halves), wider by shuffles.
        for (int o = lanes >> 1; o > 0; o >>= 1) {
            if (o == 1) {
                ox += dpp_d<kDppXor1>(ox);
                oy += dpp_d<kDppXor1>(oy);
                oz += dpp_d<kDppXor1>(oz);
            } else if (o == 2) {
                ox += dpp_d<kDppXor2>(ox);
                oy += dpp_d<kDppXor2>(oy);
                oz += dpp_d<kDppXor2>(oz);
            } else {
                ox += __shfl_xor(ox, o);
                oy += __shfl_xor(oy, o);
                oz += __shfl_xor(oz, o);
            }
        }
        uint32_t dnext = 0u;
        if (valid && l == 0) {
            double4 acc = a.gx[i];
            acc.x = fma(a.weight, ox, acc.x);
            acc.y = fma(a.weight, oy, acc.y);
            acc.z = fma(a.weight, oz, acc.z);
            a.gx[i] = acc;
            if (a.next) {
                // The same operations as kOpDriftCotangent for this slot.
                double4 y = a.lv[i];
                if (a.next_scale != 0.0) {
                    y.x = fma(a.next_scale, acc.x, y.x);
                    y.y = fma(a.next_scale, acc.y, y.y);
                    y.z = fma(a.next_scale, acc.z, y.z);
                    a.lv[i] = y;
                }
                if constexpr (PREC == LJMD_FP64) {
                    const double im = 1.0 / by_s((int)st.rec64[a.cur][i].w, a.mass);
                    ((double4 *)a.gv_next)[i] = make_double4(y.x * im, y.y * im, y.z * im, 0.0);
                } else {
                    const double im = 1.0 / by_s(st.recq[a.cur][i].w, a.mass);
                    ((float4 *)a.gv_next)[i] =
                        make_float4((float)(y.x * im), (float)(y.y * im), (float)(y.z * im), 0.f);
                }
                dnext = frame_d2_rec<PREC>(a.next_rec, st.xref, a.box, i);
            }
        }
        if (a.next) fold_disp(st.ctl, a.next_step, a.thr2, dnext);
    }
    const double v6[6] = {th.e0, th.e1, th.e2, th.s0, th.s1, th.s2};
    block_rows6(v6, a.rows + (size_t)blk * kNP, a.rows_weight, a.rows_init);
}

// Clears the cell counters after a rebuild of `step`: the list passes of the
// reverse sweep are followed by no dynamics step kernel, which does this in a
// forward run.
__global__ __launch_bounds__(kBlock) void k_adjoint_cells(State st, BoxC box, int64_t step, int forced,
                                                          float thr2) {
    if (!rebuild_due(st.ctl, step, forced, thr2)) return;
    const int64_t nthr = (int64_t)gridDim.x * blockDim.x;
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < box.ncell; c += nthr)
        st.cell_count[c] = 0;
}

// gtheta[q] = (init ? 0 : gtheta[q]) + weight * (sum of the block rows), in a
// fixed order (one block).
__global__ __launch_bounds__(kBlock) void k_adjoint_reduce(const double *part, int nrows, double weight,
                                                           double *gtheta, int init) {
    __shared__ double red[kBlock];
    for (int q = 0; q < 6; ++q) {
        double acc = 0.0;
        for (int b = threadIdx.x; b < nrows; b += kBlock) acc += part[(size_t)b * kNP + q];
        red[threadIdx.x] = acc;
        __syncthreads();
        for (int s = kBlock / 2; s > 0; s >>= 1) {
            if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
            __syncthreads();
        }
        if (threadIdx.x == 0) gtheta[q] = (init ? 0.0 : gtheta[q]) + weight * red[0];
        __syncthreads();
    }
}

struct VecArgs {
    State st;
    Geom g;
    DynC dyn;
    int cur;
    int op;
    const double *src_id;
    double *dst_id;
    double4 *a;
    double4 *b;
    void *gvec;
    double scale;
    const double *dscale;  // kOpSubForce: the device scalar c
    // kOpDriftCotangent: also fold the frame's displacement from the list
    // reference into the rebuild word of disp_step (when disp is set).
    BoxC box;
    int64_t disp_step;
    int disp;
};

template <int PREC>
__global__ __launch_bounds__(kBlock) void k_adjoint_vec(VecArgs v) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (v.disp) fold_disp(v.st.ctl, v.disp_step, v.dyn.thr2, i < v.g.n ? frame_d2_bits<PREC>(v.st, v.box, v.cur, i) : 0u);
    if (i >= v.g.n) return;
    switch (v.op) {
        case kOpGatherById: {
            const int64_t id = v.st.id[i];
            if (id >= 0 && id < v.g.n)
                v.a[i] = make_double4(v.src_id[3 * id], v.src_id[3 * id + 1], v.src_id[3 * id + 2], 0.0);
            break;
        }
        case kOpScatterById: {
            const int64_t id = v.st.id[i];
            if (id >= 0 && id < v.g.n) {
                const double4 x = v.a[i];
                v.dst_id[3 * id] = x.x;
                v.dst_id[3 * id + 1] = x.y;
                v.dst_id[3 * id + 2] = x.z;
            }
            break;
        }
        case kOpDriftCotangent: {
            double4 y = v.b[i];
            if (v.scale != 0.0) {
                const double4 x = v.a[i];
                y.x = fma(v.scale, x.x, y.x);
                y.y = fma(v.scale, x.y, y.y);
                y.z = fma(v.scale, x.z, y.z);
                v.b[i] = y;
            }
            int sp;
            if constexpr (PREC == LJMD_FP64)
                sp = (int)v.st.rec64[v.cur][i].w;
            else
                sp = v.st.recq[v.cur][i].w;
            const double im = 1.0 / by_s(sp, v.dyn.mass);
            if constexpr (PREC == LJMD_FP64)
                ((double4 *)v.gvec)[i] = make_double4(y.x * im, y.y * im, y.z * im, 0.0);
            else
                ((float4 *)v.gvec)[i] = make_float4((float)(y.x * im), (float)(y.y * im), (float)(y.z * im), 0.f);
            break;
        }
        case kOpZero:
            v.a[i] = make_double4(0, 0, 0, 0);
            break;
        case kOpSubForce: {
            double fx, fy, fz;
            if constexpr (PREC == LJMD_FP64) {
                const double4 f = v.st.frc64[i];
                fx = f.x, fy = f.y, fz = f.z;
            } else {
                const float4 f = v.st.frc32[i];
                fx = f.x, fy = f.y, fz = f.z;
            }
            const double c = *v.dscale;
            double4 y = v.a[i];
            y.x = fma(-c, fx, y.x);
            y.y = fma(-c, fy, y.y);
            y.z = fma(-c, fz, y.z);
            v.a[i] = y;
            break;
        }
        case kOpGatherG: {
            const int64_t id = v.st.id[i];
            if (id < 0 || id >= v.g.n) break;
            const double gx = v.src_id[3 * id], gy = v.src_id[3 * id + 1], gz = v.src_id[3 * id + 2];
            if constexpr (PREC == LJMD_FP64)
                ((double4 *)v.gvec)[i] = make_double4(gx, gy, gz, 0.0);
            else
                ((float4 *)v.gvec)[i] = make_float4((float)gx, (float)gy, (float)gz, 0.f);
            break;
        }
        default:
            break;
    }
}

// ------------------------------------------------------------------------
static int adjoint_blocks(const Geom &g) {
    const int per_block = (kBlock / kWave) * (kWave / g.lanes);
    return (int)((g.n + per_block - 1) / per_block);
}

template <int PREC, int NS>
static void pairs_launch(int mode, dim3 grid, hipStream_t s, const AdjArgs &aa) {
    if (mode == kAdjVjp)
        hipLaunchKernelGGL((k_adjoint_pairs<PREC, NS, kAdjVjp>), grid, dim3(kBlock), 0, s, aa);
    else
        hipLaunchKernelGGL((k_adjoint_pairs<PREC, NS, kAdjEnergy>), grid, dim3(kBlock), 0, s, aa);
}

static AdjArgs pair_args(const Launch &L, const void *gvec, double4 *gx, double weight);

hipError_t launch_adjoint_pairs(const Launch &L, int mode, const void *gvec, double4 *gx, double weight,
                                double *gtheta, int init) {
    AdjArgs aa = pair_args(L, gvec, gx, weight);
    const int nb = adjoint_blocks(*L.g);
    if (nb > L.g->max_blocks) return hipErrorInvalidValue;
    const dim3 grid(nb);
    const bool two = L.g->nspecies == 2;
    if (L.g->prec == LJMD_FP64) {
        if (two) pairs_launch<LJMD_FP64, 2>(mode, grid, L.stream, aa);
        else pairs_launch<LJMD_FP64, 1>(mode, grid, L.stream, aa);
    } else {
        if (two) pairs_launch<LJMD_FP32_DS, 2>(mode, grid, L.stream, aa);
        else pairs_launch<LJMD_FP32_DS, 1>(mode, grid, L.stream, aa);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_adjoint_reduce, dim3(1), dim3(kBlock), 0, L.stream, (const double *)L.st->partials,
                       nb, weight, gtheta, init);
    return hipGetLastError();
}

int adjoint_rows(const Geom &g) { return adjoint_blocks(g); }

hipError_t launch_adjoint_vjp_rows(const Launch &L, const void *gvec, double4 *gx, double weight, double *rows,
                                   int init, int64_t step, int forced, const AdjNext *nx) {
    AdjArgs aa = pair_args(L, gvec, gx, weight);
    if (nx) {
        aa.next = 1;
        aa.lv = nx->lv;
        aa.gv_next = nx->gv_next;
        aa.next_scale = nx->scale;
        aa.next_step = nx->step;
        aa.next_rec = nx->rec;
    }
    aa.rows = rows;
    aa.rows_weight = weight;
    aa.rows_init = init;
    aa.clear_cells = 1;
    aa.forced = forced;
    aa.step = step;
    const int nb = adjoint_blocks(*L.g);
    const dim3 grid(nb);
    const bool two = L.g->nspecies == 2;
    if (L.g->prec == LJMD_FP64) {
        if (two) pairs_launch<LJMD_FP64, 2>(kAdjVjp, grid, L.stream, aa);
        else pairs_launch<LJMD_FP64, 1>(kAdjVjp, grid, L.stream, aa);
    } else {
        if (two) pairs_launch<LJMD_FP32_DS, 2>(kAdjVjp, grid, L.stream, aa);
        else pairs_launch<LJMD_FP32_DS, 1>(kAdjVjp, grid, L.stream, aa);
    }
    return hipGetLastError();
}

hipError_t launch_adjoint_reduce(const Launch &L, const double *rows, double *gtheta) {
    hipLaunchKernelGGL(k_adjoint_reduce, dim3(1), dim3(kBlock), 0, L.stream, rows, adjoint_blocks(*L.g), 1.0,
                       gtheta, 1);
    return hipGetLastError();
}

static AdjArgs pair_args(const Launch &L, const void *gvec, double4 *gx, double weight) {
    AdjArgs aa;
    aa.st = *L.st;
    aa.g = *L.g;
    aa.box = *L.box;
    aa.pc = *L.pc;
    aa.cur = L.cur;
    aa.gvec = gvec;
    aa.gx = gx;
    aa.weight = weight;
    aa.rows = L.st->partials;
    aa.rows_weight = 1.0;
    aa.rows_init = 1;
    aa.clear_cells = 0;
    aa.forced = 0;
    aa.step = 0;
    aa.thr2 = L.dyn->thr2;
    aa.next = 0;
    aa.lv = nullptr;
    aa.gv_next = nullptr;
    aa.next_scale = 0.0;
    aa.next_step = 0;
    aa.next_rec = nullptr;
    aa.mass[0] = L.dyn->mass[0];
    aa.mass[1] = L.dyn->mass[1];
    aa.shifted = 0;
    for (int t = 0; t < 3; ++t) {
        const double c2 = L.pc->sig2[t] / L.pc->rc2[t];
        aa.c6[t] = c2 * c2 * c2;
        aa.c12[t] = aa.c6[t] * aa.c6[t];
        const double eps = L.pc->eps24[t] / 24.0;
        aa.inv_eps[t] = eps != 0.0 ? 1.0 / eps : 0.0;
        aa.inv_sig[t] = 1.0 / sqrt(L.pc->sig2[t]);
        if (L.pc->shift[t] != 0.0) aa.shifted = 1;
    }
    return aa;
}

hipError_t launch_adjoint_cells(const Launch &L, int64_t step, int forced) {
    const int nbc = (L.box->ncell + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(k_adjoint_cells, dim3(nbc < 1024 ? nbc : 1024), dim3(kBlock), 0, L.stream, *L.st,
                       *L.box, step, forced, L.dyn->thr2);
    return hipGetLastError();
}

static hipError_t vec_launch(const Launch &L, const VecArgs &v);

__global__ void k_theta_axpy(const double *dc, const double *g, double *gtheta) {
    if (threadIdx.x < 6) gtheta[threadIdx.x] = fma(*dc, g[threadIdx.x], gtheta[threadIdx.x]);
}

hipError_t launch_theta_axpy(const Launch &L, const double *dc, const double *g, double *gtheta) {
    hipLaunchKernelGGL(k_theta_axpy, dim3(1), dim3(64), 0, L.stream, dc, g, gtheta);
    return hipGetLastError();
}

hipError_t launch_adjoint_vec(const Launch &L, int op, const double *src_id, double *dst_id, double4 *a,
                              double4 *b, void *gvec, double scale, const double *dscale) {
    VecArgs v;
    v.st = *L.st;
    v.g = *L.g;
    v.dyn = *L.dyn;
    v.cur = L.cur;
    v.op = op;
    v.src_id = src_id;
    v.dst_id = dst_id;
    v.a = a;
    v.b = b;
    v.gvec = gvec;
    v.scale = scale;
    v.dscale = dscale;
    v.box = *L.box;
    v.disp_step = 0;
    v.disp = 0;
    return vec_launch(L, v);
}

hipError_t launch_adjoint_drift(const Launch &L, double4 *lx, double4 *lv, void *gvec, double scale, int64_t step,
                                int disp) {
    VecArgs v;
    v.st = *L.st;
    v.g = *L.g;
    v.dyn = *L.dyn;
    v.cur = L.cur;
    v.op = kOpDriftCotangent;
    v.src_id = nullptr;
    v.dst_id = nullptr;
    v.a = lx;
    v.b = lv;
    v.gvec = gvec;
    v.scale = scale;
    v.dscale = nullptr;
    v.box = *L.box;
    v.disp_step = step;
    v.disp = disp;
    return vec_launch(L, v);
}

static hipError_t vec_launch(const Launch &L, const VecArgs &v) {
    const dim3 grid((unsigned)((L.g->n + kBlock - 1) / kBlock));
    if (L.g->prec == LJMD_FP64)
        hipLaunchKernelGGL(k_adjoint_vec<LJMD_FP64>, grid, dim3(kBlock), 0, L.stream, v);
    else
        hipLaunchKernelGGL(k_adjoint_vec<LJMD_FP32_DS>, grid, dim3(kBlock), 0, L.stream, v);
    return hipGetLastError();
}

}  // namespace ljmd
