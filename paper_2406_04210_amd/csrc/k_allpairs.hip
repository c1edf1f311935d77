// k_allpairs.hip -- the untruncated all-to-all Lennard-Jones interaction on
// gfx950: every pair of the minimum image interacts through the plain 12-6
// potential (paper Sec. 4, "Code migration": the port started from this
// interaction combined with velocity Verlet and an Andersen-like
// thermostat; Sec. 5, "GPU Performance for All-to-All Interaction": 2,000
// particles over 20,000 steps). No lists, no cells: a context whose cutoffs
// are all infinite steps with these two launches per step.
//
//   k_ap_forces  -- block (i tile of 64 slots, j split s) stages the records
//                   of its j range in LDS, 1024 at a time; its four waves
//                   take quarters of each chunk, every lane (one particle i)
//                   reading the same record j (an LDS broadcast). The four
//                   wave partials are summed in LDS in a fixed order and
//                   written to partial row s of the tile's particles.
//   k_ap_finish  -- per particle the S partial rows in order, then the step
//                   tail of the list path (finalize, thermostat, observable
//                   terms, integrate) and the deterministic block partials.
//
// The j split S spreads a small system over the chip (N = 2,000: 32 tiles x
// 16 splits = 512 blocks, 2,048 waves); large systems take S = 1.
#include "step_common.h"

namespace ljmd {

constexpr int kApWaves = 4;            // waves per force block
constexpr int kApChunk = 1024;         // records staged in LDS at a time

// Partial rows: forces (fx, fy, fz, -) and (e, w) per split and slot.
template <int PREC>
struct ApRow {
    using F = typename std::conditional<PREC == LJMD_FP64, double4, float4>::type;
};

// Pair terms of one untruncated pair. FP32 paths: raw fixed-point
// differences in a cubic box (displacements in quanta, sigma^2 and
// 24 eps / quantum pre-scaled as in the list kernel); FP64: minimum-image
// displacements of the FP64 records.
// CUT: pairs at r >= r_c are skipped and the energy is shifted (the brute-
// force sum of the truncated potential); without it every pair interacts.
// an counts the pairs inside (one species: the shift is applied per pair
// once the sums are done).
template <int NS, bool CUT>
__device__ inline void ap_pair(const int4 &ri, const int4 &rj, const BoxC &box, const PairC &pc, float &fx,
                               float &fy, float &fz, float &sa, float &sb, int &an) {
    const float dx = (float)(int32_t)((uint32_t)ri.x - (uint32_t)rj.x);
    const float dy = (float)(int32_t)((uint32_t)ri.y - (uint32_t)rj.y);
    const float dz = (float)(int32_t)((uint32_t)ri.z - (uint32_t)rj.z);
    const float r2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
    const int t = NS == 1 ? 0 : ri.w + rj.w;
    if (CUT && !(r2 < by_t<NS>(t, box.rc2q))) return;
    an += 1;
    const float ir2 = __builtin_amdgcn_rcpf(r2);
    const float s2 = by_t<NS>(t, box.sig2q) * ir2;
    const float s6 = s2 * s2 * s2;
    float g = (s6 * ir2) * fmaf(2.0f, s6, -1.0f);
    if constexpr (NS == 2) g *= by_t<NS>(t, box.fq);
    fx = fmaf(g, dx, fx);
    fy = fmaf(g, dy, fy);
    fz = fmaf(g, dz, fz);
    if constexpr (NS == 1) {
        sa = fmaf(s6, s6, sa);
        sb += s6;
    } else {
        const float s12 = s6 * s6;
        sa += fmaf(by_t<NS>(t, pc.eps4f), s12 - s6, -by_t<NS>(t, pc.shiftf));
        sb += by_t<NS>(t, pc.eps24f) * fmaf(2.0f, s12, -s6);
    }
}

template <int NS, bool CUT>
__device__ inline void ap_pair(const double4 &ri, const double4 &rj, const BoxC &box, const PairC &pc, double &fx,
                               double &fy, double &fz, double &e, double &w, int &an) {
    const double dx = disp_d(ri.x, rj.x, box.L[0], box.invL[0]);
    const double dy = disp_d(ri.y, rj.y, box.L[1], box.invL[1]);
    const double dz = disp_d(ri.z, rj.z, box.L[2], box.invL[2]);
    const double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
    const int t = NS == 1 ? 0 : (int)ri.w + (int)rj.w;
    if (CUT && !(r2 < by_t<NS>(t, pc.rc2))) return;
    an += 1;
    double ir2 = __builtin_amdgcn_rcp(r2);
    ir2 = fma(ir2, fma(-r2, ir2, 1.0), ir2);
    ir2 = fma(ir2, fma(-r2, ir2, 1.0), ir2);
    const double s2 = by_t<NS>(t, pc.sig2) * ir2;
    const double s6 = s2 * s2 * s2;
    const double fs = by_t<NS>(t, pc.eps24) * s6 * fma(2.0, s6, -1.0) * ir2;
    fx = fma(fs, dx, fx);
    fy = fma(fs, dy, fy);
    fz = fma(fs, dz, fz);
    e += fma(by_t<NS>(t, pc.eps4) * s6, s6 - 1.0, -by_t<NS>(t, pc.shift));
    w = fma(fs, r2, w);
}

// Operands of the force pass: records (slot order) and the partial rows.
struct ApForce {
    const void *rec;    // int4 fixed-point (single precision) or double4 (FP64) records
    void *part;         // S rows of (fx, fy, fz, -) then S rows of (e, w)
    int64_t n;
    size_t stride;      // slots per row (>= n)
    int nsplit;
    BoxC box;
    PairC pc;
};

template <int PREC, int NS, bool CUT>
__global__ __launch_bounds__(kApWaves * kWave) void k_ap_forces(ApForce a, const Ctl *ctl) {
    using Rec = typename std::conditional<PREC == LJMD_FP64, double4, int4>::type;
    using Acc = typename std::conditional<PREC == LJMD_FP64, double, float>::type;
    using F = typename ApRow<PREC>::F;
    __shared__ Rec stage[kApChunk];
    __shared__ double red[kApWaves][5][kWave];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t n = a.n;
    const int nsplit = a.nsplit;
    const int tile = blockIdx.x / nsplit, split = blockIdx.x - tile * nsplit;
    const int64_t i = (int64_t)tile * kWave + lane;
    const Rec *__restrict__ rec = (const Rec *)a.rec;
    const Rec ri = i < n ? rec[i] : Rec{};
    const int64_t per = (n + nsplit - 1) / nsplit;
    const int64_t jb = split * per, je = jb + per < n ? jb + per : n;
    Acc fx = 0, fy = 0, fz = 0;
    double e = 0.0, w = 0.0;
    int an = 0;
    // One species: per-lane sums of s6^2 and s6 (the constants are applied
    // once below); two species: per-pair energies and virials.
    for (int64_t c0 = jb; c0 < je; c0 += kApChunk) {
        const int len = (int)(je - c0 < kApChunk ? je - c0 : kApChunk);
        for (int k = threadIdx.x; k < len; k += kApWaves * kWave) stage[k] = rec[c0 + k];
        __syncthreads();
        const int q0 = len * wv / kApWaves, q1 = len * (wv + 1) / kApWaves;
        Acc sa = 0, sb = 0;
        const int64_t self = i - c0;  // the particle's own slot in this chunk (if any): no self pair
#pragma unroll 4
        for (int k = q0; k < q1; ++k)
            if (k != self) ap_pair<NS, CUT>(ri, stage[k], a.box, a.pc, fx, fy, fz, sa, sb, an);
        e += (double)sa;
        w += (double)sb;
        __syncthreads();
    }
    if constexpr (PREC != LJMD_FP64 && NS == 1) {
        // sum phi_s = 4 eps (a12 - a6) - an phi(r_c), sum fs r^2 = 24 eps (2 a12 - a6).
        const double a12 = e, a6 = w;
        e = a.pc.eps4[0] * (a12 - a6) - (double)an * a.pc.shift[0];
        w = a.pc.eps24[0] * (2.0 * a12 - a6);
    }
    red[wv][0][lane] = (double)fx;
    red[wv][1][lane] = (double)fy;
    red[wv][2][lane] = (double)fz;
    red[wv][3][lane] = e;
    red[wv][4][lane] = w;
    __syncthreads();
    // The pass only reads until here; the halt check (its latency overlapping
    // the pass) gates the writes.
    if (ctl && halted(ctl)) return;
    if (wv == 0 && i < n) {
        double s[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
        for (int q = 0; q < kApWaves; ++q)
            for (int k = 0; k < 5; ++k) s[k] += red[q][k][lane];
        F *pf = (F *)a.part;
        double2 *pe = (double2 *)(pf + (size_t)nsplit * a.stride);
        const size_t row = (size_t)split * a.stride + i;
        if constexpr (PREC == LJMD_FP64) {
            pf[row] = make_double4(s[0], s[1], s[2], 0.0);
        } else {
            // FP32 forces: the four wave sums were formed in binary32.
            const float c24 = NS == 1 ? a.box.fq[0] : 1.0f;
            pf[row] = make_float4((float)s[0] * c24, (float)s[1] * c24, (float)s[2] * c24, 0.0f);
        }
        pe[row] = make_double2(s[3], s[4]);
    }
}

// One wavefront per block: a small system spreads its step tail over many
// compute units. Every lane first issues the loads of its step-tail operands
// (record, list reference, state) and of up to 16 split rows at once, then
// adds the rows in split order: a small system's step is a chain of
// latencies (N = 2,000: one round of row loads instead of four measured
// 14.2 -> 13.0 us per step).
template <int PREC, bool TH>
__global__ __launch_bounds__(kApFinishBlock) void k_ap_finish(StepArgs a, const void *part, int nsplit) {
    using F = typename ApRow<PREC>::F;
    constexpr int BS = kApFinishBlock;
    constexpr int UR = 16;  // split rows per round of loads
    Ctl *ctl = a.st.ctl;
    const int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x;
    const size_t stride = (size_t)a.g.max_blocks * BS;
    const F *pf = (const F *)part;
    const double2 *pe = (const double2 *)(pf + (size_t)nsplit * stride);
    double pu = 0.0, pw = 0.0, pk = 0.0, ppx = 0.0, ppy = 0.0, ppz = 0.0;
    uint32_t dm = 0u;
    const bool valid = i < a.g.n;
    // Everything up to the step tail only reads, so it goes ahead of the halt
    // check, whose latency then overlaps the loads.
    double4 r64;
    int si = 0;
    int4 xr;
    DsState ds;
    if (valid) {
        if constexpr (PREC == LJMD_FP64) {
            r64 = a.st.rec64[a.cur][i];
        } else {
            si = a.st.recq[a.cur][i].w;
            xr = a.st.xref[i];
            ds = ds_load(a.st.dsw, i);
        }
    }
    F f;
    double2 ew;
    if (valid) {
        for (int s0 = 0; s0 < nsplit; s0 += UR) {
            F g[UR];
            double2 h[UR];
#pragma unroll
            for (int u = 0; u < UR; ++u) {
                if (s0 + u < nsplit) {
                    g[u] = pf[(size_t)(s0 + u) * stride + i];
                    h[u] = pe[(size_t)(s0 + u) * stride + i];
                }
            }
#pragma unroll
            for (int u = 0; u < UR; ++u) {
                if (s0 + u >= nsplit) break;
                if (s0 + u == 0) {
                    f = g[0];
                    ew = h[0];
                } else {
                    f.x += g[u].x;
                    f.y += g[u].y;
                    f.z += g[u].z;
                    ew.x += h[u].x;
                    ew.y += h[u].y;
                }
            }
        }
    }
    if (halted_record(ctl, a.step, blockIdx.x == 0)) return;
    if (valid) {
        if constexpr (PREC == LJMD_FP64)
            finish_fp64<TH>(a, a.box, i, r64, f.x, f.y, f.z, ew.x, ew.y, pu, pw, pk, ppx, ppy, ppz, dm);
        else
            finish_ds<true, TH, PREC == LJMD_FP32>(a, a.box, i, si, xr, ds, f.x, f.y, f.z, ew.x, ew.y, pu, pw, pk,
                                                   ppx, ppy, ppz, dm);
    }
    block_finish<true, BS>(a, ctl, blockIdx.x, pu, pw, pk, ppx, ppy, ppz, dm);
}

// Splits of the j range: enough blocks for about 2,048 waves, at most one
// split per tile.
int allpairs_splits(int64_t n) {
    const int64_t tiles = (n + kWave - 1) / kWave;
    int64_t s = (2048 + kApWaves * tiles - 1) / (kApWaves * tiles);
    if (s > tiles) s = tiles;
    return (int)(s < 1 ? 1 : s);
}

// Bytes of the partial rows for n particles: S rows of (forces, e and w)
// per finish-kernel slot.
size_t allpairs_part_bytes(int64_t n, int prec) {
    const int bs = kApFinishBlock;
    const size_t slots = (size_t)((n + bs - 1) / bs) * bs;
    const size_t row = (prec == LJMD_FP64 ? sizeof(double4) : sizeof(float4)) + sizeof(double2);
    return (size_t)allpairs_splits(n) * slots * row;
}

hipError_t launch_allpairs_step(const Launch &L, int64_t step, int mode, int slot) {
    StepArgs a;
    a.st = *L.st;
    a.g = *L.g;
    a.box = *L.box;
    a.pc = *L.pc;
    a.dyn = *L.dyn;
    a.cur = L.cur;
    a.forced = 0;
    a.mode = mode;
    a.slot = slot;
    a.step = step;
    void *part = L.st->nbr;  // the list area holds the partial rows in this mode
    const int S = allpairs_splits(L.g->n);
    const int bs = kApFinishBlock;
    ApForce af;
    af.rec = L.g->prec == LJMD_FP64 ? (const void *)L.st->rec64[L.cur] : (const void *)L.st->recq[L.cur];
    af.part = part;
    af.n = L.g->n;
    af.stride = (size_t)L.g->max_blocks * bs;
    af.nsplit = S;
    af.box = *L.box;
    af.pc = *L.pc;
    const dim3 gf((unsigned)(((L.g->n + kWave - 1) / kWave) * S)), bf(kApWaves * kWave);
    const dim3 gn((unsigned)((L.g->n + bs - 1) / bs)), bn(bs);
    const bool th = L.dyn->thermo_on && (mode & kFinalize);
    const bool two = L.g->nspecies == 2;
#define AP(PREC)                                                                                           \
    do {                                                                                                   \
        if (two)                                                                                           \
            hipLaunchKernelGGL((k_ap_forces<PREC, 2, false>), gf, bf, 0, L.stream, af, L.st->ctl);         \
        else                                                                                               \
            hipLaunchKernelGGL((k_ap_forces<PREC, 1, false>), gf, bf, 0, L.stream, af, L.st->ctl);         \
        if (th)                                                                                            \
            hipLaunchKernelGGL((k_ap_finish<PREC, true>), gn, bn, 0, L.stream, a, (const void *)part, S);  \
        else                                                                                               \
            hipLaunchKernelGGL((k_ap_finish<PREC, false>), gn, bn, 0, L.stream, a, (const void *)part, S); \
    } while (0)
    if (L.g->prec == LJMD_FP64)
        AP(LJMD_FP64);
    else if (L.g->prec == LJMD_FP32)
        AP(LJMD_FP32);
    else
        AP(LJMD_FP32_DS);
#undef AP
    return hipGetLastError();
}

// ---- one-shot brute-force forces ----------------------------------------
// Records of a configuration given by id (slot = id): the wrap of the state
// load, then the FP64 record, or the double-single split and fixed-point
// record (single floats with zero lo parts for the plain FP32 state).
template <int PREC>
__global__ __launch_bounds__(kBlock) void k_bf_records(const double *__restrict__ x, const int32_t *__restrict__ sp,
                                                       int64_t n, int nspecies, int dim, BoxC box, void *rec) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    int s = sp[i];
    s = s < 0 ? 0 : (s >= nspecies ? nspecies - 1 : s);
    double w[3];
    for (int k = 0; k < 3; ++k) {
        const double xi = (k == 2 && dim == 2) ? 0.0 : x[3 * i + k];  // two dimensions: z = 0
        double t = xi - box.L[k] * floor(xi / box.L[k]);
        if (t >= box.L[k]) t -= box.L[k];
        w[k] = t;
    }
    if constexpr (PREC == LJMD_FP64) {
        ((double4 *)rec)[i] = make_double4(w[0], w[1], w[2], (double)s);
    } else {
        uint32_t q[3];
        for (int k = 0; k < 3; ++k) {
            float hi = (float)w[k];
            float lo = 0.0f;
            if constexpr (PREC == LJMD_FP32) {
                if (hi >= box.Lhi[k]) hi -= box.Lhi[k];
            } else {
                lo = (float)(w[k] - (double)hi);
            }
            q[k] = q_from_ds(hi, lo, box.S_hi[k], box.S_lo[k]);
        }
        ((int4 *)rec)[i] = make_int4((int)q[0], (int)q[1], (int)q[2], s);
    }
}

// Per particle the S partial rows in order -> f (FP64, by id); per block the
// sums of e/2 and w/2 in a fixed order -> blk_uw[2 * block].
template <int PREC>
__global__ __launch_bounds__(kBlock) void k_bf_sum(const void *part, int64_t n, size_t stride, int nsplit,
                                                   double *__restrict__ f, double *__restrict__ blk_uw) {
    using F = typename ApRow<PREC>::F;
    __shared__ double red[kBlock / kWave][2];
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const F *pf = (const F *)part;
    const double2 *pe = (const double2 *)(pf + (size_t)nsplit * stride);
    double u = 0.0, v = 0.0;
    if (i < n) {
        F g = pf[i];
        double2 ew = pe[i];
        for (int s = 1; s < nsplit; ++s) {
            const F h = pf[(size_t)s * stride + i];
            const double2 k = pe[(size_t)s * stride + i];
            g.x += h.x;
            g.y += h.y;
            g.z += h.z;
            ew.x += k.x;
            ew.y += k.y;
        }
        f[3 * i] = (double)g.x;
        f[3 * i + 1] = (double)g.y;
        f[3 * i + 2] = (double)g.z;
        u = 0.5 * ew.x;
        v = 0.5 * ew.y;
    }
    for (int o = 32; o > 0; o >>= 1) {
        u += __shfl_xor(u, o);
        v += __shfl_xor(v, o);
    }
    if ((threadIdx.x & 63) == 0) {
        red[threadIdx.x >> 6][0] = u;
        red[threadIdx.x >> 6][1] = v;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double su = 0.0, sv = 0.0;
        for (int q = 0; q < kBlock / kWave; ++q) {
            su += red[q][0];
            sv += red[q][1];
        }
        blk_uw[2 * blockIdx.x] = su;
        blk_uw[2 * blockIdx.x + 1] = sv;
    }
}

// uw = the block sums in a fixed order (one block).
__global__ __launch_bounds__(kBlock) void k_bf_reduce(const double *__restrict__ blk_uw, int nb, double *uw) {
    __shared__ double red[kBlock][2];
    double u = 0.0, v = 0.0;
    for (int b = threadIdx.x; b < nb; b += kBlock) {
        u += blk_uw[2 * b];
        v += blk_uw[2 * b + 1];
    }
    red[threadIdx.x][0] = u;
    red[threadIdx.x][1] = v;
    __syncthreads();
    for (int s = kBlock / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            red[threadIdx.x][0] += red[threadIdx.x + s][0];
            red[threadIdx.x][1] += red[threadIdx.x + s][1];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        uw[0] = red[0][0];
        uw[1] = red[0][1];
    }
}

// Scratch of a one-shot evaluation: records, partial rows, block sums.
struct BruteScratch {
    size_t off_rows, off_blk, total, stride;
    int nsplit, nb;
};

static BruteScratch brute_layout(int64_t n, int prec) {
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    BruteScratch b;
    const int64_t npad = (n + kBlock - 1) / kBlock * kBlock;
    b.stride = (size_t)npad;
    b.nsplit = allpairs_splits(n);
    b.nb = (int)(npad / kBlock);
    const size_t rec = prec == LJMD_FP64 ? sizeof(double4) : sizeof(int4);
    const size_t row = (prec == LJMD_FP64 ? sizeof(double4) : sizeof(float4)) + sizeof(double2);
    b.off_rows = al(rec * npad);
    b.off_blk = b.off_rows + al((size_t)b.nsplit * b.stride * row);
    b.total = b.off_blk + al(2 * sizeof(double) * (size_t)b.nb);
    return b;
}

size_t brute_scratch_bytes(int64_t n, int prec) { return brute_layout(n, prec).total; }

hipError_t launch_brute(const BoxC &box, const PairC &pc, int prec, int nspecies, int dim, int cut, int64_t n,
                        const double *x, const int32_t *sp, double *f, double *uw, uint8_t *scratch,
                        hipStream_t stream) {
    const BruteScratch bl = brute_layout(n, prec);
    ApForce af;
    af.rec = scratch;
    af.part = scratch + bl.off_rows;
    af.n = n;
    af.stride = bl.stride;
    af.nsplit = bl.nsplit;
    af.box = box;
    af.pc = pc;
    double *blk = (double *)(scratch + bl.off_blk);
    const dim3 gr((unsigned)bl.nb), b1(kBlock);
    const dim3 gf((unsigned)(((n + kWave - 1) / kWave) * bl.nsplit)), bf(kApWaves * kWave);
    const Ctl *none = nullptr;
#define BF(PREC)                                                                                              \
    do {                                                                                                      \
        hipLaunchKernelGGL(k_bf_records<PREC>, gr, b1, 0, stream, x, sp, n, nspecies, dim, box, scratch);   \
        if (nspecies == 2 && cut)                                                                             \
            hipLaunchKernelGGL((k_ap_forces<PREC, 2, true>), gf, bf, 0, stream, af, none);                   \
        else if (nspecies == 2)                                                                               \
            hipLaunchKernelGGL((k_ap_forces<PREC, 2, false>), gf, bf, 0, stream, af, none);                  \
        else if (cut)                                                                                         \
            hipLaunchKernelGGL((k_ap_forces<PREC, 1, true>), gf, bf, 0, stream, af, none);                   \
        else                                                                                                  \
            hipLaunchKernelGGL((k_ap_forces<PREC, 1, false>), gf, bf, 0, stream, af, none);                  \
        hipLaunchKernelGGL(k_bf_sum<PREC>, gr, b1, 0, stream, (const void *)af.part, n, bl.stride, bl.nsplit, \
                           f, blk);                                                                           \
    } while (0)
    if (prec == LJMD_FP64)
        BF(LJMD_FP64);
    else if (prec == LJMD_FP32)
        BF(LJMD_FP32);
    else
        BF(LJMD_FP32_DS);
#undef BF
    hipLaunchKernelGGL(k_bf_reduce, dim3(1), b1, 0, stream, (const double *)blk, bl.nb, uw);
    return hipGetLastError();
}

}  // namespace ljmd
