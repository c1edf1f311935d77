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
template <int NS>
__device__ inline void ap_pair(const int4 &ri, const int4 &rj, const BoxC &box, const PairC &pc, float &fx,
                               float &fy, float &fz, float &sa, float &sb) {
    const float dx = (float)(int32_t)((uint32_t)ri.x - (uint32_t)rj.x);
    const float dy = (float)(int32_t)((uint32_t)ri.y - (uint32_t)rj.y);
    const float dz = (float)(int32_t)((uint32_t)ri.z - (uint32_t)rj.z);
    const float r2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
    const int t = NS == 1 ? 0 : ri.w + rj.w;
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
        sa += by_t<NS>(t, pc.eps4f) * (s12 - s6);
        sb += by_t<NS>(t, pc.eps24f) * fmaf(2.0f, s12, -s6);
    }
}

template <int NS>
__device__ inline void ap_pair(const double4 &ri, const double4 &rj, const BoxC &box, const PairC &pc, double &fx,
                               double &fy, double &fz, double &e, double &w) {
    const double dx = disp_d(ri.x, rj.x, box.L[0], box.invL[0]);
    const double dy = disp_d(ri.y, rj.y, box.L[1], box.invL[1]);
    const double dz = disp_d(ri.z, rj.z, box.L[2], box.invL[2]);
    const double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
    const int t = NS == 1 ? 0 : (int)ri.w + (int)rj.w;
    double ir2 = __builtin_amdgcn_rcp(r2);
    ir2 = fma(ir2, fma(-r2, ir2, 1.0), ir2);
    ir2 = fma(ir2, fma(-r2, ir2, 1.0), ir2);
    const double s2 = by_t<NS>(t, pc.sig2) * ir2;
    const double s6 = s2 * s2 * s2;
    const double fs = by_t<NS>(t, pc.eps24) * s6 * fma(2.0, s6, -1.0) * ir2;
    fx = fma(fs, dx, fx);
    fy = fma(fs, dy, fy);
    fz = fma(fs, dz, fz);
    e += by_t<NS>(t, pc.eps4) * s6 * (s6 - 1.0);
    w = fma(fs, r2, w);
}

template <int PREC, int NS>
__global__ __launch_bounds__(kApWaves * kWave) void k_ap_forces(StepArgs a, void *part, int nsplit) {
    using Rec = typename std::conditional<PREC == LJMD_FP64, double4, int4>::type;
    using Acc = typename std::conditional<PREC == LJMD_FP64, double, float>::type;
    using F = typename ApRow<PREC>::F;
    __shared__ Rec stage[kApChunk];
    __shared__ double red[kApWaves][5][kWave];
    const State &st = a.st;
    if (halted(st.ctl)) return;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t n = a.g.n;
    const int tile = blockIdx.x / nsplit, split = blockIdx.x - tile * nsplit;
    const int64_t i = (int64_t)tile * kWave + lane;
    const Rec *__restrict__ rec;
    if constexpr (PREC == LJMD_FP64)
        rec = st.rec64[a.cur];
    else
        rec = st.recq[a.cur];
    const Rec ri = i < n ? rec[i] : Rec{};
    const int64_t per = (n + nsplit - 1) / nsplit;
    const int64_t jb = split * per, je = jb + per < n ? jb + per : n;
    Acc fx = 0, fy = 0, fz = 0;
    double e = 0.0, w = 0.0;
    // One species: per-lane sums of s6^2 and s6 (the constants are applied
    // once below); two species: per-pair energies and virials.
    for (int64_t c0 = jb; c0 < je; c0 += kApChunk) {
        const int len = (int)(je - c0 < kApChunk ? je - c0 : kApChunk);
        for (int k = threadIdx.x; k < len; k += kApWaves * kWave) stage[k] = rec[c0 + k];
        __syncthreads();
        const int q0 = len * wv / kApWaves, q1 = len * (wv + 1) / kApWaves;
        Acc sa = 0, sb = 0;
        for (int k = q0; k < q1; ++k) {
            if (c0 + k == i) continue;          // no self pair
            ap_pair<NS>(ri, stage[k], a.box, a.pc, fx, fy, fz, sa, sb);
        }
        e += (double)sa;
        w += (double)sb;
        __syncthreads();
    }
    if constexpr (PREC != LJMD_FP64 && NS == 1) {
        // sum phi = 4 eps (a12 - a6), sum fs r^2 = 24 eps (2 a12 - a6).
        const double a12 = e, a6 = w;
        e = a.pc.eps4[0] * (a12 - a6);
        w = a.pc.eps24[0] * (2.0 * a12 - a6);
    }
    red[wv][0][lane] = (double)fx;
    red[wv][1][lane] = (double)fy;
    red[wv][2][lane] = (double)fz;
    red[wv][3][lane] = e;
    red[wv][4][lane] = w;
    __syncthreads();
    if (wv == 0 && i < n) {
        double s[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
        for (int q = 0; q < kApWaves; ++q)
            for (int k = 0; k < 5; ++k) s[k] += red[q][k][lane];
        F *pf = (F *)part;
        double2 *pe = (double2 *)(pf + (size_t)nsplit * a.g.max_blocks * step_block_threads(PREC));
        const size_t row = (size_t)split * a.g.max_blocks * step_block_threads(PREC) + i;
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

template <int PREC, bool TH>
__global__ __launch_bounds__(kBlock) void k_ap_finish(StepArgs a, const void *part, int nsplit) {
    using F = typename ApRow<PREC>::F;
    constexpr int BS = PREC == LJMD_FP64 ? kBlockF64 : kBlock;
    Ctl *ctl = a.st.ctl;
    if (halted_record(ctl, a.step, blockIdx.x == 0)) return;
    const int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x;
    const size_t stride = (size_t)a.g.max_blocks * BS;
    const F *pf = (const F *)part;
    const double2 *pe = (const double2 *)(pf + (size_t)nsplit * stride);
    double pu = 0.0, pw = 0.0, pk = 0.0, ppx = 0.0, ppy = 0.0, ppz = 0.0;
    uint32_t dm = 0u;
    if (i < a.g.n) {
        F f = pf[i];
        double2 ew = pe[i];
        for (int s = 1; s < nsplit; ++s) {
            const F g = pf[(size_t)s * stride + i];
            const double2 h = pe[(size_t)s * stride + i];
            f.x += g.x;
            f.y += g.y;
            f.z += g.z;
            ew.x += h.x;
            ew.y += h.y;
        }
        if constexpr (PREC == LJMD_FP64)
            finish_fp64<TH>(a, a.box, i, a.st.rec64[a.cur][i], f.x, f.y, f.z, ew.x, ew.y, pu, pw, pk, ppx, ppy, ppz,
                            dm);
        else
            finish_ds<true, TH, PREC == LJMD_FP32>(a, a.box, i, a.st.recq[a.cur][i].w, f.x, f.y, f.z, ew.x, ew.y,
                                                   pu, pw, pk, ppx, ppy, ppz, dm);
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
    const int bs = step_block_threads(prec);
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
    const dim3 gf((unsigned)(((L.g->n + kWave - 1) / kWave) * S)), bf(kApWaves * kWave);
    const int bs = step_block_threads(L.g->prec);
    const dim3 gn((unsigned)((L.g->n + bs - 1) / bs)), bn(bs);
    const bool th = L.dyn->thermo_on && (mode & kFinalize);
    const bool two = L.g->nspecies == 2;
#define AP(PREC)                                                                                           \
    do {                                                                                                   \
        if (two)                                                                                           \
            hipLaunchKernelGGL((k_ap_forces<PREC, 2>), gf, bf, 0, L.stream, a, part, S);                   \
        else                                                                                               \
            hipLaunchKernelGGL((k_ap_forces<PREC, 1>), gf, bf, 0, L.stream, a, part, S);                   \
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

}  // namespace ljmd
