// k_rebuild.hip -- neighbour-list rebuild on gfx950: particle binning,
// canonical cell order, space-filling-curve resort and Verlet-list build
// (paper Sec. 3 "Code structure": Verlet lists built from particle binning;
// Sec. 4 "Mixed Strategy": sorting).
//
// Every kernel here is launched every step and returns at once unless the
// list is due (host-forced, or the largest displacement since the last build
// exceeded half the skin -- paper Sec. 5: more movement, more list updates).
// The decision reads one control word written by the previous step's kernel,
// so no host synchronisation is needed per step.
#include "internal.h"

namespace ljmd {

// Fixed-point coordinates of particle i in the current record buffer.
template <int PREC>
__device__ inline void load_q(const State &st, int cur, int64_t i, const BoxC &box, uint32_t *q,
                              int *sp) {
    if constexpr (PREC == LJMD_FP64) {
        double4 r = st.rec64[cur][i];
        q[0] = q_from_d(r.x, box.S[0]);
        q[1] = q_from_d(r.y, box.S[1]);
        q[2] = q_from_d(r.z, box.S[2]);
        *sp = (int)r.w;
    } else {
        int4 r = st.recq[cur][i];
        q[0] = (uint32_t)r.x;
        q[1] = (uint32_t)r.y;
        q[2] = (uint32_t)r.z;
        *sp = r.w;
    }
}

// Bin: cell of every particle, counted with an atomic per cell. The slot a
// particle lands in is arbitrary; k_canon restores a deterministic order.
template <int PREC>
__global__ __launch_bounds__(kBlock) void k_bin(State st, Geom g, BoxC box, int cur, int64_t step,
                                                int forced, float thr2) {
    if (blockIdx.x == 0 && threadIdx.x == 0) st.ctl->maxd[(step + 1) & 1] = 0u;
    if (!rebuild_due(st.ctl, step, forced, thr2)) return;
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= g.n) return;
    uint32_t q[3];
    int sp;
    load_q<PREC>(st, cur, i, box, q, &sp);
    int cx, cy, cz;
    int c = cell_of_q(q[0], q[1], q[2], box, st.rank_of, &cx, &cy, &cz);
    int slot = atomicAdd(&st.cell_count[c], 1);
    if (slot < g.cell_cap)
        st.cell_members[(int64_t)c * g.cell_cap + slot] = (int32_t)i;
    else
        atomicOr(&st.ctl->flags, kErrCell);
}

// Canonicalise: one wavefront per cell sorts the cell's particle slots
// ascending by rank counting in LDS (slots are distinct), so that list order
// and hence force summation order are reproducible run to run.
__global__ __launch_bounds__(kBlock) void k_canon(State st, Geom g, BoxC box, int64_t step,
                                                  int forced, float thr2) {
    if (!rebuild_due(st.ctl, step, forced, thr2)) return;
    extern __shared__ int32_t sm[];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t c = (int64_t)blockIdx.x * (kBlock / kWave) + wv;
    if (c >= box.ncell) return;
    const int cnt = st.cell_count[c];
    const int m = cnt < g.cell_cap ? cnt : g.cell_cap;
    if (lane == 0 && cnt > *(volatile int32_t *)&st.ctl->max_cell) atomicMax(&st.ctl->max_cell, cnt);
    int32_t *src = sm + (size_t)wv * 2 * g.cell_cap;
    int32_t *dst = src + g.cell_cap;
    int32_t *mem = st.cell_members + c * g.cell_cap;
    for (int e = lane; e < m; e += kWave) src[e] = mem[e];
    __builtin_amdgcn_wave_barrier();
    for (int e = lane; e < m; e += kWave) {
        int v = src[e];
        int r = 0;
        for (int k = 0; k < m; ++k) r += src[k] < v ? 1 : 0;
        dst[r] = v;
    }
    __builtin_amdgcn_wave_barrier();
    for (int e = lane; e < m; e += kWave) mem[e] = dst[e];
}

// Exclusive scan of the (capped) cell counts in Hilbert-rank order: the
// start of every cell in the resorted particle order. One block.
__global__ __launch_bounds__(1024) void k_scan(State st, Geom g, int ncell) {
    __shared__ int32_t wsum[16];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    int32_t carry = 0;
    for (int base = 0; base < ncell; base += 1024) {
        int idx = base + tid;
        int v = 0;
        if (idx < ncell) {
            v = st.cell_count[idx];
            v = v < g.cell_cap ? v : g.cell_cap;
        }
        int x = v;
        for (int o = 1; o < kWave; o <<= 1) {
            int y = __shfl_up(x, o);
            if (lane >= o) x += y;
        }
        if (lane == kWave - 1) wsum[wv] = x;
        __syncthreads();
        if (wv == 0) {
            int s = lane < 16 ? wsum[lane] : 0;
            for (int o = 1; o < 16; o <<= 1) {
                int y = __shfl_up(s, o);
                if (lane >= o) s += y;
            }
            if (lane < 16) wsum[lane] = s;
        }
        __syncthreads();
        int excl = x - v + (wv > 0 ? wsum[wv - 1] : 0) + carry;
        if (idx < ncell) st.cell_start[idx] = excl;
        int total = wsum[15];
        __syncthreads();
        carry += total;
    }
    if (tid == 0) st.cell_start[ncell] = carry;
}

// Resort views of the scratch region (one copy of every per-particle array).
struct ResortView {
    double4 *rec64, *vel64;
    int4 *recq;
    float4 *pos_hi, *pos_lo, *vel_hi, *vel_lo;
    int4 *img;
    int32_t *id;
};

__host__ __device__ inline ResortView resort_view(uint8_t *base, int64_t npad, int prec) {
    ResortView v{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        uint8_t *p = base + off;
        off += (bytes + 255) & ~(size_t)255;
        return p;
    };
    if (prec == LJMD_FP64) {
        v.rec64 = (double4 *)take(sizeof(double4) * npad);
        v.vel64 = (double4 *)take(sizeof(double4) * npad);
    } else {
        v.recq = (int4 *)take(sizeof(int4) * npad);
        v.pos_hi = (float4 *)take(sizeof(float4) * npad);
        v.pos_lo = (float4 *)take(sizeof(float4) * npad);
        v.vel_hi = (float4 *)take(sizeof(float4) * npad);
        v.vel_lo = (float4 *)take(sizeof(float4) * npad);
    }
    v.img = (int4 *)take(sizeof(int4) * npad);
    v.id = (int32_t *)take(sizeof(int32_t) * npad);
    return v;
}

size_t resort_scratch_bytes(int64_t npad, int prec) {
    auto r = [](size_t b) { return (b + 255) & ~(size_t)255; };
    size_t s = prec == LJMD_FP64 ? 2 * r(sizeof(double4) * npad) : 5 * r(sizeof(float4) * npad);
    return s + r(sizeof(int4) * npad) + r(sizeof(int32_t) * npad);
}

// Gather every per-particle array into scratch in (cell rank, slot) order and
// rewrite the cell members with their new slots. One thread per cell slot.
template <int PREC>
__global__ __launch_bounds__(kBlock) void k_resort_gather(State st, Geom g, BoxC box, int cur,
                                                          ResortView sv) {
    int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    int64_t c = t / g.cell_cap;
    int k = (int)(t - c * g.cell_cap);
    if (c >= box.ncell) return;
    int cnt = st.cell_count[c];
    int m = cnt < g.cell_cap ? cnt : g.cell_cap;
    if (k >= m) return;
    int64_t slot = c * g.cell_cap + k;
    int i = st.cell_members[slot];
    int s = st.cell_start[c] + k;
    if constexpr (PREC == LJMD_FP64) {
        sv.rec64[s] = st.rec64[cur][i];
        sv.vel64[s] = st.vel64[i];
    } else {
        sv.recq[s] = st.recq[cur][i];
        sv.pos_hi[s] = st.pos_hi[i];
        sv.pos_lo[s] = st.pos_lo[i];
        sv.vel_hi[s] = st.vel_hi[i];
        sv.vel_lo[s] = st.vel_lo[i];
    }
    sv.img[s] = st.img[i];
    sv.id[s] = st.id[i];
    st.cell_members[slot] = s;
}

template <int PREC>
__global__ __launch_bounds__(kBlock) void k_resort_copy(State st, Geom g, int cur, ResortView sv) {
    int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (s >= g.n) return;
    if constexpr (PREC == LJMD_FP64) {
        st.rec64[cur][s] = sv.rec64[s];
        st.vel64[s] = sv.vel64[s];
    } else {
        st.recq[cur][s] = sv.recq[s];
        st.pos_hi[s] = sv.pos_hi[s];
        st.pos_lo[s] = sv.pos_lo[s];
        st.vel_hi[s] = sv.vel_hi[s];
        st.vel_lo[s] = sv.vel_lo[s];
    }
    st.img[s] = sv.img[s];
    st.id[s] = sv.id[s];
}

// Pair-type constant by symmetric type t = a + b.
template <int NS, class T>
__device__ inline T by_type(int t, const T (&a)[3]) {
    if constexpr (NS == 1) {
        return a[0];
    } else {
        return t == 0 ? a[0] : (t == 1 ? a[1] : a[2]);
    }
}

// Verlet lists, one wavefront per home cell. Candidates are the particle
// slots of the (up to 27 distinct) surrounding cells taken cell by cell in a
// fixed stencil order (x outer, z inner), each cell's slots ascending
// (binning leaves them in atomic order; a rank count in LDS sorts them).
// The wave stages whole stencil cells into LDS in groups that fit kStage
// (all member loads of a group in flight together, so a cell costs a few
// memory latencies, not one per neighbour cell) and sweeps each group: a
// home particle gets G = 64/m lanes (m = home occupancy) that take four
// G-wide runs of candidates per trip, record gathers in flight together, so
// the whole wave touches only 4G records per trip. Hits (j != i and
// r_ij^2 < (r_c + skin)^2 under the stated sequence of the precision) are
// compacted with ballots and written in candidate order: the list order
// depends neither on G nor on the grouping and is reproducible.
constexpr int kStage = 1024;
constexpr int kNlistWaves = 4;

// Stage the slots of stencil cells [s0, s1) (tot slots; lane s of the wave
// holds cell id scell, count scnt and prefix offset soff of stencil cell s)
// into dst, each cell's slots ascending. Wave-uniform control flow: every
// lane executes every shuffle; only memory accesses are predicated.
__device__ inline void stage_cells(const State &st, const Geom &g, int lane, int s0, int s1, int tot,
                                   int scell, int scnt, int soff, int32_t *sraw, int32_t *dst) {
    const int base_off = __shfl(soff, s0);
    for (int b = 0; b < tot; b += kWave) {
        const int t = b + lane, tg = base_off + t;
        int sel = s0;
        for (int s = s0 + 1; s < s1; ++s) sel = __shfl(soff, s) <= tg ? s : sel;
        const int cs = __shfl(scell, sel), os = __shfl(soff, sel) - base_off;
        if (t < tot) {
            int v = st.cell_members[(int64_t)cs * g.cell_cap + (t - os)];
            // A slot outside [0, n) would mean corrupted cell data: replace it
            // and report, so that no later gather can leave the arrays.
            if ((unsigned)v >= (unsigned)g.n) {
                v = 0;
                atomicOr(&st.ctl->flags, kErrCell);
            }
            sraw[t] = v;
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    for (int b = 0; b < tot; b += kWave) {
        const int t = b + lane, tg = base_off + t;
        int sel = s0;
        for (int s = s0 + 1; s < s1; ++s) sel = __shfl(soff, s) <= tg ? s : sel;
        const int os = __shfl(soff, sel) - base_off, ms = __shfl(scnt, sel);
        if (t < tot) {
            const int v = sraw[t];
            int r = 0;
            for (int k = 0; k < ms; ++k) r += sraw[os + k] < v ? 1 : 0;
            dst[os + (r < ms ? r : ms - 1)] = v;
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

template <int PREC, int NS>
__global__ __launch_bounds__(kWave * kNlistWaves) void k_nlist_cell(
    State st, Geom g, BoxC box, PairC pc, int cur, int64_t step, int forced, float thr2,
    int cells_per_wave) {
    if (!rebuild_due(st.ctl, step, forced, thr2)) return;
    if (blockIdx.x == 0 && threadIdx.x == 0) st.ctl->rebuilds += 1;
    extern __shared__ int32_t lds[];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int32_t *sraw = lds + (size_t)wv * (2 * kStage + g.cell_cap);
    int32_t *sidx = sraw + kStage;
    int32_t *shome = sidx + kStage;
    const int blk = xcd_remap(blockIdx.x, gridDim.x);
    const int cbeg = (blk * kNlistWaves + wv) * cells_per_wave;
    const int cend = min(cbeg + cells_per_wave, box.ncell);
    int wave_max = 0;
    for (int c = cbeg; c < cend; ++c) {
        const int lin = st.cell_lin[c];
        const int cc[3] = {lin / (box.nc[1] * box.nc[2]), (lin / box.nc[2]) % box.nc[1],
                           lin % box.nc[2]};
        int lo[3], n3[3];
        for (int a = 0; a < 3; ++a) {
            if (box.nc[a] >= 3) {
                lo[a] = -1;
                n3[a] = 3;
            } else {
                lo[a] = -cc[a];
                n3[a] = box.nc[a];
            }
        }
        const int nst = n3[0] * n3[1] * n3[2];
        int scell = 0, scnt = 0;
        if (lane < nst) {
            const int a = lane / (n3[1] * n3[2]), b = (lane / n3[2]) % n3[1], d = lane % n3[2];
            int ax = cc[0] + lo[0] + a, ay = cc[1] + lo[1] + b, az = cc[2] + lo[2] + d;
            ax += ax < 0 ? box.nc[0] : (ax >= box.nc[0] ? -box.nc[0] : 0);
            ay += ay < 0 ? box.nc[1] : (ay >= box.nc[1] ? -box.nc[1] : 0);
            az += az < 0 ? box.nc[2] : (az >= box.nc[2] ? -box.nc[2] : 0);
            scell = st.rank_of[(ax * box.nc[1] + ay) * box.nc[2] + az];
            scnt = min(st.cell_count[scell], g.cell_cap);
        }
        int incl = scnt;
        for (int o = 1; o < kWave; o <<= 1) {
            const int y = __shfl_up(incl, o);
            if (lane >= o) incl += y;
        }
        const int soff = incl - scnt;
        const int home_s = ((-lo[0]) * n3[1] + (-lo[1])) * n3[2] + (-lo[2]);
        const int m = __shfl(scnt, home_s);
        if (m == 0) continue;
        stage_cells(st, g, lane, home_s, home_s + 1, m, scell, scnt, soff, sraw, shome);

        const int G = m >= kWave ? 1 : kWave / m;
        const int P = kWave / G;
        const int p_local = lane / G, gl = lane % G;
        const unsigned long long gbits = G >= 64 ? ~0ull : ((1ull << G) - 1ull);
        const unsigned long long below = (1ull << gl) - 1ull;
        constexpr int U = 4;
        for (int pb = 0; pb < m; pb += P) {
            const int p = pb + p_local;
            const bool active = p_local < P && p < m;
            int i = 0, si = 0;
            uint32_t qi[3] = {0, 0, 0};
            double xi[3] = {0, 0, 0};
            if (active) {
                i = shome[p];
                if constexpr (PREC == LJMD_FP64) {
                    const double4 r = st.rec64[cur][i];
                    xi[0] = r.x;
                    xi[1] = r.y;
                    xi[2] = r.z;
                    si = (int)r.w;
                } else {
                    const int4 r = st.recq[cur][i];
                    qi[0] = (uint32_t)r.x;
                    qi[1] = (uint32_t)r.y;
                    qi[2] = (uint32_t)r.z;
                    si = r.w;
                }
            }
            int k = 0;
            for (int s0 = 0; s0 < nst;) {
                // Next group of whole stencil cells that fits the stage.
                int s1 = s0, tot = 0;
                while (s1 < nst) {
                    const int cn = __shfl(scnt, s1);
                    if (tot + cn > kStage) break;
                    tot += cn;
                    ++s1;
                }
                if (s1 == s0) {  // unreachable: cell_cap <= kStage; guarantees progress
                    if (lane == 0) atomicOr(&st.ctl->flags, kErrCell);
                    s1 = s0 + 1;
                    tot = 0;
                }
                stage_cells(st, g, lane, s0, s1, tot, scell, scnt, soff, sraw, sidx);
                for (int base = 0; base < tot; base += U * G) {
                    int jj[U];
                    bool ok[U];
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        const int t = base + u * G + gl;
                        ok[u] = active && t < tot;
                        jj[u] = sidx[ok[u] ? t : 0];
                        ok[u] = ok[u] && jj[u] != i;
                    }
                    bool in[U];
                    if constexpr (PREC == LJMD_FP64) {
                        double4 rj[U];
#pragma unroll
                        for (int u = 0; u < U; ++u) rj[u] = st.rec64[cur][jj[u]];
#pragma unroll
                        for (int u = 0; u < U; ++u) {
                            const int tt = NS == 1 ? 0 : si + (int)rj[u].w;
                            const double dx = disp_d(xi[0], rj[u].x, box.L[0], box.invL[0]);
                            const double dy = disp_d(xi[1], rj[u].y, box.L[1], box.invL[1]);
                            const double dz = disp_d(xi[2], rj[u].z, box.L[2], box.invL[2]);
                            const double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
                            in[u] = ok[u] && r2 < by_type<NS>(tt, pc.rl2);
                        }
                    } else {
                        int4 rj[U];
#pragma unroll
                        for (int u = 0; u < U; ++u) rj[u] = st.recq[cur][jj[u]];
#pragma unroll
                        for (int u = 0; u < U; ++u) {
                            const int tt = NS == 1 ? 0 : si + rj[u].w;
                            const float dx = disp_q(qi[0], (uint32_t)rj[u].x, box.qs_hi[0], box.qs_lo[0]);
                            const float dy = disp_q(qi[1], (uint32_t)rj[u].y, box.qs_hi[1], box.qs_lo[1]);
                            const float dz = disp_q(qi[2], (uint32_t)rj[u].z, box.qs_hi[2], box.qs_lo[2]);
                            const float r2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
                            in[u] = ok[u] && r2 < by_type<NS>(tt, pc.rl2f);
                        }
                    }
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        const unsigned long long mask = __ballot(in[u] ? 1 : 0);
                        const unsigned long long grp = (mask >> (lane - gl)) & gbits;
                        const int pos = __popcll(grp & below);
                        if (in[u] && k + pos < g.cap) st.nbr[nbr_index(i, k + pos, g.lanes, g.cap)] = jj[u];
                        k += __popcll(grp);
                    }
                }
                s0 = s1;
            }
            if (active && gl == 0) {
                st.nbr_cnt[i] = k;
                if constexpr (PREC == LJMD_FP64)
                    st.xref[i] = make_int4((int)q_from_d(xi[0], box.S[0]), (int)q_from_d(xi[1], box.S[1]),
                                           (int)q_from_d(xi[2], box.S[2]), 0);
                else
                    st.xref[i] = make_int4((int)qi[0], (int)qi[1], (int)qi[2], 0);
                if (k > g.cap) atomicOr(&st.ctl->flags, kErrList);
            }
            wave_max = active && k > wave_max ? k : wave_max;
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        const int y = __shfl_xor(wave_max, o);
        wave_max = y > wave_max ? y : wave_max;
    }
    if (lane == 0 && wave_max > 0 && wave_max > *(volatile int32_t *)&st.ctl->max_fill)
        atomicMax(&st.ctl->max_fill, wave_max);
}

// ------------------------------------------------------------------------
constexpr int kNlistBlocks = 1024;
static inline unsigned blocks_for(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

hipError_t launch_bin(const Launch &L, int64_t step, int forced) {
    unsigned nb = blocks_for(L.g->n, kBlock);
    if (L.g->prec == LJMD_FP64)
        hipLaunchKernelGGL(k_bin<LJMD_FP64>, dim3(nb), dim3(kBlock), 0, L.stream, *L.st, *L.g,
                           *L.box, L.cur, step, forced, L.dyn->thr2);
    else
        hipLaunchKernelGGL(k_bin<LJMD_FP32_DS>, dim3(nb), dim3(kBlock), 0, L.stream, *L.st, *L.g,
                           *L.box, L.cur, step, forced, L.dyn->thr2);
    return hipGetLastError();
}

hipError_t launch_canon(const Launch &L, int64_t step, int forced) {
    const int wpb = kBlock / kWave;
    unsigned nb = blocks_for(L.box->ncell, wpb);
    size_t shm = (size_t)wpb * 2 * L.g->cell_cap * sizeof(int32_t);
    hipLaunchKernelGGL(k_canon, dim3(nb), dim3(kBlock), shm, L.stream, *L.st, *L.g, *L.box, step,
                       forced, L.dyn->thr2);
    return hipGetLastError();
}

hipError_t launch_resort(const Launch &L) {
    int64_t npad = (L.g->n + 63) / 64 * 64;
    ResortView sv = resort_view(L.st->scratch, npad, L.g->prec);
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, L.stream, *L.st, *L.g, L.box->ncell);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    unsigned nb = blocks_for((int64_t)L.box->ncell * L.g->cell_cap, kBlock);
    unsigned nc = blocks_for(L.g->n, kBlock);
    if (L.g->prec == LJMD_FP64) {
        hipLaunchKernelGGL(k_resort_gather<LJMD_FP64>, dim3(nb), dim3(kBlock), 0, L.stream, *L.st,
                           *L.g, *L.box, L.cur, sv);
        hipLaunchKernelGGL(k_resort_copy<LJMD_FP64>, dim3(nc), dim3(kBlock), 0, L.stream, *L.st,
                           *L.g, L.cur, sv);
    } else {
        hipLaunchKernelGGL(k_resort_gather<LJMD_FP32_DS>, dim3(nb), dim3(kBlock), 0, L.stream,
                           *L.st, *L.g, *L.box, L.cur, sv);
        hipLaunchKernelGGL(k_resort_copy<LJMD_FP32_DS>, dim3(nc), dim3(kBlock), 0, L.stream, *L.st,
                           *L.g, L.cur, sv);
    }
    return hipGetLastError();
}

hipError_t launch_nlist(const Launch &L, int64_t step, int forced) {
    // Contiguous runs of Hilbert-ranked cells per wave; at most kNlistBlocks
    // blocks so that the launch stays cheap on steps without a rebuild.
    const int ncell = L.box->ncell;
    const int nwaves_max = kNlistBlocks * kNlistWaves;
    const int per = (ncell + nwaves_max - 1) / nwaves_max;
    const int nwaves = (ncell + per - 1) / per;
    const unsigned grid = (unsigned)((nwaves + kNlistWaves - 1) / kNlistWaves);
    const size_t shm = (size_t)kNlistWaves * (2 * kStage + L.g->cell_cap) * sizeof(int32_t);
#define NL(P, S)                                                                              \
    hipLaunchKernelGGL((k_nlist_cell<P, S>), dim3(grid), dim3(kWave * kNlistWaves), shm,      \
                       L.stream, *L.st, *L.g, *L.box, *L.pc, L.cur, step, forced, L.dyn->thr2, per)
    if (L.g->prec == LJMD_FP64) {
        if (L.g->nspecies == 1) NL(LJMD_FP64, 1); else NL(LJMD_FP64, 2);
    } else {
        if (L.g->nspecies == 1) NL(LJMD_FP32_DS, 1); else NL(LJMD_FP32_DS, 2);
    }
#undef NL
    return hipGetLastError();
}

}  // namespace ljmd
