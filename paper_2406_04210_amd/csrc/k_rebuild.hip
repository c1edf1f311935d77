// k_rebuild.hip -- neighbour-list rebuild on gfx950: particle binning,
// canonical cell order, space-filling-curve resort and Verlet-list build
// (paper Sec. 3 "Code structure": Verlet lists built from particle binning;
// Sec. 4 "Mixed Strategy": sorting).
//
// Cells are indexed by the Hilbert rank of their position in the cell grid.
// A cell slot holds a particle's whole record -- its position record plus
// its index and species packed in the last word -- so that the list build
// reads every candidate with one contiguous 16-byte (FP32) or 32-byte (FP64)
// load instead of an index load followed by a dependent gather.
//
// bin, canon and nlist are launched every step and return at once unless
// the list is due (host-forced, or the largest displacement since the last
// build exceeded half the skin -- paper Sec. 5: more movement, more list
// updates). The decision reads one control word written by the previous
// step's kernel, so no host synchronisation is needed per step.
#include "batch.h"
#include "internal.h"

namespace ljmd {

// Binning and cell canonicalisation run as one or two 1024-thread blocks per
// compute unit and stride over their work (see rebuild_blocks): only a few
// hundred workgroups to retire when no rebuild is due.
constexpr int kRbBlock = 1024;

__host__ __device__ inline size_t canon_lds_per_wave(int cell_cap, size_t rec_bytes) {
    return (((size_t)cell_cap * (rec_bytes + sizeof(int32_t))) + 15) & ~(size_t)15;
}

// Cell-slot records: (position record, (index << 1) | species).
template <int PREC>
struct CellRec;
template <>
struct CellRec<LJMD_FP64> {
    using T = double4;
    __device__ static T pack(const double4 &r, int i) {
        return make_double4(r.x, r.y, r.z, (double)((i << 1) | ((int)r.w & 1)));
    }
    __device__ static int index(const T &c) { return ((int)c.w) >> 1; }
    __device__ static int species(const T &c) { return ((int)c.w) & 1; }
    __device__ static T with_index(const T &c, int i) {
        return make_double4(c.x, c.y, c.z, (double)((i << 1) | species(c)));
    }
};
template <>
struct CellRec<LJMD_FP32_DS> {
    using T = int4;
    __device__ static T pack(const int4 &r, int i) { return make_int4(r.x, r.y, r.z, (i << 1) | (r.w & 1)); }
    __device__ static int index(const T &c) { return (int)((uint32_t)c.w >> 1); }
    __device__ static int species(const T &c) { return c.w & 1; }
    __device__ static T with_index(const T &c, int i) {
        return make_int4(c.x, c.y, c.z, (i << 1) | species(c));
    }
};

template <int PREC>
__device__ inline typename CellRec<PREC>::T *cell_recs(const State &st) {
    return (typename CellRec<PREC>::T *)st.cell_rec;
}

// Fixed-point coordinates of a position record.
__device__ inline void rec_q(const double4 &r, const BoxC &box, uint32_t *q) {
    q[0] = q_from_d(r.x, box.S[0]);
    q[1] = q_from_d(r.y, box.S[1]);
    q[2] = q_from_d(r.z, box.S[2]);
}
__device__ inline void rec_q(const int4 &r, const BoxC &, uint32_t *q) {
    q[0] = (uint32_t)r.x;
    q[1] = (uint32_t)r.y;
    q[2] = (uint32_t)r.z;
}

template <int PREC>
__device__ inline const typename CellRec<PREC>::T *records(const State &st, int cur) {
    if constexpr (PREC == LJMD_FP64)
        return st.rec64[cur];
    else
        return st.recq[cur];
}

// Bin: cell of every particle (from its fixed-point coordinates, so always
// inside the grid), counted with an atomic per cell. The slot a particle
// lands in is arbitrary; k_canon restores a deterministic order.
template <int PREC>
__device__ inline void bin_one(const State &st, const Geom &g, const BoxC &box, const int32_t *rank_of,
                               int64_t c_off, int cur, int64_t i, Ctl *ctl) {
    using CR = CellRec<PREC>;
    const auto r = records<PREC>(st, cur)[i];
    uint32_t q[3];
    rec_q(r, box, q);
    int cx, cy, cz;
    const int64_t c = c_off + cell_of_q(q[0], q[1], q[2], box, rank_of, &cx, &cy, &cz);
    // The lanes of a wavefront that land in one cell take their slots with a
    // single atomic: consecutive particles (space-filling-curve order) share
    // a few cells. The groups and their leaders are found first (ballots
    // only, every active lane runs the same number of rounds); then the
    // leaders' atomics go out together, one memory round trip per wave.
    const int lane = threadIdx.x & 63;
    const int ci = (int)c;
    unsigned long long pending = __ballot(1);
    int leader_of = lane, rank = 0, take = 0;
    while (pending) {
        const int leader = __ffsll(pending) - 1;
        const int cl = __builtin_amdgcn_readlane(ci, leader);
        const unsigned long long same = __ballot(ci == cl);
        if (ci == cl) {
            leader_of = leader;
            rank = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(same >> 32),
                                                  __builtin_amdgcn_mbcnt_lo((uint32_t)same, 0u));
        }
        if (lane == leader) take = __popcll(same);
        pending &= ~same;
    }
    int base = 0;
    if (take > 0) base = atomicAdd(&st.cell_count[ci], take);
    const int slot = __shfl(base, leader_of) + rank;
    if (slot < g.cell_cap)
        cell_recs<PREC>(st)[c * g.cell_cap + slot] = CR::pack(r, (int)i);
    else
        atomicOr(&ctl->flags, kErrCell);
}

template <int PREC>
__global__ __launch_bounds__(kRbBlock) void k_bin(State st, Geom g, BoxC box, int cur, int64_t step,
                                                int forced, float thr2) {
    if (blockIdx.x == 0 && threadIdx.x == 0) st.ctl->maxd[(step + 1) & 1] = 0u;
    if (halted(st.ctl) || !rebuild_due(st.ctl, step, forced, thr2)) return;
    if (blockIdx.x == 0 && threadIdx.x < 8) st.ctl->nlq[threadIdx.x] = 0u;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < g.n; i += stride)
        bin_one<PREC>(st, g, box, st.rank_of, 0, cur, i, st.ctl);
}

// Canonicalise: one wavefront per cell sorts the cell's slots by particle
// index (distinct keys, rank counting in LDS), so that list order and hence
// force summation order are reproducible run to run.
template <int PREC>
__device__ inline void canon_cell(const State &st, const Geom &g, int64_t c, typename CellRec<PREC>::T *tmp,
                                  int32_t *key) {
    using CR = CellRec<PREC>;
    using T = typename CR::T;
    const int lane = threadIdx.x & 63;
    const int cnt = st.cell_count[c];
    const int m = cnt < g.cell_cap ? cnt : g.cell_cap;
    T *mem = cell_recs<PREC>(st) + c * g.cell_cap;
    for (int e = lane; e < m; e += kWave) key[e] = CR::index(mem[e]);
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    for (int e = lane; e < m; e += kWave) {
        const int v = key[e];
        int r = 0;
        for (int k = 0; k < m; ++k) r += key[k] < v ? 1 : 0;
        tmp[r < m ? r : m - 1] = mem[e];
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    for (int e = lane; e < m; e += kWave) mem[e] = tmp[e];
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

template <int PREC>
__global__ __launch_bounds__(kRbBlock) void k_canon(State st, Geom g, BoxC box, int64_t step,
                                                 int forced, float thr2) {
    if (halted(st.ctl) || !rebuild_due(st.ctl, step, forced, thr2)) return;
    using T = typename CellRec<PREC>::T;
    extern __shared__ int4 sm_raw[];
    const int wv = threadIdx.x >> 6, W = blockDim.x >> 6;
    T *tmp = (T *)((uint8_t *)sm_raw + (size_t)wv * canon_lds_per_wave(g.cell_cap, sizeof(T)));
    int32_t *key = (int32_t *)(tmp + g.cell_cap);
    for (int c = blockIdx.x * W + wv; c < box.ncell; c += gridDim.x * W) canon_cell<PREC>(st, g, c, tmp, key);
}

// Exclusive scan of the (capped) cell counts in Hilbert-rank order: the
// start of every cell in the resorted particle order. One block.
// Exclusive scan of the capped counts of cells [c_off, c_off + ncell) into
// cell_start, offset by `base` (one 1024-thread block).
__device__ inline void scan_cells(const State &st, const Geom &g, int64_t c_off, int ncell, int64_t base_slot) {
    __shared__ int32_t wsum[16];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    int32_t carry = 0;
    for (int base = 0; base < ncell; base += 1024) {
        const int idx = base + tid;
        int v = 0;
        if (idx < ncell) {
            v = st.cell_count[c_off + idx];
            v = v < g.cell_cap ? v : g.cell_cap;
        }
        int x = v;
        for (int o = 1; o < kWave; o <<= 1) {
            const int y = __shfl_up(x, o);
            if (lane >= o) x += y;
        }
        if (lane == kWave - 1) wsum[wv] = x;
        __syncthreads();
        if (wv == 0) {
            int s = lane < 16 ? wsum[lane] : 0;
            for (int o = 1; o < 16; o <<= 1) {
                const int y = __shfl_up(s, o);
                if (lane >= o) s += y;
            }
            if (lane < 16) wsum[lane] = s;
        }
        __syncthreads();
        const int excl = x - v + (wv > 0 ? wsum[wv - 1] : 0) + carry;
        if (idx < ncell) st.cell_start[c_off + idx] = (int32_t)(base_slot + excl);
        const int total = wsum[15];
        __syncthreads();
        carry += total;
    }
}

__global__ __launch_bounds__(1024) void k_scan(State st, Geom g, int ncell) {
    if (halted(st.ctl)) return;
    scan_cells(st, g, 0, ncell, 0);
}

// Resort views of the scratch region (one copy of every per-particle array).
struct ResortView {
    double4 *rec64, *vel64;
    int4 *recq;
    float4 *dsw[3];
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
        for (int k = 0; k < 3; ++k) v.dsw[k] = (float4 *)take(sizeof(float4) * npad);
    }
    v.img = (int4 *)take(sizeof(int4) * npad);
    v.id = (int32_t *)take(sizeof(int32_t) * npad);
    return v;
}

size_t resort_scratch_bytes(int64_t npad, int prec) {
    auto r = [](size_t b) { return (b + 255) & ~(size_t)255; };
    size_t s = prec == LJMD_FP64 ? 2 * r(sizeof(double4) * npad) : 4 * r(sizeof(float4) * npad);
    return s + r(sizeof(int4) * npad) + r(sizeof(int32_t) * npad);
}

size_t cell_rec_bytes(int prec) { return prec == LJMD_FP64 ? sizeof(double4) : sizeof(int4); }

// Gather every per-particle array into scratch in (cell rank, slot) order and
// give each cell slot the particle's new index. One thread per cell slot.
template <int PREC>
__global__ __launch_bounds__(kBlock) void k_resort_gather(State st, Geom g, BoxC box, int cur,
                                                          ResortView sv) {
    using CR = CellRec<PREC>;
    if (halted(st.ctl)) return;
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int64_t c = t / g.cell_cap;
    const int k = (int)(t - c * g.cell_cap);
    if (c >= box.ncell) return;
    const int cnt = st.cell_count[c];
    const int m = cnt < g.cell_cap ? cnt : g.cell_cap;
    if (k >= m) return;
    auto *cr = cell_recs<PREC>(st);
    const int64_t slot = c * g.cell_cap + k;
    const auto rc = cr[slot];
    const int i = CR::index(rc);
    const int s = st.cell_start[c] + k;
    if ((unsigned)i >= (unsigned)g.n || (unsigned)s >= (unsigned)g.n) {
        atomicOr(&st.ctl->flags, kErrCell);
        return;
    }
    if constexpr (PREC == LJMD_FP64) {
        sv.rec64[s] = st.rec64[cur][i];
        sv.vel64[s] = st.vel64[i];
    } else {
        sv.recq[s] = st.recq[cur][i];
        for (int w = 0; w < 3; ++w) sv.dsw[w][s] = st.dsw[w][i];
    }
    sv.img[s] = st.img[i];
    sv.id[s] = st.id[i];
    cr[slot] = CR::with_index(rc, s);
}

template <int PREC>
__global__ __launch_bounds__(kBlock) void k_resort_copy(State st, Geom g, int cur, ResortView sv) {
    const int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (s >= g.n || halted(st.ctl)) return;
    if constexpr (PREC == LJMD_FP64) {
        st.rec64[cur][s] = sv.rec64[s];
        st.vel64[s] = sv.vel64[s];
    } else {
        st.recq[cur][s] = sv.recq[s];
        for (int w = 0; w < 3; ++w) st.dsw[w][s] = sv.dsw[w][s];
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
        return (t & 2) ? a[2] : ((t & 1) ? a[1] : a[0]);  // t in {0, 1, 2}
    }
}

// r^2 of a candidate under the stated sequence of each precision.
__device__ inline double cand_r2(const double4 &ri, const double4 &rj, const BoxC &box) {
    const double dx = disp_d(ri.x, rj.x, box.L[0], box.invL[0]);
    const double dy = disp_d(ri.y, rj.y, box.L[1], box.invL[1]);
    const double dz = disp_d(ri.z, rj.z, box.L[2], box.invL[2]);
    return fma(dz, dz, fma(dy, dy, dx * dx));
}
__device__ inline float cand_r2(const int4 &ri, const int4 &rj, const BoxC &box) {
    const float dx = (float)(int32_t)((uint32_t)ri.x - (uint32_t)rj.x) * box.qs_hi[0];
    const float dy = (float)(int32_t)((uint32_t)ri.y - (uint32_t)rj.y) * box.qs_hi[1];
    const float dz = (float)(int32_t)((uint32_t)ri.z - (uint32_t)rj.z) * box.qs_hi[2];
    return fmaf(dz, dz, fmaf(dy, dy, dx * dx));
}
// Cubic boxes: r^2 in squared quanta from the raw wrapped differences.
__device__ inline float cand_r2q(const int4 &ri, const int4 &rj) {
    const float dx = (float)(int32_t)((uint32_t)ri.x - (uint32_t)rj.x);
    const float dy = (float)(int32_t)((uint32_t)ri.y - (uint32_t)rj.y);
    const float dz = (float)(int32_t)((uint32_t)ri.z - (uint32_t)rj.z);
    return fmaf(dz, dz, fmaf(dy, dy, dx * dx));
}

// Verlet lists, candidate-major: one wavefront per home cell. The
// candidates are the slots of the (up to 27 distinct) cells around the home
// cell, taken cell by cell in a fixed stencil order (x outer, z inner), each
// cell's slots ascending by index (canonicalised). The lanes hold 64
// consecutive candidates each (CH blocks in registers, loaded once per
// cell); the wave then loops over the home particles, every lane testing its
// candidates against the same particle (r_ij^2 < (r_c + skin)^2 under the
// stated sequence of the precision, j != i), and a ballot compacts the hits
// into the particle's list in candidate order. No lane ever idles on a
// shorter loop than its neighbours, and the list order is reproducible.
//
// The home particles (up to 64 at a time) and their running list lengths
// live in registers, one per lane; the loop over them reads both with
// readlane, so the inner loop needs no LDS traffic and no wave barrier,
// and the list stores are never waited on.
template <int PREC, bool FILT = false>
struct NlistChunk {
    // 64-candidate blocks per chunk (FILT: blocks loaded per round and per
    // queue drain; six keep the kernel within 96 VGPRs, five waves per SIMD,
    // and its two queues within 6 KiB of LDS per wave)
    static constexpr int CH = FILT ? 6 : (PREC == LJMD_FP64 ? 4 : 8);
};

// Waves per list-build block, and blocks per compute unit: with up to
// 8 cells per wave of a grid of kNlBlocksPerCu blocks per compute unit,
// each wave takes a contiguous run of cells (measured at N = 256,000: one
// cell per wave over 12 blocks per compute unit, 52.3 ms per 1000 steps,
// against 54.8 ms with three cells per wave over 5); larger grids of cells
// go through the per-XCD queues with kNlQueueBlocksPerCu blocks per compute
// unit, the five waves per SIMD that fit at once (the 4M mixture 3.99e9 ->
// 4.01e9 and the 512-replica batch 4.22e9 -> 4.33e9 particle-steps/s
// against 12).
constexpr int kNlWaves = 4;
constexpr int kNlBlocksPerCu = 12;
constexpr int kNlQueueBlocksPerCu = 5;

__device__ inline int lane_read(int v, int p) { return __builtin_amdgcn_readlane(v, p); }
__device__ inline int4 lane_read(const int4 &v, int p) {
    return make_int4(lane_read(v.x, p), lane_read(v.y, p), lane_read(v.z, p), lane_read(v.w, p));
}
__device__ inline double lane_read(double v, int p) {
    const long long b = __double_as_longlong(v);
    const unsigned lo = (unsigned)lane_read((int)(b & 0xffffffffll), p);
    const unsigned hi = (unsigned)lane_read((int)(b >> 32), p);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
__device__ inline double4 lane_read(const double4 &v, int p) {
    return make_double4(lane_read(v.x, p), lane_read(v.y, p), lane_read(v.z, p), lane_read(v.w, p));
}

// Smallest wrapped distance, in quanta along one axis, from coordinate q to
// any coordinate of [mn, mn + span] (the wrapped difference of two
// coordinates is their minimum-image displacement).
__device__ inline uint32_t gap_q(uint32_t q, uint32_t mn, uint32_t span) {
    const uint32_t t = q - mn;
    const uint32_t a = t - span, b = 0u - t;
    return t <= span ? 0u : (a < b ? a : b);
}

// Unsigned minimum (MAX false) or maximum over the wavefront, complete in
// lane 63, by DPP row moves instead of LDS permutes (every lane active):
// lane pairs and quads, half-row and row mirrors, then row broadcasts; a
// lane of a row that a broadcast does not write reads the identity.
template <int CTRL, int ROWM, bool MAX>
__device__ inline uint32_t dpp_ext(uint32_t v) {
    const uint32_t w = (uint32_t)__builtin_amdgcn_update_dpp(MAX ? 0 : -1, (int)v, CTRL, ROWM, 0xf, false);
    return MAX ? (w > v ? w : v) : (w < v ? w : v);
}
template <bool MAX>
__device__ inline uint32_t wave_ext_last(uint32_t v) {
    v = dpp_ext<0xb1, 0xf, MAX>(v);
    v = dpp_ext<0x4e, 0xf, MAX>(v);
    v = dpp_ext<0x141, 0xf, MAX>(v);
    v = dpp_ext<0x140, 0xf, MAX>(v);
    v = dpp_ext<0x142, 0xa, MAX>(v);
    v = dpp_ext<0x143, 0xc, MAX>(v);
    return v;
}
__device__ inline uint32_t wave_min_u32(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_readlane((int)wave_ext_last<false>(v), 63);
}
__device__ inline uint32_t wave_max_u32(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_readlane((int)wave_ext_last<true>(v), 63);
}

// Tests the candidate blocks cand[0 .. nbk) (lane e of block b holds one
// candidate; cv marks the real ones, thr / thr1 their FP32 bounds) against
// every home particle of the lanes in `homes` (lane p holds home record hrec
// and its list length so far in kreg) and appends the hits to the
// particles' lists in candidate order.
template <int PREC, int NS, bool QC, int LG, int CH>
__device__ inline void nlist_homes(const State &st, const Geom &g, const BoxC &box, const PairC &pc,
                                   const typename CellRec<PREC>::T &hrec, int &kreg, uint64_t homes,
                                   const typename CellRec<PREC>::T (&cand)[CH], const bool (&cv)[CH],
                                   const uint32_t (&thr)[CH], const uint32_t (&thr1)[CH], int nbk) {
    using CR = CellRec<PREC>;
    using T = typename CR::T;
    const int lane = threadIdx.x & 63;
    const int lg = LG >= 0 ? LG : (g.lanes >= 16 ? 4 : (g.lanes >= 8 ? 3 : (g.lanes >= 4 ? 2 : (g.lanes >= 2 ? 1 : 0))));
    const int lanes = LG >= 0 ? (1 << LG) : g.lanes;
    // The two-lane store table (below), held in scalar registers and opaque
    // to the compiler, so that the merge stays a single bit-field insert.
    uint64_t g4tab = 0x1C0C180814041000ull;
    asm volatile("" : "+s"(g4tab));
    for (uint64_t mk = homes; mk != 0ull; mk &= mk - 1ull) {
        const int p = __builtin_ctzll(mk);
        const T ri = lane_read(hrec, p);
        const int i = CR::index(ri);
        if ((unsigned)i >= (unsigned)g.n) continue;
        const int si = CR::species(ri);
        int k = lane_read(kreg, p);
        // Entry kk of particle i: lane kk % lanes, its entry m = kk / lanes
        // at row[(m / 4) * 256 + (kk % lanes) * 4 + m % 4], addressed by a
        // 32-bit byte offset from the particle's row.
        uint8_t *__restrict__ row = (uint8_t *)(st.nbr + nbr_index(i, 0, lanes, g.cap));
#pragma unroll
        for (int b = 0; b < CH; ++b) {
            if (b >= nbk) break;
            const int j = CR::index(cand[b]);
            bool hit;
            if constexpr (PREC == LJMD_FP64) {
                const int tt = NS == 1 ? 0 : si + CR::species(cand[b]);
                const double r2 = cand_r2(ri, cand[b], box);
                hit = cv[b] && r2 > 0.0 && r2 < by_type<NS>(tt, pc.rl2);
            } else {
                // 0 < r^2 < r_L^2 as one unsigned compare of the bit
                // patterns (r^2 >= 0); thr[b] is 0 for empty lanes.
                const uint32_t lim = (NS == 2 && si != 0) ? thr1[b] : thr[b];
                const float r2 = QC ? cand_r2q(ri, cand[b]) : cand_r2(ri, cand[b], box);
                hit = __float_as_uint(r2) - 1u < lim;
            }
            const unsigned long long mask = __builtin_amdgcn_ballot_w64(hit);
            // Entries past the capacity land on the last slot: a list that
            // overflows is only counted (its build is flagged and redone
            // with larger lists), and no branch on the count is needed.
            uint32_t kk = __builtin_amdgcn_mbcnt_hi(
                (uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, (uint32_t)k));
            kk = min(kk, (uint32_t)g.cap - 1u);
            k += __popcll(mask);
            uint32_t off;
            if constexpr (LG == 1) {
                // Two lanes: byte (kk / 8) * 1024 + 4 g(kk % 8) with
                // g(r) = 4 (r % 2) + r / 2. Byte r of a 64-bit table holds
                // 4 g(r) (one 64-bit shift by 8 kk, which the hardware takes
                // modulo 64); its bits 0..9 are exactly 4 g(r), since the
                // next byte is a multiple of 4, and they are merged into the
                // group's offset with one bit-field insert.
                const uint32_t g4 = (uint32_t)(g4tab >> ((kk << 3) & 63u));
                off = ((kk << 7) & ~0x3ffu) | (g4 & 0x3ffu);
            } else {
                off = (((kk >> (lg + 2)) << 8) | ((kk & (uint32_t)(lanes - 1)) << 2) |
                       __builtin_amdgcn_ubfe(kk, lg, 2)) << 2;
            }
            if (hit) *(int32_t *)(row + off) = j;
        }
        kreg = lane == p ? k : kreg;
    }
}

// Bit patterns of r_L^2 - 1 ulp for the candidates of a block (0 for empty
// lanes): thr for a home particle of species 0, thr1 of species 1.
template <int PREC, int NS, bool QC>
__device__ inline void nlist_bounds(const BoxC &box, const PairC &pc, const typename CellRec<PREC>::T &cand,
                                    bool cv, uint32_t &thr, uint32_t &thr1) {
    using CR = CellRec<PREC>;
    thr = 0u;
    thr1 = 0u;
    if constexpr (PREC == LJMD_FP32_DS) {
        const float *tab = QC ? box.rl2q : pc.rl2f;
        if constexpr (NS == 1) {
            thr = cv ? __float_as_uint(tab[0]) - 1u : 0u;
        } else {
            const bool sj = CR::species(cand) != 0;  // pair type = home species + sj
            thr = cv ? __float_as_uint(sj ? tab[1] : tab[0]) - 1u : 0u;
            thr1 = cv ? __float_as_uint(sj ? tab[2] : tab[1]) - 1u : 0u;
        }
    }
}

// Candidates per queue of the reduced list build: a chunk of CH blocks is
// appended to queues holding fewer than CH blocks' worth.
template <int CH>
struct NlistQueue {
    static constexpr int kCap = 2 * CH * kWave;
};

// One home cell (local Hilbert rank c of a box whose cells start at c_off in
// the flattened cell arrays; rank_of and cell_lin are that box's tables).
// QC: FP32 criterion of a cubic box, in squared quanta (raw differences
// against r_L^2 / quantum^2).
//
// With QC the home particles are split in two groups at the middle of their
// extent along z, and every candidate is first tested against the bounding
// box of each group: it is dropped for a group when its distance to the box
// (in quanta, per axis the wrapped gap to the box's extent) exceeds r_L with
// a margin of 2^-18 relative, which covers the roundings of both that bound
// and the exact test (a few units of 2^-24 each), so a dropped candidate
// fails the exact test for every home particle of the group. The survivors'
// indices go, in candidate order, to a per-group queue in LDS; whenever a
// queue holds CH blocks' worth (and once more at the end), the wave reloads
// them from the particles' records and runs the exact test for that group's
// home particles only. So the lists are the same entries in the same order
// as without the reduction, while at liquid density the exact test runs
// over about 0.7 of the (particle, block) pairs of a single reduction per
// cell (two smaller boxes, and blocks filled across chunks), at the price of
// a second, cheap test per candidate. rec: the particles' position records,
// the same as the cell slots hold. queue: 2 x NlistQueue<CH>::kCap entries
// of this wave.
// LG: log2 of the lanes per particle of the list layout when it is known at
// compile time (the shifts and masks of the entry index fold), -1 to read it
// from g.lanes. WIDE: the grid has at least 2 R + 2 cells along every axis
// (a compile-time branch, so that the box test's loop carries only the
// bounds of one form).
template <int PREC, int NS, bool QC, int LG, bool WIDE>
__device__ inline void nlist_cell_as(const State &st, const Geom &g, const BoxC &box, const PairC &pc,
                                     const int32_t *rank_of, const int32_t *cell_lin, int64_t c_off, int c,
                                     Ctl *ctl, const typename CellRec<PREC>::T *__restrict__ rec, int32_t *queue) {
    using CR = CellRec<PREC>;
    using T = typename CR::T;
    constexpr bool FILT = PREC == LJMD_FP32_DS && QC;
    constexpr int CH = NlistChunk<PREC, FILT>::CH;
    const int lane = threadIdx.x & 63;
    const T *__restrict__ cr = cell_recs<PREC>(st);
    const int lin = cell_lin[c];
    const int cc[3] = {lin / (box.nc[1] * box.nc[2]), (lin / box.nc[2]) % box.nc[1],
                       lin % box.nc[2]};
    // Stencil: the cells within box.reach cells of the home cell along each
    // axis (3 x 3 x 3 with cells of edge >= r_L, 5 x 5 x 5 with cells of
    // edge >= r_L / 2), or every cell of an axis that has fewer (each cell
    // once). Stencil cells are taken 64 at a time, one per lane.
    const int R = box.reach;
    int lo[3], n3[3];
    for (int a = 0; a < 3; ++a) {
        if (box.nc[a] >= 2 * R + 1) {
            lo[a] = -R;
            n3[a] = 2 * R + 1;
        } else {
            lo[a] = -cc[a];
            n3[a] = box.nc[a];
        }
    }
    const int nst = n3[0] * n3[1] * n3[2];
    const int home = (int)c_off + c;
    const int m = min(st.cell_count[home], g.cell_cap);
    // Largest list radius of any pair type, with the margin of the reduction.
    float reach = 0.0f;
    if constexpr (FILT) {
        reach = box.rl2q[0];
        if constexpr (NS == 2) reach = fmaxf(reach, fmaxf(box.rl2q[1], box.rl2q[2]));
        reach *= 1.0f + 0x1p-18f;
    }
    for (int h0 = 0; h0 < m; h0 += kWave) {
        const int hm = min(m - h0, kWave);
        // Lane e holds home particle h0 + e and the length of its list so far.
        T hrec;
        if (lane < hm) hrec = cr[(int64_t)home * g.cell_cap + h0 + lane];
        else hrec = T{};
        const uint64_t all = hm >= kWave ? ~0ull : ((1ull << hm) - 1ull);
        // FILT: the two groups' lane masks and bounding boxes (wrapped extent
        // per axis: start and span in quanta), their queue fills.
        uint64_t gmask[2] = {all, 0ull};
        uint32_t bmn[2][3] = {{0u, 0u, 0u}, {0u, 0u, 0u}}, bspan[2][3] = {{0u, 0u, 0u}, {0u, 0u, 0u}};
        int fill[2] = {0, 0};
        if constexpr (FILT) {
            const bool act = lane < hm;
            const uint32_t hq[3] = {(uint32_t)hrec.x, (uint32_t)hrec.y, (uint32_t)hrec.z};
            const uint32_t zmn = wave_min_u32(act ? hq[2] : 0xffffffffu);
            const uint32_t zmx = wave_max_u32(act ? hq[2] : 0u);
            const bool up = act && hq[2] - zmn > ((zmx - zmn) >> 1);
            gmask[0] = __ballot(act && !up);
            gmask[1] = __ballot(up);
            for (int gi = 0; gi < 2; ++gi) {
                const bool in = ((gmask[gi] >> lane) & 1ull) != 0ull;
                for (int a = 0; a < 3; ++a) {
                    const uint32_t mn = wave_min_u32(in ? hq[a] : 0xffffffffu);
                    const uint32_t mx = wave_max_u32(in ? hq[a] : 0u);
                    bmn[gi][a] = mn;
                    bspan[gi][a] = mx - mn;
                }
            }
        }
        // An empty group (all home particles at one z) keeps no candidate:
        // its bound is negative.
        const float greach[2] = {reach, gmask[1] != 0ull ? reach : -1.0f};
        // WIDE (along every axis the grid has at least 2 R + 2 cells): every
        // candidate then lies within half a box of the home cell, and the
        // wrapped gap to a group's box is the plain signed one (glo, ghi:
        // the box's extent relative to group 0's corner).
        int32_t glo[2][3], ghi[2][3];
        for (int gi = 0; gi < 2; ++gi)
            for (int a = 0; a < 3; ++a) {
                glo[gi][a] = (int32_t)(bmn[gi][a] - bmn[0][a]);
                ghi[gi][a] = glo[gi][a] + (int32_t)bspan[gi][a];
            }
        int kreg = 0;
        // FILT: test the home particles of group gi against the first cnt
        // queued candidates (cnt <= CH blocks), reloaded from their records.
        auto drain = [&](int gi, int cnt) {
            T cand[CH];
            bool cv[CH];
            uint32_t thr[CH], thr1[CH];
            const int nbk = (cnt + kWave - 1) / kWave;
            const int32_t *qg = queue + gi * NlistQueue<CH>::kCap;
#pragma unroll
            for (int b = 0; b < CH; ++b) {
                cv[b] = false;
                cand[b] = T{};
                thr[b] = thr1[b] = 0u;
                if (b >= nbk) continue;
                const int t = b * kWave + lane;
                cv[b] = t < cnt;
                const int j = cv[b] ? qg[t] : 0;
                if (cv[b]) cand[b] = CR::pack(rec[j], j);
            }
#pragma unroll
            for (int b = 0; b < CH; ++b) {
                if (b >= nbk) break;
                nlist_bounds<PREC, NS, QC>(box, pc, cand[b], cv[b], thr[b], thr1[b]);
            }
            nlist_homes<PREC, NS, QC, LG, CH>(st, g, box, pc, hrec, kreg, gmask[gi], cand, cv, thr, thr1, nbk);
        };
        for (int s0 = 0; s0 < nst; s0 += kWave) {
        // Stencil cells s0 .. s0 + nsp - 1: lane e holds cell s0 + e, its
        // flattened index, its (capped) count and the offset of its first
        // candidate among this part's candidates.
        const int nsp = min(nst - s0, kWave);
        int scell = 0, scnt = 0;
        if (lane < nsp) {
            const int sl = s0 + lane;
            const int a = sl / (n3[1] * n3[2]), bb = (sl / n3[2]) % n3[1], d = sl % n3[2];
            int ax = cc[0] + lo[0] + a, ay = cc[1] + lo[1] + bb, az = cc[2] + lo[2] + d;
            ax += ax < 0 ? box.nc[0] : (ax >= box.nc[0] ? -box.nc[0] : 0);
            ay += ay < 0 ? box.nc[1] : (ay >= box.nc[1] ? -box.nc[1] : 0);
            az += az < 0 ? box.nc[2] : (az >= box.nc[2] ? -box.nc[2] : 0);
            scell = (int)c_off + rank_of[(ax * box.nc[1] + ay) * box.nc[2] + az];
            scnt = min(st.cell_count[scell], g.cell_cap);
        }
        int incl = scnt;
        for (int o = 1; o < kWave; o <<= 1) {
            const int y = __shfl_up(incl, o);
            if (lane >= o) incl += y;
        }
        const int soff = incl - scnt;
        const int ncand = __builtin_amdgcn_readlane(incl, kWave - 1);  // wave-uniform, in a scalar register
        const int top = nsp > 32 ? 32 : 16;
        for (int cb = 0; cb < ncand; cb += CH * kWave) {
            // Blocks of 64 candidates this chunk holds (wave-uniform): the
            // last chunk of a cell is usually short.
            const int nbk = min(CH, (ncand - cb + kWave - 1) / kWave);
            T cand[CH];
            bool cv[CH];
#pragma unroll
            for (int b = 0; b < CH; ++b) {
                cv[b] = false;
                cand[b] = T{};
                if (b >= nbk) continue;
                const int t = cb + b * kWave + lane;
                // Largest stencil cell s of this part with soff[s] <= t: a
                // fixed 5-step (6 with more than 32 cells) binary search,
                // every lane shuffling in every step.
                int sel = 0;
                for (int stp = top; stp >= 1; stp >>= 1) {
                    const int cand_s = sel + stp;
                    const int v = __shfl(soff, cand_s < nsp ? cand_s : nsp - 1);
                    if (cand_s < nsp && v <= t) sel = cand_s;
                }
                const int cs = __shfl(scell, sel), os = __shfl(soff, sel);
                cv[b] = t < ncand;
                int e = t - os;
                e = e < 0 ? 0 : (e >= g.cell_cap ? g.cell_cap - 1 : e);
                const int64_t at = cv[b] ? (int64_t)cs * g.cell_cap + e : 0;
                cand[b] = cr[at];
                cv[b] = cv[b] && (unsigned)CR::index(cand[b]) < (unsigned)g.n;
            }
            if constexpr (FILT) {
                // Queue, per group, the candidates within reach of its box.
#pragma unroll
                for (int b = 0; b < CH; ++b) {
                    if (b >= nbk) break;
                    // Wide grids: the candidate's coordinates relative to
                    // group 0's box corner, as signed quanta (the direct
                    // image is the nearest one).
                    const int32_t dx = (int32_t)((uint32_t)cand[b].x - bmn[0][0]);
                    const int32_t dy = (int32_t)((uint32_t)cand[b].y - bmn[0][1]);
                    const int32_t dz = (int32_t)((uint32_t)cand[b].z - bmn[0][2]);
                    const unsigned long long cvm = __builtin_amdgcn_ballot_w64(cv[b]);
#pragma unroll
                    for (int gi = 0; gi < 2; ++gi) {
                        float gx, gy, gz;
                        if constexpr (WIDE) {
                            gx = (float)max(max(glo[gi][0] - dx, dx - ghi[gi][0]), 0);
                            gy = (float)max(max(glo[gi][1] - dy, dy - ghi[gi][1]), 0);
                            gz = (float)max(max(glo[gi][2] - dz, dz - ghi[gi][2]), 0);
                        } else {
                            gx = (float)gap_q((uint32_t)cand[b].x, bmn[gi][0], bspan[gi][0]);
                            gy = (float)gap_q((uint32_t)cand[b].y, bmn[gi][1], bspan[gi][1]);
                            gz = (float)gap_q((uint32_t)cand[b].z, bmn[gi][2], bspan[gi][2]);
                        }
                        // The ballot of the bare compare, masked with the
                        // real candidates' ballot in scalar registers.
                        const bool near = fmaf(gz, gz, fmaf(gy, gy, gx * gx)) <= greach[gi];
                        const unsigned long long km = __builtin_amdgcn_ballot_w64(near) & cvm;
                        const uint32_t pos = __builtin_amdgcn_mbcnt_hi(
                            (uint32_t)(km >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)km, (uint32_t)fill[gi]));
                        if (near && cv[b]) queue[gi * NlistQueue<CH>::kCap + pos] = CR::index(cand[b]);
                        fill[gi] += __popcll(km);
                    }
                }
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                __builtin_amdgcn_wave_barrier();
                // A queue holding CH blocks or more: test its first CH
                // blocks, then move the rest (fewer than CH blocks) to its
                // front.
                for (int gi = 0; gi < 2; ++gi) {
                    if (fill[gi] < CH * kWave) continue;
                    drain(gi, CH * kWave);
                    int32_t *qg = queue + gi * NlistQueue<CH>::kCap;
                    const int rest = fill[gi] - CH * kWave;
                    int32_t mv[CH];
#pragma unroll
                    for (int b = 0; b < CH; ++b) {
                        const int t = b * kWave + lane;
                        mv[b] = t < rest ? qg[CH * kWave + t] : 0;
                    }
                    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                    __builtin_amdgcn_wave_barrier();
#pragma unroll
                    for (int b = 0; b < CH; ++b) {
                        const int t = b * kWave + lane;
                        if (t < rest) qg[t] = mv[b];
                    }
                    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                    __builtin_amdgcn_wave_barrier();
                    fill[gi] = rest;
                }
            } else {
                uint32_t thr[CH], thr1[CH];
#pragma unroll
                for (int b = 0; b < CH; ++b) {
                    thr[b] = thr1[b] = 0u;
                    if (b >= nbk) continue;
                    nlist_bounds<PREC, NS, QC>(box, pc, cand[b], cv[b], thr[b], thr1[b]);
                }
                nlist_homes<PREC, NS, QC, LG, CH>(st, g, box, pc, hrec, kreg, all, cand, cv, thr, thr1, nbk);
            }
        }
        }
        if constexpr (FILT) {
            for (int gi = 0; gi < 2; ++gi)
                if (fill[gi] > 0) drain(gi, fill[gi]);
            // The next group of home particles (cells over 64) starts on
            // empty queues; make this group's reads complete first.
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
        }
        if (lane < hm) {
            const int i = CR::index(hrec);
            if ((unsigned)i < (unsigned)g.n) {
                uint32_t q[3];
                rec_q(hrec, box, q);
                st.nbr_cnt[i] = kreg;
                st.xref[i] = make_int4((int)q[0], (int)q[1], (int)q[2], CR::species(hrec));
                if (kreg > g.cap) atomicOr(&ctl->flags, kErrList);
            }
        }
    }
}

// The lists of home cell c (see nlist_cell_as).
template <int PREC, int NS, bool QC, int LG = -1>
__device__ inline void nlist_cell(const State &st, const Geom &g, const BoxC &box, const PairC &pc,
                                  const int32_t *rank_of, const int32_t *cell_lin, int64_t c_off, int c,
                                  Ctl *ctl, const typename CellRec<PREC>::T *__restrict__ rec, int32_t *queue) {
    constexpr bool FILT = PREC == LJMD_FP32_DS && QC;
    const int w = 2 * box.reach + 2;
    if (FILT && box.nc[0] >= w && box.nc[1] >= w && box.nc[2] >= w)
        nlist_cell_as<PREC, NS, QC, LG, FILT>(st, g, box, pc, rank_of, cell_lin, c_off, c, ctl, rec, queue);
    else
        nlist_cell_as<PREC, NS, QC, LG, false>(st, g, box, pc, rank_of, cell_lin, c_off, c, ctl, rec, queue);
}

// Per-block LDS of the reduced list build (FP32 cubic boxes only): two
// candidate queues per wave.
template <int PREC, bool QC>
struct NlistStage {
    static constexpr int kPerWave =
        (PREC == LJMD_FP32_DS && QC) ? 2 * NlistQueue<NlistChunk<PREC, true>::CH>::kCap : 0;
    static constexpr int kEntries = kPerWave > 0 ? kNlWaves * kPerWave : 1;
};

template <int PREC, int NS, bool QC, int LG = -1>
__global__ __launch_bounds__(kNlWaves * kWave, 6) void k_nlist(State st, Geom g, BoxC box, PairC pc, int cur,
                                                            int64_t step, int forced, float thr2) {
    if (halted(st.ctl) || !rebuild_due(st.ctl, step, forced, thr2)) return;
    if (blockIdx.x == 0 && threadIdx.x == 0) st.ctl->rebuilds += 1;
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)), W = blockDim.x >> 6;
    const int tw = gridDim.x * W;
    using Stage = NlistStage<PREC, QC>;
    __shared__ int32_t queue_all[Stage::kEntries];
    int32_t *queue = queue_all + wv * Stage::kPerWave;
    const auto *rec = records<PREC>(st, cur);
    if (box.ncell < 8 * tw) {
        // A few cells per wave: contiguous runs of Hilbert-ranked cells, each
        // XCD one contiguous share of the box.
        const int gw = xcd_remap(blockIdx.x, gridDim.x) * W + wv;
        const int per = (box.ncell + tw - 1) / tw;
        const int cbeg = gw * per, cend = min(cbeg + per, box.ncell);
        for (int c = cbeg; c < cend; ++c)
            nlist_cell<PREC, NS, QC, LG>(st, g, box, pc, st.rank_of, st.cell_lin, 0, c, st.ctl, rec, queue);
        return;
    }
    // Many cells per wave: each XCD (blocks are dispatched to XCD
    // blockIdx % 8) owns one contiguous share of the cells and its waves take
    // the next cell of that share from a queue, since cells differ in
    // occupancy. With fewer than 8 blocks, each block owns a share. Every
    // wave leaves once its share is used up.
    const int nq = gridDim.x < 8 ? (int)gridDim.x : 8;
    const int q = (int)(blockIdx.x % (unsigned)nq);
    const int lo = (int)((int64_t)box.ncell * q / nq), hi = (int)((int64_t)box.ncell * (q + 1) / nq);
    const int lane = threadIdx.x & 63;
    for (;;) {
        int c = 0;
        if (lane == 0) c = lo + (int)atomicAdd(&st.ctl->nlq[q], 1u);
        c = __builtin_amdgcn_readfirstlane(c);  // wave-uniform from here on
        if (c >= hi) break;
        nlist_cell<PREC, NS, QC, LG>(st, g, box, pc, st.rank_of, st.cell_lin, 0, c, st.ctl, rec, queue);
    }
}

// ---- batches of systems -------------------------------------------------
// Plan entry k holds flattened items [off[k], off[k + 1]): the last k with
// off[k] <= t.
__device__ inline int plan_find(const int64_t *off, int count, int64_t t) {
    int lo = 0, hi = count;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (off[mid] <= t) lo = mid;
        else hi = mid;
    }
    return lo;
}

// Plans of up to kPlanLds systems are searched in LDS: the block copies the
// offsets there once instead of every lookup walking a chain of dependent
// global loads.
constexpr int kPlanLds = 512;

// Copy off[0 .. count] into sh when it fits (every thread of the block must
// call this); true if it did.
__device__ inline bool plan_stage(const int64_t *off, int count, int64_t *sh) {
    if (count > kPlanLds) return false;
    for (int k = threadIdx.x; k <= count; k += blockDim.x) sh[k] = off[k];
    __syncthreads();
    return true;
}

// One block: per system the rebuild decision (forced, or its largest
// displacement since its last build exceeded skin/2), the reset of the
// other parity word, and the compacted list of systems that rebuild with
// prefix sums of their particle and cell counts.
__global__ __launch_bounds__(1024) void k_batch_plan(State st, const SysC *sys, int nsys, BatchPlan bp,
                                                     int64_t step, int forced, float thr2) {
    __shared__ int32_t sn[1024];
    __shared__ int64_t sp[1024], sc[1024];
    const int t = threadIdx.x;
    if (t < 8) st.ctl->nlq[t] = 0u;  // list-build queues of this step
    const int per = (nsys + 1023) / 1024;
    const int s0 = t * per, s1 = min(s0 + per, nsys);
    int cnt = 0;
    int64_t np = 0, nc = 0;
    for (int s = s0; s < s1; ++s) {
        Ctl *ctl = st.ctl + s;
        const bool d = !halted(ctl) && rebuild_due(ctl, step, forced, thr2);
        ctl->maxd[(step + 1) & 1] = 0u;
        bp.due[s] = d ? 1 : 0;
        if (d) {
            ++cnt;
            np += sys[s].n;
            nc += sys[s].box.ncell;
            ctl->rebuilds += 1;
        }
    }
    sn[t] = cnt;
    sp[t] = np;
    sc[t] = nc;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
        const int a = t >= o ? sn[t - o] : 0;
        const int64_t b = t >= o ? sp[t - o] : 0, c = t >= o ? sc[t - o] : 0;
        __syncthreads();
        sn[t] += a;
        sp[t] += b;
        sc[t] += c;
        __syncthreads();
    }
    int k = sn[t] - cnt;
    int64_t po = sp[t] - np, co = sc[t] - nc;
    for (int s = s0; s < s1; ++s) {
        if (!bp.due[s]) continue;
        bp.wl_sys[k] = s;
        bp.wl_poff[k] = po;
        bp.wl_coff[k] = co;
        ++k;
        po += sys[s].n;
        co += sys[s].box.ncell;
    }
    if (t == 1023) {
        bp.wl_count[0] = sn[1023];
        bp.wl_poff[sn[1023]] = sp[1023];
        bp.wl_coff[sn[1023]] = sc[1023];
    }
}

__global__ __launch_bounds__(kRbBlock) void k_batch_bin(State st, Geom g, const SysC *sys, BatchPlan bp, int cur) {
    __shared__ int64_t plan_sh[kPlanLds + 1];
    const int count = bp.wl_count[0];
    const bool lds = plan_stage(bp.wl_poff, count, plan_sh);
    const int64_t total = bp.wl_poff[count];
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += stride) {
        const int k = lds ? plan_find(plan_sh, count, t) : plan_find(bp.wl_poff, count, t);
        const int s = bp.wl_sys[k];
        const SysC &y = sys[s];
        const int64_t first = lds ? plan_sh[k] : bp.wl_poff[k];
        bin_one<LJMD_FP32_DS>(st, g, y.box, st.rank_of + y.c_off, y.c_off, cur, y.p_off + (t - first), st.ctl + s);
    }
}

__global__ __launch_bounds__(kRbBlock) void k_batch_canon(State st, Geom g, const SysC *sys, BatchPlan bp) {
    using T = typename CellRec<LJMD_FP32_DS>::T;
    extern __shared__ int4 sm_raw[];
    __shared__ int64_t plan_sh[kPlanLds + 1];
    const int wv = threadIdx.x >> 6, W = blockDim.x >> 6;
    T *tmp = (T *)((uint8_t *)sm_raw + (size_t)wv * canon_lds_per_wave(g.cell_cap, sizeof(T)));
    int32_t *key = (int32_t *)(tmp + g.cell_cap);
    const int count = bp.wl_count[0];
    const bool lds = plan_stage(bp.wl_coff, count, plan_sh);
    const int64_t total = bp.wl_coff[count];
    for (int64_t w = (int64_t)blockIdx.x * W + wv; w < total; w += (int64_t)gridDim.x * W) {
        const int k = lds ? plan_find(plan_sh, count, w) : plan_find(bp.wl_coff, count, w);
        const SysC &y = sys[bp.wl_sys[k]];
        const int64_t first = lds ? plan_sh[k] : bp.wl_coff[k];
        canon_cell<LJMD_FP32_DS>(st, g, y.c_off + (w - first), tmp, key);
    }
}

template <int LG>
__global__ __launch_bounds__(kNlWaves * kWave, 5) void k_batch_nlist(State st, Geom g, const SysC *sys, BatchPlan bp,
                                                                  PairC pc, int cur) {
    __shared__ int64_t plan_sh[kPlanLds + 1];
    const int count = bp.wl_count[0];
    const bool lds = plan_stage(bp.wl_coff, count, plan_sh);
    const int64_t total = bp.wl_coff[count];
    // The flattened cells of the systems due, split into one contiguous share
    // per XCD whose waves take the next cell from a queue (as k_nlist; the
    // queues live in the first system's control words, reset by the plan).
    const int nq = gridDim.x < 8 ? (int)gridDim.x : 8;
    const int q = (int)(blockIdx.x % (unsigned)nq);
    const int64_t lo = total * q / nq, hi = total * (q + 1) / nq;
    const int lane = threadIdx.x & 63;
    using Stage = NlistStage<LJMD_FP32_DS, true>;
    __shared__ int32_t queue_all[Stage::kEntries];
    int32_t *queue = queue_all + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)) * Stage::kPerWave;
    const int4 *rec = records<LJMD_FP32_DS>(st, cur);
    for (;;) {
        int64_t w = 0;
        if (lane == 0) w = lo + (int64_t)atomicAdd(&st.ctl->nlq[q], 1u);
        w = (int64_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(w >> 32)) << 32) |
                      (uint32_t)__builtin_amdgcn_readfirstlane((int)w));
        if (w >= hi) break;
        const int k = lds ? plan_find(plan_sh, count, w) : plan_find(bp.wl_coff, count, w);
        const int s = bp.wl_sys[k];
        const SysC &y = sys[s];
        const int64_t first = lds ? plan_sh[k] : bp.wl_coff[k];
        nlist_cell<LJMD_FP32_DS, 1, true, LG>(st, g, y.box, pc, st.rank_of + y.c_off, st.cell_lin + y.c_off,
                                              y.c_off, (int)(w - first), st.ctl + s, rec, queue);
    }
}

// One block per system: slot offsets of its cells for a resort.
__global__ __launch_bounds__(1024) void k_batch_scan(State st, Geom g, const SysC *sys) {
    const SysC &y = sys[blockIdx.x];
    scan_cells(st, g, y.c_off, y.box.ncell, y.p_off);
}

// ------------------------------------------------------------------------
static inline unsigned blocks_for(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

// One block per compute unit, fewer if the work is smaller.
// Blocks for a rebuild kernel: enough for the work, at most per_cu per
// compute unit. Cell canonicalisation and the batch's binning take two per
// compute unit: their waves wait on one cell's (or particle's) loads at a
// time, and twice the waves in flight measured the 512-replica batch at
// 4.40-4.43e9 particle-steps/s against 4.37e9 with one.
static inline unsigned rebuild_blocks(const Launch &L, int64_t work_items, int per_block, int per_cu = 1) {
    const unsigned need = blocks_for(work_items, per_block);
    const unsigned ncu = (L.g->ncu > 0 ? (unsigned)L.g->ncu : 256u) * (unsigned)per_cu;
    return need < ncu ? (need > 0 ? need : 1u) : ncu;
}

hipError_t launch_bin(const Launch &L, int64_t step, int forced) {
    const unsigned nb = rebuild_blocks(L, L.g->n, kRbBlock);
    if (L.g->prec == LJMD_FP64)
        hipLaunchKernelGGL(k_bin<LJMD_FP64>, dim3(nb), dim3(kRbBlock), 0, L.stream, *L.st, *L.g,
                           *L.box, L.cur, step, forced, L.dyn->thr2);
    else
        hipLaunchKernelGGL(k_bin<LJMD_FP32_DS>, dim3(nb), dim3(kRbBlock), 0, L.stream, *L.st, *L.g,
                           *L.box, L.cur, step, forced, L.dyn->thr2);
    return hipGetLastError();
}

hipError_t launch_canon(const Launch &L, int64_t step, int forced) {
    const size_t per_wave = canon_lds_per_wave(L.g->cell_cap, cell_rec_bytes(L.g->prec));
    int W = kRbBlock / kWave;
    while (W > 1 && (size_t)W * per_wave > 65536) --W;
    const unsigned nb = rebuild_blocks(L, L.box->ncell, W, 2);
    const size_t shm = (size_t)W * per_wave;
    if (L.g->prec == LJMD_FP64)
        hipLaunchKernelGGL(k_canon<LJMD_FP64>, dim3(nb), dim3(W * kWave), shm, L.stream, *L.st,
                           *L.g, *L.box, step, forced, L.dyn->thr2);
    else
        hipLaunchKernelGGL(k_canon<LJMD_FP32_DS>, dim3(nb), dim3(W * kWave), shm, L.stream, *L.st,
                           *L.g, *L.box, step, forced, L.dyn->thr2);
    return hipGetLastError();
}

hipError_t launch_resort(const Launch &L) {
    const int64_t npad = (L.g->n + 63) / 64 * 64;
    ResortView sv = resort_view(L.st->scratch, npad, L.g->prec);
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, L.stream, *L.st, *L.g, L.box->ncell);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const unsigned nb = blocks_for((int64_t)L.box->ncell * L.g->cell_cap, kBlock);
    const unsigned nc = blocks_for(L.g->n, kBlock);
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

template <int PREC, int NS>
static void nlist_launch(const Launch &L, int64_t step, int forced) {
    const unsigned need = blocks_for(L.box->ncell, kNlWaves);
    const unsigned ncu = L.g->ncu > 0 ? (unsigned)L.g->ncu : 256u;
    // The kernel takes the queue path when the cells outnumber 8 per wave.
    const bool queued = (int64_t)L.box->ncell >= (int64_t)8 * kNlWaves * kNlBlocksPerCu * ncu;
    const unsigned cap = ncu * (queued ? kNlQueueBlocksPerCu : kNlBlocksPerCu);
    const unsigned nb = need < cap ? (need > 0 ? need : 1u) : cap;
    // The common layout of the single-precision force pass (two lanes per
    // particle) has its own instantiation with the entry index folded.
    if (PREC == LJMD_FP32_DS && L.box->cubic && L.g->lanes == 2)
        hipLaunchKernelGGL((k_nlist<PREC, NS, PREC == LJMD_FP32_DS, 1>), dim3(nb), dim3(kNlWaves * kWave), 0,
                           L.stream, *L.st, *L.g, *L.box, *L.pc, L.cur, step, forced, L.dyn->thr2);
    else if (PREC == LJMD_FP32_DS && L.box->cubic)
        hipLaunchKernelGGL((k_nlist<PREC, NS, PREC == LJMD_FP32_DS>), dim3(nb), dim3(kNlWaves * kWave), 0, L.stream,
                           *L.st, *L.g, *L.box, *L.pc, L.cur, step, forced, L.dyn->thr2);
    else
        hipLaunchKernelGGL((k_nlist<PREC, NS, false>), dim3(nb), dim3(kNlWaves * kWave), 0, L.stream, *L.st,
                           *L.g, *L.box, *L.pc, L.cur, step, forced, L.dyn->thr2);
}

hipError_t launch_nlist(const Launch &L, int64_t step, int forced) {
    if (L.g->prec == LJMD_FP64) {
        if (L.g->nspecies == 1) nlist_launch<LJMD_FP64, 1>(L, step, forced);
        else nlist_launch<LJMD_FP64, 2>(L, step, forced);
    } else {
        if (L.g->nspecies == 1) nlist_launch<LJMD_FP32_DS, 1>(L, step, forced);
        else nlist_launch<LJMD_FP32_DS, 2>(L, step, forced);
    }
    return hipGetLastError();
}

hipError_t launch_batch_plan(const Launch &L, const SysC *sys, int nsys, const BatchPlan &bp, int64_t step,
                             int forced) {
    hipLaunchKernelGGL(k_batch_plan, dim3(1), dim3(1024), 0, L.stream, *L.st, sys, nsys, bp, step, forced,
                       L.dyn->thr2);
    return hipGetLastError();
}

hipError_t launch_batch_bin(const Launch &L, const SysC *sys, const BatchPlan &bp, int64_t total_particles) {
    const unsigned nb = rebuild_blocks(L, total_particles, kRbBlock, 2);
    hipLaunchKernelGGL(k_batch_bin, dim3(nb), dim3(kRbBlock), 0, L.stream, *L.st, *L.g, sys, bp, L.cur);
    return hipGetLastError();
}

hipError_t launch_batch_canon(const Launch &L, const SysC *sys, const BatchPlan &bp, int64_t total_cells) {
    const size_t per_wave = canon_lds_per_wave(L.g->cell_cap, cell_rec_bytes(LJMD_FP32_DS));
    int W = kRbBlock / kWave;
    // 64 KiB per block, the staged plan included.
    while (W > 1 && (size_t)W * per_wave + sizeof(int64_t) * (kPlanLds + 1) > 65536) --W;
    const unsigned nb = rebuild_blocks(L, total_cells, W, 2);
    hipLaunchKernelGGL(k_batch_canon, dim3(nb), dim3(W * kWave), (size_t)W * per_wave, L.stream, *L.st, *L.g, sys,
                       bp);
    return hipGetLastError();
}

hipError_t launch_batch_nlist(const Launch &L, const SysC *sys, const BatchPlan &bp, int64_t total_cells) {
    const unsigned need = blocks_for(total_cells, kNlWaves);
    const unsigned ncu = L.g->ncu > 0 ? (unsigned)L.g->ncu : 256u;
    const unsigned cap = ncu * kNlQueueBlocksPerCu;
    const unsigned nb = need < cap ? (need > 0 ? need : 1u) : cap;
    // Two lanes per particle (the usual tuned shape) with the entry index folded.
    if (L.g->lanes == 2)
        hipLaunchKernelGGL(k_batch_nlist<1>, dim3(nb), dim3(kNlWaves * kWave), 0, L.stream, *L.st, *L.g, sys, bp,
                           *L.pc, L.cur);
    else
        hipLaunchKernelGGL(k_batch_nlist<-1>, dim3(nb), dim3(kNlWaves * kWave), 0, L.stream, *L.st, *L.g, sys, bp,
                           *L.pc, L.cur);
    return hipGetLastError();
}

hipError_t launch_batch_scan(const Launch &L, const SysC *sys, int nsys) {
    hipLaunchKernelGGL(k_batch_scan, dim3((unsigned)nsys), dim3(1024), 0, L.stream, *L.st, *L.g, sys);
    return hipGetLastError();
}

// Gather and copy of a resort over every slot of the batch (one flat range).
hipError_t launch_batch_resort_move(const Launch &L, int64_t ncell_total) {
    const int64_t npad = (L.g->n + 63) / 64 * 64;
    ResortView sv = resort_view(L.st->scratch, npad, LJMD_FP32_DS);
    BoxC all = *L.box;
    all.ncell = (int32_t)ncell_total;
    const int64_t slots = (int64_t)all.ncell * L.g->cell_cap;
    hipLaunchKernelGGL(k_resort_gather<LJMD_FP32_DS>, dim3(blocks_for(slots, kBlock)), dim3(kBlock), 0, L.stream,
                       *L.st, *L.g, all, L.cur, sv);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_resort_copy<LJMD_FP32_DS>, dim3(blocks_for(L.g->n, kBlock)), dim3(kBlock), 0, L.stream,
                       *L.st, *L.g, L.cur, sv);
    return hipGetLastError();
}

}  // namespace ljmd
