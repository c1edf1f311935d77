// internal.h -- shared declarations of the gfx950 LJ MD library (device
// constants, workspace views, double-single and fixed-point helpers, kernel
// launchers). Not part of the public ABI.
//
// Every translation unit is compiled with -ffp-contract=off: multiplies and
// adds are never fused implicitly, and each fused multiply-add is written out
// with fmaf/fma. That makes the FP32 list-membership sequence and the
// error-free transformations of the double-single arithmetic exact as stated.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>
#include <stdint.h>

#include "../../include/ljmd.h"

namespace ljmd {

constexpr int kWave = 64;        // CDNA wavefront width
constexpr int kBlock = 1024;     // threads per block of the per-particle kernels
constexpr int kBlockF64 = 256;   // threads per block of the FP64 step kernel (register-heavy)
__host__ __device__ constexpr int step_block_threads(int prec) { return prec == LJMD_FP64 ? kBlockF64 : kBlock; }
constexpr int kApFinishBlock = 64;  // threads per block of the all-pairs step tail (one wavefront)
constexpr int kRing = 64;        // steps of block partials kept before an observable flush
constexpr int kNP = 8;           // doubles per partial row: U, W, K, px, py, pz, -, -

// Latched device error bits (ctl->flags).
enum : uint32_t { kErrList = 1u, kErrCell = 2u, kErrNaN = 4u };
// List slots allocated past the last row: the force loop of a cubic box
// reads up to one group row (256 entries) past a chunk's lists without
// clamping.
constexpr size_t kListPad = 8 * 64;

// Box constants. The fixed-point image coordinate q = round(x * 2^32 / L)
// mod 2^32 turns the minimum image into a wrapping 32-bit subtraction.
struct BoxC {
    double L[3], invL[3], S[3];  // S = 2^32 / L
    float Lhi[3], Llo[3];        // L as a double-single pair
    float qs_hi[3], qs_lo[3];    // quantum L * 2^-32 as a double-single pair
    float S_hi[3], S_lo[3];      // 2^32 / L as a double-single pair
    float r2c[3];                // (quantum / qs_hi)^2: removes the systematic rounding
                                 // of the single-float quantum from r^2 in the force kernel
    int32_t nc[3];               // cells per axis
    int32_t ncell;
    int32_t cubic;               // all three edges equal: forces may work in quanta
    int32_t reach;               // list-build stencil half-width in cells (1: edge >= r_L, 2: edge >= r_L / 2)
    // Cubic boxes, per pair type: r_c^2 and sigma^2 in units of the squared
    // quantum (L 2^-32)^2, and 24 eps / quantum, so that the force kernel can
    // use raw fixed-point differences as displacements.
    float rc2q[3], sig2q[3], fq[3];
    // Cubic boxes: list radius squared per pair type in squared quanta (the
    // FP32 list criterion of a cubic box compares raw differences).
    float rl2q[3];
};

// Pair constants by symmetric pair type t = a + b (0: AA, 1: AB, 2: BB).
struct PairC {
    double rc2[3], rl2[3], sig2[3], eps24[3], eps4[3], shift[3];
    float rc2f[3], rl2f[3], sig2f[3], eps24f[3], eps4f[3], shiftf[3];
};

// Integration constants per species.
struct DynC {
    double hdt_m[2];                 // dt / (2 m)
    float hdt_m_hi[2], hdt_m_lo[2];  // the same as double-single pairs
    double dt;
    float dt_hi, dt_lo;
    double mass[2];
    float massf[2];
    float thr2;                      // (skin / 2)^2: rebuild when exceeded
    // Stochastic velocity resampling (the Andersen-like thermostat): a
    // particle collides in a step when the first word of its Philox block is
    // below thermo_thr (probability rate * dt), and then takes the velocity
    // sqrt(T / m) z, z standard normal.
    int32_t thermo_on;
    uint32_t thermo_thr, seed_lo, seed_hi;
    double thermo_sd[2];             // sqrt(T / m) per species
};

// Control words in device memory.
struct Ctl {
    uint32_t maxd[2];     // max squared displacement since the last build (float bits), by drift parity
    uint32_t flags;       // latched error bits
    int32_t max_fill;     // longest current list (computed on request)
    int64_t rebuilds;     // list builds since set_state
    unsigned long long fmax[2];  // steepest descent: max |F| (double bits), by iteration parity
    int64_t halt;         // 1 + step id of the first step kernel that found an error latched (0: none)
    uint32_t nlq[8];      // list-build work queues (next cell), one per XCD; reset before each build
    double last[kNP];     // observables of the last flushed step: U, W, K, px, py, pz, rebuilt, step
};

// One system of a batch (independent boxes sharing the potential and the
// integration constants). Its particles occupy slots [p_off, p_off + n) of
// the flattened arrays, padded to whole step-kernel blocks; its cells
// are [c_off, c_off + box.ncell); its step-kernel blocks [b_off, b_off + nb).
struct SysC {
    BoxC box;
    int64_t p_off;   // first slot
    int64_t in_off;  // first row of the caller's concatenated arrays
    int32_t n;       // particles
    int32_t id;      // index of the system (its control words are ctl[id])
    int32_t c_off;   // first cell
    int32_t b_off;   // first step-kernel block
    int32_t nb;      // step-kernel blocks
    int32_t pad;
};

// Views of the caller's workspace (all device pointers).
struct State {
    // FP64 path
    double4 *rec64[2];    // gathered record (x, y, z, species) -- ping-pong by step
    double4 *vel64;       // (vx, vy, vz, 0)
    double4 *frc64;       // forces of the last step (fx, fy, fz, 0)
    // FP32 + double-single path
    int4 *recq[2];        // gathered record (qx, qy, qz, species) -- ping-pong by step
    float4 *dsw[3];       // double-single position and velocity, three unpadded words (DsState)
    float4 *frc32;
    // common
    int4 *img;            // periodic image counters (x, y, z, 0)
    int32_t *id;          // original id of the particle stored at this slot
    int4 *xref;           // q at the last list build (x, y, z) and the species
    int32_t *nbr;         // neighbour list, interleaved by wave chunk (see nbr_index)
    int32_t *nbr_cnt;     // list length per particle
    int32_t *cell_count;  // particles binned per cell (cells indexed by Hilbert rank)
    void *cell_rec;       // [ncell][cell_cap] slot records (int4 FP32 / double4 FP64):
                          // position record with (index << 1 | species) in .w,
                          // ascending by index after canonicalisation
    int32_t *cell_start;  // [ncell + 1] exclusive scan of counts (resort only)
    int32_t *rank_of;     // [ncell] Hilbert rank of the cell with linear index (ix*ny+iy)*nz+iz
    int32_t *cell_lin;    // [ncell] linear index of the cell with a given Hilbert rank
    uint8_t *scratch;     // resort staging
    double *partials;     // [kRing][max_blocks][kNP] per-block observable partials
    int32_t *rebuilt;     // [kRing] 1 if the list was rebuilt before that step's force
    Ctl *ctl;
};

struct Geom {
    int64_t n;
    int32_t cap;          // list slots per particle (multiple of 16)
    int32_t cell_cap;     // slots per cell
    int32_t lanes;        // lanes per particle in the force gather
    int32_t nspecies;
    int32_t prec;
    int32_t max_blocks;   // rows per ring slot of partials
    int32_t ncu;          // compute units of the device (grid of the per-step rebuild kernels)
    int32_t all_pairs;    // 1: untruncated all-pairs interaction (no lists, no cells)
    int32_t dim;          // 2 (motion in the x-y plane, z and v_z held at 0) or 3
};

// ------------------------------------------------------------------------
// Device helpers
// ------------------------------------------------------------------------

// Chunked, interleaved neighbour-list layout. A wave owns P = 64/lanes
// particles; particle i's entry k belongs to lane L = (i%P)*lanes + k%lanes
// of its chunk as that lane's entry m = k/lanes, and lanes keep their entries
// in groups of four:
//   chunk*(P*cap) + (m/4)*256 + L*4 + m%4,   chunk = i/P,
// so one 16-byte load per lane fetches four consecutive entries and a wave
// reads 1 KiB contiguous. cap is a multiple of 4*lanes; lanes is a power of
// two, so the index is shifts and masks only.
__host__ __device__ inline int64_t nbr_index(int64_t i, int32_t k, int32_t lanes, int32_t cap) {
    const int lg = lanes >= 16 ? 4 : (lanes >= 8 ? 3 : (lanes >= 4 ? 2 : (lanes >= 2 ? 1 : 0)));
    const int pg = 6 - lg;  // log2 of particles per chunk
    const int64_t chunk = i >> pg;
    const int32_t p = (int32_t)(i & ((1 << pg) - 1));
    const int32_t m = k >> lg, L = (p << lg) + (k & (lanes - 1));
    return ((chunk * (int64_t)cap) << pg) + ((int64_t)(m >> 2) << 8) + (L << 2) + (m & 3);
}

// Entry m of the lane whose entries start at nbl (its chunk's base + 4*L).
__device__ inline int32_t nb_entry(const int32_t *nbl, int m) { return nbl[((int64_t)(m >> 2) << 8) + (m & 3)]; }

// List capacity granule: whole groups of four entries per lane.
__host__ __device__ inline int32_t cap_granule(int32_t lanes) { return 4 * lanes > 16 ? 4 * lanes : 16; }

// Blocks are dispatched round-robin over the 8 XCDs of the chip; remap so
// that each XCD works on one contiguous eighth of the (space-filling-curve
// ordered) particles and its L2 holds one compact region of the box.
__device__ inline int xcd_remap(int b, int nb) {
    int q = nb >> 3;
    if (b >= (q << 3)) return b;
    return (b & 7) * q + (b >> 3);
}

// Error-free transformations (Knuth's TwoSum, Dekker's Fast2Sum and the
// fma-based TwoProduct) and double-single arithmetic built on them.
struct dsf {
    float hi, lo;
};

__device__ inline dsf two_sum(float a, float b) {
    float s = a + b;
    float bb = s - a;
    float e = (a - (s - bb)) + (b - bb);
    return {s, e};
}

__device__ inline dsf fast_two_sum(float a, float b) {  // requires |a| >= |b| or a == 0
    float s = a + b;
    float e = b - (s - a);
    return {s, e};
}

__device__ inline dsf ds_add(dsf a, dsf b) {
    dsf s = two_sum(a.hi, b.hi);
    float e = s.lo + (a.lo + b.lo);
    return fast_two_sum(s.hi, e);
}

// (c_hi + c_lo) * f as a double-single pair.
__device__ inline dsf ds_mul_f(float c_hi, float c_lo, float f) {
    float p = c_hi * f;
    float e = fmaf(c_hi, f, -p);
    e = fmaf(c_lo, f, e);
    return fast_two_sum(p, e);
}

// (a_hi + a_lo) * (b_hi + b_lo) as a double-single pair.
__device__ inline dsf ds_mul(dsf a, float b_hi, float b_lo) {
    float p = a.hi * b_hi;
    float e = fmaf(a.hi, b_hi, -p);
    e = fmaf(a.hi, b_lo, fmaf(a.lo, b_hi, e));
    return fast_two_sum(p, e);
}

// Double-single pair of an FP64 value: the nearest float and the rounded rest.
__device__ inline dsf ds_of(double v) {
    const float h = (float)v;
    return {h, (float)(v - (double)h)};
}

// Double-single position and velocity of one particle. Stored without
// padding as three float4 words per slot (State::dsw):
//   w0 = (x.hi, y.hi, z.hi, x.lo), w1 = (y.lo, z.lo, vx.hi, vy.hi),
//   w2 = (vz.hi, vx.lo, vy.lo, vz.lo).
// The plain single-precision state keeps every lo part zero.
struct DsState {
    dsf x, y, z, vx, vy, vz;
};
__device__ inline DsState ds_unpack(const float4 &w0, const float4 &w1, const float4 &w2) {
    DsState s;
    s.x = dsf{w0.x, w0.w};
    s.y = dsf{w0.y, w1.x};
    s.z = dsf{w0.z, w1.y};
    s.vx = dsf{w1.z, w2.y};
    s.vy = dsf{w1.w, w2.z};
    s.vz = dsf{w2.x, w2.w};
    return s;
}
__device__ inline DsState ds_load(float4 *const dsw[3], int64_t i) {
    return ds_unpack(dsw[0][i], dsw[1][i], dsw[2][i]);
}
__device__ inline void ds_store(float4 *const dsw[3], int64_t i, const DsState &s) {
    dsw[0][i] = make_float4(s.x.hi, s.y.hi, s.z.hi, s.x.lo);
    dsw[1][i] = make_float4(s.y.lo, s.z.lo, s.vx.hi, s.vy.hi);
    dsw[2][i] = make_float4(s.vz.hi, s.vx.lo, s.vy.lo, s.vz.lo);
}

// Fixed-point image coordinate of a double-single position (binary32 only):
// q = round((hi + lo) * S) mod 2^32 with S = 2^32/L given as (S_hi, S_lo).
__device__ inline uint32_t q_from_ds(float hi, float lo, float S_hi, float S_lo) {
    float p = hi * S_hi;
    float e = fmaf(hi, S_hi, -p);
    float a = hi * S_lo;
    float b = lo * S_hi;
    float c = a + b;
    float t = e + c;
    float pi = floorf(p);
    float pf = p - pi;
    float u = pf + t;
    long long q = (long long)pi + (long long)(int)rintf(u);
    return (uint32_t)(unsigned long long)q;
}

// Fixed-point coordinate of an FP64 position (used for binning and for the
// displacement check of the FP64 path).
__device__ inline uint32_t q_from_d(double x, double S) {
    return (uint32_t)(unsigned long long)(long long)rint(x * S);
}

// Minimum-image displacement from two fixed-point coordinates.
__device__ inline float disp_q(uint32_t qi, uint32_t qj, float qs_hi, float qs_lo) {
    int32_t dq = (int32_t)(qi - qj);
    float a = (float)dq;
    return fmaf(a, qs_hi, a * qs_lo);
}

// Minimum-image displacement of the FP64 path.
// Wrapped inputs give m in {-1, 0, 1}, so L*m is exact and the fused form
// equals t - L*m bit for bit.
__device__ inline double disp_d(double xi, double xj, double L, double invL) {
    double t = xi - xj;
    double m = rint(t * invL);
    return fma(-L, m, t);
}

// Cell (Hilbert rank) of a particle from its fixed-point coordinates.
__device__ inline int cell_of_q(uint32_t qx, uint32_t qy, uint32_t qz, const BoxC &b,
                                const int32_t *rank_of, int *cx, int *cy, int *cz) {
    int ix = (int)(((uint64_t)qx * (uint32_t)b.nc[0]) >> 32);
    int iy = (int)(((uint64_t)qy * (uint32_t)b.nc[1]) >> 32);
    int iz = (int)(((uint64_t)qz * (uint32_t)b.nc[2]) >> 32);
    *cx = ix;
    *cy = iy;
    *cz = iz;
    return rank_of[(ix * b.nc[1] + iy) * b.nc[2] + iz];
}

// Once an error is latched (list or cell overflow, non-finite position) no
// kernel changes the state any more, so that no step runs on a truncated
// list: the kernels return at once, and the first step kernel to see the
// error records its step (halt = step + 1), from which the host redoes the
// run after growing the list. The flags are written by earlier kernels of
// the stream (or by this kernel, for a non-finite position, after which the
// state is lost anyway), so every block of a launch sees the same value.
__device__ inline bool halted(const Ctl *ctl) { return ctl->flags != 0u; }
__device__ inline bool halted_record(Ctl *ctl, int64_t step, bool recorder) {
    if (ctl->flags == 0u) return false;
    if (recorder && threadIdx.x == 0 && ctl->halt == 0) ctl->halt = step + 1;
    return true;
}

// Whether the list is rebuilt before the force evaluation of a step: forced
// by the host (state load, resort) or the largest squared displacement since
// the last build exceeds (skin/2)^2. A NaN displacement also triggers it.
__device__ inline bool rebuild_due(const Ctl *ctl, int64_t step, int forced, float thr2) {
    if (forced) return true;
    uint32_t m = ctl->maxd[step & 1];
    return m > __float_as_uint(thr2);
}

// ------------------------------------------------------------------------
// Kernel launchers (host), one per kernel family.
// ------------------------------------------------------------------------
struct Launch {
    const State *st;
    const Geom *g;
    const BoxC *box;
    const PairC *pc;
    const DynC *dyn;
    hipStream_t stream;
    int cur;              // current ping-pong record buffer
    // Optional event pair stamped by the dispatch itself (start and end of
    // the kernel, no marker packets around it): set only for timed launches.
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
};

// Launch on L.stream; with L.ev0 set, through the extended launch that
// stamps L.ev0 / L.ev1 with the kernel's own start and end.
template <typename K, typename... Args>
inline void launch_k(const Launch &L, K kernel, dim3 grid, dim3 block, Args... args) {
    if (L.ev0)
        hipExtLaunchKernelGGL(kernel, grid, block, 0, L.stream, L.ev0, L.ev1, 0, args...);
    else
        hipLaunchKernelGGL(kernel, grid, block, 0, L.stream, args...);
}

hipError_t launch_set_state(const Launch &L, const double *x, const double *v, const int32_t *sp);
hipError_t launch_bin(const Launch &L, int64_t step, int forced);
hipError_t launch_canon(const Launch &L, int64_t step, int forced);
hipError_t launch_resort(const Launch &L);
hipError_t launch_nlist(const Launch &L, int64_t step, int forced);
// mode bits for launch_step
// kObserve: the step's observable partials (energy, virial, kinetic energy,
// momentum) will be reduced; without it the one-species cubic kernels skip
// them (positions, velocities and forces are the same either way).
enum : int { kFinalize = 1, kIntegrate = 2, kStoreForce = 4, kObserve = 8 };
// Particle slots below which the quanta force loop addresses records by a
// 32-bit byte offset.
constexpr int64_t kQuantaMaxSlots = (int64_t)1 << 28;
hipError_t launch_step(const Launch &L, int64_t step, int forced, int mode, int slot);
hipError_t launch_integrate(const Launch &L, int64_t step);
hipError_t launch_obs_reduce(const Launch &L, int64_t first_step, int count, int nblocks,
                             double *obs_dev, int64_t obs_row0);
hipError_t launch_get_state(const Launch &L, double *x, double *v, int32_t *img);
hipError_t launch_get_forces(const Launch &L, double *f);
hipError_t launch_neighbors(const Launch &L, int32_t *cnt, int32_t *ids, int32_t cap);
hipError_t launch_max_fill(const Launch &L);
hipError_t launch_sd(const Launch &L, int64_t step, int forced, int iter, double delta,
                     double clamp, double *fmax_out);
// All-pairs mode: splits of the j range, bytes of the partial rows (held in
// the list area), and the two launches of one step.
int allpairs_splits(int64_t n);
size_t allpairs_part_bytes(int64_t n, int prec);
hipError_t launch_allpairs_step(const Launch &L, int64_t step, int mode, int slot);
// One-shot brute-force forces of a configuration given by id: scratch of
// brute_scratch_bytes(n, prec) bytes (256-byte aligned); cut: truncate and
// shift at r_c (else every pair interacts). f (n*3) and uw (U, W) are FP64.
size_t brute_scratch_bytes(int64_t n, int prec);
hipError_t launch_brute(const BoxC &box, const PairC &pc, int prec, int nspecies, int dim, int cut, int64_t n,
                        const double *x, const int32_t *sp, double *f, double *uw, uint8_t *scratch,
                        hipStream_t stream);
// Box and pair constants of a parameter set (cell grid 1x1x1), and the
// parameter check of ljmd_check_params with its reason.
void box_pair_constants(const ljmd_params &p, BoxC &b, PairC &q);
int check_params_why(const ljmd_params *p, const char **why);
// Text returned by ljmd_last_error(NULL) (calls without a context).
void set_global_error(const char *msg);
size_t resort_scratch_bytes(int64_t npad, int prec);
size_t cell_rec_bytes(int prec);
int step_blocks(const Geom &g);

}  // namespace ljmd
