// k_io.hip -- boundary kernels: loading a state given by particle id,
// reading state, forces and lists back by id, and the deterministic FP64
// reduction of per-block observable partials (paper Sec. 4 "Mixed
// Strategy": reductions; Sec. 3: observables sampled between steps).
#include "batch.h"
#include "internal.h"

namespace ljmd {

// Load x, v, species (by id) into slot i = id; wrap x into [0, L) as
//   f = floor(x / L); w = x - L f; if (w >= L) { w -= L; f += 1; }
// and, in the FP32 path, split w and v into double-single pairs
// (hi = (float) w, lo = (float)(w - hi)) and form the fixed-point record.
// Slot i takes row `row` of the caller's arrays (its id).
template <int PREC>
__device__ inline void set_one(const State &st, const Geom &g, const BoxC &box, int cur, int64_t i,
                               int64_t row, const double *__restrict__ x, const double *__restrict__ v,
                               const int32_t *__restrict__ sp) {
    int s = sp[row];
    s = s < 0 ? 0 : (s >= g.nspecies ? g.nspecies - 1 : s);
    double w[3];
    int im[3];
    for (int k = 0; k < 3; ++k) {
        // Two dimensions: z is held at 0 whatever the caller passed.
        const double xi = (k == 2 && g.dim == 2) ? 0.0 : x[3 * row + k];
        double f = floor(xi / box.L[k]);
        double t = xi - box.L[k] * f;
        if (t >= box.L[k]) {
            t -= box.L[k];
            f += 1.0;
        }
        w[k] = t;
        im[k] = (int)f;
    }
    st.img[i] = make_int4(im[0], im[1], im[2], 0);
    st.id[i] = (int32_t)row;
    const double vx = v[3 * row], vy = v[3 * row + 1], vz = g.dim == 2 ? 0.0 : v[3 * row + 2];
    if constexpr (PREC == LJMD_FP64) {
        st.rec64[cur][i] = make_double4(w[0], w[1], w[2], (double)s);
        st.vel64[i] = make_double4(vx, vy, vz, 0.0);
    } else {
        // Double-single, or (plain FP32) the nearest floats with zero lo
        // parts, a coordinate that rounds up to the box edge wrapping to 0.
        constexpr bool plain = PREC == LJMD_FP32;
        float hi[3], lo[3];
        uint32_t q[3];
        for (int k = 0; k < 3; ++k) {
            hi[k] = (float)w[k];
            if (plain && hi[k] >= box.Lhi[k]) {
                hi[k] -= box.Lhi[k];
                im[k] += 1;
            }
            lo[k] = plain ? 0.0f : (float)(w[k] - (double)hi[k]);
            q[k] = q_from_ds(hi[k], lo[k], box.S_hi[k], box.S_lo[k]);
        }
        if (plain) st.img[i] = make_int4(im[0], im[1], im[2], 0);
        st.recq[cur][i] = make_int4((int)q[0], (int)q[1], (int)q[2], s);
        const float vhx = (float)vx, vhy = (float)vy, vhz = (float)vz;
        DsState d;
        d.x = dsf{hi[0], lo[0]};
        d.y = dsf{hi[1], lo[1]};
        d.z = dsf{hi[2], lo[2]};
        d.vx = dsf{vhx, plain ? 0.0f : (float)(vx - (double)vhx)};
        d.vy = dsf{vhy, plain ? 0.0f : (float)(vy - (double)vhy)};
        d.vz = dsf{vhz, plain ? 0.0f : (float)(vz - (double)vhz)};
        ds_store(st.dsw, i, d);
        // The species also rides in the list reference's last word (the
        // step kernel reads it there); its coordinates are set by the list
        // build that follows every state load.
        st.xref[i] = make_int4(0, 0, 0, s);
    }
}

template <int PREC>
__global__ __launch_bounds__(kBlock) void k_set_state(State st, Geom g, BoxC box, int cur,
                                                      const double *__restrict__ x,
                                                      const double *__restrict__ v,
                                                      const int32_t *__restrict__ sp) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= g.n) return;
    set_one<PREC>(st, g, box, cur, i, i, x, v, sp);
}

template <int PREC>
__global__ __launch_bounds__(kBlock) void k_get_state(State st, Geom g, int cur, double *x,
                                                      double *v, int32_t *img) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= g.n) return;
    const int64_t id = st.id[i];
    if (id < 0 || id >= g.n) return;
    double px, py, pz, vx, vy, vz;
    if constexpr (PREC == LJMD_FP64) {
        const double4 r = st.rec64[cur][i];
        const double4 u = st.vel64[i];
        px = r.x; py = r.y; pz = r.z;
        vx = u.x; vy = u.y; vz = u.z;
    } else {
        const DsState d = ds_load(st.dsw, i);
        px = (double)d.x.hi + (double)d.x.lo;
        py = (double)d.y.hi + (double)d.y.lo;
        pz = (double)d.z.hi + (double)d.z.lo;
        vx = (double)d.vx.hi + (double)d.vx.lo;
        vy = (double)d.vy.hi + (double)d.vy.lo;
        vz = (double)d.vz.hi + (double)d.vz.lo;
    }
    if (x) {
        x[3 * id] = px;
        x[3 * id + 1] = py;
        x[3 * id + 2] = pz;
    }
    if (v) {
        v[3 * id] = vx;
        v[3 * id + 1] = vy;
        v[3 * id + 2] = vz;
    }
    if (img) {
        const int4 m = st.img[i];
        img[3 * id] = m.x;
        img[3 * id + 1] = m.y;
        img[3 * id + 2] = m.z;
    }
}

template <int PREC>
__global__ __launch_bounds__(kBlock) void k_get_forces(State st, Geom g, double *f) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= g.n) return;
    const int64_t id = st.id[i];
    if (id < 0 || id >= g.n) return;
    if constexpr (PREC == LJMD_FP64) {
        const double4 r = st.frc64[i];
        f[3 * id] = r.x;
        f[3 * id + 1] = r.y;
        f[3 * id + 2] = r.z;
    } else {
        const float4 r = st.frc32[i];
        f[3 * id] = r.x;
        f[3 * id + 1] = r.y;
        f[3 * id + 2] = r.z;
    }
}

__global__ __launch_bounds__(kBlock) void k_neighbors(State st, Geom g, int32_t *cnt, int32_t *ids,
                                                      int32_t cap_out) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= g.n) return;
    const int64_t id = st.id[i];
    if (id < 0 || id >= g.n) return;
    const int c = st.nbr_cnt[i];
    cnt[id] = c;
    int m = c < g.cap ? c : g.cap;
    m = m < cap_out ? m : cap_out;
    for (int k = 0; k < m; ++k) {
        const int j = st.nbr[nbr_index(i, k, g.lanes, g.cap)];
        ids[id * (int64_t)cap_out + k] = (j >= 0 && j < g.n) ? st.id[j] : -1;
    }
}

// One block per step: reduce that step's per-block partial rows in a fixed
// order (strided per thread, then a fixed LDS tree), so the FP64 sums are
// bit-reproducible. Row layout out: U, K, W, px, py, pz, rebuilt, step.
__global__ __launch_bounds__(kBlock) void k_obs_reduce(State st, Geom g, int64_t first_step,
                                                       int nblocks, double *obs, int64_t row0,
                                                       int count) {
    __shared__ double red[kBlock][6];
    const int sidx = blockIdx.x;
    const int64_t step = first_step + sidx;
    const int slot = (int)(step % kRing);
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (int b = threadIdx.x; b < nblocks; b += kBlock) {
        const double *r = st.partials + ((size_t)slot * g.max_blocks + b) * kNP;
        for (int q = 0; q < 6; ++q) acc[q] += r[q];
    }
    for (int q = 0; q < 6; ++q) red[threadIdx.x][q] = acc[q];
    __syncthreads();
    for (int s = kBlock / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s)
            for (int q = 0; q < 6; ++q) red[threadIdx.x][q] += red[threadIdx.x + s][q];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        double row[kNP] = {red[0][0], red[0][2], red[0][1], red[0][3],
                           red[0][4], red[0][5], (double)st.rebuilt[slot], (double)step};
        if (obs)
            for (int q = 0; q < kNP; ++q) obs[(row0 + sidx) * kNP + q] = row[q];
        if (sidx == count - 1)
            for (int q = 0; q < kNP; ++q) st.ctl->last[q] = row[q];
    }
}

// Longest current neighbour list (one block; only run on request).
__global__ __launch_bounds__(kBlock) void k_max_fill(State st, Geom g) {
    __shared__ int32_t red[kBlock / kWave];
    int m = 0;
    for (int64_t i = threadIdx.x; i < g.n; i += kBlock) {
        const int c = st.nbr_cnt[i];
        m = c > m ? c : m;
    }
    for (int o = 32; o > 0; o >>= 1) {
        const int y = __shfl_xor(m, o);
        m = y > m ? y : m;
    }
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int q = 1; q < kBlock / kWave; ++q) m = red[q] > m ? red[q] : m;
        st.ctl->max_fill = m;
    }
}

// ---- batches of systems -------------------------------------------------
// Slot i of a batch belongs to the system sys[sys_of_g16[i >> 4]] (systems
// are padded to whole blocks of slots); slots past a system's particles are
// padding and stay inert (no id, no list, never binned or moved).
__device__ inline const SysC &sys_of(const SysC *sys, const int32_t *sys_of_g16, int64_t i) {
    return sys[sys_of_g16[i >> 4]];
}

__global__ __launch_bounds__(kBlock) void k_batch_set_state(State st, Geom g, const SysC *sys,
                                                            const int32_t *sys_of_g16, int cur,
                                                            const double *__restrict__ x,
                                                            const double *__restrict__ v,
                                                            const int32_t *__restrict__ sp) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= g.n) return;
    const SysC &y = sys_of(sys, sys_of_g16, i);
    const int64_t local = i - y.p_off;
    if (local >= y.n) {
        st.id[i] = -1;
        st.img[i] = make_int4(0, 0, 0, 0);
        st.recq[cur][i] = make_int4(0, 0, 0, 0);
        st.dsw[0][i] = st.dsw[1][i] = st.dsw[2][i] = st.frc32[i] = make_float4(0.f, 0.f, 0.f, 0.f);
        st.xref[i] = make_int4(0, 0, 0, 0);
        st.nbr_cnt[i] = 0;
        return;
    }
    set_one<LJMD_FP32_DS>(st, g, y.box, cur, i, y.in_off + local, x, v, sp);
}

__global__ __launch_bounds__(kBlock) void k_batch_get(State st, Geom g, const SysC *sys,
                                                      const int32_t *sys_of_g16, int cur, double *x,
                                                      double *v, int32_t *img, double *f) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= g.n) return;
    const SysC &y = sys_of(sys, sys_of_g16, i);
    if (i - y.p_off >= y.n) return;
    const int64_t row = st.id[i];
    if (row < y.in_off || row >= y.in_off + y.n) return;
    if (x || v) {
        const DsState d = ds_load(st.dsw, i);
        if (x) {
            x[3 * row] = (double)d.x.hi + (double)d.x.lo;
            x[3 * row + 1] = (double)d.y.hi + (double)d.y.lo;
            x[3 * row + 2] = (double)d.z.hi + (double)d.z.lo;
        }
        if (v) {
            v[3 * row] = (double)d.vx.hi + (double)d.vx.lo;
            v[3 * row + 1] = (double)d.vy.hi + (double)d.vy.lo;
            v[3 * row + 2] = (double)d.vz.hi + (double)d.vz.lo;
        }
    }
    if (img) {
        const int4 m = st.img[i];
        img[3 * row] = m.x;
        img[3 * row + 1] = m.y;
        img[3 * row + 2] = m.z;
    }
    if (f) {
        const float4 r = st.frc32[i];
        f[3 * row] = r.x;
        f[3 * row + 1] = r.y;
        f[3 * row + 2] = r.z;
    }
}

// One block per system: its step-kernel rows of ring slot `slot`, reduced in
// the same fixed order as a single box's (strided per thread, then the LDS
// tree), so a system's observables match its run as a single box.
__global__ __launch_bounds__(kBlock) void k_batch_obs(State st, Geom g, const SysC *sys, int slot, int64_t step,
                                                      double *out) {
    __shared__ double red[kBlock][6];
    const SysC &y = sys[blockIdx.x];
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (int b = threadIdx.x; b < y.nb; b += kBlock) {
        const double *r = st.partials + ((size_t)slot * g.max_blocks + y.b_off + b) * kNP;
        for (int q = 0; q < 6; ++q) acc[q] += r[q];
    }
    for (int q = 0; q < 6; ++q) red[threadIdx.x][q] = acc[q];
    __syncthreads();
    for (int s = kBlock / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s)
            for (int q = 0; q < 6; ++q) red[threadIdx.x][q] += red[threadIdx.x + s][q];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        Ctl *ctl = st.ctl + y.id;
        double row[kNP] = {red[0][0], red[0][2], red[0][1], red[0][3],
                           red[0][4], red[0][5], (double)ctl->rebuilds, (double)step};
        for (int q = 0; q < kNP; ++q) ctl->last[q] = row[q];
        if (out)
            for (int q = 0; q < kNP; ++q) out[(size_t)y.id * kNP + q] = row[q];
    }
}

// ------------------------------------------------------------------------
static inline unsigned nblk(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

hipError_t launch_max_fill(const Launch &L) {
    hipLaunchKernelGGL(k_max_fill, dim3(1), dim3(kBlock), 0, L.stream, *L.st, *L.g);
    return hipGetLastError();
}

hipError_t launch_set_state(const Launch &L, const double *x, const double *v, const int32_t *sp) {
    if (L.g->prec == LJMD_FP64)
        hipLaunchKernelGGL(k_set_state<LJMD_FP64>, dim3(nblk(L.g->n)), dim3(kBlock), 0, L.stream,
                           *L.st, *L.g, *L.box, L.cur, x, v, sp);
    else if (L.g->prec == LJMD_FP32)
        hipLaunchKernelGGL(k_set_state<LJMD_FP32>, dim3(nblk(L.g->n)), dim3(kBlock), 0,
                           L.stream, *L.st, *L.g, *L.box, L.cur, x, v, sp);
    else
        hipLaunchKernelGGL(k_set_state<LJMD_FP32_DS>, dim3(nblk(L.g->n)), dim3(kBlock), 0,
                           L.stream, *L.st, *L.g, *L.box, L.cur, x, v, sp);
    return hipGetLastError();
}

hipError_t launch_get_state(const Launch &L, double *x, double *v, int32_t *img) {
    if (L.g->prec == LJMD_FP64)
        hipLaunchKernelGGL(k_get_state<LJMD_FP64>, dim3(nblk(L.g->n)), dim3(kBlock), 0, L.stream,
                           *L.st, *L.g, L.cur, x, v, img);
    else
        hipLaunchKernelGGL(k_get_state<LJMD_FP32_DS>, dim3(nblk(L.g->n)), dim3(kBlock), 0,
                           L.stream, *L.st, *L.g, L.cur, x, v, img);
    return hipGetLastError();
}

hipError_t launch_get_forces(const Launch &L, double *f) {
    if (L.g->prec == LJMD_FP64)
        hipLaunchKernelGGL(k_get_forces<LJMD_FP64>, dim3(nblk(L.g->n)), dim3(kBlock), 0, L.stream,
                           *L.st, *L.g, f);
    else
        hipLaunchKernelGGL(k_get_forces<LJMD_FP32_DS>, dim3(nblk(L.g->n)), dim3(kBlock), 0,
                           L.stream, *L.st, *L.g, f);
    return hipGetLastError();
}

hipError_t launch_neighbors(const Launch &L, int32_t *cnt, int32_t *ids, int32_t cap) {
    hipLaunchKernelGGL(k_neighbors, dim3(nblk(L.g->n)), dim3(kBlock), 0, L.stream, *L.st, *L.g,
                       cnt, ids, cap);
    return hipGetLastError();
}

hipError_t launch_obs_reduce(const Launch &L, int64_t first_step, int count, int nblocks,
                             double *obs_dev, int64_t obs_row0) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_obs_reduce, dim3(count), dim3(kBlock), 0, L.stream, *L.st, *L.g,
                       first_step, nblocks, obs_dev, obs_row0, count);
    return hipGetLastError();
}

hipError_t launch_batch_set_state(const Launch &L, const SysC *sys, const int32_t *sys_of_g16, int64_t nslots,
                                  const double *x, const double *v, const int32_t *sp) {
    hipLaunchKernelGGL(k_batch_set_state, dim3(nblk(nslots)), dim3(kBlock), 0, L.stream, *L.st, *L.g, sys,
                       sys_of_g16, L.cur, x, v, sp);
    return hipGetLastError();
}

hipError_t launch_batch_get_state(const Launch &L, const SysC *sys, const int32_t *sys_of_g16, int64_t nslots,
                                  double *x, double *v, int32_t *img) {
    hipLaunchKernelGGL(k_batch_get, dim3(nblk(nslots)), dim3(kBlock), 0, L.stream, *L.st, *L.g, sys, sys_of_g16,
                       L.cur, x, v, img, (double *)nullptr);
    return hipGetLastError();
}

hipError_t launch_batch_get_forces(const Launch &L, const SysC *sys, const int32_t *sys_of_g16, int64_t nslots,
                                   double *f) {
    hipLaunchKernelGGL(k_batch_get, dim3(nblk(nslots)), dim3(kBlock), 0, L.stream, *L.st, *L.g, sys, sys_of_g16,
                       L.cur, (double *)nullptr, (double *)nullptr, (int32_t *)nullptr, f);
    return hipGetLastError();
}

hipError_t launch_batch_obs(const Launch &L, const SysC *sys, int nsys, int slot, int64_t step, double *out) {
    hipLaunchKernelGGL(k_batch_obs, dim3((unsigned)nsys), dim3(kBlock), 0, L.stream, *L.st, *L.g, sys, slot, step,
                       out);
    return hipGetLastError();
}

}  // namespace ljmd
