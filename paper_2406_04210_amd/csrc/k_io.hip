// k_io.hip -- boundary kernels: loading a state given by particle id,
// reading state, forces and lists back by id, and the deterministic FP64
// reduction of per-block observable partials (paper Sec. 4 "Mixed
// Strategy": reductions; Sec. 3: observables sampled between steps).
#include "internal.h"

namespace ljmd {

// Load x, v, species (by id) into slot i = id; wrap x into [0, L) as
//   f = floor(x / L); w = x - L f; if (w >= L) { w -= L; f += 1; }
// and, in the FP32 path, split w and v into double-single pairs
// (hi = (float) w, lo = (float)(w - hi)) and form the fixed-point record.
template <int PREC>
__global__ __launch_bounds__(kBlock) void k_set_state(State st, Geom g, BoxC box, int cur,
                                                      const double *__restrict__ x,
                                                      const double *__restrict__ v,
                                                      const int32_t *__restrict__ sp) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= g.n) return;
    int s = sp[i];
    s = s < 0 ? 0 : (s >= g.nspecies ? g.nspecies - 1 : s);
    double w[3];
    int im[3];
    for (int k = 0; k < 3; ++k) {
        const double xi = x[3 * i + k];
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
    st.id[i] = (int32_t)i;
    const double vx = v[3 * i], vy = v[3 * i + 1], vz = v[3 * i + 2];
    if constexpr (PREC == LJMD_FP64) {
        st.rec64[cur][i] = make_double4(w[0], w[1], w[2], (double)s);
        st.vel64[i] = make_double4(vx, vy, vz, 0.0);
    } else {
        float hi[3], lo[3];
        uint32_t q[3];
        for (int k = 0; k < 3; ++k) {
            hi[k] = (float)w[k];
            lo[k] = (float)(w[k] - (double)hi[k]);
            q[k] = q_from_ds(hi[k], lo[k], box.S_hi[k], box.S_lo[k]);
        }
        st.pos_hi[i] = make_float4(hi[0], hi[1], hi[2], 0.f);
        st.pos_lo[i] = make_float4(lo[0], lo[1], lo[2], 0.f);
        st.recq[cur][i] = make_int4((int)q[0], (int)q[1], (int)q[2], s);
        const float vhx = (float)vx, vhy = (float)vy, vhz = (float)vz;
        st.vel_hi[i] = make_float4(vhx, vhy, vhz, 0.f);
        st.vel_lo[i] = make_float4((float)(vx - (double)vhx), (float)(vy - (double)vhy),
                                   (float)(vz - (double)vhz), 0.f);
    }
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
        const float4 h = st.pos_hi[i], l = st.pos_lo[i];
        const float4 vh = st.vel_hi[i], vl = st.vel_lo[i];
        px = (double)h.x + (double)l.x;
        py = (double)h.y + (double)l.y;
        pz = (double)h.z + (double)l.z;
        vx = (double)vh.x + (double)vl.x;
        vy = (double)vh.y + (double)vl.y;
        vz = (double)vh.z + (double)vl.z;
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

}  // namespace ljmd
