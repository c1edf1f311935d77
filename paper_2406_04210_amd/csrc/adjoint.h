// adjoint.h -- launchers of the adjoint kernels (k_adjoint.hip): the force
// vector-Jacobian product with the parameter gradients, the energy parameter
// gradient, and the per-particle vector operations of the reverse
// velocity-Verlet sweep.
#pragma once

#include "internal.h"

namespace ljmd {

// Pair pass modes.
enum : int { kAdjVjp = 0, kAdjEnergy = 1 };

// Per-particle operations of the reverse sweep (slot order unless noted).
enum : int {
    kOpGatherById = 0,   // a[i] = src_id[id[i]]        (FP64 triples by original id)
    kOpScatterById = 1,  // dst_id[id[i]] = a[i]
    kOpZero = 4,         // a[i] = 0
    kOpGatherG = 5,      // gvec[i] = src_id[id[i]]     (path precision)
    kOpDriftCotangent = 6,  // b[i] += scale * a[i] (skipped when scale == 0); gvec[i] = b[i] / m_i
                            // (path precision: double4 or float4)
    kOpSubForce = 7,        // a[i] -= c * F_i with c = *dscale (device) and F the stored forces
};

// One pair pass over the current lists at the positions in record buffer
// L.cur. kAdjVjp: gx[i] += weight * ((dF/dx)^T g)_i with g = gvec (slot order),
// and gtheta[0..5] (+)= weight * d(g.F)/d(eps_t, sigma_t). kAdjEnergy:
// gtheta (+)= weight * dU/d(eps_t, sigma_t). gtheta is overwritten when init
// is set, else accumulated. Block partial rows go to the first ring slot of
// the observable partials.
hipError_t launch_adjoint_pairs(const Launch &L, int mode, const void *gvec, double4 *gx, double weight,
                                double *gtheta, int init);

// Block rows of the parameter sums of one VJP pass (launch_adjoint_vjp_rows).
int adjoint_rows(const Geom &g);

// The VJP pass of the reverse sweep: gx[i] += weight * ((dF/dx)^T g)_i, and
// row b of rows (kNP doubles per block, adjoint_rows(g) blocks) becomes
// (init ? 0 : row) + weight * that block's parameter sums; the cell counters
// are cleared if the lists were rebuilt for `step`.
// The drift of the next (earlier) frame done by a VJP pass as each slot's
// gx becomes final: lv += scale * gx (none when scale == 0), gv_next = lv / m
// (the layout of gvec), and the displacement of that frame's records `rec`
// from the list reference folded into the rebuild word of `step`. The same
// arithmetic as kOpDriftCotangent with its displacement check.
struct AdjNext {
    double4 *lv;
    void *gv_next;
    double scale;
    int64_t step;
    const void *rec;
};
hipError_t launch_adjoint_vjp_rows(const Launch &L, const void *gvec, double4 *gx, double weight, double *rows,
                                   int init, int64_t step, int forced, const AdjNext *next);

// gtheta[0..5] = the sums of the block rows, in a fixed order.
hipError_t launch_adjoint_reduce(const Launch &L, const double *rows, double *gtheta);

// kOpDriftCotangent on (lx, lv, gvec); with disp, the displacement of the
// positions in record buffer L.cur from the list reference is folded into
// the rebuild decision of `step` in the same pass.
hipError_t launch_adjoint_drift(const Launch &L, double4 *lx, double4 *lv, void *gvec, double scale, int64_t step,
                                int disp);

// Clear the cell counters if the lists were rebuilt for `step` (in a forward
// run the step kernel does this).
hipError_t launch_adjoint_cells(const Launch &L, int64_t step, int forced);

hipError_t launch_adjoint_vec(const Launch &L, int op, const double *src_id, double *dst_id, double4 *a,
                              double4 *b, void *gvec, double scale, const double *dscale = nullptr);

// gtheta[0..5] += c * g[0..5] with c = *dc (device scalars).
hipError_t launch_theta_axpy(const Launch &L, const double *dc, const double *g, double *gtheta);


}  // namespace ljmd
