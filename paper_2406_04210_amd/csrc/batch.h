// batch.h -- launchers of the batched form: many independent one-species
// cubic systems (replicas of uneven size) stepped together, every kernel
// spanning all systems at once over a flattened work list.
#pragma once

#include "internal.h"

namespace ljmd {

// Per-step rebuild plan of a batch: which systems rebuild their lists this
// step, and the prefix sums that flatten their particles and cells.
struct BatchPlan {
    int32_t *due;        // [nsys] 1 if system s rebuilds this step
    int32_t *wl_sys;     // [nsys] systems that rebuild, in order
    int64_t *wl_poff;    // [nsys + 1] prefix of their particle counts
    int64_t *wl_coff;    // [nsys + 1] prefix of their cell counts
    int32_t *wl_count;   // [1] number of systems that rebuild
};

// Decide per system (forced, or its largest displacement exceeded skin/2),
// clear the other parity word, and compact the systems that rebuild.
hipError_t launch_batch_plan(const Launch &L, const SysC *sys, int nsys, const BatchPlan &bp, int64_t step,
                             int forced);
// Binning, canonical order and list build of the systems in the plan.
hipError_t launch_batch_bin(const Launch &L, const SysC *sys, const BatchPlan &bp, int64_t total_particles);
hipError_t launch_batch_canon(const Launch &L, const SysC *sys, const BatchPlan &bp, int64_t total_cells);
hipError_t launch_batch_nlist(const Launch &L, const SysC *sys, const BatchPlan &bp, int64_t total_cells);
// Exclusive scan of each system's cell counts into slot offsets (resort).
hipError_t launch_batch_scan(const Launch &L, const SysC *sys, int nsys);
// Gather into the new order and copy back, over every slot of the batch.
hipError_t launch_batch_resort_move(const Launch &L, int64_t ncell_total);
// Fused step of every system (FP32 + double-single).
hipError_t launch_batch_step(const Launch &L, const SysC *sys, const int32_t *sys_of_g16, int nblocks,
                             int64_t step, int forced, int mode, int slot);
hipError_t launch_batch_integrate(const Launch &L, const SysC *sys, const int32_t *sys_of_g16, int64_t nslots,
                                  int64_t step);
// State I/O in the caller's concatenated order, and per-system observables.
hipError_t launch_batch_set_state(const Launch &L, const SysC *sys, const int32_t *sys_of_g16, int64_t nslots,
                                  const double *x, const double *v, const int32_t *sp);
hipError_t launch_batch_get_state(const Launch &L, const SysC *sys, const int32_t *sys_of_g16, int64_t nslots,
                                  double *x, double *v, int32_t *img);
hipError_t launch_batch_get_forces(const Launch &L, const SysC *sys, const int32_t *sys_of_g16, int64_t nslots,
                                   double *f);
hipError_t launch_batch_obs(const Launch &L, const SysC *sys, int nsys, int slot, int64_t step, double *out);

}  // namespace ljmd
