/*
 * ljmd.h -- C ABI of the MI355X (gfx950) truncated Lennard-Jones MD hot path.
 *
 * The operations follow the problem statement of the paper (arXiv 2406.04210):
 * time stepping of N particles in a periodic box (Sec. 1) under a truncated
 * pair potential whose neighbours come from Verlet lists built by particle
 * binning (Sec. 3, "Code structure"), with the two velocity-Verlet half
 * steps "integrate" and "finalize" around the force evaluation (Sec. 3 and
 * Fig. 1), the common 12-6 Lennard-Jones potential (Sec. 4), truncated
 * forces (Sec. 5, "Truncated Force Performance Study"), list updates driven
 * by particle movement (same paragraph) and reductions/sorting (Sec. 4,
 * "Mixed Strategy").
 *
 * Conventions for every function below:
 *   - Units are reduced LJ units; host-facing arrays are float64 and indexed
 *     by the ORIGINAL particle id 0..n-1 (the library reorders particles
 *     internally along a space-filling curve and hides that order).
 *   - Array arguments marked "device" are device pointers on the GPU that
 *     owns the context; "host" pointers are ordinary host memory.
 *   - All device memory is CALLER-OWNED: the caller allocates one workspace
 *     of ljmd_workspace_size() bytes and passes it to ljmd_create(). The
 *     library never allocates or frees device memory.
 *   - Work is enqueued on the hip stream given to ljmd_create() and the
 *     calls return without synchronising, except those documented as
 *     synchronising (ljmd_set_state, ljmd_run, ljmd_minimize_sd,
 *     ljmd_vv_forward and ljmd_vv_backward wait once at their end to check
 *     the lists; ljmd_sync_status, ljmd_observables).
 *   - Return value: LJMD_OK (0) or a negative ljmd_status. Functions never
 *     abort or throw. Errors detected on the device (list or cell overflow,
 *     non-finite positions) are latched in the context; from then on no
 *     kernel changes the state, so no step ever runs on a truncated list.
 *     A list overflow is recovered by the calls that wait at their end: the
 *     lists grow in place, up to what the workspace holds, and the frozen
 *     steps are redone (bitwise as with room from the start: list entries
 *     keep their order at any capacity); LJMD_ENLIST only when the workspace
 *     is full. Other errors are reported by the next synchronising call.
 *     ljmd_last_error() describes the last error.
 *   - A context is not thread-safe; separate contexts are independent.
 */
#ifndef LJMD_H
#define LJMD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LJMD_ABI_VERSION 8

enum ljmd_status {
    LJMD_OK = 0,
    LJMD_EINVAL = -1,  /* bad argument or parameter */
    LJMD_ENOMEM = -2,  /* workspace smaller than ljmd_workspace_size() */
    LJMD_EHIP = -3,    /* a HIP runtime call failed */
    LJMD_EBOX = -4,    /* box edge < 2 * largest list radius (minimum image breaks) */
    LJMD_ENLIST = -5,  /* a neighbour list exceeded nbr_capacity */
    LJMD_ENAN = -6,    /* non-finite position detected */
    LJMD_ESTATE = -7,  /* call out of order (e.g. run before set_state) */
    LJMD_ECELL = -8    /* a cell exceeded cell_capacity */
};

/* The float types of the paper's modules (Sec. 3, "Code structure": double,
 * mixed and single precision). */
enum ljmd_precision {
    LJMD_FP64 = 0,     /* positions, velocities and pair arithmetic in FP64 */
    LJMD_FP32_DS = 1,  /* FP32 pair arithmetic and force accumulation; positions and
                          velocities carried as double-single (unevaluated sums of
                          two floats); FP64 only in the energy/virial reductions */
    LJMD_FP32 = 2      /* as LJMD_FP32_DS, but positions and velocities carried as
                          single floats: each half kick and drift is one binary32
                          product and one binary32 sum (the paper's GPU single
                          precision); lists and forces as LJMD_FP32_DS */
};

/* System and run parameters. Pair tables are indexed [a*2+b] for species
 * a, b in {0, 1}; with nspecies == 1 only entry [0] is read. */
typedef struct ljmd_params {
    int64_t n;              /* number of particles, >= 2 */
    double box[3];          /* periodic box edges (orthorhombic) */
    int32_t nspecies;       /* 1 or 2 */
    int32_t shift_energy;   /* 1: pair energy shifted to vanish at the cutoff */
    double eps[4];          /* LJ well depth per pair */
    double sigma[4];        /* LJ length per pair */
    double rcut[4];         /* absolute cutoff length per pair; +inf for every used pair
                               selects the untruncated all-pairs interaction (see below) */
    double mass[2];         /* mass per species */
    double skin;            /* Verlet skin: list radius = rcut + skin */
    double dt;              /* time step */
    int32_t sort_interval;  /* reorder along the space-filling curve every k steps; 0 = never */
    int32_t precision;      /* enum ljmd_precision */
    int32_t nbr_capacity;   /* list slots per particle to start with; 0 = automatic */
    int32_t cell_capacity;  /* particle slots per cell, <= 768; 0 = automatic */
    int32_t lanes;          /* lanes per particle in the force gather: 1,2,4,8,16; 0 = automatic */
    int32_t cell_split;     /* cells per list radius along each axis for binning and the
                               list build: 1 (cell edge >= r_L, 27-cell stencil) or 2 (edge
                               >= r_L / 2, 125-cell stencil); 0 = 1. The lists are the
                               same sets either way; ljmd_autotune times both */
    int32_t dim;            /* 3 (0 = 3) or 2 (the paper's modules take the dimension as a
                               template parameter, Sec. 3): with 2 the particles move in the
                               x-y plane; the z coordinates and velocities a caller passes
                               are taken as 0 and come back as 0, box[2] is no period of
                               the system but must still be a valid edge (>= 2 list radii;
                               pass box[0] for a square box so that the fixed-point fast
                               path applies), T = 2K/(2N-2), P = rho T + W/(2A) with the
                               area A = box[0] box[1]. The gradient calls and batches are
                               three-dimensional only */
    int32_t pad;            /* must be 0 */
} ljmd_params;

/* Per-step observable row written by ljmd_run into a device array:
 * [U, K, W, px, py, pz, rebuilt, step]  (rebuilt = 1 if the neighbour list
 * was rebuilt before the force evaluation of that step). U is the total
 * (shifted) potential energy, K the kinetic energy, W = sum_{i<j} r_ij.f_ij
 * the pair virial and p the total momentum. */
#define LJMD_NOBS 8

typedef struct ljmd_obs {
    double U, K, W;         /* potential, kinetic, virial */
    double P, T, E;         /* pressure rho T + W/(3V), temperature 2K/(3N-3), U+K */
    double p[3];            /* total momentum */
    int64_t step;           /* steps taken since ljmd_set_state */
    int64_t rebuilds;       /* list builds since ljmd_set_state (including the first) */
    int32_t max_fill;       /* longest neighbour list seen */
    int32_t nbr_capacity;   /* list capacity in use */
} ljmd_obs;

typedef struct ljmd_ctx ljmd_ctx;

/* Version of this ABI (LJMD_ABI_VERSION). */
int32_t ljmd_abi_version(void);

/* Validate parameters without touching a device. Returns LJMD_OK,
 * LJMD_EINVAL (bad value, NULL) or LJMD_EBOX (box too small for the
 * minimum-image convention with the largest list radius). Host only. */
int ljmd_check_params(const ljmd_params *p);

/* Bytes of device workspace needed for these parameters (pure host
 * arithmetic, resolves the automatic capacities). 0 if p is invalid. With
 * an automatic list capacity the size includes room for lists twice as long
 * as the initial capacity (up to 4096 slots), so that a list overflow can be
 * recovered in place; with an explicit nbr_capacity it holds exactly that
 * capacity. A larger workspace passed to ljmd_create is room for longer
 * lists (the lists lie at its end): ljmd_workspace_size of the same
 * parameters with nbr_capacity = C gives the bytes for lists of C slots.
 *
 * The untruncated all-pairs interaction (every used rcut = +inf: the
 * interaction of the paper's all-to-all study, Sec. 4 and Sec. 5 "GPU
 * Performance for All-to-All Interaction"): every pair of the minimum
 * image interacts through the unshifted 12-6 potential; there are no lists
 * or cells (skin, sort_interval, nbr_capacity, cell_capacity and lanes are
 * ignored, and any box edge is accepted; the single-precision paths need a
 * cubic box). ljmd_run, ljmd_set_state, ljmd_get_*, ljmd_observables and
 * the thermostat work as for the truncated potential; the list-based calls
 * (ljmd_neighbors, ljmd_minimize_sd, the gradients and rollouts, the tuner
 * and batches) return LJMD_EINVAL. */
size_t ljmd_workspace_size(const ljmd_params *p);

/* Cell grid the binning uses for these parameters: ncell[0..2] cells per
 * axis, each edge >= the largest list radius. Host only. */
int ljmd_cell_grid(const ljmd_params *p, int32_t ncell[3]);

/* Rank of every cell of an nx*ny*nz grid along a 3D Hilbert curve
 * (Skilling's transpose algorithm, AIP Conf. Proc. 707, 2004, on the
 * smallest 2^k cube that holds the grid; ranks are then compacted to
 * 0..nx*ny*nz-1). rank_out (host, nx*ny*nz int32) is indexed
 * (ix*ny + iy)*nz + iz. This order is the particle order after a
 * space-filling-curve resort (paper Sec. 4: sorting). Host only. */
int ljmd_hilbert_ranks(int32_t nx, int32_t ny, int32_t nz, int32_t *rank_out);

/* Create a context on the current HIP device. dev_workspace (device) must
 * hold >= ljmd_workspace_size(p) bytes, 256-byte aligned, and outlive the
 * context; hip_stream is a hipStream_t (NULL = default stream). The context
 * keeps copies of p. Enqueues workspace initialisation on the stream. */
int ljmd_create(const ljmd_params *p, void *dev_workspace, size_t bytes, void *hip_stream,
                ljmd_ctx **out);

/* Release the host-side context (device memory stays the caller's). */
int ljmd_destroy(ljmd_ctx *ctx);

/* Load a state: x, v (device, n*3 float64, by id; x need not be wrapped)
 * and species (device, n int32 in [0, nspecies)). Wraps positions into the
 * box, sorts particles along the space-filling curve, builds the lists and
 * evaluates the forces of this state (the "force" slot before the first
 * "integrate"). Resets the step and rebuild counters. Waits for the device
 * at the end (a list overflow of the first build is recovered). */
int ljmd_set_state(ljmd_ctx *ctx, const double *x, const double *v, const int32_t *species);

/* Read the state by id: x (wrapped into [0, L)), v (device, n*3 float64)
 * and img (device, n*3 int32 periodic image counters, so that the
 * unwrapped position is x + img * L). Any pointer may be NULL. */
int ljmd_get_state(ljmd_ctx *ctx, double *x, double *v, int32_t *img);

/* Forces of the current state by id (device, n*3 float64). */
int ljmd_get_forces(ljmd_ctx *ctx, double *f);

/* Advance nsteps velocity-Verlet steps: per step, half kick + drift
 * ("integrate"), list rebuild if any particle moved more than skin/2 since
 * the last build (strict >) or a resort is due, force evaluation, half kick
 * ("finalize"). obs_dev (device, nsteps * LJMD_NOBS float64, or NULL)
 * receives one observable row per step. Enqueues every step, then waits
 * for the device once: if a list overflowed, the lists grow and the steps
 * from the one that stopped are redone (their observable rows rewritten). */
int ljmd_run(ljmd_ctx *ctx, int64_t nsteps, double *obs_dev);

/* Steepest descent to relax a starting configuration (random positions
 * overlap): per iteration, forces of the truncated potential with every pair
 * distance clamped from below at clamp * sigma_ab (this mode only), then
 * x_i += max_disp * F_i / max_j |F_j|, so no particle moves more than
 * max_disp; lists follow the half-skin rebuild rule. Velocities are left
 * as they are; at the end the lists are rebuilt (with a resort) and the
 * unclamped forces of the relaxed state evaluated, as after ljmd_set_state.
 * fmax_dev (device, nsteps float64, or NULL) receives max_j |F_j| at the
 * start of every iteration. Requires a loaded state. Asynchronous. */
int ljmd_minimize_sd(ljmd_ctx *ctx, int32_t nsteps, double max_disp, double clamp,
                     double *fmax_dev);

/* Neighbour lists of the last build, by id: cnt (device, n int32) list
 * lengths and ids (device, n*cap int32, row id holds the first min(cnt, cap)
 * partner ids in list order). For tests and inspection. */
int ljmd_neighbors(ljmd_ctx *ctx, int32_t *cnt, int32_t *ids, int32_t cap);

/* Synchronise the stream and return the first latched device error
 * (LJMD_ENLIST, LJMD_ECELL, LJMD_ENAN) or LJMD_OK. */
int ljmd_sync_status(ljmd_ctx *ctx);

/* Synchronise and fill *out with the observables of the current step. */
int ljmd_observables(ljmd_ctx *ctx, ljmd_obs *out);

/* Stochastic velocity resampling, the Andersen-like ("Boltzmann")
 * thermostat that the paper combines with velocity Verlet (Sec. 4, "Code
 * migration"; its truncated-force study varies the temperature, Sec. 5).
 * After the second half kick of every step s of ljmd_run, each particle
 * collides with probability rate * dt and then takes a new velocity
 * sqrt(temperature / m) z, z three standard normal deviates. The draws come
 * from the counter-based generator Philox4x32-10 (Salmon et al., SC'11)
 * keyed by seed, with counters (id, s mod 2^32, s / 2^32, 0) and
 * (id, s mod 2^32, s / 2^32, 1) for the particle's original id: the particle
 * collides iff the first word is below floor(rate dt 2^32), and z comes from
 * the Box-Muller transform of the word pairs (w1, w2) and (w3, w4), a word u
 * read as (u + 1/2) 2^-32. Results therefore depend only on the seed and
 * not on the particle order or the launch shape. rate = 0 switches it off
 * (the default). Host-side setting, takes effect from the next step;
 * LJMD_EINVAL for negative or non-finite values. ljmd_vv_forward refuses
 * to run while it is on (the dynamics would not be differentiable). */
int ljmd_set_thermostat(ljmd_ctx *ctx, double temperature, double rate, uint64_t seed);

/* Kernel timing with HIP events on the context's stream for every launch
 * of each kernel family during ljmd_run: [0] the fused step kernel (forces
 * + velocity Verlet + reductions; its events are stamped by the dispatch
 * itself through the extended launch, so they hold the kernel's own start
 * and end; the other families are bracketed by recorded events, which
 * add the marker packets' cost), [1] the rebuild sequence
 * (binning, canonical order, list build -- launched every step, working
 * only when a rebuild is due), [2] the space-filling-curve resort,
 * [3] everything else (integrate at run start, observable flushes),
 * [4] the adjoint pair pass (force VJP) of ljmd_vv_backward and
 * ljmd_force_vjp. ljmd_set_profiling(ctx, 1) starts accumulating (and
 * clears the sums); ljmd_kernel_times synchronises and writes total
 * milliseconds ms[5] and launch counts count[5] (host arrays). Events cost a
 * few microseconds of enqueue work per launch; leave profiling off for
 * throughput runs. */
#define LJMD_NKT 5
int ljmd_set_profiling(ljmd_ctx *ctx, int enable);
int ljmd_kernel_times(ljmd_ctx *ctx, double ms[LJMD_NKT], int64_t count[LJMD_NKT]);

/* ---- Gradients ------------------------------------------------------------
 * The paper computes no gradients; these differentiate its truncated 12-6
 * pair potential (Sec. 4, Sec. 5) and its velocity-Verlet step (Sec. 3,
 * Fig. 1). Only pairs inside the cutoff contribute: the force jump at r_c
 * adds nothing, so every gradient is that of the truncated function almost
 * everywhere. The cutoff r_c is a fixed length (it does not scale with
 * sigma); the energy shift moves with eps and sigma. Parameter gradients are
 * six float64 in the order
 *   [d/d eps_AA, d/d eps_AB, d/d eps_BB, d/d sigma_AA, d/d sigma_AB, d/d sigma_BB]
 * (one species: entries 0 and 3, the rest 0). Pair arithmetic runs in the
 * context's precision; parameter sums are float64 in a fixed order. */

/* Replace eps and sigma (host, 4 entries each, the ljmd_params layout
 * [AA, AB, BA, BB] with AB == BA; cutoffs, masses and skin stay). With a
 * state loaded, its forces and observables are re-evaluated (the lists
 * depend only on cutoffs and skin and are kept). Asynchronous. */
int ljmd_set_pair_params(ljmd_ctx *ctx, const double eps[4], const double sigma[4]);

/* Force vector-Jacobian product at the current state: for a cotangent g
 * (device, n*3 float64, by id) writes gx = (dF/dx)^T g (device, n*3
 * float64, by id; dF/dx is minus the Hessian of U) and gtheta =
 * d(g.F)/d(eps, sigma) (device, 6 float64). g is read before gx is
 * written, so they may alias. Uses the workspace's scratch area.
 * Asynchronous. */
int ljmd_force_vjp(ljmd_ctx *ctx, const double *g, double *gx, double *gtheta);

/* Parameter gradient of the potential energy at the current state: gtheta
 * (device, 6 float64) = dU/d(eps, sigma). The position gradient of U is -F
 * (ljmd_get_forces). Asynchronous. */
int ljmd_energy_grad(ljmd_ctx *ctx, double *gtheta);

/* Flags of a differentiable rollout. LJMD_ADJ_STORE_ALL: the forward run
 * keeps every position frame and the reverse sweep reads them instead of
 * recomputing segments (more memory, no recompute; same results bit for
 * bit, since a recompute repeats the forward run exactly). */
#define LJMD_ADJ_STORE_ALL 1

/* Device bytes ljmd_vv_forward needs for nsteps >= 1 steps with a
 * checkpoint every ckpt_every >= 1 steps (0 if an argument is invalid):
 * ceil(nsteps / ckpt_every) + 1 state copies, ckpt_every + 1 position
 * frames for the recompute (nsteps + 1 with LJMD_ADJ_STORE_ALL, plus one
 * int32 rebuild marker per step when ckpt_every <= 64), four
 * per-particle adjoint vectors and 64 bytes of parameter-gradient sums per
 * 64 particles. */
size_t ljmd_adjoint_workspace_size(const ljmd_params *p, int32_t nsteps, int32_t ckpt_every,
                                   int32_t flags);

/* Differentiable rollout: nsteps velocity-Verlet steps from the current
 * state, as ljmd_run except that (a) before every ckpt_every-th step the
 * state is stored in adj_ws and that step's list build is forced, (b) no
 * space-filling-curve resort happens, (c) the lists are rebuilt at the final
 * state. With (a) the recompute of a segment from its checkpoint repeats
 * the forward run bit for bit. adj_ws (device, >= ljmd_adjoint_workspace_size
 * bytes for the same arguments, 256-byte aligned) stays the caller's and
 * must live until the matching ljmd_vv_backward. flags: 0 or
 * LJMD_ADJ_STORE_ALL. obs_dev as in ljmd_run. Asynchronous. */
int ljmd_vv_forward(ljmd_ctx *ctx, int32_t nsteps, int32_t ckpt_every, int32_t flags, void *adj_ws,
                    size_t bytes, double *obs_dev);

/* Reverse sweep of the last ljmd_vv_forward. From lam_x = dL/dx_N and
 * lam_v = dL/dv_N (device, n*3 float64, by id) for a loss L of the final
 * state, writes gx0 = dL/dx_0 and gv0 = dL/dv_0 (device, n*3 float64, by
 * id; may alias lam_x, lam_v) and gtheta = dL/d(eps, sigma) through the
 * dynamics (device, 6 float64). gU (device, one float64, or NULL) is the
 * loss's weight dL/dU_N of the final potential energy U(x_N; theta): the
 * sweep then starts from lam_x - gU F(x_N) and gtheta also receives
 * gU dU/dtheta at x_N, so lam_x and lam_v hold only the rest of the loss. Segments are taken last first: each is
 * recomputed from its checkpoint (or read, with LJMD_ADJ_STORE_ALL) and its
 * frames swept backwards with one force VJP per frame (cotangent lam_v / m,
 * weight dt/2 at x_N and x_0, dt between). Each segment's sweep starts
 * from the list of the forward run's last build in it (for segments of at
 * most 64 steps; longer ones build the list afresh at the first frame), and
 * lists are built again whenever a frame is more than skin/2 from the last
 * build. With LJMD_ADJ_STORE_ALL and segments of at most 64 steps the call
 * waits for the device once (it reads the forward run's rebuild markers).
 * Leaves the context at the final state, as
 * ljmd_vv_forward did. LJMD_ESTATE if no rollout is recorded or the state
 * changed since. Asynchronous. */
int ljmd_vv_backward(ljmd_ctx *ctx, const double *lam_x, const double *lam_v, const double *gU,
                     double *gx0, double *gv0, double *gtheta);

/* ---- Autotuning -------------------------------------------------------------
 * The paper picks launch configurations per device (Sec. 4, 5); this
 * library's tuner times short runs of a system on the device for each
 * candidate cell size (cell_split 1 and 2: cells of edge >= r_L or >= r_L/2)
 * and force-gather shape (lanes per particle 1, 2, 4, 8, 16), keeps the
 * fastest pair, and sizes the list capacity from the longest list seen
 * (1.25x, at least +24, in units of 16). Results are cached as JSON lines
 * in cache_path (may be NULL) under a key of device architecture,
 * dimension, precision, species count, size (power of two), density (to
 * 0.05) and list radius; a cached key is returned without timing. */
typedef struct ljmd_tuning {
    int32_t lanes;          /* fastest lanes per particle */
    int32_t nbr_capacity;   /* suggested list capacity */
    int32_t cell_capacity;  /* cell capacity used (0 = automatic) */
    int32_t max_fill;       /* longest list seen while timing */
    double ms_per_step;     /* time per step of the fastest shape */
    int32_t from_cache;     /* 1 if read from the cache */
    int32_t cell_split;     /* fastest cell size (ljmd_params.cell_split) */
} ljmd_tuning;

/* Device bytes the tuner needs for p (the largest workspace of its
 * candidates; 0 if p is invalid). */
size_t ljmd_autotune_workspace_size(const ljmd_params *p);

/* Tune for the state x, v, species (device, as ljmd_set_state) with steps
 * timed steps per candidate (after 10 warm-up steps), using dev_workspace
 * (>= ljmd_autotune_workspace_size bytes) for temporary contexts. Writes the
 * result to *out (host). Synchronises. */
int ljmd_autotune(const ljmd_params *p, const double *x, const double *v, const int32_t *species,
                  void *dev_workspace, size_t bytes, void *hip_stream, int32_t steps,
                  const char *cache_path, ljmd_tuning *out);

/* ---- Batches of systems ------------------------------------------------------
 * Many independent one-species systems (replicas) of uneven size in cubic
 * boxes, stepped together: every kernel of a step spans all of them at once
 * over a flattened list of particles, cells and blocks, and each system keeps
 * its own list-rebuild decisions and observables. A system's trajectory is
 * the one it has as a single box with the same parameters (the batch is a
 * layout, not an approximation). Shared parameters (potential, masses, dt,
 * skin, sort_interval, lanes, capacities) come from one ljmd_params whose n
 * and box are ignored; nspecies must be 1 and precision LJMD_FP32_DS. The
 * paper runs one box per launch; batching is this library's addition. */
typedef struct ljmd_batch ljmd_batch;

typedef struct {
    int64_t n;   /* particles */
    double box;  /* edge of the cubic box */
} ljmd_system;

/* Device bytes a batch of these systems needs (0 if any is invalid). */
size_t ljmd_batch_workspace_size(const ljmd_params *shared, const ljmd_system *sys, int32_t nsys);

/* Create a batch on the current device (workspace as for ljmd_create).
 * Enqueues initialisation on the stream and waits for it. */
int ljmd_batch_create(const ljmd_params *shared, const ljmd_system *sys, int32_t nsys, void *dev_workspace,
                      size_t bytes, void *hip_stream, ljmd_batch **out);

int ljmd_batch_destroy(ljmd_batch *b);

/* Load every system: x, v (device, sum(n)*3 float64) and species (device,
 * sum(n) int32), system k's rows following system k-1's. Then, per system,
 * what ljmd_set_state does. */
int ljmd_batch_set_state(ljmd_batch *b, const double *x, const double *v, const int32_t *species);

/* Advance every system nsteps (as ljmd_run). obs_dev (device, nsys *
 * LJMD_NOBS float64, or NULL) receives each system's observables of the last
 * step, with column 6 holding its list builds so far. Asynchronous.
 * Whole resort periods (sort_interval steps, doubled when odd; 64 without
 * resorts) that start at a multiple of the period and do not hold the run's
 * last step are replayed from a HIP graph captured on first use (one per
 * parity of the record buffers, kept until ljmd_batch_destroy); the results
 * are bitwise those of launching every step. The stream must not be under
 * capture by the caller while graphs are enabled. */
int ljmd_batch_run(ljmd_batch *b, int64_t nsteps, double *obs_dev);

/* Enable (default) or disable the graph replay of ljmd_batch_run. */
int ljmd_batch_use_graphs(ljmd_batch *b, int32_t enable);

/* State and forces in the concatenated row order of ljmd_batch_set_state. */
int ljmd_batch_get_state(ljmd_batch *b, double *x, double *v, int32_t *img);
int ljmd_batch_get_forces(ljmd_batch *b, double *f);

/* Synchronise and copy each system's last observable row to obs_host (host,
 * nsys * LJMD_NOBS float64). */
int ljmd_batch_observables(ljmd_batch *b, double *obs_host);

/* Synchronise; the first latched device error of any system, or LJMD_OK. */
int ljmd_batch_sync_status(ljmd_batch *b);

/* Synchronise; *out (host) receives the longest neighbour list of any
 * system as built last. */
int ljmd_batch_max_fill(ljmd_batch *b, int32_t *out);

/* Batch autotuner: as ljmd_autotune, timed on the whole batch. For each
 * lanes candidate a batch of these systems is created in dev_workspace
 * (>= ljmd_batch_autotune_workspace_size bytes), loaded with x, v, species
 * (device, as ljmd_batch_set_state), warmed up 10 steps and timed over
 * steps steps; the fastest is kept, and the list capacity is sized from the
 * longest list seen. Cached under a key of the device, the number of
 * systems, their total size and mean density. Synchronises. */
size_t ljmd_batch_autotune_workspace_size(const ljmd_params *shared, const ljmd_system *sys, int32_t nsys);
int ljmd_batch_autotune(const ljmd_params *shared, const ljmd_system *sys, int32_t nsys, const double *x,
                        const double *v, const int32_t *species, void *dev_workspace, size_t bytes,
                        void *hip_stream, int32_t steps, const char *cache_path, ljmd_tuning *out);

const char *ljmd_batch_last_error(const ljmd_batch *b);

/* ---- One-shot brute-force forces --------------------------------------------
 * Forces, energy and virial of one configuration by the sum over all pairs
 * of the minimum image: the definition of the truncated, shifted pair sum
 * that the Verlet-list path reaches (paper Sec. 3 "Code structure", Sec. 5
 * "Truncated Force Performance Study"), or with every used rcut = +inf the
 * untruncated all-to-all interaction (Sec. 4 "Code migration", Sec. 5 "GPU
 * Performance for All-to-All Interaction"). O(N^2) work, no lists, no state:
 * a GPU checker for small systems and the all-pairs evaluation itself.
 * p as for ljmd_create (n, box, pair tables, nspecies, precision; the
 * single-precision paths need a cubic box and evaluate the binary32 pair
 * arithmetic of the step kernels on the fixed-point positions); x (device,
 * n*3 float64, any image), species (device, n int32) -> f (device, n*3
 * float64, same order) and uw (device, 2 float64: U = sum phi_s, W = sum
 * r_ij.f_ij over pairs i < j). ws (device, >= ljmd_brute_workspace_size(p)
 * bytes, 256-byte aligned) is scratch, the caller's. Asynchronous on
 * hip_stream. Errors: LJMD_EINVAL / LJMD_EBOX (parameters), LJMD_ENOMEM
 * (workspace too small), LJMD_EHIP; text in ljmd_last_error(NULL). */
size_t ljmd_brute_workspace_size(const ljmd_params *p);
int ljmd_brute_forces(const ljmd_params *p, const double *x, const int32_t *species, double *f, double *uw,
                      void *dev_workspace, size_t bytes, void *hip_stream);

/* ---- Allocation-free variant -----------------------------------------------
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * evaluation as ljmd_brute_forces, with the same arguments minus the
 * workspace. Its scratch is a fixed device array of
 * LJMD_BRUTE_STATIC_SCRATCH_BYTES inside the library (one per GPU, held
 * until the process ends); the call allocates and frees nothing. Sizes
 * whose scratch (ljmd_brute_workspace_size) exceeds it are rejected with
 * LJMD_ENOMEM (above about 349,000 particles in single precision, 208,000
 * in FP64). Every call on a GPU shares that GPU's array: calls that overlap on
 * one GPU (other streams, other threads) race and must be serialised by the
 * caller; calls on one stream are ordered. Nothing in the array needs to
 * start at zero. Errors as ljmd_brute_forces. */
#define LJMD_BRUTE_STATIC_SCRATCH_BYTES (16u << 20)
size_t ljmd_brute_static_scratch_bytes(void);
int ljmd_brute_forces_noalloc(const ljmd_params *p, const double *x, const int32_t *species, double *f, double *uw,
                              void *hip_stream);

/* Text of the last error of ctx (or of the last failed create when ctx is
 * NULL). The pointer stays valid until the next call on ctx. */
const char *ljmd_last_error(const ljmd_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* LJMD_H */
