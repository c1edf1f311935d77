/*
 * oracle.c -- plain, slow, obviously correct CPU reference for the truncated
 * Lennard-Jones molecular-dynamics hot path.
 *
 * TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke entry point and the
 * CPU-baseline leg of the benchmark may load this library. It shares no code,
 * header, table or constant with the GPU library, and the GPU library never
 * calls it.
 *
 * What it computes (paper: Sec. 1 time-stepping of Hamiltonian dynamics in a
 * periodic box; Sec. 3 "Code structure": truncated pair potential, Verlet
 * neighbour lists built from particle binning, velocity-Verlet half steps
 * "integrate"/"finalize"; Sec. 4: the common Lennard-Jones potential):
 *
 *   phi(r)    = 4 eps [ (sigma/r)^12 - (sigma/r)^6 ]                (textbook LJ)
 *   phi_s(r)  = phi(r) - phi(r_c)  for r < r_c, else 0   (truncated, energy-shifted)
 *   f_ij      = fs(r) * r_ij,  fs = 24 eps [ 2 (sigma/r)^12 - (sigma/r)^6 ] / r^2
 *   r_ij      = x_i - x_j under the minimum image  d - L rint(d / L)
 *   U = sum_{i<j} phi_s,  W = sum_{i<j} fs r^2,  K = sum m v^2 / 2
 *
 * Everything is IEEE FP64. Two functions additionally reproduce, in IEEE
 * binary32 with explicit fused multiply-adds, the stated FP32 operation
 * sequence that the single-precision path uses to decide list membership
 * (double-single split, fixed-point image coordinate, displacement, r^2), so
 * that neighbour sets can be compared exactly, and one evaluates the FP64
 * forces of the fixed-point positions that sequence produces. Compile with
 * -ffp-contract=off so that no other fusion happens.
 *
 * Also here: the stochastic velocity-resampling ("Boltzmann", Andersen-like)
 * thermostat the paper combines with velocity Verlet (Sec. 4), drawing from
 * the counter-based Philox4x32-10 generator (Salmon et al., SC'11); and, with
 * infinite cutoffs, the untruncated all-pairs interaction the port started
 * from (Sec. 4, Sec. 5 "GPU Performance for All-to-All Interaction"): every
 * function below accepts rcut = +inf (no shift, all pairs interact).
 */
#define _POSIX_C_SOURCE 199309L  /* clock_gettime */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Monotonic wall clock in seconds (timing of the CPU baseline). */
static double wall_seconds(void) {
    struct timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}

/* Parameters of one system (mirrored by a ctypes Structure in __init__.py). */
typedef struct {
    int32_t nspecies;       /* 1 or 2 */
    int32_t shift_energy;   /* 1: subtract phi(r_c) inside the cutoff */
    double eps[4];          /* [a*2+b] */
    double sigma[4];
    double rcut[4];         /* absolute cutoff length per pair */
    double mass[2];
    double skin;            /* list radius = rcut + skin */
    double dt;
} olj_t;

static int pair_index(const olj_t *p, int a, int b) {
    return p->nspecies == 1 ? 0 : a * 2 + b;
}

/* ---------------------------------------------------------------- O1 ---- */

/* Unshifted 12-6 Lennard-Jones potential at distance r. */
double oracle_phi(double r, double eps, double sigma) {
    double sr = sigma / r;
    double sr6 = sr * sr * sr * sr * sr * sr;
    return 4.0 * eps * (sr6 * sr6 - sr6);
}

/* fs(r) = -phi'(r) / r, so that the force on i from j is fs * (x_i - x_j). */
double oracle_fscalar(double r, double eps, double sigma) {
    double sr = sigma / r;
    double sr6 = sr * sr * sr * sr * sr * sr;
    return 24.0 * eps * (2.0 * sr6 * sr6 - sr6) / (r * r);
}

/* Truncated (and, if requested, energy-shifted) pair energy of pair type ab. */
double oracle_pair_energy(double r, int ab, const olj_t *p) {
    if (r >= p->rcut[ab]) return 0.0;
    double e = oracle_phi(r, p->eps[ab], p->sigma[ab]);
    if (p->shift_energy) e -= oracle_phi(p->rcut[ab], p->eps[ab], p->sigma[ab]);
    return e;
}

/* Truncated force scalar: fs(r) inside the cutoff, 0 outside (the force is
 * not shifted, so it jumps at r_c). */
double oracle_pair_fscalar(double r, int ab, const olj_t *p) {
    if (r >= p->rcut[ab]) return 0.0;
    return oracle_fscalar(r, p->eps[ab], p->sigma[ab]);
}

/* Minimum-image displacement x_i - x_j for any (wrapped or not) positions. */
static void min_image(const double *xi, const double *xj, const double *box, double d[3]) {
    for (int k = 0; k < 3; ++k) {
        double t = xi[k] - xj[k];
        d[k] = t - box[k] * rint(t / box[k]);
    }
}

/* ---------------------------------------------------------------- O2 ---- */

/* Brute force over all pairs i < j (the untruncated-loop definition with the
 * cutoff applied). f: n*3 output. out[0] = U, out[1] = W. */
void oracle_forces_brute(int64_t n, const double *x, const int32_t *sp, const double *box,
                         const olj_t *p, double *f, double *out) {
    /* U and W sum up to n(n-1)/2 terms (2e6 for the untruncated 2,000-particle
     * system), many of them equal on a lattice, so their FP64 roundings do not
     * cancel: a double accumulator drifts by several 1e-12 of the sum. The
     * two sums are carried in long double (64-bit significand) and rounded
     * once at the end. */
    long double U = 0.0L, W = 0.0L;
    memset(f, 0, sizeof(double) * 3 * (size_t)n);
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t j = i + 1; j < n; ++j) {
            double d[3];
            min_image(x + 3 * i, x + 3 * j, box, d);
            double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
            int ab = pair_index(p, sp[i], sp[j]);
            if (r >= p->rcut[ab]) continue;
            double fs = oracle_pair_fscalar(r, ab, p);
            for (int k = 0; k < 3; ++k) {
                f[3 * i + k] += fs * d[k];
                f[3 * j + k] -= fs * d[k];
            }
            U += (long double)oracle_pair_energy(r, ab, p);
            W += (long double)(fs * r * r);
        }
    }
    out[0] = (double)U;
    out[1] = (double)W;
}

/* ---------------------------------------------------------------- O3 ---- */

/* Wrap one coordinate into [0, L). */
static double wrap1(double x, double L) {
    double w = x - L * floor(x / L);
    if (w >= L) w -= L;
    return w;
}

/* FP64 list criterion: the stated double-precision operation sequence.
 * d = w_i - w_j; d -= L rint(d / L); r2 = fma(dz,dz, fma(dy,dy, dx*dx)). */
static double r2_fp64(const double *wi, const double *wj, const double *box) {
    double d[3];
    for (int k = 0; k < 3; ++k) {
        double t = wi[k] - wj[k];
        double m = rint(t / box[k]);
        d[k] = t - box[k] * m;
    }
    return fma(d[2], d[2], fma(d[1], d[1], d[0] * d[0]));
}

/* FP32 operation sequence of the single-precision path.
 * 1) double-single split of a wrapped FP64 coordinate: hi = (float) w,
 *    lo = (float)(w - hi)  (Dekker's split into an unevaluated float sum).
 * 2) fixed-point image coordinate q = round((hi + lo) * 2^32 / L) mod 2^32,
 *    evaluated with an error-free product (TwoProduct by fma) in binary32.
 * 3) displacement from the wrapping difference of two q's, converted to
 *    binary32 and scaled by the single-float quantum (float)(L * 2^-32):
 *    one rounding of the product.
 * 4) list membership: r^2 = fma(dz, dz, fma(dy, dy, dx * dx)) in binary32
 *    and 0 < r^2 < (float) r_L^2. In a cubic box the displacements are the
 *    converted differences themselves (no scaling), compared with
 *    (float)(r_L^2 / (L 2^-32)^2), the squared list radius in squared
 *    quanta computed in FP64 and rounded once.                              */
void oracle_ds_split(double w, float *hi, float *lo) {
    float h = (float)w;
    *hi = h;
    *lo = (float)(w - (double)h);
}

uint32_t oracle_q_from_ds(float hi, float lo, double L) {
    double S = 4294967296.0 / L;
    float S_hi = (float)S;
    float S_lo = (float)(S - (double)S_hi);
    float p = hi * S_hi;
    float e = fmaf(hi, S_hi, -p);
    float a = hi * S_lo;
    float b = lo * S_hi;
    float c = a + b;
    float t = e + c;
    float pi = floorf(p);
    float pf = p - pi;
    float u = pf + t;
    int64_t q = (int64_t)pi + (int64_t)(int32_t)rintf(u);
    return (uint32_t)(uint64_t)q;
}

float oracle_disp_q(uint32_t qi, uint32_t qj, double L) {
    float qs = (float)(L / 4294967296.0);
    int32_t dq = (int32_t)(qi - qj);
    return (float)dq * qs;
}

static float r2_fp32(const uint32_t *qi, const uint32_t *qj, const double *box) {
    float dx = oracle_disp_q(qi[0], qj[0], box[0]);
    float dy = oracle_disp_q(qi[1], qj[1], box[1]);
    float dz = oracle_disp_q(qi[2], qj[2], box[2]);
    return fmaf(dz, dz, fmaf(dy, dy, dx * dx));
}

/* Step 4 in a cubic box: r^2 in squared quanta. */
static float r2_fp32_quanta(const uint32_t *qi, const uint32_t *qj) {
    float dx = (float)(int32_t)(qi[0] - qj[0]);
    float dy = (float)(int32_t)(qi[1] - qj[1]);
    float dz = (float)(int32_t)(qi[2] - qj[2]);
    return fmaf(dz, dz, fmaf(dy, dy, dx * dx));
}

/* Full Verlet lists {j : 0 < r_ij^2 < (rcut_ab + skin)^2} by particle index
 * (a particle is never its own partner, nor is one at exactly its position),
 * built with cell binning (cells of edge >= the largest list radius; a
 * particle's partners then lie in the 27 surrounding cells). With fewer than
 * three cells along an axis every particle is a candidate (plain all-pairs).
 * mode 0: FP64 criterion; mode 1: the FP32 sequence above (step 4).
 * cnt[i] = list length; nbr[i*cap + k] = k-th partner (first cap stored).
 * Returns the largest list length (may exceed cap, in which case the lists
 * are truncated and the caller must retry with a larger cap). */
int32_t oracle_build_lists(int64_t n, const double *x, const int32_t *sp, const double *box,
                           const olj_t *p, int32_t mode, int32_t cap, int32_t *cnt, int32_t *nbr) {
    double rl_max = 0.0;
    double rl2[4];
    float rl2f[4];
    const int cubic = box[0] == box[1] && box[1] == box[2];
    const double quantum = box[0] / 4294967296.0;
    for (int ab = 0; ab < 4; ++ab) {
        double rl = p->rcut[ab] + p->skin;
        rl2[ab] = rl * rl;
        rl2f[ab] = cubic ? (float)(rl * rl / (quantum * quantum)) : (float)(rl * rl);
        int used = p->nspecies == 2 || ab == 0;
        if (used && rl > rl_max) rl_max = rl;
    }
    double *w = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    uint32_t *q = (uint32_t *)malloc(sizeof(uint32_t) * 3 * (size_t)n);
    for (int64_t i = 0; i < n; ++i)
        for (int k = 0; k < 3; ++k) {
            w[3 * i + k] = wrap1(x[3 * i + k], box[k]);
            float hi, lo;
            oracle_ds_split(w[3 * i + k], &hi, &lo);
            q[3 * i + k] = oracle_q_from_ds(hi, lo, box[k]);
        }
    int nc[3];
    int brute = 0;
    for (int k = 0; k < 3; ++k) {
        nc[k] = (int)floor(box[k] / (rl_max * (1.0 + 1e-9)));
        if (nc[k] < 3) brute = 1;
    }
    int64_t ncell = brute ? 1 : (int64_t)nc[0] * nc[1] * nc[2];
    int64_t *cell_of = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    int64_t *start = (int64_t *)calloc((size_t)ncell + 1, sizeof(int64_t));
    int64_t *members = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    for (int64_t i = 0; i < n; ++i) {
        int64_t c = 0;
        if (!brute) {
            int ci[3];
            for (int k = 0; k < 3; ++k) {
                ci[k] = (int)floor(w[3 * i + k] / box[k] * nc[k]);
                if (ci[k] >= nc[k]) ci[k] = nc[k] - 1;
                if (ci[k] < 0) ci[k] = 0;
            }
            c = ((int64_t)ci[0] * nc[1] + ci[1]) * nc[2] + ci[2];
        }
        cell_of[i] = c;
        start[c + 1]++;
    }
    for (int64_t c = 0; c < ncell; ++c) start[c + 1] += start[c];
    {
        int64_t *fill = (int64_t *)calloc((size_t)ncell, sizeof(int64_t));
        for (int64_t i = 0; i < n; ++i) {  /* increasing index: stable */
            int64_t c = cell_of[i];
            members[start[c] + fill[c]++] = i;
        }
        free(fill);
    }
    int32_t maxcnt = 0;
#pragma omp parallel for schedule(dynamic, 256) reduction(max : maxcnt)
    for (int64_t i = 0; i < n; ++i) {
        int32_t k = 0;
        int64_t cells[27];
        int ncand = 0;
        if (brute) {
            cells[0] = 0;
            ncand = 1;
        } else {
            int64_t c = cell_of[i];
            int cz = (int)(c % nc[2]), cy = (int)((c / nc[2]) % nc[1]), cx = (int)(c / ((int64_t)nc[1] * nc[2]));
            for (int dx = -1; dx <= 1; ++dx)
                for (int dy = -1; dy <= 1; ++dy)
                    for (int dz = -1; dz <= 1; ++dz) {
                        int ax = (cx + dx + nc[0]) % nc[0];
                        int ay = (cy + dy + nc[1]) % nc[1];
                        int az = (cz + dz + nc[2]) % nc[2];
                        cells[ncand++] = ((int64_t)ax * nc[1] + ay) * nc[2] + az;
                    }
        }
        for (int s = 0; s < ncand; ++s) {
            int64_t c = cells[s];
            for (int64_t m = start[c]; m < start[c + 1]; ++m) {
                int64_t j = members[m];
                if (j == i) continue;
                int ab = pair_index(p, sp[i], sp[j]);
                int in;
                if (mode == 0) {
                    double r2 = r2_fp64(w + 3 * i, w + 3 * j, box);
                    in = r2 > 0.0 && r2 < rl2[ab];
                } else {
                    float r2 = cubic ? r2_fp32_quanta(q + 3 * i, q + 3 * j) : r2_fp32(q + 3 * i, q + 3 * j, box);
                    in = r2 > 0.0f && r2 < rl2f[ab];
                }
                if (in) {
                    if (k < cap) nbr[(size_t)i * cap + k] = (int32_t)j;
                    k++;
                }
            }
        }
        cnt[i] = k;
        if (k > maxcnt) maxcnt = k;
    }
    free(w);
    free(q);
    free(cell_of);
    free(start);
    free(members);
    return maxcnt;
}

/* ---------------------------------------------------------------- O4 ---- */

/* Forces, energy and virial from full Verlet lists: f_i = sum_j fs r_ij over
 * list partners with r < r_c; each pair appears in both lists, so U and W
 * take half of every list term. out = [U, W]. */
void oracle_forces_list(int64_t n, const double *x, const int32_t *sp, const double *box,
                        const olj_t *p, int32_t cap, const int32_t *cnt, const int32_t *nbr,
                        double *f, double *out) {
    double U = 0.0, W = 0.0;
#pragma omp parallel for schedule(static) reduction(+ : U, W)
    for (int64_t i = 0; i < n; ++i) {
        double fi[3] = {0.0, 0.0, 0.0};
        double ui = 0.0, wi = 0.0;
        int32_t m = cnt[i] < cap ? cnt[i] : cap;
        for (int32_t k = 0; k < m; ++k) {
            int64_t j = nbr[(size_t)i * cap + k];
            double d[3];
            min_image(x + 3 * i, x + 3 * j, box, d);
            double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
            int ab = pair_index(p, sp[i], sp[j]);
            if (r >= p->rcut[ab]) continue;
            double fs = oracle_pair_fscalar(r, ab, p);
            for (int c = 0; c < 3; ++c) fi[c] += fs * d[c];
            ui += 0.5 * oracle_pair_energy(r, ab, p);
            wi += 0.5 * fs * r * r;
        }
        for (int c = 0; c < 3; ++c) f[3 * i + c] = fi[c];
        U += ui;
        W += wi;
    }
    out[0] = U;
    out[1] = W;
}

/* O10b -- FP64 forces of the positions the FP32 path represents. Every
 * coordinate is first carried through steps 1 and 2 of the FP32 sequence
 * above (double-single split of the wrapped coordinate, fixed-point image
 * coordinate q); a pair displacement is then the wrapped 32-bit difference
 * q_i - q_j times the quantum L 2^-32, formed in FP64 (exact: an integer of
 * at most 31 bits times a power-of-two multiple of L, rounded once). From
 * there on everything is oracle_forces_list: FP64 pair forces over the full
 * lists, the cutoff decided in FP64 on these displacements. What remains
 * between this and the FP32 path is the binary32 arithmetic of the path
 * itself (and the cutoff decision at ties).
 * out = [U, W]; fabs (nullable) receives per particle the sum over its
 * partners inside the cutoff of the pair-force magnitudes |fs| r, the scale
 * against which the rounding of a sum of pair forces is measured. */
void oracle_forces_fixed(int64_t n, const double *x, const int32_t *sp, const double *box,
                         const olj_t *p, int32_t cap, const int32_t *cnt, const int32_t *nbr,
                         double *f, double *out, double *fabs_sum) {
    uint32_t *q = (uint32_t *)malloc(sizeof(uint32_t) * 3 * (size_t)n);
    double quantum[3];
    for (int k = 0; k < 3; ++k) quantum[k] = box[k] / 4294967296.0;
    for (int64_t i = 0; i < n; ++i)
        for (int k = 0; k < 3; ++k) {
            float hi, lo;
            oracle_ds_split(wrap1(x[3 * i + k], box[k]), &hi, &lo);
            q[3 * i + k] = oracle_q_from_ds(hi, lo, box[k]);
        }
    double U = 0.0, W = 0.0;
#pragma omp parallel for schedule(static) reduction(+ : U, W)
    for (int64_t i = 0; i < n; ++i) {
        double fi[3] = {0.0, 0.0, 0.0};
        double ui = 0.0, wi = 0.0, ai = 0.0;
        int32_t m = cnt[i] < cap ? cnt[i] : cap;
        for (int32_t k = 0; k < m; ++k) {
            int64_t j = nbr[(size_t)i * cap + k];
            double d[3];
            for (int c = 0; c < 3; ++c)
                d[c] = (double)(int32_t)(q[3 * i + c] - q[3 * j + c]) * quantum[c];
            double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
            int ab = pair_index(p, sp[i], sp[j]);
            if (r >= p->rcut[ab]) continue;
            double fs = oracle_pair_fscalar(r, ab, p);
            for (int c = 0; c < 3; ++c) fi[c] += fs * d[c];
            ui += 0.5 * oracle_pair_energy(r, ab, p);
            wi += 0.5 * fs * r * r;
            ai += fabs(fs) * r;
        }
        for (int c = 0; c < 3; ++c) f[3 * i + c] = fi[c];
        if (fabs_sum) fabs_sum[i] = ai;
        U += ui;
        W += wi;
    }
    free(q);
    out[0] = U;
    out[1] = W;
}

/* Kinetic energy and momentum: out = [K, px, py, pz]. */
void oracle_kinetic(int64_t n, const double *v, const int32_t *sp, const olj_t *p, double *out) {
    double K = 0.0, px = 0.0, py = 0.0, pz = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double m = p->mass[p->nspecies == 2 ? sp[i] : 0];
        const double *vi = v + 3 * i;
        K += 0.5 * m * (vi[0] * vi[0] + vi[1] * vi[1] + vi[2] * vi[2]);
        px += m * vi[0];
        py += m * vi[1];
        pz += m * vi[2];
    }
    out[0] = K;
    out[1] = px;
    out[2] = py;
    out[3] = pz;
}

/* ---------------------------------------------------------------- O11 --- */

/* Philox4x32-10, the counter-based generator of Salmon, Moraes, Dror and
 * Shaw, "Parallel random numbers: as easy as 1, 2, 3" (SC'11): ten rounds of
 *   (hi0, lo0) = M0 * c0,  (hi1, lo1) = M1 * c2   (32 x 32 -> 64-bit products)
 *   c = (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0)
 * with the key bumped by the Weyl constants (W0, W1) after every round but
 * the last. M0 = 0xD2511F53, M1 = 0xCD9E8D57, W0 = 0x9E3779B9,
 * W1 = 0xBB67AE85. */
void oracle_philox4x32(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        c0 = hi1 ^ c1 ^ k0;
        c1 = lo1;
        c2 = hi0 ^ c3 ^ k1;
        c3 = lo0;
        if (r < 9) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

/* Settings of the stochastic velocity-resampling ("Boltzmann", Andersen-type)
 * thermostat. rate = collision frequency nu per unit time; 0 disables it. */
typedef struct {
    double temperature;
    double rate;
    uint64_t seed;
    int32_t dim;    /* 2: motion in the x-y plane (a resampled v_z is 0); else 3 */
    int32_t pad;
} othermo_t;

/* Collision threshold: a particle collides in a step iff its first draw u0
 * (a uniform 32-bit integer) is below floor(nu dt 2^32), so that the
 * collision probability per step is nu dt (to 2^-32). */
uint32_t oracle_thermo_threshold(double rate, double dt) {
    double t = floor(rate * dt * 4294967296.0);
    if (!(t > 0.0)) return 0u;
    if (t >= 4294967295.0) return 0xFFFFFFFFu;
    return (uint32_t)t;
}

/* Uniform in (0, 1) from a 32-bit integer: (u + 1/2) 2^-32 (exact in FP64). */
static double u01(uint32_t u) { return ((double)u + 0.5) * (1.0 / 4294967296.0); }

/* The thermostat's draws for particle `id` at step `step`: two Philox blocks
 * with counters (id, step_lo, step_hi, 0) and (id, step_lo, step_hi, 1) under
 * the key (seed_lo, seed_hi). Returns 1 if the particle collides (first word
 * below the threshold) and then writes three standard normal deviates from
 * the Box-Muller transform (z0, z1) = sqrt(-2 ln a) (cos 2 pi b, sin 2 pi b)
 * of the pairs (a, b) = (w1, w2) and (w3, w4) of the eight words (z1 of the
 * second pair unused). */
int32_t oracle_thermo_draw(uint64_t seed, int64_t id, int64_t step, uint32_t threshold, double z[3]) {
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t ctr[4] = {(uint32_t)id, (uint32_t)(uint64_t)step, (uint32_t)((uint64_t)step >> 32), 0u};
    uint32_t a[4], b[4];
    oracle_philox4x32(ctr, key, a);
    if (a[0] >= threshold) return 0;
    ctr[3] = 1u;
    oracle_philox4x32(ctr, key, b);
    const double two_pi = 6.283185307179586476925286766559;
    double r1 = sqrt(-2.0 * log(u01(a[1]))), t1 = two_pi * u01(a[2]);
    double r2 = sqrt(-2.0 * log(u01(a[3]))), t2 = two_pi * u01(b[0]);
    z[0] = r1 * cos(t1);
    z[1] = r1 * sin(t1);
    z[2] = r2 * cos(t2);
    return 1;
}

/* Order-independent 64-bit signature of the set of unordered pairs i < j
 * inside their cutoff (from full lists): the sum of a 64-bit mix of (i, j).
 * Two configurations with the same signature have, but for a 2^-64 chance,
 * the same pairs inside the cutoff. */
static uint64_t mix64(uint64_t z) {
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static uint64_t cutoff_signature(int64_t n, const double *x, const int32_t *sp, const double *box,
                                 const olj_t *p, int32_t cap, const int32_t *cnt, const int32_t *nbr) {
    uint64_t s = 0;
    for (int64_t i = 0; i < n; ++i) {
        int32_t m = cnt[i] < cap ? cnt[i] : cap;
        for (int32_t k = 0; k < m; ++k) {
            int64_t j = nbr[(size_t)i * cap + k];
            if (j <= i) continue;
            double d[3];
            min_image(x + 3 * i, x + 3 * j, box, d);
            double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
            if (r >= p->rcut[pair_index(p, sp[i], sp[j])]) continue;
            s += mix64(((uint64_t)i << 32) | (uint64_t)j);
        }
    }
    return s;
}

/* ---------------------------------------------------------------- O5 ---- */

typedef struct {
    int64_t n;
    int32_t cap;
    int32_t *cnt, *nbr;
    double *xref;
} olist_t;

static int build(olist_t *L, const double *x, const int32_t *sp, const double *box,
                 const olj_t *p) {
    for (;;) {
        int32_t mx = oracle_build_lists(L->n, x, sp, box, p, 0, L->cap, L->cnt, L->nbr);
        if (mx <= L->cap) break;
        L->cap = mx + 16;
        free(L->nbr);
        L->nbr = (int32_t *)malloc(sizeof(int32_t) * (size_t)L->n * L->cap);
        if (!L->nbr) return -1;
    }
    memcpy(L->xref, x, sizeof(double) * 3 * (size_t)L->n);
    return 0;
}

/* The list stays valid while no particle has moved more than half the skin
 * since the last build; rebuild when the largest displacement exceeds s/2. */
static int needs_rebuild(const olist_t *L, const double *x, double skin) {
    double lim2 = 0.25 * skin * skin;
    for (int64_t i = 0; i < 3 * L->n; i += 3) {
        double dx = x[i] - L->xref[i], dy = x[i + 1] - L->xref[i + 1], dz = x[i + 2] - L->xref[i + 2];
        if (dx * dx + dy * dy + dz * dz > lim2) return 1;
    }
    return 0;
}

/* Velocity-Verlet NVE (Sec. 3: the "integrate" half step updates momenta and
 * positions, a force evaluation follows, "finalize" completes the momenta):
 *   v <- v + dt/2 F/m ; x <- x + dt v ; [rebuild if needed] ; F <- F(x) ;
 *   v <- v + dt/2 F/m ; [thermostat].
 * With a thermostat (Sec. 4: velocity Verlet combined with a stochastic
 * Andersen-like thermostat), after the second half kick of step s every
 * particle that collides (oracle_thermo_draw with its id and s) takes a new
 * velocity sqrt(T/m) z from the Maxwell-Boltzmann distribution at T.
 * x (unwrapped) and v are updated in place, particles keep their order (the
 * id of row i is i). obs (nullable) receives (nsteps + 1) rows
 * [U, K, W, px, py, pz] for steps 0..nsteps. f_out (nullable) receives the
 * final forces; thermo (nullable) enables the thermostat; sig (nullable)
 * receives, for steps 0..nsteps, the signature of the pairs inside the
 * cutoff; loop_seconds (nullable) the wall time of the step loop alone
 * (after the initial list build and forces). Returns the number of list
 * builds (including the initial one), or -1 on allocation failure. */
int64_t oracle_run_nve(int64_t n, double *x, double *v, const int32_t *sp, const double *box,
                       const olj_t *p, int64_t nsteps, double *obs, double *f_out,
                       const othermo_t *thermo, uint64_t *sig, double *loop_seconds) {
    olist_t L;
    L.n = n;
    L.cap = 160;
    L.cnt = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    L.nbr = (int32_t *)malloc(sizeof(int32_t) * (size_t)n * L.cap);
    L.xref = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    double *f = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    double *invm = (double *)malloc(sizeof(double) * (size_t)n);
    if (!L.cnt || !L.nbr || !L.xref || !f || !invm) return -1;
    for (int64_t i = 0; i < n; ++i) invm[i] = 1.0 / p->mass[p->nspecies == 2 ? sp[i] : 0];
    int64_t builds = 0;
    if (build(&L, x, sp, box, p)) return -1;
    builds++;
    double uw[2], kp[4];
    oracle_forces_list(n, x, sp, box, p, L.cap, L.cnt, L.nbr, f, uw);
    if (obs) {
        oracle_kinetic(n, v, sp, p, kp);
        double row[6] = {uw[0], kp[0], uw[1], kp[1], kp[2], kp[3]};
        memcpy(obs, row, sizeof row);
    }
    if (sig) sig[0] = cutoff_signature(n, x, sp, box, p, L.cap, L.cnt, L.nbr);
    const int thermo_on = thermo && thermo->rate > 0.0;
    const uint32_t thr = thermo_on ? oracle_thermo_threshold(thermo->rate, p->dt) : 0u;
    double h = 0.5 * p->dt;
    double t0 = wall_seconds();
    for (int64_t s = 1; s <= nsteps; ++s) {
        for (int64_t i = 0; i < n; ++i)
            for (int k = 0; k < 3; ++k) {
                v[3 * i + k] += h * f[3 * i + k] * invm[i];
                x[3 * i + k] += p->dt * v[3 * i + k];
            }
        if (needs_rebuild(&L, x, p->skin)) {
            if (build(&L, x, sp, box, p)) return -1;
            builds++;
        }
        oracle_forces_list(n, x, sp, box, p, L.cap, L.cnt, L.nbr, f, uw);
        for (int64_t i = 0; i < n; ++i)
            for (int k = 0; k < 3; ++k) v[3 * i + k] += h * f[3 * i + k] * invm[i];
        if (thermo_on)
            for (int64_t i = 0; i < n; ++i) {
                double z[3];
                if (!oracle_thermo_draw(thermo->seed, i, s, thr, z)) continue;
                double sd = sqrt(thermo->temperature * invm[i]);
                if (thermo->dim == 2) z[2] = 0.0;
                for (int k = 0; k < 3; ++k) v[3 * i + k] = sd * z[k];
            }
        if (sig) sig[s] = cutoff_signature(n, x, sp, box, p, L.cap, L.cnt, L.nbr);
        if (obs) {
            oracle_kinetic(n, v, sp, p, kp);
            double row[6] = {uw[0], kp[0], uw[1], kp[1], kp[2], kp[3]};
            memcpy(obs + 6 * s, row, sizeof row);
        }
    }
    if (loop_seconds) *loop_seconds = wall_seconds() - t0;
    if (f_out) memcpy(f_out, f, sizeof(double) * 3 * (size_t)n);
    free(L.cnt);
    free(L.nbr);
    free(L.xref);
    free(f);
    free(invm);
    return builds;
}

/* ---------------------------------------------------------------- O6 ---- */

/* Steepest descent used to relax random starting positions (the 4M-particle
 * mixture workload) before dynamics:
 *   F = forces of the truncated potential with every pair distance clamped
 *       from below at clamp * sigma_ab (random positions overlap; the clamp
 *       keeps forces finite and is used only here);
 *   F_max = max_i |F_i|;   x_i <- x_i + delta * F_i / F_max,
 * so that no particle moves more than delta per step. Lists are rebuilt with
 * the same half-skin rule as the dynamics. x (unwrapped) is updated in place.
 * u_out (nullable) receives nsteps+1 clamped energies U_k (before step k+1 and
 * after the last step); fmax_out (nullable) the nsteps+1 values F_max.
 * Returns the number of list builds, -1 on allocation failure. */
static void forces_list_clamped(int64_t n, const double *x, const int32_t *sp, const double *box,
                                const olj_t *p, int32_t cap, const int32_t *cnt,
                                const int32_t *nbr, double clamp, double *f, double *U_out) {
    double U = 0.0;
#pragma omp parallel for schedule(static) reduction(+ : U)
    for (int64_t i = 0; i < n; ++i) {
        double fi[3] = {0.0, 0.0, 0.0};
        double ui = 0.0;
        int32_t m = cnt[i] < cap ? cnt[i] : cap;
        for (int32_t k = 0; k < m; ++k) {
            int64_t j = nbr[(size_t)i * cap + k];
            double d[3];
            min_image(x + 3 * i, x + 3 * j, box, d);
            double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
            int ab = pair_index(p, sp[i], sp[j]);
            if (r >= p->rcut[ab]) continue;
            double rmin = clamp * p->sigma[ab];
            double re = r < rmin ? rmin : r;
            double fs = oracle_pair_fscalar(re, ab, p);
            for (int c = 0; c < 3; ++c) fi[c] += fs * d[c];
            ui += 0.5 * oracle_pair_energy(re, ab, p);
        }
        for (int c = 0; c < 3; ++c) f[3 * i + c] = fi[c];
        U += ui;
    }
    *U_out = U;
}

int64_t oracle_minimize_sd(int64_t n, double *x, const int32_t *sp, const double *box,
                           const olj_t *p, int64_t nsteps, double delta, double clamp,
                           double *u_out, double *fmax_out) {
    olist_t L;
    L.n = n;
    L.cap = 160;
    L.cnt = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    L.nbr = (int32_t *)malloc(sizeof(int32_t) * (size_t)n * L.cap);
    L.xref = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    double *f = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    if (!L.cnt || !L.nbr || !L.xref || !f) return -1;
    int64_t builds = 0;
    if (build(&L, x, sp, box, p)) return -1;
    builds++;
    for (int64_t s = 0; s <= nsteps; ++s) {
        if (s > 0 && needs_rebuild(&L, x, p->skin)) {
            if (build(&L, x, sp, box, p)) return -1;
            builds++;
        }
        double U;
        forces_list_clamped(n, x, sp, box, p, L.cap, L.cnt, L.nbr, clamp, f, &U);
        double fmax = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            double a = sqrt(f[3 * i] * f[3 * i] + f[3 * i + 1] * f[3 * i + 1] + f[3 * i + 2] * f[3 * i + 2]);
            if (a > fmax) fmax = a;
        }
        if (u_out) u_out[s] = U;
        if (fmax_out) fmax_out[s] = fmax;
        if (s == nsteps || fmax == 0.0) {
            for (int64_t t = s + 1; t <= nsteps; ++t) {
                if (u_out) u_out[t] = U;
                if (fmax_out) fmax_out[t] = fmax;
            }
            break;
        }
        double scale = delta / fmax;
        for (int64_t k = 0; k < 3 * n; ++k) x[k] += scale * f[k];
    }
    free(L.cnt);
    free(L.nbr);
    free(L.xref);
    free(f);
    return builds;
}

/* ---------------------------------------------------------------- O7 ---- */

/* Pair-type index of the symmetric parameter: 0 = AA, 1 = AB, 2 = BB. */
static int sym_type(const olj_t *p, int a, int b) { return p->nspecies == 1 ? 0 : a + b; }

/* Unordered pairs i < j within the cutoff, from full lists (j > i). The
 * callback receives the minimum-image displacement d = x_i - x_j and r^2. */
typedef void (*pair_fn)(void *ctx, int64_t i, int64_t j, const double d[3], double r2, int ab);

static int for_each_pair(int64_t n, const double *x, const int32_t *sp, const double *box,
                         const olj_t *p, pair_fn fn, void *ctx) {
    int32_t cap = 160;
    int32_t *cnt = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *nbr = NULL;
    if (!cnt) return -1;
    for (;;) {
        free(nbr);
        nbr = (int32_t *)malloc(sizeof(int32_t) * (size_t)n * cap);
        if (!nbr) return -1;
        int32_t mx = oracle_build_lists(n, x, sp, box, p, 0, cap, cnt, nbr);
        if (mx <= cap) break;
        cap = mx + 16;
    }
    for (int64_t i = 0; i < n; ++i)
        for (int32_t k = 0; k < cnt[i]; ++k) {
            int64_t j = nbr[(size_t)i * cap + k];
            if (j <= i) continue;
            double d[3];
            min_image(x + 3 * i, x + 3 * j, box, d);
            double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            int ab = pair_index(p, sp[i], sp[j]);
            if (r2 >= p->rcut[ab] * p->rcut[ab]) continue;
            fn(ctx, i, j, d, r2, ab);
        }
    free(cnt);
    free(nbr);
    return 0;
}

typedef struct {
    const olj_t *p;
    const int32_t *sp;
    const double *g;
    double *gx;
    double gt[6];  /* d/d eps_t (t = 0..2), d/d sigma_t */
} vjp_ctx;

/* Vector-Jacobian product of the forces: for a cotangent g (N x 3),
 *   gx_i = sum_j [ fs D + 2 (dfs/dr^2) (d.D) d ],  D = g_i - g_j,
 * i.e. (dF/dx)^T g, with fs = 24 eps (2 s12 - s6) / r^2 and
 * dfs/d(r^2) = -(24 eps / r^4)(14 s12 - 4 s6), s6 = (sigma/r)^6, s12 = s6^2;
 * and the parameter gradients of g.F summed per symmetric pair type:
 *   d(g.F)/d eps   += D.f_ij / eps,
 *   d(g.F)/d sigma += (D.d) (144 eps / sigma) (4 s12 - s6) / r^2.
 * The force is differentiated where it is smooth (r < r_c); its jump at
 * r_c has no derivative term. */
static void vjp_pair(void *vc, int64_t i, int64_t j, const double d[3], double r2, int ab) {
    vjp_ctx *c = (vjp_ctx *)vc;
    const olj_t *p = c->p;
    double eps = p->eps[ab], sig = p->sigma[ab];
    double s2 = sig * sig / r2, s6 = s2 * s2 * s2, s12 = s6 * s6;
    double fs = 24.0 * eps * (2.0 * s12 - s6) / r2;
    double dfs = -(24.0 * eps / (r2 * r2)) * (14.0 * s12 - 4.0 * s6);
    double D[3], dD = 0.0;
    for (int k = 0; k < 3; ++k) {
        D[k] = c->g[3 * i + k] - c->g[3 * j + k];
        dD += d[k] * D[k];
    }
    for (int k = 0; k < 3; ++k) {
        double t = fs * D[k] + 2.0 * dfs * dD * d[k];
        c->gx[3 * i + k] += t;
        c->gx[3 * j + k] -= t;
    }
    int t = sym_type(p, c->sp[i], c->sp[j]);
    if (eps != 0.0) c->gt[t] += fs * dD / eps;
    c->gt[3 + t] += dD * (144.0 * eps / sig) * (4.0 * s12 - s6) / r2;
}

int32_t oracle_force_vjp(int64_t n, const double *x, const int32_t *sp, const double *box,
                         const olj_t *p, const double *g, double *gx, double *gtheta) {
    vjp_ctx c;
    c.p = p;
    c.sp = sp;
    c.g = g;
    c.gx = gx;
    memset(gx, 0, sizeof(double) * 3 * (size_t)n);
    memset(c.gt, 0, sizeof c.gt);
    if (for_each_pair(n, x, sp, box, p, vjp_pair, &c)) return -1;
    memcpy(gtheta, c.gt, sizeof c.gt);
    return 0;
}

/* Parameter gradient of the truncated, shifted potential energy, with r_c a
 * fixed length and the shift phi(r_c; eps, sigma) differentiated too:
 *   dU/d eps_t   = sum phi_s / eps,
 *   dU/d sigma_t = sum (4 eps / sigma) [(12 s12 - 6 s6) - (12 s12 - 6 s6)|_{r_c}]. */
typedef struct {
    const olj_t *p;
    const int32_t *sp;
    double gt[6];
} eg_ctx;

static void eg_pair(void *vc, int64_t i, int64_t j, const double d[3], double r2, int ab) {
    (void)d;
    eg_ctx *c = (eg_ctx *)vc;
    const olj_t *p = c->p;
    double eps = p->eps[ab], sig = p->sigma[ab], rc = p->rcut[ab];
    double s2 = sig * sig / r2, s6 = s2 * s2 * s2, s12 = s6 * s6;
    double c2 = sig * sig / (rc * rc), c6 = c2 * c2 * c2, c12 = c6 * c6;
    int t = sym_type(p, c->sp[i], c->sp[j]);
    double phis = 4.0 * (s12 - s6) - (p->shift_energy ? 4.0 * (c12 - c6) : 0.0);
    c->gt[t] += phis;
    double dsig = (12.0 * s12 - 6.0 * s6) - (p->shift_energy ? (12.0 * c12 - 6.0 * c6) : 0.0);
    c->gt[3 + t] += 4.0 * eps / sig * dsig;
}

int32_t oracle_energy_grad(int64_t n, const double *x, const int32_t *sp, const double *box,
                           const olj_t *p, double *gtheta) {
    eg_ctx c;
    c.p = p;
    c.sp = sp;
    memset(c.gt, 0, sizeof c.gt);
    if (for_each_pair(n, x, sp, box, p, eg_pair, &c)) return -1;
    memcpy(gtheta, c.gt, sizeof c.gt);
    return 0;
}

/* Forces of a configuration via freshly built lists (any N). Returns 0/-1. */
static int forces_fresh(int64_t n, const double *x, const int32_t *sp, const double *box,
                        const olj_t *p, double *f, double *uw) {
    int32_t cap = 160;
    int32_t *cnt = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *nbr = NULL;
    if (!cnt) return -1;
    for (;;) {
        free(nbr);
        nbr = (int32_t *)malloc(sizeof(int32_t) * (size_t)n * cap);
        if (!nbr) return -1;
        int32_t mx = oracle_build_lists(n, x, sp, box, p, 0, cap, cnt, nbr);
        if (mx <= cap) break;
        cap = mx + 16;
    }
    oracle_forces_list(n, x, sp, box, p, cap, cnt, nbr, f, uw);
    free(cnt);
    free(nbr);
    return 0;
}

/* ---------------------------------------------------------------- O9 ---- */

/* Adjoint of nsteps velocity-Verlet steps (every frame stored; no
 * checkpointing). Forward: v' = v_n + dt/2 a(x_n); x_{n+1} = x_n + dt v';
 * v_{n+1} = v' + dt/2 a(x_{n+1}), a = F/m. Given lam_x = dL/dx_N and
 * lam_v = dL/dv_N (in place: on return they hold dL/dx_0 and dL/dv_0 of the
 * dynamics part), the reverse sweep is, for n = N-1 .. 0,
 *   lam_v' = lam_v;  lam_x += dt/2 J(x_{n+1})^T lam_v;  g_th += dt/2 da/dth^T lam_v
 *   lam_v' += dt lam_x
 *   lam_v = lam_v';  lam_x += dt/2 J(x_n)^T lam_v';      g_th += dt/2 da/dth^T lam_v'
 * with J^T lam = (dF/dx)^T (lam / m) (a force VJP with the cotangent divided
 * by the mass). gtheta (6) accumulates. Returns 0, or -1 on failure. */
int32_t oracle_vv_adjoint(int64_t n, const double *x0, const double *v0, const int32_t *sp,
                          const double *box, const olj_t *p, int64_t nsteps, double *lam_x,
                          double *lam_v, double *gtheta) {
    size_t nn = 3 * (size_t)n;
    double *frames = (double *)malloc(sizeof(double) * nn * (size_t)(nsteps + 1));
    double *x = (double *)malloc(sizeof(double) * nn);
    double *v = (double *)malloc(sizeof(double) * nn);
    double *f = (double *)malloc(sizeof(double) * nn);
    double *g = (double *)malloc(sizeof(double) * nn);
    double *gx = (double *)malloc(sizeof(double) * nn);
    double *invm = (double *)malloc(sizeof(double) * (size_t)n);
    if (!frames || !x || !v || !f || !g || !gx || !invm) return -1;
    for (int64_t i = 0; i < n; ++i) invm[i] = 1.0 / p->mass[p->nspecies == 2 ? sp[i] : 0];
    memcpy(x, x0, sizeof(double) * nn);
    memcpy(v, v0, sizeof(double) * nn);
    memcpy(frames, x, sizeof(double) * nn);
    double uw[2];
    if (forces_fresh(n, x, sp, box, p, f, uw)) return -1;
    double h = 0.5 * p->dt;
    for (int64_t s = 1; s <= nsteps; ++s) {
        for (size_t k = 0; k < nn; ++k) {
            v[k] += h * f[k] * invm[k / 3];
            x[k] += p->dt * v[k];
        }
        if (forces_fresh(n, x, sp, box, p, f, uw)) return -1;
        for (size_t k = 0; k < nn; ++k) v[k] += h * f[k] * invm[k / 3];
        memcpy(frames + nn * (size_t)s, x, sizeof(double) * nn);
    }
    double gt[6];
    for (int64_t s = nsteps - 1; s >= 0; --s) {
        /* second half kick of step s -> s+1, at x_{s+1} */
        for (size_t k = 0; k < nn; ++k) g[k] = lam_v[k] * invm[k / 3];
        if (oracle_force_vjp(n, frames + nn * (size_t)(s + 1), sp, box, p, g, gx, gt)) return -1;
        for (size_t k = 0; k < nn; ++k) lam_x[k] += h * gx[k];
        for (int q = 0; q < 6; ++q) gtheta[q] += h * gt[q];
        /* drift */
        for (size_t k = 0; k < nn; ++k) lam_v[k] += p->dt * lam_x[k];
        /* first half kick, at x_s */
        for (size_t k = 0; k < nn; ++k) g[k] = lam_v[k] * invm[k / 3];
        if (oracle_force_vjp(n, frames + nn * (size_t)s, sp, box, p, g, gx, gt)) return -1;
        for (size_t k = 0; k < nn; ++k) lam_x[k] += h * gx[k];
        for (int q = 0; q < 6; ++q) gtheta[q] += h * gt[q];
    }
    free(frames);
    free(x);
    free(v);
    free(f);
    free(g);
    free(gx);
    free(invm);
    return 0;
}

/* Threads of the OpenMP loops from now on (n >= 1). */
void oracle_set_threads(int32_t n) {
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int32_t oracle_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
