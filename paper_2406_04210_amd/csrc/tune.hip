// tune.hip -- the autotuner: picks the cell size of the binning and list
// build (cells of edge >= r_L, or >= r_L / 2 with the 125-cell stencil) and
// the launch shape of the force gather (lanes per particle) for a system by
// timing short runs on the device, and sizes the list capacity from the
// longest list seen. Results are cached in a
// text file of JSON lines keyed by device, precision, species count, size
// and density, so a known shape is reused without timing (the paper tunes
// launch configurations per device, Sec. 4-5; the search here is this
// library's own).
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "internal.h"

namespace {

constexpr int kLaneCandidates[] = {1, 2, 4, 8, 16};
constexpr int kSplitCandidates[] = {1, 2};

std::string tune_key(const ljmd_params *p) {
    hipDeviceProp_t prop;
    int dev = 0;
    std::string arch = "unknown";
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
        arch = prop.gcnArchName;
    for (char &ch : arch)
        if (ch == '"' || ch == ' ') ch = '_';
    // Density per volume, or per area in two dimensions (box[2] is no period there).
    const double vol = p->dim == 2 ? p->box[0] * p->box[1] : p->box[0] * p->box[1] * p->box[2];
    const double rho = (double)p->n / vol;
    char buf[256];
    // Dimension, size in powers of two, density to 0.05, the list radius to 0.1 sigma.
    std::snprintf(buf, sizeof buf, "%s|dim%d|prec%d|ns%d|n2^%d|rho%.2f|rl%.1f", arch.c_str(), p->dim == 2 ? 2 : 3,
                  p->precision, p->nspecies, (int)std::lround(std::log2((double)p->n)),
                  std::round(rho * 20.0) / 20.0, p->rcut[0] + p->skin);
    return buf;
}

bool cache_lookup(const char *path, const std::string &key, ljmd_tuning *out) {
    FILE *f = std::fopen(path, "r");
    if (!f) return false;
    char line[1024];
    const std::string want = "\"key\": \"" + key + "\"";
    bool found = false;
    while (std::fgets(line, sizeof line, f)) {
        if (!std::strstr(line, want.c_str())) continue;
        int lanes = 0, cap = 0, cc = 0, fill = 0;
        double ms = 0.0;
        const char *q = std::strstr(line, "\"lanes\":");
        const char *r = std::strstr(line, "\"nbr_capacity\":");
        const char *s = std::strstr(line, "\"cell_capacity\":");
        const char *t = std::strstr(line, "\"ms_per_step\":");
        const char *u = std::strstr(line, "\"max_fill\":");
        const char *v = std::strstr(line, "\"cell_split\":");
        if (!q || !r || !s || !t || !u || !v) continue;
        int split = 0;
        if (std::sscanf(v, "\"cell_split\": %d", &split) != 1) continue;
        if (std::sscanf(q, "\"lanes\": %d", &lanes) != 1 || std::sscanf(r, "\"nbr_capacity\": %d", &cap) != 1 ||
            std::sscanf(s, "\"cell_capacity\": %d", &cc) != 1 || std::sscanf(t, "\"ms_per_step\": %lf", &ms) != 1 ||
            std::sscanf(u, "\"max_fill\": %d", &fill) != 1)
            continue;
        out->lanes = lanes;
        out->nbr_capacity = cap;
        out->cell_capacity = cc;
        out->ms_per_step = ms;
        out->max_fill = fill;
        out->cell_split = split;
        found = true;  // the last matching line wins
    }
    std::fclose(f);
    return found;
}

void cache_store(const char *path, const std::string &key, const ljmd_tuning &t) {
    FILE *f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f,
                 "{\"key\": \"%s\", \"cell_split\": %d, \"lanes\": %d, \"nbr_capacity\": %d, "
                 "\"cell_capacity\": %d, \"ms_per_step\": %.6f, \"max_fill\": %d}\n",
                 key.c_str(), t.cell_split, t.lanes, t.nbr_capacity, t.cell_capacity, t.ms_per_step, t.max_fill);
    std::fclose(f);
}

std::string batch_key(const ljmd_params *p, const ljmd_system *sys, int32_t nsys) {
    hipDeviceProp_t prop;
    int dev = 0;
    std::string arch = "unknown";
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
        arch = prop.gcnArchName;
    for (char &ch : arch)
        if (ch == '"' || ch == ' ') ch = '_';
    double ntot = 0.0, vol = 0.0;
    for (int32_t k = 0; k < nsys; ++k) {
        ntot += (double)sys[k].n;
        vol += sys[k].box * sys[k].box * sys[k].box;
    }
    char buf[256];
    std::snprintf(buf, sizeof buf, "batch|%s|nsys%d|n2^%d|rho%.2f|rl%.1f", arch.c_str(), nsys,
                  (int)std::lround(std::log2(ntot)), std::round(ntot / vol * 20.0) / 20.0, p->rcut[0] + p->skin);
    return buf;
}

// List capacity from the longest list seen: a margin for density
// fluctuations, in whole 16-slot units.
int capacity_for(int fill) {
    int cap = (int)std::ceil(std::fmax(1.25 * fill, fill + 24.0));
    cap = (cap + 15) / 16 * 16;
    return cap < 16 ? 16 : (cap > 4096 ? 4096 : cap);
}

}  // namespace

extern "C" {

size_t ljmd_autotune_workspace_size(const ljmd_params *p) {
    if (ljmd_check_params(p) != LJMD_OK) return 0;
    size_t best = 0;
    for (int split : kSplitCandidates)
        for (int lanes : kLaneCandidates) {
            ljmd_params q = *p;
            q.lanes = lanes;
            q.cell_split = split;
            const size_t s = ljmd_workspace_size(&q);
            if (s == 0) return 0;
            best = s > best ? s : best;
        }
    return best;
}

int ljmd_autotune(const ljmd_params *p, const double *x, const double *v, const int32_t *species, void *ws,
                  size_t bytes, void *stream, int32_t steps, const char *cache_path, ljmd_tuning *out) {
    if (!p || !x || !v || !species || !ws || !out || steps < 1) return LJMD_EINVAL;
    int r = ljmd_check_params(p);
    if (r != LJMD_OK) return r;
    if (std::isinf(p->rcut[0])) return LJMD_EINVAL;  // the all-pairs interaction has no lists to tune
    std::memset(out, 0, sizeof *out);
    const std::string key = tune_key(p);
    if (cache_path && cache_lookup(cache_path, key, out)) {
        out->from_cache = 1;
        return LJMD_OK;
    }
    if (bytes < ljmd_autotune_workspace_size(p)) return LJMD_ENOMEM;
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return LJMD_EHIP;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return LJMD_EHIP;
    }
    double best_ms = 0.0;
    int rc = LJMD_OK;
    for (int split : kSplitCandidates)
    for (int lanes : kLaneCandidates) {
        ljmd_params q = *p;
        q.lanes = lanes;
        q.cell_split = split;
        ljmd_ctx *c = nullptr;
        if ((rc = ljmd_create(&q, ws, bytes, stream, &c)) != LJMD_OK) break;
        float ms = 0.f;
        ljmd_obs o;
        rc = ljmd_set_state(c, x, v, species);
        if (rc == LJMD_OK) rc = ljmd_run(c, 10, nullptr);  // warm-up
        if (rc == LJMD_OK) rc = ljmd_sync_status(c);
        if (rc == LJMD_OK && hipEventRecord(e0, s) != hipSuccess) rc = LJMD_EHIP;
        if (rc == LJMD_OK) rc = ljmd_run(c, steps, nullptr);
        if (rc == LJMD_OK && hipEventRecord(e1, s) != hipSuccess) rc = LJMD_EHIP;
        if (rc == LJMD_OK && hipEventSynchronize(e1) != hipSuccess) rc = LJMD_EHIP;
        if (rc == LJMD_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) rc = LJMD_EHIP;
        if (rc == LJMD_OK) rc = ljmd_observables(c, &o);
        ljmd_destroy(c);
        if (rc != LJMD_OK) break;
        const double per = (double)ms / steps;
        if (out->lanes == 0 || per < best_ms) {
            best_ms = per;
            out->lanes = lanes;
            out->cell_split = split;
            out->cell_capacity = q.cell_capacity;
        }
        out->max_fill = o.max_fill > out->max_fill ? o.max_fill : out->max_fill;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != LJMD_OK) return rc;
    out->nbr_capacity = capacity_for(out->max_fill);
    out->ms_per_step = best_ms;
    out->from_cache = 0;
    if (cache_path) cache_store(cache_path, key, *out);
    return LJMD_OK;
}

size_t ljmd_batch_autotune_workspace_size(const ljmd_params *shared, const ljmd_system *sys, int32_t nsys) {
    if (!shared || !sys || nsys < 1) return 0;
    size_t best = 0;
    for (int split : kSplitCandidates)
        for (int lanes : kLaneCandidates) {
            ljmd_params q = *shared;
            q.lanes = lanes;
            q.cell_split = split;
            const size_t s = ljmd_batch_workspace_size(&q, sys, nsys);
            if (s == 0) return 0;
            best = s > best ? s : best;
        }
    return best;
}

int ljmd_batch_autotune(const ljmd_params *shared, const ljmd_system *sys, int32_t nsys, const double *x,
                        const double *v, const int32_t *species, void *ws, size_t bytes, void *stream,
                        int32_t steps, const char *cache_path, ljmd_tuning *out) {
    if (!shared || !sys || nsys < 1 || !x || !v || !species || !ws || !out || steps < 1) return LJMD_EINVAL;
    std::memset(out, 0, sizeof *out);
    const size_t need = ljmd_batch_autotune_workspace_size(shared, sys, nsys);
    if (need == 0) return LJMD_EINVAL;
    const std::string key = batch_key(shared, sys, nsys);
    if (cache_path && cache_lookup(cache_path, key, out)) {
        out->from_cache = 1;
        return LJMD_OK;
    }
    if (bytes < need) return LJMD_ENOMEM;
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return LJMD_EHIP;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return LJMD_EHIP;
    }
    double best_ms = 0.0;
    int rc = LJMD_OK;
    for (int split : kSplitCandidates)
    for (int lanes : kLaneCandidates) {
        ljmd_params q = *shared;
        q.lanes = lanes;
        q.cell_split = split;
        ljmd_batch *b = nullptr;
        if ((rc = ljmd_batch_create(&q, sys, nsys, ws, bytes, stream, &b)) != LJMD_OK) break;
        float ms = 0.f;
        int32_t fill = 0;
        rc = ljmd_batch_set_state(b, x, v, species);
        if (rc == LJMD_OK) rc = ljmd_batch_run(b, 10, nullptr);  // warm-up
        if (rc == LJMD_OK) rc = ljmd_batch_sync_status(b);
        if (rc == LJMD_OK && hipEventRecord(e0, s) != hipSuccess) rc = LJMD_EHIP;
        if (rc == LJMD_OK) rc = ljmd_batch_run(b, steps, nullptr);
        if (rc == LJMD_OK && hipEventRecord(e1, s) != hipSuccess) rc = LJMD_EHIP;
        if (rc == LJMD_OK && hipEventSynchronize(e1) != hipSuccess) rc = LJMD_EHIP;
        if (rc == LJMD_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) rc = LJMD_EHIP;
        if (rc == LJMD_OK) rc = ljmd_batch_sync_status(b);
        if (rc == LJMD_OK) rc = ljmd_batch_max_fill(b, &fill);
        ljmd_batch_destroy(b);
        if (rc != LJMD_OK) break;
        const double per = (double)ms / steps;
        if (out->lanes == 0 || per < best_ms) {
            best_ms = per;
            out->lanes = lanes;
            out->cell_split = split;
            out->cell_capacity = q.cell_capacity;
        }
        out->max_fill = fill > out->max_fill ? fill : out->max_fill;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != LJMD_OK) return rc;
    out->nbr_capacity = capacity_for(out->max_fill);
    out->ms_per_step = best_ms;
    out->from_cache = 0;
    if (cache_path) cache_store(cache_path, key, *out);
    return LJMD_OK;
}

}  // extern "C"
