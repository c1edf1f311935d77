// brute.hip -- one-shot evaluation of the forces, energy and virial of a
// configuration by the brute-force sum over all pairs (the definition that
// the Verlet-list path reaches: paper Sec. 3, truncated pair forces; with
// infinite cutoffs the all-to-all interaction of Sec. 4). No context and no
// state: the scratch comes from a caller workspace.
#include <cmath>
#include <cstdio>
#include <string>

#include "internal.h"

using namespace ljmd;

namespace {

bool cut_of(const ljmd_params *p) { return !std::isinf(p->rcut[0]); }

int brute_fail(int code, const char *msg) {
    set_global_error(msg);
    return code;
}

// Parameters of a one-shot evaluation: the checks of ljmd_check_params,
// and a cubic box for the single-precision paths (fixed-point quanta).
int brute_check(const ljmd_params *p) {
    const char *why = "";
    const int r = check_params_why(p, &why);
    if (r != LJMD_OK) return brute_fail(r, why);
    if (p->precision != LJMD_FP64 && !(p->box[0] == p->box[1] && p->box[1] == p->box[2]))
        return brute_fail(LJMD_EINVAL, "brute forces in single precision need a cubic box");
    return LJMD_OK;
}

}  // namespace

extern "C" {

size_t ljmd_brute_workspace_size(const ljmd_params *p) {
    if (check_params_why(p, nullptr) != LJMD_OK) return 0;
    return brute_scratch_bytes(p->n, p->precision);
}

int ljmd_brute_forces(const ljmd_params *p, const double *x, const int32_t *species, double *f, double *uw,
                      void *ws, size_t bytes, void *stream) {
    int r = brute_check(p);
    if (r != LJMD_OK) return r;
    if (!x || !species || !f || !uw || !ws) return brute_fail(LJMD_EINVAL, "brute_forces: NULL argument");
    if (((uintptr_t)ws & 255) != 0) return brute_fail(LJMD_EINVAL, "brute_forces: workspace must be 256-byte aligned");
    if (bytes < brute_scratch_bytes(p->n, p->precision))
        return brute_fail(LJMD_ENOMEM, "brute_forces: workspace smaller than ljmd_brute_workspace_size");
    BoxC box;
    PairC pc;
    box_pair_constants(*p, box, pc);
    const hipError_t e = launch_brute(box, pc, p->precision, p->nspecies, cut_of(p) ? 1 : 0, p->n, x, species, f, uw,
                                      (uint8_t *)ws, (hipStream_t)stream);
    if (e != hipSuccess) return brute_fail(LJMD_EHIP, hipGetErrorString(e));
    return LJMD_OK;
}

}  // extern "C"
