// brute.hip -- one-shot evaluation of the forces, energy and virial of a
// configuration by the brute-force sum over all pairs (the definition that
// the Verlet-list path reaches: paper Sec. 3, truncated pair forces; with
// infinite cutoffs the all-to-all interaction of Sec. 4). No context and no
// state: the scratch comes from a caller workspace.
#include <cmath>
#include <cstdio>
#include <mutex>
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

// Scratch of the allocation-free entry point: a fixed array in device
// memory, one copy per GPU the library runs on, held until the process
// ends. Host code never passes its name to a kernel (on the host the name
// is a stand-in, not a device address): it uses the address that
// hipGetSymbolAddress returned for the current device.
constexpr size_t kStaticScratchBytes = (size_t)LJMD_BRUTE_STATIC_SCRATCH_BYTES;
__device__ __align__(256) uint8_t scratch[kStaticScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
uint8_t *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per
// device (with that device current).
int static_scratch(uint8_t **out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return brute_fail(LJMD_EHIP, hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return brute_fail(LJMD_EINVAL, "brute_forces_noalloc: device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return brute_fail(LJMD_EHIP, e != hipSuccess ? hipGetErrorString(e) : "scratch symbol has no address");
        g_scratch_ptr[dev] = (uint8_t *)ptr;
    }
    *out = g_scratch_ptr[dev];
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
    const int dim = p->dim == 2 ? 2 : 3;
    const hipError_t e = launch_brute(box, pc, p->precision, p->nspecies, dim, cut_of(p) ? 1 : 0, p->n, x, species,
                                      f, uw, (uint8_t *)ws, (hipStream_t)stream);
    if (e != hipSuccess) return brute_fail(LJMD_EHIP, hipGetErrorString(e));
    return LJMD_OK;
}

size_t ljmd_brute_static_scratch_bytes(void) { return kStaticScratchBytes; }

int ljmd_brute_forces_noalloc(const ljmd_params *p, const double *x, const int32_t *species, double *f,
                              double *uw, void *stream) {
    int r = brute_check(p);
    if (r != LJMD_OK) return r;
    if (!x || !species || !f || !uw) return brute_fail(LJMD_EINVAL, "brute_forces_noalloc: NULL argument");
    const size_t need = brute_scratch_bytes(p->n, p->precision);
    if (need > kStaticScratchBytes) {
        char msg[160];
        std::snprintf(msg, sizeof msg,
                      "brute_forces_noalloc: n=%lld needs %zu bytes of scratch, above the fixed %zu "
                      "(use ljmd_brute_forces with a workspace)",
                      (long long)p->n, need, kStaticScratchBytes);
        return brute_fail(LJMD_ENOMEM, msg);
    }
    uint8_t *ptr = nullptr;
    if ((r = static_scratch(&ptr)) != LJMD_OK) return r;
    BoxC box;
    PairC pc;
    box_pair_constants(*p, box, pc);
    const int dim = p->dim == 2 ? 2 : 3;
    const hipError_t e = launch_brute(box, pc, p->precision, p->nspecies, dim, cut_of(p) ? 1 : 0, p->n, x, species,
                                      f, uw, ptr, (hipStream_t)stream);
    if (e != hipSuccess) return brute_fail(LJMD_EHIP, hipGetErrorString(e));
    return LJMD_OK;
}

}  // extern "C"
