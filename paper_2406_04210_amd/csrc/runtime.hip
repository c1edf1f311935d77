// runtime.hip -- host side of the C ABI declared in include/ljmd.h:
// parameter validation, workspace planning, the Hilbert cell order, context
// lifetime and the per-step launch sequence (paper Sec. 3 Fig. 1: integrate,
// force, finalize, sample; list updates as particles move, Sec. 5).
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "adjoint.h"
#include "batch.h"
#include "internal.h"

namespace ljmd {
}

using namespace ljmd;

// Workspace layout of a differentiable rollout (ljmd_vv_forward).
struct AdjPlan {
    int32_t nsteps = 0, every = 0, nseg = 0;
    bool store_all = false;   // every frame kept by the forward run
    size_t ckpt_stride = 0;   // bytes of one stored state
    size_t off_ckpt = 0;      // (nseg + 1) stored states
    size_t frame_stride = 0;  // bytes of one position frame (record buffer)
    size_t off_frames = 0;    // every + 1 frames (nsteps + 1 when store_all)
    size_t off_lx = 0, off_lv = 0, off_g = 0, off_g2 = 0;  // off_g2: second cotangent buffer
    // Rebuild markers of every forward step (int32, store_all with segments
    // of at most kRing steps): where each segment's last list build was.
    size_t off_marks = 0;
    // Parameter-gradient rows of the sweep's VJP passes (kNP doubles for
    // each of at most ceil(n / 64) blocks), summed once at the end.
    size_t off_rows = 0;
    size_t total = 0;
    // The sweep starts each segment from the list of the forward run's last
    // build in it (segments of at most kRing steps, whose markers the step
    // kernels' ring still holds when the segment ends).
    bool reuse_lists() const { return every <= kRing; }
};

// The rollout recorded by the last ljmd_vv_forward.
struct AdjRecord {
    bool valid = false;
    AdjPlan plan;
    uint8_t *ws = nullptr;
    int64_t step0 = 0;
    uint64_t gen = 0;
};

struct ljmd_ctx {
    ljmd_params p;
    Geom g;
    BoxC box;
    PairC pc;
    DynC dyn;
    State st;
    hipStream_t stream = nullptr;
    int device = 0;
    int cur = 0;
    int64_t step = 0;
    bool have_state = false;
    int nblocks = 0;
    std::string err;
    // Kernel timing (ljmd_set_profiling): event pairs per family, resolved lazily.
    bool profiling = false;
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    std::vector<std::pair<int, size_t>> ev_marks;  // (family, index of start event)
    double ms[LJMD_NKT] = {};
    int64_t count[LJMD_NKT] = {};
    // The workspace: lists start at off_nbr and may grow to its end.
    uint8_t *ws = nullptr;
    size_t ws_bytes = 0, off_nbr = 0;
    int64_t npad = 0;
    int32_t recoveries = 0;  // list overflows recovered since ljmd_create
    // Bumped by every call that changes the dynamical state or the potential.
    uint64_t gen = 0;
    AdjRecord adj;
    ~ljmd_ctx() {
        for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
    }
};

static thread_local std::string g_create_err;

namespace {

constexpr double kTwo32 = 4294967296.0;

int fail(ljmd_ctx *c, int code, const char *fmt, ...) __attribute__((format(printf, 3, 4)));
int fail(ljmd_ctx *c, int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c)
        c->err = buf;
    else
        g_create_err = buf;
    return code;
}

int hip_fail(ljmd_ctx *c, hipError_t e, const char *what) {
    return fail(c, LJMD_EHIP, "%s: %s", what, hipGetErrorString(e));
}

bool used_pair(const ljmd_params *p, int ab) { return p->nspecies == 2 || ab == 0; }

// Every used cutoff infinite: the untruncated all-pairs interaction.
bool all_pairs(const ljmd_params *p) {
    for (int ab = 0; ab < 4; ++ab)
        if (used_pair(p, ab) && !std::isinf(p->rcut[ab])) return false;
    return true;
}

double list_radius_max(const ljmd_params *p) {
    double r = 0.0;
    for (int ab = 0; ab < 4; ++ab)
        if (used_pair(p, ab)) r = std::max(r, p->rcut[ab] + p->skin);
    return r;
}

int validate(const ljmd_params *p, std::string *why) {
    auto bad = [&](const char *m) {
        if (why) *why = m;
        return LJMD_EINVAL;
    };
    if (!p) return bad("params is NULL");
    if (p->n < 2 || p->n > (int64_t)INT32_MAX - 1024) return bad("n must be in [2, 2^31 - 1024)");
    for (int k = 0; k < 3; ++k)
        if (!(p->box[k] > 0.0) || !std::isfinite(p->box[k])) return bad("box edges must be finite and > 0");
    if (p->nspecies != 1 && p->nspecies != 2) return bad("nspecies must be 1 or 2");
    for (int ab = 0; ab < 4; ++ab) {
        if (!used_pair(p, ab)) continue;
        if (!(p->eps[ab] >= 0.0) || !std::isfinite(p->eps[ab])) return bad("eps must be finite and >= 0");
        if (!(p->sigma[ab] > 0.0) || !std::isfinite(p->sigma[ab])) return bad("sigma must be finite and > 0");
        if (!(p->rcut[ab] > 0.0)) return bad("rcut must be > 0 (or +inf for the all-pairs interaction)");
    }
    bool any_inf = false;
    for (int ab = 0; ab < 4; ++ab) any_inf = any_inf || (used_pair(p, ab) && std::isinf(p->rcut[ab]));
    if (any_inf && !all_pairs(p)) return bad("rcut: either every used cutoff is +inf (all pairs) or none");
    if (p->nspecies == 2 &&
        (p->eps[1] != p->eps[2] || p->sigma[1] != p->sigma[2] || p->rcut[1] != p->rcut[2]))
        return bad("pair tables must be symmetric ([1] == [2])");
    for (int s = 0; s < p->nspecies; ++s)
        if (!(p->mass[s] > 0.0) || !std::isfinite(p->mass[s])) return bad("masses must be finite and > 0");
    if (!(p->skin >= 0.0) || !std::isfinite(p->skin)) return bad("skin must be finite and >= 0");
    if (!(p->dt > 0.0) || !std::isfinite(p->dt)) return bad("dt must be finite and > 0");
    if (p->sort_interval < 0) return bad("sort_interval must be >= 0");
    if (p->precision != LJMD_FP64 && p->precision != LJMD_FP32_DS && p->precision != LJMD_FP32)
        return bad("unknown precision");
    if (p->nbr_capacity < 0 || p->nbr_capacity > 4096) return bad("nbr_capacity must be in [0, 4096]");
    if (p->cell_capacity < 0 || p->cell_capacity > 768) return bad("cell_capacity must be in [0, 768]");
    if (p->lanes != 0 && p->lanes != 1 && p->lanes != 2 && p->lanes != 4 && p->lanes != 8 && p->lanes != 16)
        return bad("lanes must be 0, 1, 2, 4, 8 or 16");
    if (p->cell_split < 0 || p->cell_split > 2) return bad("cell_split must be 0, 1 or 2");
    if (p->dim != 0 && p->dim != 2 && p->dim != 3) return bad("dim must be 0, 2 or 3");
    if (p->pad != 0) return bad("pad must be 0");
    if (all_pairs(p)) {
        // Minimum image of every pair; the single-precision paths work in
        // fixed-point quanta of a cubic box.
        if (p->precision != LJMD_FP64 && !(p->box[0] == p->box[1] && p->box[1] == p->box[2]))
            return bad("the all-pairs interaction in single precision needs a cubic box");
        return LJMD_OK;
    }
    const double rl = list_radius_max(p);
    for (int k = 0; k < 3; ++k)
        if (p->box[k] < 2.0 * rl) {
            if (why) *why = "box edge < 2 * (rcut + skin): minimum image would be ambiguous";
            return LJMD_EBOX;
        }
    return LJMD_OK;
}

// Cells per list radius along each axis (ljmd_params.cell_split).
int cell_split(const ljmd_params *p) { return p->cell_split == 2 ? 2 : 1; }

// Spatial dimension of a parameter set (0 reads as 3).
int dim_of(const ljmd_params *p) { return p->dim == 2 ? 2 : 3; }

void grid_dims(const ljmd_params *p, int nc[3]) {
    const double edge = list_radius_max(p) / cell_split(p);
    for (int k = 0; k < 3; ++k) {
        double f = std::floor(p->box[k] / (edge * (1.0 + 1e-6)));
        nc[k] = (int)std::max(1.0, std::min(f, 1024.0));
    }
    // In two dimensions every particle sits at z = 0: one layer of cells.
    if (dim_of(p) == 2) nc[2] = 1;
}

struct Plan {
    int64_t npad;
    int32_t cap, cell_cap, lanes;
    int32_t cap_reserve;  // list slots per particle the workspace holds (>= cap): room to grow
    int nc[3];
    int ncell;
    int max_blocks;
    // byte offsets
    size_t off_rec[2], off_vel, off_frc, off_dsw[3], off_img, off_id,
        off_xref, off_nbr, off_cnt, off_ccount, off_cmem, off_cstart, off_rank, off_lin, off_scratch,
        off_part, off_rebuilt, off_ctl;
    size_t total;
};

inline size_t al(size_t b) { return (b + 255) & ~(size_t)255; }

// Bytes of the neighbour lists of npad slots with cap entries each.
inline size_t list_bytes(int64_t npad, int32_t cap) { return sizeof(int32_t) * ((size_t)npad * cap + kListPad); }

int32_t round_up(int32_t v, int32_t m) { return (v + m - 1) / m * m; }

void lay_out(Plan &pl, int prec, int nctl);

Plan make_plan(const ljmd_params *p) {
    Plan pl{};
    pl.npad = (p->n + 63) / 64 * 64;
    grid_dims(p, pl.nc);
    pl.ncell = pl.nc[0] * pl.nc[1] * pl.nc[2];
    if (all_pairs(p)) {
        // No lists and one (unused) cell; the list area holds the partial
        // force rows of the j splits, one particle per lane of the step tail.
        pl.lanes = 1;
        pl.cell_cap = 8;
        const size_t pb = allpairs_part_bytes(p->n, p->precision);
        pl.cap = 16;
        pl.cap_reserve = std::max<int32_t>(
            16, round_up((int32_t)((pb + sizeof(int32_t) * pl.npad - 1) / (sizeof(int32_t) * pl.npad)), 16));
        pl.max_blocks = (int)((p->n + kApFinishBlock - 1) / kApFinishBlock);
        lay_out(pl, p->precision, 1);
        return pl;
    }
    const double vol = p->box[0] * p->box[1] * p->box[2];
    const double rho = (double)p->n / vol;
    const double rl = list_radius_max(p);
    const double nl = 4.0 / 3.0 * M_PI * rl * rl * rl * rho;
    int32_t cap = p->nbr_capacity;
    if (cap == 0) {
        double c = std::max(1.5 * nl, nl + 40.0);
        cap = (int32_t)std::min<double>(c, 4096.0);
        cap = std::min<int64_t>(cap, p->n);
    }
    // Measured on MI355X at N=256,000: 2 lanes per particle for FP32, 4 for FP64.
    pl.lanes = p->lanes != 0 ? p->lanes : (p->precision == LJMD_FP64 ? 4 : 2);
    pl.cap = std::max<int32_t>(16, round_up(cap, cap_granule(pl.lanes)));
    // With an automatic capacity the workspace holds twice the initial list
    // (up to 4096 slots), so that an overflow can be recovered by growing the
    // list in place; an explicit capacity reserves exactly itself (a larger
    // workspace passed to ljmd_create adds room).
    pl.cap_reserve = p->nbr_capacity == 0
                         ? std::max(pl.cap, std::min<int32_t>(4096 / cap_granule(pl.lanes) * cap_granule(pl.lanes),
                                                              2 * pl.cap))
                         : pl.cap;
    int32_t cc = p->cell_capacity;
    if (cc == 0) {
        double cellv = vol / pl.ncell;
        double mean = rho * cellv;
        cc = (int32_t)std::min<double>(2.0 * mean + 32.0, 768.0);
        cc = (int32_t)std::min<int64_t>(cc, p->n);
    }
    pl.cell_cap = std::max<int32_t>(8, round_up(cc, 8));
    if (pl.cell_cap > 768) pl.cell_cap = 768;
    const int per_block = (step_block_threads(p->precision) / kWave) * (kWave / pl.lanes);
    pl.max_blocks = (int)((p->n + per_block - 1) / per_block);
    lay_out(pl, p->precision, 1);
    return pl;
}

// Byte offsets of every array in a workspace for pl.npad slots, pl.ncell
// cells, pl.max_blocks step-kernel blocks and nctl control-word sets.
void lay_out(Plan &pl, int prec, int nctl) {
    const int64_t N = pl.npad;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += al(bytes);
        return o;
    };
    if (prec == LJMD_FP64) {
        pl.off_rec[0] = take(sizeof(double4) * N);
        pl.off_rec[1] = take(sizeof(double4) * N);
        pl.off_vel = take(sizeof(double4) * N);
        pl.off_frc = take(sizeof(double4) * N);
    } else {
        pl.off_rec[0] = take(sizeof(int4) * N);
        pl.off_rec[1] = take(sizeof(int4) * N);
        for (int k = 0; k < 3; ++k) pl.off_dsw[k] = take(sizeof(float4) * N);
        pl.off_frc = take(sizeof(float4) * N);
    }
    pl.off_img = take(sizeof(int4) * N);
    pl.off_id = take(sizeof(int32_t) * N);
    pl.off_xref = take(sizeof(int4) * N);
    pl.off_cnt = take(sizeof(int32_t) * N);
    pl.off_ccount = take(sizeof(int32_t) * pl.ncell);
    pl.off_cmem = take(cell_rec_bytes(prec) * (size_t)pl.ncell * pl.cell_cap);
    pl.off_cstart = take(sizeof(int32_t) * (pl.ncell + 1));
    pl.off_rank = take(sizeof(int32_t) * pl.ncell);
    pl.off_lin = take(sizeof(int32_t) * pl.ncell);
    pl.off_scratch = take(resort_scratch_bytes(N, prec));
    pl.off_part = take(sizeof(double) * (size_t)kRing * pl.max_blocks * kNP);
    pl.off_rebuilt = take(sizeof(int32_t) * kRing);
    pl.off_ctl = take(sizeof(Ctl) * (size_t)nctl);
    // Lists last, so that a larger workspace is room for longer lists; one
    // row block past the end: the force kernel reads a few entries beyond a
    // list (they hold valid indices and are not used).
    pl.off_nbr = take(list_bytes(N, std::max(pl.cap, pl.cap_reserve)));
    pl.total = off;
}

// Skilling's transform from axes to the transposed Hilbert index (AIP Conf.
// Proc. 707, 381 (2004)), then bit interleaving to a scalar index.
uint64_t hilbert_index3(uint32_t x, uint32_t y, uint32_t z, int bits) {
    uint32_t X[3] = {x, y, z};
    if (bits <= 0) return 0;
    const uint32_t M = 1u << (bits - 1);
    for (uint32_t Q = M; Q > 1; Q >>= 1) {
        const uint32_t P = Q - 1;
        for (int i = 0; i < 3; ++i) {
            if (X[i] & Q) {
                X[0] ^= P;
            } else {
                const uint32_t t = (X[0] ^ X[i]) & P;
                X[0] ^= t;
                X[i] ^= t;
            }
        }
    }
    for (int i = 1; i < 3; ++i) X[i] ^= X[i - 1];
    uint32_t t = 0;
    for (uint32_t Q = M; Q > 1; Q >>= 1)
        if (X[2] & Q) t ^= Q - 1;
    for (int i = 0; i < 3; ++i) X[i] ^= t;
    uint64_t h = 0;
    for (int b = bits - 1; b >= 0; --b)
        for (int i = 0; i < 3; ++i) h = (h << 1) | ((X[i] >> b) & 1u);
    return h;
}

void fill_pairs(PairC &q, const ljmd_params &p);
void fill_quanta(BoxC &b, const PairC &q, double L);

void fill_constants(ljmd_ctx *c, const Plan &pl) {
    const ljmd_params &p = c->p;
    BoxC &b = c->box;
    for (int k = 0; k < 3; ++k) {
        const double L = p.box[k];
        b.L[k] = L;
        b.invL[k] = 1.0 / L;
        b.S[k] = kTwo32 / L;
        b.Lhi[k] = (float)L;
        b.Llo[k] = (float)(L - (double)b.Lhi[k]);
        const double qs = L / kTwo32;
        b.qs_hi[k] = (float)qs;
        b.qs_lo[k] = (float)(qs - (double)b.qs_hi[k]);
        const double ratio = qs / (double)b.qs_hi[k];
        b.r2c[k] = (float)(ratio * ratio);
        const double S = kTwo32 / L;
        b.S_hi[k] = (float)S;
        b.S_lo[k] = (float)(S - (double)b.S_hi[k]);
        b.nc[k] = pl.nc[k];
    }
    b.ncell = pl.ncell;
    b.cubic = (p.box[0] == p.box[1] && p.box[1] == p.box[2]) ? 1 : 0;
    b.reach = cell_split(&p);
    fill_pairs(c->pc, p);
    fill_quanta(b, c->pc, p.box[0]);
    DynC &d = c->dyn;
    for (int s = 0; s < 2; ++s) {
        const double m = p.mass[p.nspecies == 2 ? s : 0];
        d.mass[s] = m;
        d.massf[s] = (float)m;
        d.hdt_m[s] = 0.5 * p.dt / m;
        d.hdt_m_hi[s] = (float)d.hdt_m[s];
        d.hdt_m_lo[s] = (float)(d.hdt_m[s] - (double)d.hdt_m_hi[s]);
    }
    d.dt = p.dt;
    d.dt_hi = (float)p.dt;
    d.dt_lo = (float)(p.dt - (double)d.dt_hi);
    d.thr2 = (float)(0.25 * p.skin * p.skin);
}

// Pair constants per symmetric type (AA, AB, BB) from the 4-entry tables.
void fill_pairs(PairC &q, const ljmd_params &p) {
    const int src[3] = {0, 1, 3};
    for (int t = 0; t < 3; ++t) {
        const int ab = p.nspecies == 1 ? 0 : src[t];
        const double rc = p.rcut[ab], rl = p.rcut[ab] + p.skin;
        const double eps = p.eps[ab], sig = p.sigma[ab];
        q.rc2[t] = rc * rc;
        q.rl2[t] = rl * rl;
        q.sig2[t] = sig * sig;
        q.eps24[t] = 24.0 * eps;
        q.eps4[t] = 4.0 * eps;
        const double sr6 = std::pow(sig / rc, 6.0);
        q.shift[t] = p.shift_energy ? 4.0 * eps * (sr6 * sr6 - sr6) : 0.0;
        q.rc2f[t] = (float)q.rc2[t];
        q.rl2f[t] = (float)(rl * rl);
        q.sig2f[t] = (float)q.sig2[t];
        q.eps24f[t] = (float)q.eps24[t];
        q.eps4f[t] = (float)q.eps4[t];
        q.shiftf[t] = (float)q.shift[t];
    }
}

// Pair constants in units of the quantum of a cubic box of edge L.
void fill_quanta(BoxC &b, const PairC &q, double L) {
    const double qs = L / kTwo32;
    for (int t = 0; t < 3; ++t) {
        b.rc2q[t] = (float)(q.rc2[t] / (qs * qs));
        b.sig2q[t] = (float)(q.sig2[t] / (qs * qs));
        b.fq[t] = (float)(q.eps24[t] / qs);
        b.rl2q[t] = (float)(q.rl2[t] / (qs * qs));
    }
}

// Timing bracket around a group of launches of one kernel family. A
// stamped bracket records nothing itself: its two events go to a single
// launch (Launch::ev0 / ev1) that the dispatch stamps with the kernel's own
// start and end, so the measured time holds no marker packets.
struct Bracket {
    ljmd_ctx *c;
    int fam;
    size_t start = 0;
    bool on = false, stamp = false;
    Bracket(ljmd_ctx *cc, int f, bool stamped = false) : c(cc), fam(f), stamp(stamped) {
        if (!c->profiling) return;
        if (c->ev_used + 2 > c->ev_pool.size()) {
            for (int k = 0; k < 64; ++k) {
                hipEvent_t e;
                if (hipEventCreate(&e) != hipSuccess) return;
                c->ev_pool.push_back(e);
            }
        }
        start = c->ev_used;
        c->ev_used += 2;
        on = stamp || hipEventRecord(c->ev_pool[start], c->stream) == hipSuccess;
    }
    // Events for a stamped launch (null when not profiling).
    hipEvent_t ev(int k) const { return on && stamp ? c->ev_pool[start + k] : nullptr; }
    ~Bracket() {
        if (!on) return;
        if (stamp || hipEventRecord(c->ev_pool[start + 1], c->stream) == hipSuccess)
            c->ev_marks.push_back({fam, start});
    }
};

// Resolve recorded brackets into the per-family sums (synchronises).
int resolve_times(ljmd_ctx *c) {
    if (c->ev_marks.empty()) return LJMD_OK;
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "synchronise");
    for (auto &m : c->ev_marks) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, c->ev_pool[m.second], c->ev_pool[m.second + 1]) == hipSuccess) {
            c->ms[m.first] += ms;
            c->count[m.first] += 1;
        }
    }
    c->ev_marks.clear();
    c->ev_used = 0;
    return LJMD_OK;
}

Launch launcher(ljmd_ctx *c) {
    Launch L;
    L.st = &c->st;
    L.g = &c->g;
    L.box = &c->box;
    L.pc = &c->pc;
    L.dyn = &c->dyn;
    L.stream = c->stream;
    L.cur = c->cur;
    return L;
}

// The list rebuild of one step: binning, canonical cell order, [resort],
// list build. All kernels decide on the device whether to do anything.
int rebuild_sequence(ljmd_ctx *c, int64_t step, int forced, bool resort) {
    if (c->g.all_pairs) return LJMD_OK;  // no lists to build
    Launch L = launcher(c);
    hipError_t e;
    if (resort) {
        {
            Bracket b(c, 1);
            if ((e = launch_bin(L, step, forced)) != hipSuccess) return hip_fail(c, e, "bin");
            if ((e = launch_canon(L, step, forced)) != hipSuccess) return hip_fail(c, e, "canon");
        }
        {
            Bracket b(c, 2);
            if ((e = launch_resort(L)) != hipSuccess) return hip_fail(c, e, "resort");
        }
        Bracket b(c, 1);
        if ((e = launch_nlist(L, step, forced)) != hipSuccess) return hip_fail(c, e, "nlist");
        return LJMD_OK;
    }
    Bracket b(c, 1);
    if ((e = launch_bin(L, step, forced)) != hipSuccess) return hip_fail(c, e, "bin");
    if ((e = launch_canon(L, step, forced)) != hipSuccess) return hip_fail(c, e, "canon");
    if ((e = launch_nlist(L, step, forced)) != hipSuccess) return hip_fail(c, e, "nlist");
    return LJMD_OK;
}

int64_t padded(int64_t n) { return (n + 63) / 64 * 64; }

size_t rec_bytes(int prec) { return prec == LJMD_FP64 ? sizeof(double4) : sizeof(int4); }

void *rec_ptr(const ljmd_ctx *c, int which) {
    return c->g.prec == LJMD_FP64 ? (void *)c->st.rec64[which] : (void *)c->st.recq[which];
}

// Point record buffer `which` at other device memory of the same size (the
// kernels take the buffers from the state at each launch).
void set_rec_ptr(ljmd_ctx *c, int which, void *p) {
    if (c->g.prec == LJMD_FP64)
        c->st.rec64[which] = (double4 *)p;
    else
        c->st.recq[which] = (int4 *)p;
}

// Puts the context's own record buffers back on restore() and on scope exit.
struct RecBuffers {
    ljmd_ctx *c;
    void *p0, *p1;
    explicit RecBuffers(ljmd_ctx *ctx) : c(ctx), p0(rec_ptr(ctx, 0)), p1(rec_ptr(ctx, 1)) {}
    void restore() {
        set_rec_ptr(c, 0, p0);
        set_rec_ptr(c, 1, p1);
    }
    ~RecBuffers() { restore(); }
};

struct RunOpts {
    bool force_first = false;   // force the list build of the first step
    bool allow_resort = true;   // space-filling-curve resort every sort_interval steps
    bool final_obs = true;      // refresh the stored observables when obs_dev is NULL
    uint8_t *frames = nullptr;  // if set: record buffer before the run and after every step
    size_t frame_stride = 0;
};

// Steps s0 .. s0 + n - 1 from a state at rest before the list build of step
// s0: positions x_{s0} in record buffer c->cur, velocities half kicked. Row
// k of obs_dev (nullable) receives the observables of step s0 + k. With
// frames, every step writes its new records straight into frame k0 + k + 2
// (k0: the frame offset of step s0 - 1's records). Leaves c->cur at the last
// step's records and c->step at s0 + n - 1.
int step_range(ljmd_ctx *c, int64_t s0, int64_t n, double *obs_dev, const RunOpts &o, bool force_first,
               int64_t k0) {
    hipError_t e;
    const bool redirect = o.frames != nullptr;
    Launch L = launcher(c);
    int64_t first = s0;
    int pending = 0;
    int64_t row = 0;
    for (int64_t k = 0; k < n; ++k) {
        const int64_t s = s0 + k;
        const bool resort = o.allow_resort && c->p.sort_interval > 0 && s % c->p.sort_interval == 0;
        const int forced = (resort || (force_first && k == 0)) ? 1 : 0;
        int r = rebuild_sequence(c, s, forced, resort);
        if (r) return r;
        const bool last = k == n - 1;
        const bool observe = obs_dev != nullptr || (last && o.final_obs);
        const int mode = kFinalize | (last ? kStoreForce : kIntegrate) | (observe ? kObserve : 0);
        // Records of step s are frame k0 + k + 1; the integrate half writes frame k0 + k + 2.
        if (redirect && !last) set_rec_ptr(c, c->cur ^ 1, o.frames + (size_t)(k0 + k + 2) * o.frame_stride);
        L = launcher(c);
        {
            Bracket b(c, 0, !c->g.all_pairs);
            L.ev0 = b.ev(0);
            L.ev1 = b.ev(1);
            e = launch_step(L, s, forced, mode, (int)(s % kRing));
            L.ev0 = L.ev1 = nullptr;
            if (e != hipSuccess) return hip_fail(c, e, "step");
        }
        if (!last) c->cur ^= 1;
        ++pending;
        if (obs_dev && (pending == kRing || last)) {
            Bracket b(c, 3);
            if ((e = launch_obs_reduce(L, first, pending, c->nblocks, obs_dev, row)) != hipSuccess)
                return hip_fail(c, e, "obs");
            row += pending;
            first += pending;
            pending = 0;
        }
    }
    if (!obs_dev && o.final_obs) {
        Bracket b(c, 3);
        if ((e = launch_obs_reduce(L, s0 + n - 1, 1, c->nblocks, nullptr, 0)) != hipSuccess)
            return hip_fail(c, e, "obs");
    }
    c->step = s0 + n - 1;
    return LJMD_OK;
}

// nsteps velocity-Verlet steps from a state at rest (positions, velocities
// and forces of step c->step): integrate from the stored forces, then per
// step the rebuild sequence and the fused step kernel.
int run_steps(ljmd_ctx *c, int64_t nsteps, double *obs_dev, const RunOpts &o) {
    hipError_t e;
    const size_t fb = rec_bytes(c->g.prec) * (size_t)c->g.n;
    // With frames, every step writes its new records straight into the next
    // frame (the record buffers are pointed there); the buffers are restored
    // and the last frame copied back at the end.
    const bool redirect = o.frames && nsteps > 0;
    RecBuffers own(c);
    if (o.frames && (e = hipMemcpyAsync(o.frames, rec_ptr(c, c->cur), fb, hipMemcpyDeviceToDevice,
                                        c->stream)) != hipSuccess)
        return hip_fail(c, e, "frame copy");
    if (redirect) set_rec_ptr(c, c->cur ^ 1, o.frames + o.frame_stride);
    Launch L = launcher(c);
    {
        Bracket b(c, 3);
        if ((e = launch_integrate(L, c->step)) != hipSuccess) return hip_fail(c, e, "integrate");
    }
    c->cur ^= 1;
    RunOpts so = o;
    if (!redirect) so.frames = nullptr;
    const int64_t s0 = c->step + 1;
    int r = step_range(c, s0, nsteps, obs_dev, so, o.force_first, 0);
    if (r) return r;
    if (redirect) {
        void *final_frame = rec_ptr(c, c->cur);
        own.restore();
        if ((e = hipMemcpyAsync(rec_ptr(c, c->cur), final_frame, fb, hipMemcpyDeviceToDevice, c->stream)) !=
            hipSuccess)
            return hip_fail(c, e, "frame copy");
    }
    // Keep the event pool bounded on long profiled runs.
    if (c->profiling && c->ev_used > 8192) return resolve_times(c);
    return LJMD_OK;
}

// ---- list overflow: freeze, grow, redo ---------------------------------------

// Control words after the work enqueued so far (synchronises).
int read_ctl(ljmd_ctx *c, Ctl *h) {
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "synchronise");
    e = hipMemcpy(h, c->st.ctl, sizeof *h, hipMemcpyDeviceToHost);
    return e == hipSuccess ? LJMD_OK : hip_fail(c, e, "read control words");
}

int flags_status(ljmd_ctx *c, uint32_t flags) {
    if (flags & kErrNaN) return fail(c, LJMD_ENAN, "non-finite position detected");
    if (flags & kErrCell) return fail(c, LJMD_ECELL, "a cell exceeded cell_capacity=%d", c->g.cell_cap);
    if (flags & kErrList) return fail(c, LJMD_ENLIST, "a neighbour list exceeded nbr_capacity=%d", c->g.cap);
    return LJMD_OK;
}

// Largest list capacity the workspace holds.
int32_t cap_limit(const ljmd_ctx *c) {
    const size_t room = c->ws_bytes - c->off_nbr;
    const size_t pad = sizeof(int32_t) * kListPad;
    if (room <= pad) return 0;
    const int64_t slots = (int64_t)((room - pad) / sizeof(int32_t) / (size_t)c->npad);
    const int32_t gr = cap_granule(c->g.lanes);
    return (int32_t)std::min<int64_t>(4096, slots / gr * gr);
}

// After a list overflow (lists of `need` entries): a larger capacity within
// the workspace, the list area cleared to valid indices, the error and halt
// words and the cell counters cleared. LJMD_ENLIST if the workspace is too
// small.
int grow_lists(ljmd_ctx *c, int32_t need) {
    const int32_t gr = cap_granule(c->g.lanes);
    const int32_t want = round_up(std::max<int32_t>(need + 16, (int32_t)std::ceil(1.25 * need)), gr);
    const int32_t lim = cap_limit(c);
    if (need > lim)
        return fail(c, LJMD_ENLIST, "a neighbour list of %d entries exceeds the %d slots the workspace holds "
                                    "(nbr_capacity=%d)", need, lim, c->g.cap);
    c->g.cap = std::min(want, lim);
    hipError_t e = hipMemsetAsync(c->st.nbr, 0, list_bytes(c->npad, c->g.cap), c->stream);
    if (e == hipSuccess) e = hipMemsetAsync(&c->st.ctl->flags, 0, sizeof(uint32_t), c->stream);
    if (e == hipSuccess) e = hipMemsetAsync(&c->st.ctl->halt, 0, sizeof(int64_t), c->stream);
    if (e == hipSuccess) e = hipMemsetAsync(c->st.cell_count, 0, sizeof(int32_t) * c->box.ncell, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "grow lists");
    ++c->recoveries;
    return LJMD_OK;
}

// Check the latched errors; for a list overflow that the workspace can hold,
// grow the lists and set *redo (the caller repeats from ctl.halt). Any other
// error is returned.
int check_overflow(ljmd_ctx *c, Ctl *h, bool *redo) {
    *redo = false;
    hipError_t e = launch_max_fill(launcher(c));
    if (e != hipSuccess) return hip_fail(c, e, "max_fill");
    int r = read_ctl(c, h);
    if (r) return r;
    if (h->flags == 0u) return LJMD_OK;
    if (h->flags != kErrList) return flags_status(c, h->flags);
    if ((r = grow_lists(c, h->max_fill))) return r;
    *redo = true;
    return LJMD_OK;
}

// ---- differentiable rollout ----------------------------------------------
// A stored state is the record buffer in use plus the dynamical arrays:
// positions (double-single parts), velocities, forces of the step and image
// counters -- everything the next "integrate" reads.
int ckpt_elems(int prec, size_t elem[8]) {
    int k = 0;
    elem[k++] = rec_bytes(prec);
    if (prec == LJMD_FP64) {
        elem[k++] = sizeof(double4);  // velocities
        elem[k++] = sizeof(double4);  // forces
    } else {
        for (int q = 0; q < 4; ++q) elem[k++] = sizeof(float4);  // double-single state words, forces
    }
    elem[k++] = sizeof(int4);  // image counters
    return k;
}

AdjPlan adj_plan(const ljmd_params *p, int32_t nsteps, int32_t every, int32_t flags) {
    AdjPlan a;
    const int64_t npad = padded(p->n);
    size_t elem[8];
    const int ne = ckpt_elems(p->precision, elem);
    for (int q = 0; q < ne; ++q) a.ckpt_stride += al(elem[q] * (size_t)npad);
    a.nsteps = nsteps;
    a.every = every;
    a.nseg = (nsteps + every - 1) / every;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += al(bytes);
        return o;
    };
    a.off_ckpt = take((size_t)(a.nseg + 1) * a.ckpt_stride);
    a.frame_stride = al(rec_bytes(p->precision) * (size_t)npad);
    a.store_all = (flags & LJMD_ADJ_STORE_ALL) != 0;
    const int32_t nframes = a.store_all ? nsteps + 1 : std::min(every, nsteps) + 1;
    a.off_frames = take((size_t)nframes * a.frame_stride);
    a.off_lx = take(sizeof(double4) * (size_t)npad);
    a.off_lv = take(sizeof(double4) * (size_t)npad);
    a.off_g = take(sizeof(double4) * (size_t)npad);
    a.off_g2 = take(sizeof(double4) * (size_t)npad);
    if (a.store_all && a.reuse_lists()) a.off_marks = take(sizeof(int32_t) * (size_t)nsteps);
    a.off_rows = take(sizeof(double) * kNP * (size_t)((p->n + 63) / 64));
    a.total = off;
    return a;
}

// Copy the state into (save) or out of (restore) one stored state.
int ckpt_copy(ljmd_ctx *c, uint8_t *dst, bool save) {
    void *arr[8];
    int k = 0;
    arr[k++] = rec_ptr(c, c->cur);
    if (c->g.prec == LJMD_FP64) {
        arr[k++] = c->st.vel64;
        arr[k++] = c->st.frc64;
    } else {
        arr[k++] = c->st.dsw[0];
        arr[k++] = c->st.dsw[1];
        arr[k++] = c->st.dsw[2];
        arr[k++] = c->st.frc32;
    }
    arr[k++] = c->st.img;
    size_t elem[8];
    const int ne = ckpt_elems(c->g.prec, elem);
    if (ne != k) return fail(c, LJMD_EINVAL, "internal: checkpoint layout");
    const int64_t npad = padded(c->g.n);
    size_t off = 0;
    for (int q = 0; q < ne; ++q) {
        const size_t bytes = elem[q] * (size_t)c->g.n;
        hipError_t e = save ? hipMemcpyAsync(dst + off, arr[q], bytes, hipMemcpyDeviceToDevice, c->stream)
                            : hipMemcpyAsync(arr[q], dst + off, bytes, hipMemcpyDeviceToDevice, c->stream);
        if (e != hipSuccess) return hip_fail(c, e, save ? "checkpoint save" : "checkpoint restore");
        off += al(elem[q] * (size_t)npad);
    }
    return LJMD_OK;
}

// Lists built for `step` at the positions in use, cell counters cleared:
// the state at rest that ljmd_vv_forward leaves and ljmd_vv_backward restores.
int rebuild_at_rest(ljmd_ctx *c, int64_t step) {
    int r = rebuild_sequence(c, step, 1, false);
    if (r) return r;
    hipError_t e = launch_adjoint_cells(launcher(c), step, 1);
    return e == hipSuccess ? LJMD_OK : hip_fail(c, e, "clear cells");
}

// Device pointers of every array of a workspace laid out by lay_out.
void bind_state(State &s, const Plan &pl, uint8_t *b, int prec) {
    std::memset(&s, 0, sizeof s);
    if (prec == LJMD_FP64) {
        s.rec64[0] = (double4 *)(b + pl.off_rec[0]);
        s.rec64[1] = (double4 *)(b + pl.off_rec[1]);
        s.vel64 = (double4 *)(b + pl.off_vel);
        s.frc64 = (double4 *)(b + pl.off_frc);
    } else {
        s.recq[0] = (int4 *)(b + pl.off_rec[0]);
        s.recq[1] = (int4 *)(b + pl.off_rec[1]);
        for (int k = 0; k < 3; ++k) s.dsw[k] = (float4 *)(b + pl.off_dsw[k]);
        s.frc32 = (float4 *)(b + pl.off_frc);
    }
    s.img = (int4 *)(b + pl.off_img);
    s.id = (int32_t *)(b + pl.off_id);
    s.xref = (int4 *)(b + pl.off_xref);
    s.nbr = (int32_t *)(b + pl.off_nbr);
    s.nbr_cnt = (int32_t *)(b + pl.off_cnt);
    s.cell_count = (int32_t *)(b + pl.off_ccount);
    s.cell_rec = (void *)(b + pl.off_cmem);
    s.cell_start = (int32_t *)(b + pl.off_cstart);
    s.rank_of = (int32_t *)(b + pl.off_rank);
    s.cell_lin = (int32_t *)(b + pl.off_lin);
    s.scratch = b + pl.off_scratch;
    s.partials = (double *)(b + pl.off_part);
    s.rebuilt = (int32_t *)(b + pl.off_rebuilt);
    s.ctl = (Ctl *)(b + pl.off_ctl);
}

// ---- batches of systems ------------------------------------------------------

// Host description of a batch: per-system geometry and the flattened layout.
struct BatchGeom {
    std::vector<SysC> sys;
    std::vector<int32_t> sys_of_g16;
    std::vector<std::vector<int32_t>> rank;  // per system, local Hilbert ranks
    int64_t nslots = 0, ntot = 0, ncell = 0;
    int32_t cap = 0, cell_cap = 0, lanes = 0;
    int nblocks = 0;
    std::string why;
};

// Parameters of system k: the shared ones with its own count and cubic edge.
ljmd_params system_params(const ljmd_params *shared, const ljmd_system &y) {
    ljmd_params q = *shared;
    q.n = y.n;
    q.box[0] = q.box[1] = q.box[2] = y.box;
    return q;
}

int batch_geom(const ljmd_params *shared, const ljmd_system *ys, int32_t nsys, BatchGeom &bg, bool ranks) {
    if (!shared || !ys || nsys < 1 || nsys > 65536) {
        bg.why = "batch: NULL argument or nsys outside [1, 65536]";
        return LJMD_EINVAL;
    }
    if (shared->nspecies != 1 || shared->precision != LJMD_FP32_DS || all_pairs(shared) || dim_of(shared) != 3) {
        bg.why = "batch: one species, three dimensions and the FP32 + double-single path only";
        return LJMD_EINVAL;
    }
    bg.sys.resize(nsys);
    bg.lanes = shared->lanes != 0 ? shared->lanes : 2;
    const int per_block = (kBlock / kWave) * (kWave / bg.lanes);
    int64_t p_off = 0, in_off = 0, c_off = 0;
    int b_off = 0;
    int32_t cap = 0, cc = 0;
    for (int k = 0; k < nsys; ++k) {
        const ljmd_params q = system_params(shared, ys[k]);
        std::string why;
        const int r = validate(&q, &why);
        if (r != LJMD_OK) {
            bg.why = "batch system " + std::to_string(k) + ": " + why;
            return r;
        }
        const Plan pk = make_plan(&q);
        cap = std::max(cap, pk.cap);
        cc = std::max(cc, pk.cell_cap);
        SysC &y = bg.sys[k];
        std::memset(&y, 0, sizeof y);
        const int64_t npad = (q.n + per_block - 1) / per_block * per_block;
        y.p_off = p_off;
        y.in_off = in_off;
        y.n = (int32_t)q.n;
        y.id = k;
        y.c_off = (int32_t)c_off;
        y.b_off = b_off;
        y.nb = (int)(npad / per_block);
        // Box constants exactly as a single box of these parameters has them.
        BoxC &b = y.box;
        for (int a = 0; a < 3; ++a) {
            const double L = q.box[a];
            b.L[a] = L;
            b.invL[a] = 1.0 / L;
            b.S[a] = kTwo32 / L;
            b.Lhi[a] = (float)L;
            b.Llo[a] = (float)(L - (double)b.Lhi[a]);
            const double qs = L / kTwo32;
            b.qs_hi[a] = (float)qs;
            b.qs_lo[a] = (float)(qs - (double)b.qs_hi[a]);
            const double ratio = qs / (double)b.qs_hi[a];
            b.r2c[a] = (float)(ratio * ratio);
            b.S_hi[a] = (float)b.S[a];
            b.S_lo[a] = (float)(b.S[a] - (double)b.S_hi[a]);
            b.nc[a] = pk.nc[a];
        }
        b.ncell = pk.ncell;
        b.cubic = 1;
        b.reach = cell_split(&q);
        PairC pc;
        fill_pairs(pc, q);
        fill_quanta(b, pc, q.box[0]);
        if (ranks) {
            std::vector<int32_t> rk(pk.ncell);
            ljmd_hilbert_ranks(pk.nc[0], pk.nc[1], pk.nc[2], rk.data());
            bg.rank.push_back(std::move(rk));
        }
        p_off += npad;
        in_off += q.n;
        c_off += pk.ncell;
        b_off += y.nb;
    }
    if (p_off >= kQuantaMaxSlots) {
        bg.why = "batch: 2^28 particle slots or more";
        return LJMD_EINVAL;
    }
    bg.nslots = p_off;
    bg.ntot = in_off;
    bg.ncell = c_off;
    bg.nblocks = b_off;
    bg.cap = std::max<int32_t>(
        16, round_up(shared->nbr_capacity != 0 ? shared->nbr_capacity : cap, cap_granule(bg.lanes)));
    bg.cell_cap = shared->cell_capacity != 0 ? std::min<int32_t>(768, std::max<int32_t>(8, round_up(shared->cell_capacity, 8))) : cc;
    bg.sys_of_g16.resize(bg.nslots / 16);
    for (int k = 0; k < nsys; ++k) {
        const SysC &y = bg.sys[k];
        const int64_t npad = (int64_t)y.nb * per_block;
        for (int64_t g = y.p_off / 16; g < (y.p_off + npad) / 16; ++g) bg.sys_of_g16[g] = k;
    }
    return LJMD_OK;
}

// Workspace of a batch: the single-box layout over every slot and cell, one
// set of control words per system, then the system tables and the plan.
struct BatchLayout {
    Plan pl;
    size_t off_sys = 0, off_g16 = 0, off_due = 0, off_wlsys = 0, off_wlpoff = 0, off_wlcoff = 0,
           off_wlcnt = 0, total = 0;
};

BatchLayout batch_layout(const BatchGeom &bg, int nsys) {
    BatchLayout bl;
    Plan &pl = bl.pl;
    pl = Plan{};
    pl.npad = bg.nslots;
    pl.ncell = (int)bg.ncell;
    pl.cap = bg.cap;
    pl.cap_reserve = bg.cap;
    pl.cell_cap = bg.cell_cap;
    pl.lanes = bg.lanes;
    pl.max_blocks = bg.nblocks;
    lay_out(pl, LJMD_FP32_DS, nsys);
    size_t off = pl.total;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += al(bytes);
        return o;
    };
    bl.off_sys = take(sizeof(SysC) * (size_t)nsys);
    bl.off_g16 = take(sizeof(int32_t) * bg.sys_of_g16.size());
    bl.off_due = take(sizeof(int32_t) * (size_t)nsys);
    bl.off_wlsys = take(sizeof(int32_t) * (size_t)nsys);
    bl.off_wlpoff = take(sizeof(int64_t) * (size_t)(nsys + 1));
    bl.off_wlcoff = take(sizeof(int64_t) * (size_t)(nsys + 1));
    bl.off_wlcnt = take(sizeof(int32_t));
    bl.total = off;
    return bl;
}

}  // namespace

namespace ljmd {

void box_pair_constants(const ljmd_params &p, BoxC &b, PairC &q) {
    std::memset(&b, 0, sizeof b);
    for (int k = 0; k < 3; ++k) {
        const double L = p.box[k];
        b.L[k] = L;
        b.invL[k] = 1.0 / L;
        b.S[k] = kTwo32 / L;
        b.Lhi[k] = (float)L;
        b.Llo[k] = (float)(L - (double)b.Lhi[k]);
        const double qs = L / kTwo32;
        b.qs_hi[k] = (float)qs;
        b.qs_lo[k] = (float)(qs - (double)b.qs_hi[k]);
        const double ratio = qs / (double)b.qs_hi[k];
        b.r2c[k] = (float)(ratio * ratio);
        b.S_hi[k] = (float)b.S[k];
        b.S_lo[k] = (float)(b.S[k] - (double)b.S_hi[k]);
        b.nc[k] = 1;
    }
    b.ncell = 1;
    b.cubic = (p.box[0] == p.box[1] && p.box[1] == p.box[2]) ? 1 : 0;
    b.reach = 1;
    fill_pairs(q, p);
    fill_quanta(b, q, p.box[0]);
}

int check_params_why(const ljmd_params *p, const char **why) {
    static thread_local std::string w;
    w.clear();
    const int r = validate(p, &w);
    if (why) *why = w.c_str();
    return r;
}

void set_global_error(const char *msg) { g_create_err = msg; }

}  // namespace ljmd

extern "C" {

int32_t ljmd_abi_version(void) { return LJMD_ABI_VERSION; }

int ljmd_check_params(const ljmd_params *p) { return validate(p, nullptr); }

size_t ljmd_workspace_size(const ljmd_params *p) {
    if (validate(p, nullptr) != LJMD_OK) return 0;
    return make_plan(p).total;
}

int ljmd_cell_grid(const ljmd_params *p, int32_t ncell[3]) {
    int r = validate(p, nullptr);
    if (r != LJMD_OK) return r;
    if (!ncell) return LJMD_EINVAL;
    int nc[3];
    grid_dims(p, nc);
    for (int k = 0; k < 3; ++k) ncell[k] = nc[k];
    return LJMD_OK;
}

int ljmd_hilbert_ranks(int32_t nx, int32_t ny, int32_t nz, int32_t *rank_out) {
    if (nx < 1 || ny < 1 || nz < 1 || !rank_out) return LJMD_EINVAL;
    if ((int64_t)nx * ny * nz > (int64_t)1 << 28) return LJMD_EINVAL;
    int bits = 0;
    while ((1 << bits) < std::max(nx, std::max(ny, nz))) ++bits;
    const int64_t nc = (int64_t)nx * ny * nz;
    std::vector<std::pair<uint64_t, int32_t>> keys;
    try {
        keys.resize(nc);
    } catch (...) {
        return LJMD_EINVAL;
    }
    for (int32_t x = 0; x < nx; ++x)
        for (int32_t y = 0; y < ny; ++y)
            for (int32_t z = 0; z < nz; ++z) {
                const int32_t lin = (x * ny + y) * nz + z;
                keys[lin] = {hilbert_index3(x, y, z, bits), lin};
            }
    std::sort(keys.begin(), keys.end());
    for (int64_t r = 0; r < nc; ++r) rank_out[keys[r].second] = (int32_t)r;
    return LJMD_OK;
}

int ljmd_create(const ljmd_params *p, void *ws, size_t bytes, void *stream, ljmd_ctx **out) {
    if (!out) return fail(nullptr, LJMD_EINVAL, "out is NULL");
    *out = nullptr;
    std::string why;
    int r = validate(p, &why);
    if (r != LJMD_OK) return fail(nullptr, r, "%s", why.c_str());
    if (!ws) return fail(nullptr, LJMD_EINVAL, "workspace is NULL");
    if (((uintptr_t)ws & 255) != 0) return fail(nullptr, LJMD_EINVAL, "workspace must be 256-byte aligned");
    Plan pl = make_plan(p);
    if (bytes < pl.total)
        return fail(nullptr, LJMD_ENOMEM, "workspace has %zu bytes, needs %zu", bytes, pl.total);
    ljmd_ctx *c = new (std::nothrow) ljmd_ctx();
    if (!c) return fail(nullptr, LJMD_ENOMEM, "host allocation failed");
    c->p = *p;
    c->stream = (hipStream_t)stream;
    if (hipGetDevice(&c->device) != hipSuccess) c->device = -1;
    fill_constants(c, pl);
    Geom &g = c->g;
    g.n = p->n;
    g.cap = pl.cap;
    g.cell_cap = pl.cell_cap;
    g.lanes = pl.lanes;
    g.nspecies = p->nspecies;
    g.prec = p->precision;
    g.max_blocks = pl.max_blocks;
    g.all_pairs = all_pairs(p) ? 1 : 0;
    g.dim = dim_of(p);
    g.ncu = 256;
    if (c->device >= 0) {
        int ncu = 0;
        if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, c->device) ==
                hipSuccess &&
            ncu > 0)
            g.ncu = ncu;
    }
    c->nblocks = pl.max_blocks;
    c->ws = (uint8_t *)ws;
    c->ws_bytes = bytes;
    c->off_nbr = pl.off_nbr;
    c->npad = pl.npad;
    uint8_t *b = (uint8_t *)ws;
    State &s = c->st;
    bind_state(s, pl, b, p->precision);

    std::vector<int32_t> rank(pl.ncell), lin(pl.ncell);
    ljmd_hilbert_ranks(pl.nc[0], pl.nc[1], pl.nc[2], rank.data());
    for (int k = 0; k < pl.ncell; ++k) lin[rank[k]] = k;
    hipError_t e = hipMemcpyAsync(s.rank_of, rank.data(), sizeof(int32_t) * pl.ncell,
                                  hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(s.cell_lin, lin.data(), sizeof(int32_t) * pl.ncell, hipMemcpyHostToDevice,
                           c->stream);
    if (e == hipSuccess) e = hipMemsetAsync(s.cell_count, 0, sizeof(int32_t) * pl.ncell, c->stream);
    if (e == hipSuccess) e = hipMemsetAsync(s.ctl, 0, sizeof(Ctl), c->stream);
    if (e == hipSuccess) e = hipMemsetAsync(s.nbr_cnt, 0, sizeof(int32_t) * pl.npad, c->stream);
    // Every list slot holds a valid particle index from the start (0).
    if (e == hipSuccess) e = hipMemsetAsync(s.nbr, 0, list_bytes(pl.npad, pl.cap), c->stream);
    // The rank table comes from pageable host memory: finish before it goes away.
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        int rc = fail(nullptr, LJMD_EHIP, "workspace initialisation: %s", hipGetErrorString(e));
        delete c;
        return rc;
    }
    *out = c;
    return LJMD_OK;
}

int ljmd_destroy(ljmd_ctx *c) {
    delete c;
    return LJMD_OK;
}

int ljmd_set_state(ljmd_ctx *c, const double *x, const double *v, const int32_t *species) {
    if (!c) return LJMD_EINVAL;
    if (!x || !v || !species) return fail(c, LJMD_EINVAL, "set_state: NULL array");
    c->cur = 0;
    c->step = 0;
    ++c->gen;
    hipError_t e = hipMemsetAsync(c->st.ctl, 0, sizeof(Ctl), c->stream);
    if (e == hipSuccess) e = hipMemsetAsync(c->st.cell_count, 0, sizeof(int32_t) * c->box.ncell, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "set_state memset");
    Launch L = launcher(c);
    if ((e = launch_set_state(L, x, v, species)) != hipSuccess) return hip_fail(c, e, "set_state");
    int r = rebuild_sequence(c, 0, 1, true);
    if (r) return r;
    for (;;) {
        L = launcher(c);
        if ((e = launch_step(L, 0, 1, kStoreForce | kObserve, 0)) != hipSuccess) return hip_fail(c, e, "force");
        if ((e = launch_obs_reduce(L, 0, 1, c->nblocks, nullptr, 0)) != hipSuccess)
            return hip_fail(c, e, "obs");
        // A list overflow of the first build: grow the lists and build again
        // (the positions stay where the state load put them).
        Ctl h;
        bool redo = false;
        if ((r = check_overflow(c, &h, &redo))) return r;
        if (!redo) break;
        if ((r = rebuild_sequence(c, 0, 1, false))) return r;
    }
    c->have_state = true;
    return LJMD_OK;
}

int ljmd_run(ljmd_ctx *c, int64_t nsteps, double *obs_dev) {
    if (!c) return LJMD_EINVAL;
    if (!c->have_state) return fail(c, LJMD_ESTATE, "run before set_state");
    if (nsteps < 0) return fail(c, LJMD_EINVAL, "nsteps < 0");
    if (nsteps == 0) return LJMD_OK;
    ++c->gen;
    const int64_t first = c->step + 1, last = c->step + nsteps;
    const int cur_first = c->cur ^ 1;  // the records of step `first`, written by the integrate half
    int r = run_steps(c, nsteps, obs_dev, RunOpts{});
    if (r) return r;
    // One wait at the end: a list that overflowed froze every later kernel
    // (no step ran on a truncated list); grow the lists and redo from the
    // step that stopped, until the run is through or the workspace is full.
    for (;;) {
        Ctl h;
        bool redo = false;
        if ((r = check_overflow(c, &h, &redo))) return r;
        if (!redo) return LJMD_OK;
        const int64_t hs = h.halt - 1;
        if (h.halt == 0 || hs < first || hs > last)
            return fail(c, LJMD_ENLIST, "internal: list overflow without a halted step in the run");
        c->cur = cur_first ^ (int)((hs - first) & 1);
        RunOpts o;
        if ((r = step_range(c, hs, last - hs + 1, obs_dev ? obs_dev + (size_t)(hs - first) * LJMD_NOBS : nullptr, o,
                            true, 0)))
            return r;
    }
}

int ljmd_set_thermostat(ljmd_ctx *c, double temperature, double rate, uint64_t seed) {
    if (!c) return LJMD_EINVAL;
    if (!(rate >= 0.0) || !std::isfinite(rate) || !(temperature >= 0.0) || !std::isfinite(temperature))
        return fail(c, LJMD_EINVAL, "set_thermostat: temperature and rate must be finite and >= 0");
    DynC &d = c->dyn;
    // Threshold floor(rate dt 2^32), saturated to the largest 32-bit word.
    const double t = std::floor(rate * c->p.dt * 4294967296.0);
    d.thermo_thr = !(t > 0.0) ? 0u : (t >= 4294967295.0 ? 0xFFFFFFFFu : (uint32_t)t);
    d.thermo_on = rate > 0.0 ? 1 : 0;
    d.seed_lo = (uint32_t)seed;
    d.seed_hi = (uint32_t)(seed >> 32);
    for (int s = 0; s < 2; ++s) d.thermo_sd[s] = std::sqrt(temperature / d.mass[s]);
    ++c->gen;
    return LJMD_OK;
}

int ljmd_set_profiling(ljmd_ctx *c, int enable) {
    if (!c) return LJMD_EINVAL;
    int r = resolve_times(c);
    for (int k = 0; k < LJMD_NKT; ++k) {
        c->ms[k] = 0.0;
        c->count[k] = 0;
    }
    c->profiling = enable != 0;
    return r;
}

int ljmd_kernel_times(ljmd_ctx *c, double ms[LJMD_NKT], int64_t count[LJMD_NKT]) {
    if (!c || !ms || !count) return LJMD_EINVAL;
    int r = resolve_times(c);
    for (int k = 0; k < LJMD_NKT; ++k) {
        ms[k] = c->ms[k];
        count[k] = c->count[k];
    }
    return r;
}

int ljmd_minimize_sd(ljmd_ctx *c, int32_t nsteps, double max_disp, double clamp, double *fmax_dev) {
    if (!c) return LJMD_EINVAL;
    if (c->g.all_pairs) return fail(c, LJMD_EINVAL, "minimize_sd: not available for the all-pairs interaction");
    if (!c->have_state) return fail(c, LJMD_ESTATE, "minimize_sd before set_state");
    if (nsteps < 0 || !(max_disp > 0.0) || !std::isfinite(max_disp) || !(clamp >= 0.0) ||
        !std::isfinite(clamp))
        return fail(c, LJMD_EINVAL, "minimize_sd: bad arguments");
    ++c->gen;
    hipError_t e = hipMemsetAsync(c->st.ctl->fmax, 0, sizeof(c->st.ctl->fmax), c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "minimize_sd memset");
    // Iteration s uses the control-word parity of id c->step + 1 + s; the
    // final state load below uses c->step again, as after ljmd_set_state.
    // After a list overflow (every later kernel frozen) the lists grow and
    // the iterations resume from the one that stopped.
    int32_t s_from = 0;
    bool final_only = false;
    for (;;) {
        for (int32_t s = final_only ? nsteps : s_from; s < nsteps; ++s) {
            const int64_t t = c->step + 1 + s;
            const int first = s == s_from ? 1 : 0;
            int r = rebuild_sequence(c, t, first, false);
            if (r) return r;
            if ((e = launch_sd(launcher(c), t, first, s, max_disp, clamp, fmax_dev)) != hipSuccess)
                return hip_fail(c, e, "steepest descent");
        }
        int r = rebuild_sequence(c, c->step, 1, true);
        if (r) return r;
        Launch L = launcher(c);
        if ((e = launch_step(L, c->step, 1, kStoreForce | kObserve, (int)(c->step % kRing))) != hipSuccess)
            return hip_fail(c, e, "force");
        if ((e = launch_obs_reduce(L, c->step, 1, c->nblocks, nullptr, 0)) != hipSuccess)
            return hip_fail(c, e, "obs");
        Ctl h;
        bool redo = false;
        if ((r = check_overflow(c, &h, &redo))) return r;
        if (!redo) return LJMD_OK;
        // halt = 1 + the step id that stopped: c->step for the final force,
        // c->step + 1 + s for iteration s.
        if (h.halt == c->step + 1) {
            final_only = true;
        } else if (h.halt >= c->step + 2 && h.halt <= c->step + 1 + nsteps) {
            s_from = (int32_t)(h.halt - c->step - 2);
            final_only = false;
        } else {
            return fail(c, LJMD_ENLIST, "internal: list overflow without a halted iteration");
        }
    }
}

int ljmd_get_state(ljmd_ctx *c, double *x, double *v, int32_t *img) {
    if (!c) return LJMD_EINVAL;
    if (!c->have_state) return fail(c, LJMD_ESTATE, "get_state before set_state");
    hipError_t e = launch_get_state(launcher(c), x, v, img);
    return e == hipSuccess ? LJMD_OK : hip_fail(c, e, "get_state");
}

int ljmd_get_forces(ljmd_ctx *c, double *f) {
    if (!c) return LJMD_EINVAL;
    if (!c->have_state) return fail(c, LJMD_ESTATE, "get_forces before set_state");
    if (!f) return fail(c, LJMD_EINVAL, "get_forces: NULL array");
    hipError_t e = launch_get_forces(launcher(c), f);
    return e == hipSuccess ? LJMD_OK : hip_fail(c, e, "get_forces");
}

int ljmd_neighbors(ljmd_ctx *c, int32_t *cnt, int32_t *ids, int32_t cap) {
    if (!c) return LJMD_EINVAL;
    if (c->g.all_pairs) return fail(c, LJMD_EINVAL, "neighbors: not available for the all-pairs interaction");
    if (!c->have_state) return fail(c, LJMD_ESTATE, "neighbors before set_state");
    if (!cnt || !ids || cap < 1) return fail(c, LJMD_EINVAL, "neighbors: bad arguments");
    hipError_t e = launch_neighbors(launcher(c), cnt, ids, cap);
    return e == hipSuccess ? LJMD_OK : hip_fail(c, e, "neighbors");
}

int ljmd_sync_status(ljmd_ctx *c) {
    if (!c) return LJMD_EINVAL;
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "synchronise");
    uint32_t flags = 0;
    e = hipMemcpy(&flags, &c->st.ctl->flags, sizeof flags, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(c, e, "read flags");
    return flags_status(c, flags);
}

int ljmd_observables(ljmd_ctx *c, ljmd_obs *out) {
    if (!c || !out) return LJMD_EINVAL;
    if (!c->have_state) return fail(c, LJMD_ESTATE, "observables before set_state");
    hipError_t e0 = launch_max_fill(launcher(c));
    if (e0 != hipSuccess) return hip_fail(c, e0, "max_fill");
    int r = ljmd_sync_status(c);
    Ctl h;
    hipError_t e = hipMemcpy(&h, c->st.ctl, sizeof h, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(c, e, "read observables");
    const double n = (double)c->p.n;
    const double d = (double)c->g.dim;
    const double vol = c->g.dim == 2 ? c->p.box[0] * c->p.box[1] : c->p.box[0] * c->p.box[1] * c->p.box[2];
    out->U = h.last[0];
    out->K = h.last[1];
    out->W = h.last[2];
    out->p[0] = h.last[3];
    out->p[1] = h.last[4];
    out->p[2] = h.last[5];
    out->T = 2.0 * out->K / (d * n - d);
    out->P = n / vol * out->T + out->W / (d * vol);
    out->E = out->U + out->K;
    out->step = c->step;
    out->rebuilds = h.rebuilds;
    out->max_fill = h.max_fill;
    out->nbr_capacity = c->g.cap;
    return r;
}

const char *ljmd_last_error(const ljmd_ctx *c) {
    return c ? c->err.c_str() : g_create_err.c_str();
}

// ---- gradients --------------------------------------------------------------

int ljmd_set_pair_params(ljmd_ctx *c, const double eps[4], const double sigma[4]) {
    if (!c) return LJMD_EINVAL;
    if (!eps || !sigma) return fail(c, LJMD_EINVAL, "set_pair_params: NULL array");
    ljmd_params q = c->p;
    for (int k = 0; k < 4; ++k) {
        q.eps[k] = eps[k];
        q.sigma[k] = sigma[k];
    }
    std::string why;
    int r = validate(&q, &why);
    if (r != LJMD_OK) return fail(c, r, "set_pair_params: %s", why.c_str());
    c->p = q;
    fill_pairs(c->pc, c->p);
    fill_quanta(c->box, c->pc, c->p.box[0]);
    ++c->gen;
    if (!c->have_state) return LJMD_OK;
    // Forces and observables of the current positions under the new values.
    Launch L = launcher(c);
    hipError_t e;
    if ((e = launch_step(L, c->step, 0, kStoreForce | kObserve, (int)(c->step % kRing))) != hipSuccess)
        return hip_fail(c, e, "force");
    if ((e = launch_obs_reduce(L, c->step, 1, c->nblocks, nullptr, 0)) != hipSuccess)
        return hip_fail(c, e, "obs");
    return LJMD_OK;
}

int ljmd_force_vjp(ljmd_ctx *c, const double *g, double *gx, double *gtheta) {
    if (!c) return LJMD_EINVAL;
    if (c->g.all_pairs) return fail(c, LJMD_EINVAL, "force_vjp: not available for the all-pairs interaction");
    if (c->g.dim != 3) return fail(c, LJMD_EINVAL, "force_vjp: three dimensions only");
    if (!c->have_state) return fail(c, LJMD_ESTATE, "force_vjp before set_state");
    if (!g || !gx || !gtheta) return fail(c, LJMD_EINVAL, "force_vjp: NULL array");
    // Scratch: the FP64 accumulator, then the cotangent in the path precision.
    const int64_t npad = padded(c->g.n);
    const size_t need = 2 * al(sizeof(double4) * (size_t)npad);
    if (resort_scratch_bytes(npad, c->g.prec) < need) return fail(c, LJMD_ENOMEM, "internal: scratch");
    uint8_t *scr = (uint8_t *)c->st.scratch;
    double4 *acc = (double4 *)scr;
    void *gv = scr + al(sizeof(double4) * (size_t)npad);
    Launch L = launcher(c);
    hipError_t e;
    if ((e = launch_adjoint_vec(L, kOpGatherG, g, nullptr, nullptr, nullptr, gv, 0.0)) != hipSuccess ||
        (e = launch_adjoint_vec(L, kOpZero, nullptr, nullptr, acc, nullptr, nullptr, 0.0)) != hipSuccess)
        return hip_fail(c, e, "force_vjp setup");
    {
        Bracket b(c, 4);
        if ((e = launch_adjoint_pairs(L, kAdjVjp, gv, acc, 1.0, gtheta, 1)) != hipSuccess)
            return hip_fail(c, e, "force_vjp");
    }
    if ((e = launch_adjoint_vec(L, kOpScatterById, nullptr, gx, acc, nullptr, nullptr, 0.0)) != hipSuccess)
        return hip_fail(c, e, "force_vjp scatter");
    return LJMD_OK;
}

int ljmd_energy_grad(ljmd_ctx *c, double *gtheta) {
    if (!c) return LJMD_EINVAL;
    if (c->g.all_pairs) return fail(c, LJMD_EINVAL, "energy_grad: not available for the all-pairs interaction");
    if (c->g.dim != 3) return fail(c, LJMD_EINVAL, "energy_grad: three dimensions only");
    if (!c->have_state) return fail(c, LJMD_ESTATE, "energy_grad before set_state");
    if (!gtheta) return fail(c, LJMD_EINVAL, "energy_grad: NULL array");
    hipError_t e = launch_adjoint_pairs(launcher(c), kAdjEnergy, nullptr, nullptr, 1.0, gtheta, 1);
    return e == hipSuccess ? LJMD_OK : hip_fail(c, e, "energy_grad");
}

size_t ljmd_adjoint_workspace_size(const ljmd_params *p, int32_t nsteps, int32_t ckpt_every,
                                   int32_t flags) {
    if (validate(p, nullptr) != LJMD_OK || nsteps < 1 || ckpt_every < 1 || (flags & ~LJMD_ADJ_STORE_ALL))
        return 0;
    return adj_plan(p, nsteps, ckpt_every, flags).total;
}

int ljmd_vv_forward(ljmd_ctx *c, int32_t nsteps, int32_t ckpt_every, int32_t flags, void *adj_ws,
                    size_t bytes, double *obs_dev) {
    if (!c) return LJMD_EINVAL;
    if (!c->have_state) return fail(c, LJMD_ESTATE, "vv_forward before set_state");
    if (nsteps < 1 || ckpt_every < 1) return fail(c, LJMD_EINVAL, "vv_forward: nsteps and ckpt_every must be >= 1");
    if (flags & ~LJMD_ADJ_STORE_ALL) return fail(c, LJMD_EINVAL, "vv_forward: unknown flags");
    if (c->g.all_pairs) return fail(c, LJMD_EINVAL, "vv_forward: not available for the all-pairs interaction");
    if (c->g.dim != 3) return fail(c, LJMD_EINVAL, "vv_forward: three dimensions only");
    if (c->dyn.thermo_on)
        return fail(c, LJMD_EINVAL, "vv_forward: the thermostat makes the dynamics stochastic (switch it off)");
    if (!adj_ws || ((uintptr_t)adj_ws & 255) != 0)
        return fail(c, LJMD_EINVAL, "vv_forward: workspace must be non-NULL and 256-byte aligned");
    const AdjPlan P = adj_plan(&c->p, nsteps, ckpt_every, flags);
    if (bytes < P.total)
        return fail(c, LJMD_ENOMEM, "vv_forward: workspace has %zu bytes, needs %zu", bytes, P.total);
    c->adj = AdjRecord{};
    ++c->gen;
    uint8_t *ws = (uint8_t *)adj_ws;
    const int64_t step0 = c->step;
    RunOpts o;
    o.force_first = true;
    o.allow_resort = false;
    o.frame_stride = P.frame_stride;
    for (;;) {
    for (int32_t seg = 0; seg < P.nseg; ++seg) {
        int r = ckpt_copy(c, ws + P.off_ckpt + (size_t)seg * P.ckpt_stride, true);
        if (r) return r;
        const int32_t s0 = seg * ckpt_every;
        const int32_t n = std::min(ckpt_every, nsteps - s0);
        if (P.store_all) o.frames = ws + P.off_frames + (size_t)s0 * P.frame_stride;
        const int64_t sb = c->step + 1;  // step id of the segment's first step
        if ((r = run_steps(c, n, obs_dev ? obs_dev + (size_t)s0 * LJMD_NOBS : nullptr, o))) return r;
        if (P.store_all && P.reuse_lists()) {
            // Step sb + k rebuilt (or not) from frame k + 1 of the segment.
            int32_t *marks = (int32_t *)(ws + P.off_marks) + s0;
            for (int32_t k = 0; k < n;) {
                const int slot = (int)((sb + k) % kRing);
                const int32_t len = std::min(n - k, (int32_t)(kRing - slot));
                hipError_t e = hipMemcpyAsync(marks + k, c->st.rebuilt + slot, sizeof(int32_t) * (size_t)len,
                                              hipMemcpyDeviceToDevice, c->stream);
                if (e != hipSuccess) return hip_fail(c, e, "rebuild markers");
                k += len;
            }
        }
    }
    int r = ckpt_copy(c, ws + P.off_ckpt + (size_t)P.nseg * P.ckpt_stride, true);
    if (r) return r;
    if ((r = rebuild_at_rest(c, c->step))) return r;
    // A list overflow froze the rollout: grow the lists and run it again
    // from the first stored state.
    Ctl h;
    bool redo = false;
    if ((r = check_overflow(c, &h, &redo))) return r;
    if (!redo) break;
    if ((r = ckpt_copy(c, ws + P.off_ckpt, false))) return r;
    c->step = step0;
    }
    c->adj.valid = true;
    c->adj.plan = P;
    c->adj.ws = ws;
    c->adj.step0 = step0;
    c->adj.gen = c->gen;
    return LJMD_OK;
}

int ljmd_vv_backward(ljmd_ctx *c, const double *lam_x, const double *lam_v, const double *gU, double *gx0,
                     double *gv0, double *gtheta) {
    if (!c) return LJMD_EINVAL;
    if (!c->adj.valid || c->adj.gen != c->gen)
        return fail(c, LJMD_ESTATE, "vv_backward without a matching vv_forward (state changed since)");
    if (!lam_x || !lam_v || !gx0 || !gv0 || !gtheta) return fail(c, LJMD_EINVAL, "vv_backward: NULL array");
    const AdjPlan &P = c->adj.plan;
    uint8_t *ws = c->adj.ws;
    double4 *lx = (double4 *)(ws + P.off_lx);
    double4 *lv = (double4 *)(ws + P.off_lv);
    // Cotangent buffers: a frame's VJP reads one while its epilogue writes
    // the next frame's into the other.
    void *gvb[2] = {ws + P.off_g, ws + P.off_g2};
    int gb = 0;
    double *rows = (double *)(ws + P.off_rows);
    if ((size_t)adjoint_rows(c->g) > (size_t)((c->g.n + 63) / 64))
        return fail(c, LJMD_EINVAL, "internal: adjoint rows");
    uint8_t *frames = ws + P.off_frames;
    const int64_t N = P.nsteps;
    const double dt = c->p.dt, h = 0.5 * c->p.dt;
    hipError_t e;
    // The sweep reads each frame in place (the current record buffer is
    // pointed at it); the context's buffers come back before every segment's
    // recompute, at the end and on any error.
    RecBuffers own(c);
    const int cur_entry = c->cur;
    const int64_t step_entry = c->step;
    Launch L;
    uint8_t *final_state = ws + P.off_ckpt + (size_t)P.nseg * P.ckpt_stride;
    for (;;) {
    // The final state (its stored forces F(x_N) too), whatever an earlier
    // attempt left.
    int r0 = ckpt_copy(c, final_state, false);
    if (r0) return r0;
    L = launcher(c);
    if ((e = launch_adjoint_vec(L, kOpGatherById, lam_x, nullptr, lx, nullptr, nullptr, 0.0)) != hipSuccess ||
        (e = launch_adjoint_vec(L, kOpGatherById, lam_v, nullptr, lv, nullptr, nullptr, 0.0)) != hipSuccess)
        return hip_fail(c, e, "vv_backward gather");
    // A loss term gU U(x_N): dU/dx_N = -F(x_N).
    if (gU && (e = launch_adjoint_vec(L, kOpSubForce, nullptr, nullptr, lx, nullptr, nullptr, 0.0, gU)) != hipSuccess)
        return hip_fail(c, e, "vv_backward energy cotangent");
    RunOpts o;
    o.force_first = true;
    o.allow_resort = false;
    o.final_obs = false;
    o.frames = frames;
    o.frame_stride = P.frame_stride;
    bool first = true;
    gb = 0;
    const bool reuse = P.reuse_lists();
    std::vector<int32_t> marks;
    if (reuse && P.store_all) {
        marks.resize((size_t)N);
        if ((e = hipMemcpyAsync(marks.data(), ws + P.off_marks, sizeof(int32_t) * (size_t)N, hipMemcpyDeviceToHost,
                                c->stream)) != hipSuccess ||
            (e = hipStreamSynchronize(c->stream)) != hipSuccess)
            return hip_fail(c, e, "vv_backward markers");
    }
    for (int32_t seg = P.nseg - 1; seg >= 0; --seg) {
        const int32_t s0 = seg * P.every;
        const int32_t n = std::min(P.every, P.nsteps - s0);
        int r;
        uint8_t *seg_frames = frames;
        // Frames the sweep of this segment reads: 0 .. n for the last
        // segment, 0 .. n - 1 for the others (their frame n is the next
        // segment's frame 0, already swept), so the recompute stops one step
        // short of the segment's end (segments of one step excepted).
        const int32_t nrec = (seg == P.nseg - 1 || n == 1) ? n : n - 1;
        if (P.store_all) {
            seg_frames = frames + (size_t)s0 * P.frame_stride;
            c->step = c->adj.step0 + s0 + nrec;
        } else {
            // Recompute the segment from its stored state, keeping its frames.
            own.restore();
            if ((r = ckpt_copy(c, ws + P.off_ckpt + (size_t)seg * P.ckpt_stride, false))) return r;
            c->step = c->adj.step0 + s0;
            if ((r = run_steps(c, nrec, nullptr, o))) return r;
        }
        // Sweep the frames backwards, with step ids that continue after the
        // segment's end (parity of the displacement words). With reuse, the
        // sweep starts from the list of the forward run's last build in the
        // segment: the recompute has just left it in place (and the
        // displacement word of step id c->step + 1 clear); with stored frames
        // it is built again from the frame the markers name, so both ways
        // give the same lists bit for bit. Every frame, the first included,
        // then follows the half-skin rule. Without reuse the lists are built
        // afresh at the first frame.
        int64_t t = c->step + 1;
        const int32_t top = seg == P.nseg - 1 ? n : n - 1;
        if (reuse && P.store_all) {
            int32_t fl = 1;
            for (int32_t k = 0; k < nrec; ++k)
                if (marks[(size_t)s0 + k]) fl = k + 1;
            L = launcher(c);
            set_rec_ptr(c, c->cur, seg_frames + (size_t)fl * P.frame_stride);
            if ((r = rebuild_sequence(c, t - 1, 1, false))) return r;
            if ((e = launch_adjoint_cells(L, t - 1, 1)) != hipSuccess) return hip_fail(c, e, "clear cells");
        }
        for (int32_t j = top; j >= 0; --j, ++t) {
            const int64_t s = (int64_t)s0 + j;
            const int forced = (!reuse && j == top) ? 1 : 0;
            L = launcher(c);
            set_rec_ptr(c, c->cur, seg_frames + (size_t)j * P.frame_stride);
            // Drift (lambda_v += dt lambda_x, none at the last frame), the
            // force cotangent lambda_v / m and, unless the list is forced,
            // the frame's displacement from the last build, in one pass: at
            // the segment's first frame on its own, later in the epilogue of
            // the previous frame's VJP.
            if (j == top &&
                (e = launch_adjoint_drift(L, lx, lv, gvb[gb], s != N ? dt : 0.0, t, forced ? 0 : 1)) != hipSuccess)
                return hip_fail(c, e, "vv_backward drift and cotangent");
            if ((r = rebuild_sequence(c, t, forced, false))) return r;
            // The VJP pass also clears the cell counters after a rebuild;
            // its parameter sums stay in block rows until the sweep ends.
            const double w = (s == N || s == 0) ? h : dt;
            AdjNext nx{lv, gvb[gb ^ 1], dt, t + 1, j > 0 ? seg_frames + (size_t)(j - 1) * P.frame_stride : nullptr};
            Bracket b(c, 4);
            if ((e = launch_adjoint_vjp_rows(L, gvb[gb], lx, w, rows, first ? 1 : 0, t, forced, j > 0 ? &nx : nullptr)) !=
                hipSuccess)
                return hip_fail(c, e, "vv_backward vjp");
            first = false;
            gb ^= 1;
        }
    }
    // The sweep builds lists at frames the forward run did not: a list that
    // overflowed there froze the recompute and spoilt the VJP passes. Grow
    // the lists and sweep again (the cotangent inputs are read again; the
    // outputs are written only after this check).
    {
        Ctl h;
        bool redo = false;
        int r = check_overflow(c, &h, &redo);
        if (r) return r;
        if (!redo) break;
        own.restore();
        c->cur = cur_entry;
        c->step = step_entry;
    }
    }
    L = launcher(c);
    if ((e = launch_adjoint_reduce(L, rows, gtheta)) != hipSuccess) return hip_fail(c, e, "vv_backward theta");
    if ((e = launch_adjoint_vec(L, kOpScatterById, nullptr, gx0, lx, nullptr, nullptr, 0.0)) != hipSuccess ||
        (e = launch_adjoint_vec(L, kOpScatterById, nullptr, gv0, lv, nullptr, nullptr, 0.0)) != hipSuccess)
        return hip_fail(c, e, "vv_backward scatter");
    // Back to the final state of the rollout, lists as ljmd_vv_forward left them.
    own.restore();
    int r = ckpt_copy(c, final_state, false);
    if (r) return r;
    c->step = c->adj.step0 + N;
    if ((r = rebuild_at_rest(c, c->step))) return r;
    if (gU) {
        // gtheta += gU dU/dtheta at x_N (the sweep's parameter rows are free
        // again and hold the six sums).
        L = launcher(c);
        if ((e = launch_adjoint_pairs(L, kAdjEnergy, nullptr, nullptr, 1.0, rows, 1)) != hipSuccess ||
            (e = launch_theta_axpy(L, gU, rows, gtheta)) != hipSuccess)
            return hip_fail(c, e, "vv_backward energy gradient");
    }
    return LJMD_OK;
}

}  // extern "C"

struct ljmd_batch {
    ljmd_params p;  // shared parameters
    int nsys = 0;
    BatchGeom bg;
    BatchLayout bl;
    Geom g;
    BoxC all;       // only ncell (every cell of the batch) is used
    PairC pc;
    DynC dyn;
    State st;
    SysC *sys = nullptr;
    int32_t *g16 = nullptr;
    BatchPlan bp;
    hipStream_t stream = nullptr;
    int device = 0;
    int cur = 0;
    int64_t step = 0;
    bool have_state = false;
    std::string err;
    // Graph replay of whole periods of steps (see batch_period): one graph
    // per value of cur at the period's start, captured on first use on a
    // private stream and launched on the batch's stream.
    bool graphs = true;
    hipStream_t cap_stream = nullptr;
    hipGraph_t period_graph[2] = {nullptr, nullptr};
    hipGraphExec_t period_exec[2] = {nullptr, nullptr};
    ~ljmd_batch() {
        for (int k = 0; k < 2; ++k) {
            if (period_exec[k]) (void)hipGraphExecDestroy(period_exec[k]);
            if (period_graph[k]) (void)hipGraphDestroy(period_graph[k]);
        }
        if (cap_stream) (void)hipStreamDestroy(cap_stream);
    }
};

namespace {

int bfail(ljmd_batch *b, int code, const char *fmt, ...) __attribute__((format(printf, 3, 4)));
int bfail(ljmd_batch *b, int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (b)
        b->err = buf;
    else
        g_create_err = buf;
    return code;
}

int bhip(ljmd_batch *b, hipError_t e, const char *what) {
    return bfail(b, LJMD_EHIP, "%s: %s", what, hipGetErrorString(e));
}

Launch blauncher(ljmd_batch *b) {
    Launch L;
    L.st = &b->st;
    L.g = &b->g;
    L.box = &b->all;
    L.pc = &b->pc;
    L.dyn = &b->dyn;
    L.stream = b->stream;
    L.cur = b->cur;
    return L;
}

// The list rebuild of one step for every system that needs it; a resort
// (every sort_interval steps, and at a state load) forces all of them.
int batch_rebuild(ljmd_batch *b, int64_t step, int forced, bool resort) {
    Launch L = blauncher(b);
    hipError_t e;
    if ((e = launch_batch_plan(L, b->sys, b->nsys, b->bp, step, forced)) != hipSuccess) return bhip(b, e, "plan");
    if ((e = launch_batch_bin(L, b->sys, b->bp, b->bg.ntot)) != hipSuccess) return bhip(b, e, "bin");
    if ((e = launch_batch_canon(L, b->sys, b->bp, b->bg.ncell)) != hipSuccess) return bhip(b, e, "canon");
    if (resort) {
        if ((e = launch_batch_scan(L, b->sys, b->nsys)) != hipSuccess) return bhip(b, e, "scan");
        if ((e = launch_batch_resort_move(L, b->bg.ncell)) != hipSuccess) return bhip(b, e, "resort");
    }
    if ((e = launch_batch_nlist(L, b->sys, b->bp, b->bg.ncell)) != hipSuccess) return bhip(b, e, "nlist");
    return LJMD_OK;
}

// One step s of every system: rebuild if due, then forces and both
// velocity-Verlet halves (the last step of a run stores forces and
// observables instead of starting the next step).
int batch_one_step(ljmd_batch *b, int64_t s, bool last) {
    const bool resort = b->p.sort_interval > 0 && s % b->p.sort_interval == 0;
    const int forced = resort ? 1 : 0;
    int r = batch_rebuild(b, s, forced, resort);
    if (r) return r;
    Launch L = blauncher(b);
    hipError_t e = launch_batch_step(L, b->sys, b->g16, b->bg.nblocks, s, forced,
                                     kFinalize | (last ? kStoreForce | kObserve : kIntegrate), (int)(s % kRing));
    if (e != hipSuccess) return bhip(b, e, "batch step");
    if (!last) b->cur ^= 1;
    return LJMD_OK;
}

// Steps per replayed graph: the resort period (doubled when odd), or 64
// without resorts. Every kernel of a step depends on the step number only
// through its parity, the resort schedule and the partials slot of observed
// steps (never inside a period), so a period captured at one multiple of
// this length replays unchanged at every other; its length is even, so the
// record buffer in use (cur) is the same at its start and end.
int64_t batch_period(const ljmd_batch *b) {
    const int64_t si = b->p.sort_interval;
    if (si <= 0) return 64;
    return si % 2 == 0 ? si : 2 * si;
}

// Steps s0 + 1 .. s0 + period as one graph launch (s0 a multiple of the
// period, none of them the last step of the run).
int batch_period_graph(ljmd_batch *b, int64_t s0) {
    const int64_t P = batch_period(b);
    const int k = b->cur;
    hipError_t e;
    if (!b->period_exec[k]) {
        if (!b->cap_stream && (e = hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking)) != hipSuccess)
            return bhip(b, e, "capture stream");
        hipStream_t user = b->stream;
        const int cur0 = b->cur;
        if ((e = hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal)) != hipSuccess)
            return bhip(b, e, "begin capture");
        b->stream = b->cap_stream;
        int r = LJMD_OK;
        for (int64_t q = 1; q <= P && r == LJMD_OK; ++q) r = batch_one_step(b, s0 + q, false);
        b->stream = user;
        b->cur = cur0;
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(b->cap_stream, &g);
        if (r != LJMD_OK) {
            if (g) (void)hipGraphDestroy(g);
            return r;
        }
        if (e != hipSuccess) return bhip(b, e, "end capture");
        hipGraphExec_t x = nullptr;
        if ((e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0)) != hipSuccess) {
            (void)hipGraphDestroy(g);
            return bhip(b, e, "graph instantiate");
        }
        b->period_graph[k] = g;
        b->period_exec[k] = x;
    }
    if ((e = hipGraphLaunch(b->period_exec[k], b->stream)) != hipSuccess) return bhip(b, e, "graph launch");
    return LJMD_OK;
}

}  // namespace

extern "C" {

size_t ljmd_batch_workspace_size(const ljmd_params *shared, const ljmd_system *sys, int32_t nsys) {
    BatchGeom bg;
    if (batch_geom(shared, sys, nsys, bg, false) != LJMD_OK) return 0;
    return batch_layout(bg, nsys).total;
}

int ljmd_batch_create(const ljmd_params *shared, const ljmd_system *sys, int32_t nsys, void *ws, size_t bytes,
                      void *stream, ljmd_batch **out) {
    if (!out) return bfail(nullptr, LJMD_EINVAL, "out is NULL");
    *out = nullptr;
    if (!ws) return bfail(nullptr, LJMD_EINVAL, "workspace is NULL");
    if (((uintptr_t)ws & 255) != 0) return bfail(nullptr, LJMD_EINVAL, "workspace must be 256-byte aligned");
    ljmd_batch *b = new (std::nothrow) ljmd_batch();
    if (!b) return bfail(nullptr, LJMD_ENOMEM, "host allocation failed");
    int r = batch_geom(shared, sys, nsys, b->bg, true);
    if (r != LJMD_OK) {
        bfail(nullptr, r, "%s", b->bg.why.c_str());
        delete b;
        return r;
    }
    b->bl = batch_layout(b->bg, nsys);
    if (bytes < b->bl.total) {
        delete b;
        return bfail(nullptr, LJMD_ENOMEM, "workspace has %zu bytes, needs %zu", bytes, b->bl.total);
    }
    b->p = *shared;
    b->nsys = nsys;
    b->stream = (hipStream_t)stream;
    if (hipGetDevice(&b->device) != hipSuccess) b->device = -1;
    // Shared constants from the first system's parameters (the potential,
    // masses, time step and skin are common).
    const ljmd_params q0 = system_params(shared, sys[0]);
    fill_pairs(b->pc, q0);
    DynC &d = b->dyn;
    for (int s = 0; s < 2; ++s) {
        const double m = q0.mass[0];
        d.mass[s] = m;
        d.massf[s] = (float)m;
        d.hdt_m[s] = 0.5 * q0.dt / m;
        d.hdt_m_hi[s] = (float)d.hdt_m[s];
        d.hdt_m_lo[s] = (float)(d.hdt_m[s] - (double)d.hdt_m_hi[s]);
    }
    d.dt = q0.dt;
    d.dt_hi = (float)q0.dt;
    d.dt_lo = (float)(q0.dt - (double)d.dt_hi);
    d.thr2 = (float)(0.25 * q0.skin * q0.skin);
    std::memset(&b->all, 0, sizeof b->all);
    b->all.ncell = (int32_t)b->bg.ncell;
    Geom &g = b->g;
    g.n = b->bg.nslots;
    g.cap = b->bg.cap;
    g.cell_cap = b->bg.cell_cap;
    g.lanes = b->bg.lanes;
    g.nspecies = 1;
    g.prec = LJMD_FP32_DS;
    g.max_blocks = b->bg.nblocks;
    g.dim = 3;
    g.ncu = 256;
    if (b->device >= 0) {
        int ncu = 0;
        if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, b->device) == hipSuccess && ncu > 0)
            g.ncu = ncu;
    }
    uint8_t *base = (uint8_t *)ws;
    const Plan &pl = b->bl.pl;
    bind_state(b->st, pl, base, LJMD_FP32_DS);
    b->sys = (SysC *)(base + b->bl.off_sys);
    b->g16 = (int32_t *)(base + b->bl.off_g16);
    b->bp.due = (int32_t *)(base + b->bl.off_due);
    b->bp.wl_sys = (int32_t *)(base + b->bl.off_wlsys);
    b->bp.wl_poff = (int64_t *)(base + b->bl.off_wlpoff);
    b->bp.wl_coff = (int64_t *)(base + b->bl.off_wlcoff);
    b->bp.wl_count = (int32_t *)(base + b->bl.off_wlcnt);
    // Tables: concatenated Hilbert ranks and their inverses, systems, slot groups.
    std::vector<int32_t> rank(b->bg.ncell), lin(b->bg.ncell);
    for (int k = 0; k < nsys; ++k) {
        const SysC &y = b->bg.sys[k];
        const std::vector<int32_t> &rk = b->bg.rank[k];
        for (int c = 0; c < y.box.ncell; ++c) {
            rank[y.c_off + c] = rk[c];
            lin[y.c_off + rk[c]] = c;
        }
    }
    hipError_t e = hipMemcpyAsync(b->st.rank_of, rank.data(), sizeof(int32_t) * rank.size(), hipMemcpyHostToDevice,
                                  b->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->st.cell_lin, lin.data(), sizeof(int32_t) * lin.size(), hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->sys, b->bg.sys.data(), sizeof(SysC) * nsys, hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->g16, b->bg.sys_of_g16.data(), sizeof(int32_t) * b->bg.sys_of_g16.size(),
                           hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) e = hipMemsetAsync(b->st.cell_count, 0, sizeof(int32_t) * b->bg.ncell, b->stream);
    if (e == hipSuccess) e = hipMemsetAsync(b->st.ctl, 0, sizeof(Ctl) * nsys, b->stream);
    if (e == hipSuccess) e = hipMemsetAsync(b->st.nbr_cnt, 0, sizeof(int32_t) * pl.npad, b->stream);
    if (e == hipSuccess)
        e = hipMemsetAsync(b->st.nbr, 0, sizeof(int32_t) * ((size_t)pl.npad * pl.cap + kListPad), b->stream);
    // The tables come from pageable host memory: finish before they go away.
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) {
        int rc = bfail(nullptr, LJMD_EHIP, "batch workspace initialisation: %s", hipGetErrorString(e));
        delete b;
        return rc;
    }
    *out = b;
    return LJMD_OK;
}

int ljmd_batch_destroy(ljmd_batch *b) {
    delete b;
    return LJMD_OK;
}

int ljmd_batch_max_fill(ljmd_batch *b, int32_t *out) {
    if (!b || !out) return LJMD_EINVAL;
    if (!b->have_state) return bfail(b, LJMD_ESTATE, "batch_max_fill before batch_set_state");
    hipError_t e = launch_max_fill(blauncher(b));
    if (e != hipSuccess) return bhip(b, e, "max_fill");
    // k_max_fill scans every slot of the batch into the first control set.
    if ((e = hipMemcpyAsync(out, &b->st.ctl->max_fill, sizeof(int32_t), hipMemcpyDeviceToHost, b->stream)) !=
            hipSuccess ||
        (e = hipStreamSynchronize(b->stream)) != hipSuccess)
        return bhip(b, e, "read max_fill");
    return LJMD_OK;
}

int ljmd_batch_use_graphs(ljmd_batch *b, int32_t enable) {
    if (!b) return LJMD_EINVAL;
    b->graphs = enable != 0;
    return LJMD_OK;
}

int ljmd_batch_set_state(ljmd_batch *b, const double *x, const double *v, const int32_t *species) {
    if (!b) return LJMD_EINVAL;
    if (!x || !v || !species) return bfail(b, LJMD_EINVAL, "batch_set_state: NULL array");
    b->cur = 0;
    b->step = 0;
    hipError_t e = hipMemsetAsync(b->st.ctl, 0, sizeof(Ctl) * b->nsys, b->stream);
    if (e == hipSuccess) e = hipMemsetAsync(b->st.cell_count, 0, sizeof(int32_t) * b->bg.ncell, b->stream);
    if (e != hipSuccess) return bhip(b, e, "batch_set_state memset");
    Launch L = blauncher(b);
    if ((e = launch_batch_set_state(L, b->sys, b->g16, b->bg.nslots, x, v, species)) != hipSuccess)
        return bhip(b, e, "batch_set_state");
    int r = batch_rebuild(b, 0, 1, true);
    if (r) return r;
    L = blauncher(b);
    if ((e = launch_batch_step(L, b->sys, b->g16, b->bg.nblocks, 0, 1, kStoreForce | kObserve, 0)) != hipSuccess)
        return bhip(b, e, "batch force");
    if ((e = launch_batch_obs(L, b->sys, b->nsys, 0, 0, nullptr)) != hipSuccess) return bhip(b, e, "batch obs");
    b->have_state = true;
    return LJMD_OK;
}

int ljmd_batch_run(ljmd_batch *b, int64_t nsteps, double *obs_dev) {
    if (!b) return LJMD_EINVAL;
    if (!b->have_state) return bfail(b, LJMD_ESTATE, "batch_run before batch_set_state");
    if (nsteps < 0) return bfail(b, LJMD_EINVAL, "nsteps < 0");
    if (nsteps == 0) return LJMD_OK;
    hipError_t e;
    Launch L = blauncher(b);
    if ((e = launch_batch_integrate(L, b->sys, b->g16, b->bg.nslots, b->step)) != hipSuccess)
        return bhip(b, e, "batch integrate");
    b->cur ^= 1;
    // Whole periods that do not hold the run's last step replay a captured
    // graph; the other steps are launched one by one.
    const int64_t P = batch_period(b);
    int64_t k = 0;
    while (k < nsteps) {
        const int64_t s = b->step + 1 + k;
        int r;
        if (b->graphs && (s - 1) % P == 0 && nsteps - k > P) {
            r = batch_period_graph(b, s - 1);
            k += P;
        } else {
            r = batch_one_step(b, s, k == nsteps - 1);
            ++k;
        }
        if (r) return r;
    }
    L = blauncher(b);
    b->step += nsteps;
    if ((e = launch_batch_obs(L, b->sys, b->nsys, (int)(b->step % kRing), b->step, obs_dev)) != hipSuccess)
        return bhip(b, e, "batch obs");
    return LJMD_OK;
}

int ljmd_batch_get_state(ljmd_batch *b, double *x, double *v, int32_t *img) {
    if (!b) return LJMD_EINVAL;
    if (!b->have_state) return bfail(b, LJMD_ESTATE, "batch_get_state before batch_set_state");
    hipError_t e = launch_batch_get_state(blauncher(b), b->sys, b->g16, b->bg.nslots, x, v, img);
    return e == hipSuccess ? LJMD_OK : bhip(b, e, "batch_get_state");
}

int ljmd_batch_get_forces(ljmd_batch *b, double *f) {
    if (!b) return LJMD_EINVAL;
    if (!b->have_state) return bfail(b, LJMD_ESTATE, "batch_get_forces before batch_set_state");
    if (!f) return bfail(b, LJMD_EINVAL, "batch_get_forces: NULL array");
    hipError_t e = launch_batch_get_forces(blauncher(b), b->sys, b->g16, b->bg.nslots, f);
    return e == hipSuccess ? LJMD_OK : bhip(b, e, "batch_get_forces");
}

int ljmd_batch_observables(ljmd_batch *b, double *obs_host) {
    if (!b || !obs_host) return LJMD_EINVAL;
    if (!b->have_state) return bfail(b, LJMD_ESTATE, "batch_observables before batch_set_state");
    int r = ljmd_batch_sync_status(b);
    std::vector<Ctl> h(b->nsys);
    hipError_t e = hipMemcpy(h.data(), b->st.ctl, sizeof(Ctl) * b->nsys, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return bhip(b, e, "read observables");
    for (int k = 0; k < b->nsys; ++k)
        for (int q = 0; q < LJMD_NOBS; ++q) obs_host[(size_t)k * LJMD_NOBS + q] = h[k].last[q];
    return r;
}

int ljmd_batch_sync_status(ljmd_batch *b) {
    if (!b) return LJMD_EINVAL;
    hipError_t e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return bhip(b, e, "synchronise");
    std::vector<Ctl> h(b->nsys);
    e = hipMemcpy(h.data(), b->st.ctl, sizeof(Ctl) * b->nsys, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return bhip(b, e, "read flags");
    for (int k = 0; k < b->nsys; ++k) {
        const uint32_t flags = h[k].flags;
        if (flags & kErrNaN) return bfail(b, LJMD_ENAN, "system %d: non-finite position detected", k);
        if (flags & kErrCell) return bfail(b, LJMD_ECELL, "system %d: a cell exceeded cell_capacity=%d", k, b->g.cell_cap);
        if (flags & kErrList)
            return bfail(b, LJMD_ENLIST, "system %d: a neighbour list exceeded nbr_capacity=%d", k, b->g.cap);
    }
    return LJMD_OK;
}

const char *ljmd_batch_last_error(const ljmd_batch *b) { return b ? b->err.c_str() : g_create_err.c_str(); }

}  // extern "C"

