"""ctypes binding of libljmd.so, the gfx950 truncated-LJ MD library.

Argument marshalling only: every step of the method runs in the library's
HIP kernels. PyTorch supplies device memory (the workspace and the I/O
tensors) and the stream. There is no CPU fallback: importing this module
raises if the library is missing, and creating a ``System`` raises if no
GPU is present.

Function names mirror include/ljmd.h.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libljmd.so")

ABI_VERSION = 8
FP64 = 0
FP32_DS = 1
FP32 = 2
ADJ_STORE_ALL = 1
NOBS = 8
OBS_FIELDS = ("U", "K", "W", "px", "py", "pz", "rebuilt", "step")

STATUS = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EHIP", -4: "EBOX", -5: "ENLIST",
          -6: "ENAN", -7: "ESTATE", -8: "ECELL"}


class LJMDError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"ljmd {STATUS.get(code, code)} ({code}): {msg}")
        self.code = code


class Params(C.Structure):
    _fields_ = [("n", C.c_int64), ("box", C.c_double * 3), ("nspecies", C.c_int32),
                ("shift_energy", C.c_int32), ("eps", C.c_double * 4), ("sigma", C.c_double * 4),
                ("rcut", C.c_double * 4), ("mass", C.c_double * 2), ("skin", C.c_double),
                ("dt", C.c_double), ("sort_interval", C.c_int32), ("precision", C.c_int32),
                ("nbr_capacity", C.c_int32), ("cell_capacity", C.c_int32), ("lanes", C.c_int32),
                ("cell_split", C.c_int32), ("dim", C.c_int32), ("pad", C.c_int32)]


class Obs(C.Structure):
    _fields_ = [("U", C.c_double), ("K", C.c_double), ("W", C.c_double), ("P", C.c_double),
                ("T", C.c_double), ("E", C.c_double), ("p", C.c_double * 3),
                ("step", C.c_int64), ("rebuilds", C.c_int64), ("max_fill", C.c_int32),
                ("nbr_capacity", C.c_int32)]


class SystemDesc(C.Structure):
    _fields_ = [("n", C.c_int64), ("box", C.c_double)]


class Tuning(C.Structure):
    _fields_ = [("lanes", C.c_int32), ("nbr_capacity", C.c_int32), ("cell_capacity", C.c_int32),
                ("max_fill", C.c_int32), ("ms_per_step", C.c_double), ("from_cache", C.c_int32),
                ("cell_split", C.c_int32)]


# Every exported function: name -> (restype, argtypes).
_vp, _dp, _ip = C.c_void_p, C.c_void_p, C.c_void_p
SIGNATURES = {
    "ljmd_abi_version": (C.c_int32, []),
    "ljmd_check_params": (C.c_int, [C.POINTER(Params)]),
    "ljmd_workspace_size": (C.c_size_t, [C.POINTER(Params)]),
    "ljmd_cell_grid": (C.c_int, [C.POINTER(Params), C.POINTER(C.c_int32)]),
    "ljmd_hilbert_ranks": (C.c_int, [C.c_int32, C.c_int32, C.c_int32, C.POINTER(C.c_int32)]),
    "ljmd_create": (C.c_int, [C.POINTER(Params), _vp, C.c_size_t, _vp, C.POINTER(_vp)]),
    "ljmd_destroy": (C.c_int, [_vp]),
    "ljmd_set_state": (C.c_int, [_vp, _dp, _dp, _ip]),
    "ljmd_get_state": (C.c_int, [_vp, _dp, _dp, _ip]),
    "ljmd_get_forces": (C.c_int, [_vp, _dp]),
    "ljmd_run": (C.c_int, [_vp, C.c_int64, _dp]),
    "ljmd_neighbors": (C.c_int, [_vp, _ip, _ip, C.c_int32]),
    "ljmd_minimize_sd": (C.c_int, [_vp, C.c_int32, C.c_double, C.c_double, _dp]),
    "ljmd_sync_status": (C.c_int, [_vp]),
    "ljmd_observables": (C.c_int, [_vp, C.POINTER(Obs)]),
    "ljmd_set_thermostat": (C.c_int, [_vp, C.c_double, C.c_double, C.c_uint64]),
    "ljmd_set_profiling": (C.c_int, [_vp, C.c_int]),
    "ljmd_kernel_times": (C.c_int, [_vp, C.POINTER(C.c_double), C.POINTER(C.c_int64)]),
    "ljmd_last_error": (C.c_char_p, [_vp]),
    "ljmd_set_pair_params": (C.c_int, [_vp, C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "ljmd_force_vjp": (C.c_int, [_vp, _dp, _dp, _dp]),
    "ljmd_energy_grad": (C.c_int, [_vp, _dp]),
    "ljmd_adjoint_workspace_size": (C.c_size_t, [C.POINTER(Params), C.c_int32, C.c_int32, C.c_int32]),
    "ljmd_vv_forward": (C.c_int, [_vp, C.c_int32, C.c_int32, C.c_int32, _vp, C.c_size_t, _dp]),
    "ljmd_vv_backward": (C.c_int, [_vp, _dp, _dp, _dp, _dp, _dp, _dp]),
    "ljmd_batch_workspace_size": (C.c_size_t, [C.POINTER(Params), C.POINTER(SystemDesc), C.c_int32]),
    "ljmd_batch_create": (C.c_int, [C.POINTER(Params), C.POINTER(SystemDesc), C.c_int32, _vp, C.c_size_t, _vp,
                                    C.POINTER(_vp)]),
    "ljmd_batch_destroy": (C.c_int, [_vp]),
    "ljmd_batch_set_state": (C.c_int, [_vp, _dp, _dp, _ip]),
    "ljmd_batch_run": (C.c_int, [_vp, C.c_int64, _dp]),
    "ljmd_batch_use_graphs": (C.c_int, [_vp, C.c_int32]),
    "ljmd_batch_get_state": (C.c_int, [_vp, _dp, _dp, _ip]),
    "ljmd_batch_get_forces": (C.c_int, [_vp, _dp]),
    "ljmd_batch_observables": (C.c_int, [_vp, C.POINTER(C.c_double)]),
    "ljmd_batch_sync_status": (C.c_int, [_vp]),
    "ljmd_batch_last_error": (C.c_char_p, [_vp]),
    "ljmd_batch_max_fill": (C.c_int, [_vp, C.POINTER(C.c_int32)]),
    "ljmd_batch_autotune_workspace_size": (C.c_size_t, [C.POINTER(Params), C.POINTER(SystemDesc), C.c_int32]),
    "ljmd_batch_autotune": (C.c_int, [C.POINTER(Params), C.POINTER(SystemDesc), C.c_int32, _dp, _dp, _ip, _vp,
                                      C.c_size_t, _vp, C.c_int32, C.c_char_p, C.POINTER(Tuning)]),
    "ljmd_brute_workspace_size": (C.c_size_t, [C.POINTER(Params)]),
    "ljmd_brute_forces": (C.c_int, [C.POINTER(Params), _dp, _ip, _dp, _dp, _vp, C.c_size_t, _vp]),
    "ljmd_brute_static_scratch_bytes": (C.c_size_t, []),
    "ljmd_brute_forces_noalloc": (C.c_int, [C.POINTER(Params), _dp, _ip, _dp, _dp, _vp]),
    "ljmd_autotune_workspace_size": (C.c_size_t, [C.POINTER(Params)]),
    "ljmd_autotune": (C.c_int, [C.POINTER(Params), _dp, _dp, _ip, _vp, C.c_size_t, _vp, C.c_int32, C.c_char_p,
                                C.POINTER(Tuning)]),
}
NKT = 5
KERNEL_FAMILIES = ("step", "rebuild", "resort", "other", "adjoint")
# Parameter-gradient layout of the library: (eps_AA, eps_AB, eps_BB,
# sigma_AA, sigma_AB, sigma_BB); entries 1, 2, 4, 5 are unused with one species.
THETA_FIELDS = ("eps_AA", "eps_AB", "eps_BB", "sigma_AA", "sigma_AB", "sigma_BB")


def _load():
    # torch must be loaded first: libljmd.so then binds to the HIP runtime
    # torch already mapped (same soname), so the process holds exactly one
    # HIP/HSA runtime and torch's device pointers and streams are ours too.
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -c 'import __graft_entry__ as g; g.build()'` "
                          "(there is no CPU fallback)")
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


lib = _load()


def last_error(ctx=None) -> str:
    s = lib.ljmd_last_error(ctx)
    return s.decode() if s else ""


def _check(code: int, ctx=None):
    if code != 0:
        raise LJMDError(code, last_error(ctx))


def make_params(n: int, box, p, precision: int = FP32_DS, sort_interval: int = 100,
                nbr_capacity: int = 0, cell_capacity: int = 0, lanes: int = 0, cell_split: int = 0) -> Params:
    """Build the C parameter struct from an LJParams-like object ``p``."""
    s = Params()
    s.n = int(n)
    for k in range(3):
        s.box[k] = float(box[k])
    s.nspecies = int(p.nspecies)
    s.shift_energy = int(p.shift_energy)
    for k in range(4):
        s.eps[k] = float(p.eps[k])
        s.sigma[k] = float(p.sigma[k])
        s.rcut[k] = float(p.rcut[k])
    for k in range(2):
        s.mass[k] = float(p.mass[k])
    s.skin = float(p.skin)
    s.dt = float(p.dt)
    s.sort_interval = int(sort_interval)
    s.precision = int(precision)
    s.nbr_capacity = int(nbr_capacity)
    s.cell_capacity = int(cell_capacity)
    s.lanes = int(lanes)
    s.cell_split = int(cell_split)
    s.dim = int(getattr(p, "dim", 3))
    s.pad = 0
    return s


def check_params(params: Params) -> int:
    return int(lib.ljmd_check_params(C.byref(params)))


def workspace_size(params: Params) -> int:
    return int(lib.ljmd_workspace_size(C.byref(params)))


def cell_grid(params: Params):
    out = (C.c_int32 * 3)()
    _check(lib.ljmd_cell_grid(C.byref(params), out))
    return tuple(out)


def hilbert_ranks(nx: int, ny: int, nz: int) -> np.ndarray:
    out = np.zeros(nx * ny * nz, dtype=np.int32)
    _check(lib.ljmd_hilbert_ranks(nx, ny, nz, out.ctypes.data_as(C.POINTER(C.c_int32))))
    return out


def _ptr(t) -> int:
    return t.data_ptr()


class System:
    """One simulation box on the current GPU.

    ``p`` is an LJParams-like object; ``precision`` is FP64 or FP32_DS. The
    workspace is a torch uint8 tensor owned by this object; work is enqueued
    on torch's current stream.
    """

    def __init__(self, n: int, box, p, precision: int = FP32_DS, sort_interval: int = 100,
                 nbr_capacity: int = 0, cell_capacity: int = 0, lanes: int = 0, device=None,
                 nbr_capacity_max: int = 0, cell_split: int = 0):
        """nbr_capacity_max > nbr_capacity gives the workspace room for lists of
        that many entries: a list overflow then grows the lists in place and
        redoes the steps (ljmd_run), instead of reporting LJMD_ENLIST."""
        import torch
        self.torch = torch
        if not torch.cuda.is_available():
            raise RuntimeError("ljmd.System needs a HIP GPU; none is visible")
        self.device = torch.device(device if device is not None else "cuda")
        self.params = make_params(n, box, p, precision, sort_interval, nbr_capacity,
                                  cell_capacity, lanes, cell_split)
        self.n = int(n)
        self.box = np.asarray(box, dtype=np.float64)
        _check(check_params(self.params))
        size = workspace_size(self.params)
        if nbr_capacity_max > 0:
            room = make_params(n, box, p, precision, sort_interval, nbr_capacity_max, cell_capacity, lanes,
                               cell_split)
            size = max(size, workspace_size(room))
        self.workspace = torch.empty(size, dtype=torch.uint8, device=self.device)
        self.stream = torch.cuda.current_stream(self.device)
        ctx = C.c_void_p()
        code = lib.ljmd_create(C.byref(self.params), C.c_void_p(_ptr(self.workspace)), size,
                               C.c_void_p(self.stream.cuda_stream), C.byref(ctx))
        if code != 0:
            raise LJMDError(code, last_error(None))
        self.ctx = ctx
        self._gen = 0

    def close(self):
        if getattr(self, "ctx", None):
            lib.ljmd_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _dev(self, a, dtype):
        t = self.torch
        if isinstance(a, np.ndarray):
            a = t.from_numpy(np.ascontiguousarray(a))
        return a.to(device=self.device, dtype=dtype).contiguous()

    def set_state(self, x, v, species):
        t = self.torch
        x = self._dev(x, t.float64).reshape(self.n, 3)
        v = self._dev(v, t.float64).reshape(self.n, 3)
        s = self._dev(species, t.int32).reshape(self.n)
        _check(lib.ljmd_set_state(self.ctx, _ptr(x), _ptr(v), _ptr(s)), self.ctx)
        self._keep = (x, v, s)
        self._gen += 1

    def gen(self) -> int:
        """Counter of calls that changed the state or the potential."""
        return self._gen

    def run(self, nsteps: int, observe: bool = True):
        """Advance nsteps; returns a (nsteps, 8) float64 device tensor of
        per-step observables (U, K, W, px, py, pz, rebuilt, step) or None."""
        t = self.torch
        obs = t.empty((max(nsteps, 1), NOBS), dtype=t.float64, device=self.device) if observe else None
        self._gen += 1
        _check(lib.ljmd_run(self.ctx, int(nsteps), _ptr(obs) if obs is not None else None), self.ctx)
        return obs[:nsteps] if obs is not None else None

    def minimize_sd(self, nsteps: int, max_disp: float = 0.01, clamp: float = 0.6,
                    record: bool = True):
        """Steepest-descent relaxation; returns the (nsteps,) device tensor of
        max |F| at the start of every iteration (or None)."""
        t = self.torch
        fm = t.zeros(max(nsteps, 1), dtype=t.float64, device=self.device) if record else None
        self._gen += 1
        _check(lib.ljmd_minimize_sd(self.ctx, int(nsteps), float(max_disp), float(clamp),
                                    _ptr(fm) if fm is not None else None), self.ctx)
        return fm[:nsteps] if fm is not None else None

    def get_state(self):
        t = self.torch
        x = t.empty((self.n, 3), dtype=t.float64, device=self.device)
        v = t.empty_like(x)
        img = t.empty((self.n, 3), dtype=t.int32, device=self.device)
        _check(lib.ljmd_get_state(self.ctx, _ptr(x), _ptr(v), _ptr(img)), self.ctx)
        return x, v, img

    def unwrapped_positions(self):
        x, _, img = self.get_state()
        return x + img.to(x.dtype) * self.torch.as_tensor(self.box, device=self.device)

    def forces(self):
        t = self.torch
        f = t.empty((self.n, 3), dtype=t.float64, device=self.device)
        _check(lib.ljmd_get_forces(self.ctx, _ptr(f)), self.ctx)
        return f

    def neighbors(self, cap: int = 256):
        t = self.torch
        cnt = t.empty(self.n, dtype=t.int32, device=self.device)
        ids = t.full((self.n, cap), -1, dtype=t.int32, device=self.device)
        _check(lib.ljmd_neighbors(self.ctx, _ptr(cnt), _ptr(ids), int(cap)), self.ctx)
        return cnt, ids

    def sync(self):
        _check(lib.ljmd_sync_status(self.ctx), self.ctx)

    def set_thermostat(self, temperature: float, rate: float, seed: int = 0):
        """Andersen-like velocity resampling at `temperature` with collision
        rate `rate` per unit time (0 switches it off)."""
        _check(lib.ljmd_set_thermostat(self.ctx, float(temperature), float(rate), int(seed)), self.ctx)
        self._gen += 1

    def set_profiling(self, enable: bool):
        _check(lib.ljmd_set_profiling(self.ctx, int(bool(enable))), self.ctx)

    def kernel_times(self) -> dict:
        """{family: (total ms, launches)} accumulated since set_profiling(True)."""
        ms = (C.c_double * NKT)()
        cnt = (C.c_int64 * NKT)()
        _check(lib.ljmd_kernel_times(self.ctx, ms, cnt), self.ctx)
        return {KERNEL_FAMILIES[k]: (ms[k], cnt[k]) for k in range(NKT)}

    def observables(self) -> dict:
        o = Obs()
        _check(lib.ljmd_observables(self.ctx, C.byref(o)), self.ctx)
        return {"U": o.U, "K": o.K, "W": o.W, "P": o.P, "T": o.T, "E": o.E,
                "p": (o.p[0], o.p[1], o.p[2]), "step": o.step, "rebuilds": o.rebuilds,
                "max_fill": o.max_fill, "nbr_capacity": o.nbr_capacity}

    # ---- gradients -----------------------------------------------------------

    def theta(self) -> np.ndarray:
        """Current (eps_AA, eps_AB, eps_BB, sigma_AA, sigma_AB, sigma_BB)."""
        e, s = self.params.eps, self.params.sigma
        return np.array([e[0], e[1], e[3], s[0], s[1], s[3]], dtype=np.float64)

    def set_pair_params(self, eps, sigma):
        """Replace eps and sigma (4 entries each, [AA, AB, BA, BB]); the
        forces of a loaded state are re-evaluated."""
        e = (C.c_double * 4)(*[float(v) for v in eps])
        s = (C.c_double * 4)(*[float(v) for v in sigma])
        _check(lib.ljmd_set_pair_params(self.ctx, e, s), self.ctx)
        for k in range(4):
            self.params.eps[k] = e[k]
            self.params.sigma[k] = s[k]
        self._gen += 1

    def set_theta(self, theta):
        """set_pair_params from the 6-entry gradient layout (one species: only
        entries 0 and 3 are used)."""
        t = [float(v) for v in theta]
        if self.params.nspecies == 1:
            eps, sig = [t[0]] * 4, [t[3]] * 4
        else:
            eps, sig = [t[0], t[1], t[1], t[2]], [t[3], t[4], t[4], t[5]]
        self.set_pair_params(eps, sig)

    def force_vjp(self, g):
        """(dF/dx)^T g by id and d(g.F)/dtheta at the current state."""
        t = self.torch
        g = self._dev(g, t.float64).reshape(self.n, 3)
        gx = t.empty((self.n, 3), dtype=t.float64, device=self.device)
        gth = t.empty(6, dtype=t.float64, device=self.device)
        _check(lib.ljmd_force_vjp(self.ctx, _ptr(g), _ptr(gx), _ptr(gth)), self.ctx)
        self._keep_g = g
        return gx, gth

    def energy_grad(self):
        """dU/dtheta at the current state (dU/dx = -forces())."""
        t = self.torch
        gth = t.empty(6, dtype=t.float64, device=self.device)
        _check(lib.ljmd_energy_grad(self.ctx, _ptr(gth)), self.ctx)
        return gth

    def adjoint_workspace_size(self, nsteps: int, every: int, store_all: bool = False) -> int:
        return int(lib.ljmd_adjoint_workspace_size(C.byref(self.params), int(nsteps), int(every),
                                                   ADJ_STORE_ALL if store_all else 0))

    def vv_forward(self, nsteps: int, every: int = 10, observe: bool = True,
                   store_all: bool = False):
        """Differentiable rollout of nsteps with a stored state every `every`
        steps (and every frame kept if store_all); returns the (nsteps, 8)
        observables (or None)."""
        t = self.torch
        flags = ADJ_STORE_ALL if store_all else 0
        size = self.adjoint_workspace_size(nsteps, every, store_all)
        if size == 0:
            raise LJMDError(-1, "vv_forward: invalid nsteps/every")
        ws = getattr(self, "_adj_ws", None)
        if ws is None or ws.numel() < size:
            ws = t.empty(size, dtype=t.uint8, device=self.device)
            self._adj_ws = ws
        obs = t.empty((nsteps, NOBS), dtype=t.float64, device=self.device) if observe else None
        self._gen += 1
        _check(lib.ljmd_vv_forward(self.ctx, int(nsteps), int(every), flags, C.c_void_p(_ptr(ws)),
                                   ws.numel(), _ptr(obs) if obs is not None else None), self.ctx)
        return obs

    def vv_backward(self, lam_x, lam_v, gU=None):
        """(dL/dx_0, dL/dv_0, dL/dtheta) of the last rollout from dL/dx_N and
        dL/dv_N (by id) and, if given, the weight gU = dL/dU_N of the final
        potential energy in the loss (a device scalar tensor or a float)."""
        t = self.torch
        lx = self._dev(lam_x, t.float64).reshape(self.n, 3)
        lv = self._dev(lam_v, t.float64).reshape(self.n, 3)
        gu = None
        if gU is not None:
            gu = (gU.detach() if isinstance(gU, t.Tensor) else t.tensor(float(gU)))
            gu = gu.to(device=self.device, dtype=t.float64).reshape(1).contiguous()
        gx0 = t.empty((self.n, 3), dtype=t.float64, device=self.device)
        gv0 = t.empty_like(gx0)
        gth = t.empty(6, dtype=t.float64, device=self.device)
        _check(lib.ljmd_vv_backward(self.ctx, _ptr(lx), _ptr(lv), _ptr(gu) if gu is not None else None,
                                    _ptr(gx0), _ptr(gv0), _ptr(gth)), self.ctx)
        self._keep_l = (lx, lv, gu)
        return gx0, gv0, gth


def autotune(n: int, box, p, x, v, species, precision: int = FP32_DS, steps: int = 20,
             cache_path: str | None = None, sort_interval: int = 100) -> dict:
    """Time every cell size (cell_split 1, 2) and force-gather shape (lanes)
    on this state and return the fastest pair with a list capacity sized
    from the longest list seen; a cached result (same device, precision,
    species count, size and density) is returned without timing."""
    import torch
    params = make_params(n, box, p, precision, sort_interval)
    _check(check_params(params))
    size = int(lib.ljmd_autotune_workspace_size(C.byref(params)))
    ws = torch.empty(size, dtype=torch.uint8, device="cuda")
    dev = lambda a, dt: (torch.from_numpy(np.ascontiguousarray(a)) if isinstance(a, np.ndarray) else a).to(
        device="cuda", dtype=dt).contiguous()
    xs, vs, sp = dev(x, torch.float64), dev(v, torch.float64), dev(species, torch.int32)
    out = Tuning()
    stream = torch.cuda.current_stream()
    code = lib.ljmd_autotune(C.byref(params), _ptr(xs), _ptr(vs), _ptr(sp), C.c_void_p(_ptr(ws)), size,
                             C.c_void_p(stream.cuda_stream), int(steps),
                             cache_path.encode() if cache_path else None, C.byref(out))
    _check(code)
    return {"lanes": out.lanes, "cell_split": out.cell_split, "nbr_capacity": out.nbr_capacity,
            "cell_capacity": out.cell_capacity, "max_fill": out.max_fill, "ms_per_step": out.ms_per_step,
            "from_cache": bool(out.from_cache)}


def autotune_batch(sizes, edges, p, x, v, species, steps: int = 20, cache_path: str | None = None,
                   sort_interval: int = 100) -> dict:
    """ljmd_batch_autotune: time every cell size and force-gather shape on the whole batch
    (systems of the given sizes and cubic box edges, state concatenated as
    for Batch.set_state) and return the fastest with a list capacity sized
    from the longest list of any system; cached like autotune()."""
    import torch
    sizes = np.asarray(sizes, dtype=np.int64)
    edges = np.asarray(edges, dtype=np.float64)
    params = make_params(int(sizes[0]), [edges[0]] * 3, p, FP32_DS, sort_interval)
    desc = (SystemDesc * len(sizes))(*[SystemDesc(int(n), float(L)) for n, L in zip(sizes, edges)])
    size = int(lib.ljmd_batch_autotune_workspace_size(C.byref(params), desc, len(sizes)))
    if size == 0:
        raise LJMDError(-1, "invalid batch (see ljmd_check_params for each system)")
    ws = torch.empty(size, dtype=torch.uint8, device="cuda")
    dev = lambda a, dt: (torch.from_numpy(np.ascontiguousarray(a)) if isinstance(a, np.ndarray) else a).to(
        device="cuda", dtype=dt).contiguous()
    xs, vs, sp = dev(x, torch.float64), dev(v, torch.float64), dev(species, torch.int32)
    out = Tuning()
    stream = torch.cuda.current_stream()
    code = lib.ljmd_batch_autotune(C.byref(params), desc, len(sizes), _ptr(xs), _ptr(vs), _ptr(sp),
                                   C.c_void_p(_ptr(ws)), size, C.c_void_p(stream.cuda_stream), int(steps),
                                   cache_path.encode() if cache_path else None, C.byref(out))
    if code != 0:
        raise LJMDError(code, lib.ljmd_batch_last_error(None).decode())
    return {"lanes": out.lanes, "cell_split": out.cell_split, "nbr_capacity": out.nbr_capacity,
            "cell_capacity": out.cell_capacity, "max_fill": out.max_fill, "ms_per_step": out.ms_per_step,
            "from_cache": bool(out.from_cache)}


def brute_forces(n: int, box, p, x, species, precision: int = FP64):
    """ljmd_brute_forces: forces (n, 3), U and W of one configuration by the
    sum over all pairs (device tensors; the scratch is a torch tensor)."""
    import torch
    params = make_params(n, box, p, precision, 0)
    size = int(lib.ljmd_brute_workspace_size(C.byref(params)))
    if size == 0:
        _check(check_params(params))
        raise LJMDError(-1, "invalid parameters")
    dev = lambda a, dt: (torch.from_numpy(np.ascontiguousarray(a)) if isinstance(a, np.ndarray) else a).to(
        device="cuda", dtype=dt).contiguous()
    xs, sp = dev(x, torch.float64).reshape(n, 3), dev(species, torch.int32).reshape(n)
    ws = torch.empty(size, dtype=torch.uint8, device="cuda")
    f = torch.empty((n, 3), dtype=torch.float64, device="cuda")
    uw = torch.empty(2, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()
    code = lib.ljmd_brute_forces(C.byref(params), _ptr(xs), _ptr(sp), _ptr(f), _ptr(uw), C.c_void_p(_ptr(ws)), size,
                                 C.c_void_p(stream.cuda_stream))
    if code != 0:
        raise LJMDError(code, last_error(None))
    return f, uw


def brute_forces_noalloc(n: int, box, p, x, species, precision: int = FP64):
    """ljmd_brute_forces_noalloc: as brute_forces, with the library's fixed
    per-GPU scratch instead of a workspace (the call allocates nothing on the
    device; only the outputs here are torch tensors)."""
    import torch
    params = make_params(n, box, p, precision, 0)
    dev = lambda a, dt: (torch.from_numpy(np.ascontiguousarray(a)) if isinstance(a, np.ndarray) else a).to(
        device="cuda", dtype=dt).contiguous()
    xs, sp = dev(x, torch.float64).reshape(n, 3), dev(species, torch.int32).reshape(n)
    f = torch.empty((n, 3), dtype=torch.float64, device="cuda")
    uw = torch.empty(2, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()
    code = lib.ljmd_brute_forces_noalloc(C.byref(params), _ptr(xs), _ptr(sp), _ptr(f), _ptr(uw),
                                         C.c_void_p(stream.cuda_stream))
    if code != 0:
        raise LJMDError(code, last_error(None))
    return f, uw


class Batch:
    """Independent one-species systems in cubic boxes, stepped together.

    ``sizes`` and ``edges`` give each system's particle count and box edge;
    ``p`` (an LJParams-like object) the shared potential and integration
    settings. State arrays are the systems' rows concatenated in order.
    """

    def __init__(self, sizes, edges, p, sort_interval: int = 100, nbr_capacity: int = 0,
                 cell_capacity: int = 0, lanes: int = 0, device=None, cell_split: int = 0):
        import torch
        self.torch = torch
        if not torch.cuda.is_available():
            raise RuntimeError("ljmd.Batch needs a HIP GPU; none is visible")
        self.device = torch.device(device if device is not None else "cuda")
        self.sizes = np.asarray(sizes, dtype=np.int64)
        self.edges = np.asarray(edges, dtype=np.float64)
        if self.sizes.shape != self.edges.shape or self.sizes.ndim != 1:
            raise ValueError("sizes and edges must be equal-length 1-D sequences")
        self.nsys = len(self.sizes)
        self.ntot = int(self.sizes.sum())
        self.offsets = np.concatenate([[0], np.cumsum(self.sizes)])
        self.params = make_params(int(self.sizes[0]), [self.edges[0]] * 3, p, FP32_DS, sort_interval,
                                  nbr_capacity, cell_capacity, lanes, cell_split)
        self.desc = (SystemDesc * self.nsys)(*[SystemDesc(int(n), float(L))
                                               for n, L in zip(self.sizes, self.edges)])
        size = int(lib.ljmd_batch_workspace_size(C.byref(self.params), self.desc, self.nsys))
        if size == 0:
            raise LJMDError(-1, "invalid batch (see ljmd_check_params for each system)")
        self.workspace = torch.empty(size, dtype=torch.uint8, device=self.device)
        self.stream = torch.cuda.current_stream(self.device)
        b = C.c_void_p()
        code = lib.ljmd_batch_create(C.byref(self.params), self.desc, self.nsys,
                                     C.c_void_p(_ptr(self.workspace)), size,
                                     C.c_void_p(self.stream.cuda_stream), C.byref(b))
        if code != 0:
            raise LJMDError(code, lib.ljmd_batch_last_error(None).decode())
        self.b = b

    def _err(self, code):
        if code != 0:
            raise LJMDError(code, lib.ljmd_batch_last_error(self.b).decode())

    def close(self):
        if getattr(self, "b", None):
            lib.ljmd_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _dev(self, a, dtype):
        t = self.torch
        if isinstance(a, np.ndarray):
            a = t.from_numpy(np.ascontiguousarray(a))
        return a.to(device=self.device, dtype=dtype).contiguous()

    def set_state(self, x, v, species):
        t = self.torch
        x = self._dev(x, t.float64).reshape(self.ntot, 3)
        v = self._dev(v, t.float64).reshape(self.ntot, 3)
        s = self._dev(species, t.int32).reshape(self.ntot)
        self._err(lib.ljmd_batch_set_state(self.b, _ptr(x), _ptr(v), _ptr(s)))
        self._keep = (x, v, s)

    def use_graphs(self, enable: bool):
        """Replay whole resort periods of run() from captured HIP graphs
        (default) or launch every step."""
        self._err(lib.ljmd_batch_use_graphs(self.b, 1 if enable else 0))

    def run(self, nsteps: int, observe: bool = False):
        """Advance every system; returns the (nsys, 8) device tensor of each
        system's last-step observables when observe is set."""
        t = self.torch
        obs = t.empty((self.nsys, NOBS), dtype=t.float64, device=self.device) if observe else None
        self._err(lib.ljmd_batch_run(self.b, int(nsteps), _ptr(obs) if obs is not None else None))
        return obs

    def get_state(self):
        t = self.torch
        x = t.empty((self.ntot, 3), dtype=t.float64, device=self.device)
        v = t.empty_like(x)
        img = t.empty((self.ntot, 3), dtype=t.int32, device=self.device)
        self._err(lib.ljmd_batch_get_state(self.b, _ptr(x), _ptr(v), _ptr(img)))
        return x, v, img

    def forces(self):
        t = self.torch
        f = t.empty((self.ntot, 3), dtype=t.float64, device=self.device)
        self._err(lib.ljmd_batch_get_forces(self.b, _ptr(f)))
        return f

    def observables(self) -> np.ndarray:
        out = np.zeros((self.nsys, NOBS), dtype=np.float64)
        self._err(lib.ljmd_batch_observables(self.b, out.ctypes.data_as(C.POINTER(C.c_double))))
        return out

    def sync(self):
        self._err(lib.ljmd_batch_sync_status(self.b))

    def max_fill(self) -> int:
        """Longest neighbour list of any system as built last (synchronises)."""
        out = C.c_int32(0)
        self._err(lib.ljmd_batch_max_fill(self.b, C.byref(out)))
        return int(out.value)


# ---- torch.autograd front ends ----------------------------------------------
# theta is a float64 tensor of 6 entries in THETA_FIELDS order. The System's
# state is overwritten by every call (the functions load x and theta first).

def _autograd():
    import torch

    class LJForceFn(torch.autograd.Function):
        """F(x; theta) by id for a System; backward is the library's force VJP."""

        @staticmethod
        def forward(ctx, x, theta, system, species):
            system.set_theta(theta.detach().cpu().numpy())
            x = x.detach()
            system.set_state(x, torch.zeros_like(x), species)
            ctx.system, ctx.species = system, species
            ctx.gen = system.gen()
            ctx.save_for_backward(x, theta)
            return system.forces()

        @staticmethod
        def backward(ctx, gF):
            x, theta = ctx.saved_tensors
            s = ctx.system
            if s.gen() != ctx.gen:
                # The System was used since: load x and theta again.
                s.set_theta(theta.detach().cpu().numpy())
                s.set_state(x, torch.zeros_like(x), ctx.species)
            gx, gth = s.force_vjp(gF.contiguous())
            return gx, gth.to(theta.device), None, None

    class VVRollout(torch.autograd.Function):
        """(x_N unwrapped, v_N, U_N) after nsteps velocity-Verlet steps from
        (x0, v0) under theta; backward recomputes from checkpoints."""

        @staticmethod
        def forward(ctx, x0, v0, theta, system, species, nsteps, every):
            system.set_theta(theta.detach().cpu().numpy())
            system.set_state(x0.detach(), v0.detach(), species)
            obs = system.vv_forward(nsteps, every)
            xN = system.unwrapped_positions()
            _, vN, _ = system.get_state()
            ctx.system, ctx.species, ctx.nsteps, ctx.every = system, species, nsteps, every
            ctx.gen = system.gen()
            ctx.save_for_backward(x0, v0, theta)
            return xN, vN, obs[-1, 0].clone()

        @staticmethod
        def backward(ctx, gxN, gvN, gU):
            x0, v0, theta = ctx.saved_tensors
            s = ctx.system
            if s.gen() != ctx.gen:
                # The System was used since: repeat the (deterministic) forward.
                s.set_theta(theta.detach().cpu().numpy())
                s.set_state(x0.detach(), v0.detach(), ctx.species)
                s.vv_forward(ctx.nsteps, ctx.every, observe=False)
            lam_x = gxN.contiguous() if gxN is not None else torch.zeros((s.n, 3), dtype=torch.float64,
                                                                         device=s.device)
            lam_v = gvN.contiguous() if gvN is not None else torch.zeros_like(lam_x)
            # The final-energy term (dU/dx_N = -F(x_N), dU/dtheta at x_N) is
            # applied by the library from gU.
            gx0, gv0, gth = s.vv_backward(lam_x, lam_v, gU)
            return gx0, gv0, gth.to(theta.device), None, None, None, None

    return LJForceFn, VVRollout


LJForceFn, VVRollout = _autograd()
