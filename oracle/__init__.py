"""CPU oracle for the truncated Lennard-Jones MD hot path (ctypes binding).

TEST INFRASTRUCTURE ONLY: the test suite, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` are the only users. The GPU library never
imports, links or calls anything here, and this package imports nothing from
the GPU package.

The arithmetic lives in ``oracle.c`` (plain FP64 C, OpenMP over particles);
this module only marshals numpy arrays. Functions and the passages of the
paper they follow:

* ``phi``, ``fscalar``, ``pair_energy``, ``pair_fscalar`` -- the 12-6
  Lennard-Jones pair potential, truncated and energy-shifted (Sec. 3 "Code
  structure": truncation of the interaction range; Sec. 4: the common
  Lennard-Jones potential).
* ``forces_brute`` -- the O(N^2) all-pairs sum with the cutoff applied
  (Sec. 4: the all-to-all interaction the port started from).
* ``build_lists`` -- Verlet neighbour lists from particle binning (Sec. 3).
* ``forces_list``, ``kinetic`` -- forces, energy, virial, kinetic energy and
  momentum from the lists.
* ``run_nve`` -- velocity-Verlet time stepping with the list rebuilt when
  particles have moved far enough (Sec. 3 signals integrate/force/finalize;
  Sec. 5: list updates become more frequent as particles move faster),
  optionally with the stochastic Andersen-like ("Boltzmann") thermostat the
  paper combines with velocity Verlet (Sec. 4).
* ``forces_fixed`` -- FP64 forces of the positions the single-precision path
  represents (32-bit fixed-point image coordinates from the stated FP32
  sequence); what remains against that path is its binary32 arithmetic.
* ``philox4x32``, ``thermo_draw`` -- the counter-based generator (Salmon et
  al., SC'11) and the thermostat's per-particle draws.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import time

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "oracle.c")

CFLAGS = ["-O3", "-march=x86-64-v3", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
          "-fPIC", "-shared", "-std=c11", "-Wall"]


def build(verbose: bool = False) -> str:
    """Compile oracle.c into liboracle.so (gcc)."""
    tmp = _LIB_PATH + f".tmp{os.getpid()}"
    cmd = ["gcc", *CFLAGS, _SRC, "-o", tmp, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class OThermo(C.Structure):
    _fields_ = [("temperature", C.c_double), ("rate", C.c_double), ("seed", C.c_uint64),
                ("dim", C.c_int32), ("pad", C.c_int32)]


class OLJ(C.Structure):
    _fields_ = [("nspecies", C.c_int32), ("shift_energy", C.c_int32),
                ("eps", C.c_double * 4), ("sigma", C.c_double * 4), ("rcut", C.c_double * 4),
                ("mass", C.c_double * 2), ("skin", C.c_double), ("dt", C.c_double)]


def make_params(p) -> OLJ:
    """Build the C parameter struct from an object with the LJParams fields."""
    s = OLJ()
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
    return s


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = C.CDLL(_LIB_PATH)
        dp, ip, up = C.POINTER(C.c_double), C.POINTER(C.c_int32), C.POINTER(C.c_uint32)
        fp = C.POINTER(C.c_float)
        pp = C.POINTER(OLJ)
        L.oracle_phi.restype = C.c_double
        L.oracle_phi.argtypes = [C.c_double, C.c_double, C.c_double]
        L.oracle_fscalar.restype = C.c_double
        L.oracle_fscalar.argtypes = [C.c_double, C.c_double, C.c_double]
        L.oracle_pair_energy.restype = C.c_double
        L.oracle_pair_energy.argtypes = [C.c_double, C.c_int, pp]
        L.oracle_pair_fscalar.restype = C.c_double
        L.oracle_pair_fscalar.argtypes = [C.c_double, C.c_int, pp]
        L.oracle_forces_brute.restype = None
        L.oracle_forces_brute.argtypes = [C.c_int64, dp, ip, dp, pp, dp, dp]
        L.oracle_build_lists.restype = C.c_int32
        L.oracle_build_lists.argtypes = [C.c_int64, dp, ip, dp, pp, C.c_int32, C.c_int32, ip, ip]
        L.oracle_forces_list.restype = None
        L.oracle_forces_list.argtypes = [C.c_int64, dp, ip, dp, pp, C.c_int32, ip, ip, dp, dp]
        L.oracle_kinetic.restype = None
        L.oracle_kinetic.argtypes = [C.c_int64, dp, ip, pp, dp]
        L.oracle_run_nve.restype = C.c_int64
        L.oracle_run_nve.argtypes = [C.c_int64, dp, dp, ip, dp, pp, C.c_int64, dp, dp,
                                     C.POINTER(OThermo), C.POINTER(C.c_uint64), dp]
        L.oracle_forces_fixed.restype = None
        L.oracle_forces_fixed.argtypes = [C.c_int64, dp, ip, dp, pp, C.c_int32, ip, ip, dp, dp, dp]
        L.oracle_philox4x32.restype = None
        L.oracle_philox4x32.argtypes = [up, up, up]
        L.oracle_thermo_threshold.restype = C.c_uint32
        L.oracle_thermo_threshold.argtypes = [C.c_double, C.c_double]
        L.oracle_thermo_draw.restype = C.c_int32
        L.oracle_thermo_draw.argtypes = [C.c_uint64, C.c_int64, C.c_int64, C.c_uint32, dp]
        L.oracle_set_threads.restype = None
        L.oracle_set_threads.argtypes = [C.c_int32]
        L.oracle_ds_split.restype = None
        L.oracle_ds_split.argtypes = [C.c_double, fp, fp]
        L.oracle_q_from_ds.restype = C.c_uint32
        L.oracle_q_from_ds.argtypes = [C.c_float, C.c_float, C.c_double]
        L.oracle_disp_q.restype = C.c_float
        L.oracle_disp_q.argtypes = [C.c_uint32, C.c_uint32, C.c_double]
        L.oracle_minimize_sd.restype = C.c_int64
        L.oracle_minimize_sd.argtypes = [C.c_int64, dp, ip, dp, pp, C.c_int64, C.c_double,
                                         C.c_double, dp, dp]
        L.oracle_force_vjp.restype = C.c_int32
        L.oracle_force_vjp.argtypes = [C.c_int64, dp, ip, dp, pp, dp, dp, dp]
        L.oracle_energy_grad.restype = C.c_int32
        L.oracle_energy_grad.argtypes = [C.c_int64, dp, ip, dp, pp, dp]
        L.oracle_vv_adjoint.restype = C.c_int32
        L.oracle_vv_adjoint.argtypes = [C.c_int64, dp, dp, ip, dp, pp, C.c_int64, dp, dp, dp]
        L.oracle_num_threads.restype = C.c_int32
        L.oracle_num_threads.argtypes = []
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _i(a):
    return a.ctypes.data_as(C.POINTER(C.c_int32))


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def phi(r, eps=1.0, sigma=1.0):
    return lib().oracle_phi(float(r), float(eps), float(sigma))


def fscalar(r, eps=1.0, sigma=1.0):
    return lib().oracle_fscalar(float(r), float(eps), float(sigma))


def pair_energy(r, ab, params):
    s = make_params(params)
    return lib().oracle_pair_energy(float(r), int(ab), C.byref(s))


def pair_fscalar(r, ab, params):
    s = make_params(params)
    return lib().oracle_pair_fscalar(float(r), int(ab), C.byref(s))


def forces_brute(x, species, box, params):
    """All-pairs forces. Returns (F (N,3), U, W)."""
    x = _f64(x, (-1, 3))
    n = x.shape[0]
    sp, bx = _i32(species), _f64(box)
    f = np.zeros((n, 3))
    out = np.zeros(2)
    s = make_params(params)
    lib().oracle_forces_brute(n, _d(x), _i(sp), _d(bx), C.byref(s), _d(f), _d(out))
    return f, float(out[0]), float(out[1])


def build_lists(x, species, box, params, mode: int = 0, cap: int = 160):
    """Full Verlet lists. mode 0: FP64 criterion, 1: the FP32 sequence.
    Returns (cnt (N,), nbr (N, cap)); grows cap until every list fits."""
    x = _f64(x, (-1, 3))
    n = x.shape[0]
    sp, bx = _i32(species), _f64(box)
    s = make_params(params)
    while True:
        cnt = np.zeros(n, dtype=np.int32)
        nbr = np.full((n, cap), -1, dtype=np.int32)
        mx = lib().oracle_build_lists(n, _d(x), _i(sp), _d(bx), C.byref(s), int(mode), int(cap),
                                      _i(cnt), _i(nbr))
        if mx <= cap:
            return cnt, nbr
        cap = int(mx) + 16


def neighbor_sets(cnt, nbr):
    return [frozenset(nbr[i, : cnt[i]].tolist()) for i in range(len(cnt))]


def forces_list(x, species, box, params, cnt, nbr):
    x = _f64(x, (-1, 3))
    n = x.shape[0]
    sp, bx = _i32(species), _f64(box)
    nbr = np.ascontiguousarray(nbr, dtype=np.int32)
    cnt = _i32(cnt)
    f = np.zeros((n, 3))
    out = np.zeros(2)
    s = make_params(params)
    lib().oracle_forces_list(n, _d(x), _i(sp), _d(bx), C.byref(s), nbr.shape[1], _i(cnt), _i(nbr),
                             _d(f), _d(out))
    return f, float(out[0]), float(out[1])


def forces(x, species, box, params):
    """Forces via lists (any N). Returns (F, U, W)."""
    cnt, nbr = build_lists(x, species, box, params, 0)
    return forces_list(x, species, box, params, cnt, nbr)


def kinetic(v, species, params):
    v = _f64(v, (-1, 3))
    sp = _i32(species)
    out = np.zeros(4)
    s = make_params(params)
    lib().oracle_kinetic(v.shape[0], _d(v), _i(sp), C.byref(s), _d(out))
    return float(out[0]), out[1:].copy()


def run_nve(x, v, species, box, params, nsteps: int, want_obs: bool = True, thermostat=None,
            want_sig: bool = False):
    """Velocity-Verlet NVE (or, with ``thermostat=(T, rate, seed)``, with the
    Andersen-like thermostat; in a two-dimensional system (params.dim == 2,
    z = 0) the resampled v_z is 0). Returns dict with x, v (unwrapped, final),
    f (final forces), obs ((nsteps+1, 6): U, K, W, px, py, pz), builds,
    seconds (wall time of the whole call), loop_seconds (wall time of the
    step loop alone, after the initial list build and forces), sig
    ((nsteps+1,) uint64 signatures of the pairs inside the cutoff, or None)."""
    x = _f64(x, (-1, 3)).copy()
    v = _f64(v, (-1, 3)).copy()
    n = x.shape[0]
    sp, bx = _i32(species), _f64(box)
    obs = np.zeros((nsteps + 1, 6)) if want_obs else None
    sig = np.zeros(nsteps + 1, dtype=np.uint64) if want_sig else None
    f = np.zeros((n, 3))
    s = make_params(params)
    th = None
    if thermostat is not None:
        dim = int(thermostat[3]) if len(thermostat) > 3 else int(getattr(params, "dim", 3))
        th = OThermo(float(thermostat[0]), float(thermostat[1]), int(thermostat[2]), dim, 0)
    loop = C.c_double(0.0)
    t0 = time.perf_counter()
    builds = lib().oracle_run_nve(n, _d(x), _d(v), _i(sp), _d(bx), C.byref(s), int(nsteps),
                                  _d(obs) if obs is not None else None, _d(f),
                                  C.byref(th) if th is not None else None,
                                  sig.ctypes.data_as(C.POINTER(C.c_uint64)) if sig is not None else None,
                                  C.byref(loop))
    dt = time.perf_counter() - t0
    if builds < 0:
        raise MemoryError("oracle_run_nve: allocation failed")
    return {"x": x, "v": v, "f": f, "obs": obs, "builds": int(builds), "seconds": dt,
            "loop_seconds": loop.value, "sig": sig}


def forces_fixed(x, species, box, params, cnt=None, nbr=None):
    """FP64 forces of the positions the FP32 path represents (fixed-point
    displacements). Returns (F, U, W, fabs) with fabs (N,) the per-particle
    sum of pair-force magnitudes inside the cutoff."""
    x = _f64(x, (-1, 3))
    n = x.shape[0]
    sp, bx = _i32(species), _f64(box)
    if cnt is None:
        cnt, nbr = build_lists(x, species, box, params, 0)
    nbr = np.ascontiguousarray(nbr, dtype=np.int32)
    cnt = _i32(cnt)
    f = np.zeros((n, 3))
    fa = np.zeros(n)
    out = np.zeros(2)
    s = make_params(params)
    lib().oracle_forces_fixed(n, _d(x), _i(sp), _d(bx), C.byref(s), nbr.shape[1], _i(cnt), _i(nbr),
                              _d(f), _d(out), _d(fa))
    return f, float(out[0]), float(out[1]), fa


def philox4x32(ctr, key):
    """Philox4x32-10 block for a 4-word counter and 2-word key."""
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    o = np.zeros(4, dtype=np.uint32)
    up = C.POINTER(C.c_uint32)
    lib().oracle_philox4x32(c.ctypes.data_as(up), k.ctypes.data_as(up), o.ctypes.data_as(up))
    return o


def thermo_threshold(rate: float, dt: float) -> int:
    return int(lib().oracle_thermo_threshold(float(rate), float(dt)))


def thermo_draw(seed: int, pid: int, step: int, threshold: int):
    """(collides, z (3,)) of particle pid at step for the thermostat."""
    z = np.zeros(3)
    hit = lib().oracle_thermo_draw(int(seed), int(pid), int(step), int(threshold), _d(z))
    return bool(hit), z


def set_threads(n: int):
    """Threads of the oracle's OpenMP loops from now on."""
    lib().oracle_set_threads(int(n))


def minimize_sd(x, species, box, params, nsteps: int, delta: float = 0.01, clamp: float = 0.6):
    """Steepest descent with capped step and clamped pair distance.
    Returns dict x (relaxed, unwrapped), U ((nsteps+1,) clamped energies),
    fmax ((nsteps+1,)), builds."""
    x = _f64(x, (-1, 3)).copy()
    sp, bx = _i32(species), _f64(box)
    u = np.zeros(nsteps + 1)
    fm = np.zeros(nsteps + 1)
    s = make_params(params)
    b = lib().oracle_minimize_sd(x.shape[0], _d(x), _i(sp), _d(bx), C.byref(s), int(nsteps),
                                 float(delta), float(clamp), _d(u), _d(fm))
    if b < 0:
        raise MemoryError("oracle_minimize_sd: allocation failed")
    return {"x": x, "U": u, "fmax": fm, "builds": int(b)}


def force_vjp(x, species, box, params, g):
    """(dF/dx)^T g and the parameter gradient of g.F per symmetric pair type.
    Returns (gx (N,3), geps (3,), gsig (3,)) with types [AA, AB, BB]."""
    x = _f64(x, (-1, 3))
    g = _f64(g, (-1, 3))
    sp, bx = _i32(species), _f64(box)
    gx = np.zeros_like(x)
    gt = np.zeros(6)
    s = make_params(params)
    if lib().oracle_force_vjp(x.shape[0], _d(x), _i(sp), _d(bx), C.byref(s), _d(g), _d(gx), _d(gt)):
        raise MemoryError("oracle_force_vjp")
    return gx, gt[:3].copy(), gt[3:].copy()


def energy_grad(x, species, box, params):
    """dU/d(eps_t), dU/d(sigma_t) per symmetric pair type [AA, AB, BB]."""
    x = _f64(x, (-1, 3))
    sp, bx = _i32(species), _f64(box)
    gt = np.zeros(6)
    s = make_params(params)
    if lib().oracle_energy_grad(x.shape[0], _d(x), _i(sp), _d(bx), C.byref(s), _d(gt)):
        raise MemoryError("oracle_energy_grad")
    return gt[:3].copy(), gt[3:].copy()


def vv_adjoint(x0, v0, species, box, params, nsteps, lam_x, lam_v):
    """Adjoint of nsteps velocity-Verlet steps from (x0, v0): given dL/dx_N and
    dL/dv_N returns (dL/dx_0, dL/dv_0, geps (3,), gsig (3,)) of the dynamics."""
    x0 = _f64(x0, (-1, 3))
    v0 = _f64(v0, (-1, 3))
    lx = _f64(lam_x, (-1, 3)).copy()
    lv = _f64(lam_v, (-1, 3)).copy()
    sp, bx = _i32(species), _f64(box)
    gt = np.zeros(6)
    s = make_params(params)
    if lib().oracle_vv_adjoint(x0.shape[0], _d(x0), _d(v0), _i(sp), _d(bx), C.byref(s),
                               int(nsteps), _d(lx), _d(lv), _d(gt)):
        raise MemoryError("oracle_vv_adjoint")
    return lx, lv, gt[:3].copy(), gt[3:].copy()


def with_params(params, eps=None, sigma=None):
    """Copy of params with per-type (AA, AB, BB) eps/sigma replaced; cutoffs
    stay the same absolute lengths."""
    q = params.copy()
    for name, vals in (("eps", eps), ("sigma", sigma)):
        if vals is None:
            continue
        arr = getattr(q, name)
        vals = np.atleast_1d(np.asarray(vals, dtype=np.float64))
        if q.nspecies == 1:
            arr[:] = vals[0]
        else:
            arr[0], arr[1], arr[2], arr[3] = vals[0], vals[1], vals[1], vals[2]
    return q


def ds_split(w: float):
    hi, lo = C.c_float(), C.c_float()
    lib().oracle_ds_split(float(w), C.byref(hi), C.byref(lo))
    return np.float32(hi.value), np.float32(lo.value)


def q_from_ds(hi, lo, L):
    return int(lib().oracle_q_from_ds(float(hi), float(lo), float(L)))


def disp_q(qi, qj, L):
    return np.float32(lib().oracle_disp_q(int(qi) & 0xFFFFFFFF, int(qj) & 0xFFFFFFFF, float(L)))


def num_threads() -> int:
    return int(lib().oracle_num_threads())
