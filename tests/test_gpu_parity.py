"""Parity of the HIP path with the CPU oracle, through the C ABI.

Inputs come from the shared seeded generators; every expected value comes
from the oracle. Tolerances:
  * neighbour sets: identical (FP64 criterion in the FP64 path, the stated
    FP32 sequence in the FP32 path, both evaluated from the same FP64 input);
  * forces (metrics in force_metrics.py), after the tie allowance |F(r_c)|
    per partner at a cutoff tie (the truncated force jumps there):
    FP64 against the oracle's FP64 forces, max_i |dF_i| / max(rms_j |F_j|, 1)
    <= 1e-12; FP32+DS against the oracle's FP64 forces of the fixed-point
    positions the path represents, max_i |dF_i| / A_i <= 1e-5 with A_i the
    sum of particle i's pair-force magnitudes inside the cutoff (binary32
    pair arithmetic leaves a few 1e-7 of each pair force; every test prints
    the rms-relative and per-particle errors beside it);
  * U/N, W/N: relative 1e-12 (FP64), 5e-6 (FP32+DS). The FP32 bound follows
    from the arithmetic: s^12 = u^6 multiplies the relative error of r^2
    (~2e-7 from the binary32 displacement) and of the 1-ulp reciprocal
    (1.2e-7) six times, so a repulsion-dominated energy sum can be off by
    ~2.6e-6 relative (each test prints the measured error);
  * 100-step trajectories (N=2048): max |dx| <= 1e-10 sigma, |dv| <= 1e-9
    (FP64); <= 1e-4 and <= 1e-3 (FP32+DS).
"""
import math

import numpy as np
import pytest

import oracle
from force_metrics import bound_key, force_errors, reference, report, tie_allowance
from paper_2406_04210_amd import workloads as W

pytestmark = pytest.mark.gpu

FP64, FP32 = 0, 1
TOL_F = {FP64: 1e-12, FP32: 1e-5}
TOL_E = {FP64: 1e-12, FP32: 5e-6}


@pytest.fixture(scope="module")
def ljmd():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2406_04210_amd import ljmd as L
    return L


def jittered_fcc(m, amp, seed, rho=0.8442):
    x, L = W.fcc_lattice(m, rho)
    rng = np.random.default_rng(seed)
    x = x + amp * rng.standard_normal(x.shape)
    return x, np.full(3, L)


def cases():
    """(name, x, v, species, box, params) small parity cases that span several
    wave chunks, a ragged tail, two cells per axis and the mixture."""
    out = []
    w = W.config_small()
    out.append(("fcc8_lattice_mb", w.x, w.v, w.species, w.box, w.params))
    x, box = jittered_fcc(8, 0.1, 3)
    out.append(("fcc8_jitter", x, w.v, w.species, box, w.params))
    r = W.random_dense(777, 0.8442, seed=5)          # ragged: 777 = 12*64 + 9
    out.append(("random777", r.x, r.v, r.species, r.box, r.params))
    r = W.random_dense(256, 0.8442, seed=6)          # 2 cells per axis
    out.append(("random256_2cells", r.x, r.v, r.species, r.box, r.params))
    r = W.random_dense(1500, 1.1, seed=7, nspecies=2, min_dist=0.75)
    out.append(("mixture1500", r.x, r.v, r.species, r.box, r.params))
    # Two cells per axis holding 80 particles each: the list build takes a
    # cell's home particles in two passes of at most 64.
    r = W.random_dense(640, 1.1, seed=9, min_dist=0.75)
    out.append(("random640_80percell", r.x, r.v, r.species, r.box, r.params))
    # Unequal box edges (the scaled-displacement paths): the jittered 8^3
    # lattice cut to 6 of its 8 cells along z, which keeps it periodic; once
    # with one species and once as an 80:20 mixture.
    x, L = W.fcc_lattice(8, 0.8442)
    a = L / 8.0
    x = x[x[:, 2] < 6.0 * a - 1e-9]
    box = np.array([L, L, 6.0 * a])
    rng = np.random.default_rng(12)
    x = np.ascontiguousarray((x + 0.05 * rng.standard_normal(x.shape)) % box)
    sp1 = np.zeros(len(x), np.int32)
    v = W.maxwell_boltzmann(len(x), 1.0, w.params.mass, sp1, rng)
    out.append(("fcc8x8x6_noncubic", x, v, sp1, box, w.params))
    pm = W.binary_mixture_params()
    sp2 = np.ones(len(x), np.int32)
    sp2[rng.permutation(len(x))[: int(round(0.8 * len(x)))]] = 0
    v2 = W.maxwell_boltzmann(len(x), 1.0, pm.mass, sp2, rng)
    out.append(("fcc8x8x6_noncubic_mixture", x, v2, sp2, box, pm))
    return out


CASES = cases()
IDS = [c[0] for c in CASES]


def make_system(ljmd, x, v, sp, box, p, prec, **kw):
    s = ljmd.System(len(x), box, p, precision=prec, **kw)
    s.set_state(x, v, sp)
    return s


@pytest.mark.parametrize("prec", [FP64, FP32])
@pytest.mark.parametrize("case", CASES, ids=IDS)
def test_neighbor_sets_exact(ljmd, case, prec):
    name, x, v, sp, box, p = case
    s = make_system(ljmd, x, v, sp, box, p, prec)
    cnt, ids = s.neighbors(cap=256)
    s.sync()
    cnt, ids = cnt.cpu().numpy(), ids.cpu().numpy()
    oc, on = oracle.build_lists(x, sp, box, p, mode=0 if prec == FP64 else 1)
    assert np.array_equal(cnt, oc)
    for i in range(len(x)):
        assert set(ids[i, : cnt[i]].tolist()) == set(on[i, : oc[i]].tolist()), (name, i)


HALF_CELL_CASES = [c for c in CASES if c[0] in ("random777", "random256_2cells", "mixture1500",
                                                 "fcc8x8x6_noncubic_mixture")]


@pytest.mark.parametrize("prec", [FP64, FP32])
@pytest.mark.parametrize("case", HALF_CELL_CASES, ids=[c[0] for c in HALF_CELL_CASES])
def test_half_size_cells_lists_and_forces(ljmd, case, prec):
    # Cells of edge >= r_L / 2 and the 125-cell stencil (taken in two parts
    # of at most 64 cells; random256 has 4 cells per axis, fewer than the
    # stencil's 5, so each of its cells is visited once): the same neighbour
    # sets and the same forces as the oracle.
    name, x, v, sp, box, p = case
    s = make_system(ljmd, x, v, sp, box, p, prec, cell_split=2)
    nc = ljmd.cell_grid(s.params)
    print(f"half cells {name}: grid {nc}", flush=True)
    cnt, ids = s.neighbors(cap=256)
    s.sync()
    cnt, ids = cnt.cpu().numpy(), ids.cpu().numpy()
    oc, on = oracle.build_lists(x, sp, box, p, mode=0 if prec == FP64 else 1)
    assert np.array_equal(cnt, oc)
    for i in range(len(x)):
        assert set(ids[i, : cnt[i]].tolist()) == set(on[i, : oc[i]].tolist()), (name, i)
    f = s.forces().cpu().numpy()
    o = s.observables()
    U, Wv = check_forces(f"{name} half cells prec={prec}", f, x, sp, box, p, prec)
    eu, ew = energy_errors(f"{name} half cells prec={prec}", o, U, Wv, len(x))
    assert eu <= TOL_E[prec] and ew <= TOL_E[prec]


@pytest.mark.parametrize("prec", [FP64, FP32])
def test_half_size_cells_trajectory(ljmd, prec):
    # 100 steps with resorts every 25 on the 125-cell stencil: the oracle's
    # trajectory to the same bounds as with full-size cells.
    w = W.config_small()
    s, obs, xu, v = _trajectory(ljmd, w, prec, 100, sort_interval=25, cell_split=2)
    r = oracle.run_nve(w.x, w.v, w.species, w.box, w.params, 100)
    dx = np.abs(xu - r["x"]).max()
    dv = np.abs(v - r["v"]).max()
    tol_x, tol_v = (1e-10, 1e-9) if prec == FP64 else (1e-4, 1e-3)
    assert dx <= tol_x and dv <= tol_v, (dx, dv)


def list_radius_ties(nspecies, seed):
    """Sparse cubic box of partner pairs at the list radius of their pair type
    times (1 + delta), delta from -3e-7 to 3e-7 (a few units of the FP32
    rounding of r^2 in quanta), in random directions. Most cells hold one or
    two particles, so the candidate reduction of the list build bounds the
    distance to a home box that is (nearly) a point: the list must still
    match the oracle pair for pair."""
    p = W.single_species_params() if nspecies == 1 else W.binary_mixture_params()
    L = 20.0
    rng = np.random.default_rng(seed)
    deltas = [-3e-7, -1e-7, -3e-8, 0.0, 3e-8, 1e-7, 3e-7]
    xs, sps = [], []
    for k in range(240):
        si, sj = (int(rng.integers(0, 2)), int(rng.integers(0, 2))) if nspecies == 2 else (0, 0)
        ab = si + sj if nspecies == 2 else 0
        rl = float(p.rcut[[0, 1, 3][ab]] + p.skin)
        u = rng.standard_normal(3)
        if k % 3 == 0:
            u = np.eye(3)[k % 9 // 3] * rng.choice([-1.0, 1.0])  # along an axis
        u /= np.linalg.norm(u)
        c = rng.uniform(0.0, L, 3)
        xs += [c, c + rl * (1.0 + deltas[k % len(deltas)]) * u]
        sps += [si, sj]
    x = np.ascontiguousarray(np.array(xs) % L)
    sp = np.array(sps, np.int32)
    return x, sp, np.full(3, L), p


@pytest.mark.parametrize("prec", [FP64, FP32])
@pytest.mark.parametrize("nspecies", [1, 2])
def test_neighbor_sets_at_list_radius_ties(ljmd, nspecies, prec):
    x, sp, box, p = list_radius_ties(nspecies, 40 + nspecies)
    v = np.zeros_like(x)
    s = make_system(ljmd, x, v, sp, box, p, prec)
    cnt, ids = s.neighbors(cap=256)
    s.sync()
    cnt, ids = cnt.cpu().numpy(), ids.cpu().numpy()
    oc, on = oracle.build_lists(x, sp, box, p, mode=0 if prec == FP64 else 1)
    assert np.array_equal(cnt, oc)
    for i in range(len(x)):
        assert set(ids[i, : cnt[i]].tolist()) == set(on[i, : oc[i]].tolist()), i


def check_forces(tag, f, x, sp, box, p, prec, tol=None):
    ref, U, Wv, A = reference(x, sp, box, p, prec)
    m = report(tag, force_errors(f, ref, A, tie_allowance(x, sp, box, p, prec)))
    assert m[bound_key(prec)] <= (TOL_F[prec] if tol is None else tol), (tag, m)
    return U, Wv


def energy_errors(tag, o, U, Wv, n):
    eu = abs(o["U"] - U) / max(1.0, abs(U))
    ew = abs(o["W"] - Wv) / max(1.0, abs(Wv))
    print(f"energy errors [{tag}]: U rel {eu:.3e} W rel {ew:.3e}", flush=True)
    return eu, ew


@pytest.mark.parametrize("prec", [FP64, FP32])
@pytest.mark.parametrize("case", CASES, ids=IDS)
def test_forces_energy_virial(ljmd, case, prec):
    name, x, v, sp, box, p = case
    s = make_system(ljmd, x, v, sp, box, p, prec)
    f = s.forces().cpu().numpy()
    o = s.observables()
    U, Wv = check_forces(f"{name} prec={prec}", f, x, sp, box, p, prec)
    K, mom = oracle.kinetic(v, sp, p)
    n = len(x)
    eu, ew = energy_errors(f"{name} prec={prec}", o, U, Wv, n)
    assert eu <= TOL_E[prec] and ew <= TOL_E[prec]
    assert o["K"] == pytest.approx(K, rel=1e-12 if prec == FP64 else 1e-6)
    assert o["rebuilds"] == 1 and o["step"] == 0


@pytest.mark.parametrize("lanes", [1, 2, 4, 8, 16])
@pytest.mark.parametrize("prec", [FP64, FP32])
def test_gather_lanes_agree(ljmd, lanes, prec):
    name, x, v, sp, box, p = CASES[4]
    s = make_system(ljmd, x, v, sp, box, p, prec, lanes=lanes)
    f = s.forces().cpu().numpy()
    check_forces(f"{name} lanes={lanes} prec={prec}", f, x, sp, box, p, prec)


def _trajectory(ljmd, w, prec, nsteps, **kw):
    s = make_system(ljmd, w.x, w.v, w.species, w.box, w.params, prec, **kw)
    obs = s.run(nsteps)
    s.sync()
    xu = s.unwrapped_positions().cpu().numpy()
    _, v, _ = s.get_state()
    return s, obs.cpu().numpy(), xu, v.cpu().numpy()


@pytest.mark.parametrize("prec", [FP64, FP32])
def test_trajectory_100_steps(ljmd, prec):
    w = W.config_small()
    s, obs, xu, v = _trajectory(ljmd, w, prec, 100, sort_interval=25)
    r = oracle.run_nve(w.x, w.v, w.species, w.box, w.params, 100)
    dx = np.abs(xu - r["x"]).max()
    dv = np.abs(v - r["v"]).max()
    tol_x, tol_v = (1e-10, 1e-9) if prec == FP64 else (1e-4, 1e-3)
    assert dx <= tol_x and dv <= tol_v, (dx, dv)
    n = w.n
    U, K = obs[:, 0], obs[:, 1]
    ro = r["obs"][1:]
    tol = 1e-10 if prec == FP64 else 1e-5
    assert np.abs(U - ro[:, 0]).max() / n <= tol
    assert np.abs(K - ro[:, 1]).max() / n <= tol
    assert np.array_equal(obs[:, 7], np.arange(1, 101))
    # Momentum stays zero.
    assert np.abs(obs[:, 3:6]).max() < (1e-10 if prec == FP64 else 1e-3)
    o = s.observables()
    assert o["step"] == 100 and o["rebuilds"] == 1 + int(obs[:, 6].sum())


@pytest.mark.parametrize("prec", [FP64, FP32])
def test_trajectory_unequal_masses(ljmd, prec):
    # Species masses 1 and 2 (every other case has unit masses): the half
    # kicks divide by the particle's own mass, K and p are mass-weighted.
    # The lattice-start fluid (the calibrated trajectory case) as two species
    # with the same potential: every other particle has mass 2.
    r0 = W.config_small()
    sp = (np.arange(r0.n) % 2).astype(np.int32)
    p = r0.params.copy()
    p.nspecies = 2
    p.mass = np.array([1.0, 2.0])
    r0.species = sp
    v = W.maxwell_boltzmann(r0.n, 1.0, p.mass, sp, np.random.default_rng(70))
    v = v + np.array([0.05, -0.02, 0.03])          # a non-zero total momentum
    s = make_system(ljmd, r0.x, v, r0.species, r0.box, p, prec, sort_interval=25)
    obs = s.run(100).cpu().numpy()
    s.sync()
    xu = s.unwrapped_positions().cpu().numpy()
    _, vg, _ = s.get_state()
    vg = vg.cpu().numpy()
    r = oracle.run_nve(r0.x, v, r0.species, r0.box, p, 100)
    dx = np.abs(xu - r["x"]).max()
    dv = np.abs(vg - r["v"]).max()
    print(f"unequal masses prec={prec}: max|dx|={dx:.3e} max|dv|={dv:.3e}", flush=True)
    tol_x, tol_v = (1e-10, 1e-9) if prec == FP64 else (1e-4, 1e-3)
    assert dx <= tol_x and dv <= tol_v, (dx, dv)
    ro = r["obs"][1:]
    tol = 1e-10 if prec == FP64 else 1e-5
    assert np.abs(obs[:, 1] - ro[:, 1]).max() / r0.n <= tol          # K = sum m v^2 / 2
    assert np.abs(obs[:, 0] - ro[:, 0]).max() / r0.n <= tol
    P0 = (p.mass[r0.species][:, None] * v).sum(axis=0)
    assert np.abs(obs[:, 3:6] - P0[None, :]).max() <= (1e-10 if prec == FP64 else 1e-4) * np.abs(P0).max()
    assert np.abs(ro[:, 3:6] - P0[None, :]).max() <= 1e-10 * np.abs(P0).max()


@pytest.mark.parametrize("nspecies", [1, 2])
def test_observing_steps_does_not_change_the_trajectory(ljmd, nspecies):
    # Steps whose observables are not reduced skip the energy and virial
    # terms; positions, velocities and forces are bitwise those of a run that
    # observes every step, and the last step's observables agree.
    import torch
    if nspecies == 1:
        w = W.config_small()
    else:
        w = W.config_mixture(n=3000, seed_index=2)
    runs = []
    for observe in (True, False):
        s = make_system(ljmd, w.x, w.v, w.species, w.box, w.params, FP32)
        if nspecies == 2:
            s.minimize_sd(100, 0.05, 0.6, record=False)
            x, _, _ = s.get_state()
            s.set_state(x, torch.as_tensor(w.v, device="cuda"), torch.as_tensor(w.species, device="cuda"))
        s.run(40, observe=observe)
        s.run(25, observe=observe)
        x, v, img = s.get_state()
        f = s.forces()
        o = s.observables()
        s.sync()
        runs.append((x, v, img, f, o))
    a, b = runs
    for k in range(4):
        assert torch.equal(a[k], b[k]), k
    for key in ("U", "K", "W", "step", "rebuilds"):
        assert a[4][key] == b[4][key], key


@pytest.mark.parametrize("prec", [FP64, FP32])
def test_split_runs_and_resort_do_not_change_results(ljmd, prec):
    w = W.config_small()
    s1 = make_system(ljmd, w.x, w.v, w.species, w.box, w.params, prec, sort_interval=0)
    s1.run(60, observe=False)
    x1 = s1.unwrapped_positions().cpu().numpy()
    s2 = make_system(ljmd, w.x, w.v, w.species, w.box, w.params, prec, sort_interval=7)
    for k in (1, 13, 46):
        s2.run(k, observe=False)
    x2 = s2.unwrapped_positions().cpu().numpy()
    s2.sync()
    # Same physics; only summation order may differ after a resort.
    tol = 1e-11 if prec == FP64 else 1e-4
    assert np.abs(x1 - x2).max() <= tol


@pytest.mark.parametrize("prec", [FP64, FP32])
def test_bitwise_reproducible(ljmd, prec):
    w = W.config_small()
    res = []
    for _ in range(2):
        s = make_system(ljmd, w.x, w.v, w.species, w.box, w.params, prec, sort_interval=10)
        obs = s.run(40)
        x, v, img = s.get_state()
        res.append((obs.cpu().numpy(), x.cpu().numpy(), v.cpu().numpy()))
    for a, b in zip(res[0], res[1]):
        assert np.array_equal(a, b)


def test_free_flight_ds_matches_closed_form(ljmd):
    # eps = 0: x_n = x_0 + n dt v exactly; double-single keeps ~48 bits.
    w = W.config_small()
    p = w.params.copy()
    p.eps[:] = 0.0
    s = make_system(ljmd, w.x, w.v, w.species, w.box, p, FP32, sort_interval=0)
    nsteps = 20000
    s.run(nsteps, observe=False)
    xu = s.unwrapped_positions().cpu().numpy()
    s.sync()
    want = w.x + (nsteps * p.dt) * w.v
    err_ds = np.abs(xu - want).max()
    assert err_ds < 1e-9
    # A plain FP32 accumulation of the same walk is far worse (negative control).
    xf = w.x.astype(np.float32)
    step = (np.float32(p.dt) * w.v.astype(np.float32)).astype(np.float32)
    for _ in range(2000):
        xf = (xf + step).astype(np.float32)
    err_f32 = np.abs(xf - (w.x + 2000 * p.dt * w.v)).max()
    assert err_f32 > 100 * err_ds


def test_nbr_overflow_without_room_is_reported(ljmd):
    # An explicit capacity reserves no room to grow: the state load (which
    # waits for its first list build) reports LJMD_ENLIST.
    w = W.config_small()
    s = ljmd.System(w.n, w.box, w.params, precision=FP64, nbr_capacity=32)
    with pytest.raises(ljmd.LJMDError) as e:
        s.set_state(w.x, w.v, w.species)
        s.sync()
    assert e.value.code == -5


@pytest.mark.parametrize("prec", [FP64, FP32])
def test_nbr_overflow_recovered_in_state_load_and_run(ljmd, prec):
    # Capacity 80 holds the lattice's 78 partners but not the liquid's longer
    # lists; with room for 256 the lists grow in place and the overflowing
    # steps are redone. The trajectory is bitwise that of a system that had
    # room from the start (list entries keep their order at any capacity),
    # and matches the oracle. Capacity 32 already overflows at the state load.
    w = W.config_small()
    ref = make_system(ljmd, w.x, w.v, w.species, w.box, w.params, prec, sort_interval=25)
    obs_ref = ref.run(100).cpu().numpy()
    x_ref = ref.unwrapped_positions().cpu().numpy()
    o_ref = ref.observables()
    for cap in (80, 32):
        s = make_system(ljmd, w.x, w.v, w.species, w.box, w.params, prec, sort_interval=25, nbr_capacity=cap,
                        nbr_capacity_max=256)
        obs = s.run(100).cpu().numpy()
        s.sync()
        o = s.observables()
        print(f"overflow recovery prec={prec} cap={cap}: capacity now {o['nbr_capacity']}, "
              f"max fill {o['max_fill']} (room-from-start max fill {o_ref['max_fill']})", flush=True)
        assert o["nbr_capacity"] > cap and o["nbr_capacity"] >= o["max_fill"]
        xu = s.unwrapped_positions().cpu().numpy()
        assert np.array_equal(xu, x_ref)
        # Observables of every step, the redone ones included (the rebuild
        # counter also counts the build that overflowed).
        assert np.array_equal(obs[:, [0, 1, 2, 3, 4, 5, 7]], obs_ref[:, [0, 1, 2, 3, 4, 5, 7]])
    r = oracle.run_nve(w.x, w.v, w.species, w.box, w.params, 100)
    tol_x = 1e-10 if prec == FP64 else 1e-4
    assert np.abs(xu - r["x"]).max() <= tol_x


@pytest.mark.parametrize("prec", [FP64, FP32])
def test_nbr_overflow_recovered_in_rollout_and_sweep(ljmd, prec):
    # The differentiable rollout (forward) and its reverse sweep with lists
    # that overflow: the forward run is repeated from its first stored state
    # with longer lists, the sweep checks before writing its outputs; the
    # gradient equals bitwise that of a system with room from the start.
    w = W.config_small()
    rng = np.random.default_rng(5)
    lam_x, lam_v = rng.standard_normal(w.x.shape), rng.standard_normal(w.x.shape)
    out = []
    for cap, room in ((0, 0), (80, 256)):
        s = make_system(ljmd, w.x, w.v, w.species, w.box, w.params, prec, nbr_capacity=cap, nbr_capacity_max=room)
        s.vv_forward(60, 10)
        g = s.vv_backward(lam_x, lam_v)
        s.sync()
        out.append([t.cpu().numpy() for t in g] + [s.observables()["nbr_capacity"]])
    assert out[1][3] > 80
    for a, b in zip(out[0][:3], out[1][:3]):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("prec", [FP64, FP32])
def test_nonfinite_velocity_is_reported(ljmd, prec):
    # A NaN velocity gives a NaN position at the next drift, which has no
    # fixed-point image: the run reports LJMD_ENAN at the next synchronising
    # call instead of going on with a wrapped coordinate.
    w = W.config_small()
    v = w.v.copy()
    v[17, 1] = np.nan
    s = make_system(ljmd, w.x, v, w.species, w.box, w.params, prec)
    with pytest.raises(ljmd.LJMDError) as e:
        s.run(3)
        s.sync()
    assert e.value.code == -6


def test_run_before_state_is_rejected(ljmd):
    w = W.config_small()
    s = ljmd.System(w.n, w.box, w.params, precision=FP64)
    with pytest.raises(ljmd.LJMDError) as e:
        s.run(1)
    assert e.value.code == -7


@pytest.mark.parametrize("prec", [FP64, FP32])
def test_full_size_forces_and_sampled_lists(ljmd, prec):
    # The headline workload at full size: N = 256,000 (FCC 40^3, rho 0.8442),
    # jittered so that forces are non-trivial.
    w = W.config_headline()
    x, box = jittered_fcc(40, 0.08, 17)
    s = make_system(ljmd, x, w.v, w.species, box, w.params, prec)
    f = s.forces().cpu().numpy()
    o = s.observables()
    Uo, Wo = check_forces(f"headline n=256000 prec={prec}", f, x, w.species, box, w.params, prec)
    eu, ew = energy_errors(f"headline n=256000 prec={prec}", o, Uo, Wo, len(x))
    assert eu <= TOL_E[prec] and ew <= TOL_E[prec]
    cnt, ids = s.neighbors(cap=256)
    cnt, ids = cnt.cpu().numpy(), ids.cpu().numpy()
    oc, on = oracle.build_lists(x, w.species, box, w.params, mode=0 if prec == FP64 else 1)
    assert np.array_equal(cnt, oc)
    rng = np.random.default_rng(1)
    for i in rng.choice(len(x), 2000, replace=False):
        assert set(ids[i, : cnt[i]].tolist()) == set(on[i, : oc[i]].tolist())


def test_full_size_mixture_after_relaxation(ljmd):
    # The binary-mixture workload at full size (N = 4,000,000, rho = 1.2) in
    # the bench's configuration: 200 steepest-descent steps, then the forces
    # and lists of the relaxed state (two-species quanta kernels; the list
    # build takes cells from per-XCD queues at this size).
    import torch
    w = W.config_mixture()
    s = make_system(ljmd, w.x, w.v, w.species, w.box, w.params, FP32)
    s.minimize_sd(200, 0.05, 0.6, record=False)
    x, _, _ = s.get_state()
    s.set_state(x, torch.as_tensor(w.v, device="cuda"), torch.as_tensor(w.species, device="cuda"))
    f = s.forces().cpu().numpy()
    o = s.observables()
    cnt, ids = s.neighbors(cap=160)
    cnt, ids = cnt.cpu().numpy(), ids.cpu().numpy()
    s.sync()
    del s
    xh = x.cpu().numpy()
    # Reference: the oracle's FP64 forces of the fixed-point positions the
    # FP32 path holds. In this dense relaxed liquid (rho = 1.2 after steepest
    # descent) the net forces are ~1/50 of the pair forces that form them, so
    # the FP32 bound (1e-5 of the particle's pair-force magnitude sum) and the
    # rms-relative error differ most here; both are printed.
    ref, Uo, Wo, A = reference(xh, w.species, w.box, w.params, FP32)
    m = report("mixture n=4000000 relaxed", force_errors(f, ref, A, tie_allowance(xh, w.species, w.box,
                                                                                   w.params, FP32)))
    assert m[bound_key(FP32)] <= TOL_F[FP32], m
    eu, ew = energy_errors("mixture n=4000000 relaxed", o, Uo, Wo, len(xh))
    assert eu <= TOL_E[FP32] and ew <= TOL_E[FP32]
    oc, on = oracle.build_lists(xh, w.species, w.box, w.params, mode=1, cap=160)
    assert np.array_equal(cnt, oc)
    rng = np.random.default_rng(2)
    for i in rng.choice(len(xh), 2000, replace=False):
        assert set(ids[i, : cnt[i]].tolist()) == set(on[i, : oc[i]].tolist())


def test_fp32_energy_conservation_tracks_fp64(ljmd):
    w = W.config_small()
    drifts = {}
    for prec in (FP64, FP32):
        s = make_system(ljmd, w.x, w.v, w.species, w.box, w.params, prec)
        obs = s.run(1000).cpu().numpy()
        E = (obs[:, 0] + obs[:, 1]) / w.n
        late = E[200:]
        drifts[prec] = (np.polyfit(np.arange(len(late)) * w.params.dt, late, 1)[0],
                        np.abs(E - E.mean()).max())
    slope64, fl64 = drifts[FP64]
    slope32, fl32 = drifts[FP32]
    assert abs(slope32) < 5e-5 and abs(slope64) < 5e-5
    assert fl32 < 1.5 * fl64 + 1e-5


@pytest.mark.parametrize("prec", [FP64, FP32])
def test_steepest_descent_matches_oracle(ljmd, prec):
    # Uniform random binary mixture (overlapping pairs): the relaxation path.
    w = W.config_mixture(n=1500, seed_index=2)
    nsteps = 30
    s = make_system(ljmd, w.x, w.v, w.species, w.box, w.params, prec)
    fm = s.minimize_sd(nsteps, 0.01, 0.6).cpu().numpy()
    xu = s.unwrapped_positions().cpu().numpy()
    f = s.forces().cpu().numpy()
    s.sync()
    r = oracle.minimize_sd(w.x, w.species, w.box, w.params, nsteps, delta=0.01, clamp=0.6)
    tol_f, tol_x = (1e-10, 1e-9) if prec == FP64 else (1e-5, 1e-4)
    assert np.abs(fm - r["fmax"][:nsteps]).max() <= tol_f * r["fmax"][0]
    assert np.abs(xu - r["x"]).max() <= tol_x
    # After relaxation the context holds the unclamped forces of the new state.
    fo, _, _ = oracle.forces(r["x"], w.species, w.box, w.params)
    rms = np.sqrt((fo ** 2).sum(axis=1).mean())
    assert np.abs(f - fo).max() <= (1e-9 if prec == FP64 else 1e-3) * max(rms, np.abs(fo).max())
