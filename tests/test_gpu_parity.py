"""Parity of the HIP path with the CPU oracle, through the C ABI.

Inputs come from the shared seeded generators; every expected value comes
from the oracle. Tolerances:
  * neighbour sets: identical (FP64 criterion in the FP64 path, the stated
    FP32 sequence in the FP32 path, both evaluated from the same FP64 input);
  * forces: relative error per particle, max_i |dF_i| / s_i <= 1e-12 (FP64),
    <= 1e-5 (FP32+DS), with the scale s_i = max(|F_i|, rms_j |F_j|, 1 eps/sigma):
    relative to the particle's own force, floored at the rms force (for
    forces that nearly cancel) and at the unit force (perfect lattice); a
    particle with a partner at a cutoff tie (|r^2 - r_c^2| within rounding of
    the path's precision, found from the FP64 positions) may additionally
    differ by the force jump |F(r_c)| per such partner, because the truncated
    force is discontinuous there and binary32 decides r^2 < r_c^2;
  * U/N, W/N: relative 1e-12 (FP64), 5e-6 (FP32+DS). The FP32 bound follows
    from the arithmetic: s^12 = u^6 multiplies the relative error of r^2
    (~2e-7 from the binary32 displacement) and of the 1-ulp reciprocal
    (1.2e-7) six times, so a repulsion-dominated energy sum can be off by
    ~2.6e-6 relative;
  * 100-step trajectories (N=2048): max |dx| <= 1e-10 sigma, |dv| <= 1e-9
    (FP64); <= 1e-4 and <= 1e-3 (FP32+DS).
"""
import math

import numpy as np
import pytest

import oracle
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


def tie_allowance(x, sp, box, p, prec):
    """Per-particle sum of |F(r_c)| over partners at a cutoff tie."""
    x = np.asarray(x, dtype=np.float64)
    n = len(x)
    cnt, nbr = oracle.build_lists(x, sp, box, p, mode=0)
    i = np.repeat(np.arange(n), cnt)
    j = nbr[np.arange(nbr.shape[1])[None, :] < cnt[:, None]]
    d = x[i] - x[j]
    d -= box * np.rint(d / box)
    r2 = (d * d).sum(axis=1)
    ab = sp[i] * 2 + sp[j] if p.nspecies == 2 else np.zeros(len(i), dtype=np.int64)
    rc = np.asarray(p.rcut)[ab]
    window = 1e-12 if prec == FP64 else 2e-6
    tie = np.abs(r2 - rc * rc) <= window * rc * rc
    out = np.zeros(n)
    for k in np.nonzero(tie)[0]:
        a = int(ab[k])
        jump = abs(oracle.pair_fscalar(rc[k] * (1 - 1e-15), a, p)) * rc[k]
        out[i[k]] += 1.001 * jump
    return out


def representation_allowance(x, sp, box, p, chunk=250000):
    """Per-particle force error the FP32 path's representation admits:
    sum over partners within the cutoff of sqrt(3) * (L / 2^32) * (|dF/dr| +
    |F| / r) (pair displacement from 32-bit fixed-point coordinates) plus
    3e-6 |F| (binary32 pair arithmetic and per-lane sums). Pair forces from
    the oracle's FP64 lists and the textbook LJ formulas."""
    x = np.asarray(x, dtype=np.float64)
    n = len(x)
    cnt, nbr = oracle.build_lists(x, sp, box, p, mode=0)
    qs = float(np.max(box)) / 2.0 ** 32
    src = [0, 1, 3] if p.nspecies == 2 else [0, 0, 0]
    sig_t = np.array([p.sigma[a] for a in src]); eps_t = np.array([p.eps[a] for a in src])
    rc_t = np.array([p.rcut[a] for a in src])
    out = np.zeros(n)
    for a in range(0, n, chunk):
        b = min(n, a + chunk)
        c = cnt[a:b]
        ii = np.repeat(np.arange(a, b), c)
        jj = nbr[a:b][np.arange(nbr.shape[1])[None, :] < c[:, None]]
        d = x[ii] - x[jj]
        d -= box * np.rint(d / box)
        r = np.sqrt((d * d).sum(axis=1))
        t = (sp[ii] + sp[jj]) if p.nspecies == 2 else np.zeros(len(ii), dtype=np.int64)
        u = sig_t[t] / r
        F = 24.0 * eps_t[t] * (2.0 * u ** 12 - u ** 6) / r
        dF = 24.0 * eps_t[t] * (-26.0 * u ** 12 + 7.0 * u ** 6) / r ** 2
        inside = r < rc_t[t]
        wgt = (math.sqrt(3.0) * qs * (np.abs(dF) + np.abs(F) / r) + 3e-6 * np.abs(F)) * inside
        out[a:b] += np.bincount(ii - a, weights=wgt, minlength=b - a)
    return out


def rel_force_err(f, g, allowance=None):
    rms = math.sqrt(float((g ** 2).sum(axis=1).mean()))
    scale = np.maximum(np.maximum(np.linalg.norm(g, axis=1), rms), 1.0)
    err = np.linalg.norm(f - g, axis=1)
    if allowance is not None:
        err = np.maximum(err - allowance, 0.0)
    return float((err / scale).max())


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


@pytest.mark.parametrize("prec", [FP64, FP32])
@pytest.mark.parametrize("case", CASES, ids=IDS)
def test_forces_energy_virial(ljmd, case, prec):
    name, x, v, sp, box, p = case
    s = make_system(ljmd, x, v, sp, box, p, prec)
    f = s.forces().cpu().numpy()
    o = s.observables()
    fb, Ub, Wb = oracle.forces_brute(x, sp, box, p)
    K, mom = oracle.kinetic(v, sp, p)
    assert rel_force_err(f, fb, tie_allowance(x, sp, box, p, prec)) <= TOL_F[prec], name
    n = len(x)
    assert abs(o["U"] - Ub) / n <= TOL_E[prec] * max(1.0, abs(Ub) / n)
    assert abs(o["W"] - Wb) / n <= TOL_E[prec] * max(1.0, abs(Wb) / n)
    assert o["K"] == pytest.approx(K, rel=1e-12 if prec == FP64 else 1e-6)
    assert o["rebuilds"] == 1 and o["step"] == 0


@pytest.mark.parametrize("lanes", [1, 2, 4, 8, 16])
@pytest.mark.parametrize("prec", [FP64, FP32])
def test_gather_lanes_agree(ljmd, lanes, prec):
    name, x, v, sp, box, p = CASES[4]
    s = make_system(ljmd, x, v, sp, box, p, prec, lanes=lanes)
    f = s.forces().cpu().numpy()
    fb, _, _ = oracle.forces_brute(x, sp, box, p)
    assert rel_force_err(f, fb, tie_allowance(x, sp, box, p, prec)) <= TOL_F[prec]


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


def test_nbr_overflow_is_reported(ljmd):
    w = W.config_small()
    s = ljmd.System(w.n, w.box, w.params, precision=FP64, nbr_capacity=32)
    s.set_state(w.x, w.v, w.species)
    with pytest.raises(ljmd.LJMDError) as e:
        s.sync()
    assert e.value.code == -5


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
    fo, Uo, Wo = oracle.forces(x, w.species, box, w.params)
    allow = tie_allowance(x, w.species, box, w.params, prec)
    assert rel_force_err(f, fo, allow) <= TOL_F[prec]
    # Away from cutoff ties the plain per-particle bound holds.
    clean = allow == 0
    assert rel_force_err(f[clean], fo[clean]) <= TOL_F[prec]
    assert abs(o["U"] - Uo) <= TOL_E[prec] * abs(Uo)
    assert abs(o["W"] - Wo) <= TOL_E[prec] * abs(Wo)
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
    fo, Uo, Wo = oracle.forces(xh, w.species, w.box, w.params)
    # Per-particle bound: 1e-5 of max(|F_i|, rms |F|, 1), plus what the
    # representation allows in a dense, relaxed liquid (net forces far below
    # the pair forces): pair displacements come from 32-bit fixed-point
    # coordinates (an error up to sqrt(3) L 2^-32 per pair) and each pair
    # force from ~10 binary32 operations summed over a few dozen pairs per
    # lane (3e-6 |F_ij|). A particle above it must owe the excess to
    # partners at a cutoff tie (found by brute force for those few only).
    rms = math.sqrt(float((fo ** 2).sum(axis=1).mean()))
    scale = np.maximum(np.maximum(np.linalg.norm(fo, axis=1), rms), 1.0)
    allow = representation_allowance(xh, w.species, w.box, w.params)
    err = np.linalg.norm(f - fo, axis=1)
    over = np.nonzero(err > TOL_F[FP32] * scale + allow)[0]
    assert len(over) <= 100, len(over)
    p = w.params
    for i in over:
        d = xh - xh[i]
        d -= w.box * np.rint(d / w.box)
        r2 = (d * d).sum(axis=1)
        ab = w.species[i] * 2 + w.species
        rc = np.asarray(p.rcut)[ab]
        near = np.nonzero((np.abs(r2 - rc * rc) <= 2e-6 * rc * rc) & (np.arange(len(xh)) != i))[0]
        tie = sum(1.001 * abs(oracle.pair_fscalar(rc[j] * (1 - 1e-15), int(ab[j]), p)) * rc[j] for j in near)
        assert err[i] - tie <= TOL_F[FP32] * scale[i] + allow[i], (i, err[i], tie)
    assert abs(o["U"] - Uo) <= TOL_E[FP32] * abs(Uo)
    assert abs(o["W"] - Wo) <= TOL_E[FP32] * abs(Wo)
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
