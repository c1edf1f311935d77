"""The two-dimensional variant (ljmd_params.dim = 2; the dimension template
of the paper's modules, Sec. 3) through the C ABI, against the oracle on
the same planar configurations: neighbour sets exact, forces, energy and
virial within the tolerances of test_gpu_parity.py, a 100-step trajectory,
the 2D temperature and pressure, the thermostat (v_z stays 0, draws equal
to the oracle's), and z inputs ignored.

Cases: a jittered triangular lattice in its rectangular periodic cell (the
general displacement path) and a jittered square lattice in a square box
(the fixed-point fast path of square boxes)."""
import numpy as np
import pytest

import oracle
from force_metrics import bound_key, force_errors, reference, report, tie_allowance
from paper_2406_04210_amd import workloads as W

pytestmark = pytest.mark.gpu
FP64, FP32_DS, FP32 = 0, 1, 2
TOL_F = {FP64: 1e-12, FP32_DS: 1e-5, FP32: 1e-5}
TOL_E = {FP64: 1e-12, FP32_DS: 5e-6, FP32: 5e-6}


@pytest.fixture(scope="module")
def ljmd():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2406_04210_amd import ljmd as L
    return L


def square_fluid(m=40, rho=0.7, seed=21):
    rng = np.random.default_rng(seed)
    a = 1.0 / np.sqrt(rho)
    g = np.stack(np.meshgrid(np.arange(m), np.arange(m), indexing="ij"), axis=-1).reshape(-1, 2) * a
    x = np.zeros((m * m, 3))
    x[:, :2] = (g + 0.05 * rng.standard_normal(g.shape)) % (m * a)
    L = np.full(3, m * a)
    p = W.single_species_params()
    p.dim = 2
    sp = np.zeros(len(x), np.int32)
    v = W.maxwell_boltzmann_2d(len(x), 1.0, p.mass, sp, rng)
    return "square1600", x, v, sp, L, p


def tri_fluid():
    w = W.lj_fluid_2d(m=24, rho=0.7)              # 1152 particles, ragged tail
    return "tri1152", w.x, w.v, w.species, w.box, w.params


CASES = [tri_fluid(), square_fluid()]
IDS = [c[0] for c in CASES]


def fp32_ref(prec):
    return FP64 if prec == FP64 else 1


@pytest.mark.parametrize("prec", [FP64, FP32_DS, FP32])
@pytest.mark.parametrize("case", CASES, ids=IDS)
def test_lists_forces_energy_in_the_plane(ljmd, case, prec):
    name, x, v, sp, box, p = case
    s = ljmd.System(len(x), box, p, precision=prec)
    assert ljmd.cell_grid(s.params)[2] == 1
    s.set_state(x, v, sp)
    if prec == FP32:
        # The plain single-precision state holds float positions and
        # velocities: the oracle takes the values the path holds.
        xg, vg, _ = s.get_state()
        x, v = xg.cpu().numpy(), vg.cpu().numpy()
    cnt, ids = s.neighbors(cap=256)
    s.sync()
    cnt, ids = cnt.cpu().numpy(), ids.cpu().numpy()
    oc, on = oracle.build_lists(x, sp, box, p, mode=0 if prec == FP64 else 1)
    assert np.array_equal(cnt, oc)
    for i in range(len(x)):
        assert set(ids[i, : cnt[i]].tolist()) == set(on[i, : oc[i]].tolist()), (name, i)
    f = s.forces().cpu().numpy()
    assert np.all(f[:, 2] == 0.0)
    r = fp32_ref(prec)
    ref, U, Wv, A = reference(x, sp, box, p, r)
    m = report(f"2d {name} prec={prec}", force_errors(f, ref, A, tie_allowance(x, sp, box, p, r)))
    assert m[bound_key(r)] <= TOL_F[prec], m
    o = s.observables()
    n = len(x)
    assert abs(o["U"] - U) / abs(U) <= TOL_E[prec] and abs(o["W"] - Wv) / max(1.0, abs(Wv)) <= TOL_E[prec]
    K, _ = oracle.kinetic(v, sp, p)
    area = box[0] * box[1]
    T = 2.0 * K / (2 * n - 2)
    assert o["T"] == pytest.approx(T, rel=1e-12 if prec == FP64 else 1e-6)
    assert o["P"] == pytest.approx(n / area * T + Wv / (2.0 * area), rel=1e-10 if prec == FP64 else 1e-5)


@pytest.mark.parametrize("prec", [FP64, FP32_DS])
@pytest.mark.parametrize("case", CASES, ids=IDS)
def test_trajectory_in_the_plane(ljmd, case, prec):
    name, x, v, sp, box, p = case
    s = ljmd.System(len(x), box, p, precision=prec, sort_interval=25)
    s.set_state(x, v, sp)
    obs = s.run(100)
    s.sync()
    xu = s.unwrapped_positions().cpu().numpy()
    _, vg, _ = s.get_state()
    vg = vg.cpu().numpy()
    assert np.all(xu[:, 2] == 0.0) and np.all(vg[:, 2] == 0.0)
    r = oracle.run_nve(x, v, sp, box, p, 100)
    dx = np.abs(xu - r["x"]).max()
    dv = np.abs(vg - r["v"]).max()
    tol_x, tol_v = (1e-10, 1e-9) if prec == FP64 else (1e-4, 1e-3)
    print(f"2d trajectory {name} prec={prec}: dx {dx:.3e} dv {dv:.3e}", flush=True)
    assert dx <= tol_x and dv <= tol_v, (dx, dv)
    o = obs.cpu().numpy()
    tol = 1e-10 if prec == FP64 else 1e-5
    assert np.abs(o[:, 0] - r["obs"][1:, 0]).max() / len(x) <= tol


@pytest.mark.parametrize("prec", [FP64, FP32_DS])
def test_thermostat_in_the_plane(ljmd, prec):
    name, x, v, sp, box, p = CASES[0]
    s = ljmd.System(len(x), box, p, precision=prec)
    s.set_state(x, v, sp)
    s.set_thermostat(1.4, 4.0, seed=77)
    s.run(50, observe=False)
    s.sync()
    xu = s.unwrapped_positions().cpu().numpy()
    _, vg, _ = s.get_state()
    vg = vg.cpu().numpy()
    assert np.all(vg[:, 2] == 0.0) and np.all(xu[:, 2] == 0.0)
    r = oracle.run_nve(x, v, sp, box, p, 50, thermostat=(1.4, 4.0, 77))
    tol_x, tol_v = (1e-10, 1e-9) if prec == FP64 else (1e-4, 1e-3)
    assert np.abs(xu - r["x"]).max() <= tol_x and np.abs(vg - r["v"]).max() <= tol_v


def test_z_inputs_are_ignored(ljmd):
    name, x, v, sp, box, p = CASES[1]
    xz, vz = x.copy(), v.copy()
    xz[:, 2] = 3.7
    vz[:, 2] = -0.9
    s = ljmd.System(len(x), box, p, precision=FP64)
    s.set_state(xz, vz, sp)
    f = s.forces().cpu().numpy()
    xg, vg, _ = s.get_state()
    assert np.all(xg.cpu().numpy()[:, 2] == 0.0) and np.all(vg.cpu().numpy()[:, 2] == 0.0)
    ref, _, _ = oracle.forces(x, sp, box, p)
    assert np.abs(f - ref).max() <= 1e-12 * max(1.0, float(np.sqrt((ref ** 2).sum(1).mean())))


def test_gradient_calls_and_batches_are_three_dimensional(ljmd):
    name, x, v, sp, box, p = CASES[1]
    s = ljmd.System(len(x), box, p, precision=FP64)
    s.set_state(x, v, sp)
    with pytest.raises(ljmd.LJMDError):
        s.energy_grad()
    with pytest.raises(ljmd.LJMDError):
        s.vv_forward(5, 5)
    with pytest.raises(Exception):
        ljmd.Batch([len(x)], [box[0]], p)


def test_brute_forces_in_the_plane(ljmd):
    # The one-shot brute force with dim = 2 also takes z as 0.
    name, x, v, sp, box, p = CASES[1]
    xz = x.copy()
    xz[:, 2] = 1.25
    f, uw = ljmd.brute_forces(len(x), box, p, xz, sp, precision=FP64)
    f, uw = f.cpu().numpy(), uw.cpu().numpy()
    fb, Ub, Wb = oracle.forces_brute(x, sp, box, p)
    rms = float(np.sqrt((fb ** 2).sum(1).mean()))
    assert np.all(f[:, 2] == 0.0)
    assert np.abs(f - fb).max() <= 1e-12 * max(rms, 1.0)
    assert abs(uw[0] - Ub) <= 1e-12 * abs(Ub) and abs(uw[1] - Wb) <= 1e-12 * max(1.0, abs(Wb))
