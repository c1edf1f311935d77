"""The Andersen-like ("Boltzmann") thermostat on the GPU against the oracle,
through the C ABI.

Both sides draw from Philox4x32-10 keyed by the seed with counters (original
id, step), so the collision decisions are integer comparisons taken
identically; the resampled velocities sqrt(T/m) z go through log, sqrt, cos
and sin, which the device and host libraries round within an ulp or so of
each other. A collision decided differently would move a velocity by O(1);
the trajectories agree to the tolerances of the NVE parity tests, so every
decision matched.
"""
import numpy as np
import pytest

import oracle
from paper_2406_04210_amd import workloads as W

pytestmark = pytest.mark.gpu
FP64, FP32 = 0, 1


@pytest.fixture(scope="module")
def ljmd():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2406_04210_amd import ljmd as L
    return L


def run_gpu(ljmd, w, prec, nsteps, thermo, sort_interval=25, p=None):
    p = w.params if p is None else p
    s = ljmd.System(w.n, w.box, p, precision=prec, sort_interval=sort_interval)
    s.set_state(w.x, w.v, w.species)
    if thermo is not None:
        s.set_thermostat(*thermo)
    obs = s.run(nsteps).cpu().numpy()
    s.sync()
    xu = s.unwrapped_positions().cpu().numpy()
    _, v, _ = s.get_state()
    return obs, xu, v.cpu().numpy()


@pytest.mark.parametrize("prec", [FP64, FP32])
def test_thermostat_trajectory_matches_oracle(ljmd, prec):
    w = W.config_small()
    thermo = (1.5, 10.0, 2024)             # T, collision rate (probability 0.05 per step), seed
    obs, xu, v = run_gpu(ljmd, w, prec, 100, thermo)
    r = oracle.run_nve(w.x, w.v, w.species, w.box, w.params, 100, thermostat=thermo)
    dx, dv = np.abs(xu - r["x"]).max(), np.abs(v - r["v"]).max()
    dk = np.abs(obs[:, 1] - r["obs"][1:, 1]).max() / w.n
    print(f"thermostat prec={prec}: max|dx| {dx:.3e} max|dv| {dv:.3e} max|dK|/N {dk:.3e}", flush=True)
    tol_x, tol_v, tol_k = (1e-10, 1e-9, 1e-10) if prec == FP64 else (1e-4, 1e-3, 1e-5)
    assert dx <= tol_x and dv <= tol_v and dk <= tol_k
    # The kinetic energy moved towards the bath (T 1.0 -> 1.5).
    assert obs[-1, 1] > obs[0, 1]


def test_thermostat_unequal_masses_matches_oracle(ljmd):
    r0 = W.random_dense(1500, 1.1, seed=7, nspecies=2, min_dist=0.75)
    p = r0.params.copy()
    p.mass = np.array([1.0, 2.0])
    thermo = (0.9, 20.0, 77)
    obs, xu, v = run_gpu(ljmd, r0, FP64, 60, thermo, p=p)
    r = oracle.run_nve(r0.x, r0.v, r0.species, r0.box, p, 60, thermostat=thermo)
    assert np.abs(xu - r["x"]).max() <= 1e-10 and np.abs(v - r["v"]).max() <= 1e-9


def test_thermostat_draws_follow_ids_not_order(ljmd):
    # A resort every 7 steps reorders the particles; draws are keyed by the
    # original id, so the run matches the one without resorts (up to force
    # summation order).
    w = W.config_small()
    thermo = (1.2, 30.0, 5)
    _, xa, va = run_gpu(ljmd, w, FP64, 60, thermo, sort_interval=7)
    _, xb, vb = run_gpu(ljmd, w, FP64, 60, thermo, sort_interval=0)
    assert np.abs(xa - xb).max() <= 1e-11 and np.abs(va - vb).max() <= 1e-10


@pytest.mark.parametrize("prec", [FP64, FP32])
def test_rate_zero_is_nve_bitwise(ljmd, prec):
    w = W.config_small()
    a = run_gpu(ljmd, w, prec, 40, None)
    b = run_gpu(ljmd, w, prec, 40, (3.0, 0.0, 9))
    for u, t in zip(a, b):
        assert np.array_equal(u, t)


def test_thermostat_relaxes_to_the_bath_temperature(ljmd):
    x, L = W.fcc_lattice(10, 0.8442)
    sp = np.zeros(len(x), np.int32)
    p = W.single_species_params()
    v = W.maxwell_boltzmann(len(x), 0.5, p.mass, sp, np.random.default_rng(3))
    s = ljmd.System(len(x), np.full(3, L), p, precision=FP32)
    s.set_state(x, v, sp)
    s.set_thermostat(1.0, 10.0, 11)
    obs = s.run(3000).cpu().numpy()
    s.sync()
    T = 2.0 * obs[1500:, 1] / (3 * len(x) - 3)
    assert T.mean() == pytest.approx(1.0, abs=0.03)


def test_thermostat_rejects_bad_values_and_rollouts(ljmd):
    w = W.config_small()
    s = ljmd.System(w.n, w.box, w.params, precision=FP64)
    s.set_state(w.x, w.v, w.species)
    with pytest.raises(ljmd.LJMDError):
        s.set_thermostat(1.0, -1.0, 0)
    s.set_thermostat(1.0, 5.0, 0)
    with pytest.raises(ljmd.LJMDError):
        s.vv_forward(5, 5)
