"""Pins of the oracle's mass handling: every other pin uses unit masses, so
these use species masses 1 and 2 (or 3), where a mass in place of its
inverse, or the masses of the two species swapped, changes the answer.

* A dimer of unequal masses oscillates with omega = sqrt(phi''(r_min) / mu),
  mu = m1 m2 / (m1 + m2) (two-body reduction, textbook mechanics), shifted by
  velocity Verlet as cos(omega' dt) = 1 - (omega dt)^2 / 2.
* Internal forces conserve the total momentum sum m v exactly (Newton's
  third law), also when it is not zero, and the centre of mass then moves
  uniformly; with the masses swapped in the kicks neither holds.
* K = sum m v^2 / 2 and p = sum m v for a hand-computed case.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2406_04210_amd import workloads as W

RMIN = 2.0 ** (1.0 / 6.0)


def two_species_equal_potential(m0, m1):
    p = W.single_species_params()
    p.nspecies = 2
    p.mass = np.array([m0, m1], dtype=np.float64)
    return p


def test_kinetic_energy_and_momentum_by_hand():
    p = two_species_equal_potential(1.0, 2.0)
    v = np.array([[1.0, 0.0, 0.0], [0.0, 2.0, -1.0], [0.5, 0.5, 0.5]])
    sp = np.array([0, 1, 1], np.int32)
    K, mom = oracle.kinetic(v, sp, p)
    assert K == 0.5 * 1.0 * 1.0 + 0.5 * 2.0 * 5.0 + 0.5 * 2.0 * 0.75
    assert np.array_equal(mom, np.array([1.0 + 1.0, 4.0 + 1.0, -2.0 + 1.0]))


@pytest.mark.parametrize("masses", [(1.0, 2.0), (2.0, 1.0), (1.0, 3.0)])
def test_unequal_mass_dimer_frequency(masses):
    m0, m1 = masses
    p = two_species_equal_potential(m0, m1)
    box = np.full(3, 10.0)
    amp = 0.005
    x = np.array([[5.0 - 0.5 * (RMIN + amp), 5.0, 5.0], [5.0 + 0.5 * (RMIN + amp), 5.0, 5.0]])
    sp = np.array([0, 1], np.int32)
    xs, vs = x, np.zeros((2, 3))
    seps = [x[1, 0] - x[0, 0]]
    for _ in range(1500):
        r = oracle.run_nve(xs, vs, sp, box, p, 1, want_obs=False)
        xs, vs = r["x"], r["v"]
        seps.append(xs[1, 0] - xs[0, 0])
        # Momentum stays zero: m0 v0 + m1 v1 = 0 along the axis.
        assert abs(m0 * vs[0, 0] + m1 * vs[1, 0]) < 1e-13
    s = np.array(seps) - RMIN
    t = [k + s[k] / (s[k] - s[k + 1]) for k in range(len(s) - 1) if s[k] < 0 <= s[k + 1]]
    period_steps = (t[-1] - t[0]) / (len(t) - 1)
    mu = m0 * m1 / (m0 + m1)
    omega = math.sqrt(72.0 * 2.0 ** (-1.0 / 3.0) / mu)
    wdt = omega * p.dt
    want = 2.0 * math.pi / (math.acos(1.0 - wdt * wdt / 2.0) / p.dt) / p.dt
    assert period_steps == pytest.approx(want, rel=2e-3)
    # The unit-mass period differs by far more than the tolerance.
    w1 = math.sqrt(2.0 * 72.0 * 2.0 ** (-1.0 / 3.0)) * p.dt
    assert abs(2.0 * math.pi / math.acos(1.0 - w1 * w1 / 2.0) - want) > 0.05 * want


def test_momentum_and_centre_of_mass_with_unequal_masses():
    w = W.random_dense(500, 0.9, seed=21, nspecies=2, min_dist=0.8)
    p = w.params.copy()
    p.mass = np.array([1.0, 3.0])
    m = p.mass[w.species][:, None]
    v = W.maxwell_boltzmann(w.n, 1.0, p.mass, w.species, np.random.default_rng(4))
    v = v + np.array([0.3, -0.2, 0.1])            # a non-zero total momentum
    P0 = (m * v).sum(axis=0)
    M = m.sum()
    R0 = (m * w.x).sum(axis=0) / M
    nsteps = 200
    r = oracle.run_nve(w.x, v, w.species, w.box, p, nsteps)
    P = (m * r["v"]).sum(axis=0)
    assert np.abs(P - P0).max() <= 1e-11 * np.abs(P0).max()
    assert np.abs(r["obs"][:, 3:] - P0[None, :]).max() <= 1e-11 * np.abs(P0).max()
    R = (m * r["x"]).sum(axis=0) / M
    assert np.abs(R - (R0 + nsteps * p.dt * P0 / M)).max() < 1e-11
    # The kinetic energy is mass-weighted: K equals sum m v^2 / 2 of the final state.
    K, _ = oracle.kinetic(r["v"], w.species, p)
    assert r["obs"][-1, 1] == K
    # Negative control: with the species masses swapped the momentum drifts.
    q = p.copy()
    q.mass = np.array([3.0, 1.0])
    r2 = oracle.run_nve(w.x, v, w.species, w.box, q, nsteps)
    P2 = (m * r2["v"]).sum(axis=0)
    assert np.abs(P2 - P0).max() > 1e-6
