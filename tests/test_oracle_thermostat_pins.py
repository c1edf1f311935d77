"""Pins of the oracle's stochastic velocity-resampling thermostat (the
Andersen-like "Boltzmann" thermostat the paper combines with velocity
Verlet, Sec. 4) and of its counter-based generator.

* Philox4x32-10 reproduces the known-answer vectors its authors publish.
* Collisions happen with probability rate * dt per particle and step
  (binomial bounds), and resampled velocities follow N(0, T/m) per
  component (moments, with masses 1 and 2).
* Rate 0 leaves velocity Verlet untouched bit for bit; a thermostatted
  fluid relaxes to the target temperature from above and below.
* Draws depend only on (seed, id, step): relabelling the particles
  relabels the draws.
"""
import math
import os

import numpy as np
import pytest

import oracle
from paper_2406_04210_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def kat_rows():
    rows = []
    with open(GOLDEN) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            w = [int(t, 16) for t in line.split()]
            rows.append((w[0:4], w[4:6], w[6:10]))
    return rows


@pytest.mark.parametrize("row", kat_rows())
def test_philox_known_answers(row):
    ctr, key, want = row
    assert oracle.philox4x32(ctr, key).tolist() == want


def test_collision_rate_and_maxwell_boltzmann_moments():
    rate, dt, T = 2.0, 0.005, 1.3
    thr = oracle.thermo_threshold(rate, dt)
    assert thr == math.floor(rate * dt * 2.0 ** 32)
    hits, zs = 0, []
    trials = 0
    for step in range(1, 41):
        for pid in range(2000):
            trials += 1
            hit, z = oracle.thermo_draw(12345, pid, step, thr)
            if hit:
                hits += 1
                zs.append(z)
    pr = rate * dt
    sd = math.sqrt(trials * pr * (1 - pr))
    assert abs(hits - trials * pr) < 5 * sd
    # Every particle draws N(0,1) deviates when the threshold is 2^32 - 1.
    z = np.array([oracle.thermo_draw(7, pid, 3, 0xFFFFFFFF)[1] for pid in range(40000)])
    n = z.size
    assert abs(z.mean()) < 5 / math.sqrt(n)
    assert abs(z.var() - 1.0) < 5 * math.sqrt(2.0 / n)
    assert abs((z ** 4).mean() / (z ** 2).mean() ** 2 - 3.0) < 0.1
    # Components are uncorrelated.
    c = np.corrcoef(z.T)
    assert np.abs(c - np.eye(3)).max() < 5 / math.sqrt(40000)


def test_rate_zero_is_plain_velocity_verlet():
    w = W.config_small()
    a = oracle.run_nve(w.x, w.v, w.species, w.box, w.params, 30)
    b = oracle.run_nve(w.x, w.v, w.species, w.box, w.params, 30, thermostat=(1.0, 0.0, 9))
    assert np.array_equal(a["x"], b["x"]) and np.array_equal(a["v"], b["v"])


def test_resampled_velocities_and_mass_scaling():
    # Rate so high that every particle collides every step: after one step
    # every velocity is sqrt(T/m) z with z from its own draw.
    w = W.random_dense(600, 0.8, seed=5, nspecies=2, min_dist=0.85)
    p = w.params.copy()
    p.mass = np.array([1.0, 2.0])
    T = 1.7
    big = 1e12
    r = oracle.run_nve(w.x, w.v, w.species, w.box, p, 1, thermostat=(T, big, 77))
    thr = oracle.thermo_threshold(big, p.dt)
    assert thr == 0xFFFFFFFF
    for pid in range(0, w.n, 37):
        hit, z = oracle.thermo_draw(77, pid, 1, thr)
        assert hit
        want = math.sqrt(T / p.mass[w.species[pid]]) * z
        assert np.array_equal(r["v"][pid], want)
    m = p.mass[w.species][:, None]
    kT = (m * r["v"] ** 2).mean()
    assert kT == pytest.approx(T, rel=5 * math.sqrt(2.0 / (3 * w.n)))


@pytest.mark.parametrize("t0", [0.5, 2.0])
def test_thermostat_relaxes_to_target_temperature(t0):
    x, L = W.fcc_lattice(5, 0.8442)
    sp = np.zeros(len(x), np.int32)
    p = W.single_species_params()
    v = W.maxwell_boltzmann(len(x), t0, p.mass, sp, np.random.default_rng(3))
    box = np.full(3, L)
    r = oracle.run_nve(x, v, sp, box, p, 3000, thermostat=(1.0, 10.0, 2024))
    K = r["obs"][1500:, 1]
    T = 2.0 * K / (3 * len(x) - 3)
    assert T.mean() == pytest.approx(1.0, abs=0.06)


def test_draws_follow_ids_not_rows():
    w = W.random_dense(300, 0.8, seed=9)
    perm = np.random.default_rng(1).permutation(w.n)
    thr = oracle.thermo_threshold(20.0, w.params.dt)
    rows = [oracle.thermo_draw(5, pid, 4, thr) for pid in range(w.n)]
    rows_p = [oracle.thermo_draw(5, pid, 4, thr) for pid in perm]
    for k, pid in enumerate(perm):
        assert rows_p[k][0] == rows[pid][0]
        if rows[pid][0]:
            assert np.array_equal(rows_p[k][1], rows[pid][1])
