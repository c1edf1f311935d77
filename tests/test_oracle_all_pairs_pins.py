"""Pins of the oracle's untruncated all-pairs mode (the all-to-all
Lennard-Jones interaction the paper's port started from, Sec. 4 and Sec. 5
"GPU Performance for All-to-All Interaction"): with an infinite cutoff every
pair of the minimum image interacts through the plain 12-6 potential, with
no shift (phi(inf) = 0).

* A dimer and a collinear trimer: U and F equal the closed forms.
* F = -grad U by finite differences of the untruncated energy.
* Newton's third law; the untruncated energy equals the truncated-shifted
  energy plus, per pair, phi(r_c) inside the cutoff and phi(r) outside it.
* The list-based forces with an infinite cutoff equal the brute force.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2406_04210_amd import workloads as W


def untruncated(p):
    q = p.copy()
    q.rcut = np.full(4, np.inf)
    return q


def test_dimer_and_trimer_closed_forms():
    p = untruncated(W.single_species_params())
    box = np.full(3, 30.0)
    sp = np.zeros(3, np.int32)
    x = np.array([[1.0, 1.0, 1.0], [4.2, 1.0, 1.0], [6.0, 1.0, 1.0]])
    f, U, Wv = oracle.forces_brute(x, sp, box, p)
    r12, r23, r13 = 3.2, 1.8, 5.0
    phi = lambda r: 4.0 * (r ** -12 - r ** -6)
    fsr = lambda r: 24.0 * (2.0 * r ** -13 - r ** -7)        # -phi'(r)
    assert U == pytest.approx(phi(r12) + phi(r23) + phi(r13), rel=1e-14)
    assert Wv == pytest.approx(fsr(r12) * r12 + fsr(r23) * r23 + fsr(r13) * r13, rel=1e-14)
    assert f[0, 0] == pytest.approx(-fsr(r12) - fsr(r13), rel=1e-13)
    assert f[2, 0] == pytest.approx(fsr(r23) + fsr(r13), rel=1e-13)
    assert np.abs(f[:, 1:]).max() == 0.0


def test_force_is_minus_gradient_and_newton_third_law():
    w = W.random_dense(200, 0.8, seed=31, nspecies=2, min_dist=0.8)
    p = untruncated(w.params)
    f, U, _ = oracle.forces_brute(w.x, w.species, w.box, p)
    rms = np.sqrt((f ** 2).sum(1).mean())
    assert np.abs(f.sum(0)).max() <= 1e-12 * math.sqrt(w.n) * rms
    rng = np.random.default_rng(3)
    h = 2e-5
    for _ in range(5):
        i, k = int(rng.integers(w.n)), int(rng.integers(3))

        def E(s):
            x = w.x.copy()
            x[i, k] += s
            return oracle.forces_brute(x, w.species, w.box, p)[1]

        g = (-E(2 * h) + 8 * E(h) - 8 * E(-h) + E(-2 * h)) / (12 * h)
        assert -g == pytest.approx(f[i, k], rel=2e-7, abs=2e-7 * np.abs(f).max())


def test_untruncated_minus_truncated_is_the_pair_tail():
    w = W.random_dense(300, 0.85, seed=32)
    p = w.params
    q = untruncated(p)
    _, Ut, _ = oracle.forces_brute(w.x, w.species, w.box, p)
    _, Uu, _ = oracle.forces_brute(w.x, w.species, w.box, q)
    d = w.x[:, None, :] - w.x[None, :, :]
    d -= w.box * np.rint(d / w.box)
    r = np.sqrt((d * d).sum(-1))[np.triu_indices(w.n, 1)]
    rc = p.rcut[0]
    tail = sum(oracle.phi(rc) if rr < rc else oracle.phi(rr) for rr in r)
    assert Uu == pytest.approx(Ut + tail, rel=1e-12)


def test_list_forces_with_infinite_cutoff_equal_brute_force():
    w = W.random_dense(400, 0.8442, seed=33)
    p = untruncated(w.params)
    fb, Ub, Wb = oracle.forces_brute(w.x, w.species, w.box, p)
    fl, Ul, Wl = oracle.forces(w.x, w.species, w.box, p)
    rms = np.sqrt((fb ** 2).sum(1).mean())
    assert np.abs(fl - fb).max() <= 1e-12 * rms
    assert Ul == pytest.approx(Ub, rel=1e-12)


def test_brute_sums_are_correctly_rounded_on_the_2000_particle_fluid():
    # The all-to-all workload (2,000 particles, 2e6 pairs, many of them at
    # equal lattice distances): the oracle's U and W equal the correctly
    # rounded sums (math.fsum) of the pair terms to a few units of the last
    # place. A plain double accumulator misses them by ~6e-12 relative.
    w = W.all_pairs_fluid()
    x, n, L = w.x, w.n, w.box
    _, U, Wv = oracle.forces_brute(x, w.species, w.box, w.params)
    i, j = np.triu_indices(n, 1)
    d = x[i] - x[j]
    d -= L * np.rint(d / L)
    r2 = (d * d).sum(axis=1)
    s6 = (1.0 / r2) ** 3
    U_exact = math.fsum((4.0 * (s6 * s6 - s6)).tolist())
    W_exact = math.fsum((24.0 * (2.0 * s6 * s6 - s6)).tolist())
    assert abs(U - U_exact) <= 1e-14 * abs(U_exact)
    assert abs(Wv - W_exact) <= 1e-14 * abs(W_exact)
