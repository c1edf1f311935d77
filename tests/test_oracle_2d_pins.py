"""Pins of the oracle in two dimensions (the dimension template of the
paper's modules, Sec. 3): particles in the plane z = 0 of a box whose third
edge only sizes an unused axis.

* A perfect triangular lattice: every force vanishes (each site is a centre
  of symmetry), and U/N equals half the sum of phi_s over the lattice
  vectors inside the cutoff, enumerated here from the two primitive vectors
  of the infinite lattice (independent of the oracle's box, cells and
  minimum image).
* Forces stay in the plane: a jittered lattice gets F_z = 0 exactly, and a
  run keeps z and v_z exactly 0.
* The thermostat in the plane: resampled velocities have v_z = 0 and in-plane
  components of variance T/m, and a thermostatted fluid settles at
  sum m v^2 / (2N - 2) = T (two degrees of freedom per particle).
"""
import math

import numpy as np
import pytest

import oracle
from paper_2406_04210_amd import workloads as W


def lattice_energy_per_site(rho, p):
    a = math.sqrt(2.0 / (math.sqrt(3.0) * rho))
    a1 = np.array([a, 0.0])
    a2 = np.array([0.5 * a, 0.5 * math.sqrt(3.0) * a])
    rc = p.rcut[0]
    kmax = int(math.ceil(rc / (0.5 * a))) + 2
    terms = []
    for i in range(-kmax, kmax + 1):
        for j in range(-kmax, kmax + 1):
            if i == 0 and j == 0:
                continue
            r = float(np.linalg.norm(i * a1 + j * a2))
            if r < rc:
                terms.append(oracle.phi(r) - oracle.phi(rc))
    return 0.5 * math.fsum(terms), a


def test_triangular_lattice_forces_vanish_and_energy_is_the_lattice_sum():
    p = W.single_species_params()
    p.dim = 2
    rho = 0.7
    x, L = W.triangular_lattice(16, rho)
    sp = np.zeros(len(x), np.int32)
    u_site, a = lattice_energy_per_site(rho, p)
    # No lattice shell within 2% of r_c: the cutoff decision is unambiguous.
    for k2 in (1, 3, 4, 7, 9):
        assert abs(math.sqrt(k2) * a - p.rcut[0]) > 0.02 * p.rcut[0]
    f, U, Wv = oracle.forces(x, sp, L, p)
    assert np.abs(f).max() <= 1e-12
    assert U / len(x) == pytest.approx(u_site, rel=1e-13)
    fb, Ub, _ = oracle.forces_brute(x, sp, L, p)
    assert Ub == pytest.approx(U, rel=1e-13)


def test_forces_and_motion_stay_in_the_plane():
    w = W.lj_fluid_2d(m=12, rho=0.7)
    f, U, Wv = oracle.forces(w.x, w.species, w.box, w.params)
    assert np.all(f[:, 2] == 0.0)
    assert np.abs(f[:, :2]).max() > 1.0          # the jittered lattice is not in balance
    r = oracle.run_nve(w.x, w.v, w.species, w.box, w.params, 60)
    assert np.all(r["x"][:, 2] == 0.0) and np.all(r["v"][:, 2] == 0.0)
    # Momentum stays zero in the plane (Newton's third law).
    assert np.abs(r["obs"][:, 3:6]).max() < 1e-11


def test_thermostat_in_the_plane():
    w = W.lj_fluid_2d(m=12, rho=0.7, temperature=1.0)
    T = 1.6
    r = oracle.run_nve(w.x, w.v, w.species, w.box, w.params, 2500, thermostat=(T, 5.0, 99))
    v = r["v"]
    assert np.all(v[:, 2] == 0.0)
    n = len(v)
    K = r["obs"][:, 1]
    t_series = 2.0 * K / (2 * n - 2)
    # Samples of 288 particles scatter by ~6 %; 2,000 steps average that to ~1 %.
    t_mean = t_series[500:].mean()
    assert t_mean == pytest.approx(T, rel=0.03), t_mean
    # In-plane components of the draws themselves: N(0, T/m), v_z = 0.
    thr = oracle.thermo_threshold(5.0, w.params.dt)
    zs = []
    for pid in range(800):
        for step in range(1, 60):
            hit, z = oracle.thermo_draw(99, pid, step, thr)
            if hit:
                zs.append(z[:2])
    zs = np.array(zs)
    assert len(zs) > 1000
    assert zs.mean() == pytest.approx(0.0, abs=0.1)
    assert zs.var() == pytest.approx(1.0, rel=0.1)
