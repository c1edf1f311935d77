"""Pins of the oracle's fixed-point force mode (forces of the positions the
single-precision path represents: 32-bit fixed-point image coordinates).

* In a box of edge 16 with coordinates on the 2^-20 grid, every coordinate
  is a float (so its double-single split is exact) and q = x 2^28 exactly:
  the fixed-point displacements are then the exact displacements, and the
  mode must give bitwise the plain FP64 list forces. A wrong sign, quantum
  or image in the mode fails this.
* For general positions the mode differs from plain FP64 by at most what
  one quantum per coordinate can change (per pair sqrt(3) L 2^-32 times
  |dF/dr| + |F|/r, the pair force's Lipschitz bound), and it does differ.
* The per-particle sum of pair-force magnitudes bounds the net force
  (triangle inequality) and is zero exactly for particles without partners
  inside the cutoff.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2406_04210_amd import workloads as W


def grid_positions(n, L, rho_seed):
    x, _ = W.fcc_lattice(8, 0.8442)
    x = x[:n] * (L / (8 * (4.0 / 0.8442) ** (1.0 / 3.0)))
    rng = np.random.default_rng(rho_seed)
    x = (x + 0.05 * rng.standard_normal(x.shape)) % L
    return np.round(x * 2.0 ** 20) / 2.0 ** 20 % L


@pytest.mark.parametrize("nspecies", [1, 2])
def test_exact_grid_positions_give_plain_forces_bitwise(nspecies):
    L = 16.0
    x = grid_positions(2048, L, 3)
    box = np.full(3, L)
    p = W.single_species_params() if nspecies == 1 else W.binary_mixture_params()
    sp = np.zeros(len(x), np.int32) if nspecies == 1 else (np.arange(len(x)) % 5 == 0).astype(np.int32)
    cnt, nbr = oracle.build_lists(x, sp, box, p, 0)
    f0, U0, W0 = oracle.forces_list(x, sp, box, p, cnt, nbr)
    f1, U1, W1, fa = oracle.forces_fixed(x, sp, box, p, cnt, nbr)
    assert np.abs(f0).max() > 1.0
    assert np.array_equal(f0, f1)
    # (U and W are OpenMP reductions: equal up to the order of the thread sums.)
    assert U1 == pytest.approx(U0, rel=1e-13) and W1 == pytest.approx(W0, rel=1e-13)


def test_general_positions_within_one_quantum_per_coordinate():
    x, L = W.fcc_lattice(8, 0.8442)
    rng = np.random.default_rng(8)
    x = x + 0.07 * rng.standard_normal(x.shape)
    box = np.full(3, L)
    sp = np.zeros(len(x), np.int32)
    p = W.single_species_params()
    cnt, nbr = oracle.build_lists(x, sp, box, p, 0)
    f0, _, _ = oracle.forces_list(x, sp, box, p, cnt, nbr)
    f1, _, _, fa = oracle.forces_fixed(x, sp, box, p, cnt, nbr)
    qs = L / 2.0 ** 32
    # Lipschitz bound of the pair force over a displacement change of at most
    # sqrt(3) quanta per pair (each coordinate rounded to the nearest quantum
    # up to one unit: two particles, so up to 2 quanta per axis).
    n = len(x)
    i = np.repeat(np.arange(n), cnt)
    j = nbr[np.arange(nbr.shape[1])[None, :] < cnt[:, None]]
    d = x[i] - x[j]
    d -= box * np.rint(d / box)
    r = np.sqrt((d * d).sum(1))
    inside = r < p.rcut[0] - 1e-9
    u = 1.0 / r
    F = 24.0 * (2.0 * u ** 13 - u ** 7)
    dF = 24.0 * (-26.0 * u ** 14 + 7.0 * u ** 8)
    bound = np.bincount(i, weights=inside * 2.0 * math.sqrt(3.0) * qs * (np.abs(dF) + np.abs(F) / r),
                        minlength=n)
    err = np.linalg.norm(f1 - f0, axis=1)
    assert np.all(err <= bound * 1.01 + 1e-13)
    assert err.max() > 0.0
    # Triangle inequality, and the magnitude sum itself.
    assert np.all(np.linalg.norm(f1, axis=1) <= fa * (1 + 1e-12))
    want = np.bincount(i, weights=inside * np.abs(F), minlength=n)
    assert np.allclose(fa, want, rtol=1e-6)


def test_isolated_particle_has_zero_magnitude_sum():
    p = W.single_species_params()
    box = np.full(3, 12.0)
    x = np.array([[1.0, 1.0, 1.0], [2.1, 1.0, 1.0], [7.0, 7.0, 7.0]])
    sp = np.zeros(3, np.int32)
    f, U, Wv, fa = oracle.forces_fixed(x, sp, box, p)
    assert fa[2] == 0.0 and np.all(f[2] == 0.0)
    assert fa[0] == pytest.approx(abs(oracle.fscalar(1.1)) * 1.1, rel=1e-7)
    assert f[0, 0] == pytest.approx(-f[1, 0], rel=1e-15)
