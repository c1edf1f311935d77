"""Edge and degenerate inputs through the C ABI, against the oracle:

* the smallest systems: a dimer (N = 2) oscillating for 200 steps and a
  collinear trimer, in a box of one or two cells per axis;
* a dilute gas where most particles have no partner (empty lists, zero
  forces);
* two particles at the same position (never partners: the pair
  interaction is undefined at r = 0, and the list criterion is 0 < r^2);
* coordinates outside [0, L) and exactly at L (wrapped on load, images
  counted);
* the smallest box the minimum image allows (L = 2 r_L) and one just below
  it (LJMD_EBOX)."""
import numpy as np
import pytest

import oracle
from force_metrics import bound_key, force_errors, reference, report, tie_allowance
from paper_2406_04210_amd import workloads as W

pytestmark = pytest.mark.gpu
FP64, FP32_DS = 0, 1


@pytest.fixture(scope="module")
def ljmd():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2406_04210_amd import ljmd as L
    return L


def lists_equal(ljmd, s, x, sp, box, p, prec):
    cnt, ids = s.neighbors(cap=256)
    s.sync()
    cnt, ids = cnt.cpu().numpy(), ids.cpu().numpy()
    oc, on = oracle.build_lists(x, sp, box, p, mode=0 if prec == FP64 else 1)
    assert np.array_equal(cnt, oc)
    for i in range(len(x)):
        assert set(ids[i, : cnt[i]].tolist()) == set(on[i, : oc[i]].tolist())
    return cnt


@pytest.mark.parametrize("prec", [FP64, FP32_DS])
def test_dimer_trajectory(ljmd, prec):
    p = W.single_species_params()
    box = np.full(3, 6.0)
    x = np.array([[1.0, 2.0, 3.0], [2.2, 2.05, 2.9]])
    v = np.array([[0.3, -0.1, 0.05], [-0.3, 0.1, -0.05]])
    sp = np.zeros(2, np.int32)
    s = ljmd.System(2, box, p, precision=prec, sort_interval=50)
    s.set_state(x, v, sp)
    assert list(lists_equal(ljmd, s, x, sp, box, p, prec)) == [1, 1]
    s.run(200, observe=False)
    s.sync()
    xu = s.unwrapped_positions().cpu().numpy()
    r = oracle.run_nve(x, v, sp, box, p, 200)
    tol = 1e-10 if prec == FP64 else 1e-5
    assert np.abs(xu - r["x"]).max() <= tol


@pytest.mark.parametrize("prec", [FP64, FP32_DS])
def test_trimer_forces(ljmd, prec):
    p = W.single_species_params()
    box = np.full(3, 7.0)
    x = np.array([[1.0, 1.0, 1.0], [2.15, 1.0, 1.0], [3.4, 1.0, 1.0]])
    sp = np.zeros(3, np.int32)
    s = ljmd.System(3, box, p, precision=prec)
    s.set_state(x, np.zeros_like(x), sp)
    f = s.forces().cpu().numpy()
    fb, Ub, Wb = oracle.forces_brute(x, sp, box, p)
    scale = np.abs(fb).max()
    assert np.abs(f - fb).max() <= (1e-12 if prec == FP64 else 1e-5) * scale
    o = s.observables()
    assert o["U"] == pytest.approx(Ub, rel=1e-12 if prec == FP64 else 5e-6)


@pytest.mark.parametrize("prec", [FP64, FP32_DS])
def test_dilute_gas_with_isolated_particles(ljmd, prec):
    rng = np.random.default_rng(31)
    p = W.single_species_params()
    box = np.full(3, 40.0)
    x = rng.uniform(0.0, 40.0, size=(64, 3))
    sp = np.zeros(64, np.int32)
    s = ljmd.System(64, box, p, precision=prec)
    s.set_state(x, np.zeros_like(x), sp)
    cnt = lists_equal(ljmd, s, x, sp, box, p, prec)
    assert (cnt == 0).sum() > 20                     # most have no partner
    f = s.forces().cpu().numpy()
    fo, _, _ = oracle.forces(x, sp, box, p)
    assert np.all(f[cnt == 0] == 0.0)
    r = 1 if prec == FP32_DS else FP64
    ref, _, _, A = reference(x, sp, box, p, r)
    m = report(f"dilute prec={prec}", force_errors(f, ref, A, tie_allowance(x, sp, box, p, r)))
    assert m[bound_key(r)] <= (1e-12 if prec == FP64 else 1e-5)


@pytest.mark.parametrize("prec", [FP64, FP32_DS])
def test_coincident_particles_are_not_partners(ljmd, prec):
    w = W.random_dense(300, 0.8442, seed=13)
    x = w.x.copy()
    x[7] = x[150]                                    # particle 7 on top of particle 150
    s = ljmd.System(len(x), w.box, w.params, precision=prec)
    s.set_state(x, np.zeros_like(x), w.species)
    cnt, ids = s.neighbors(cap=256)
    s.sync()
    cnt, ids = cnt.cpu().numpy(), ids.cpu().numpy()
    assert 150 not in ids[7, : cnt[7]] and 7 not in ids[150, : cnt[150]]
    lists_equal(ljmd, s, x, w.species, w.box, w.params, prec)
    f = s.forces().cpu().numpy()
    assert np.isfinite(f).all()
    r = 1 if prec == FP32_DS else FP64
    ref, _, _, A = reference(x, w.species, w.box, w.params, r)
    m = report(f"coincident prec={prec}", force_errors(f, ref, A, tie_allowance(x, w.species, w.box, w.params, r)))
    assert m[bound_key(r)] <= (1e-12 if prec == FP64 else 1e-5)


@pytest.mark.parametrize("prec", [FP64, FP32_DS])
def test_coordinates_outside_the_box_are_wrapped(ljmd, prec):
    w = W.random_dense(400, 0.8442, seed=17)
    L = w.box[0]
    shift = np.random.default_rng(5).integers(-3, 4, size=w.x.shape)
    x = w.x + shift * L
    x[0] = [L, 0.0, 2 * L]                           # exactly at the edge: wraps to 0
    s = ljmd.System(len(x), w.box, w.params, precision=prec)
    s.set_state(x, np.zeros_like(x), w.species)
    f = s.forces().cpu().numpy()
    xw = x - L * np.floor(x / L)
    xw[xw >= L] -= L
    r = 1 if prec == FP32_DS else FP64
    ref, _, _, A = reference(xw, w.species, w.box, w.params, r)
    m = report(f"wrapped prec={prec}", force_errors(f, ref, A, tie_allowance(xw, w.species, w.box, w.params, r)))
    assert m[bound_key(r)] <= (1e-12 if prec == FP64 else 1e-5)
    xu = s.unwrapped_positions().cpu().numpy()
    assert np.abs(xu - x).max() <= 1e-12 * 4 * L


def test_smallest_box_and_one_below(ljmd):
    p = W.single_species_params()
    rl = p.rcut[0] + p.skin
    L = 2.0 * rl
    n = 120
    w = W.random_dense(n, n / L ** 3, seed=43)
    s = ljmd.System(n, np.full(3, L), p, precision=FP64)
    s.set_state(w.x, np.zeros_like(w.x), w.species)
    lists_equal(ljmd, s, w.x, w.species, np.full(3, L), p, FP64)
    f = s.forces().cpu().numpy()
    fo, _, _ = oracle.forces(w.x, w.species, np.full(3, L), p)
    assert np.abs(f - fo).max() <= 1e-12 * max(1.0, float(np.sqrt((fo ** 2).sum(1).mean())))
    with pytest.raises(ljmd.LJMDError) as err:
        ljmd.System(n, np.full(3, L * (1 - 1e-9)), p, precision=FP64)
    assert err.value.code == -4                       # LJMD_EBOX


@pytest.mark.parametrize("prec", [FP64, FP32_DS])
@pytest.mark.parametrize("ncell_axis", [3, 5])
def test_crowded_cell_lists(ljmd, prec, ncell_axis):
    # One cell holding about 150 particles (a cluster dropped into a sparse
    # gas): the list build takes a cell's particles 64 at a time, splits
    # them in two groups along z and queues each group's candidates; with 3
    # cells per axis the box test takes the wrapped gap, with 5 the signed
    # one. Lists must match the oracle's sets exactly.
    p = W.single_species_params()
    rl = p.rcut[0] + p.skin
    L = ncell_axis * rl * 1.01
    edge = L / ncell_axis
    rng = np.random.default_rng(31 + ncell_axis)
    x = np.concatenate([rng.uniform(0.0, L, size=(300, 3)),
                        edge + rng.uniform(0.02 * edge, 0.98 * edge, size=(140, 3))])
    sp = np.zeros(len(x), dtype=np.int32)
    box = (L, L, L)
    s = ljmd.System(len(x), box, p, precision=prec, nbr_capacity=384, cell_capacity=256)
    s.set_state(x, np.zeros_like(x), sp)
    cnt, ids = s.neighbors(cap=512)
    s.sync()
    cnt, ids = cnt.cpu().numpy(), ids.cpu().numpy()
    oc, on = oracle.build_lists(x, sp, box, p, mode=0 if prec == FP64 else 1, cap=512)
    assert oc.max() > 64 and oc.max() <= 384
    assert np.array_equal(cnt, oc)
    for i in range(len(x)):
        assert set(ids[i, : cnt[i]].tolist()) == set(on[i, : oc[i]].tolist()), i
