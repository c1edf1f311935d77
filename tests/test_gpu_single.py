"""The plain single-precision path (LJMD_FP32: positions and velocities as
single floats, the paper's GPU precision) through the C ABI.

* Free flight (eps = 0): every step is x <- fl(x + fl(dt v)) with the wrap
  x -= L in floats, so the GPU walk equals, bit for bit, the same binary32
  recurrence done by numpy; and it is far from the closed form, where the
  double-single path stays within 1e-9 (the negative control of the
  double-single state).
* Lists and forces of the rounded positions: the lists equal the oracle's
  stated FP32 sequence and the forces the oracle's forces of the fixed-point
  positions, as for the double-single path.
* A 100-step trajectory against the FP64 oracle.
"""
import numpy as np
import pytest

import oracle
from force_metrics import bound_key, force_errors, reference, report, tie_allowance
from paper_2406_04210_amd import workloads as W

pytestmark = pytest.mark.gpu
FP32_PLAIN, FP32_DS = 2, 1


@pytest.fixture(scope="module")
def ljmd():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2406_04210_amd import ljmd as L
    return L


def test_plain_free_flight_is_the_binary32_recurrence(ljmd):
    w = W.config_small()
    p = w.params.copy()
    p.eps[:] = 0.0
    nsteps = 3000
    s = ljmd.System(w.n, w.box, p, precision=FP32_PLAIN, sort_interval=0)
    s.set_state(w.x, w.v, w.species)
    s.run(nsteps, observe=False)
    x, _, img = s.get_state()
    s.sync()
    x, img = x.cpu().numpy(), img.cpu().numpy()
    L = np.float32(w.box[0])
    xf = w.x.astype(np.float32)
    vf = w.v.astype(np.float32)
    im = np.zeros(xf.shape, np.int64)
    dt = np.float32(p.dt)
    for _ in range(nsteps):
        xf = (xf + (dt * vf).astype(np.float32)).astype(np.float32)
        lo, hi = xf < 0, xf >= L
        xf = np.where(lo, xf + L, np.where(hi, xf - L, xf)).astype(np.float32)
        im += hi.astype(np.int64) - lo.astype(np.int64)
        again = xf >= L
        xf = np.where(again, xf - L, xf).astype(np.float32)
    assert np.array_equal(x, xf.astype(np.float64))
    assert np.array_equal(img, im)
    want = w.x + nsteps * p.dt * w.v
    err_plain = np.abs(x + img * w.box - want).max()
    s2 = ljmd.System(w.n, w.box, p, precision=FP32_DS, sort_interval=0)
    s2.set_state(w.x, w.v, w.species)
    s2.run(nsteps, observe=False)
    err_ds = np.abs(s2.unwrapped_positions().cpu().numpy() - want).max()
    print(f"free flight {nsteps} steps: plain FP32 err {err_plain:.3e}, double-single err {err_ds:.3e}", flush=True)
    assert err_ds < 1e-9 and err_plain > 1000 * err_ds


@pytest.mark.parametrize("nspecies", [1, 2])
def test_plain_lists_and_forces(ljmd, nspecies):
    if nspecies == 1:
        x, L = W.fcc_lattice(8, 0.8442)
        x = x + 0.1 * np.random.default_rng(3).standard_normal(x.shape)
        box, sp, p = np.full(3, L), np.zeros(len(x), np.int32), W.single_species_params()
    else:
        r = W.random_dense(1500, 1.1, seed=7, nspecies=2, min_dist=0.75)
        x, box, sp, p = r.x, r.box, r.species, r.params
    s = ljmd.System(len(x), box, p, precision=FP32_PLAIN)
    s.set_state(x, np.zeros_like(x), sp)
    f = s.forces().cpu().numpy()
    xg, _, _ = s.get_state()
    cnt, ids = s.neighbors(cap=256)
    s.sync()
    xr = xg.cpu().numpy()                      # the float positions the path holds
    assert np.array_equal(xr, xr.astype(np.float32).astype(np.float64))
    cnt, ids = cnt.cpu().numpy(), ids.cpu().numpy()
    oc, on = oracle.build_lists(xr, sp, box, p, mode=1)
    assert np.array_equal(cnt, oc)
    for i in range(0, len(xr), 7):
        assert set(ids[i, :cnt[i]].tolist()) == set(on[i, :oc[i]].tolist())
    ref, _, _, A = reference(xr, sp, box, p, 1)
    m = report(f"plain fp32 nspecies={nspecies}", force_errors(f, ref, A, tie_allowance(xr, sp, box, p, 1)))
    assert m[bound_key(1)] <= 1e-5


def test_plain_trajectory_against_oracle(ljmd):
    w = W.config_small()
    s = ljmd.System(w.n, w.box, w.params, precision=FP32_PLAIN, sort_interval=25)
    s.set_state(w.x, w.v, w.species)
    obs = s.run(100).cpu().numpy()
    s.sync()
    xu = s.unwrapped_positions().cpu().numpy()
    r = oracle.run_nve(w.x, w.v, w.species, w.box, w.params, 100)
    dx = np.abs(xu - r["x"]).max()
    dE = np.abs((obs[:, 0] + obs[:, 1]) - (r["obs"][1:, 0] + r["obs"][1:, 1])).max() / w.n
    print(f"plain fp32 100 steps: max|dx| {dx:.3e}, max|dE|/N {dE:.3e}", flush=True)
    assert dx <= 2e-4 and dE <= 1e-4
