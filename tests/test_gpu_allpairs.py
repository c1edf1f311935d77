"""The untruncated all-pairs interaction (infinite cutoffs: every pair of
the minimum image, plain 12-6 potential, no shift) on the GPU against the
oracle's brute force, through the C ABI. Tolerances as for the truncated
path: forces 1e-12 (FP64) and 1e-5 (FP32 paths, against the oracle's forces
of the fixed-point positions) of the rms force; U and W 1e-12 / 5e-6;
100-step trajectories 1e-10 / 1e-4.
"""
import numpy as np
import pytest

import oracle
from force_metrics import bound_key, force_errors, reference, report
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


def cases():
    w = W.all_pairs_fluid()
    out = [("fluid2000", w.x, w.v, w.species, w.box, w.params)]
    r = W.random_dense(777, 0.8442, seed=15)
    p = r.params.copy()
    p.rcut = np.full(4, np.inf)
    out.append(("random777", r.x, r.v, r.species, r.box, p))
    r = W.random_dense(900, 1.0, seed=16, nspecies=2, min_dist=0.8)
    p = r.params.copy()
    p.rcut = np.full(4, np.inf)
    out.append(("mixture900", r.x, r.v, r.species, r.box, p))
    # More partners than one LDS chunk of records holds in either precision.
    w = W.all_pairs_fluid(n=4500, seed_index=3)
    out.append(("fluid4500", w.x, w.v, w.species, w.box, w.params))
    return out


CASES = cases()


@pytest.mark.parametrize("prec", [FP64, FP32_DS, FP32])
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_all_pairs_forces_energy_virial(ljmd, case, prec):
    name, x, v, sp, box, p = case
    s = ljmd.System(len(x), box, p, precision=prec)
    s.set_state(x, v, sp)
    f = s.forces().cpu().numpy()
    o = s.observables()
    xg, _, _ = s.get_state()
    s.sync()
    xr = xg.cpu().numpy() if prec == FP32 else x        # plain FP32 holds rounded positions
    ref, U, Wv, A = reference(xr, sp, box, p, FP64 if prec == FP64 else 1)
    fb, Ub, Wb = oracle.forces_brute(xr, sp, box, p)
    if prec == FP64:
        assert np.abs(ref - fb).max() <= 1e-12 * np.abs(fb).max()
    m = report(f"all pairs {name} prec={prec}", force_errors(f, ref, A))
    assert m[bound_key(FP64 if prec == FP64 else 1)] <= TOL_F[prec]
    eu, ew = abs(o["U"] - U) / abs(U), abs(o["W"] - Wv) / abs(Wv)
    print(f"all pairs {name} prec={prec}: U rel {eu:.3e} W rel {ew:.3e}", flush=True)
    assert eu <= TOL_E[prec] and ew <= TOL_E[prec]


@pytest.mark.parametrize("prec", [FP64, FP32_DS])
def test_all_pairs_trajectory(ljmd, prec):
    w = W.all_pairs_fluid()
    s = ljmd.System(w.n, w.box, w.params, precision=prec)
    s.set_state(w.x, w.v, w.species)
    obs = s.run(100).cpu().numpy()
    s.sync()
    xu = s.unwrapped_positions().cpu().numpy()
    r = oracle.run_nve(w.x, w.v, w.species, w.box, w.params, 100)
    dx = np.abs(xu - r["x"]).max()
    dU = np.abs(obs[:, 0] - r["obs"][1:, 0]).max() / w.n
    print(f"all pairs trajectory prec={prec}: max|dx| {dx:.3e} max|dU|/N {dU:.3e}", flush=True)
    assert dx <= (1e-10 if prec == FP64 else 1e-4)
    assert dU <= (1e-10 if prec == FP64 else 1e-5)
    # FP32 sums ~2,000 pair forces per particle, each with a few 1e-7 of its
    # magnitude: the total momentum drifts by that much per particle.
    assert np.abs(obs[:, 3:6]).max() < (1e-10 if prec == FP64 else 1e-5 * w.n)


def test_all_pairs_with_thermostat(ljmd):
    # The paper's all-to-all setup: velocity Verlet with the Andersen-like thermostat.
    w = W.all_pairs_fluid()
    thermo = (1.2, 5.0, 31)
    s = ljmd.System(w.n, w.box, w.params, precision=FP64)
    s.set_state(w.x, w.v, w.species)
    s.set_thermostat(*thermo)
    s.run(60, observe=False)
    s.sync()
    xu = s.unwrapped_positions().cpu().numpy()
    r = oracle.run_nve(w.x, w.v, w.species, w.box, w.params, 60, thermostat=thermo)
    assert np.abs(xu - r["x"]).max() <= 1e-10


def test_all_pairs_rejects_list_calls(ljmd):
    w = W.all_pairs_fluid()
    s = ljmd.System(w.n, w.box, w.params, precision=FP64)
    s.set_state(w.x, w.v, w.species)
    for call in (lambda: s.neighbors(), lambda: s.minimize_sd(2), lambda: s.vv_forward(2, 1),
                 lambda: s.energy_grad()):
        with pytest.raises(ljmd.LJMDError):
            call()
