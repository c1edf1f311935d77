"""Pins of the oracle's adjoint (force VJP, parameter gradients, velocity-
Verlet adjoint) against finite differences, symmetries and exact identities.

The force VJP is (dF/dx)^T g, and dF/dx = -Hessian is symmetric; the force
and the energy are homogeneous of degree one in eps; with a fixed cutoff
length the energy obeys sigma dU/dsigma = W + n_c r_c phi'(r_c) (a scaling
identity). Finite differences are taken where no pair crosses the cutoff
(checked), because the truncated force jumps there.
"""
import numpy as np
import pytest

import oracle
from paper_2406_04210_amd import workloads as W


def jittered(m, amp, seed, rho=0.8442):
    x, L = W.fcc_lattice(m, rho)
    rng = np.random.default_rng(seed)
    return x + amp * rng.standard_normal(x.shape), np.full(3, L)


def pair_distances(x, box, p, sp):
    cnt, nbr = oracle.build_lists(x, sp, box, p)
    n = len(x)
    i = np.repeat(np.arange(n), cnt)
    j = nbr[np.arange(nbr.shape[1])[None, :] < cnt[:, None]]
    d = x[i] - x[j]
    d -= box * np.rint(d / box)
    return np.sqrt((d * d).sum(1)), i, j


def no_cutoff_crossing(x, box, p, sp, h, dlt):
    """No pair distance can cross its cutoff between x - h dlt and x + h dlt
    (|dr| <= h (|dlt_i| + |dlt_j|))."""
    r, i, j = pair_distances(x, box, p, sp)
    nrm = np.linalg.norm(dlt, axis=1)
    ab = sp[i] * 2 + sp[j] if p.nspecies == 2 else np.zeros(len(i), dtype=np.int64)
    rc = np.asarray(p.rcut)[ab]
    return bool(np.all(np.abs(r - rc) > h * (nrm[i] + nrm[j])))


@pytest.mark.parametrize("nspecies", [1, 2])
def test_force_vjp_matches_directional_fd(nspecies):
    if nspecies == 1:
        x, box = jittered(5, 0.06, 1)
        sp = np.zeros(len(x), np.int32)
        p = W.single_species_params()
    else:
        w = W.random_dense(400, 1.0, seed=2, nspecies=2, min_dist=0.8)
        x, box, sp, p = w.x, w.box, w.species, w.params
    rng = np.random.default_rng(3)
    g = rng.standard_normal(x.shape)
    gx, _, _ = oracle.force_vjp(x, sp, box, p, g)
    h = 1e-6
    done = 0
    while done < 3:
        dlt = rng.standard_normal(x.shape)
        if not no_cutoff_crossing(x, box, p, sp, h, dlt):
            continue
        done += 1
        fp, _, _ = oracle.forces_brute(x + h * dlt, sp, box, p)
        fm, _, _ = oracle.forces_brute(x - h * dlt, sp, box, p)
        fd = (g * (fp - fm)).sum() / (2 * h)
        assert (gx * dlt).sum() == pytest.approx(fd, rel=1e-7)


def test_force_vjp_symmetry_and_translation():
    x, box = jittered(5, 0.06, 4)
    sp = np.zeros(len(x), np.int32)
    p = W.single_species_params()
    rng = np.random.default_rng(5)
    u, v = rng.standard_normal(x.shape), rng.standard_normal(x.shape)
    hu, _, _ = oracle.force_vjp(x, sp, box, p, u)
    hv, _, _ = oracle.force_vjp(x, sp, box, p, v)
    assert (hu * v).sum() == pytest.approx((hv * u).sum(), rel=1e-12)
    # A uniform translation is a zero mode of the Hessian.
    ht, _, _ = oracle.force_vjp(x, sp, box, p, np.tile([0.3, -1.2, 0.7], (len(x), 1)))
    assert np.abs(ht).max() < 1e-10


def test_parameter_gradients_identities_and_fd():
    x, box = jittered(6, 0.05, 6)
    sp = np.zeros(len(x), np.int32)
    p = W.single_species_params()
    rng = np.random.default_rng(7)
    g = rng.standard_normal(x.shape)
    f, U, Wv = oracle.forces_brute(x, sp, box, p)
    _, ge, gs = oracle.force_vjp(x, sp, box, p, g)
    ue, us = oracle.energy_grad(x, sp, box, p)
    # Homogeneity in eps.
    assert 1.0 * ge[0] == pytest.approx((g * f).sum(), rel=1e-12)
    assert 1.0 * ue[0] == pytest.approx(U, rel=1e-12)
    # sigma dU/dsigma = W + n_c r_c phi'(r_c) (fixed cutoff length).
    r, _, _ = pair_distances(x, box, p, sp)
    nc = int((r < p.rcut[0]).sum()) // 2
    rc = p.rcut[0]
    dphi_rc = -rc * oracle.fscalar(rc)
    assert 1.0 * us[0] == pytest.approx(Wv + nc * rc * dphi_rc, rel=1e-11)
    # Central differences in eps and sigma.
    for k, grad_f, grad_u in (("eps", ge[0], ue[0]), ("sigma", gs[0], us[0])):
        h = 1e-6
        pp = oracle.with_params(p, **{k: 1.0 + h})
        pm = oracle.with_params(p, **{k: 1.0 - h})
        fp, Up, _ = oracle.forces_brute(x, sp, box, pp)
        fm, Um, _ = oracle.forces_brute(x, sp, box, pm)
        assert grad_f == pytest.approx((g * (fp - fm)).sum() / (2 * h), rel=1e-7)
        assert grad_u == pytest.approx((Up - Um) / (2 * h), rel=1e-7)


def test_mixture_parameter_gradients_fd():
    w = W.random_dense(500, 1.0, seed=8, nspecies=2, min_dist=0.8)
    x, box, sp, p = w.x, w.box, w.species, w.params
    rng = np.random.default_rng(9)
    g = rng.standard_normal(x.shape)
    _, ge, gs = oracle.force_vjp(x, sp, box, p, g)
    ue, us = oracle.energy_grad(x, sp, box, p)
    base_e = np.array([p.eps[0], p.eps[1], p.eps[3]])
    base_s = np.array([p.sigma[0], p.sigma[1], p.sigma[3]])
    h = 1e-6
    for t in range(3):
        for name, base, gf, gu in (("eps", base_e, ge, ue), ("sigma", base_s, gs, us)):
            up, dn = base.copy(), base.copy()
            up[t] += h
            dn[t] -= h
            fp, Up, _ = oracle.forces_brute(x, sp, box, oracle.with_params(p, **{name: up}))
            fm, Um, _ = oracle.forces_brute(x, sp, box, oracle.with_params(p, **{name: dn}))
            assert gf[t] == pytest.approx((g * (fp - fm)).sum() / (2 * h), rel=2e-6, abs=1e-6)
            assert gu[t] == pytest.approx((Up - Um) / (2 * h), rel=2e-6, abs=1e-6)


def rollout_loss(x0, v0, sp, box, p, nsteps, gU, gX):
    """A linear functional of the final state: <gX, x_N> + <gU, v_N>."""
    r = oracle.run_nve(x0, v0, sp, box, p, nsteps, want_obs=False)
    return (gX * r["x"]).sum() + (gU * r["v"]).sum()


def test_vv_adjoint_matches_tangent_fd():
    x0, box = jittered(5, 0.04, 10)
    sp = np.zeros(len(x0), np.int32)
    p = W.single_species_params()
    rng = np.random.default_rng(11)
    v0 = W.maxwell_boltzmann(len(x0), 0.5, p.mass, sp, rng)
    nsteps = 12
    gX, gV = rng.standard_normal(x0.shape), rng.standard_normal(x0.shape)
    lx, lv, ge, gs = oracle.vv_adjoint(x0, v0, sp, box, p, nsteps, gX, gV)
    h = 1e-7
    for _ in range(2):
        dx, dv = rng.standard_normal(x0.shape), rng.standard_normal(x0.shape)
        fd = (rollout_loss(x0 + h * dx, v0 + h * dv, sp, box, p, nsteps, gV, gX)
              - rollout_loss(x0 - h * dx, v0 - h * dv, sp, box, p, nsteps, gV, gX)) / (2 * h)
        fd2 = (rollout_loss(x0 + 2 * h * dx, v0 + 2 * h * dv, sp, box, p, nsteps, gV, gX)
               - rollout_loss(x0 - 2 * h * dx, v0 - 2 * h * dv, sp, box, p, nsteps, gV, gX)) / (4 * h)
        assert fd == pytest.approx(fd2, rel=1e-5)      # no cutoff crossing between the runs
        assert (lx * dx).sum() + (lv * dv).sum() == pytest.approx(fd, rel=1e-6)
    # Parameter gradient of the rollout by central differences in eps and sigma.
    for name, gth in (("eps", ge[0]), ("sigma", gs[0])):
        hp = 1e-6
        Lp = rollout_loss(x0, v0, sp, box, oracle.with_params(p, **{name: 1 + hp}), nsteps, gV, gX)
        Lm = rollout_loss(x0, v0, sp, box, oracle.with_params(p, **{name: 1 - hp}), nsteps, gV, gX)
        assert gth == pytest.approx((Lp - Lm) / (2 * hp), rel=1e-5)


def test_full_loss_gradient_matches_fd_n2048():
    # The differentiable workload at the size named for its finite-difference
    # check: jittered FCC 8^3 (N = 2048), 50 velocity-Verlet steps, target
    # parameters within 5 %. The oracle's gradient (force VJP + rollout
    # adjoint + energy gradient) against central differences of the loss
    # along seeded directions in (x0, v0, eps, sigma), FP64, with a step h
    # at which no pair changes side of its cutoff in any of the 51 frames
    # (checked by the cutoff signature of both runs).
    import loss4
    w, eps_t, sig_t = W.jittered_fcc(8)
    nsteps = 50
    p = w.params
    f_star, _, _ = oracle.forces(w.x, w.species, w.box, oracle.with_params(p, eps=[eps_t[0]] * 3,
                                                                          sigma=[sig_t[0]] * 3))
    gx, gv, ge, gs = loss4.grad(w.x, w.v, w.species, w.box, p, 1.0, 1.0, f_star, nsteps)
    rng = np.random.default_rng(2048)
    for _ in range(2):
        dx, dv = rng.standard_normal(w.x.shape), rng.standard_normal(w.x.shape)
        de, ds = float(rng.standard_normal()), float(rng.standard_normal())
        fd, dx, dv, de, ds = loss4.fd_directional(w.x, w.v, w.species, w.box, p, 1.0, 1.0, f_star, nsteps,
                                                  dx, dv, de, ds, 1e-8, rng)
        an = (gx * dx).sum() + (gv * dv).sum() + ge * de + gs * ds
        assert an == pytest.approx(fd, rel=1e-6)
