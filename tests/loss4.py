"""The differentiable workload's loss, evaluated and differentiated by the
oracle only (test infrastructure shared by the CPU pin and the GPU parity
test of the full loss).

  L(x0, v0, eps, sigma) = |F(x0; th) - F*|^2 / (3N) + U(x_K; th) / N,

K velocity-Verlet steps from (x0, v0); F* = F(x0; th*) is target data,
computed once and held fixed under differentiation; the cutoff is a fixed
length. Gradient: force VJP of the matching term at x0, plus the adjoint of
the rollout seeded with dU/dx_K = -F(x_K) and dU/dv_K = 0, plus dU/dth at
x_K.
"""
import numpy as np

import oracle


def theta_params(p, eps, sig):
    return oracle.with_params(p, eps=[eps] * 3, sigma=[sig] * 3)


def loss(x0, v0, sp, box, p, eps, sig, f_star, nsteps, want_sig=False):
    q = theta_params(p, eps, sig)
    n = len(x0)
    f0, _, _ = oracle.forces(x0, sp, box, q)
    r = oracle.run_nve(x0, v0, sp, box, q, nsteps, want_obs=True, want_sig=want_sig)
    val = ((f0 - f_star) ** 2).sum() / (3 * n) + r["obs"][-1, 0] / n
    return val, r["sig"]


def grad(x0, v0, sp, box, p, eps, sig, f_star, nsteps):
    """(dL/dx0, dL/dv0, dL/deps, dL/dsigma)."""
    q = theta_params(p, eps, sig)
    n = len(x0)
    f0, _, _ = oracle.forces(x0, sp, box, q)
    gF = 2.0 * (f0 - f_star) / (3 * n)
    gx_a, ge_a, gs_a = oracle.force_vjp(x0, sp, box, q, gF)
    r = oracle.run_nve(x0, v0, sp, box, q, nsteps, want_obs=False)
    lam_x = -r["f"] / n
    lx, lv, ge_r, gs_r = oracle.vv_adjoint(x0, v0, sp, box, q, nsteps, lam_x, np.zeros_like(lam_x))
    ue, us = oracle.energy_grad(r["x"], sp, box, q)
    return gx_a + lx, lv, ge_a[0] + ge_r[0] + ue[0] / n, gs_a[0] + gs_r[0] + us[0] / n


def fd_directional(x0, v0, sp, box, p, eps, sig, f_star, nsteps, dx, dv, de, ds, h, rng, tries=8):
    """Central difference of L along (dx, dv, de, ds) with step h, taken only
    when the +h and -h runs have the same pairs inside the cutoff at every
    step (the truncated force jumps at r_c); otherwise the direction is
    redrawn (same distribution) up to `tries` times. Returns (fd, dx, dv, de, ds)."""
    for _ in range(tries):
        lp, sp_ = loss(x0 + h * dx, v0 + h * dv, sp, box, p, eps + h * de, sig + h * ds, f_star, nsteps, True)
        lm, sm_ = loss(x0 - h * dx, v0 - h * dv, sp, box, p, eps - h * de, sig - h * ds, f_star, nsteps, True)
        if np.array_equal(sp_, sm_):
            return (lp - lm) / (2 * h), dx, dv, de, ds
        dx, dv = rng.standard_normal(dx.shape), rng.standard_normal(dv.shape)
        de, ds = float(rng.standard_normal()), float(rng.standard_normal())
    raise RuntimeError("every direction crossed the cutoff")
