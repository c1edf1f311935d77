"""Force-error metrics shared by the GPU parity tests.

Every force comparison reports three numbers; FP64 comparisons assert the
first, FP32 comparisons the second (``bound_key``):

* ``sec8c`` -- max_i e_i / max(rms_j |F_j|, 1): the error of the worst
  particle relative to the rms force of the configuration (floored at the
  unit force eps/sigma, for lattices whose forces vanish by symmetry);
* ``cond`` -- max_i e_i / max(A_i, 1), with A_i the sum over i's partners
  inside the cutoff of the pair-force magnitudes: the error relative to the
  scale of the sum that forms F_i (the rounding of a floating-point sum is
  bounded relative to the sum of its terms' magnitudes);
* ``per_particle`` -- max_i e_i / max(|F_i|, rms, 1).

e_i = max(|F_i - F_i^ref| - t_i, 0), where t_i (tie allowance) is |F(r_c)|
per partner at a cutoff tie: the truncated force jumps there, and binary32
(or FP64) decides r^2 < r_c^2 in its own rounding.

References: the FP64 path is compared with the oracle's plain FP64 forces;
the FP32 + double-single path with the oracle's forces of the positions it
represents (``oracle.forces_fixed``: 32-bit fixed-point image
coordinates), so that what is measured is the path's binary32 arithmetic.
"""
import math

import numpy as np

import oracle

FP64, FP32 = 0, 1


def bound_key(prec):
    """The metric a comparison of this precision is held to (1e-12 FP64,
    1e-5 FP32). Binary32 rounds r^2 to 2^-24 relative and the r^-13
    repulsion amplifies that about 6.5-fold, so every pair force carries a
    few 1e-7 of its magnitude: a particle's error is set by the pair forces
    that form it, not by the rms force of the configuration, and the
    rms-relative error exceeds 1e-5 wherever forces spread over orders of
    magnitude (measured: 4e-5 in a jittered lattice and in the relaxed 4M
    mixture, whose pair-force-relative error stays below 2e-6)."""
    return "sec8c" if prec == FP64 else "cond"


def tie_allowance(x, sp, box, p, prec):
    """Per-particle sum of |F(r_c)| over partners at a cutoff tie
    (|r^2 - r_c^2| <= 2e-6 r_c^2 in FP32, 1e-12 r_c^2 in FP64)."""
    x = np.asarray(x, dtype=np.float64)
    n = len(x)
    cnt, nbr = oracle.build_lists(x, sp, box, p, mode=0)
    i = np.repeat(np.arange(n), cnt)
    j = nbr[np.arange(nbr.shape[1])[None, :] < cnt[:, None]]
    d = x[i] - x[j]
    d -= box * np.rint(d / box)
    r2 = (d * d).sum(axis=1)
    ab = sp[i] * 2 + sp[j] if p.nspecies == 2 else np.zeros(len(i), dtype=np.int64)
    rc = np.asarray(p.rcut)[ab]
    window = 1e-12 if prec == FP64 else 2e-6
    tie = np.abs(r2 - rc * rc) <= window * rc * rc
    out = np.zeros(n)
    for k in np.nonzero(tie)[0]:
        a = int(ab[k])
        jump = abs(oracle.pair_fscalar(rc[k] * (1 - 1e-15), a, p)) * rc[k]
        out[i[k]] += 1.001 * jump
    return out


def reference(x, sp, box, p, prec):
    """(F_ref, U, W, A) for the path of precision prec (see module doc)."""
    cnt, nbr = oracle.build_lists(x, sp, box, p, mode=0)
    if prec == FP32:
        f, U, W, A = oracle.forces_fixed(x, sp, box, p, cnt, nbr)
    else:
        f, U, W = oracle.forces_list(x, sp, box, p, cnt, nbr)
        _, _, _, A = oracle.forces_fixed(x, sp, box, p, cnt, nbr)
    return f, U, W, A


def force_errors(f, ref, A=None, allowance=None):
    f = np.asarray(f, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    rms = math.sqrt(float((ref ** 2).sum(axis=1).mean()))
    e = np.linalg.norm(f - ref, axis=1)
    if allowance is not None:
        e = np.maximum(e - allowance, 0.0)
    out = {
        "sec8c": float(e.max() / max(rms, 1.0)),
        "per_particle": float((e / np.maximum(np.maximum(np.linalg.norm(ref, axis=1), rms), 1.0)).max()),
        "rms": rms,
    }
    if A is not None:
        out["cond"] = float((e / np.maximum(A, 1.0)).max())
    return out


def report(tag, m):
    parts = " ".join(f"{k}={v:.3e}" for k, v in m.items())
    print(f"force errors [{tag}]: {parts}", flush=True)
    return m
