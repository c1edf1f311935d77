"""Batched systems (replicas of uneven size stepped together) through the
C ABI: every system of a batch follows exactly the trajectory it has as a
single box (the batch is a memory layout, not an approximation), and its
forces match the oracle.

Expected values: the single-box path of this library for the bitwise
comparison (itself pinned to the oracle by test_gpu_parity.py), and the
oracle for the forces (FP32 tolerance as in test_gpu_parity.py).
"""
import math

import numpy as np
import pytest

import oracle
from paper_2406_04210_amd import workloads as W
from force_metrics import bound_key, force_errors, reference, report, tie_allowance

pytestmark = pytest.mark.gpu
FP32 = 1


@pytest.fixture(scope="module")
def ljmd():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2406_04210_amd import ljmd as L
    return L


@pytest.fixture(scope="module")
def replicas():
    # A seeded subset of the replica draws: uneven N (500 .. 32000), rho in
    # [0.7, 1.2], T in [0.7, 1.5]; the smallest boxes have two cells per axis.
    return W.replica_draws(nrep=7)


def concat(ws):
    x = np.concatenate([w.x for w in ws])
    v = np.concatenate([w.v for w in ws])
    sp = np.concatenate([w.species for w in ws])
    return x, v, sp


def make_batch(ljmd, ws, **kw):
    b = ljmd.Batch([w.n for w in ws], [w.box[0] for w in ws], ws[0].params, **kw)
    b.set_state(*concat(ws))
    return b


@pytest.mark.parametrize("cell_split", [1, 2])
def test_batch_matches_single_boxes_bitwise(ljmd, replicas, cell_split):
    import torch
    ws = replicas
    b = make_batch(ljmd, ws, sort_interval=50, cell_split=cell_split)
    b.run(60)
    b.run(75)                       # crosses resorts at steps 50 and 100
    xb, vb, ib = b.get_state()
    fb = b.forces()
    ob = b.observables()
    b.sync()
    off = np.concatenate([[0], np.cumsum([w.n for w in ws])])
    for k, w in enumerate(ws):
        s = ljmd.System(w.n, w.box, w.params, precision=FP32, sort_interval=50, cell_split=cell_split)
        s.set_state(w.x, w.v, w.species)
        s.run(60, observe=False)
        s.run(75, observe=False)
        x, v, img = s.get_state()
        f = s.forces()
        o = s.observables()
        s.sync()
        sl = slice(off[k], off[k + 1])
        assert torch.equal(x, xb[sl]), (k, w.name)
        assert torch.equal(v, vb[sl]), (k, w.name)
        assert torch.equal(img, ib[sl]), (k, w.name)
        assert torch.equal(f, fb[sl]), (k, w.name)
        # Observables: the same FP64 reduction order per system.
        assert ob[k, 0] == o["U"] and ob[k, 1] == o["K"] and ob[k, 2] == o["W"], (k, ob[k], o)
        assert int(ob[k, 6]) == o["rebuilds"] and int(ob[k, 7]) == o["step"] == 135


def batch_snapshot(b):
    x, v, img = b.get_state()
    f = b.forces()
    o = b.observables()
    b.sync()
    return x, v, img, f, o


@pytest.mark.parametrize("sort_interval,runs", [(20, (70, 55, 41)), (15, (100, 61))])
def test_batch_graph_replay_matches_eager_bitwise(ljmd, replicas, sort_interval, runs):
    # Whole resort periods (20 steps; 30 for the odd interval 15) replay a
    # captured graph; the eager batch launches every step. After every run
    # (graph replays, eager steps and host synchronisation in between) both
    # hold bitwise the same state, forces and observables.
    import torch
    ws = replicas[:5]
    a = make_batch(ljmd, ws, sort_interval=sort_interval)
    e = make_batch(ljmd, ws, sort_interval=sort_interval)
    e.use_graphs(False)
    for n in runs:
        a.run(n)
        e.run(n)
        sa, se = batch_snapshot(a), batch_snapshot(e)
        for k in range(4):
            assert torch.equal(sa[k], se[k]), (n, k)
        assert np.array_equal(sa[4], se[4]), n


def test_batch_forces_match_oracle(ljmd, replicas):
    ws = replicas[:4]
    b = make_batch(ljmd, ws)
    f = b.forces().cpu().numpy()
    b.sync()
    off = np.concatenate([[0], np.cumsum([w.n for w in ws])])
    for k, w in enumerate(ws):
        # The FP32 bound of test_gpu_parity.py: 1e-5 of the rms force against
        # the oracle's forces of the fixed-point positions, after the tie
        # allowance (lattice-with-vacancy states can hold cutoff ties).
        ref, _, _, A = reference(w.x, w.species, w.box, w.params, FP32)
        m = report(f"batch replica {k} {w.name}",
                   force_errors(f[off[k]:off[k + 1]], ref, A, tie_allowance(w.x, w.species, w.box, w.params, FP32)))
        assert m[bound_key(1)] <= 1e-5, (k, m)


def test_batch_rejects_small_box(ljmd):
    p = W.single_species_params()
    with pytest.raises(ljmd.LJMDError):
        ljmd.Batch([500, 500], [7.5, 4.0], p)      # 4.0 < 2 (r_c + skin)


def test_full_batch_sampled_systems(ljmd):
    # The 512-replica workload at full size (sum N about 3.9 million), in the
    # bench's launch configuration: 120 steps (a graph-replayed resort period
    # and eager steps, list builds from per-XCD cell queues), then sampled
    # systems against single-box runs (bitwise) and the oracle (forces).
    import torch
    ws = W.replica_draws(512)
    b = make_batch(ljmd, ws, sort_interval=100)
    b.run(120)
    xb, vb, ib = b.get_state()
    fb = b.forces()
    b.sync()
    off = np.concatenate([[0], np.cumsum([w.n for w in ws])])
    rng = np.random.default_rng(4)
    for k in rng.choice(len(ws), 3, replace=False):
        w = ws[k]
        s = ljmd.System(w.n, w.box, w.params, precision=FP32, sort_interval=100)
        s.set_state(w.x, w.v, w.species)
        s.run(120, observe=False)
        x, v, img = s.get_state()
        f = s.forces()
        s.sync()
        sl = slice(off[k], off[k + 1])
        assert torch.equal(x, xb[sl]) and torch.equal(v, vb[sl]) and torch.equal(f, fb[sl]), (k, w.name)
    fh = fb.cpu().numpy()
    xh = xb.cpu().numpy()
    for k in rng.choice(len(ws), 6, replace=False):
        w = ws[k]
        sl = slice(off[k], off[k + 1])
        ref, _, _, A = reference(xh[sl], w.species, w.box, w.params, FP32)
        # The FP32 bound of test_gpu_parity.py (1e-5 of the rms force against
        # the fixed-point positions' forces, ties allowed for).
        m = report(f"full batch replica {k} {w.name}",
                   force_errors(fh[sl], ref, A, tie_allowance(xh[sl], w.species, w.box, w.params, FP32)))
        assert m[bound_key(1)] <= 1e-5, (k, w.name, m)


def test_many_systems_plan_searched_in_global_memory(ljmd):
    # 700 small replicas: every system rebuilds on the first step, so the
    # rebuild plan holds more systems than the list-build kernels stage in
    # LDS (512) and they search it in global memory instead. Sampled systems
    # (the first, the last and two drawn) against single-box runs (bitwise,
    # rebuild counts included) and two against the oracle (forces).
    import torch
    ws = W.replica_draws(700, nmin=500, nmax=1500)
    b = make_batch(ljmd, ws, sort_interval=25)
    b.run(40)
    xb, vb, ib = b.get_state()
    fb = b.forces()
    ob = b.observables()
    b.sync()
    assert int(ob[:, 6].min()) >= 1
    off = np.concatenate([[0], np.cumsum([w.n for w in ws])])
    rng = np.random.default_rng(6)
    picks = [0, len(ws) - 1] + [int(k) for k in rng.choice(np.arange(1, len(ws) - 1), 2, replace=False)]
    for k in picks:
        w = ws[k]
        s = ljmd.System(w.n, w.box, w.params, precision=FP32, sort_interval=25)
        s.set_state(w.x, w.v, w.species)
        s.run(40, observe=False)
        x, v, img = s.get_state()
        f = s.forces()
        o = s.observables()
        s.sync()
        sl = slice(off[k], off[k + 1])
        assert torch.equal(x, xb[sl]) and torch.equal(v, vb[sl]), (k, w.name)
        assert torch.equal(img, ib[sl]) and torch.equal(f, fb[sl]), (k, w.name)
        assert int(ob[k, 6]) == o["rebuilds"] and int(ob[k, 7]) == o["step"] == 40, (k, ob[k], o)
    fh = fb.cpu().numpy()
    xh = xb.cpu().numpy()
    for k in picks[2:]:
        w = ws[k]
        sl = slice(off[k], off[k + 1])
        ref, _, _, A = reference(xh[sl], w.species, w.box, w.params, FP32)
        m = report(f"many-system batch replica {k} {w.name}",
                   force_errors(fh[sl], ref, A, tie_allowance(xh[sl], w.species, w.box, w.params, FP32)))
        assert m[bound_key(1)] <= 1e-5, (k, w.name, m)
