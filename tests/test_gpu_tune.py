"""The autotuner through the C ABI: it times every cell size (cells of edge
>= r_L or >= r_L / 2) and force-gather shape on the device, returns the
fastest pair with a list capacity above the longest list seen, caches the
result and reads it back; a system built with the tuned cell size, shape and
capacity gives the forces of the oracle."""
import pytest

import oracle
from paper_2406_04210_amd import workloads as W
from force_metrics import bound_key, force_errors, reference, report, tie_allowance

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ljmd():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2406_04210_amd import ljmd as L
    return L


def test_autotune_times_caches_and_runs(ljmd, tmp_path):
    w = W.config_small()
    cache = str(tmp_path / "tune.jsonl")
    t = ljmd.autotune(w.n, w.box, w.params, w.x, w.v, w.species, steps=10, cache_path=cache)
    print("tuned", t, flush=True)
    assert t["lanes"] in (1, 2, 4, 8, 16) and t["cell_split"] in (1, 2)
    assert t["ms_per_step"] > 0.0 and not t["from_cache"]
    assert t["max_fill"] > 0 and t["nbr_capacity"] >= t["max_fill"] + 16 and t["nbr_capacity"] % 16 == 0
    again = ljmd.autotune(w.n, w.box, w.params, w.x, w.v, w.species, steps=10, cache_path=cache)
    assert again["from_cache"]
    assert {k: again[k] for k in ("lanes", "cell_split", "nbr_capacity", "max_fill")} == \
           {k: t[k] for k in ("lanes", "cell_split", "nbr_capacity", "max_fill")}
    with open(cache) as fh:
        assert len(fh.readlines()) == 1
    s = ljmd.System(w.n, w.box, w.params, lanes=t["lanes"], nbr_capacity=t["nbr_capacity"],
                    cell_split=t["cell_split"])
    s.set_state(w.x, w.v, w.species)
    s.run(50, observe=False)
    s.sync()
    x, v, _ = s.get_state()
    f = s.forces().cpu().numpy()
    xh = x.cpu().numpy()
    ref, _, _, A = reference(xh, w.species, w.box, w.params, 1)
    # Forces of the state the GPU reached, to the FP32 tolerance of
    # test_gpu_parity.py (with its allowance at cutoff ties).
    m = report("tuned system", force_errors(f, ref, A, tie_allowance(xh, w.species, w.box, w.params, 1)))
    assert m[bound_key(1)] <= 1e-5, m


def test_batch_autotune_times_caches_and_runs(ljmd, tmp_path):
    import numpy as np
    ws = W.replica_draws(nrep=5)
    sizes, edges = [w.n for w in ws], [w.box[0] for w in ws]
    x = np.concatenate([w.x for w in ws])
    v = np.concatenate([w.v for w in ws])
    sp = np.concatenate([w.species for w in ws])
    cache = str(tmp_path / "tune_batch.jsonl")
    t = ljmd.autotune_batch(sizes, edges, ws[0].params, x, v, sp, steps=10, cache_path=cache)
    print("tuned batch", t, flush=True)
    assert t["lanes"] in (1, 2, 4, 8, 16) and t["cell_split"] in (1, 2)
    assert t["ms_per_step"] > 0.0 and not t["from_cache"]
    assert t["max_fill"] > 0 and t["nbr_capacity"] >= t["max_fill"] + 16 and t["nbr_capacity"] % 16 == 0
    again = ljmd.autotune_batch(sizes, edges, ws[0].params, x, v, sp, steps=10, cache_path=cache)
    assert again["from_cache"] and again["lanes"] == t["lanes"] and again["nbr_capacity"] == t["nbr_capacity"]
    assert again["cell_split"] == t["cell_split"]
    b = ljmd.Batch(sizes, edges, ws[0].params, lanes=t["lanes"], nbr_capacity=t["nbr_capacity"],
                   cell_split=t["cell_split"])
    b.set_state(x, v, sp)
    assert 0 < b.max_fill() <= t["nbr_capacity"]
    f = b.forces().cpu().numpy()
    b.sync()
    off = np.concatenate([[0], np.cumsum(sizes)])
    for k, w in enumerate(ws):
        ref, _, _, A = reference(w.x, w.species, w.box, w.params, 1)
        g = f[off[k]:off[k + 1]]
        # FP32 pair arithmetic, allowance at cutoff ties as in test_gpu_parity.py.
        m = report(f"tuned batch replica {k}",
                   force_errors(g, ref, A, tie_allowance(w.x, w.species, w.box, w.params, 1)))
        assert m[bound_key(1)] <= 1e-5, (k, m)
