"""ljmd_brute_forces_noalloc (the allocation-free variant of ljmd_brute_forces,
scratch in a fixed per-GPU device array) against ljmd_brute_forces with a
caller workspace, through the C ABI: the same kernels in the same order, so
the outputs must agree bit for bit. Two calls in a row, the second on a
smaller input (the array keeps the first call's contents), in both
precisions and with and without the cutoff; sizes beyond the fixed scratch
are rejected before any launch."""
import numpy as np
import pytest

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


def inputs():
    big = W.random_dense(1500, 1.1, seed=7, nspecies=2, min_dist=0.75)
    small = W.random_dense(300, 0.8442, seed=11)
    allp = W.all_pairs_fluid(n=900)
    return [("mixture1500", big), ("fluid300", small), ("allpairs900", allp)]


@pytest.mark.parametrize("prec", [FP64, FP32_DS])
def test_noalloc_matches_workspace_call(ljmd, prec):
    import torch
    seq = inputs()
    # Big first, then smaller ones: the shared array holds the earlier
    # call's records and partial rows when the next one starts.
    for name, w in seq:
        n = len(w.x)
        print(f"noalloc case={name} n={n} prec={prec}", flush=True)
        f0, uw0 = ljmd.brute_forces(n, w.box, w.params, w.x, w.species, precision=prec)
        f1, uw1 = ljmd.brute_forces_noalloc(n, w.box, w.params, w.x, w.species, precision=prec)
        torch.cuda.synchronize()
        a, b = f0.cpu().numpy(), f1.cpu().numpy()
        assert np.array_equal(a.view(np.uint64), b.view(np.uint64)), (name, np.abs(a - b).max())
        assert np.array_equal(uw0.cpu().numpy().view(np.uint64), uw1.cpu().numpy().view(np.uint64)), name
        assert np.isfinite(a).all()


def test_noalloc_rejects_sizes_beyond_scratch(ljmd):
    import ctypes as C
    limit = int(ljmd.lib.ljmd_brute_static_scratch_bytes())
    p = W.single_species_params()
    n = 400_000
    L = (n / 0.8442) ** (1.0 / 3.0)
    params = ljmd.make_params(n, np.full(3, L), p, FP32_DS, 0)
    need = int(ljmd.lib.ljmd_brute_workspace_size(C.byref(params)))
    assert need > limit
    # Rejected on the host before any pointer is touched.
    code = ljmd.lib.ljmd_brute_forces_noalloc(C.byref(params), C.c_void_p(16), C.c_void_p(16), C.c_void_p(16),
                                              C.c_void_p(16), None)
    assert code == -2  # LJMD_ENOMEM
    assert "scratch" in ljmd.last_error(None)
