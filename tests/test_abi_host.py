"""Host-side checks of the C ABI (no GPU): the library loads, exports every
function include/ljmd.h declares, validates parameters, plans its workspace
and orders cells along a Hilbert curve."""
import os
import re
import subprocess

import numpy as np
import pytest

from paper_2406_04210_amd import ljmd
from paper_2406_04210_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ljmd.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ljmd_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    names = declared_functions()
    assert len(names) >= 15
    out = subprocess.run(["nm", "-D", "--defined-only", ljmd.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT (ljmd_\w+)", out))
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    # The binding declares exactly the header's functions.
    assert sorted(ljmd.SIGNATURES) == names


def test_abi_version():
    hdr = open(os.path.join(ROOT, "include", "ljmd.h")).read()
    declared = int(re.search(r"#define LJMD_ABI_VERSION (\d+)", hdr).group(1))
    assert ljmd.lib.ljmd_abi_version() == declared == ljmd.ABI_VERSION


def _params(**kw):
    w = W.config_small()
    p = ljmd.make_params(w.n, w.box, w.params)
    for k, v in kw.items():
        if isinstance(v, tuple):
            arr = getattr(p, k)
            for i, x in enumerate(v):
                arr[i] = x
        else:
            setattr(p, k, v)
    return p


def test_valid_params_and_workspace():
    p = _params()
    assert ljmd.check_params(p) == 0
    ws = ljmd.workspace_size(p)
    assert ws > 2048 * 100
    assert ljmd.cell_grid(p) == (4, 4, 4)
    p64 = _params(precision=ljmd.FP64)
    assert ljmd.workspace_size(p64) > 0
    # Larger capacity -> larger workspace.
    assert ljmd.workspace_size(_params(nbr_capacity=512)) > ws


@pytest.mark.parametrize("field,value,code", [
    ("n", 1, -1), ("n", 0, -1), ("nspecies", 3, -1), ("precision", 7, -1), ("dt", 0.0, -1),
    ("dt", float("nan"), -1), ("skin", -0.1, -1), ("sort_interval", -1, -1),
    ("nbr_capacity", -5, -1), ("lanes", 3, -1), ("cell_split", 3, -1), ("cell_split", -1, -1), ("cell_capacity", 769, -1),
    ("box", (4.0, 13.4, 13.4), -4), ("box", (0.0, 13.4, 13.4), -1), ("mass", (0.0, 1.0), -1),
    ("sigma", (0.0, 1.0, 1.0, 1.0), -1),
])
def test_parameter_validation(field, value, code):
    p = _params(**{field: value})
    assert ljmd.check_params(p) == code
    assert ljmd.workspace_size(p) == 0


def test_asymmetric_mixture_rejected():
    w = W.config_mixture(n=4000, seed_index=2)
    p = ljmd.make_params(w.n, w.box, w.params)
    assert ljmd.check_params(p) == 0
    p.eps[2] = 2.0
    assert ljmd.check_params(p) == -1


def test_create_rejects_bad_arguments():
    import ctypes as C
    p = _params()
    ctx = C.c_void_p()
    # NULL workspace
    assert ljmd.lib.ljmd_create(C.byref(p), None, 0, None, C.byref(ctx)) == -1
    assert "workspace" in ljmd.last_error(None)
    # too small workspace (pointer never dereferenced on this path)
    assert ljmd.lib.ljmd_create(C.byref(p), C.c_void_p(256), 1024, None, C.byref(ctx)) == -2
    # misaligned
    assert ljmd.lib.ljmd_create(C.byref(p), C.c_void_p(257), 1 << 40, None, C.byref(ctx)) == -1
    assert ljmd.lib.ljmd_run(None, 1, None) == -1


def _hilbert_order(n):
    r = ljmd.hilbert_ranks(n, n, n)
    assert sorted(r.tolist()) == list(range(n ** 3))      # a bijection onto 0..n^3-1
    cells = np.empty((n ** 3, 3), dtype=np.int64)
    lin = np.arange(n ** 3)
    cells[r] = np.stack([lin // (n * n), (lin // n) % n, lin % n], axis=1)
    return cells


@pytest.mark.parametrize("n", [2, 4, 8, 16, 32])
def test_hilbert_consecutive_cells_are_face_adjacent(n):
    cells = _hilbert_order(n)
    steps = np.abs(np.diff(cells, axis=0)).sum(axis=1)
    assert np.all(steps == 1)


@pytest.mark.parametrize("dims", [(23, 23, 23), (3, 5, 7), (1, 1, 1), (2, 9, 4)])
def test_hilbert_ranks_are_a_bijection_on_any_grid(dims):
    r = ljmd.hilbert_ranks(*dims)
    assert sorted(r.tolist()) == list(range(int(np.prod(dims))))
    # Compacting a 2^k curve keeps locality: most consecutive cells are close.
    nx, ny, nz = dims
    lin = np.arange(nx * ny * nz)
    cells = np.empty((len(lin), 3), dtype=np.int64)
    cells[r] = np.stack([lin // (ny * nz), (lin // nz) % ny, lin % nz], axis=1)
    if len(lin) > 8:
        steps = np.abs(np.diff(cells, axis=0)).sum(axis=1)
        assert np.mean(steps == 1) > 0.6
