"""The C-ABI library on the CPU: it loads, exports every declared entry point,
and rejects malformed input on the host before touching the GPU."""
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "phmg.h")


def _lib():
    from paper_2407_07253_amd import _lib
    return _lib


def test_every_declared_function_is_exported():
    lib = _lib()
    text = open(HEADER).read()
    declared = sorted(set(re.findall(r"\b(phmg_[a-z_0-9]+)\s*\(", text)))
    assert declared, "no declarations found"
    import ctypes
    so = ctypes.CDLL(lib.LIB_PATH)
    for name in declared:
        assert hasattr(so, name), name
    assert sorted(lib.EXPORTED) == declared


def _tiny_hierarchy():
    from paper_2407_07253_amd import frontend
    fh = frontend.build_hierarchy("tiny4")
    L0, L1 = fh.levels
    K = [[L0.K.rowptr.copy(), L0.K.col.copy(), L0.K.val.copy(), L0.K.nrows, L0.K.ncols],
         [L1.K.rowptr.copy(), L1.K.col.copy(), L1.K.val.copy(), L1.K.nrows, L1.K.ncols]]
    P = [[L1.P.rowptr.copy(), L1.P.col.copy(), L1.P.val.copy(), L1.P.nrows, L1.P.ncols]]
    pts = [[L0.patch_ptr.copy(), L0.patch_dofs.copy(), L0.patch_weight.copy()]]
    return K, P, pts, L1.null_vector()


def _create(K, P, pts, z, **kw):
    lib = _lib()
    return lib.Hierarchy(K, P, pts, z, stream=0, **kw)


def _expect_einval(K, P, pts, z, match, **kw):
    lib = _lib()
    with pytest.raises(lib.PhmgError) as e:
        _create(K, P, pts, z, **kw)
    assert e.value.status == lib.PHMG_EINVAL
    assert re.search(match, str(e.value)), str(e.value)


def test_rejects_unsorted_columns():
    K, P, pts, z = _tiny_hierarchy()
    r = 5
    a, b = K[0][0][r], K[0][0][r + 1]
    K[0][1][a:b] = K[0][1][a:b][::-1].copy()
    _expect_einval(K, P, pts, z, r"level 0: K: columns not strictly ascending in row 5")


def test_rejects_column_out_of_range_and_nan():
    K, P, pts, z = _tiny_hierarchy()
    K[1][1][3] = 10 ** 6
    _expect_einval(K, P, pts, z, r"level 1: K: column index out of range")
    K, P, pts, z = _tiny_hierarchy()
    K[0][2][7] = np.nan
    _expect_einval(K, P, pts, z, r"level 0: K: non-finite value")


def test_rejects_level_size_mismatch():
    K, P, pts, z = _tiny_hierarchy()
    P[0][4] = P[0][4] - 1
    _expect_einval(K, P, pts, z, r"P|column index")


def test_rejects_bad_patches():
    K, P, pts, z = _tiny_hierarchy()
    pts[0][1][pts[0][0][3]] = K[0][3] + 5
    _expect_einval(K, P, pts, z, r"level 0: patch 3 dof out of range")
    K, P, pts, z = _tiny_hierarchy()
    s = pts[0][0][2]
    pts[0][1][s], pts[0][1][s + 1] = pts[0][1][s + 1], pts[0][1][s]
    _expect_einval(K, P, pts, z, r"level 0: patch 2 dofs not strictly ascending")
    K, P, pts, z = _tiny_hierarchy()
    pts[0][2][0] = np.inf
    _expect_einval(K, P, pts, z, r"non-finite weight")


def test_rejects_bad_options():
    K, P, pts, z = _tiny_hierarchy()
    _expect_einval(K, P, pts, z, r"cycle options", n_v=0)
    _expect_einval(K, P, pts, z, r"cycle options", n_plevels=5)


@pytest.mark.parametrize("seed", range(12))
def test_host_hessenberg_qr_matches_lapack(seed):
    """The host QR that turns Arnoldi's Hessenberg matrix into the Chebyshev bound."""
    lib = _lib()
    rng = np.random.default_rng(seed)
    k = int(rng.integers(1, 31))
    H = np.triu(rng.standard_normal((k + 1, k)), -1)
    if seed % 3 == 0:                      # clustered spectrum like the smoother's
        H[:k, :k] += np.diag(10.0 + 1e-3 * rng.standard_normal(k))
    ref = np.linalg.eigvals(H[:k, :k]).real.max()
    got = lib.ritz_max_real(H, k)
    assert abs(got - ref) <= 1e-9 * max(1.0, abs(ref)), (k, got, ref)


def test_host_hessenberg_qr_rejects_bad_input():
    lib = _lib()
    H = np.zeros((3, 2))
    H[0, 0] = np.nan
    with pytest.raises(lib.PhmgError):
        lib.ritz_max_real(H, 2)


def test_batched_entry_points_reject_bad_arguments_on_the_host():
    """The batched calls validate before any launch (null context, nrhs range)."""
    import ctypes
    lib = _lib()
    it = (ctypes.c_int32 * 4)()
    rr = (ctypes.c_double * 4)()
    assert lib._fgmres_b(None, 4, 1, 2, 1e-8, 30, 100, it, rr) == lib.PHMG_EINVAL
    assert "null context" in lib.last_error()
    assert lib._vcycle_b(None, 0, 1, 2) == lib.PHMG_EINVAL
    assert lib._apply_b(None, 0, 17, 1, 2, 1) == lib.PHMG_EINVAL
