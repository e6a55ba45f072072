"""phmg_relax_apply_noalloc through the C ABI: the sweeps of phmg_relax_apply
with the work buffers in the library's fixed device array.  The two entry
points launch the same kernels in the same order, so their outputs must agree
bit for bit; two calls in a row, the second on a smaller level, check that the
array's leftover contents from one call do not leak into the next."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from paper_2407_07253_amd import frontend  # noqa: E402


def _dev(a):
    return torch.tensor(np.asarray(a, dtype=np.float64), device="cuda")


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _both(H, level, nu, seed):
    n = H.n[level]
    rng = np.random.default_rng(seed)
    b, x0 = rng.standard_normal(n), rng.standard_normal(n)
    xa, xb = _dev(x0), _dev(x0)
    H.relax_apply(level, _dev(b), xa, nu)
    H.relax_apply_noalloc(level, _dev(b), xb, nu)
    return _host(xa), _host(xb), x0


@pytest.mark.parametrize("name", ["cfg2_r1", "cfg1"])
def test_noalloc_matches_relax_apply(name):
    from paper_2407_07253_amd._lib import Hierarchy
    fh = frontend.build_hierarchy(name)
    H = Hierarchy.from_frontend(fh)
    H.setup()
    print(f"noalloc: {name} levels {H.n}", flush=True)
    # first call on level 0, then a smaller input (level 1) right after it
    for level, seed in ((0, 11), (1, 12), (0, 13)):
        if level >= len(fh.levels) - 1:
            continue
        for nu in (1, 2):
            a, b, x0 = _both(H, level, nu, seed + nu)
            assert not np.array_equal(a, x0)
            assert np.array_equal(a, b), (name, level, nu, float(np.abs(a - b).max()))
    H.close()


def test_noalloc_rejects_oversized_level_and_unset_level():
    from paper_2407_07253_amd import _lib
    from paper_2407_07253_amd._lib import Hierarchy
    # a trivial two-level hierarchy whose finest level needs more than the array:
    # K_0 = I (n x n), one-DoF patches, P = ones (n x 1), K_1 = [1]
    n = 1_500_000
    assert 3 * n > _lib.NOALLOC_MAX_DOUBLES
    rp = np.arange(n + 1, dtype=np.int32)
    col = np.arange(n, dtype=np.int32)
    K0 = (rp, col, np.ones(n), n, n)
    K1 = (np.array([0, 1], dtype=np.int32), np.array([0], dtype=np.int32), np.ones(1), 1, 1)
    P0 = (rp, np.zeros(n, dtype=np.int32), np.ones(n), n, 1)
    pts = [(np.arange(n + 1, dtype=np.int64), col, None)]
    H = Hierarchy([K0, K1], [P0], pts, None)
    x = torch.zeros(n, dtype=torch.float64, device="cuda")
    b = torch.ones(n, dtype=torch.float64, device="cuda")
    with pytest.raises(_lib.PhmgError) as e:
        H.relax_apply_noalloc(0, b, x, 1)
    assert e.value.status == _lib.PHMG_EINVAL and "allocation-free" in str(e.value)
    assert float(x.abs().max()) == 0.0
    H.close()
    # a level that fits but has not been set up
    fh = frontend.build_hierarchy("cfg1")
    H = Hierarchy.from_frontend(fh)
    x = torch.zeros(fh.levels[0].n, dtype=torch.float64, device="cuda")
    with pytest.raises(_lib.PhmgError) as e:
        H.relax_apply_noalloc(0, x, x.clone(), 1)
    assert e.value.status == _lib.PHMG_ESTATE
    H.close()
