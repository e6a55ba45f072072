"""Failure handling and the pressure-kernel projection, through the C ABI.

* A NaN or Inf in b (or in the initial x) is rejected with PHMG_EINVAL before
  any iteration (the device norm of b - K x_0 is not finite) and x is left as
  it was; the batched solve names the offending system.
* maxit reached: PHMG_ENOCONV, iters = maxit, and x is the last iterate, i.e.
  what the oracle's FGMRES (Section 4) returns after the same number of steps.
* phmg_project_kernel removes the component along the constant pressure (the
  kernel of K with Dirichlet data on the whole boundary, Section 2): for
  z = [0; 1_p] that is the pressure mean, checked against numpy.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import fgmres as ofgmres  # noqa: E402
from oracle import multigrid as omg  # noqa: E402
from oracle import problems as oproblems  # noqa: E402
from paper_2407_07253_amd import frontend  # noqa: E402


def _dev(a):
    return torch.tensor(np.ascontiguousarray(a, dtype=np.float64), device="cuda")


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


_H = {}


def _hier(name="cfg1"):
    if name not in _H:
        from paper_2407_07253_amd._lib import Hierarchy
        fh = frontend.build_hierarchy(name)
        H = Hierarchy.from_frontend(fh)
        H.setup()
        _H[name] = (fh, H)
    return _H[name]


@pytest.mark.parametrize("bad", [np.nan, np.inf, -np.inf])
def test_nonfinite_right_hand_side_is_rejected(bad):
    from paper_2407_07253_amd._lib import PhmgError, PHMG_EINVAL
    fh, H = _hier()
    b = np.array(fh.b[0])
    b[17] = bad
    x0 = np.random.default_rng(1).standard_normal(b.size)
    x = _dev(x0)
    with pytest.raises(PhmgError) as e:
        H.fgmres(_dev(b), x, rtol=1e-8)
    assert e.value.status == PHMG_EINVAL and "NaN or Inf" in str(e.value)
    assert np.array_equal(_host(x), x0)
    # a non-finite initial guess with a finite b
    x1 = x0.copy()
    x1[3] = bad
    xg = _dev(x1)
    with pytest.raises(PhmgError) as e:
        H.fgmres(_dev(fh.b[0]), xg, rtol=1e-8)
    assert e.value.status == PHMG_EINVAL
    # batched: the offending system is named
    B = np.stack([fh.b[0], b, fh.b[0]])
    X = _dev(np.zeros_like(B))
    with pytest.raises(PhmgError) as e:
        H.fgmres_batched(_dev(B), X, rtol=1e-8)
    assert e.value.status == PHMG_EINVAL and "system 1" in str(e.value)
    # the context stays usable
    x = _dev(np.zeros(b.size))
    its, rr, conv = H.fgmres(_dev(fh.b[0]), x, rtol=1e-8)
    assert conv


@pytest.mark.parametrize("maxit", [1, 3, 7])
def test_maxit_returns_enoconv_with_the_last_iterate(maxit):
    fh, H = _hier()
    ol, od, oopts, ob = oproblems.build("cfg1")
    omg.setup(ol, oopts)
    K = ol[0].K
    res = ofgmres.fgmres(lambda v: K @ v, lambda v: omg.vcycle(ol, oopts, v), ob, rtol=1e-12, maxit=maxit)
    assert not res.converged and res.iters == maxit
    x = _dev(np.zeros_like(ob))
    iters, relres, conv = H.fgmres(_dev(fh.b[0]), x, rtol=1e-12, maxit=maxit)
    got = _host(x)
    nfu = od[0].nfu
    g, o = got.copy(), res.x.copy()
    g[2 * nfu:] -= g[2 * nfu:].mean()
    o[2 * nfu:] -= o[2 * nfu:].mean()
    err = np.linalg.norm(g - o) / np.linalg.norm(o)
    print(f"maxit {maxit}: ENOCONV={not conv}, iters {iters}, relres {relres:.3e} (oracle {res.relres:.3e}), "
          f"iterate rel err {err:.2e}")
    assert not conv and iters == maxit
    assert abs(relres - res.relres) <= 1e-8 * res.relres
    assert err <= 1e-10
    # the batched solve reports the same
    X = _dev(np.stack([fh.b[0] * 0.0, fh.b[0]]))
    Xs = torch.zeros_like(X)
    its, rrs, ok = H.fgmres_batched(X, Xs, rtol=1e-12, maxit=maxit)
    assert not ok and its[1] == maxit and its[0] == 0


def test_project_kernel_removes_the_pressure_mean():
    fh, H = _hier()
    L0 = fh.levels[0]
    n, p0 = L0.n, L0.dim * L0.nfu
    rng = np.random.default_rng(5)
    for nrhs in (1, 3, 16):
        X = rng.standard_normal((nrhs, n)) + 3.0
        Xg = _dev(X)
        H.project_kernel(Xg)
        want = X.copy()
        want[:, p0:] -= want[:, p0:].mean(axis=1, keepdims=True)
        got = _host(Xg)
        err = np.abs(got - want).max() / np.abs(want).max()
        print(f"nrhs {nrhs}: projection rel err {err:.2e}")
        assert err <= 1e-14
        assert np.abs(got[:, p0:].sum(axis=1)).max() <= 1e-11 * np.abs(got).max() * (n - p0)


def test_project_kernel_needs_a_kernel_vector():
    from paper_2407_07253_amd._lib import PhmgError, PHMG_ESTATE, PHMG_EINVAL
    fh, H = _hier()
    n = fh.levels[0].n
    X = _dev(np.ones((1, n)))
    H.set_kernel_vector(None)
    with pytest.raises(PhmgError) as e:
        H.project_kernel(X)
    assert e.value.status == PHMG_ESTATE
    with pytest.raises(PhmgError) as e:
        H.set_kernel_vector(np.zeros(n))
    assert e.value.status == PHMG_EINVAL
    H.set_kernel_vector(fh.levels[0].null_vector())
    H.project_kernel(X)
