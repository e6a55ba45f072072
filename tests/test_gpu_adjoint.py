"""Adjoint (transposed) GPU operators against the oracle's transposed cycle.

The library's transposed sweep reuses the forward factors: in the general layout
K_i^{-T} = P_i^T B_i^T with the stored B_i = (P_i K_i)^{-1}; in the symmetric
strip layout (storage "auto" on symmetric levels) the stored S_i = sym(K_i^{-1})
is its own transpose.  The oracle solves with its own LU transposed
(oracle/lu.py lu_solve_transposed).  Both layouts are tested.  Tolerances as in the forward
parity tests.  The adjoint identity <y, B x> = <B^T y, x> is checked on the GPU
alone as a property that holds for any correct pair.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import fgmres as ofgmres  # noqa: E402
from oracle import multigrid as omg  # noqa: E402
from oracle import problems as oproblems  # noqa: E402
from paper_2407_07253_amd import frontend  # noqa: E402

_CACHE = {}


def _pair(name, storage="auto"):
    key = (name, storage)
    if key not in _CACHE:
        from paper_2407_07253_amd._lib import Hierarchy
        fh = frontend.build_hierarchy(name)
        H = Hierarchy.from_frontend(fh)
        for l in range(len(fh.levels) - 1):
            H.set_patch_storage(l, storage)
        H.setup()
        base = _CACHE.get((name, "auto")) or _CACHE.get((name, "general"))
        if base is None:
            ol, od, oopts, ob = oproblems.build(name)
            omg.setup(ol, oopts)
        else:
            ol, od, oopts, ob = base[2:]
        _CACHE[key] = (fh, H, ol, od, oopts, ob)
    return _CACHE[key]


def _dev(a):
    return torch.tensor(np.ascontiguousarray(a, dtype=np.float64), device="cuda")


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def _normalise(x, nfu):
    y = np.array(x, copy=True)
    y[2 * nfu:] -= y[2 * nfu:].mean()
    return y


NAMES = ["cfg1", "cfg2_r1", "sv_small"]


@pytest.mark.parametrize("name", NAMES)
@pytest.mark.parametrize("nu", [1, 2])
@pytest.mark.parametrize("storage", ["auto", "general"])
def test_transposed_relax_matches_oracle(name, nu, storage):
    fh, H, ol, od, oopts, ob = _pair(name, storage)
    rng = np.random.default_rng(500 + nu)
    for l in range(len(ol) - 1):
        n = ol[l].n
        b, x = rng.standard_normal(n), rng.standard_normal(n)
        xg = _dev(x)
        H.relax_apply_transposed(l, _dev(b), xg, nu)
        got = _host(xg)
        ref = omg._relax(ol[l], oopts, b, x, nu, True)
        err = _rel(got, ref)
        print(f"{name} level {l} nu={nu}: transposed sweep rel err {err:.2e}")
        assert err <= 1e-11, (l, err)


@pytest.mark.parametrize("name", NAMES)
@pytest.mark.parametrize("storage", ["auto", "general"])
def test_transposed_vcycle_matches_oracle(name, storage):
    fh, H, ol, od, oopts, ob = _pair(name, storage)
    rng = np.random.default_rng(8)
    b = rng.standard_normal(ol[0].n)
    z = _dev(np.full(ol[0].n, np.nan))
    H.vcycle_transposed(_dev(b), z)
    got = _host(z)
    ref = omg.vcycle(ol, oopts, b, transpose=True)
    err = _rel(got, ref)
    print(f"{name} transposed vcycle rel err {err:.2e}")
    assert err <= 1e-11


@pytest.mark.parametrize("name", NAMES)
@pytest.mark.parametrize("storage", ["auto", "general"])
def test_transposed_vcycle_is_the_adjoint(name, storage):
    """<y, B x> = <B^T y, x> for random x, y (B the forward V-cycle operator)."""
    fh, H, ol, od, oopts, ob = _pair(name, storage)
    rng = np.random.default_rng(9)
    n = ol[0].n
    worst = 0.0
    for _ in range(3):
        x, y = rng.standard_normal(n), rng.standard_normal(n)
        bx, bty = _dev(np.zeros(n)), _dev(np.zeros(n))
        H.vcycle(_dev(x), bx)
        H.vcycle_transposed(_dev(y), bty)
        Bx, BTy = _host(bx), _host(bty)
        lhs, rhs = y @ Bx, BTy @ x
        scale = np.linalg.norm(y) * np.linalg.norm(Bx)
        worst = max(worst, abs(lhs - rhs) / scale)
    print(f"{name}: |<y,Bx> - <B^T y,x>| / (|y||Bx|) = {worst:.2e}")
    assert worst <= 1e-12


@pytest.mark.parametrize("name", NAMES)
@pytest.mark.parametrize("storage", ["auto", "general"])
def test_transposed_fgmres_matches_oracle(name, storage):
    fh, H, ol, od, oopts, ob = _pair(name, storage)
    rng = np.random.default_rng(10)
    g = rng.standard_normal(ol[0].n)
    g[2 * od[0].nfu:] -= g[2 * od[0].nfu:].mean()       # consistent: orthogonal to the pressure kernel
    x = _dev(np.zeros_like(g))
    iters, relres, conv = H.fgmres_transposed(_dev(g), x, rtol=1e-8)
    got = _host(x)
    KT = ol[0].K.T.tocsr()
    res = ofgmres.fgmres(lambda v: KT @ v, lambda v: omg.vcycle(ol, oopts, v, transpose=True), g, rtol=1e-8)
    nfu = od[0].nfu
    err = np.linalg.norm(_normalise(got, nfu) - _normalise(res.x, nfu)) / np.linalg.norm(_normalise(res.x, nfu))
    print(f"{name}: transposed FGMRES GPU iters {iters} relres {relres:.3e}; oracle iters {res.iters} "
          f"relres {res.relres:.3e}; solution rel err {err:.2e}")
    assert conv and res.converged
    assert iters == res.iters
    assert err <= 1e-10


@pytest.mark.parametrize("storage", ["auto", "general"])
@pytest.mark.parametrize("prec", ["f32", "bf16"])
def test_transposed_reduced_precision_is_the_adjoint(prec, storage):
    """With FP32 / BF16 inverses the transposed sweep is still the adjoint of the forward
    one up to float32 rounding of the two products."""
    from paper_2407_07253_amd._lib import Hierarchy
    fh = frontend.build_hierarchy("cfg2_r1")
    H = Hierarchy.from_frontend(fh)
    for l in range(len(fh.levels) - 1):
        H.set_precision(l, prec)
        H.set_patch_storage(l, storage)
    H.setup()
    n = fh.levels[0].n
    rng = np.random.default_rng(12)
    x, y = rng.standard_normal(n), rng.standard_normal(n)
    bx, bty = _dev(np.zeros(n)), _dev(np.zeros(n))
    H.vcycle(_dev(x), bx)
    H.vcycle_transposed(_dev(y), bty)
    Bx, BTy = _host(bx), _host(bty)
    d = abs(y @ Bx - BTy @ x) / (np.linalg.norm(y) * np.linalg.norm(Bx))
    print(f"{prec} ({storage}): adjoint defect {d:.2e}")
    assert d <= 1e-5
    H.close()


@pytest.mark.parametrize("name,nrhs", [("cfg1", 3), ("cfg2_r1", 16), ("sv_small", 5)])
def test_batched_transposed_vcycle_matches_oracle(name, nrhs):
    """Every column of the block adjoint cycle equals the oracle's transposed V-cycle."""
    fh, H, ol, od, oopts, ob = _pair(name, "auto")
    for l in range(len(ol) - 1):
        assert H.level_info(l)["symmetric_storage"], l
    rng = np.random.default_rng(40 + nrhs)
    B = rng.standard_normal((nrhs, ol[0].n))
    Z = _dev(np.full((nrhs, ol[0].n), np.nan))      # content on entry is ignored
    H.vcycle_batched_transposed(_dev(B), Z)
    got = _host(Z)
    worst = max(_rel(got[c], omg.vcycle(ol, oopts, B[c], transpose=True)) for c in range(nrhs))
    print(f"{name} batched transposed vcycle nrhs={nrhs}: worst column rel err {worst:.2e}")
    assert worst <= 1e-11


@pytest.mark.parametrize("name,nrhs", [("cfg1", 2), ("cfg2_r1", 6), ("sv_small", 3)])
def test_batched_transposed_fgmres_equals_single_system_path(name, nrhs):
    """Each column of the lockstep adjoint solve takes the iterations of its own transposed solve."""
    fh, H, ol, od, oopts, ob = _pair(name, "auto")
    rng = np.random.default_rng(60 + nrhs)
    nfu = od[0].nfu
    G = rng.standard_normal((nrhs, ol[0].n))
    G[:, 2 * nfu:] -= G[:, 2 * nfu:].mean(axis=1, keepdims=True)
    G[0] = 0.0                                          # a zero column converges at 0 iterations
    X = _dev(np.zeros_like(G))
    iters, relres, conv = H.fgmres_batched_transposed(_dev(G), X, rtol=1e-8)
    got = _host(X)
    assert conv and iters[0] == 0 and np.all(got[0] == 0.0)
    KT = ol[0].K.T.tocsr()
    for c in range(1, nrhs):
        x1 = _dev(np.zeros(ol[0].n))
        it1, rr1, conv1 = H.fgmres_transposed(_dev(G[c]), x1, rtol=1e-8)
        one = _normalise(_host(x1), nfu)
        err = np.linalg.norm(_normalise(got[c], nfu) - one) / np.linalg.norm(one)
        true_rel = np.linalg.norm(G[c] - KT @ got[c]) / np.linalg.norm(G[c])
        print(f"{name} column {c}: batched iters {iters[c]} relres {relres[c]:.3e}; single iters {it1} "
              f"relres {rr1:.3e}; rel diff {err:.2e}; true relres {true_rel:.3e}")
        assert conv1 and iters[c] == it1
        assert err <= 1e-10
        assert true_rel <= 1e-8 * (1 + 1e-6)


def test_batched_transposed_needs_symmetric_layout():
    from paper_2407_07253_amd._lib import PhmgError
    fh, H, ol, od, oopts, ob = _pair("cfg1", "general")
    n = ol[0].n
    with pytest.raises(PhmgError):
        H.vcycle_batched_transposed(_dev(np.ones((2, n))), _dev(np.zeros((2, n))))
    with pytest.raises(PhmgError):
        H.fgmres_batched_transposed(_dev(np.ones((2, n))), _dev(np.zeros((2, n))))
