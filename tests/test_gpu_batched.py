"""Batched (multi-right-hand-side) GPU path against the oracle and the single-system path.

Every column of a batched call must equal what the oracle computes for that
system alone: the block kernels (block SpMM, the MFMA patch product, the block
scatter, the block coarse solve) never mix columns.  Tolerances as for the
single-system parity tests: one sweep / one V-cycle to 1e-11 relative (max
norm), FGMRES identical iteration counts per column and solutions equal to
1e-10 relative after removing the pressure mean.  Against the single-system GPU
path the columns agree to rounding of the different summation order (1e-12).
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


def _pair(name, nrhs, storage="auto"):
    """name 'cfg3_r1:k3': the workload with velocity order 3 (Taylor-Hood P3/P2)."""
    key = (name, nrhs, storage)
    if key not in _CACHE:
        from paper_2407_07253_amd._lib import Hierarchy
        base, k = (name.split(":k")[0], int(name.split(":k")[1])) if ":k" in name else (name, None)
        forcing = "bumps" if base.startswith("cfg3") else "mms"
        fh = frontend.build_hierarchy(base, k=k, forcing=forcing, nrhs=nrhs)
        H = Hierarchy.from_frontend(fh)
        for l in range(len(fh.levels) - 1):
            H.set_patch_storage(l, storage)
        H.setup()
        ol, od, oopts, ob = oproblems.build(base, k=k, forcing=forcing, nrhs=nrhs)
        omg.setup(ol, oopts)
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
    y[..., 2 * nfu:] -= y[..., 2 * nfu:].mean(axis=-1, keepdims=True)
    return y


@pytest.mark.parametrize("storage", ["auto", "general"])
@pytest.mark.parametrize("name,nrhs", [("cfg1", 3), ("cfg3_r1", 16), ("sv_small", 5), ("cfg3_r1:k3", 16)])
@pytest.mark.parametrize("nu", [1, 2])
def test_batched_relax_matches_oracle(name, nrhs, nu, storage):
    fh, H, ol, od, oopts, ob = _pair(name, 1, storage)
    rng = np.random.default_rng(300 + nu + nrhs)
    for l in range(len(ol) - 1):
        n = ol[l].n
        B, X = rng.standard_normal((nrhs, n)), rng.standard_normal((nrhs, n))
        Xg = _dev(X)
        H.relax_apply_batched(l, _dev(B), Xg, nu)
        got = _host(Xg)
        worst = 0.0
        for c in range(nrhs):
            ref = omg._relax(ol[l], oopts, B[c], X[c], nu, False)
            worst = max(worst, _rel(got[c], ref))
        print(f"{name} ({storage}) level {l} nu={nu} nrhs={nrhs}: worst column rel err {worst:.2e}")
        assert worst <= 1e-11, (l, worst)


@pytest.mark.parametrize("name,nrhs", [("cfg1", 1), ("cfg2_r1", 4), ("cfg3_r1", 16)])
def test_batched_vcycle_matches_oracle(name, nrhs):
    fh, H, ol, od, oopts, ob = _pair(name, 1)
    rng = np.random.default_rng(11 + nrhs)
    B = rng.standard_normal((nrhs, ol[0].n))
    Z = _dev(np.full((nrhs, ol[0].n), np.nan))      # content on entry is ignored
    H.vcycle_batched(_dev(B), Z)
    got = _host(Z)
    worst = max(_rel(got[c], omg.vcycle(ol, oopts, B[c])) for c in range(nrhs))
    print(f"{name} batched vcycle nrhs={nrhs}: worst column rel err {worst:.2e}")
    assert worst <= 1e-11


@pytest.mark.parametrize("name", ["cfg3_r1", "cfg3_r1:k3"])
def test_batched_fgmres_matches_oracle_per_column(name):
    """cfg3_r1 (16x16 TH P4/P3 and P3/P2, bump forcings): per-column iteration counts and solutions."""
    nrhs = 3
    fh, H, ol, od, oopts, ob = _pair(name, nrhs)
    X = _dev(np.zeros((nrhs, ol[0].n)))
    iters, relres, conv = H.fgmres_batched(_dev(fh.b), X, rtol=1e-8, restart=30, maxit=1000)
    got = _host(X)
    K = ol[0].K
    nfu = od[0].nfu
    assert conv
    for c in range(nrhs):
        res = ofgmres.fgmres(lambda v: K @ v, lambda v: omg.vcycle(ol, oopts, v), ob[c], rtol=1e-8, restart=30,
                             maxit=1000)
        ref = _normalise(res.x, nfu)
        err = np.linalg.norm(_normalise(got[c], nfu) - ref) / np.linalg.norm(ref)
        print(f"column {c}: GPU iters {iters[c]} relres {relres[c]:.3e}; oracle iters {res.iters} "
              f"relres {res.relres:.3e}; solution rel err {err:.2e}")
        assert res.converged
        assert iters[c] == res.iters
        assert err <= 1e-10
        true_rel = np.linalg.norm(ob[c] - K @ got[c]) / np.linalg.norm(ob[c])
        assert true_rel <= 1e-8 * (1 + 1e-6)


@pytest.mark.parametrize("name,nrhs", [("cfg3_r1", 16), ("cfg2_r1", 5), ("cfg1", 2)])
def test_batched_fgmres_equals_single_system_path(name, nrhs):
    """Each column of the lockstep solve takes the iterations of its own single-system solve."""
    fh, H, ol, od, oopts, ob = _pair(name, 1)
    rng = np.random.default_rng(5)
    if name.startswith("cfg3"):
        B = frontend.build_hierarchy(name, forcing="bumps", nrhs=nrhs).b
    else:
        # the manufactured right-hand side and random multiples / perturbations of it; the
        # perturbation is kept orthogonal to the constant-pressure kernel (consistent systems)
        E = rng.standard_normal((nrhs, ol[0].n))
        E[:, 2 * od[0].nfu:] -= E[:, 2 * od[0].nfu:].mean(axis=1, keepdims=True)
        B = fh.b[0][None, :] * rng.uniform(0.5, 2.0, size=(nrhs, 1)) + 1e-3 * E
    X = _dev(np.zeros_like(B))
    iters, relres, conv = H.fgmres_batched(_dev(B), X, rtol=1e-8)
    got = _host(X)
    nfu = od[0].nfu
    assert conv
    for c in range(nrhs):
        x1 = _dev(np.zeros(ol[0].n))
        it1, rr1, conv1 = H.fgmres(_dev(B[c]), x1, rtol=1e-8)
        one = _normalise(_host(x1), nfu)
        err = np.linalg.norm(_normalise(got[c], nfu) - one) / np.linalg.norm(one)
        print(f"{name} column {c}: batched iters {iters[c]} relres {relres[c]:.3e}; single iters {it1} "
              f"relres {rr1:.3e}; rel diff {err:.2e}")
        assert conv1 and iters[c] == it1
        assert err <= 1e-10


def test_batched_zero_and_converged_columns():
    """A zero right-hand side converges at 0 iterations and stays zero; the others are unaffected."""
    fh, H, ol, od, oopts, ob = _pair("cfg1", 1)
    n = ol[0].n
    B = np.stack([fh.b[0], np.zeros(n), 2.0 * fh.b[0]])
    X = _dev(np.zeros((3, n)))
    iters, relres, conv = H.fgmres_batched(_dev(B), X, rtol=1e-8)
    got = _host(X)
    assert conv and iters[1] == 0 and relres[1] == 0.0
    assert np.all(got[1] == 0.0)
    assert iters[0] == iters[2]
    assert _rel(got[2], 2.0 * got[0]) <= 1e-12


@pytest.mark.parametrize("prec", ["f32", "bf16"])
def test_batched_mixed_precision_reaches_fp64_residual(prec):
    """Patch inverses stored in FP32 / BF16 (MFMA, float32 accumulation), FP64 FGMRES: every
    column reaches the FP64 residual target measured with the oracle's operator."""
    from paper_2407_07253_amd._lib import Hierarchy
    nrhs = 16
    fh = frontend.build_hierarchy("cfg3_r1", forcing="bumps", nrhs=nrhs)
    ol, od, oopts, ob = oproblems.build("cfg3_r1", forcing="bumps", nrhs=nrhs)
    H = Hierarchy.from_frontend(fh)
    for l in range(len(fh.levels) - 1):
        H.set_precision(l, prec)
    H.setup()
    X = _dev(np.zeros((nrhs, ol[0].n)))
    iters, relres, conv = H.fgmres_batched(_dev(ob), X, rtol=1e-8)
    got = _host(X)
    K = ol[0].K
    fh64, H64, *_ = _pair("cfg3_r1", 1)
    X64 = _dev(np.zeros((nrhs, ol[0].n)))
    it64, _, conv64 = H64.fgmres_batched(_dev(ob), X64, rtol=1e-8)
    ref = _host(X64)
    nfu = od[0].nfu
    assert conv and conv64
    for c in range(nrhs):
        true_rel = np.linalg.norm(ob[c] - K @ got[c]) / np.linalg.norm(ob[c])
        err = np.linalg.norm(_normalise(got[c] - ref[c], nfu)) / np.linalg.norm(_normalise(ref[c], nfu))
        print(f"{prec} column {c}: iters {iters[c]} (fp64 {it64[c]}), true relres {true_rel:.3e}, "
              f"error vs fp64 solution {err:.2e}")
        assert true_rel <= 1.05e-8
        assert err <= 1e-5
    H.close()


def test_batched_graph_replays_equal_eager():
    """The captured block V-cycle gives bitwise the eager launches, replay after replay."""
    fh, H, ol, od, oopts, ob = _pair("cfg2_r1", 1)
    rng = np.random.default_rng(21)
    outs = []
    for graphs in (False, True, True, True):
        H.set_graphs(graphs)
        B = _dev(rng.standard_normal((6, ol[0].n)))
        Z1 = _dev(np.zeros((6, ol[0].n)))
        H.vcycle_batched(B, Z1)
        torch.cuda.synchronize()
        H.set_graphs(False)
        Z0 = _dev(np.zeros((6, ol[0].n)))
        H.vcycle_batched(B, Z0)
        outs.append((_host(Z1), _host(Z0)))
    H.set_graphs(True)
    for a, b in outs:
        assert np.array_equal(a, b)


def test_batched_argument_errors():
    from paper_2407_07253_amd._lib import PhmgError
    fh, H, ol, od, oopts, ob = _pair("cfg1", 1)
    n = ol[0].n
    with pytest.raises(ValueError):
        H.vcycle_batched(_dev(np.zeros((17, n))), _dev(np.zeros((17, n))))
    with pytest.raises(ValueError):
        H.vcycle_batched(_dev(np.zeros((2, n))), _dev(np.zeros((3, n))))
    with pytest.raises(PhmgError):
        H.relax_apply_batched(len(ol) - 1, _dev(np.zeros((2, ol[-1].n))), _dev(np.zeros((2, ol[-1].n))))
    with pytest.raises(PhmgError):
        H.fgmres_batched(_dev(np.ones((2, n))), _dev(np.zeros((2, n))), restart=40)


@pytest.mark.parametrize("storage", ["auto", "general"])
@pytest.mark.parametrize("prec", ["f32", "bf16"])
def test_batched_reduced_precision_sweep_matches_single_path(prec, storage):
    """With FP32 / BF16 patch inverses the MFMA block product (float32 accumulation) and the
    single-system streaming kernel use the same rounded factors and right-hand sides; they
    differ only in float32 summation order, so a sweep agrees to ~1e-6 in norm.  A wrong
    MFMA lane layout would permute rows inside 16-row tiles and give O(1) differences."""
    from paper_2407_07253_amd._lib import Hierarchy
    fh = frontend.build_hierarchy("cfg3_r1")
    H = Hierarchy.from_frontend(fh)
    for l in range(len(fh.levels) - 1):
        H.set_precision(l, prec)
        H.set_patch_storage(l, storage)
    H.setup()
    rng = np.random.default_rng(77)
    nrhs = 7
    for l in range(len(fh.levels) - 1):
        n = fh.levels[l].n
        B, X = rng.standard_normal((nrhs, n)), rng.standard_normal((nrhs, n))
        Xg = _dev(X)
        H.relax_apply_batched(l, _dev(B), Xg, 1)
        got = _host(Xg)
        worst = 0.0
        for c in range(nrhs):
            x1 = _dev(X[c])
            H.relax_apply(l, _dev(B[c]), x1, 1)
            one = _host(x1)
            worst = max(worst, float(np.linalg.norm(got[c] - one) / np.linalg.norm(one - X[c])))
        print(f"{prec} ({storage}) level {l}: worst column ||batched - single|| / ||correction|| = {worst:.2e}")
        assert worst <= 1e-4
    H.close()


@pytest.mark.parametrize("prec,storage", [("f64", "auto"), ("f64", "general"), ("f32", "auto"), ("bf16", "auto")])
def test_block_variants_bit_identical(prec, storage):
    """Every shape of the multi-right-hand-side patch solve deals rows and columns to lanes
    differently but sums each product in the same order: one sweep with each shape forced
    must give the same bits.  cfg2_r1 level 0 has patches of 64-210 DoFs, so the row groups
    of every shape (16 to 128 rows per pass) end in ragged tails; FP64 shape 0 is also checked
    against the oracle."""
    from paper_2407_07253_amd._lib import Hierarchy, PhmgError
    fh = frontend.build_hierarchy("cfg2_r1")
    H = Hierarchy.from_frontend(fh)
    nl = len(fh.levels)
    for l in range(nl - 1):
        H.set_precision(l, prec)
        H.set_patch_storage(l, storage)
    H.setup()
    rng = np.random.default_rng(91)
    nrhs = 5
    if prec == "f64":
        ol, od, oopts, ob = oproblems.build("cfg2_r1", forcing="mms", nrhs=1)
        omg.setup(ol, oopts)
    for l in range(nl - 1):
        info = H.level_info(l)
        if info["npatch"] == 0:
            continue
        nv = info["block_variants"]
        assert nv >= 4
        n = fh.levels[l].n
        B, X = rng.standard_normal((nrhs, n)), rng.standard_normal((nrhs, n))
        outs = []
        for v in range(nv):
            H.set_block_variant(l, v)
            assert H.level_info(l)["block_variant"] == v
            Xg = _dev(X)
            H.relax_apply_batched(l, _dev(B), Xg, 1)
            outs.append(_host(Xg))
        for v in range(1, nv):
            assert np.array_equal(outs[v], outs[0]), (l, v, float(np.abs(outs[v] - outs[0]).max()))
        if prec == "f64":
            worst = max(_rel(outs[0][c], omg._relax(ol[l], oopts, B[c], X[c], 1, False)) for c in range(nrhs))
            print(f"{storage} level {l}: {nv} shapes identical, rel err vs oracle {worst:.2e}")
            assert worst <= 1e-11, (l, worst)
        with pytest.raises(PhmgError):
            H.set_block_variant(l, nv)
    H.close()


def test_every_block_spmm_shape_gives_the_same_sweep_and_cycle():
    """Every block SpMM shape (16 lanes per row with 1, 2 or 4 groups of entries in flight, 4 or 2
    lanes per row with 4 or 8 systems each; plain or XCD-contiguous rows), forced on K, P and R of
    every level: the shapes that add each row's entries in row order (0, 3, 6-9) give the same
    bits for a batched sweep and a batched V-cycle, the others agree to rounding (1e-12
    relative), and shape 0 matches the oracle's sweep.  cfg2_r1 rows have 20-200 entries, so
    every shape's chunks end in ragged tails."""
    from paper_2407_07253_amd._lib import Hierarchy, PhmgError
    fh = frontend.build_hierarchy("cfg2_r1")
    H = Hierarchy.from_frontend(fh)
    H.setup()
    ol, od, oopts, ob = oproblems.build("cfg2_r1", forcing="mms", nrhs=1)
    omg.setup(ol, oopts)
    nl = len(fh.levels)
    rng = np.random.default_rng(29)
    nrhs = 5
    n0 = fh.levels[0].n
    B, X = rng.standard_normal((nrhs, n0)), rng.standard_normal((nrhs, n0))
    sweeps, cycles = {}, {}
    for v in range(10):
        for l in range(nl):
            H.set_spmm_variant(l, "K", v)
            if l < nl - 1:
                H.set_spmm_variant(l, "P", v)
                H.set_spmm_variant(l, "R", v)
        Xg = _dev(X)
        H.relax_apply_batched(0, _dev(B), Xg, 2)
        sweeps[v] = _host(Xg)
        Xc = _dev(np.zeros((nrhs, n0)))
        H.vcycle_batched(_dev(B), Xc)
        cycles[v] = _host(Xc)
    for v in (3, 6, 7, 8, 9):
        assert np.array_equal(sweeps[v], sweeps[0]), v
        assert np.array_equal(cycles[v], cycles[0]), v
    for v in (1, 2, 4, 5):
        assert _rel(sweeps[v], sweeps[0]) <= 1e-12, (v, _rel(sweeps[v], sweeps[0]))
        assert _rel(cycles[v], cycles[0]) <= 1e-12, (v, _rel(cycles[v], cycles[0]))
    worst = max(_rel(sweeps[0][c], omg._relax(ol[0], oopts, B[c], X[c], 2, False)) for c in range(nrhs))
    assert worst <= 1e-11, worst
    with pytest.raises(PhmgError):
        H.set_spmm_variant(0, "K", 10)
    with pytest.raises(PhmgError):
        H.set_spmm_variant(nl - 1, "P", 0)
    H.close()
