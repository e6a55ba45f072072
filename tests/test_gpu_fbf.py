"""Full-block-factorisation preconditioner (Section 3.3, eq. "eq:fbf") on the GPU against the oracle.

The velocity-block hierarchy (star patches, velocity transfers) runs through the same
library calls as the monolithic one; the FBF object adds the B, B^T and S~^{-1} products.
Tolerances as for the monolithic parity tests.
"""
import time

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import fbf as ofbf  # noqa: E402
from oracle import fgmres as ofgmres  # noqa: E402
from oracle import multigrid as omg  # noqa: E402
from oracle import problems as oproblems  # noqa: E402
from paper_2407_07253_amd import frontend  # noqa: E402


def _dev(a):
    return torch.tensor(np.ascontiguousarray(a, dtype=np.float64), device="cuda")


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _gpu_fbf(fh):
    from paper_2407_07253_amd._lib import Fbf, Hierarchy
    d = frontend.fbf_inputs(fh)
    K = [(a.rowptr, a.col, a.val, a.nrows, a.ncols) for a in d["A"]]
    P = [(p.rowptr, p.col, p.val, p.nrows, p.ncols) for p in d["P"]]
    Hv = Hierarchy(K, P, d["patches"], None, **d["opts"])
    Hv.setup()
    return Fbf(Hv, d["K"], d["B"], d["S_inv"]), Hv


def _oracle_fbf(name):
    ol, od, oopts, ob = oproblems.build(name)
    vl = ofbf.velocity_levels(ol, od)
    omg.setup(vl, oopts)
    nu = 2 * od[0].nfu
    B = ol[0].K[nu:, :nu].tocsr()
    return ol, od, oopts, ob, vl, B, ofbf.pressure_mass_inverse(od[0])


def test_fbf_apply_and_fgmres_match_oracle():
    fh = frontend.build_hierarchy("sv_small")
    F, Hv = _gpu_fbf(fh)
    ol, od, oopts, ob, vl, B, Sinv = _oracle_fbf("sv_small")
    n = ol[0].n
    rng = np.random.default_rng(41)
    r = rng.standard_normal(n)
    z = _dev(np.zeros(n))
    F.apply(_dev(r), z)
    ref = ofbf.fbf_apply(vl, oopts, B, Sinv, r)
    err = float(np.abs(_host(z) - ref).max() / np.abs(ref).max())
    for l in range(len(vl) - 1):
        assert abs(Hv.level_info(l)["lambda_max"] - vl[l].lmax) <= 1e-11 * vl[l].lmax
    x = _dev(np.zeros(n))
    iters, relres, conv = F.fgmres(_dev(ob), x, rtol=1e-8)
    K = ol[0].K
    res = ofgmres.fgmres(lambda v: K @ v, lambda v: ofbf.fbf_apply(vl, oopts, B, Sinv, v), ob, rtol=1e-8)
    p0 = 2 * od[0].nfu
    got, want = _host(x), np.array(res.x)
    got[p0:] -= got[p0:].mean()
    want[p0:] -= want[p0:].mean()
    xerr = np.linalg.norm(got - want) / np.linalg.norm(want)
    print(f"sv_small FBF: apply rel err {err:.2e}; FGMRES GPU {iters} (relres {relres:.2e}), oracle {res.iters}; "
          f"solution rel err {xerr:.2e}")
    assert err <= 1e-11
    assert conv and res.converged and iters == res.iters
    assert xerr <= 1e-10
    F.close()


def test_fbf_full_size_sv():
    """cfg4 (SV P4/P3disc on the Alfeld split of the jittered 16x16 mesh refined twice): FBF-FGMRES
    converges to 1e-8 (true residual); iterations and time next to the monolithic phMG."""
    from paper_2407_07253_amd._lib import Hierarchy
    fh = frontend.build_hierarchy("cfg4")
    F, Hv = _gpu_fbf(fh)
    b = _dev(fh.b[0])
    x = _dev(np.zeros_like(fh.b[0]))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    iters, relres, conv = F.fgmres(b, x, rtol=1e-8)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    H = Hierarchy.from_frontend(fh)
    H.setup()
    xm = _dev(np.zeros_like(fh.b[0]))
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    im, rm, cm = H.fgmres(b, xm, rtol=1e-8)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    r = _dev(np.zeros_like(fh.b[0]))
    H.residual(0, b, x, r)
    true_rel = float(torch.linalg.norm(r) / torch.linalg.norm(b))
    print(f"cfg4 FBF: {iters} iterations, {1e3 * (t1 - t0):.1f} ms, true relres {true_rel:.2e}; "
          f"monolithic phMG: {im} iterations, {1e3 * (t3 - t2):.1f} ms")
    assert conv and true_rel <= 1.05e-8
    F.close()
    H.close()
