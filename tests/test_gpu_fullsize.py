"""Full-size GPU checks on the benchmark workloads (through the C ABI).

The oracle cannot run whole solves at these sizes in seconds, so the checks
are (a) sampled outputs the oracle computes one by one -- one relaxation
sweep at ~60 sampled DoFs, using only the patches that contain them -- and
(b) properties that hold at any size: the true residual of the FGMRES
solution measured with the oracle's own assembled K and b, and the
Scott-Vogelius pointwise divergence, evaluated in extended precision.
Full solves against the oracle are in test_gpu_fullsize_golden.py.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

import synth  # noqa: E402
from oracle.discretization import assemble_stokes  # noqa: E402
from oracle.lu import lu_factor, lu_solve  # noqa: E402
from oracle.patches import vanka_star_patches  # noqa: E402
from oracle.problems import SEEDS, level_specs  # noqa: E402
from paper_2407_07253_amd import frontend  # noqa: E402


def _dev(a):
    return torch.tensor(np.asarray(a, dtype=np.float64), device="cuda")


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _oracle_level0(name):
    meshes = synth.config_mesh_hierarchy(name)[::-1]
    specs, _ = level_specs(name)
    mi, k, kind = specs[0]
    A = synth.mms_amplitude(SEEDS[name])
    return assemble_stokes(meshes[mi], k, kind, forcing=lambda x, y: synth.mms_forcing(x, y, A),
                           dirichlet=lambda x, y: synth.mms_velocity(x, y, A))


def test_cfg2_relax_sweep_sampled_against_oracle():
    from paper_2407_07253_amd._lib import Hierarchy
    fh = frontend.build_hierarchy("cfg2")
    omega = 0.37
    H = Hierarchy.from_frontend(fh, weights=False, smoother="richardson", omega=omega)
    H.setup(0)
    d = _oracle_level0("cfg2")
    n = d.n
    rng = np.random.default_rng(42)
    b, x = rng.standard_normal(n), rng.standard_normal(n)
    xg = _dev(x)
    H.relax_apply(0, _dev(b), xg, 1)
    got = _host(xg)
    patches = vanka_star_patches(d)
    sample = np.sort(rng.choice(n, size=60, replace=False))
    r = b - d.K @ x
    want = x[sample].copy()
    for i, S in enumerate(patches):
        pos = np.searchsorted(S, sample)
        hit = (pos < len(S)) & (S[np.minimum(pos, len(S) - 1)] == sample)
        if not hit.any():
            continue
        LU, piv = lu_factor(d.K[S][:, S].toarray())
        y = lu_solve(LU, piv, r[S])
        want[hit] += omega * y[pos[hit]]
    err = np.abs(got[sample] - want).max() / np.abs(want).max()
    print(f"cfg2 sampled sweep: rel err {err:.2e} over {len(sample)} DoFs")
    assert err <= 1e-11
    H.close()


def test_cfg2_fgmres_true_residual_with_oracle_operator():
    from paper_2407_07253_amd._lib import Hierarchy
    fh = frontend.build_hierarchy("cfg2")
    H = Hierarchy.from_frontend(fh)
    H.setup()
    d = _oracle_level0("cfg2")
    assert np.abs(fh.b[0] - d.b).max() <= 1e-12 * np.abs(d.b).max()
    for prec in ("f64", "f32", "bf16"):
        for l in range(len(fh.levels) - 1):
            H.set_precision(l, prec)
        H.setup()
        x = _dev(np.zeros(d.n))
        iters, relres, conv = H.fgmres(_dev(d.b), x, rtol=1e-8, maxit=600)
        xs = _host(x)
        true = np.linalg.norm(d.b - d.K @ xs) / np.linalg.norm(d.b)
        print(f"cfg2 {prec}: {iters} iterations, library relres {relres:.3e}, oracle-operator residual {true:.3e}")
        assert conv
        assert true <= 1.05e-8
    H.close()


def _pressure_residual_extended(K, b, x, lo):
    """Rows lo.. of b - K x accumulated in extended precision (numpy longdouble, 64-bit
    mantissa on x86), then rounded to float64: the FP64 rounding of the sum, which would
    be of the size of the pressure residual itself, is out of the way."""
    K = K.tocsr()
    rp = K.indptr[lo:]
    cols = K.indices[rp[0]:rp[-1]]
    prod = K.data[rp[0]:rp[-1]].astype(np.longdouble) * np.asarray(x, dtype=np.longdouble)[cols]
    sums = np.add.reduceat(prod, rp[:-1] - rp[0]) if len(prod) else np.zeros(0, dtype=np.longdouble)
    sums[np.diff(rp) == 0] = 0
    return (np.asarray(b[lo:], dtype=np.longdouble) - sums).astype(np.float64), \
        (abs(K[lo:]) @ np.abs(x)).astype(np.float64)


def test_cfg4_scott_vogelius_divergence_free_after_tight_solve():
    """Section 2.1: the Scott-Vogelius velocity is pointwise divergence free, ||div u_h||_inf < 1e-10.

    div u_h lies in the discontinuous pressure space, so on every cell T it is fixed by the
    pressure rows of the residual: div u_h|_T = psi^T M_T^{-1} r_p,T (r_p = b_p - B u_h, M_T
    the cell pressure mass matrix).  On this mesh ||psi M_T^{-1}||_inf reaches 5.7e6 (small
    Alfeld cells), so 1e-10 needs |r_p| below ~2e-17 while the terms of (B u_h)_i are of size
    sum_j |B_ij| |u_j| ~ 0.03-0.17: an FP64 evaluation of r_p has a floor of ~1e-10 in div and
    cannot certify the bound.  Here r_p is formed with the library's own operator K in
    extended precision; the evaluation's own floor, eps_ext * nnz_row * sum_j |B_ij| |u_j|
    propagated through M_T^{-1}, is computed and must lie below 1e-11.  The solve runs to a
    relative residual of 2e-11: FP64's attainable level on this system is bounded by
    eps ||(|K| |x|)|| / ||b|| ~ 4e-11 relative (measured on the CPU), so 1e-12 stagnates, and
    1e-11 lies at the edge: it was reached, or missed by a hair (1.09e-11 after 300
    iterations), depending on the summation order inside the patch solve.
    """
    from paper_2407_07253_amd._lib import Hierarchy
    from oracle import element
    from oracle.discretization import cell_geometry
    fh = frontend.build_hierarchy("cfg4")
    H = Hierarchy.from_frontend(fh)
    H.setup()
    d = _oracle_level0("cfg4")
    b = fh.b[0]
    x = _dev(np.zeros(d.n))
    iters, relres, conv = H.fgmres(_dev(b), x, rtol=2e-11, maxit=300)
    xs = _host(x)
    H.close()
    lo = 2 * d.nfu
    rp, scale = _pressure_residual_extended(fh.levels[0].K.to_scipy(), b, xs, lo)
    nrow = np.diff(fh.levels[0].K.to_scipy().tocsr().indptr)[lo:]
    eps_ext = float(np.finfo(np.longdouble).eps)
    assert eps_ext < 1e-18, "needs an extended-precision longdouble"
    k = d.k
    qp, qw = element.quadrature(2 * k)
    psi, _ = element.eval_basis(k - 1, qp)
    verts, cells = d.mesh.verts, d.mesh.cells
    div_max = floor = 0.0
    for c in range(cells.shape[0]):
        _, _, adet, _ = cell_geometry(verts, cells[c])
        M = np.einsum("q,qi,qj->ij", qw * adet, psi, psi)
        rows = d.Q.cell_dofs[c]                     # the cell's pressure DoFs (rows lo + rows of K)
        G = psi @ np.linalg.inv(M)
        div_max = max(div_max, np.abs(G @ rp[rows]).max())
        floor = max(floor, (np.abs(G) @ (eps_ext * nrow[rows] * scale[rows])).max())
    print(f"cfg4: {iters} iterations, relres {relres:.2e}; pressure residual max {np.abs(rp).max():.2e} "
          f"(FP64 rounding of its terms up to {np.finfo(float).eps * scale.max():.1e}); "
          f"max |div u_h| {div_max:.3e}; extended-precision evaluation floor {floor:.2e}")
    assert conv and relres <= 2e-11
    assert floor < 1e-11
    assert div_max < 1e-10
