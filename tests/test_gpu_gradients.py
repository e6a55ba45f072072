"""Gradients through the GPU solve (torch.autograd with the library's adjoint).

Reference 1 (oracle): state and adjoint from sparse direct solves of the
oracle's own variable-viscosity assembly, contracted element by element
(oracle/adjoint.py).  The GPU solves to rtol 1e-12, so the gradients agree to
about 1e-9 relative; the test asks for 1e-7.

Reference 2 (central finite differences, h = 1e-6, FP64): J is re-evaluated
through the GPU forward solve with the perturbed log-viscosity (a new
hierarchy, set-up and solve each time); the difference quotient carries
O(h^2) truncation and solve-tolerance / h rounding, about 1e-6 relative.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

import synth  # noqa: E402
from oracle import adjoint as oadj  # noqa: E402
from oracle import problems as oproblems  # noqa: E402

NAME = "cfg3_r1"
NRHS = 4


def _direct(K, z, b):
    Kb = sp.bmat([[K, sp.csr_matrix(z[:, None])], [sp.csr_matrix(z[None, :]), None]], format="csc")
    return spla.spsolve(Kb, np.concatenate([b, [0.0]]))[:-1]


def _inputs(batched_adjoint=True):
    from paper_2407_07253_amd.adjoint import StokesProblem
    problem = StokesProblem(NAME, rtol=1e-12, batched_adjoint=batched_adjoint)
    lv = synth.log_viscosity(problem.mesh.verts, seed=5)
    fh, H = problem.hierarchy(lv)
    n0, p0, nf = problem.sizes
    coords = fh.levels[0].V.coords
    C, W, D = synth.gaussian_bump_params(NRHS, 6)
    fn = np.zeros((NRHS, 2, coords.shape[0]))
    for b in range(NRHS):
        fn[b, 0], fn[b, 1] = synth.gaussian_bump_forcing(coords[:, 0], coords[:, 1], C[b], W[b], D[b])
    T = np.random.default_rng(11).standard_normal((NRHS, n0)) * 0.01
    return problem, lv, fn, T, p0


def _J(problem, f, l, T, p0):
    """1/2 sum_c ||u_c - t_c||^2 over the free velocity DoFs (entries before the pressure block)."""
    X = problem.solve(f, l)
    Tt = torch.tensor(T, device="cuda")
    return 0.5 * ((X[:, :p0] - Tt[:, :p0]) ** 2).sum()


@pytest.mark.parametrize("batched_adjoint", [True, False])
def test_gradients_match_oracle_adjoint(batched_adjoint):
    problem, lv, fn, T, p0 = _inputs(batched_adjoint)
    f = torch.tensor(fn.reshape(NRHS, -1), device="cuda", requires_grad=True)
    l = torch.tensor(lv, device="cuda", requires_grad=True)
    J = _J(problem, f, l, T, p0)
    J.backward()
    gl, gf = l.grad.cpu().numpy(), f.grad.cpu().numpy().reshape(NRHS, 2, -1)
    print(f"forward iters {problem.last_iters}, adjoint iters {problem.last_adjoint_iters}")
    _, od, _, _ = oproblems.build(NAME, with_rhs=False, log_visc=lv)
    d = od[0]
    B = oadj.forcing_rhs(d, fn)
    z = d.null_vector()
    Xo = np.stack([_direct(d.K, z, b) for b in B])
    Go = oadj.objective_gradient(Xo, T, d.nfu)
    KT = d.K.T.tocsr()
    Lo = np.stack([_direct(KT, z, g) for g in Go])
    Jo = oadj.objective(Xo, T, d.nfu)
    glo = oadj.viscosity_gradient(d, Xo, Lo)
    gfo = oadj.forcing_gradient(d, Lo)
    eJ = abs(float(J) - Jo) / abs(Jo)
    el = np.abs(gl - glo).max() / np.abs(glo).max()
    ef = np.abs(gf - gfo).max() / np.abs(gfo).max()
    print(f"J {float(J):.12e} oracle {Jo:.12e} (rel {eJ:.2e}); dJ/dl rel err {el:.2e}; dJ/df rel err {ef:.2e}")
    assert eJ <= 1e-10
    assert el <= 1e-7
    assert ef <= 1e-7


def test_gradients_match_central_differences():
    problem, lv, fn, T, p0 = _inputs()
    f = torch.tensor(fn.reshape(NRHS, -1), device="cuda", requires_grad=True)
    l = torch.tensor(lv, device="cuda", requires_grad=True)
    _J(problem, f, l, T, p0).backward()
    gl, gf = l.grad.clone(), f.grad.clone()
    rng = np.random.default_rng(13)
    h = 1e-6
    with torch.no_grad():
        for trial in range(2):
            dl = torch.tensor(rng.standard_normal(lv.shape), device="cuda")
            Jp = float(_J(problem, f, l + h * dl, T, p0))
            Jm = float(_J(problem, f, l - h * dl, T, p0))
            fd = (Jp - Jm) / (2 * h)
            an = float((gl * dl).sum())
            print(f"log-viscosity direction {trial}: adjoint {an:.10e} central difference {fd:.10e} "
                  f"rel {abs(an - fd) / abs(fd):.2e}")
            assert abs(an - fd) <= 1e-5 * abs(fd)
        df = torch.tensor(rng.standard_normal(fn.reshape(NRHS, -1).shape), device="cuda")
        Jp = float(_J(problem, f + h * df, l, T, p0))
        Jm = float(_J(problem, f - h * df, l, T, p0))
        fd = (Jp - Jm) / (2 * h)
        an = float((gf * df).sum())
        print(f"forcing direction: adjoint {an:.10e} central difference {fd:.10e} rel {abs(an - fd) / abs(fd):.2e}")
        assert abs(an - fd) <= 1e-5 * abs(fd)
