"""Pins of the oracle's Stokes discretisation (not gpu).

Closed forms, invariants and manufactured-solution rates; none of them
re-types the assembly formula.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import synth
from oracle.discretization import assemble_stokes, divergence_at_quadrature, l2_errors


def _mms(seed=1):
    A = synth.mms_amplitude(seed)
    return (lambda x, y: synth.mms_velocity(x, y, A), lambda x, y: synth.mms_pressure(x, y, A),
            lambda x, y: synth.mms_forcing(x, y, A))


def _direct(d):
    z = d.null_vector()
    Kb = sp.bmat([[d.K, sp.csr_matrix(z[:, None])], [sp.csr_matrix(z[None, :]), None]], format="csc")
    return spla.spsolve(Kb, np.concatenate([d.b, [0.0]]))[:-1]


@pytest.mark.parametrize("k,N", [(2, 8), (3, 4), (4, 3)])
def test_dof_count_closed_form_structured(k, N):
    d = assemble_stokes(synth.structured_square(N), k, "TH")
    # free velocity nodes (kN-1)^2 per component, continuous P_{k-1} pressure ((k-1)N+1)^2
    assert d.nfu == (k * N - 1) ** 2
    assert d.nq == ((k - 1) * N + 1) ** 2
    assert d.n == 2 * (k * N - 1) ** 2 + ((k - 1) * N + 1) ** 2


def test_cfg1_size():
    d = assemble_stokes(synth.config_mesh_hierarchy("cfg1")[-1], 2, "TH")
    assert d.n == 531


@pytest.mark.parametrize("kind,k,mesh", [
    ("TH", 2, synth.structured_square(3)),
    ("TH", 4, synth.delaunay_square(10, seed=5)),
    ("SV", 3, synth.alfeld_split(synth.structured_square(2))),
])
def test_symmetry_spd_and_pressure_kernel(kind, k, mesh):
    d = assemble_stokes(mesh, k, kind)
    K = d.K.toarray()
    assert np.abs(K - K.T).max() <= 1e-13 * np.abs(K).max()
    A = K[: 2 * d.nfu, : 2 * d.nfu]
    assert np.linalg.eigvalsh(A).min() > 0
    assert np.abs(K[2 * d.nfu:, 2 * d.nfu:]).max() == 0.0
    # constant pressure is in ker K (all-Dirichlet boundary, Section 2)
    assert np.abs(K @ d.null_vector()).max() < 1e-12 * np.abs(K).max()


@pytest.mark.parametrize("kind,k,mesh", [
    ("TH", 2, synth.structured_square(3)),
    ("TH", 3, synth.delaunay_square(10, seed=3)),
    ("SV", 4, synth.alfeld_split(synth.structured_square(2))),
])
def test_divergence_of_interpolated_curl_is_zero(kind, k, mesh):
    # u = curl(psi) with psi a polynomial of degree k+1 lies in P_k and is divergence free,
    # so the full (pre-elimination) divergence rows annihilate its nodal interpolant.
    rng = np.random.default_rng(7)
    c = rng.standard_normal((k + 2, k + 2))

    def psi_grad(x, y):
        gx = np.zeros_like(x)
        gy = np.zeros_like(x)
        for i in range(k + 2):
            for j in range(k + 2 - i):
                if i + j > k + 1:
                    continue
                if i:
                    gx += c[i, j] * i * x ** (i - 1) * y ** j
                if j:
                    gy += c[i, j] * j * x ** i * y ** (j - 1)
        return gx, gy

    d = assemble_stokes(mesh, k, kind)
    X = d.V.coords
    gx, gy = psi_grad(X[:, 0], X[:, 1])
    ux, uy = gy, -gx
    div = d.Bx_full @ ux + d.By_full @ uy
    scale = np.abs(d.Bx_full).max() * np.abs(ux).max()
    assert np.abs(div).max() < 1e-12 * scale
    # and a non-solenoidal field is not annihilated (guards a vacuous check)
    assert np.abs(d.Bx_full @ X[:, 0]).max() > 1e-3


CASES = [
    ("TH", 2, [synth.structured_square(n) for n in (4, 8, 16)]),
    ("TH", 3, [synth.structured_square(n) for n in (4, 8, 16)]),
    ("TH", 4, [synth.structured_square(n) for n in (2, 4, 8)]),
    ("SV", 3, [synth.alfeld_split(synth.structured_square(n)) for n in (4, 8, 16)]),
    ("SV", 4, [synth.alfeld_split(synth.structured_square(n)) for n in (2, 4, 8)]),
]


@pytest.mark.parametrize("kind,k,meshes", CASES, ids=[f"{c[0]}{c[1]}" for c in CASES])
def test_mms_convergence_rates(kind, k, meshes):
    """L2 velocity error O(h^{k+1}) and pressure error O(h^k) (standard TH / SV theory)."""
    u, p, f = _mms()
    errs = []
    for m in meshes:
        d = assemble_stokes(m, k, kind, forcing=f, dirichlet=u)
        errs.append(l2_errors(d, _direct(d), u, p))
    errs = np.array(errs)
    ru = np.log2(errs[-2, 0] / errs[-1, 0])
    rp = np.log2(errs[-2, 1] / errs[-1, 1])
    assert ru > k + 1 - 0.35, (ru, errs)
    assert rp > k - 0.4, (rp, errs)


def test_sv_velocity_is_pointwise_divergence_free_th_is_not():
    """Section 2.1: Scott-Vogelius velocities are pointwise divergence free; Taylor-Hood's are not."""
    u, p, f = _mms()
    m = synth.alfeld_split(synth.structured_square(4))
    dsv = assemble_stokes(m, 4, "SV", forcing=f, dirichlet=u)
    xsv = _direct(dsv)
    divsv = divergence_at_quadrature(dsv, xsv)
    dth = assemble_stokes(m, 4, "TH", forcing=f, dirichlet=u)
    divth = divergence_at_quadrature(dth, _direct(dth))
    assert np.abs(divsv).max() < 1e-9
    assert np.abs(divth).max() > 1e-6


def test_sv_divergence_lies_in_pressure_space():
    """div V_h is inside the discontinuous pressure space for SV (Section 2.1): the direct evaluation
    of div u_h equals -M_T^{-1} (B u_h)_T on every cell for an arbitrary velocity; not so for TH."""
    from oracle.discretization import divergence_projected
    m = synth.alfeld_split(synth.delaunay_square(6, seed=8))
    d = assemble_stokes(m, 3, "SV")
    rng = np.random.default_rng(5)
    x = rng.standard_normal(d.n)
    direct = divergence_at_quadrature(d, x)
    proj = divergence_projected(d, x)
    assert np.abs(direct - proj).max() <= 1e-9 * np.abs(direct).max()
    dth = assemble_stokes(m, 3, "TH")
    dth.kind = "SV"          # force the identity on TH to show it fails there
    xt = rng.standard_normal(dth.n)
    gap = np.abs(divergence_at_quadrature(dth, xt) - divergence_projected(dth, xt)).max()
    assert gap > 1e-2 * np.abs(divergence_at_quadrature(dth, xt)).max()


@pytest.mark.parametrize("k,mesh", [(4, synth.delaunay_square(12, seed=3)), (4, synth.structured_square(3))])
def test_load_vector_integrates_polynomials_exactly(k, mesh):
    """sum_i b_i v_i = int f . psi for a constant force f and the interpolant v
    of psi = x(1-x)y(1-y) (zero on the boundary, degree 4 so I_h psi = psi):
    int psi over the unit square is 1/36."""
    from oracle.discretization import interpolate, load_vector
    d = assemble_stokes(mesh, k, "TH")
    cx, cy = 0.7, -1.3
    b = load_vector(d, lambda x, y: (np.full_like(x, cx), np.full_like(y, cy)))
    psi = lambda x, y: x * (1 - x) * y * (1 - y)
    v = interpolate(d, lambda x, y: (psi(x, y), psi(x, y)))
    assert abs(b @ v - (cx + cy) / 36.0) <= 1e-14
    assert np.all(b[2 * d.nfu:] == 0.0)          # no Dirichlet lift: pressure rows vanish


def test_load_vector_equals_assembly_rhs():
    """The separate load-vector routine reproduces the right-hand side that
    assemble_stokes builds together with K (manufactured forcing and lift)."""
    from oracle.discretization import load_vector
    A = synth.mms_amplitude(2)
    f = lambda x, y: synth.mms_forcing(x, y, A)
    g = lambda x, y: synth.mms_velocity(x, y, A)
    d = assemble_stokes(synth.jitter_interior(synth.structured_square(4), 0.05, seed=1), 3, "TH",
                        forcing=f, dirichlet=g)
    assert np.abs(load_vector(d, f) - d.b).max() <= 1e-13 * np.abs(d.b).max()
