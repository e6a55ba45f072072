"""Benchmark hierarchies assembled by the oracle.

Level 0 is the finest.  A level is (mesh, order k, element kind); the
transfer between two consecutive levels is a p-transfer when they share a
mesh (Section 3.2) and an h-transfer between nested meshes otherwise
(Section 3.1).  Direct p-coarsening (Section 4, "phMG(direct)") goes from
P_k/P_{k-1} straight to P_2/P_1 on the finest mesh; Scott-Vogelius level 0 is
coarsened through Taylor-Hood levels (Section 3.2).

Workloads (synthetic stand-ins for the paper's cavity / step problems):
  * cfg1: TH P2/P1 on the structured 8x8 mesh, hMG with the 4x4 mesh as the
    coarse direct solve; nu = 2 damped Richardson sweeps with omega = 0.5 and
    the partition-of-unity weights W_i = diag(1/c_j).
  * cfg2: TH P4/P3 on a Delaunay mesh refined 3 times -> TH P2/P1 on the same
    mesh -> P2/P1 on the 3 coarser meshes (direct solve on the base mesh).
  * cfg3: TH P4/P3 (or P3/P2) on the structured 128x128 mesh -> TH P2/P1 on
    the same mesh -> P2/P1 on 64x64 ... 8x8 (direct solve); 16 right-hand
    sides from seeded Gaussian-bump forcings, homogeneous Dirichlet data.
    cfg3_r1 / cfg3_r2 are the same recipe on 16x16 / 32x32.
  * cfg4: SV P4/P3disc on the Alfeld split of a jittered 16x16 mesh refined
    twice -> TH P2/P1 on the Alfeld mesh -> TH P2/P1 on the 3 macro meshes.
  * cfg2, cfg3 and cfg4 name no smoother; they use the paper's: nu = 2 Chebyshev
    iterations over the basic additive Schwarz operator (W_i = I), interval
    [0.1, 1.1] * lambda_max, lambda_max the largest real Ritz value of 20
    Arnoldi steps on M^{-1} K.
"""
from __future__ import annotations

from typing import List, Tuple

import numpy as np

import synth
from .discretization import assemble_stokes, load_vector
from .multigrid import CycleOpts, Level
from .patches import multiplicity_weights, vanka_star_patches
from .transfer import prolongation

SEEDS = {"cfg1": 1, "cfg2": 2, "cfg3": 3, "cfg4": 4, "cfg5": 5, "cube": 5}


def level_specs(name: str, k: int = None, schedule: str = "direct") -> Tuple[List[Tuple[int, int, str]], CycleOpts]:
    """(mesh index from the finest, order, kind) per level, and cycle options.

    schedule "direct": P_k straight to P_2 on the finest mesh ("phMG(direct)");
    "gradual": the velocity orders of gradual_schedule(k) on the finest mesh,
    every order above 2 a p-level ("phMG(gradual)", Section 4).
    """
    cheb = dict(smoother="chebyshev", cheb_lo=0.1, cheb_hi=1.1, eig_iters=20)
    if name in ("cfg1", "tiny2", "tiny4"):
        return [(0, 2, "TH"), (1, 2, "TH")], CycleOpts(nu_p=2, nu_h=2, n_v=1, n_plevels=0, omega=0.5)
    if name.startswith("cfg2") or name.startswith("cfg3"):
        nref = {"cfg2": 3, "cfg2_r2": 2, "cfg2_r1": 1, "cfg3": 4, "cfg3_r2": 2, "cfg3_r1": 1, "cfg3_r0": 0}[name]
        kk = 4 if k is None else k
        orders = gradual_schedule(kk) if schedule == "gradual" else ([kk, 2] if kk != 2 else [2])
        specs = [(0, o, "TH") for o in orders[:-1]] + [(i, 2, "TH") for i in range(nref + 1)]
        return specs, CycleOpts(nu_p=2, nu_h=2, n_v=1, n_plevels=len(orders) - 1, omega=0.5, **cheb)
    if name in ("cfg5", "cfg5_r1", "cube_tiny"):
        nlev = {"cfg5": 3, "cfg5_r1": 2, "cube_tiny": 2}[name]
        return [(i, 2, "TH") for i in range(nlev)], CycleOpts(nu_p=2, nu_h=2, n_v=1, n_plevels=0, omega=0.5, **cheb)
    if name in ("cfg4", "cfg4_r0", "sv_small"):
        nmac = {"cfg4": 3, "cfg4_r0": 1, "sv_small": 2}[name]
        kk = 4 if k is None else k
        specs = [(0, kk, "SV"), (0, 2, "TH")] + [(i, 2, "TH") for i in range(1, nmac + 1)]
        return specs, CycleOpts(nu_p=2, nu_h=2, n_v=1, n_plevels=1, omega=0.5, **cheb)
    raise KeyError(name)


def gradual_schedule(k: int) -> List[int]:
    """Velocity orders of the gradual p-coarsening schedule (figure "fig:pmg_schedule").

    k in [2,5] goes straight to P2, k in [6,7] through P4, k in [8,10] through P5.
    """
    if 2 <= k <= 5:
        return [k, 2] if k != 2 else [2]
    if k in (6, 7):
        return [k, 4, 2]
    if 8 <= k <= 10:
        return [k, 5, 2]
    raise ValueError(k)


def build(name: str, k: int = None, weights: str = None, with_rhs: bool = True,
          specs=None, opts=None, forcing: str = "mms", nrhs: int = 1, log_visc=None, schedule: str = "direct"):
    """Assemble every level, its patches and the transfers.  Returns (levels, discs, opts, b).

    forcing "mms": b is the manufactured-solution right-hand side (n,).
    forcing "bumps": b is (nrhs, n), one seeded Gaussian-bump forcing per row,
    homogeneous Dirichlet data.
    log_visc: nodal log-viscosity on the finest mesh's vertices (variable
    viscosity nu_h = P1 interpolant of exp(l)); every level is rediscretised
    with l injected to its own vertices (nested meshes keep vertex ids).
    """
    meshes = synth.config_mesh_hierarchy(name)[::-1]          # finest first
    if meshes[0].meta.get("dim") == 3:
        return _build3d(name, meshes, weights, with_rhs, specs, opts, forcing, nrhs, log_visc)
    if specs is None:
        specs, opts = level_specs(name, k, schedule)
    if weights is None:
        weights = "none" if opts.smoother == "chebyshev" else "pou"
    seed = SEEDS.get(name.split("_")[0], 1)
    f = g = None
    if with_rhs and forcing == "mms":
        A = synth.mms_amplitude(seed)
        f = lambda x, y: synth.mms_forcing(x, y, A)
        g = lambda x, y: synth.mms_velocity(x, y, A)
    discs = []
    for li, (mi, kk, kind) in enumerate(specs):
        lv = None
        if log_visc is not None:
            nv = meshes[mi].verts.shape[0]
            assert np.array_equal(meshes[mi].verts, meshes[0].verts[:nv])
            lv = np.asarray(log_visc, dtype=np.float64)[:nv]
        d = assemble_stokes(meshes[mi], kk, kind, forcing=f if li == 0 else None, dirichlet=g if li == 0 else None,
                            log_visc=lv)
        discs.append(d)
    levels = []
    for li, d in enumerate(discs):
        L = Level(K=d.K)
        if li < len(discs) - 1:
            L.patches = vanka_star_patches(d)
            L.weights = multiplicity_weights(L.patches, d.n) if weights == "pou" else None
        if li > 0:
            mf = specs[li - 1][0]
            mc = specs[li][0]
            parent = None if mf == mc else meshes[mf].parent
            L.P = prolongation(discs[li - 1], d, parent)
        levels.append(L)
    levels[-1].null = discs[-1].null_vector()
    b = None
    if with_rhs and forcing == "mms":
        b = discs[0].b
    elif with_rhs and forcing == "bumps":
        C, W, D = synth.gaussian_bump_params(nrhs, seed)
        b = np.stack([load_vector(discs[0], lambda x, y, i=i: synth.gaussian_bump_forcing(x, y, C[i], W[i], D[i]))
                      for i in range(nrhs)])
    elif with_rhs:
        raise KeyError(forcing)
    return levels, discs, opts, b


def _build3d(name, meshes, weights, with_rhs, specs, opts, forcing, nrhs, log_visc):
    """3D Taylor-Hood P2/P1 hierarchy on nested Kuhn cube meshes (hMG, h-levels only)."""
    from . import stokes3d
    if specs is None:
        specs, opts = level_specs(name)
    if weights is None:
        weights = "none" if opts.smoother == "chebyshev" else "pou"
    discs = []
    for mi, kk, kind in specs:
        lv = None
        if log_visc is not None:
            nv = meshes[mi].verts.shape[0]
            assert np.array_equal(meshes[mi].verts, meshes[0].verts[:nv])
            lv = np.asarray(log_visc, dtype=np.float64)[:nv]
        discs.append(stokes3d.assemble(meshes[mi], kk, log_visc=lv))
    levels = []
    for li, d in enumerate(discs):
        L = Level(K=d.K)
        if li < len(discs) - 1:
            L.patches = stokes3d.vanka_star_patches(d)
            L.weights = multiplicity_weights(L.patches, d.n) if weights == "pou" else None
        if li > 0:
            L.P = stokes3d.prolongation(discs[li - 1], d, meshes[specs[li - 1][0]].parent)
        levels.append(L)
    levels[-1].null = discs[-1].null_vector()
    b = None
    if with_rhs and forcing == "bumps":
        seed = SEEDS.get(name.split("_")[0], 5)
        C, W, D = synth.gaussian_bump_params3d(nrhs, seed)
        X = discs[0].V.coords
        fn = np.zeros((nrhs, 3, X.shape[0]))
        for i in range(nrhs):
            fn[i] = synth.gaussian_bump_forcing3d(X[:, 0], X[:, 1], X[:, 2], C[i], W[i], D[i])
        b = stokes3d.forcing_rhs(discs[0], fn)
    elif with_rhs:
        raise KeyError(f"3D workloads take forcing='bumps' (got {forcing!r})")
    return levels, discs, opts, b


def build_and_setup(name: str, **kw):
    levels, discs, opts, b = build(name, **kw)
    from .multigrid import setup
    setup(levels, opts)
    return levels, discs, opts, b
