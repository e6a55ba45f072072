"""Analytic problem data: manufactured solution and seeded forcings.

The Stokes problem is -lap u + grad p = f, -div u = 0 (Section 2, eq.
"eq:stokes-eq").  The manufactured solution used for the benchmark workloads
is u = curl(psi) with psi = A sin^2(pi x) sin^2(pi y), which is divergence
free and vanishes on the boundary of the unit square, and p = A cos(pi x)
cos(pi y), which has zero mean.  f = -lap u + grad p is written out below.
A is drawn from U[0.5, 2] with a seeded generator.

These are plain function evaluations (inputs), not solver arithmetic.
"""
from __future__ import annotations

import numpy as np

PI = np.pi


def mms_amplitude(seed: int) -> float:
    return float(np.random.default_rng(seed).uniform(0.5, 2.0))


def mms_velocity(x: np.ndarray, y: np.ndarray, A: float):
    ux = A * PI * np.sin(PI * x) ** 2 * np.sin(2 * PI * y)
    uy = -A * PI * np.sin(2 * PI * x) * np.sin(PI * y) ** 2
    return ux, uy


def mms_pressure(x: np.ndarray, y: np.ndarray, A: float):
    return A * np.cos(PI * x) * np.cos(PI * y)


def mms_forcing(x: np.ndarray, y: np.ndarray, A: float):
    # lap u_x = A pi^3 sin(2 pi y) (2 cos(2 pi x) - 4 sin^2(pi x))
    # lap u_y = -A pi^3 sin(2 pi x) (2 cos(2 pi y) - 4 sin^2(pi y))
    lap_ux = A * PI ** 3 * np.sin(2 * PI * y) * (2 * np.cos(2 * PI * x) - 4 * np.sin(PI * x) ** 2)
    lap_uy = -A * PI ** 3 * np.sin(2 * PI * x) * (2 * np.cos(2 * PI * y) - 4 * np.sin(PI * y) ** 2)
    dpx = -A * PI * np.sin(PI * x) * np.cos(PI * y)
    dpy = -A * PI * np.cos(PI * x) * np.sin(PI * y)
    return -lap_ux + dpx, -lap_uy + dpy


def gaussian_bump_params(nrhs: int, seed: int):
    """Centres U[0.15,0.85]^2, widths U[0.05,0.2], random unit directions."""
    rng = np.random.default_rng(seed)
    centres = rng.uniform(0.15, 0.85, size=(nrhs, 2))
    widths = rng.uniform(0.05, 0.2, size=nrhs)
    ang = rng.uniform(0.0, 2 * PI, size=nrhs)
    dirs = np.stack([np.cos(ang), np.sin(ang)], axis=1)
    return centres, widths, dirs


def gaussian_bump_forcing(x: np.ndarray, y: np.ndarray, centre, width, direction):
    g = np.exp(-((x - centre[0]) ** 2 + (y - centre[1]) ** 2) / (2.0 * width ** 2))
    return direction[0] * g, direction[1] * g


def fourier_field_params(seed: int, nmodes: int = 8, dim: int = 2, kmax: int = 2):
    """A smooth random field g(x) = sum_m a_m cos(2 pi k_m . x + phi_m): integer wave
    vectors k_m in [-kmax, kmax]^dim (never zero), a_m ~ N(0, 1/nmodes), phi_m ~ U[0, 2 pi)."""
    rng = np.random.default_rng(seed)
    ks = rng.integers(-kmax, kmax + 1, size=(nmodes, dim))
    for m in range(nmodes):
        if not ks[m].any():
            ks[m, 0] = 1
    amp = rng.standard_normal(nmodes) / np.sqrt(nmodes)
    phase = rng.uniform(0.0, 2 * PI, size=nmodes)
    return ks.astype(np.float64), amp, phase


def fourier_field(pts: np.ndarray, params) -> np.ndarray:
    """Evaluate the field at points (N, dim)."""
    ks, amp, phase = params
    return np.cos(2 * PI * pts @ ks.T + phase[None, :]) @ amp


def log_viscosity(verts: np.ndarray, seed: int, scale: float = 0.5) -> np.ndarray:
    """Nodal log-viscosity of the gradient workload: l = scale * g at the mesh vertices."""
    return scale * fourier_field(verts, fourier_field_params(seed, dim=verts.shape[1]))


def gaussian_bump_params3d(nrhs: int, seed: int):
    """3D bumps: centres U[0.15,0.85]^3, widths U[0.05,0.2], random unit directions."""
    rng = np.random.default_rng(seed)
    centres = rng.uniform(0.15, 0.85, size=(nrhs, 3))
    widths = rng.uniform(0.05, 0.2, size=nrhs)
    d = rng.standard_normal((nrhs, 3))
    dirs = d / np.linalg.norm(d, axis=1, keepdims=True)
    return centres, widths, dirs


def gaussian_bump_forcing3d(x: np.ndarray, y: np.ndarray, z: np.ndarray, centre, width, direction):
    g = np.exp(-((x - centre[0]) ** 2 + (y - centre[1]) ** 2 + (z - centre[2]) ** 2) / (2.0 * width ** 2))
    return direction[0] * g, direction[1] * g, direction[2] * g
