"""Pins of the oracle's additive Schwarz sweep against the dense eq. "eq:ASM"."""
import numpy as np
import pytest

import synth
from oracle import relax
from oracle.discretization import assemble_stokes
from oracle.patches import multiplicity_weights, vanka_star_patches


def _dense_Minv(K, patches, weights):
    n = K.shape[0]
    M = np.zeros((n, n))
    for i, S in enumerate(patches):
        inv = np.linalg.inv(K[np.ix_(S, S)])
        if weights is not None:
            inv = weights[i][:, None] * inv
        M[np.ix_(S, S)] += inv
    return M


CASES = [("TH", 2, synth.structured_square(2)), ("TH", 3, synth.structured_square(4)),
         ("SV", 2, synth.alfeld_split(synth.structured_square(1))),
         ("SV", 4, synth.alfeld_split(synth.structured_square(2)))]


@pytest.mark.parametrize("kind,k,mesh", CASES, ids=[f"{c[0]}{c[1]}" for c in CASES])
@pytest.mark.parametrize("weighted", [False, True])
def test_sweep_equals_dense_operator(kind, k, mesh, weighted):
    d = assemble_stokes(mesh, k, kind)
    patches = vanka_star_patches(d)
    W = multiplicity_weights(patches, d.n) if weighted else None
    factors = relax.setup_patches(d.K, patches)
    K = d.K.toarray()
    Minv = _dense_Minv(K, patches, W)
    rng = np.random.default_rng(11)
    b, x = rng.standard_normal(d.n), rng.standard_normal(d.n)
    w = 0.37
    x1 = relax.asm_sweeps(d.K, patches, factors, W, w, b, x, 1)
    ref = x + w * Minv @ (b - K @ x)
    assert np.abs(x1 - ref).max() <= 1e-12 * np.abs(ref).max()
    S = np.eye(d.n) - w * Minv @ K
    x3 = relax.asm_sweeps(d.K, patches, factors, W, w, b, x, 3)
    ref3 = x.copy()
    for _ in range(3):
        ref3 = S @ ref3 + w * Minv @ b
    assert np.abs(x3 - ref3).max() <= 1e-11 * np.abs(ref3).max()
    xt = relax.asm_sweeps(d.K, patches, factors, W, w, b, x, 1, transpose=True)
    reft = x + w * Minv.T @ (b - K.T @ x)
    assert np.abs(xt - reft).max() <= 1e-12 * np.abs(reft).max()
