"""Pins of the oracle's V-cycles against dense forms of eqs. "eq:TG-operator" / "eq:DC-TG-operator"."""
import numpy as np
import pytest

from oracle import multigrid, problems
from oracle.multigrid import CycleOpts


def _dense_minv(L):
    K = L.K.toarray()
    M = np.zeros_like(K)
    for i, S in enumerate(L.patches):
        inv = np.linalg.inv(K[np.ix_(S, S)])
        if L.weights is not None:
            inv = L.weights[i][:, None] * inv
        M[np.ix_(S, S)] += inv
    return M


def _dense_cycle_operator(levels, opts, l, nu_of):
    """T_l with x_out = T_l b for a cycle from x = 0 on level l (dense algebra only)."""
    L = levels[l]
    K = L.K.toarray()
    n = K.shape[0]
    if l == len(levels) - 1:
        z = L.null
        Kb = np.block([[K, z[:, None]], [z[None, :], np.zeros((1, 1))]])
        return np.linalg.inv(Kb)[:n, :n]
    nu = nu_of(l)
    Minv = _dense_minv(L)
    S = np.eye(n) - opts.omega * Minv @ K
    Anu = sum(np.linalg.matrix_power(S, t) for t in range(nu)) @ (opts.omega * Minv)
    P = levels[l + 1].P.toarray()
    Kc = levels[l + 1].K.toarray()
    Tc = _dense_cycle_operator(levels, opts, l + 1, nu_of)
    if l + 1 == opts.n_plevels and l + 1 != len(levels) - 1:
        # G_1 = n_V stationary hMG iterations: T <- T + (I - T K) T1
        T1 = Tc
        T = np.zeros_like(T1)
        for _ in range(opts.n_v):
            T = T + T1 @ (np.eye(Kc.shape[0]) - Kc @ T)
        Tc = T
    C = np.eye(n) - P @ Tc @ P.T @ K
    Snu = np.linalg.matrix_power(S, nu)
    return Snu @ (C @ Anu + P @ Tc @ P.T) + Anu


def _check(levels, opts):
    multigrid.setup(levels)
    n = levels[0].n
    nu_of = lambda l: opts.nu_p if l < opts.n_plevels else opts.nu_h
    T = _dense_cycle_operator(levels, opts, 0, nu_of)
    rng = np.random.default_rng(5)
    for _ in range(3):
        b = rng.standard_normal(n)
        got = multigrid.vcycle(levels, opts, b)
        ref = T @ b
        assert np.abs(got - ref).max() <= 1e-11 * np.abs(ref).max()
        got_t = multigrid.vcycle(levels, opts, b, transpose=True)
        ref_t = T.T @ b
        assert np.abs(got_t - ref_t).max() <= 1e-11 * np.abs(ref_t).max()


def test_coarse_bordered_solve_is_min_norm_least_squares():
    levels, discs, opts, b = problems.build("tiny4")
    multigrid.setup(levels)
    C = levels[-1]
    Kc = C.K.toarray()
    rhs = Kc @ np.random.default_rng(1).standard_normal(C.n)      # consistent right-hand side
    got = multigrid.coarse_solve(C, rhs)
    ref = np.linalg.lstsq(Kc, rhs, rcond=None)[0]
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


def test_two_level_hmg_equals_dense_propagator():
    levels, discs, opts, b = problems.build("tiny4")
    _check(levels, CycleOpts(nu_p=2, nu_h=2, n_v=1, n_plevels=0, omega=0.5))


def test_hmg_with_two_cycles_from_zero():
    levels, discs, opts, b = problems.build("tiny4")
    opts = CycleOpts(nu_p=2, nu_h=1, n_v=2, n_plevels=0, omega=0.6)
    multigrid.setup(levels)
    # two stationary cycles: x1 = T b, x2 = x1 + T (b - K x1)
    nu_of = lambda l: opts.nu_h
    T = _dense_cycle_operator(levels, CycleOpts(1, 1, 1, 0, 0.6), 0, nu_of)
    K = levels[0].K.toarray()
    bb = np.random.default_rng(2).standard_normal(levels[0].n)
    x1 = T @ bb
    ref = x1 + T @ (bb - K @ x1)
    got = multigrid.vcycle(levels, opts, bb)
    assert np.abs(got - ref).max() <= 1e-11 * np.abs(ref).max()


@pytest.mark.parametrize("n_v", [1, 2])
def test_phmg_defect_correction_equals_dense(n_v):
    specs = [(0, 3, "TH"), (0, 2, "TH"), (1, 2, "TH")]
    opts = CycleOpts(nu_p=2, nu_h=1, n_v=n_v, n_plevels=1, omega=0.55)
    levels, discs, _, b = problems.build("tiny4", specs=specs, opts=opts)
    _check(levels, opts)
