"""Pins for the oracle's GMRES / FGMRES and Algorithm 1 (oracle/krylov.py)."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import workloads as wl
from oracle import krylov, matfun, operator as op


def _prob(n=(32, 28), layer=6, inh=False):
    return wl.small_problem(n, layer=layer, ppw=10, inhomogeneous=inh, seed=11)


def test_gmres_matches_direct_solve():
    prob = _prob()
    A = op.helmholtz(prob, 0.0)
    b = op.rhs(wl.delta_source(prob, (16, 14)))
    res = krylov.gmres(lambda v: A @ v, b, 1e-12, restart=30, maxit=20000)
    ref = spla.splu(A.tocsc()).solve(b)
    assert res.converged
    assert np.linalg.norm(res.x - ref) <= 1e-9 * np.linalg.norm(ref)
    # estimates are monotone non-increasing within a cycle
    h = np.array(res.history[:31])
    assert np.all(np.diff(h) <= 1e-12 * h[0])


def test_gmres_exact_in_n_steps_on_small_dense():
    # GMRES without restart reaches the exact solution in at most N steps
    rng = np.random.default_rng(0)
    N = 12
    M = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N)) + 4 * np.eye(N)
    b = rng.standard_normal(N) + 0j
    res = krylov.gmres(lambda v: M @ v, b, 1e-14, restart=N, maxit=N)
    assert np.linalg.norm(M @ res.x - b) <= 1e-11 * np.linalg.norm(b)


@pytest.mark.parametrize("inh", [False, True])
def test_matexpre_fgmres_matches_direct_solve(inh):
    # P8: brute force.  Tight outer tolerance so the iterate is a parity quantity.
    prob = _prob(inh=inh)
    f = wl.delta_source(prob, (16, 14))
    res = krylov.matexpre_solve(prob, f, prob.default_t(), prob.default_shift(), fprtol=0.08,
                                rtol=1e-12)
    ref = krylov.direct_solve(prob, f)
    assert res.converged
    assert np.linalg.norm(res.u - ref) <= 1e-10 * np.linalg.norm(ref)
    assert res.true_relres <= 1e-12


def test_unshifted_exact_inner_solve_converges_in_one_outer_iteration():
    # P9: s = 0 and an (almost) exact inner solve make M a multiple of A^{-1}
    prob = _prob(n=(20, 18), layer=4)
    f = wl.delta_source(prob, (10, 9))
    res = krylov.matexpre_solve(prob, f, prob.default_t(), 0.0, fprtol=1e-13, rtol=1e-8,
                                inner_restart=200, max_inner=2000)
    assert res.outer_iterations == 1
    assert res.true_relres <= 1e-8


def test_precond_is_scaled_inverse_when_inner_solve_is_exact():
    # Algorithm 1 with fprtol -> 0 returns (i/t) A_s^{-1} r  (constant -i t dropped)
    prob = _prob(n=(14, 12), layer=3)
    s = prob.default_shift()
    As = op.helmholtz(prob, s)
    t = prob.default_t()
    r = wl.random_vector(prob.npts, 2)
    pr = krylov.precond_apply(As, t, r, 1e-13, restart=200, maxit=2000)
    ref = spla.splu(As.tocsc()).solve(r) / (-1j * t)
    assert np.linalg.norm(pr.w - ref) <= 1e-9 * np.linalg.norm(ref)


def test_inner_stop_is_relative_to_phi1_residual():
    prob = _prob(n=(24, 20), layer=4)
    s = prob.default_shift()
    As = op.helmholtz(prob, s)
    t = prob.default_t()
    r = wl.random_vector(prob.npts, 9)
    pr = krylov.precond_apply(As, t, r, 0.08)
    rhat = matfun.phi1_action(As, t, r)
    true_res = np.linalg.norm(rhat - (pr.w - matfun.exp_action(As, t, pr.w)))
    assert true_res <= 0.08 * np.linalg.norm(rhat) * (1 + 1e-8)
    assert pr.rhat_norm == pytest.approx(np.linalg.norm(rhat))
    assert pr.inner_iterations >= 1
