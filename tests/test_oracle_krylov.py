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


def test_fixed_point_iteration_is_the_neumann_series():
    # Theorem 2.1's iteration from zero: v_k = sum_{n<k} E^n b, residual E^k b.
    # For a diagonal E the stopping index is known in closed form.
    rng = np.random.default_rng(3)
    N = 40
    lam = 0.95 * rng.uniform(0.2, 1.0, N) * np.exp(2j * np.pi * rng.uniform(size=N))
    E = np.diag(lam)
    b = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    tol = 1e-3
    v, its = krylov.fixed_point_iteration(lambda x: E @ x, b, tol, 10000, np.linalg.norm(b))
    k = next(k for k in range(1, 10000) if np.linalg.norm(lam ** k * b) <= tol * np.linalg.norm(b))
    assert its == k
    partial = sum(lam ** n * b for n in range(k))
    assert np.allclose(v, partial, rtol=1e-12, atol=1e-12)
    # iteration limit: the iterate after the last step is returned, untested
    v2, its2 = krylov.fixed_point_iteration(lambda x: E @ x, b, tol, 3, np.linalg.norm(b))
    assert its2 == 3 and np.allclose(v2, sum(lam ** n * b for n in range(4)))
    # tolerance met at v_0 = 0 only when tol >= 1
    v3, its3 = krylov.fixed_point_iteration(lambda x: E @ x, b, 1.0, 10, np.linalg.norm(b))
    assert its3 == 0 and not v3.any()


def test_fixed_point_precond_meets_its_tolerance_and_solve_converges():
    prob = _prob(n=(24, 22), layer=5)
    t, s = prob.default_t(), prob.default_shift()
    As = op.helmholtz(prob, s)
    r = wl.random_vector(prob.npts, 5)
    pr = krylov.precond_apply(As, t, r, 0.08, inner="fixed_point")
    rhat = matfun.phi1_action(As, t, r)
    resid = rhat - (pr.w - matfun.exp_action(As, t, pr.w))
    assert np.linalg.norm(resid) <= 0.08 * np.linalg.norm(rhat)
    assert pr.inner_iterations >= 1
    # with the shift the plain iteration converges and the solve reaches the direct solution
    f = wl.delta_source(prob, (12, 11))
    res = krylov.matexpre_solve(prob, f, t, s, fprtol=0.08, rtol=1e-12, inner_solver="fixed_point")
    ref = krylov.direct_solve(prob, f)
    assert res.converged and np.linalg.norm(res.u - ref) <= 1e-10 * np.linalg.norm(ref)


def test_psi2_form_precond_is_scaled_inverse_when_inner_solve_is_exact():
    # (I - psi_1(i t A_s))^{-1} psi_2(i t A_s) r = (i / t) A_s^{-1} r (Section 3.1)
    prob = wl.small_problem((14, 12), layer=3, ppw=10, inhomogeneous=True, seed=2)
    s = 1.0 / prob.freq
    As = op.helmholtz(prob, s)
    t = prob.default_t()
    r = wl.random_vector(prob.npts, 9)
    pr = krylov.precond_apply(As, t, r, 1e-12, restart=200, maxit=400, form="psi2")
    ref = (1j / t) * spla.spsolve(As.tocsc(), r)
    assert np.linalg.norm(pr.w - ref) <= 1e-9 * np.linalg.norm(ref)


def test_psi2_form_fixed_point_meets_tolerance_and_solve_converges():
    prob = wl.small_problem((16, 14), layer=3, ppw=10, inhomogeneous=False, seed=3)
    s = 1.0 / prob.freq
    As = op.helmholtz(prob, s)
    t = prob.default_t()
    r = wl.random_vector(prob.npts, 10)
    pr = krylov.precond_apply(As, t, r, 0.08, inner="fixed_point", form="psi2")
    rhat = matfun.phi2_action(As, t, r)
    res = rhat - (pr.w - matfun.phi1_action(As, t, pr.w))
    assert np.linalg.norm(res) <= 0.08 * np.linalg.norm(rhat) * (1 + 1e-12)
    assert pr.inner_iterations >= 1
    f = wl.delta_source(prob, tuple(k // 2 for k in prob.n))
    for inner in ("gmres", "fixed_point"):
        sol = krylov.matexpre_solve(prob, f, t, s, inner_solver=inner, form="psi2")
        assert sol.converged
        A = op.helmholtz(prob, 0.0)
        b = op.rhs(f)
        assert np.linalg.norm(b - A @ sol.u) <= 1e-6 * np.linalg.norm(b) * (1 + 1e-9)
