"""Krylov solvers and the MatExPre preconditioner (oracle side).

Paper passages followed:
  * fixed-point system (I - exp(i t A)) v = b accelerated by GMRES  (Section 3.4, eq. fixed-point)
  * complex shift A_s = A + i omega^2 s D used inside the preconditioner (Section 3.4)
  * outer flexible GMRES, constant -i t dropped                      (Section 3.4)
  * Algorithm 1: r <- psi_1(i t A_s) r, keep ||r|| as the reference;
    GMRES on (I - exp(i t A_s)) w = r to relative tolerance fprtol;
    return w                                                         (Section 3.4, Algorithm 1)
  * restart 30, outer relative tolerance                             (Section 4 intro)
  * variant: the plain fixed-point iteration v <- exp(i t A) v + b from
    zero instead of GMRES on the same system                         (Section 2.1, Theorem 2.1)
  * variant: the second inverse formula, (I - psi_1(i t A_s)) w =
    psi_2(i t A_s) r, by GMRES or by its fixed-point iteration, the
    matrix form of the time-averaged map            (Section 3.1; Section 2.2, Theorem 2.2)

Readings: inner GMRES starts from w = 0 and stops on the Arnoldi residual
estimate relative to ||psi_1(i t A_s) r||; outer FGMRES starts from the given
initial guess, stops on the Arnoldi estimate relative to ||b|| and then
confirms with the true residual ||b - A u|| (restarting if it is not yet
met).  Orthogonalisation is modified Gram--Schmidt; the small least-squares
problem is solved directly with numpy.linalg.lstsq at every step.

Parity: pinned by the brute-force direct solve (scipy splu) at tight
tolerance, by the one-iteration special case (s = 0, exact inner solve), and
by the closed-form identities of Section 3 on dense tiny grids.
"""
from __future__ import annotations

import dataclasses
from typing import Callable, List, Optional

import numpy as np
import scipy.sparse.linalg as spla

from . import matfun


def _lsq_residual(H: np.ndarray, beta: float, k: int):
    """Solve min ||beta e1 - H[:k+1,:k] y|| and return (y, residual norm)."""
    Hk = H[: k + 1, :k]
    rhs = np.zeros(k + 1, dtype=np.complex128)
    rhs[0] = beta
    y, *_ = np.linalg.lstsq(Hk, rhs, rcond=None)
    res = np.linalg.norm(rhs - Hk @ y)
    return y, res


@dataclasses.dataclass
class GmresResult:
    x: np.ndarray
    iterations: int
    converged: bool
    history: List[float]


def gmres(apply: Callable[[np.ndarray], np.ndarray], b: np.ndarray, tol: float,
          restart: int = 30, maxit: int = 300, ref: Optional[float] = None) -> GmresResult:
    """Restarted GMRES(restart) from x0 = 0 for apply(x) = b; stops when the
    Arnoldi residual estimate is <= tol * ref (ref defaults to ||b||).
    Iterations count Arnoldi steps; the residual recomputed at a restart is
    one extra operator application that is not counted."""
    b = np.asarray(b, dtype=np.complex128)
    N = b.size
    ref = np.linalg.norm(b) if ref is None else ref
    x = np.zeros(N, dtype=np.complex128)
    r = b.copy()
    beta = np.linalg.norm(r)
    its = 0
    history = [beta]
    if beta <= tol * ref or beta == 0.0:
        return GmresResult(x, 0, True, history)
    while True:
        V = np.zeros((restart + 1, N), dtype=np.complex128)
        H = np.zeros((restart + 1, restart), dtype=np.complex128)
        V[0] = r / beta
        k = 0
        converged = False
        res = beta
        for j in range(restart):
            w = apply(V[j])
            its += 1
            for i in range(j + 1):
                H[i, j] = np.vdot(V[i], w)
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            k = j + 1
            _, res = _lsq_residual(H, beta, k)
            history.append(res)
            breakdown = H[j + 1, j].real <= 1e-14 * beta
            if not breakdown:
                V[j + 1] = w / H[j + 1, j]
            if res <= tol * ref or breakdown:
                converged = True
                break
            if its >= maxit:
                break
        y, _ = _lsq_residual(H, beta, k)
        x = x + V[:k].T @ y
        if converged or its >= maxit:
            return GmresResult(x, its, converged, history)
        r = b - apply(x)
        beta = np.linalg.norm(r)
        if beta <= tol * ref:
            return GmresResult(x, its, True, history)


@dataclasses.dataclass
class PrecondResult:
    w: np.ndarray
    inner_iterations: int
    rhat_norm: float


def fixed_point_iteration(apply_E: Callable[[np.ndarray], np.ndarray], b: np.ndarray, tol: float,
                          maxit: int, ref: float):
    """The plain fixed-point iteration v_{k+1} = E v_k + b from v_0 = 0
    (Section 2.1, Theorem 2.1).  Its residual b - (I - E) v_k is the step
    v_{k+1} - v_k.  Returns the first iterate whose residual norm is at most
    tol * ref (v_0 = 0 when ||b|| already is) and the number of E applications
    made; v_1 = b takes none."""
    v = np.zeros_like(b)
    if np.linalg.norm(b) <= tol * ref:
        return v, 0
    v = b.copy()
    its = 0
    while its < maxit:
        step = apply_E(v) + b - v
        its += 1
        if np.linalg.norm(step) <= tol * ref:
            break
        v = v + step
    return v, its


def precond_apply(As, t: float, r: np.ndarray, fprtol: float, restart: int = 30,
                  maxit: int = 300, inner: str = "gmres", form: str = "exp") -> PrecondResult:
    """Algorithm 1: M(r) with the constant -i t dropped.  inner = "gmres"
    (the paper's) or "fixed_point" (Theorem 2.1's plain iteration).

    form = "exp" solves (I - exp(i t A_s)) w = psi_1(i t A_s) r (eq. inverse-1);
    form = "psi2" solves (I - psi_1(i t A_s)) w = psi_2(i t A_s) r, the second
    inverse formula of Section 3.1, whose fixed-point iteration is the matrix
    form of the time-averaged map of Theorem 2.2."""
    if form == "exp":
        rhat = matfun.phi1_action(As, t, r)

        def E(v):
            return matfun.exp_action(As, t, v)
    elif form == "psi2":
        rhat = matfun.phi2_action(As, t, r)

        def E(v):
            return matfun.phi1_action(As, t, v)
    else:
        raise ValueError("form must be 'exp' or 'psi2'")
    z = np.linalg.norm(rhat)
    if inner == "fixed_point":
        if z == 0.0:
            return PrecondResult(np.zeros_like(rhat), 0, z)
        w, its = fixed_point_iteration(E, rhat, fprtol, maxit, z)
        return PrecondResult(w, its, z)
    if inner != "gmres":
        raise ValueError("inner must be 'gmres' or 'fixed_point'")

    def fixed_point_op(v):
        return v - E(v)

    res = gmres(fixed_point_op, rhat, fprtol, restart=restart, maxit=maxit, ref=z)
    return PrecondResult(res.x, res.iterations, z)


@dataclasses.dataclass
class SolveResult:
    u: np.ndarray
    outer_iterations: int
    inner_iterations: List[int]
    converged: bool
    true_relres: float
    history: List[float]

    @property
    def inner_mean(self) -> float:
        return float(np.mean(self.inner_iterations)) if self.inner_iterations else 0.0

    @property
    def inner_std(self) -> float:
        return float(np.std(self.inner_iterations)) if self.inner_iterations else 0.0


def fgmres(A, b: np.ndarray, precond: Callable[[np.ndarray], np.ndarray], rtol: float,
           restart: int = 30, maxit: int = 500, x0: Optional[np.ndarray] = None,
           inner_counter: Optional[List[int]] = None) -> SolveResult:
    """Right-preconditioned flexible GMRES(restart) for A u = b (Saad 1993):
    z_j = M(v_j), w = A z_j, Arnoldi on w, u = u0 + Z y."""
    b = np.asarray(b, dtype=np.complex128)
    N = b.size
    bnorm = np.linalg.norm(b)
    x = np.zeros(N, dtype=np.complex128) if x0 is None else np.array(x0, dtype=np.complex128)
    r = b - A @ x if x0 is not None else b.copy()
    beta = np.linalg.norm(r)
    its = 0
    history = [beta / bnorm]
    inner = inner_counter if inner_counter is not None else []
    if beta <= rtol * bnorm:
        return SolveResult(x, 0, inner, True, beta / bnorm, history)
    while True:
        V = np.zeros((restart + 1, N), dtype=np.complex128)
        Z = np.zeros((restart, N), dtype=np.complex128)
        H = np.zeros((restart + 1, restart), dtype=np.complex128)
        V[0] = r / beta
        k = 0
        est_ok = False
        for j in range(restart):
            Z[j] = precond(V[j])
            w = A @ Z[j]
            its += 1
            for i in range(j + 1):
                H[i, j] = np.vdot(V[i], w)
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            k = j + 1
            _, res = _lsq_residual(H, beta, k)
            history.append(res / bnorm)
            breakdown = H[j + 1, j].real <= 1e-14 * beta
            if not breakdown:
                V[j + 1] = w / H[j + 1, j]
            if res <= rtol * bnorm or breakdown:
                est_ok = True
                break
            if its >= maxit:
                break
        y, _ = _lsq_residual(H, beta, k)
        x = x + Z[:k].T @ y
        r = b - A @ x
        beta = np.linalg.norm(r)
        true_rel = beta / bnorm
        if (est_ok and true_rel <= rtol) or its >= maxit:
            return SolveResult(x, its, inner, true_rel <= rtol, true_rel, history)
        if true_rel <= rtol:
            return SolveResult(x, its, inner, True, true_rel, history)


def matexpre_solve(prob, f: np.ndarray, t: float, shift: float, fprtol: float = 0.08,
                   rtol: float = 1e-6, outer_restart: int = 30, inner_restart: int = 30,
                   max_outer: int = 500, max_inner: int = 300, inner_solver: str = "gmres",
                   form: str = "exp") -> SolveResult:
    """FGMRES on A u = -f preconditioned by Algorithm 1 with A_s."""
    from . import operator as op
    A = op.helmholtz(prob, 0.0)
    As = op.helmholtz(prob, shift)
    b = op.rhs(f)
    inner: List[int] = []

    def M(v):
        pr = precond_apply(As, t, v, fprtol, restart=inner_restart, maxit=max_inner, inner=inner_solver,
                           form=form)
        inner.append(pr.inner_iterations)
        return pr.w

    return fgmres(A, b, M, rtol, restart=outer_restart, maxit=max_outer, inner_counter=inner)


def unpreconditioned_gmres(prob, f: np.ndarray, rtol: float, restart: int = 30,
                           maxit: int = 100000) -> GmresResult:
    """Baseline: plain GMRES(restart) on A u = -f."""
    from . import operator as op
    A = op.helmholtz(prob, 0.0)
    b = op.rhs(f)
    return gmres(lambda v: A @ v, b, rtol, restart=restart, maxit=maxit)


def direct_solve(prob, f: np.ndarray, shift: float = 0.0) -> np.ndarray:
    """Brute force: sparse LU of A_s (shift 0 gives A) applied to -f."""
    from . import operator as op
    A = op.helmholtz(prob, shift).tocsc()
    return spla.splu(A).solve(op.rhs(f))
