"""Matrix functions of the shifted Helmholtz operator (oracle side).

Paper passages followed:
  * psi functions: psi_0 = exp, psi_{l+1}(z) = (psi_l(z) - 1/l!)/z   (Section 3.1, Def. psi)
  * int_0^t exp(i tau A) d tau = t psi_1(i t A)                     (Section 3.1, eq. inverse-1)
  * exp / psi_1 actions evaluated by an established matrix-function
    method (the paper cites Al-Mohy--Higham and uses a restarted
    Krylov method, Section 4 intro)

  * double time integral: (1/t) int_0^t int_0^s exp(i sigma A) d sigma ds
    = t psi_2(i t A), and the second inverse formula
    A^{-1} = -i t (I - psi_1(i t A))^{-1} psi_2(i t A)     (Section 3.1, after eq. inverse-1)

Routes:
  (i)  dense: scipy.linalg.expm on the full matrix (tiny grids);
  (ii) scipy.sparse.linalg.expm_multiply (Al-Mohy--Higham 2011), with psi_1
       from the augmented matrix [[M, v], [0, 0]] whose exponential carries
       psi_1(M) v in its last column, and psi_2 from
       [[M, v, 0], [0, 0, 1], [0, 0, 0]] (last column: psi_2(M) v);
  (iii) closed form for the homogeneous operator without a layer: A_s is
       diagonalised by the type-I discrete sine transform.

Parity: routes (i) and (ii) are pinned against each other and against the
closed form (iii); (iii) is pinned against the textbook DST eigenpairs.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.fft
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def psi_scalar(l: int, z: complex) -> complex:
    """psi_l(z) by Definition psi.  For |z| < 1 the recurrence cancels, so the
    equivalent power series sum_k z^k/(k+l)! is summed instead."""
    z = complex(z)
    if abs(z) < 1.0:
        total = 0j
        term = 1.0 / math.factorial(l)
        k = 0
        while True:
            total += term
            k += 1
            term = term * z / (k + l)
            if abs(term) < 1e-18 * max(abs(total), 1e-300) or k > 60:
                break
        return total
    val = complex(np.exp(z))
    for j in range(l):
        val = (val - 1.0 / math.factorial(j)) / z
    return val


def exp_action(As: sp.spmatrix, t: float, v: np.ndarray) -> np.ndarray:
    """exp(i t A_s) v via expm_multiply."""
    return spla.expm_multiply((1j * t) * As.tocsr(), np.asarray(v, dtype=np.complex128))


def _unit_column(v: np.ndarray):
    """v / ||v||_1 and ||v||_1.  psi_l(X) v is linear in v, so the augmented
    exponentials below take the unit column and scale the result back: the
    column's norm then does not inflate the augmented matrix's 1-norm, which
    sets expm_multiply's step count."""
    v = np.asarray(v, dtype=np.complex128)
    beta = float(np.abs(v).sum())
    return (v / beta if beta > 0 else v), beta


def phi1_action(As: sp.spmatrix, t: float, v: np.ndarray) -> np.ndarray:
    """psi_1(i t A_s) v via the exponential of the augmented matrix
    [[i t A_s, v], [0, 0]] applied to the last unit vector."""
    N = As.shape[0]
    v, beta = _unit_column(v)
    if beta == 0:
        return np.zeros(N, dtype=np.complex128)
    M = (1j * t) * As.tocsc()
    col = sp.csc_matrix(v.reshape(-1, 1))
    top = sp.hstack([M, col])
    bottom = sp.csc_matrix((1, N + 1), dtype=np.complex128)
    aug = sp.vstack([top, bottom]).tocsr()
    e = np.zeros(N + 1, dtype=np.complex128)
    e[-1] = 1.0
    return beta * spla.expm_multiply(aug, e)[:N]


def phi2_action(As: sp.spmatrix, t: float, v: np.ndarray) -> np.ndarray:
    """psi_2(i t A_s) v via the exponential of the augmented matrix
    [[i t A_s, v, 0], [0, 0, 1], [0, 0, 0]] applied to the last unit vector:
    its top block is int_0^1 (1 - u) exp(u i t A_s) v du = psi_2(i t A_s) v."""
    N = As.shape[0]
    v, beta = _unit_column(v)
    if beta == 0:
        return np.zeros(N, dtype=np.complex128)
    M = (1j * t) * As.tocsc()
    cols = sp.csc_matrix(np.stack([v, np.zeros_like(v)], axis=1))
    top = sp.hstack([M, cols])
    J = sp.csc_matrix(np.array([[0.0, 1.0], [0.0, 0.0]], dtype=np.complex128))
    bottom = sp.hstack([sp.csc_matrix((2, N), dtype=np.complex128), J])
    aug = sp.vstack([top, bottom]).tocsr()
    e = np.zeros(N + 2, dtype=np.complex128)
    e[-1] = 1.0
    return beta * spla.expm_multiply(aug, e)[:N]


def exp_dense(As, t: float) -> np.ndarray:
    """exp(i t A_s) as a dense matrix (tiny grids)."""
    Ad = As.toarray() if sp.issparse(As) else np.asarray(As)
    return sla.expm((1j * t) * Ad)


def phi1_dense(As, t: float) -> np.ndarray:
    """psi_1(i t A_s) as a dense matrix, from the augmented exponential."""
    Ad = As.toarray() if sp.issparse(As) else np.asarray(As)
    N = Ad.shape[0]
    aug = np.zeros((2 * N, 2 * N), dtype=np.complex128)
    aug[:N, :N] = (1j * t) * Ad
    aug[:N, N:] = np.eye(N)
    return sla.expm(aug)[:N, N:]


def phi2_dense(As, t: float) -> np.ndarray:
    """psi_2(i t A_s) as a dense matrix: the top-right block of
    exp([[M, I, 0], [0, 0, I], [0, 0, 0]]), M = i t A_s."""
    Ad = As.toarray() if sp.issparse(As) else np.asarray(As)
    N = Ad.shape[0]
    aug = np.zeros((3 * N, 3 * N), dtype=np.complex128)
    aug[:N, :N] = (1j * t) * Ad
    aug[:N, N:2 * N] = np.eye(N)
    aug[N:2 * N, 2 * N:] = np.eye(N)
    return sla.expm(aug)[:N, 2 * N:]


def dirichlet_eigs(n: int, h: float) -> np.ndarray:
    """Eigenvalues of the 1D second difference (1/h^2) tridiag(1,-2,1) with zero
    Dirichlet ghosts; eigenvector k is sin(pi (j+1) (k+1)/(n+1))."""
    k = np.arange(1, n + 1)
    return -4.0 * np.sin(np.pi * k / (2 * (n + 1))) ** 2 / (h * h)


def exp_action_dst(n, h: float, diag: complex, t: float, v: np.ndarray) -> np.ndarray:
    """exp(i t (diag I + Lap_D)) v for the Dirichlet Laplacian without a layer,
    exactly, through the orthonormal type-I DST in every axis.
    n: nodes per axis (x first); v flat with x fastest."""
    n = tuple(n)
    shape = tuple(reversed(n))
    V = np.asarray(v, dtype=np.complex128).reshape(shape)
    lam = np.full(shape, complex(diag))
    for ax_x, nd in enumerate(n):
        ax = len(n) - 1 - ax_x
        sh = [1] * len(n)
        sh[ax] = nd
        lam = lam + dirichlet_eigs(nd, h).reshape(sh)
    W = scipy.fft.dstn(V, type=1, norm="ortho")
    W = W * np.exp(1j * t * lam)
    return scipy.fft.idstn(W, type=1, norm="ortho").ravel()
