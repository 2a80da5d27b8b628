"""Discrete Helmholtz operator with a perfectly matched layer (oracle side).

Paper passages followed:
  * Helmholtz equation omega^2/c^2 u + Lap u = -f            (Section 1, eq. helmholtz)
  * 1D stretched operator (1/s) d/dx((1/s) du/dx), quadratic
    profile s = 1 + i C_pml/(delta omega) (dist/delta)^2     (Section 3.3, eq. pml-1d-s)
  * three-point FD per axis; five-point 2D / seven-point 3D  (Section 3.3, Section 4 intro)
  * zero Dirichlet outside the layer                          (Section 4 intro)
  * shifted operator A_s = A + i omega^2 s D, D = diag(1/c^2)  (Section 3.4)
  * absorbing potential instead of the layer: omega^2 u + c^2 Lap u + i W u
    = -c^2 f, i.e. omega^2/c^2 u + Lap u + i (W/c^2) u = -f, with zero
    Dirichlet values and W >= 0 vanishing inside      (Section 2.1, eq. helmholtz-absorbing)
  * boundary conditions instead of a layer: a sound-hard face (zero normal
    derivative) and first-order absorbing faces, discretised with ghost
    points                                             (Section 4.3.4, Marmousi-II)

Readings where the paper is silent (also listed in the design notes):
  * multi-dimensional layer: sum over axes of (1/s_d) d_d((1/s_d) d_d u), each
    s_d depending on x_d only; the node value 1/s_d(x_i) multiplies the flux
    difference and the half-node values 1/s_d(x_{i+-1/2}) sit in the fluxes;
  * the layer is part of the given grid: the outermost L nodes of each face,
    delta = L h, distance measured from the inner edge x_a = L h,
    x_b = (N-1-L) h; ghost nodes at indices -1 and N are zero;
  * C_pml = 20, power 2;
  * the potential's profile: W/c^2 = 2 omega^2 sum_d sigma_d(x_d) with sigma_d
    the layer profile above, so that a normally incident plane wave decays at
    the stretch's rate to first order (k = sqrt(omega^2 + i W/c^2) ~ omega +
    i omega sigma against k = omega (1 + i sigma)).

  * the first-order absorbing condition in the paper's time convention
    (outgoing waves e^{i k r}, Section 2): du/dn = i k u on the face, k =
    omega/c at the boundary node, n the outward normal; the ghost value comes
    from the central difference of du/dn at the boundary node, and the grid's
    end nodes are unknowns of the problem (no Dirichlet ghost);
  * every face of such a problem is either sound-hard or absorbing, and a
    corner node takes the ghost rows of each of its axes.

Parity: pinned by the tests (plane-wave consistency of the interior stencil,
second-order consistency of the 1D stretched operator against its analytic
form, closed-form DST spectrum without a layer, Green's function decay with a
layer, and Im(eig) >= 0).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def pml_sigma(x: np.ndarray, n: int, L: int, h: float, omega: float,
              C: float = 20.0, power: int = 2) -> np.ndarray:
    """Imaginary part sigma(x) of the stretch s(x) = 1 + i sigma(x) along one axis
    of n nodes with L layer cells on each face (eq. pml-1d-s)."""
    x = np.asarray(x, dtype=float)
    sig = np.zeros_like(x)
    if L <= 0:
        return sig
    delta = L * h
    xa = L * h
    xb = (n - 1 - L) * h
    lo = x < xa
    hi = x > xb
    sig[lo] = C / (delta * omega) * ((xa - x[lo]) / delta) ** power
    sig[hi] = C / (delta * omega) * ((x[hi] - xb) / delta) ** power
    return sig


def axis_matrix(n: int, L: int, h: float, omega: float, C: float = 20.0,
                power: int = 2) -> sp.csr_matrix:
    """n x n three-point discretisation of (1/s) d/dx((1/s) du/dx) with zero
    Dirichlet ghosts.  Row i:  (1/s_i) [ (u_{i+1}-u_i)/(s_{i+1/2} h)
    - (u_i-u_{i-1})/(s_{i-1/2} h) ] / h."""
    x = np.arange(n) * h
    s_node = 1 + 1j * pml_sigma(x, n, L, h, omega, C, power)
    s_left = 1 + 1j * pml_sigma(x - h / 2, n, L, h, omega, C, power)
    s_right = 1 + 1j * pml_sigma(x + h / 2, n, L, h, omega, C, power)
    w_left = 1.0 / (s_node * s_left * h * h)     # coefficient of u_{i-1}
    w_right = 1.0 / (s_node * s_right * h * h)   # coefficient of u_{i+1}
    rows = []
    cols = []
    vals = []
    for i in range(n):
        rows.append(i); cols.append(i); vals.append(-(w_left[i] + w_right[i]))
        if i > 0:
            rows.append(i); cols.append(i - 1); vals.append(w_left[i])
        if i < n - 1:
            rows.append(i); cols.append(i + 1); vals.append(w_right[i])
    return sp.csr_matrix((np.array(vals, dtype=np.complex128), (rows, cols)), shape=(n, n))


def laplacian_pml(n, L, h, omega, C: float = 20.0, power: int = 2) -> sp.csr_matrix:
    """Sum over axes of the stretched second difference, as a Kronecker sum on
    the flattened index i + n0*(j + n1*k)."""
    n = tuple(n)
    N = int(np.prod(n))
    lap = sp.csr_matrix((N, N), dtype=np.complex128)
    for ax, nd in enumerate(n):
        Ld = axis_matrix(nd, L, h, omega, C, power)
        inner = int(np.prod(n[:ax]))        # faster axes
        outer = int(np.prod(n[ax + 1:]))    # slower axes
        lap = lap + sp.kron(sp.identity(outer), sp.kron(Ld, sp.identity(inner)))
    return lap.tocsr()


def ghost_axis_matrix(n: int, h: float) -> sp.csr_matrix:
    """n x n second difference of one axis whose end nodes are unknowns with a
    ghost node beyond each end.  Eliminating the ghost with the central
    difference of the face's normal derivative, du/dn = q u at the end node
    (q = 0 sound-hard, q = i k absorbing), gives u_ghost = u_inner + 2 h q u_end,
    so the end row (u_ghost - 2 u_end + u_inner)/h^2 becomes
    (2 u_inner - 2 u_end)/h^2 + (2 q/h) u_end.  This matrix holds the part
    without q; the absorbing part is absorbing_boundary_diag."""
    rows, cols, vals = [], [], []
    w = 1.0 / (h * h)
    for i in range(n):
        rows.append(i); cols.append(i); vals.append(-2.0 * w)
        if i > 0:
            rows.append(i); cols.append(i - 1); vals.append(2.0 * w if i == n - 1 else w)
        if i < n - 1:
            rows.append(i); cols.append(i + 1); vals.append(2.0 * w if i == 0 else w)
    return sp.csr_matrix((np.array(vals, dtype=np.complex128), (rows, cols)), shape=(n, n))


def absorbing_boundary_diag(prob) -> np.ndarray:
    """Per node, flattened: the sum over the absorbing faces the node lies on
    of (2/h) i k with k = omega/c at the node (the q u_end term of the ghost
    elimination, q = i k).  Sound-hard faces (prob.hard_faces, pairs (axis,
    side)) contribute nothing."""
    n = tuple(prob.n)
    c = prob.c_array()
    k = prob.omega / c  # shape n[::-1]
    total = np.zeros(tuple(reversed(n)), dtype=np.complex128)
    hard = set(tuple(f) for f in prob.hard_faces)
    for ax, nd in enumerate(n):
        for side, idx in ((0, 0), (1, nd - 1)):
            if (ax, side) in hard:
                continue
            sl = [slice(None)] * len(n)
            sl[len(n) - 1 - ax] = idx
            total[tuple(sl)] += (2.0 / prob.h) * 1j * k[tuple(sl)]
    return total.ravel()


def ghost_similarity(prob) -> np.ndarray:
    """Diagonal w of the similarity that symmetrises the ghost rows: 1/2 at an
    axis' end nodes, 1 elsewhere, multiplied over the axes.  W^{1/2} A W^{-1/2}
    has a real symmetric second difference (end-row weight 2/h^2 against 1/h^2
    becomes sqrt 2/h^2 both ways) plus a diagonal with Im >= 0."""
    n = tuple(prob.n)
    w = np.ones(tuple(reversed(n)))
    for ax, nd in enumerate(n):
        wa = np.ones(nd)
        wa[0] = wa[-1] = 0.5
        sh = [1] * len(n)
        sh[len(n) - 1 - ax] = nd
        w = w * wa.reshape(sh)
    return w.ravel()


def cap_potential(prob) -> np.ndarray:
    """W/c^2 per node, flattened (x fastest): 2 omega^2 times the sum over axes
    of the layer profile at the node's coordinate."""
    n = tuple(prob.n)
    total = np.zeros(tuple(reversed(n)))
    for ax, nd in enumerate(n):
        sig = pml_sigma(np.arange(nd) * prob.h, nd, prob.layer, prob.h, prob.omega, prob.pml_C, prob.pml_power)
        sh = [1] * len(n)
        sh[len(n) - 1 - ax] = nd
        total = total + sig.reshape(sh)
    return (2.0 * prob.omega ** 2 * total).ravel()


def _absorber(prob) -> str:
    a = getattr(prob, "absorber", "pml")
    if a not in ("pml", "cap", "abc"):
        raise ValueError("absorber must be 'pml', 'cap' or 'abc'")
    return a


def _ghost_laplacian(n, h) -> sp.csr_matrix:
    n = tuple(n)
    N = int(np.prod(n))
    lap = sp.csr_matrix((N, N), dtype=np.complex128)
    for ax, nd in enumerate(n):
        inner = int(np.prod(n[:ax]))
        outer = int(np.prod(n[ax + 1:]))
        lap = lap + sp.kron(sp.identity(outer), sp.kron(ghost_axis_matrix(nd, h), sp.identity(inner)))
    return lap.tocsr()


def inverse_c2(prob) -> np.ndarray:
    """Diagonal of D = 1/c^2, flattened."""
    c = prob.c_array().ravel().astype(float)
    return 1.0 / (c * c)


def helmholtz(prob, shift: float = 0.0) -> sp.csr_matrix:
    """A_s = omega^2 (1 + i s) D + Lap_PML; shift = 0 gives A itself.  With the
    absorbing potential: A_s = omega^2 (1 + i s) D + Lap + i W/c^2.  With
    boundary conditions (sound-hard and first-order absorbing faces, ghost
    points): A_s = omega^2 (1 + i s) D + Lap_ghost + absorbing_boundary_diag."""
    D = inverse_c2(prob)
    diag = prob.omega ** 2 * (1 + 1j * shift) * D
    if _absorber(prob) == "abc":
        return (_ghost_laplacian(prob.n, prob.h) + sp.diags(diag + absorbing_boundary_diag(prob))).tocsr()
    if _absorber(prob) == "cap":
        lap = laplacian_pml(prob.n, 0, prob.h, prob.omega)
        diag = diag + 1j * cap_potential(prob)
    else:
        lap = laplacian_pml(prob.n, prob.layer, prob.h, prob.omega, prob.pml_C, prob.pml_power)
    return (lap + sp.diags(diag)).tocsr()


def rhs(f: np.ndarray) -> np.ndarray:
    """b = -f (eq. helmholtz)."""
    return -np.asarray(f, dtype=np.complex128).ravel()


def apply_rows(prob, shift: float, x: np.ndarray, points: np.ndarray) -> np.ndarray:
    """(A_s x) at selected flat indices, computed one row at a time from the
    stencil definition (for spot checks at sizes where assembling A is too big).
    x: flat complex vector; points: flat indices."""
    n = prob.n
    d = len(n)
    h, om, L = prob.h, prob.omega, prob.layer
    cap = _absorber(prob) == "cap"
    abc = _absorber(prob) == "abc"
    hard = set(tuple(f) for f in getattr(prob, "hard_faces", ()))
    D = inverse_c2(prob)
    out = np.empty(len(points), dtype=np.complex128)
    strides = [int(np.prod(n[:ax])) for ax in range(d)]
    for q, p in enumerate(np.asarray(points, dtype=np.int64)):
        idx = [(p // strides[ax]) % n[ax] for ax in range(d)]
        acc = om * om * (1 + 1j * shift) * D[p] * x[p]
        for ax in range(d):
            i = idx[ax]
            if abc:
                # ghost rows at the ends; the absorbing faces add (2/h) i omega/c
                wl = 0.0 if i == 0 else (2.0 if i == n[ax] - 1 else 1.0) / (h * h)
                wr = 0.0 if i == n[ax] - 1 else (2.0 if i == 0 else 1.0) / (h * h)
                um = x[p - strides[ax]] if i > 0 else 0.0
                up = x[p + strides[ax]] if i < n[ax] - 1 else 0.0
                acc += wl * um + wr * up - (2.0 / (h * h)) * x[p]
                for side, end in ((0, 0), (1, n[ax] - 1)):
                    if i == end and (ax, side) not in hard:
                        acc += (2.0 / h) * 1j * om * np.sqrt(D[p]) * x[p]
                continue
            xi = i * h
            sig = pml_sigma(np.array([xi - h / 2, xi, xi + h / 2]), n[ax], L, h, om, prob.pml_C, prob.pml_power)
            if cap:
                # the potential's share of this axis; no stretch
                acc += 1j * 2.0 * om * om * sig[1] * x[p]
                sig = np.zeros(3)
            s0 = 1 + 1j * sig[1]
            sl = 1 + 1j * sig[0]
            sr = 1 + 1j * sig[2]
            wl = 1 / (s0 * sl * h * h)
            wr = 1 / (s0 * sr * h * h)
            um = x[p - strides[ax]] if i > 0 else 0.0
            up = x[p + strides[ax]] if i < n[ax] - 1 else 0.0
            acc += wl * um + wr * up - (wl + wr) * x[p]
        out[q] = acc
    return out
