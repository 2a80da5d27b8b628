"""Pins for the oracle's operator assembly (oracle/operator.py)."""
import dataclasses
import math

import numpy as np
import pytest

import workloads as wl
from oracle import operator as op
from oracle import krylov, matfun
from scipy.sparse.linalg import splu


def test_dirichlet_eigs_match_dense_second_difference():
    # textbook: eig of (1/h^2) tridiag(1,-2,1) are -4 sin^2(k pi/(2(n+1)))/h^2
    n, h = 17, 0.1
    T = (np.diag(-2 * np.ones(n)) + np.diag(np.ones(n - 1), 1) + np.diag(np.ones(n - 1), -1)) / h**2
    ev = np.sort(np.linalg.eigvalsh(T))
    assert np.allclose(np.sort(matfun.dirichlet_eigs(n, h)), ev, rtol=1e-12, atol=1e-9)


def test_no_layer_operator_is_dirichlet_laplacian_plus_diagonal():
    prob = wl.small_problem((9, 7), layer=0)
    A = op.helmholtz(prob, shift=0.3).toarray()
    n0, n1 = prob.n
    h = prob.h
    T0 = (np.diag(-2 * np.ones(n0)) + np.diag(np.ones(n0 - 1), 1) + np.diag(np.ones(n0 - 1), -1)) / h**2
    T1 = (np.diag(-2 * np.ones(n1)) + np.diag(np.ones(n1 - 1), 1) + np.diag(np.ones(n1 - 1), -1)) / h**2
    ref = np.kron(np.eye(n1), T0) + np.kron(T1, np.eye(n0)) + prob.omega**2 * (1 + 0.3j) * np.eye(n0 * n1)
    assert np.abs(A - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("dim", [2, 3])
def test_plane_wave_interior_residual_vanishes(dim):
    # P5: e^{i k.x} with sum_d 4 sin^2(k_d h/2)/h^2 = omega^2/c^2 is annihilated by
    # the interior stencil.  c = 2 (constant) so a D = c^2 slip would show.
    n = (40, 36, 30)[:dim]
    prob = wl.small_problem(n, layer=6, ppw=12)
    prob.c = np.full(prob.shape, 2.0)
    h, om, c = prob.h, prob.omega, 2.0
    dirs = np.array([0.6, 0.5, 0.62][:dim])
    dirs = dirs / np.linalg.norm(dirs)
    # solve for |k|: sum 4 sin^2(k d_i h/2)/h^2 = (om/c)^2
    lo, hi = 0.0, math.pi / h
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        val = np.sum(4 * np.sin(mid * dirs * h / 2) ** 2) / h**2
        lo, hi = (mid, hi) if val < (om / c) ** 2 else (lo, mid)
    k = 0.5 * (lo + hi) * dirs
    axes = [np.arange(m) * h for m in n]
    grids = np.meshgrid(*reversed(axes), indexing="ij")
    phase = sum(g * kk for g, kk in zip(grids, reversed(k)))
    u = np.exp(1j * phase).ravel()
    A = op.helmholtz(prob, 0.0)
    r = (A @ u).reshape(prob.shape)
    L = prob.layer
    inner = tuple(slice(L + 2, m - L - 2) for m in reversed(n))
    assert np.abs(r[inner]).max() <= 1e-9 * (om / c) ** 2
    # and the residual is O(1) relative if omega^2 is dropped (sanity of the pin)
    assert np.abs((A @ u - om**2 / c**2 * u).reshape(prob.shape)[inner]).max() > 0.5 * (om / c) ** 2


def _analytic_stretched(x, u, du, d2u, sig, dsig):
    s = 1 + 1j * sig
    ds = 1j * dsig
    return (1 / s) * (d2u / s - du * ds / s**2)


def test_pml_axis_operator_second_order_consistent():
    # (1/s) d/dx((1/s) du/dx) on u vanishing at the ghost nodes; error must fall
    # like h^2 where the profile is smooth (quadratic profile: sigma' continuous).
    errs = []
    for n in (161, 321):
        h = 1.0 / (n - 1)
        L = (n - 1) // 8
        omega = 40.0
        C = 20.0
        A = op.axis_matrix(n, L, h, omega, C).toarray()
        x = np.arange(n) * h
        a, b = -h, n * h
        w = math.pi / (b - a)
        beta = 7.0
        u = np.sin(w * (x - a)) * np.exp(1j * beta * x)
        du = (w * np.cos(w * (x - a)) + 1j * beta * np.sin(w * (x - a))) * np.exp(1j * beta * x)
        d2u = (-w * w * np.sin(w * (x - a)) + 2j * beta * w * np.cos(w * (x - a))
               - beta * beta * np.sin(w * (x - a))) * np.exp(1j * beta * x)
        delta = L * h
        xa, xb = L * h, (n - 1 - L) * h
        sig = op.pml_sigma(x, n, L, h, omega, C)
        dsig = np.where(x < xa, -2 * C / (delta * omega) * (xa - x) / delta**2,
                        np.where(x > xb, 2 * C / (delta * omega) * (x - xb) / delta**2, 0.0))
        ref = _analytic_stretched(x, u, du, d2u, sig, dsig)
        got = A @ u
        mask = (np.abs(x - xa) > 2.5 * h) & (np.abs(x - xb) > 2.5 * h)
        errs.append(np.abs(got - ref)[mask].max() / np.abs(ref).max())
    assert errs[1] < errs[0] / 3.0, errs
    assert errs[1] < 2e-3  # a swapped left/right half-node stretch gives ~1.2


def test_pml_sigma_profile_values():
    # eq. pml-1d-s: zero inside, C/(delta omega) at distance delta, quadratic between
    n, L, h, om, C = 41, 8, 0.025, 50.0, 20.0
    x = np.arange(n) * h
    sig = op.pml_sigma(x, n, L, h, om, C)
    assert np.all(sig[L:n - L] == 0)
    assert sig[0] == pytest.approx(C / (L * h * om))
    assert sig[L // 2] == pytest.approx(C / (L * h * om) * 0.25)
    assert sig[n - 1] == pytest.approx(sig[0])


def test_spectrum_upper_half_plane_and_shift():
    # P3: min Im eig(A) >= 0 with the layer; homogeneous: eig(A_s) = eig(A) + i omega^2 s
    prob = wl.small_problem((24, 20), layer=5)
    A = op.helmholtz(prob, 0.0).toarray()
    ev = np.linalg.eigvals(A)
    assert ev.imag.min() > -1e-8 * np.abs(ev).max()
    s = 0.05
    evs = np.linalg.eigvals(op.helmholtz(prob, s).toarray())
    shifted = ev + 1j * prob.omega**2 * s
    d = np.abs(np.sort_complex(evs)[:, None] - shifted[None, :]).min(axis=1)
    assert d.max() <= 1e-8 * np.abs(ev).max()


@pytest.mark.parametrize("absorber", ["pml", "cap"])
def test_apply_rows_matches_assembled_matrix(absorber):
    prob = dataclasses.replace(wl.small_problem((13, 11, 9), layer=3, inhomogeneous=True, seed=3),
                               absorber=absorber)
    x = wl.random_vector(prob.npts, 7)
    As = op.helmholtz(prob, 0.07)
    pts = np.array([0, 5, 100, 500, prob.npts - 1, 13 * 11 * 4 + 13 * 5 + 6])
    assert np.allclose(op.apply_rows(prob, 0.07, x, pts), (As @ x)[pts], rtol=1e-13, atol=0)


def test_greens_function_2d_outgoing():
    # P6: delta source, homogeneous, with the layer: u ~ (i/4) H0^(1)(k r)
    # (e^{-i omega t} convention).  ppw 30 keeps dispersion error ~1%.
    from scipy.special import hankel1
    n = 161
    prob = wl.small_problem((n, n), layer=30, ppw=30)
    f = wl.delta_source(prob, (n // 2, n // 2))
    u = op.helmholtz(prob, 0.0)
    import scipy.sparse.linalg as spla
    sol = spla.splu(u.tocsc()).solve(op.rhs(f)).reshape(prob.shape)
    h = prob.h
    y, x = np.meshgrid(np.arange(n) * h, np.arange(n) * h, indexing="ij")
    r = np.hypot(x - (n // 2) * h, y - (n // 2) * h)
    ann = (r > 10 * h) & (r < 0.3)
    green = 0.25j * hankel1(0, prob.omega * r[ann])
    rel = np.linalg.norm(sol[ann] - green) / np.linalg.norm(green)
    assert rel < 0.05, rel
    # incoming (H0^(2)) must be far off: guards the sign of the layer
    wrong = 0.25j * np.conj(hankel1(0, prob.omega * r[ann]))
    assert np.linalg.norm(sol[ann] - wrong) / np.linalg.norm(wrong) > 0.5


def _cap(prob):
    return dataclasses.replace(prob, absorber="cap")


def test_cap_eigenvalues_follow_the_potential():
    # Section 2.1 proposition, discrete form: A = omega^2 D + Lap + i W/c^2 with Lap real
    # symmetric, so for A phi = lambda phi, Im(lambda) = sum (W/c^2)|phi|^2 / sum |phi|^2 >= 0
    prob = _cap(wl.small_problem((12, 10), layer=3, ppw=10, inhomogeneous=True, seed=5))
    A = op.helmholtz(prob, 0.0).toarray()
    lam, V = np.linalg.eig(A)
    W = op.cap_potential(prob)
    assert W.min() == 0.0 and W.max() > 0.0
    quot = (W[:, None] * np.abs(V) ** 2).sum(axis=0) / (np.abs(V) ** 2).sum(axis=0)
    assert np.abs(lam.imag - quot).max() <= 1e-9 * W.max()
    assert lam.imag.min() > 0.0
    # the shift adds omega^2 s D to the same quotient
    As = op.helmholtz(prob, 0.2).toarray()
    lam_s, V_s = np.linalg.eig(As)
    Dd = op.inverse_c2(prob)
    quot_s = ((W + prob.omega**2 * 0.2 * Dd)[:, None] * np.abs(V_s) ** 2).sum(axis=0) / (np.abs(V_s) ** 2).sum(axis=0)
    assert np.abs(lam_s.imag - quot_s).max() <= 1e-9 * W.max()


def test_cap_is_the_plain_laplacian_plus_potential():
    # no stretch: off-diagonal entries are 1/h^2 everywhere, the layer only in the diagonal
    prob = _cap(wl.small_problem((9, 8, 7), layer=2, ppw=10, inhomogeneous=True, seed=6))
    A = op.helmholtz(prob, 0.0).tocoo()
    off = A.row != A.col
    assert np.allclose(A.data[off], 1.0 / prob.h**2, rtol=0, atol=1e-9 / prob.h**2)
    plain = op.helmholtz(dataclasses.replace(prob, layer=0), 0.0).toarray()
    diff = np.diag(A.toarray() - plain)
    assert np.allclose(diff, 1j * op.cap_potential(prob), rtol=1e-14, atol=0)


def test_cap_decays_like_the_pml_inside_the_layer():
    # the potential's scale: a wave crossing the layer loses amplitude at the stretch's
    # rate, exp(-omega int sigma) to first order; with half the potential it would keep
    # e^{+1.1} more amplitude at depth 30 cells here
    import scipy.sparse.linalg as spla
    n, L = 161, 40
    sols = {}
    for absorber in ("pml", "cap"):
        prob = dataclasses.replace(wl.small_problem((n, n), layer=L, ppw=30), absorber=absorber)
        f = wl.delta_source(prob, (n // 2, n // 2))
        sols[absorber] = spla.splu(op.helmholtz(prob, 0.0).tocsc()).solve(op.rhs(f)).reshape(prob.shape)
    row = n // 2
    for depth in (0, 10, 20, 30):
        i = n - 1 - L + depth
        env = {k: np.sqrt(np.mean(np.abs(v[row, i - 7:i + 8]) ** 2)) for k, v in sols.items()}
        assert 0.9 < env["cap"] / env["pml"] < 1.1, (depth, env)
    # the PML itself decays by about exp(-omega int sigma) over those 30 cells
    prob = wl.small_problem((n, n), layer=L, ppw=30)
    x = np.arange(n) * prob.h
    sig = op.pml_sigma(x, n, L, prob.h, prob.omega)
    i0, i1 = n - 1 - L, n - 1 - L + 30
    pred = prob.omega * sig[i0:i1].sum() * prob.h
    env0 = np.sqrt(np.mean(np.abs(sols["pml"][row, i0 - 7:i0 + 8]) ** 2))
    env1 = np.sqrt(np.mean(np.abs(sols["pml"][row, i1 - 7:i1 + 8]) ** 2))
    # the 2D field also spreads (amplitude ~ r^-1/2) over that distance
    spread = 0.5 * np.log((i1 - n // 2) / (i0 - n // 2))
    assert abs(np.log(env0 / env1) - spread - pred) <= 0.25 * pred


def test_greens_function_2d_outgoing_with_cap():
    # as P6, with the absorbing potential (a wider layer: the potential reflects more)
    from scipy.special import hankel1
    import scipy.sparse.linalg as spla
    n, L = 161, 40
    prob = dataclasses.replace(wl.small_problem((n, n), layer=L, ppw=30), absorber="cap")
    f = wl.delta_source(prob, (n // 2, n // 2))
    sol = spla.splu(op.helmholtz(prob, 0.0).tocsc()).solve(op.rhs(f)).reshape(prob.shape)
    h = prob.h
    y, x = np.meshgrid(np.arange(n) * h, np.arange(n) * h, indexing="ij")
    r = np.hypot(x - (n // 2) * h, y - (n // 2) * h)
    ann = (r > 10 * h) & (r < 0.22)
    green = 0.25j * hankel1(0, prob.omega * r[ann])
    assert np.linalg.norm(sol[ann] - green) / np.linalg.norm(green) < 0.05
    wrong = 0.25j * np.conj(hankel1(0, prob.omega * r[ann]))
    assert np.linalg.norm(sol[ann] - wrong) / np.linalg.norm(wrong) > 0.5


# ---------------------------------------------------------------------------
# Boundary conditions in place of a layer (Section 4.3.4): a sound-hard face
# and first-order absorbing faces by ghost points.


def _abc_1d(N, h, omega, c, hard_left=True):
    return wl.Problem("abc1d", (N,), h, omega, 0, None, c, absorber="abc",
                      hard_faces=((0, 0),) if hard_left else ())


@pytest.mark.parametrize("ppw", [6.0, 10.0, 20.0])
def test_abc_1d_reflection_closed_form(ppw):
    """A plane wave driven from the left meets the absorbing right end.  The
    interior rows hold exactly for u_j = a z^j + b z^-j with z = e^{i xi h},
    2 - 2 cos(xi h) = (k h)^2; the ghost row u_N = u_{N-2} + 2 i h k u_{N-1}
    then gives |b/a| = |sin(xi h) - k h| / (sin(xi h) + k h) = tan^2(xi h / 4).
    c = 2 so that k = omega / c is tested (a k from 1/c^2 or a flipped sign,
    which reflects more than it sends, fails)."""
    N, h, c = 60, 1.0 / 59, 2.0
    k = 2 * np.pi / (ppw * h)
    omega = k * c
    prob = _abc_1d(N, h, omega, c)
    A = op.helmholtz(prob, 0.0).tolil()
    A[0, :] = 0
    A[0, 0] = 1.0  # drive u_0 = 1
    rhs = np.zeros(N, dtype=complex)
    rhs[0] = 1.0
    u = splu(A.tocsc()).solve(rhs)
    xi_h = np.arccos(1 - (k * h) ** 2 / 2)
    z = np.exp(1j * xi_h)
    M = np.array([[z ** 1, z ** -1], [z ** 2, z ** -2]])
    a, b = np.linalg.solve(M, u[1:3])
    # the two-mode form holds on every node the interior rows cover
    j = np.arange(N)
    assert np.allclose(a * z ** j + b * z ** -j, u, rtol=0, atol=1e-10 * abs(a))
    assert abs(abs(b / a) - np.tan(xi_h / 4) ** 2) <= 1e-9
    assert abs(b / a) < 0.1


def test_abc_sound_hard_face_is_a_mirror():
    """A sound-hard face is a mirror: the problem on a half domain with the
    hard face at y = 0 equals, on its nodes, the problem on the domain
    reflected across that face (speed and source mirrored, all faces
    absorbing), because the ghost value u_{-1} = u_1 is what the symmetric
    solution has there."""
    rng = np.random.default_rng(5)
    nx, ny = 15, 9
    h = 1.0 / 14
    omega = wl.omega_for(8, h)
    c_half = rng.uniform(1.0, 2.0, (ny, nx))
    f_half = rng.standard_normal((ny, nx)) + 1j * rng.standard_normal((ny, nx))
    half = wl.Problem("half", (nx, ny), h, omega, 0, c_half, absorber="abc", hard_faces=((1, 0),))
    full_rows = np.concatenate([np.arange(ny - 1, 0, -1), np.arange(ny)])  # mirrored row index |j|
    full = wl.Problem("full", (nx, 2 * ny - 1), h, omega, 0, c_half[full_rows], absorber="abc")
    s = 0.05
    u_half = krylov.direct_solve(half, f_half.ravel(), shift=s).reshape(ny, nx)
    u_full = krylov.direct_solve(full, f_half[full_rows].ravel(), shift=s).reshape(2 * ny - 1, nx)
    assert np.linalg.norm(u_full[ny - 1:] - u_half) <= 1e-11 * np.linalg.norm(u_half)
    # with the face absorbing instead, the two differ at O(1)
    half_abs = wl.Problem("half-abs", (nx, ny), h, omega, 0, c_half, absorber="abc")
    u_abs = krylov.direct_solve(half_abs, f_half.ravel(), shift=s).reshape(ny, nx)
    assert np.linalg.norm(u_full[ny - 1:] - u_abs) > 1e-2 * np.linalg.norm(u_half)


def test_abc_spectrum_and_symmetrised_field_of_values():
    """The paper states that every eigenvalue of the matrix from these
    conditions has a non-negative imaginary part.  The diagonal similarity
    W^{1/2} A W^{-1/2} (w = 1/2 at each axis' end nodes) is complex symmetric
    with a real second difference, and its skew-Hermitian part is a diagonal
    >= 0, so its field of values lies in the upper half-plane: the bound the
    library's schedule design takes, times the condition number of the
    similarity."""
    rng = np.random.default_rng(8)
    n = (9, 8)
    h = 1.0 / 8
    c = rng.uniform(1.0, 3.0, (n[1], n[0]))
    prob = wl.Problem("abc-small", n, h, wl.omega_for(6, h), 0, c, absorber="abc", hard_faces=((1, 0),))
    A = op.helmholtz(prob, 0.0).toarray()
    ev = np.linalg.eigvals(A)
    scale = np.abs(ev).max()
    assert ev.imag.min() >= -1e-12 * scale
    ev_s = np.linalg.eigvals(op.helmholtz(prob, 0.1).toarray())
    assert ev_s.imag.min() > 0
    w = op.ghost_similarity(prob)
    S = np.sqrt(w)[:, None] * A / np.sqrt(w)[None, :]
    assert np.abs(S - S.T).max() <= 1e-12 * np.abs(S).max()
    K = (S - S.conj().T) / 2j
    assert np.linalg.eigvalsh(K).min() >= -1e-12 * scale
    # the absorbing faces are what makes it non-Hermitian: with every face hard
    # the matrix is similar to a real symmetric one (real spectrum)
    hard_all = wl.Problem("hard", n, h, prob.omega, 0, c, absorber="abc",
                          hard_faces=((0, 0), (0, 1), (1, 0), (1, 1)))
    assert np.abs(np.linalg.eigvals(op.helmholtz(hard_all, 0.0).toarray()).imag).max() <= 1e-9 * scale


def test_abc_rows_against_the_assembled_matrix():
    rng = np.random.default_rng(9)
    n = (7, 6, 5)
    prob = wl.Problem("abc3", n, 1.0 / 6, 20.0, 0, rng.uniform(1, 2, n[::-1]), absorber="abc",
                      hard_faces=((2, 0),))
    x = rng.standard_normal(prob.npts) + 1j * rng.standard_normal(prob.npts)
    A = op.helmholtz(prob, 0.2)
    pts = np.arange(prob.npts)
    assert np.abs(op.apply_rows(prob, 0.2, x, pts) - A @ x).max() <= 1e-12 * np.abs(A @ x).max()
