"""Pins for the oracle's matrix functions (oracle/matfun.py) and the identities
of Section 3 (inverse identity, truncated preconditioner spectrum)."""
import math

import numpy as np
import pytest
import scipy.linalg as sla

import workloads as wl
from oracle import matfun, operator as op


def _psi_closed(l, z):
    z = complex(z)
    if l == 1:
        return np.expm1(z) / z if z.imag == 0 else (np.exp(z) - 1) / z
    return (np.exp(z) - 1 - z) / z**2


@pytest.mark.parametrize("z", [0.3 + 0.2j, -0.9j, 0.999, 1.5 - 2j, 25j, -30.0, 0.02 + 0.01j])
@pytest.mark.parametrize("l", [1, 2])
def test_psi_scalar(z, l):
    ref = _psi_closed(l, z)
    tol = 1e-13 if abs(z) > 0.1 else 1e-9  # closed forms themselves cancel near 0
    assert abs(matfun.psi_scalar(l, z) - ref) <= tol * abs(ref)


def test_psi_scalar_small_argument_series():
    # psi_1(z) -> 1 + z/2 + z^2/6 as z -> 0 (no cancellation in the series branch)
    z = 1e-7 + 2e-7j
    assert abs(matfun.psi_scalar(1, z) - (1 + z / 2 + z * z / 6)) < 1e-20
    assert abs(matfun.psi_scalar(0, 0.5) - math.exp(0.5)) < 1e-15


def _tiny(shift=0.0, dim=2, inh=False):
    n = (10, 9, 8)[:dim]
    prob = wl.small_problem(n, layer=2, ppw=10, inhomogeneous=inh, seed=1)
    t = prob.default_t()
    return prob, op.helmholtz(prob, shift), t


def test_exp_routes_agree_dense_vs_expm_multiply():
    prob, As, t = _tiny(shift=0.1, inh=True)
    v = wl.random_vector(prob.npts, 3)
    E = matfun.exp_dense(As, t)
    assert np.linalg.norm(matfun.exp_action(As, t, v) - E @ v) <= 1e-12 * np.linalg.norm(E @ v)


def test_phi1_routes_agree_and_match_integral():
    # P7: t psi_1(i t A) = int_0^t exp(i tau A) d tau (Section 3.1); Gauss-Legendre in tau
    prob, As, t = _tiny(shift=0.05, dim=3)
    v = wl.random_vector(prob.npts, 4)
    P = matfun.phi1_dense(As, t)
    got = matfun.phi1_action(As, t, v)
    assert np.linalg.norm(got - P @ v) <= 1e-12 * np.linalg.norm(P @ v)
    xg, wg = np.polynomial.legendre.leggauss(60)
    Ad = As.toarray()
    lam, X = np.linalg.eig(Ad)
    Xi = np.linalg.inv(X)
    integ = np.zeros(prob.npts, dtype=complex)
    # split [0, t] into panels to resolve the oscillation
    panels = 64
    for p in range(panels):
        a, b = p * t / panels, (p + 1) * t / panels
        for x, w in zip(xg, wg):
            tau = 0.5 * (b - a) * x + 0.5 * (a + b)
            integ += 0.5 * (b - a) * w * (X @ (np.exp(1j * tau * lam) * (Xi @ v)))
    assert np.linalg.norm(t * (P @ v) - integ) <= 1e-8 * np.linalg.norm(integ)


def test_phi1_dense_closed_form_when_invertible():
    # psi_1(M) = M^{-1}(e^M - I) for invertible M
    prob, As, t = _tiny(shift=0.02)
    M = 1j * t * As.toarray()
    ref = np.linalg.solve(M, sla.expm(M) - np.eye(M.shape[0]))
    P = matfun.phi1_dense(As, t)
    assert np.abs(P - ref).max() <= 1e-10 * np.abs(ref).max()


def test_dst_closed_form_matches_expm_multiply_without_layer():
    # P4: homogeneous, no layer: exp(itA_s) is diagonal in the DST-I basis
    prob = wl.small_problem((48, 40), layer=0)
    s = 0.04
    As = op.helmholtz(prob, s)
    t = prob.default_t()
    v = wl.random_vector(prob.npts, 5)
    ref = matfun.exp_action_dst(prob.n, prob.h, prob.omega**2 * (1 + 1j * s), t, v)
    got = matfun.exp_action(As, t, v)
    assert np.linalg.norm(got - ref) <= 1e-11 * np.linalg.norm(ref)


def test_dst_closed_form_3d_matches_dense():
    prob = wl.small_problem((7, 6, 5), layer=0)
    As = op.helmholtz(prob, 0.1)
    t = prob.default_t()
    v = wl.random_vector(prob.npts, 6)
    ref = matfun.exp_dense(As, t) @ v
    got = matfun.exp_action_dst(prob.n, prob.h, prob.omega**2 * (1 + 0.1j), t, v)
    assert np.linalg.norm(got - ref) <= 1e-12 * np.linalg.norm(ref)


def test_inverse_identity():
    # P1 (eq. magic-inverse / inverse-1): A^{-1} = -i t (I - e^{itA})^{-1} psi_1(itA)
    prob, A, t = _tiny(shift=0.0)
    Ad = A.toarray()
    E = matfun.exp_dense(A, t)
    P = matfun.phi1_dense(A, t)
    lhs = -1j * t * np.linalg.solve(np.eye(Ad.shape[0]) - E, P)
    Ainv = np.linalg.inv(Ad)
    assert np.abs(lhs - Ainv).max() <= 1e-10 * np.abs(Ainv).max()


@pytest.mark.parametrize("N", [0, 2, 5])
def test_truncated_preconditioner_spectrum(N):
    # P2 (Section 3.2 and Thm 3.1): eig(P_N A) = 1 - exp(i(N+1) t lambda_k), inside the
    # disk |z-1| <= exp(-(N+1) t lambda*), lambda* = min Im lambda_k (attained).
    prob, A, t = _tiny(shift=0.0)
    Ad = A.toarray()
    E = matfun.exp_dense(A, t)
    P = matfun.phi1_dense(A, t)
    S = np.zeros_like(E)
    En = np.eye(E.shape[0], dtype=complex)
    for _ in range(N + 1):
        S = S + En
        En = En @ E
    PN = -1j * t * S @ P
    mu = np.linalg.eigvals(PN @ Ad)
    lam = np.linalg.eigvals(Ad)
    pred = 1 - np.exp(1j * (N + 1) * t * lam)
    d = np.abs(mu[:, None] - pred[None, :]).min(axis=1)
    assert d.max() <= 1e-9
    lam_star = lam.imag.min()
    radius = math.exp(-(N + 1) * t * lam_star)
    assert np.abs(mu - 1).max() <= radius * (1 + 1e-9) + 1e-12
    assert np.abs(mu - 1).max() >= radius * (1 - 1e-6)


def test_phi2_routes_agree_and_match_double_integral():
    # t^2 psi_2(i t A) v = int_0^t (t - tau) exp(i tau A) v d tau, the double time
    # integral of Section 3.1 with the inner integral done; Gauss-Legendre in tau over
    # the eigendecomposition (independent of the augmented-exponential routes)
    prob, As, t = _tiny(shift=0.05, dim=2, inh=True)
    v = wl.random_vector(prob.npts, 7)
    P2 = matfun.phi2_dense(As, t)
    got = matfun.phi2_action(As, t, v)
    assert np.linalg.norm(got - P2 @ v) <= 1e-12 * np.linalg.norm(P2 @ v)
    xg, wg = np.polynomial.legendre.leggauss(60)
    lam, X = np.linalg.eig(As.toarray())
    c = np.linalg.solve(X, v)
    integ = np.zeros(prob.npts, dtype=complex)
    panels = 64
    for p in range(panels):
        a, b = p * t / panels, (p + 1) * t / panels
        for x, w in zip(xg, wg):
            tau = 0.5 * (b - a) * x + 0.5 * (a + b)
            integ += 0.5 * (b - a) * w * (t - tau) * (X @ (np.exp(1j * tau * lam) * c))
    assert np.linalg.norm(t * t * (P2 @ v) - integ) <= 1e-8 * np.linalg.norm(integ)


def test_phi2_dense_closed_form_when_invertible():
    # psi_2(M) = M^{-2}(e^M - I - M) for invertible M (Definition psi)
    prob, As, t = _tiny(shift=0.02)
    M = 1j * t * As.toarray()
    I = np.eye(M.shape[0])
    ref = np.linalg.solve(M, np.linalg.solve(M, sla.expm(M) - I - M))
    P2 = matfun.phi2_dense(As, t)
    assert np.abs(P2 - ref).max() <= 1e-9 * np.abs(ref).max()


def test_phi2_action_matches_dst_closed_form_without_layer():
    # no layer: psi_2(i t A_s) is diagonal in the DST-I basis with entries psi_2(i t lambda_k)
    import scipy.fft
    prob = wl.small_problem((24, 20), layer=0)
    s = 0.04
    As = op.helmholtz(prob, s)
    t = prob.default_t()
    v = wl.random_vector(prob.npts, 8)
    shape = tuple(reversed(prob.n))
    lam = np.full(shape, prob.omega**2 * (1 + 1j * s))
    lam = lam + matfun.dirichlet_eigs(prob.n[0], prob.h)[None, :] + matfun.dirichlet_eigs(prob.n[1], prob.h)[:, None]
    W = scipy.fft.dstn(v.reshape(shape), type=1, norm="ortho")
    W = W * np.vectorize(lambda z: matfun.psi_scalar(2, 1j * t * z))(lam)
    ref = scipy.fft.idstn(W, type=1, norm="ortho").ravel()
    got = matfun.phi2_action(As, t, v)
    assert np.linalg.norm(got - ref) <= 1e-11 * np.linalg.norm(ref)


@pytest.mark.parametrize("shift", [0.0, 0.1])
def test_second_inverse_identity(shift):
    # Section 3.1: A^{-1} = -i t (I - psi_1(i t A))^{-1} psi_2(i t A)
    prob, A, t = _tiny(shift=shift, inh=True)
    Ad = A.toarray()
    P1 = matfun.phi1_dense(A, t)
    P2 = matfun.phi2_dense(A, t)
    lhs = -1j * t * np.linalg.solve(np.eye(Ad.shape[0]) - P1, P2)
    Ainv = np.linalg.inv(Ad)
    assert np.abs(lhs - Ainv).max() <= 1e-9 * np.abs(Ainv).max()


def test_time_averaged_map_contraction_per_mode():
    # Theorem 2.2's per-mode factor: for Im(lambda) >= 0 the eigenvalue psi_1(i t lambda)
    # of the time-averaged map has modulus at most min(1, 2 / (|lambda| t))
    prob, A, t = _tiny(shift=0.0)
    lam = np.linalg.eigvals(A.toarray())
    assert lam.imag.min() > 0
    mu = np.linalg.eigvals(matfun.phi1_dense(A, t))
    bound = np.minimum(1.0, 2.0 / (np.abs(lam) * t))
    # match each computed eigenvalue of psi_1(i t A) to psi_1(i t lambda_k)
    pred = np.array([matfun.psi_scalar(1, 1j * t * z) for z in lam])
    d = np.abs(mu[:, None] - pred[None, :])
    assert d.min(axis=1).max() <= 1e-9
    assert np.all(np.abs(pred) <= bound * (1 + 1e-12))
    assert np.abs(mu).max() < 1.0
