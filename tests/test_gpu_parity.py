"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Sizes are small enough for the oracle yet span several 64x4 workgroup tiles
with ragged edges in every axis.  Bars: FP64 paths <= 1e-10 relative (actions
<= 1e-11), complex-float forms <= 1e-5, iteration counts within +-1."""
import numpy as np
import pytest

import workloads as wl
from oracle import krylov, matfun, operator as op

from gpu_util import announce, rel, to_dev, to_host

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2506_03617_amd as mxp  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    c = mxp.Context(0)
    yield c
    c.close()


CASES = {
    "2d-homog": dict(n=(67, 45), layer=8, inh=False),
    "2d-inh": dict(n=(67, 45), layer=8, inh=True),
    "3d-homog": dict(n=(33, 29, 21), layer=4, inh=False),
    "3d-inh": dict(n=(33, 29, 21), layer=4, inh=True),
    # z chunks of 16 planes with a ragged last chunk, ragged x and y tiles
    "3d-ragged": dict(n=(70, 9, 37), layer=3, inh=True),
}


def make(name, ppw=10.0):
    c = CASES[name]
    return wl.small_problem(c["n"], layer=c["layer"], ppw=ppw, inhomogeneous=c["inh"], seed=7, name=name)


def forced_precond_parity(P, As, o, r, tol, inner="gmres", form="exp"):
    """One preconditioner apply compared element by element with the oracle's
    at the same inner iteration count.  The count is fixed on both sides: the
    oracle's natural count k under o.fprtol (checked against the library's to
    +-1), then both run exactly k inner iterations (max_inner = k, fprtol
    1e-14) and w is compared at `tol`."""
    import copy
    rd = to_dev(r)
    wd = torch.empty_like(rd)
    its = mxp.mxp_apply_precond(P, o, rd, wd)
    natural = krylov.precond_apply(As, o.t, r, o.fprtol, inner=inner, form=form)
    assert abs(its - natural.inner_iterations) <= 1
    k = max(natural.inner_iterations, 1)
    of = copy.copy(o)
    of.fprtol = 1e-14
    of.max_inner = k
    its_f = mxp.mxp_apply_precond(P, of, rd, wd)
    ref = krylov.precond_apply(As, o.t, r, 1e-14, maxit=k, inner=inner, form=form)
    assert its_f == k == ref.inner_iterations
    err = rel(to_host(wd), ref.w)
    assert err <= tol, (k, err)
    return its, natural.inner_iterations


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("dt", ["c128", "c64"])
def test_apply_A(ctx, name, dt):
    prob = make(name)
    announce("apply_A", name, dt, prob.n)
    P = mxp.Problem(ctx, prob)
    s = prob.default_shift()
    x = wl.random_vector(prob.npts, 1)
    tdt = torch.complex128 if dt == "c128" else torch.complex64
    xd = to_dev(x, tdt)
    yd = torch.empty_like(xd)
    mxp.mxp_apply_A(P, s, xd, yd)
    torch.cuda.synchronize()
    xr = to_host(xd)  # the rounded input actually used
    As = op.helmholtz(prob, s)
    ref = As @ xr
    bound = abs(As) @ np.abs(xr)
    eps = 2.0**-53 if dt == "c128" else 2.0**-24
    assert np.linalg.norm(to_host(yd) - ref) <= 16 * eps * np.linalg.norm(bound)


@pytest.mark.parametrize("name", ["2d-homog", "2d-inh", "3d-inh"])
def test_apply_A_smooth_input_cancellation(ctx, name):
    # smooth x: the Laplacian cancels, so the normwise |A||x| bound is the right one
    prob = make(name)
    announce("apply_A smooth", name)
    P = mxp.Problem(ctx, prob)
    axes = [np.sin(np.pi * (np.arange(m) + 1) / (m + 1)) for m in prob.n]
    x = axes[0]
    for a in axes[1:]:
        x = np.multiply.outer(a, x)
    x = (x * (1 + 0.5j)).ravel()
    xd = to_dev(x)
    yd = torch.empty_like(xd)
    mxp.mxp_apply_A(P, 0.0, xd, yd)
    As = op.helmholtz(prob, 0.0)
    assert np.linalg.norm(to_host(yd) - As @ x) <= 16 * 2.0**-53 * np.linalg.norm(abs(As) @ np.abs(x))


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("dt,tol", [("c128", 1e-11), ("c64", 1e-5)])
def test_apply_exp(ctx, name, dt, tol):
    prob = make(name)
    announce("apply_exp", name, dt)
    P = mxp.Problem(ctx, prob)
    t, s = prob.default_t(), prob.default_shift()
    x = wl.random_vector(prob.npts, 2)
    tdt = torch.complex128 if dt == "c128" else torch.complex64
    xd = to_dev(x, tdt)
    yd = torch.empty_like(xd)
    mxp.mxp_apply_exp(P, t, s, xd, yd)
    ref = matfun.exp_action(op.helmholtz(prob, s), t, to_host(xd))
    assert rel(to_host(yd), ref) <= tol


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("dt,tol", [("c128", 1e-11), ("c64", 1e-5)])
def test_apply_psi1(ctx, name, dt, tol):
    prob = make(name)
    announce("apply_psi1", name, dt)
    P = mxp.Problem(ctx, prob)
    t, s = prob.default_t(), prob.default_shift()
    x = wl.random_vector(prob.npts, 3)
    tdt = torch.complex128 if dt == "c128" else torch.complex64
    xd = to_dev(x, tdt)
    yd = torch.empty_like(xd)
    mxp.mxp_apply_psi1(P, t, s, xd, yd)
    ref = matfun.phi1_action(op.helmholtz(prob, s), t, to_host(xd))
    assert rel(to_host(yd), ref) <= tol


def test_apply_exp_delta_source_and_unshifted(ctx):
    prob = make("2d-homog")
    announce("apply_exp delta s=0")
    P = mxp.Problem(ctx, prob)
    t = prob.default_t()
    f = wl.delta_source(prob, (33, 22)).ravel()
    xd = to_dev(f)
    yd = torch.empty_like(xd)
    mxp.mxp_apply_exp(P, t, 0.0, xd, yd)
    assert rel(to_host(yd), matfun.exp_action(op.helmholtz(prob, 0.0), t, f)) <= 1e-11


@pytest.mark.parametrize("name", ["2d-homog", "2d-inh", "3d-inh"])
@pytest.mark.parametrize("prec", [0, 1])
def test_apply_precond(ctx, name, prec):
    prob = make(name)
    announce("apply_precond", name, prec)
    P = mxp.Problem(ctx, prob)
    o = P.default_opts()
    o.precision = prec
    r = wl.random_vector(prob.npts, 4)
    forced_precond_parity(P, op.helmholtz(prob, o.shift), o, r, 1e-10 if prec == 0 else 1e-5)


@pytest.mark.parametrize("name", ["2d-homog", "2d-inh", "3d-homog", "3d-inh"])
@pytest.mark.parametrize("prec", [0, 1])
def test_solve_counts_and_tight_solution(ctx, name, prec):
    prob = make(name)
    announce("solve", name, prec)
    P = mxp.Problem(ctx, prob)
    centre = tuple(m // 2 for m in prob.n)
    f = wl.delta_source(prob, centre).ravel()
    o = P.default_opts()
    o.precision = prec
    fd = to_dev(f)
    ud = torch.zeros_like(fd)
    st = mxp.mxp_solve(P, o, fd, ud)
    ref = krylov.matexpre_solve(prob, f, o.t, o.shift, o.fprtol, o.rtol)
    assert st["status"] == mxp.MXP_OK
    assert st["true_relres"] <= o.rtol
    assert abs(st["outer_its"] - ref.outer_iterations) <= 1
    assert abs(st["inner_mean"] - ref.inner_mean) <= 1.0
    # the iterate itself is a parity quantity once both are solved tightly
    o.rtol = 1e-12
    ud.zero_()
    st = mxp.mxp_solve(P, o, fd, ud)
    tight = krylov.direct_solve(prob, f)
    assert st["true_relres"] <= 1e-12
    assert rel(to_host(ud), tight) <= (1e-10 if prec == 0 else 1e-5)


def test_solve_edge_cases(ctx):
    prob = wl.small_problem((3, 3), layer=0)
    announce("edge 3x3")
    P = mxp.Problem(ctx, prob)
    o = P.default_opts()
    f = np.zeros(prob.npts, complex)
    fd = to_dev(f)
    ud = torch.ones_like(fd)
    st = mxp.mxp_solve(P, o, fd, ud)
    assert st["status"] == mxp.MXP_OK and np.all(to_host(ud) == 0)
    f[4] = 1.0
    fd = to_dev(f)
    ud = torch.zeros_like(fd)
    st = mxp.mxp_solve(P, o, fd, ud)
    assert st["status"] == mxp.MXP_OK
    assert rel(to_host(ud), krylov.direct_solve(prob, f)) <= 1e-6 * 1e3
    # iteration limit -> NOT_CONVERGED with the statistics filled in
    prob = make("2d-homog")
    P = mxp.Problem(ctx, prob)
    o = P.default_opts()
    o.max_outer = 1
    fd = to_dev(wl.delta_source(prob, (33, 22)).ravel())
    ud = torch.zeros_like(fd)
    st = mxp.mxp_solve(P, o, fd, ud)
    assert st["status"] == mxp.MXP_NOT_CONVERGED and st["outer_its"] == 1
    assert 0 < st["true_relres"] < 1
    # a nearly degenerate preconditioner (fprtol just below 1: one inner step) still converges
    o = P.default_opts()
    o.fprtol = 0.99
    ud.zero_()
    st = mxp.mxp_solve(P, o, fd, ud)
    assert st["status"] == mxp.MXP_OK and st["true_relres"] <= 1e-6


def test_argument_errors(ctx):
    prob = make("2d-homog")
    P = mxp.Problem(ctx, prob)
    xd = to_dev(np.zeros(prob.npts, complex))
    with pytest.raises(mxp.MxpError) as e:
        mxp.mxp_apply_A(P, 0.0, xd, xd)
    assert e.value.status == mxp.MXP_ERR_INVALID_ARG
    o = P.default_opts()
    o.fprtol = 0.0
    with pytest.raises(mxp.MxpError):
        mxp.mxp_solve(P, o, xd, torch.zeros_like(xd))
    with pytest.raises(mxp.MxpError):
        mxp.mxp_apply_exp(P, -1.0, 0.1, xd, torch.zeros_like(xd))


@pytest.mark.parametrize("Ly", [13, 4])
@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("NX", [1, 2])
@pytest.mark.parametrize("K", [1, 2, 3, 4, 5, 6, 7, 8])
def test_fused_passes_every_tile_shape(ctx, K, NX, prec, Ly):
    # every level count a final pass can have, both lane widths, segments that
    # do not divide the grid (67 x 45 with Ly = 13) and segments shorter than
    # the halo (Ly = 4), against the oracle
    if prec == 0 and NX == 2 and K > 3:
        pytest.skip("register-limited shape, never selected")
    prob = make("2d-inh")
    announce("fused tiles", K, NX, prec, Ly)
    P = mxp.Problem(ctx, prob)
    mxp.mxp_set_tiles(P, prec, K, NX, Ly)
    t, s = prob.default_t(), prob.default_shift()
    x = wl.random_vector(prob.npts, 8)
    tdt = torch.complex128 if prec == 0 else torch.complex64
    xd = to_dev(x, tdt)
    yd = torch.empty_like(xd)
    As = op.helmholtz(prob, s)
    mxp.mxp_apply_exp(P, t, s, xd, yd)
    assert rel(to_host(yd), matfun.exp_action(As, t, to_host(xd))) <= (1e-11 if prec == 0 else 1e-5)
    mxp.mxp_apply_psi1(P, t, s, xd, yd)
    assert rel(to_host(yd), matfun.phi1_action(As, t, to_host(xd))) <= (1e-11 if prec == 0 else 1e-5)
    assert mxp.mxp_get_tiles(P, prec)["K"] == K


def test_autotuned_tiles_are_recorded(ctx):
    prob = make("2d-homog")
    P = mxp.Problem(ctx, prob)
    assert mxp.mxp_get_tiles(P, 1)["K"] == 0
    xd = to_dev(wl.random_vector(prob.npts, 1), torch.complex64)
    yd = torch.empty_like(xd)
    mxp.mxp_apply_exp(P, prob.default_t(), prob.default_shift(), xd, yd)
    tiles = mxp.mxp_get_tiles(P, 1)
    assert 1 <= tiles["K"] <= 8 and tiles["NX"] in (1, 2) and tiles["us_per_level"] > 0


@pytest.mark.parametrize("levels,zc", [(2, 1), (3, 1), (3, 2), (3, 3), (3, 0)])
@pytest.mark.parametrize("name", ["3d-homog", "3d-inh", "3d-ragged"])
@pytest.mark.parametrize("prec", [0, 1])
def test_multi_level_3d_passes(ctx, name, prec, levels, zc):
    # the two- and three-level 3D passes (tiles K = 2, 3): 62 x 14 and 60 x 12
    # tiles with ragged edges, short z-chunks (chunk boundaries inside the
    # grid; 1-, 2- and 3-plane chunks give 5, 6 and 7 plane steps, every
    # remainder of the complex-float loop unrolled by three) and the default,
    # odd and even series degrees (remainders of one and two levels) through
    # exp and psi_1
    prob = make(name)
    announce("3d multi-level passes", name, prec, levels, zc)
    P = mxp.Problem(ctx, prob)
    mxp.mxp_set_tiles(P, prec, levels, 1, zc)
    t, s = prob.default_t(), prob.default_shift()
    x = wl.random_vector(prob.npts, 9)
    tdt = torch.complex128 if prec == 0 else torch.complex64
    xd = to_dev(x, tdt)
    yd = torch.empty_like(xd)
    As = op.helmholtz(prob, s)
    tol = 1e-11 if prec == 0 else 1e-5
    mxp.mxp_apply_exp(P, t, s, xd, yd)
    assert rel(to_host(yd), matfun.exp_action(As, t, to_host(xd))) <= tol
    mxp.mxp_apply_psi1(P, t, s, xd, yd)
    assert rel(to_host(yd), matfun.phi1_action(As, t, to_host(xd))) <= tol


@pytest.mark.parametrize("prec", [0, 1])
def test_3d_kernel_choice_is_tuned_and_matches_the_oracle(ctx, prec):
    # the first action on a 3D problem times a sweep against two- and
    # three-level passes and keeps the fastest per level (K = 1 with an
    # automatic z-chunk, or K = 2, 3); the chosen kernel's action matches the oracle, and a grid with
    # per-node absorbing faces always takes sweeps
    prob = make("3d-inh")
    announce("3d kernel choice", prec)
    P = mxp.Problem(ctx, prob)
    assert mxp.mxp_get_tiles(P, prec)["K"] == 0
    tdt = torch.complex128 if prec == 0 else torch.complex64
    xd = to_dev(wl.random_vector(prob.npts, 5), tdt)
    yd = torch.empty_like(xd)
    t, s = prob.default_t(), prob.default_shift()
    mxp.mxp_apply_exp(P, t, s, xd, yd)
    tiles = mxp.mxp_get_tiles(P, prec)
    assert tiles["K"] in (1, 2, 3) and tiles["us_per_level"] > 0
    assert tiles["K"] >= 2 or tiles["Ly"] == 0
    tol = 1e-11 if prec == 0 else 1e-5
    assert rel(to_host(yd), matfun.exp_action(op.helmholtz(prob, s), t, to_host(xd))) <= tol
    P.close()
    pa = make_abc("3d-ragged")
    Pa = mxp.Problem(ctx, pa)
    xa = to_dev(wl.random_vector(pa.npts, 6), tdt)
    ya = torch.empty_like(xa)
    mxp.mxp_apply_exp(Pa, pa.default_t(), pa.default_shift(), xa, ya)
    assert mxp.mxp_get_tiles(Pa, prec)["K"] == 1
    Pa.close()


@pytest.mark.parametrize("name,levels", [("2d-inh", 0), ("3d-inh", 0), ("3d-inh", 3)])
@pytest.mark.parametrize("prec", [0, 1])
def test_graph_replayed_actions_match_direct_launches(ctx, name, levels, prec):
    # every exp / psi_1 action after the first of its kind replays a captured
    # HIP graph, with the solver's own eager kernels and synchronisations in
    # between; solutions and statistics must equal the directly launched solve
    # (with the tuner's tiles, and in 3D also with three-level passes pinned in
    # both precisions, as the mixed form's double iterations use them too)
    prob = make(name)
    announce("graphs", name, levels, prec)
    P = mxp.Problem(ctx, prob)
    if levels:
        for pr in (0, 1):
            mxp.mxp_set_tiles(P, pr, levels, 1, 0)
    centre = tuple(m // 2 for m in prob.n)
    fd = to_dev(wl.delta_source(prob, centre).ravel())
    o = P.default_opts()
    o.precision = prec
    ud = torch.zeros_like(fd)
    ref = mxp.mxp_solve(P, o, fd, ud)
    u_ref = ud.clone()
    o.use_graphs = 1
    for _ in range(2):
        ud.zero_()
        st = mxp.mxp_solve(P, o, fd, ud)
        assert torch.equal(ud, u_ref)
        for key in ("outer_its", "inner_its_total", "stencil_steps", "fn_actions", "true_relres"):
            assert st[key] == ref[key], key
    r = to_dev(wl.random_vector(prob.npts, 21))
    w_ref = torch.empty_like(r)
    o.use_graphs = 0
    its = mxp.mxp_apply_precond(P, o, r, w_ref)
    o.use_graphs = 1
    w = torch.empty_like(r)
    assert mxp.mxp_apply_precond(P, o, r, w) == its
    assert torch.equal(w, w_ref)


@pytest.mark.parametrize("name", ["2d-inh", "3d-inh"])
@pytest.mark.parametrize("prec", [0, 1])
def test_fixed_point_inner_solver(ctx, name, prec):
    # Theorem 2.1's plain iteration in place of inner GMRES: one apply against
    # the oracle's, then whole solves (counts, and the iterate at rtol 1e-12)
    prob = make(name)
    announce("fixed-point inner", name, prec)
    P = mxp.Problem(ctx, prob)
    o = P.default_opts()
    o.precision = prec
    o.inner_solver = mxp.MXP_INNER_FIXED_POINT
    r = wl.random_vector(prob.npts, 4)
    forced_precond_parity(P, op.helmholtz(prob, o.shift), o, r, 1e-10 if prec == 0 else 1e-5, inner="fixed_point")
    centre = tuple(m // 2 for m in prob.n)
    f = wl.delta_source(prob, centre).ravel()
    fd = to_dev(f)
    ud = torch.zeros_like(fd)
    st = mxp.mxp_solve(P, o, fd, ud)
    sref = krylov.matexpre_solve(prob, f, o.t, o.shift, o.fprtol, o.rtol, inner_solver="fixed_point")
    assert st["status"] == mxp.MXP_OK and st["true_relres"] <= o.rtol
    assert abs(st["outer_its"] - sref.outer_iterations) <= 1
    assert abs(st["inner_mean"] - sref.inner_mean) <= 1.0
    o.rtol = 1e-12
    ud.zero_()
    st = mxp.mxp_solve(P, o, fd, ud)
    assert st["true_relres"] <= 1e-12
    assert rel(to_host(ud), krylov.direct_solve(prob, f)) <= (1e-10 if prec == 0 else 1e-5)


@pytest.mark.parametrize("name,tfac", [(n, 1.0) for n in CASES] + [("2d-inh", f) for f in (0.3, 0.15, 0.05)]
                         + [("3d-ragged", f) for f in (0.3, 0.15, 0.05)])
@pytest.mark.parametrize("dt,tol", [("c128", 1e-11), ("c64", 1e-5)])
def test_apply_psi2(ctx, name, tfac, dt, tol):
    # t scaled down so that the substep count runs through S = 1, 2, 3 and >= 5
    prob = make(name)
    announce("apply_psi2", name, tfac, dt)
    P = mxp.Problem(ctx, prob)
    t, s = prob.default_t() * tfac, prob.default_shift()
    x = wl.random_vector(prob.npts, 13)
    tdt = torch.complex128 if dt == "c128" else torch.complex64
    xd = to_dev(x, tdt)
    yd = torch.empty_like(xd)
    mxp.mxp_apply_psi2(P, t, s, xd, yd)
    ref = matfun.phi2_action(op.helmholtz(prob, s), t, to_host(xd))
    assert rel(to_host(yd), ref) <= tol


@pytest.mark.parametrize("name,prec,inner", [("2d-inh", p, i) for p in (0, 1) for i in ("gmres", "fixed_point")]
                         + [("3d-inh", p, "gmres") for p in (0, 1)])
def test_psi2_form_inner_solver(ctx, name, prec, inner):
    # the second inverse formula (I - psi_1) w = psi_2 r, by GMRES or by the
    # time-averaged fixed-point map: one apply, then whole solves
    prob = make(name)
    announce("psi2 form", name, prec, inner)
    P = mxp.Problem(ctx, prob)
    o = P.default_opts()
    o.precision = prec
    o.inner_solver = mxp.MXP_INNER_PSI2_GMRES if inner == "gmres" else mxp.MXP_INNER_PSI2_FIXED_POINT
    r = wl.random_vector(prob.npts, 14)
    forced_precond_parity(P, op.helmholtz(prob, o.shift), o, r, 1e-10 if prec == 0 else 1e-5, inner=inner,
                          form="psi2")
    centre = tuple(m // 2 for m in prob.n)
    f = wl.delta_source(prob, centre).ravel()
    fd = to_dev(f)
    ud = torch.zeros_like(fd)
    st = mxp.mxp_solve(P, o, fd, ud)
    sref = krylov.matexpre_solve(prob, f, o.t, o.shift, o.fprtol, o.rtol, inner_solver=inner, form="psi2")
    assert st["status"] == mxp.MXP_OK and st["true_relres"] <= o.rtol
    assert abs(st["outer_its"] - sref.outer_iterations) <= 1
    assert abs(st["inner_mean"] - sref.inner_mean) <= 1.0
    o.rtol = 1e-12
    ud.zero_()
    st = mxp.mxp_solve(P, o, fd, ud)
    assert st["true_relres"] <= 1e-12
    assert rel(to_host(ud), krylov.direct_solve(prob, f)) <= (1e-10 if prec == 0 else 1e-5)


CAP_CASES = {
    "2d-inh": dict(n=(67, 45), layer=8),
    # ragged x and y tiles and z chunks, as "3d-ragged", with a layer wide enough
    # for complex-float stepping
    "3d-ragged": dict(n=(70, 17, 37), layer=6),
}


@pytest.mark.parametrize("name", list(CAP_CASES))
def test_cap_absorber(ctx, name):
    # the complex absorbing potential in place of the stretch: the operator in both
    # precisions, the exp action, one preconditioner apply and whole solves
    import dataclasses
    c = CAP_CASES[name]
    prob = dataclasses.replace(wl.small_problem(c["n"], layer=c["layer"], ppw=10.0, inhomogeneous=True, seed=7,
                                                name=name), absorber="cap")
    announce("cap", name)
    P = mxp.Problem(ctx, prob)
    s = prob.default_shift()
    As = op.helmholtz(prob, s)
    x = wl.random_vector(prob.npts, 21)
    for tdt, eps in ((torch.complex128, 2.0**-53), (torch.complex64, 2.0**-24)):
        xd = to_dev(x, tdt)
        yd = torch.empty_like(xd)
        mxp.mxp_apply_A(P, s, xd, yd)
        xr = to_host(xd)
        bound = np.linalg.norm(abs(As) @ np.abs(xr))
        assert np.linalg.norm(to_host(yd) - As @ xr) <= 16 * eps * bound
    t = prob.default_t()
    for tdt, tol in ((torch.complex128, 1e-11), (torch.complex64, 1e-5)):
        xd = to_dev(x, tdt)
        yd = torch.empty_like(xd)
        mxp.mxp_apply_exp(P, t, s, xd, yd)
        assert rel(to_host(yd), matfun.exp_action(As, t, to_host(xd))) <= tol
    o = P.default_opts()
    forced_precond_parity(P, As, o, x, 1e-10)
    centre = tuple(m // 2 for m in prob.n)
    f = wl.delta_source(prob, centre).ravel()
    fd = to_dev(f)
    sref = krylov.matexpre_solve(prob, f, o.t, o.shift, o.fprtol, o.rtol)
    for prec in (0, 1):
        o = P.default_opts()
        o.precision = prec
        ud = torch.zeros_like(fd)
        st = mxp.mxp_solve(P, o, fd, ud)
        assert st["status"] == mxp.MXP_OK and st["true_relres"] <= o.rtol
        assert abs(st["outer_its"] - sref.outer_iterations) <= 1
        assert abs(st["inner_mean"] - sref.inner_mean) <= 1.0
        o.rtol = 1e-12
        ud.zero_()
        st = mxp.mxp_solve(P, o, fd, ud)
        assert st["true_relres"] <= 1e-12
        assert rel(to_host(ud), krylov.direct_solve(prob, f)) <= (1e-10 if prec == 0 else 1e-5)


def test_cap_thin_layer_refuses_complex_float_stepping(ctx):
    # a 3-cell layer makes the potential taller than the Laplacian is wide: complex-float
    # schedules are refused, while complex-double actions stay exact
    import dataclasses
    prob = dataclasses.replace(make("3d-ragged"), absorber="cap")
    announce("cap thin layer")
    P = mxp.Problem(ctx, prob)
    t, s = prob.default_t(), prob.default_shift()
    x = wl.random_vector(prob.npts, 22)
    xd = to_dev(x)
    yd = torch.empty_like(xd)
    mxp.mxp_apply_exp(P, t, s, xd, yd)
    assert rel(to_host(yd), matfun.exp_action(op.helmholtz(prob, s), t, x)) <= 1e-11
    with pytest.raises(mxp.MxpError) as e:
        mxp.mxp_apply_exp(P, t, s, to_dev(x, torch.complex64), torch.empty(prob.npts, dtype=torch.complex64,
                                                                            device="cuda:0"))
    assert e.value.status == mxp.MXP_ERR_UNSUPPORTED
    o = P.default_opts()
    o.precision = mxp.MXP_PREC_MIXED
    with pytest.raises(mxp.MxpError) as e:
        mxp.mxp_solve(P, o, xd, torch.zeros_like(xd))
    assert e.value.status == mxp.MXP_ERR_UNSUPPORTED


@pytest.mark.parametrize("name", ["2d-inh", "3d-inh"])
@pytest.mark.parametrize("psi", [False, True])
def test_krylov_matrix_function(ctx, name, psi):
    # the Arnoldi route to exp / psi_1 against the oracle's; the stop estimate is
    # relative to ||x|| and conservative, so 1e-10 gives <= 1e-8 relative to the result
    prob = make(name)
    announce("krylov action", name, psi)
    P = mxp.Problem(ctx, prob)
    # in 3D, t ||A|| is about 1.5 times larger: the default t needs more than 250
    # vectors, so the action restarts by time stepping
    t, s = prob.default_t(), prob.default_shift()
    x = wl.random_vector(prob.npts, 23)
    xd = to_dev(x)
    yd = torch.full_like(xd, 7.0)  # the output is overwritten, whatever it held
    st, dim = mxp.mxp_apply_fn_krylov(P, psi, t, s, 1e-10, 250, xd, yd)
    assert st == mxp.MXP_OK and 8 <= dim
    assert (dim <= 250) == (prob.dim == 2)  # one basis in 2D; substeps in 3D
    As = op.helmholtz(prob, s)
    ref = matfun.phi1_action(As, t, x) if psi else matfun.exp_action(As, t, x)
    assert rel(to_host(yd), ref) <= 1e-8
    # a small cap restarts by time stepping and still meets the tolerance
    st, dim2 = mxp.mxp_apply_fn_krylov(P, psi, t, s, 1e-10, 48, xd, yd)
    assert st == mxp.MXP_OK and dim2 > 48
    assert rel(to_host(yd), ref) <= 1e-8
    # a cap no substep count can meet reports NOT_CONVERGED and leaves an approximation
    st, _ = mxp.mxp_apply_fn_krylov(P, psi, t, s, 1e-10, 2, xd, yd)
    assert st == mxp.MXP_NOT_CONVERGED
    assert np.isfinite(to_host(yd)).all()


def test_krylov_matrix_function_invariant_space(ctx):
    # 3x3 nodes: the Krylov space is at most 9-dimensional, so the basis breaks
    # down and the result is exact
    prob = wl.small_problem((3, 3), layer=0)
    announce("krylov breakdown 3x3")
    P = mxp.Problem(ctx, prob)
    t, s = prob.default_t(), 0.1
    x = wl.random_vector(prob.npts, 24)
    xd = to_dev(x)
    yd = torch.empty_like(xd)
    st, dim = mxp.mxp_apply_fn_krylov(P, False, t, s, 1e-12, 50, xd, yd)
    assert st == mxp.MXP_OK and dim <= 9
    assert rel(to_host(yd), matfun.exp_dense(op.helmholtz(prob, s), t) @ x) <= 1e-11
    zd = torch.zeros_like(xd)
    st, dim = mxp.mxp_apply_fn_krylov(P, True, t, s, 1e-12, 50, zd, yd)
    assert st == mxp.MXP_OK and dim == 0 and not to_host(yd).any()


# Boundary conditions in place of a layer (Section 4.3.4): first-order
# absorbing faces and a sound-hard face by ghost points.
ABC_CASES = {
    "2d-inh": dict(n=(67, 45), hard=((1, 0),), inh=True),
    "2d-homog": dict(n=(67, 45), hard=((1, 0),), inh=False),
    "3d-ragged": dict(n=(70, 17, 37), hard=((2, 0),), inh=True),
}


def make_abc(name):
    import dataclasses
    c = ABC_CASES[name]
    base = wl.small_problem(c["n"], layer=0, ppw=10.0, inhomogeneous=c["inh"], seed=17, name="abc-" + name)
    return dataclasses.replace(base, absorber="abc", hard_faces=c["hard"])


@pytest.mark.parametrize("name", list(ABC_CASES))
def test_abc_operator_actions_and_precond(ctx, name):
    prob = make_abc(name)
    announce("abc", name, prob.n)
    P = mxp.Problem(ctx, prob)
    s = prob.default_shift()
    As = op.helmholtz(prob, s)
    x = wl.random_vector(prob.npts, 23)
    for tdt, eps in ((torch.complex128, 2.0**-53), (torch.complex64, 2.0**-24)):
        xd = to_dev(x, tdt)
        yd = torch.empty_like(xd)
        mxp.mxp_apply_A(P, s, xd, yd)
        xr = to_host(xd)
        bound = np.linalg.norm(abs(As) @ np.abs(xr))
        assert np.linalg.norm(to_host(yd) - As @ xr) <= 16 * eps * bound, tdt
    t = prob.default_t()
    for tdt, tol in ((torch.complex128, 1e-11), (torch.complex64, 1e-5)):
        xd = to_dev(x, tdt)
        yd = torch.empty_like(xd)
        mxp.mxp_apply_exp(P, t, s, xd, yd)
        assert rel(to_host(yd), matfun.exp_action(As, t, to_host(xd))) <= tol, tdt
        mxp.mxp_apply_psi1(P, t, s, xd, yd)
        assert rel(to_host(yd), matfun.phi1_action(As, t, to_host(xd))) <= tol, tdt
    for prec in (0, 1):
        o = P.default_opts()
        o.precision = prec
        forced_precond_parity(P, As, o, x, 1e-10 if prec == 0 else 1e-5)
    P.close()


@pytest.mark.parametrize("name", ["2d-inh", "3d-ragged"])
@pytest.mark.parametrize("prec", [0, 1])
def test_abc_solve(ctx, name, prec):
    prob = make_abc(name)
    announce("abc solve", name, prec)
    P = mxp.Problem(ctx, prob)
    # a source next to the sound-hard face, centred on the other axes
    node = [m // 2 for m in prob.n]
    node[ABC_CASES[name]["hard"][0][0]] = 2
    f = wl.delta_source(prob, tuple(node)).ravel()
    fd = to_dev(f)
    ud = torch.zeros_like(fd)
    o = P.default_opts()
    o.precision = prec
    st = mxp.mxp_solve(P, o, fd, ud)
    ref = krylov.matexpre_solve(prob, f, o.t, o.shift, o.fprtol, o.rtol)
    assert st["status"] == mxp.MXP_OK and st["true_relres"] <= o.rtol
    assert abs(st["outer_its"] - ref.outer_iterations) <= 1
    assert abs(st["inner_mean"] - ref.inner_mean) <= 1.0
    o.rtol = 1e-12
    ud.zero_()
    st = mxp.mxp_solve(P, o, fd, ud)
    assert st["true_relres"] <= 1e-12
    assert rel(to_host(ud), krylov.direct_solve(prob, f)) <= (1e-10 if prec == 0 else 1e-5)
    P.close()


def test_abc_batch_equals_separate_solves(ctx):
    """A batched solve over an absorbing-face problem (3D, varying speed) and a
    layer problem equals the separate solves bit for bit."""
    probs = [make_abc("3d-ragged"), make("3d-inh")]
    announce("abc batch", [p.n for p in probs])
    Ps = [mxp.Problem(ctx, p) for p in probs]
    fs, us, opts, refs = [], [], [], []
    for p, P in zip(probs, Ps):
        f = to_dev(wl.random_vector(p.npts, 31))
        o = P.default_opts()
        o.precision = mxp.MXP_PREC_MIXED
        u = torch.zeros_like(f)
        mxp.mxp_solve(P, o, f, u)
        refs.append(u.clone())
        fs.append(f)
        us.append(torch.zeros_like(f))
        opts.append(o)
    status, stats = mxp.mxp_solve_batch(ctx, Ps, opts, fs, us)
    assert status == mxp.MXP_OK
    for u, r in zip(us, refs):
        assert torch.equal(u, r)
    for P in Ps:
        P.close()
