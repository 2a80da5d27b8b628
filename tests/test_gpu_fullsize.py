"""GPU parity at the full workload sizes, in the launch configuration the
benchmark times (autotuned fused 2D passes, 3D Clenshaw steps).

Where the oracle cannot run the whole workload, it checks what it can compute
at that size:
  * sampled rows of A_s x, one row at a time from the stencil definition;
  * exact exp actions without a layer, by the type-I DST (a textbook
    diagonalisation of the Dirichlet Laplacian);
  * identities of the matrix functions that hold at any size
    (Section 3.1: e^{itA} - I = itA psi_1(itA); the semigroup property);
  * true residuals of full solves with the oracle's own sparse matrix;
  * the 128^2 iteration counts against a stored oracle run
    (tests/golden/config1_oracle.json, written by make_config1.py)."""
import json
import os

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

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module")
def ctx():
    c = mxp.Context(0)
    yield c
    c.close()


def sample_points(n, count, seed):
    """Random flat indices plus every corner, face centre and layer edge node."""
    rng = np.random.default_rng(seed)
    npts = int(np.prod(n))
    pts = set(rng.integers(0, npts, count).tolist())
    strides = [int(np.prod(n[:a])) for a in range(len(n))]
    specials = []
    for a in range(len(n)):
        specials.append([0, 1, n[a] // 2, n[a] - 2, n[a] - 1])
    grid = np.array(np.meshgrid(*specials, indexing="ij")).reshape(len(n), -1).T
    for idx in grid:
        pts.add(int(sum(int(i) * s for i, s in zip(idx, strides))))
    return np.array(sorted(pts), dtype=np.int64)


def neighbour_abs(prob, x, pts):
    """sum over the stencil of |x| weighted as a bound on |A_s| (|1/(s s')| <= 1
    because every stretch factor is 1 + i sigma with sigma >= 0)."""
    n = prob.n
    strides = [int(np.prod(n[:a])) for a in range(len(n))]
    ax = np.abs(x)
    out = np.zeros(len(pts))
    for a in range(len(n)):
        i = (pts // strides[a]) % n[a]
        lo = np.where(i > 0, ax[np.maximum(pts - strides[a], 0)], 0.0)
        hi = np.where(i < n[a] - 1, ax[np.minimum(pts + strides[a], x.size - 1)], 0.0)
        out += (lo + hi + 2 * ax[pts]) / prob.h ** 2
    return out


WORKLOADS = {
    "2d-grf-2048": wl.config2,
    "3d-homog-256": wl.config3,
    "3d-layered-512x512x256": wl.config4_main,
}


@pytest.mark.parametrize("name", list(WORKLOADS))
@pytest.mark.parametrize("dt", ["c128", "c64"])
def test_apply_A_sampled_rows_full_size(ctx, name, dt):
    prob = WORKLOADS[name]()
    announce("apply_A full size", name, dt, prob.n)
    P = mxp.Problem(ctx, prob)
    s = prob.default_shift()
    tdt = torch.complex128 if dt == "c128" else torch.complex64
    xd = to_dev(wl.random_vector(prob.npts, 11), tdt)
    yd = torch.empty_like(xd)
    mxp.mxp_apply_A(P, s, xd, yd)
    torch.cuda.synchronize()
    pts = sample_points(prob.n, 3000, 5)
    x = to_host(xd)
    y = to_host(yd)[pts]
    del xd, yd
    ref = op.apply_rows(prob, s, x, pts)
    D = op.inverse_c2(prob).ravel()[pts]
    bound = abs(prob.omega ** 2 * (1 + 1j * s)) * D * np.abs(x[pts]) + neighbour_abs(prob, x, pts)
    eps = 2.0 ** -53 if dt == "c128" else 2.0 ** -24
    assert np.all(np.abs(y - ref) <= 16 * eps * bound)
    P.close()


@pytest.mark.parametrize("n", [(2048, 2048), (256, 256, 256)])
@pytest.mark.parametrize("dt,tol", [("c128", 1e-11), ("c64", 1e-5)])
def test_exp_full_size_against_dst(ctx, n, dt, tol):
    # bare Dirichlet box (no layer), c = 1, 8 points per wavelength: the shifted
    # operator is diagonalised exactly by the type-I DST
    h = 1.0 / (n[0] - 1)
    prob = wl.Problem("nolayer-" + "x".join(map(str, n)), tuple(n), h, wl.omega_for(8, h), 0, None, 1.0)
    announce("exp full size vs DST", prob.name, dt)
    P = mxp.Problem(ctx, prob)
    t, s = prob.default_t(), prob.default_shift()
    tdt = torch.complex128 if dt == "c128" else torch.complex64
    xd = to_dev(wl.random_vector(prob.npts, 12), tdt)
    yd = torch.empty_like(xd)
    mxp.mxp_apply_exp(P, t, s, xd, yd)
    torch.cuda.synchronize()
    x, y = to_host(xd), to_host(yd)
    del xd, yd
    P.close()
    ref = matfun.exp_action_dst(prob.n, h, prob.omega ** 2 * (1 + 1j * s), t, x)
    assert rel(y, ref) <= tol


@pytest.fixture(scope="module")
def grf_oracle():
    """The 2048^2 random-field workload (32-cell layer), its operator in the
    oracle's CSR form, a seeded input and the oracle's exp and psi_1 actions at
    t/16 (expm_multiply; about 3.4 s each on the host)."""
    prob = wl.config2()
    s = prob.default_shift()
    t = prob.default_t() / 16
    As = op.helmholtz(prob, s)
    x = wl.random_vector(prob.npts, 31)
    return {"prob": prob, "s": s, "t": t, "x": x,
            "exp": matfun.exp_action(As, t, x), "psi1": matfun.phi1_action(As, t, x)}


@pytest.mark.parametrize("fn,dt,tol", [("exp", "c128", 1e-11), ("exp", "c64", 1e-5), ("psi1", "c128", 1e-11),
                                       ("psi1", "c64", 1e-5)])
def test_actions_full_size_grf_against_oracle(ctx, grf_oracle, fn, dt, tol):
    # element by element at the benchmark's 2048^2 shape, with the layer and the
    # random-field speed, in the launch configuration the benchmark times
    # (autotuned fused 2D passes); t/16 keeps the oracle's action to seconds
    g = grf_oracle
    prob = g["prob"]
    announce("action full size vs oracle", prob.name, fn, dt)
    P = mxp.Problem(ctx, prob)
    tdt = torch.complex128 if dt == "c128" else torch.complex64
    xd = to_dev(g["x"], tdt)
    yd = torch.empty_like(xd)
    (mxp.mxp_apply_exp if fn == "exp" else mxp.mxp_apply_psi1)(P, g["t"], g["s"], xd, yd)
    torch.cuda.synchronize()
    y = to_host(yd)
    del xd, yd
    P.close()
    # (a complex-float input is the rounded x: that changes the action by about
    # 6e-8 relative, far below the complex-float bar)
    assert rel(y, g[fn]) <= tol


@pytest.fixture(scope="module")
def cube_oracle():
    """The 256^3 workload (20-cell layer, c = 1), its operator in the oracle's
    CSR form, a seeded input and the oracle's exp and psi_1 actions at t/32
    (expm_multiply; about 15 s each on the host)."""
    prob = wl.config3()
    s = prob.default_shift()
    t = prob.default_t() / 32
    As = op.helmholtz(prob, s)
    x = wl.random_vector(prob.npts, 33)
    out = {"prob": prob, "s": s, "t": t, "x": x, "exp": matfun.exp_action(As, t, x)}
    out["psi1"] = matfun.phi1_action(As, t, x)
    return out


@pytest.mark.parametrize("tiles", ["tuned", "three-level"])
@pytest.mark.parametrize("fn,dt,tol", [("exp", "c128", 1e-11), ("exp", "c64", 1e-5), ("psi1", "c128", 1e-11),
                                       ("psi1", "c64", 1e-5)])
def test_actions_full_size_3d_layer_against_oracle(ctx, cube_oracle, fn, dt, tol, tiles):
    # element by element at the benchmark's 256^3 shape with its absorbing
    # layer: the 3D kernel the autotuner picks for this problem, and the
    # three-level pass over its default 32-plane chunks (the complex-double
    # solve's kernel at this size)
    g = cube_oracle
    prob = g["prob"]
    announce("3d action full size vs oracle", prob.name, fn, dt, tiles)
    P = mxp.Problem(ctx, prob)
    prec = 0 if dt == "c128" else 1
    if tiles == "three-level":
        mxp.mxp_set_tiles(P, prec, 3, 1, 0)
    tdt = torch.complex128 if dt == "c128" else torch.complex64
    xd = to_dev(g["x"], tdt)
    yd = torch.empty_like(xd)
    (mxp.mxp_apply_exp if fn == "exp" else mxp.mxp_apply_psi1)(P, g["t"], g["s"], xd, yd)
    torch.cuda.synchronize()
    chosen = mxp.mxp_get_tiles(P, prec)
    y = to_host(yd)
    del xd, yd
    P.close()
    assert chosen["K"] in (1, 2, 3)
    if tiles == "three-level":
        assert chosen["K"] == 3
    assert rel(y, g[fn]) <= tol


def test_matfun_identities_full_size_grf(ctx):
    # with the layer and the random-field speed at full size:
    #   e^{itA_s} v - v = i t A_s psi_1(itA_s) v                       (Section 3.1)
    #   e^{i2tA_s} v = e^{itA_s}(e^{itA_s} v)  (different schedules)
    # in complex double, and the complex-float actions against them
    prob = wl.config2()
    announce("identities full size", prob.name)
    P = mxp.Problem(ctx, prob)
    t, s = prob.default_t(), prob.default_shift()
    v = to_dev(wl.random_vector(prob.npts, 13))
    e = torch.empty_like(v)
    p = torch.empty_like(v)
    z = torch.empty_like(v)
    mxp.mxp_apply_exp(P, t, s, v, e)
    mxp.mxp_apply_psi1(P, t, s, v, p)
    mxp.mxp_apply_A(P, s, p, z)
    vn = torch.linalg.vector_norm(v).item()
    lhs = e - v
    assert torch.linalg.vector_norm(lhs - 1j * t * z).item() <= 1e-8 * vn
    assert torch.linalg.vector_norm(lhs).item() > 1e-2 * vn  # not a trivial pass
    e2 = torch.empty_like(v)
    ee = torch.empty_like(v)
    mxp.mxp_apply_exp(P, 2 * t, s, v, e2)
    mxp.mxp_apply_exp(P, t, s, e, ee)
    assert torch.linalg.vector_norm(e2 - ee).item() <= 1e-10 * vn
    # complex-float actions against the complex-double ones
    v32 = v.to(torch.complex64)
    e32 = torch.empty_like(v32)
    p32 = torch.empty_like(v32)
    mxp.mxp_apply_exp(P, t, s, v32, e32)
    mxp.mxp_apply_psi1(P, t, s, v32, p32)
    ve = v32.to(torch.complex128)
    e_ref = torch.empty_like(v)
    p_ref = torch.empty_like(v)
    mxp.mxp_apply_exp(P, t, s, ve, e_ref)
    mxp.mxp_apply_psi1(P, t, s, ve, p_ref)
    assert (torch.linalg.vector_norm(e32.to(torch.complex128) - e_ref) / torch.linalg.vector_norm(e_ref)).item() <= 1e-5
    assert (torch.linalg.vector_norm(p32.to(torch.complex128) - p_ref) / torch.linalg.vector_norm(p_ref)).item() <= 1e-5
    P.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_config1_counts_against_stored_oracle_run(ctx, prec):
    with open(os.path.join(GOLDEN, "config1_oracle.json")) as fh:
        gold = json.load(fh)
    prob = wl.config1()
    announce("config1 counts", prec)
    P = mxp.Problem(ctx, prob)
    f = wl.delta_source(prob, (64, 64)).ravel()
    o = P.default_opts()
    o.precision = prec
    assert abs(o.t - gold["t"]) <= 1e-15 and abs(o.shift - gold["shift"]) <= 1e-15
    fd = to_dev(f)
    ud = torch.zeros_like(fd)
    st = mxp.mxp_solve(P, o, fd, ud)
    assert st["status"] == mxp.MXP_OK and st["true_relres"] <= 1e-6
    assert abs(st["outer_its"] - gold["outer_iterations"]) <= 1
    assert abs(st["inner_mean"] - gold["inner_mean"]) <= 1.0
    o.rtol = 1e-12
    ud.zero_()
    st = mxp.mxp_solve(P, o, fd, ud)
    assert st["true_relres"] <= 1e-12
    assert rel(to_host(ud), krylov.direct_solve(prob, f)) <= (1e-10 if prec == 0 else 1e-5)
    P.close()


def test_full_solve_2048_true_residual(ctx):
    # the mixed solve at 2048^2: outer count within +-1 of the complex-double
    # solve's, its solution close to that one, and its residual recomputed with
    # the oracle's matrix
    prob = wl.config2()
    announce("full solve", prob.name)
    P = mxp.Problem(ctx, prob)
    f = wl.delta_source(prob, (1024, 1024)).ravel()
    fd = to_dev(f)
    u64 = torch.zeros_like(fd)
    st64 = mxp.mxp_solve(P, P.default_opts(), fd, u64)
    o = P.default_opts()
    o.precision = mxp.MXP_PREC_MIXED
    ud = torch.zeros_like(fd)
    st = mxp.mxp_solve(P, o, fd, ud)
    assert st64["status"] == mxp.MXP_OK
    assert abs(st["outer_its"] - st64["outer_its"]) <= 1, (st["outer_its"], st64["outer_its"])
    # both meet 1e-6 in the residual; the solutions differ by about the same
    # relative amount (measured 1.8e-6)
    assert ((ud - u64).norm() / u64.norm()).item() <= 1e-5
    u = to_host(ud)
    del fd, ud, u64
    P.close()
    assert st["status"] == mxp.MXP_OK
    A = op.helmholtz(prob, 0.0)
    b = op.rhs(f)
    relres = np.linalg.norm(b - A @ u) / np.linalg.norm(b)
    assert relres <= 1e-6 * (1 + 1e-6)
    assert abs(relres - st["true_relres"]) <= 1e-3 * relres


def test_full_solve_256cube_true_residual(ctx):
    prob = wl.config3()
    announce("full solve", prob.name)
    P = mxp.Problem(ctx, prob)
    f = wl.gaussian_source(prob, (128 * prob.h,) * 3, 2 * prob.h).ravel()
    o = P.default_opts()
    o.precision = mxp.MXP_PREC_MIXED
    o.outer_restart = 20
    fd = to_dev(f)
    ud = torch.zeros_like(fd)
    st = mxp.mxp_solve(P, o, fd, ud)
    u = to_host(ud)
    del fd, ud
    P.close()
    assert st["status"] == mxp.MXP_OK
    A = op.helmholtz(prob, 0.0)
    b = op.rhs(f)
    relres = np.linalg.norm(b - A @ u) / np.linalg.norm(b)
    assert relres <= 1e-6 * (1 + 1e-6)
    assert abs(relres - st["true_relres"]) <= 1e-3 * relres
