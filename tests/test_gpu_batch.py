"""GPU tests of the batched solve (many right-hand sides, uneven grids).

Every right-hand side of a batch runs the same arithmetic as a separate
mxp_solve on the same problem (the lockstep batching only reorders launches
across right-hand sides, and the batched 3D sweep and 2D pass compute each
grid point as the single-grid kernels do), so solutions and statistics must
agree bit for bit.  The separate solves are themselves pinned to the oracle by the parity
tests; here a few batched right-hand sides are also checked against the oracle
directly, and the full-size layered batch against its true residuals."""
import numpy as np
import pytest

import workloads as wl
from oracle import krylov

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


def uneven_set():
    """Three 3D grids of different sizes and one 2D grid, with sources."""
    probs = [
        wl.small_problem((33, 29, 21), layer=4, ppw=10, inhomogeneous=True, seed=3, name="a"),
        wl.small_problem((24, 20, 18), layer=3, ppw=10, inhomogeneous=False, seed=4, name="b"),
        wl.small_problem((40, 17, 27), layer=4, ppw=10, inhomogeneous=True, seed=5, name="c"),
        wl.small_problem((67, 45), layer=8, ppw=10, inhomogeneous=True, seed=6, name="d"),
    ]
    nrhs = [3, 1, 2, 2]
    rhs = []
    for q, (p, k) in enumerate(zip(probs, nrhs)):
        rng = np.random.default_rng(100 + q)
        fs = []
        for r in range(k):
            node = tuple(int(rng.integers(p.layer + 1, m - p.layer - 1)) for m in p.n)
            fs.append(wl.delta_source(p, node).ravel())
        rhs.append(np.stack(fs))
    return probs, rhs


def run_batch(ctx, handles, opts, rhs, max_resident=0):
    f_list = [to_dev(f) for f in rhs]
    u_list = [torch.zeros_like(f) for f in f_list]
    status, stats = mxp.mxp_solve_batch(ctx, handles, opts, f_list, u_list, max_resident)
    return status, stats, [to_host(u).reshape(f.shape) for u, f in zip(u_list, rhs)]


@pytest.mark.parametrize("levels", [1, 2, 3])
@pytest.mark.parametrize("prec", [0, 1])
def test_batch_equals_separate_solves_bit_for_bit(ctx, prec, levels):
    probs, rhs = uneven_set()
    announce("batch vs separate", prec, levels)
    handles = [mxp.Problem(ctx, p) for p in probs]
    # the 3D grids run sweeps, two-level (batched k_cheb3d) or three-level
    # passes (batched k_cheb3d3), the mixed form's double iterations included
    for h, p in zip(handles, probs):
        if p.dim == 3:
            for pr in (0, 1):
                mxp.mxp_set_tiles(h, pr, levels, 1, 0 if levels > 1 else 16)
    opts = []
    for h in handles:
        o = h.default_opts()
        o.precision = prec
        o.outer_restart = 20
        opts.append(o)
    status, stats, us = run_batch(ctx, handles, opts, rhs)
    assert status == mxp.MXP_OK
    k = 0
    for q, h in enumerate(handles):
        for r in range(rhs[q].shape[0]):
            fd = to_dev(rhs[q][r])
            ud = torch.zeros_like(fd)
            st = mxp.mxp_solve(h, opts[q], fd, ud)
            assert st["status"] == mxp.MXP_OK and stats[k]["status"] == mxp.MXP_OK
            for key in ("outer_its", "inner_its_total", "stencil_steps", "fn_actions", "true_relres"):
                assert stats[k][key] == st[key], (q, r, key)
            assert np.array_equal(us[q][r], to_host(ud)), (q, r)
            k += 1
    for h in handles:
        h.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_batched_2d_passes_equal_separate_solves(ctx, prec):
    """Uneven 2D grids in one batch: each step's fused passes go out as one
    persistent launch per (K, NX) over every grid (two tile shapes here, so
    two groups), and every right-hand side keeps the separate solve's bits.
    The last grid's two-row segments give 1,350 workgroup indices per pass,
    more than the device holds at once, so the persistent loop strides."""
    probs = [wl.small_problem((97, 61), layer=8, ppw=10, inhomogeneous=True, seed=31, name="e"),
             wl.small_problem((130, 45), layer=8, ppw=10, inhomogeneous=True, seed=32, name="f"),
             wl.small_problem((70, 83), layer=8, ppw=10, inhomogeneous=False, seed=33, name="g"),
             wl.small_problem((1000, 600), layer=12, ppw=10, inhomogeneous=True, seed=34, name="h")]
    tiles = [(4, 1, 8), (6, 1, 12), (4, 1, 8), (4, 1, 2)]
    nrhs = [2, 2, 2, 1]
    rhs = []
    for q, p in enumerate(probs):
        rng = np.random.default_rng(200 + q)
        fs = [wl.delta_source(p, tuple(int(rng.integers(p.layer + 1, m - p.layer - 1)) for m in p.n)).ravel()
              for _ in range(nrhs[q])]
        rhs.append(np.stack(fs))
    announce("batched 2D passes", prec, [p.n for p in probs])
    handles = [mxp.Problem(ctx, p) for p in probs]
    opts = []
    for h, (K, NX, Ly) in zip(handles, tiles):
        mxp.mxp_set_tiles(h, prec, K, NX, Ly)
        o = h.default_opts()
        o.precision = prec
        opts.append(o)
    status, stats, us = run_batch(ctx, handles, opts, rhs)
    assert status == mxp.MXP_OK
    k = 0
    for q, h in enumerate(handles):
        for r in range(rhs[q].shape[0]):
            fd = to_dev(rhs[q][r])
            ud = torch.zeros_like(fd)
            st = mxp.mxp_solve(h, opts[q], fd, ud)
            assert st["status"] == mxp.MXP_OK and stats[k]["status"] == mxp.MXP_OK
            for key in ("outer_its", "inner_its_total", "stencil_steps", "fn_actions", "true_relres"):
                assert stats[k][key] == st[key], (q, r, key)
            assert np.array_equal(us[q][r], to_host(ud)), (q, r)
            k += 1
    for h in handles:
        h.close()


@pytest.mark.parametrize("inner_solver", [1, 2, 3])
@pytest.mark.parametrize("prec", [0, 1])
def test_batch_inner_solver_variants_equal_separate_solves(ctx, prec, inner_solver):
    # the fixed-point and psi_2 forms of Algorithm 1 in a batch: the same actions,
    # recorded per right-hand side and launched together, give the separate solves' bits
    probs, rhs = uneven_set()
    probs, rhs = [probs[1], probs[3]], [rhs[1], rhs[3]]
    announce("batch variants", prec, inner_solver)
    handles = [mxp.Problem(ctx, p) for p in probs]
    opts = []
    for h in handles:
        o = h.default_opts()
        o.precision = prec
        o.inner_solver = inner_solver
        opts.append(o)
    status, stats, us = run_batch(ctx, handles, opts, rhs)
    assert status == mxp.MXP_OK
    k = 0
    for q, h in enumerate(handles):
        for r in range(rhs[q].shape[0]):
            fd = to_dev(rhs[q][r])
            ud = torch.zeros_like(fd)
            st = mxp.mxp_solve(h, opts[q], fd, ud)
            assert st["status"] == mxp.MXP_OK and stats[k]["status"] == mxp.MXP_OK
            for key in ("outer_its", "inner_its_total", "stencil_steps", "fn_actions", "true_relres"):
                assert stats[k][key] == st[key], (q, r, key)
            assert np.array_equal(us[q][r], to_host(ud)), (q, r)
            k += 1
    for h in handles:
        h.close()


def test_batch_against_oracle_and_admission_limits(ctx):
    probs, rhs = uneven_set()
    announce("batch vs oracle")
    handles = [mxp.Problem(ctx, p) for p in probs]
    opts = [h.default_opts() for h in handles]
    for o in opts:
        o.rtol = 1e-12
    status, stats, us = run_batch(ctx, handles, opts, rhs)
    assert status == mxp.MXP_OK
    k = 0
    for q, p in enumerate(probs):
        for r in range(rhs[q].shape[0]):
            assert stats[k]["true_relres"] <= 1e-12
            assert rel(us[q][r], krylov.direct_solve(p, rhs[q][r])) <= 1e-10
            k += 1
    # one or two right-hand sides resident at a time: same results
    for cap in (1, 2):
        status2, stats2, us2 = run_batch(ctx, handles, opts, rhs, max_resident=cap)
        assert status2 == mxp.MXP_OK
        for a, b in zip(us, us2):
            assert np.array_equal(a, b)
        assert [s["outer_its"] for s in stats] == [s["outer_its"] for s in stats2]
    for h in handles:
        h.close()


def test_batch_counts_against_oracle(ctx):
    probs, rhs = uneven_set()
    announce("batch counts vs oracle")
    handles = [mxp.Problem(ctx, p) for p in probs[:2]]
    opts = [h.default_opts() for h in handles]
    status, stats, _ = run_batch(ctx, handles, opts, rhs[:2])
    assert status == mxp.MXP_OK
    k = 0
    for q in range(2):
        o = opts[q]
        for r in range(rhs[q].shape[0]):
            ref = krylov.matexpre_solve(probs[q], rhs[q][r], o.t, o.shift, o.fprtol, o.rtol)
            assert abs(stats[k]["outer_its"] - ref.outer_iterations) <= 1
            assert abs(stats[k]["inner_mean"] - ref.inner_mean) <= 1.0
            k += 1
    for h in handles:
        h.close()


def test_batch_status_and_errors(ctx):
    probs, rhs = uneven_set()
    announce("batch status")
    handles = [mxp.Problem(ctx, p) for p in probs[:2]]
    opts = [h.default_opts() for h in handles]
    opts[1].max_outer = 1  # cannot converge in one outer iteration
    status, stats, _ = run_batch(ctx, handles, opts, rhs[:2])
    assert status == mxp.MXP_NOT_CONVERGED
    assert [s["status"] for s in stats] == [mxp.MXP_OK] * 3 + [mxp.MXP_NOT_CONVERGED]
    # a zero right-hand side converges at once with u = 0
    zero = [np.zeros((1, probs[0].npts), complex)]
    status, stats, us = run_batch(ctx, handles[:1], [handles[0].default_opts()], zero)
    assert status == mxp.MXP_OK and stats[0]["outer_its"] == 0 and not np.any(us[0])
    # invalid options are rejected before any work
    bad = handles[0].default_opts()
    bad.fprtol = 0.0
    with pytest.raises(mxp.MxpError) as e:
        run_batch(ctx, handles[:1], [bad], rhs[:1])
    assert e.value.status == mxp.MXP_ERR_INVALID_ARG
    for h in handles:
        h.close()


def test_layered_batch_full_size(ctx):
    # the layered workload at full size: two of the 32 surface sources on the
    # 512 x 512 x 256 grid plus the 16 uneven 96^3..192^3 problems, one launch
    # per sweep step over all of them, mixed precision, FGMRES(20).  One outer
    # iteration each (a whole preconditioner apply: psi_1 action and the inner
    # GMRES with its exp actions), compared bit for bit with separate solves
    # and with residuals recomputed by the stencil (pinned to the oracle row
    # by row at this size) and, for one extra problem, the oracle's matrix.
    from oracle import operator as op
    main = wl.config4_main()
    extras = wl.config4_extras()
    announce("layered batch full size")
    probs = [main] + extras
    handles = [mxp.Problem(ctx, p) for p in probs]
    rhs = [wl.config4_sources(main, [0, 31])]
    for p in extras:
        centre = (p.n[0] // 2, p.n[1] // 2, p.layer + 2)
        rhs.append(wl.delta_source(p, centre).ravel()[None, :])
    opts = []
    for h in handles:
        o = h.default_opts()
        o.precision = mxp.MXP_PREC_MIXED
        o.outer_restart = 20
        o.max_outer = 1
        opts.append(o)
    f_list = [to_dev(f) for f in rhs]
    u_list = [torch.zeros_like(f) for f in f_list]
    status, stats = mxp.mxp_solve_batch(ctx, handles, opts, f_list, u_list, 0)
    assert status == mxp.MXP_NOT_CONVERGED
    assert all(s["status"] == mxp.MXP_NOT_CONVERGED and s["outer_its"] == 1 for s in stats)
    assert all(0 < s["true_relres"] < 1 for s in stats)
    k = 0
    for q, h in enumerate(handles):
        n = probs[q].npts
        for r in range(rhs[q].shape[0]):
            u = u_list[q].view(-1)[r * n:(r + 1) * n]
            f = f_list[q].view(-1)[r * n:(r + 1) * n]
            Au = torch.empty_like(u)
            mxp.mxp_apply_A(h, 0.0, u, Au)
            relres = (torch.linalg.vector_norm(Au + f) / torch.linalg.vector_norm(f)).item()
            assert abs(relres - stats[k]["true_relres"]) <= 1e-6 * relres
            if (q, r) in ((0, 0), (1, 0), (16, 0)):
                ud = torch.zeros_like(f)
                st = mxp.mxp_solve(h, opts[q], f.clone(), ud)
                for key in ("inner_its_total", "stencil_steps", "true_relres"):
                    assert st[key] == stats[k][key], (q, key)
                assert torch.equal(ud, u), q
            if q == 16:
                A = op.helmholtz(probs[q], 0.0)
                b = op.rhs(rhs[q][r])
                res = np.linalg.norm(b - A @ to_host(u)) / np.linalg.norm(b)
                assert abs(res - stats[k]["true_relres"]) <= 1e-6 * res
            k += 1
    for h in handles:
        h.close()
