"""GPU solves against iteration counts the paper prints (the tables in
tests/golden/paper_tables.json, each with its citation).

The paper's matrix functions come from a restarted Krylov method and ours
from Chebyshev series, and its Krylov solvers orthogonalise differently, so
counts need not be identical; the bar is the one for oracle parity: outer
iterations within +-1 and mean inner iterations within +-1.  Sizes here are
the paper's smaller ones (a few seconds each); bench.py --workload
paper-tables runs every entry that fits one GPU."""
import json
import os

import pytest

import workloads as wl

from gpu_util import announce

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2506_03617_amd as mxp  # noqa: E402

TABLES = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_tables.json")))


@pytest.fixture(scope="module")
def ctx():
    c = mxp.Context(0)
    yield c
    c.close()


def solve(ctx, prob, f, shift, fprtol, prec):
    P = mxp.Problem(ctx, prob)
    o = P.default_opts()
    o.precision = prec
    o.rtol = 1e-5          # the paper's outer tolerance
    o.shift = shift
    o.fprtol = fprtol
    fd = torch.from_numpy(f.ravel()).to("cuda:0")
    u = torch.zeros_like(fd)
    st = mxp.mxp_solve(P, o, fd, u)
    P.close()
    assert st["status"] == mxp.MXP_OK and st["true_relres"] <= o.rtol
    return st


def check(st, row):
    assert abs(st["outer_its"] - row["outer"]) <= 1, (st["outer_its"], row)
    assert abs(st["inner_mean"] - row["inner"]) <= 1.0, (st["inner_mean"], row)


@pytest.mark.parametrize("freq", [40, 80])
def test_shift_table_2d(ctx, freq):
    prob = wl.homog_problem(2, freq)
    f = wl.dipole_source(prob)
    for row in (r for r in TABLES["shift_2d"]["rows"] if r["freq"] == freq):
        announce("paper shift table 2d", freq, row["k"])
        check(solve(ctx, prob, f, row["k"] / freq, 0.01, mxp.MXP_PREC_FP64), row)


@pytest.mark.parametrize("freq", [10, 20])
def test_fprtol_table_3d(ctx, freq):
    prob = wl.homog_problem(3, freq)
    f = wl.dipole_source(prob)
    for row in (r for r in TABLES["fprtol_3d"]["rows"] if r["freq"] == freq):
        announce("paper fprtol table 3d", freq, row["fprtol"])
        check(solve(ctx, prob, f, 1.0 / freq, row["fprtol"], mxp.MXP_PREC_FP64), row)


@pytest.mark.parametrize("dim,freq,prec", [(2, 40, 0), (2, 40, 1), (2, 80, 0), (3, 10, 0), (3, 10, 1)])
def test_lens_table(ctx, dim, freq, prec):
    row = next(r for r in TABLES["lens"]["rows"] if r["dim"] == dim and r["freq"] == freq)
    announce("paper lens table", dim, freq, prec)
    prob = wl.lens_problem(dim, freq)
    check(solve(ctx, prob, wl.lens_source(prob), 1.0 / freq, 0.08, prec), row)


@pytest.mark.parametrize("freq", [40, 80])
def test_unshifted_table_2d_first_iteration(ctx, freq):
    # s = 0: the paper tabulates each outer iteration.  The number of outer
    # iterations and the first one (its inner count and the residual after it)
    # are compared; later inner counts depend on where each inner solve of an
    # undamped fixed-point system crosses fprtol and are not pinned.
    row = next(r for r in TABLES["noshift_2d"]["rows"] if r["freq"] == freq)
    announce("paper unshifted table 2d", freq)
    prob = wl.homog_problem(2, freq)
    P = mxp.Problem(ctx, prob)
    o = P.default_opts()
    o.precision = mxp.MXP_PREC_FP64
    o.rtol = 1e-5
    o.shift = 0.0
    o.fprtol = 0.01
    fd = torch.from_numpy(wl.dipole_source(prob).ravel()).to("cuda:0")
    u = torch.zeros_like(fd)
    st = mxp.mxp_solve(P, o, fd, u)
    inner, res = mxp.mxp_solve_history(P)
    P.close()
    assert st["status"] == mxp.MXP_OK
    assert len(inner) == st["outer_its"] == len(res)
    assert abs(len(inner) - len(row["inner"])) <= 1
    assert abs(inner[0] - row["inner"][0]) <= 1
    assert abs(res[0] - row["res"][0]) <= 0.05 * row["res"][0]
