"""mxp_apply_exp_noalloc: the exponential action with no device allocation
(fixed device scratch), through the C ABI, against mxp_apply_exp on two calls
in a row, the second with a smaller input, to the parity bars (complex double
1e-10, complex float 1e-5 relative)."""
import ctypes

import numpy as np
import pytest

import workloads as wl

from gpu_util import announce, rel, to_dev, to_host

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2506_03617_amd as mxp  # noqa: E402


class CountingAllocator(mxp.TorchAllocator):
    def __init__(self):
        super().__init__(0, torch.cuda.current_stream(0))
        self.calls = 0
        inner = self._alloc

        def counted(nbytes, user):
            self.calls += 1
            return inner(nbytes, user)
        self.alloc = mxp.MXP_ALLOC_FN(counted)


def _raw(P, t, s, x, y):
    """The entry point called through ctypes directly (status returned)."""
    dt = mxp.MXP_C128 if x.dtype == torch.complex128 else mxp.MXP_C64
    return mxp.lib.mxp_apply_exp_noalloc(P.handle, ctypes.c_double(t), ctypes.c_double(s), dt,
                                         ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()))


@pytest.mark.parametrize("dt,tol", [("c128", 1e-10), ("c64", 1e-5)])
def test_noalloc_exp_matches_the_allocating_entry_point(dt, tol):
    hooks = CountingAllocator()
    ctx = mxp.Context(0, allocator=hooks)
    tdt = torch.complex128 if dt == "c128" else torch.complex64
    # two calls in a row: a 2D grid of several tiles with ragged edges, then a
    # smaller 3D grid (ragged in every axis)
    probs = [wl.small_problem((301, 213), layer=12, ppw=10, inhomogeneous=True, seed=21, name="na2d"),
             wl.small_problem((60, 31, 23), layer=5, ppw=10, inhomogeneous=True, seed=22, name="na3d")]
    assert probs[1].npts < probs[0].npts
    handles = [mxp.Problem(ctx, p) for p in probs]
    results = []
    for prob, P in zip(probs, handles):
        announce("noalloc exp", dt, prob.n)
        o = P.default_opts()
        x = to_dev(wl.random_vector(prob.npts, 5), tdt)
        y = torch.full_like(x, 7.0)  # every entry must be written
        before = hooks.calls
        assert _raw(P, o.t, o.shift, x, y) == mxp.MXP_OK, mxp.lib.mxp_last_error().decode()
        torch.cuda.synchronize()
        assert hooks.calls == before, "the no-allocation action allocated"
        results.append((prob, P, o, x, y))
    refs = []
    for prob, P, o, x, y in results:
        ref = torch.empty_like(x)
        mxp.mxp_apply_exp(P, o.t, o.shift, x, ref)  # the allocating entry point
        err = rel(to_host(y), to_host(ref))
        assert err <= tol, (prob.n, err)
        assert torch.isfinite(y).all()
        refs.append(ref)
    # the larger call again after the smaller one: the shared scratch keeps no
    # state between calls (2D now runs the tiles mxp_apply_exp tuned)
    for (prob, P, o, x, y), ref in zip(results, refs):
        y2 = torch.full_like(x, -3.0)
        before = hooks.calls
        assert _raw(P, o.t, o.shift, x, y2) == mxp.MXP_OK
        assert hooks.calls == before
        assert rel(to_host(y2), to_host(ref)) <= tol
    for P in handles:
        P.close()
    ctx.close()


def test_noalloc_rejects_inputs_beyond_its_scratch():
    ctx = mxp.Context(0)
    # 300^3 complex double needs about 2.6 GB of buffers: refused before any device work
    prob = wl.Problem("big", (300, 300, 300), 1.0 / 299, wl.omega_for(8, 1.0 / 299), 10, None, 1.0)
    announce("noalloc oversize", prob.n)
    P = mxp.Problem(ctx, prob)
    x = torch.zeros(8, dtype=torch.complex128, device="cuda:0")  # never touched
    y = torch.zeros_like(x)
    st = _raw(P, 1e-5, 0.0, x, y)
    assert st == mxp.MXP_ERR_INVALID_ARG
    assert "scratch" in mxp.lib.mxp_last_error().decode()
    P.close()
    ctx.close()
