"""Device memory through the context's hooks (mxp_context_create's alloc /
release), and the complex-float argument form of mxp_solve and
mxp_apply_precond.

A counting allocator wraps PyTorch's caching allocator.  Every buffer the
library keeps must come from it and go back to it, a call must reserve its
workspace before its device work (no late allocation), and a repeated call
must allocate nothing."""
import ctypes

import numpy as np
import pytest

import workloads as wl

from gpu_util import announce, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2506_03617_amd as mxp  # noqa: E402


class CountingAllocator:
    """Hooks that take memory from torch's caching allocator and record it."""

    def __init__(self, device=0):
        self.stream = torch.cuda.current_stream(device)
        self.device = device
        self.live = {}  # pointer -> bytes
        self.calls = 0
        self.bytes = 0
        self.bad_frees = 0
        self.alloc = mxp.MXP_ALLOC_FN(self._alloc)
        self.free = mxp.MXP_FREE_FN(self._free)

    def _alloc(self, nbytes, user):
        p = torch.cuda.caching_allocator_alloc(int(nbytes), self.device, self.stream)
        self.live[p] = int(nbytes)
        self.calls += 1
        self.bytes += int(nbytes)
        return p

    def _free(self, ptr, user):
        if ptr not in self.live:
            self.bad_frees += 1
            return
        del self.live[ptr]
        torch.cuda.caching_allocator_delete(ptr)


def _stats_agree(ctx, hooks):
    st = ctx.alloc_stats()
    assert st["allocs"] == hooks.calls
    assert st["bytes_live"] == sum(hooks.live.values())
    assert hooks.bad_frees == 0
    return st


@pytest.mark.parametrize("dims", [2, 3])
def test_every_device_byte_comes_from_the_hooks(dims):
    hooks = CountingAllocator()
    ctx = mxp.Context(0, allocator=hooks)
    n = (67, 45) if dims == 2 else (33, 29, 21)
    prob = wl.small_problem(n, layer=6 if dims == 2 else 4, ppw=10, inhomogeneous=True, seed=3, name="alloc")
    announce("alloc hooks", dims, n)
    P = mxp.Problem(ctx, prob)
    assert hooks.calls > 0  # tables and D = 1/c^2 at problem creation
    _stats_agree(ctx, hooks)
    f = to_dev(wl.delta_source(prob, tuple(m // 2 for m in prob.n)))
    for prec in (mxp.MXP_PREC_FP64, mxp.MXP_PREC_MIXED):
        o = P.default_opts()
        o.precision = prec
        u = torch.zeros_like(f)
        st = mxp.mxp_solve(P, o, f, u)
        assert st["status"] == mxp.MXP_OK
        s1 = _stats_agree(ctx, hooks)
        assert s1["late"] == 0, "a solve allocated after reserving its workspace"
        # the same solve again: everything is reserved already
        calls = hooks.calls
        u.zero_()
        st2 = mxp.mxp_solve(P, o, f, u)
        assert st2["outer_its"] == st["outer_its"]
        assert hooks.calls == calls
        # preconditioner apply and actions reuse the solve's workspace
        w = torch.empty_like(f)
        mxp.mxp_apply_precond(P, o, f, w)
        assert hooks.calls == calls
        assert ctx.alloc_stats()["late"] == 0
    # the other building blocks reserve at their entry too
    x = torch.empty_like(f)
    mxp.mxp_apply_psi2(P, o.t, o.shift, f, x)
    mxp.mxp_apply_fn_krylov(P, True, o.t / 8, o.shift, 1e-8, 40, f, x)
    mxp.mxp_apply_exp(P, o.t, o.shift, f.to(torch.complex64), x.to(torch.complex64))
    assert ctx.alloc_stats()["late"] == 0
    P.close()
    st = _stats_agree(ctx, hooks)
    assert st["bytes_live"] == 0 and not hooks.live, "destroy returned every buffer"
    assert st["allocs"] == st["frees"]
    ctx.close()


def test_batched_solve_uses_the_hooks():
    hooks = CountingAllocator()
    ctx = mxp.Context(0, allocator=hooks)
    probs = [wl.small_problem(n, layer=4, ppw=10, inhomogeneous=True, seed=s, name=f"b{s}")
             for s, n in ((1, (33, 29, 21)), (2, (25, 31, 19)))]
    announce("alloc hooks batch", [p.n for p in probs])
    Ps = [mxp.Problem(ctx, p) for p in probs]
    fs, us, opts = [], [], []
    for p, P in zip(probs, Ps):
        f = np.stack([wl.delta_source(p, tuple(m // 2 for m in p.n)).ravel(),
                      wl.random_vector(p.npts, 5)])
        fs.append(to_dev(f))
        us.append(torch.zeros_like(fs[-1]))
        o = P.default_opts()
        o.precision = mxp.MXP_PREC_MIXED
        opts.append(o)
    status, stats = mxp.mxp_solve_batch(ctx, Ps, opts, fs, us)
    assert status == mxp.MXP_OK and len(stats) == 4
    st = _stats_agree(ctx, hooks)
    assert st["late"] == 0, "a batched right-hand side allocated after its reservation"
    for P in Ps:
        P.close()
    st = _stats_agree(ctx, hooks)
    assert st["bytes_live"] == 0 and st["allocs"] == st["frees"]
    ctx.close()


def test_failing_allocator_reports_oom_without_leaks():
    """An allocator that runs dry: OOM status at problem creation or at a
    solve's reservation, and whatever was taken is given back."""
    hooks = CountingAllocator()
    budget = {"left": 3}
    inner = hooks._alloc

    def limited(nbytes, user):
        if budget["left"] <= 0:
            return None
        budget["left"] -= 1
        return inner(nbytes, user)

    hooks.alloc = mxp.MXP_ALLOC_FN(limited)
    ctx = mxp.Context(0, allocator=hooks)
    prob = wl.small_problem((40, 36), layer=6, ppw=10, inhomogeneous=True, seed=1, name="oom")
    announce("alloc hooks oom", prob.n)
    # the problem needs more than three buffers: creation fails cleanly
    with pytest.raises(mxp.MxpError) as ei:
        mxp.Problem(ctx, prob)
    assert ei.value.status == mxp.MXP_ERR_OOM
    assert not hooks.live
    budget["left"] = 10 ** 9
    P = mxp.Problem(ctx, prob)
    f = to_dev(wl.delta_source(prob, (20, 18)))
    u = torch.zeros_like(f)
    budget["left"] = 2  # the solve's reservation runs dry
    with pytest.raises(mxp.MxpError) as ei:
        mxp.mxp_solve(P, P.default_opts(), f, u)
    assert ei.value.status == mxp.MXP_ERR_OOM
    budget["left"] = 10 ** 9  # and recovers once memory is back
    st = mxp.mxp_solve(P, P.default_opts(), f, u)
    assert st["status"] == mxp.MXP_OK
    P.close()
    assert not hooks.live and hooks.bad_frees == 0
    ctx.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_complex_float_arguments_equal_the_widened_double_call(prec):
    """mxp_solve / mxp_apply_precond on complex64 vectors widen them exactly and
    round the result once: the answer equals the complex128 call on the widened
    input, rounded, bit for bit."""
    ctx = mxp.Context(0)
    prob = wl.small_problem((67, 45), layer=8, ppw=10, inhomogeneous=True, seed=4, name="c64io")
    announce("complex-float arguments", prec, prob.n)
    P = mxp.Problem(ctx, prob)
    o = P.default_opts()
    o.precision = prec
    f32 = to_dev(wl.random_vector(prob.npts, 9), torch.complex64)
    f64 = f32.to(torch.complex128)
    u64 = torch.zeros_like(f64)
    st64 = mxp.mxp_solve(P, o, f64, u64)
    u32 = torch.zeros_like(f32)
    st32 = mxp.mxp_solve(P, o, f32, u32)
    assert st32["outer_its"] == st64["outer_its"] and st32["stencil_steps"] == st64["stencil_steps"]
    assert st32["true_relres"] == st64["true_relres"]
    assert torch.equal(u32, u64.to(torch.complex64))
    w64 = torch.empty_like(f64)
    w32 = torch.empty_like(f32)
    its64 = mxp.mxp_apply_precond(P, o, f64, w64)
    its32 = mxp.mxp_apply_precond(P, o, f32, w32)
    assert its32 == its64
    assert torch.equal(w32, w64.to(torch.complex64))
    with pytest.raises(TypeError):
        mxp.mxp_solve(P, o, f32, u64)
    P.close()
    ctx.close()
