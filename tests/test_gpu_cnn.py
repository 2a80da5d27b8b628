"""GPU tests of the learned stage: the bf16 matrix-core network kernels against
the float64 oracle (oracle/conv.py), training steps, and solves that use the
network with the MatExPre fallback.

Tolerance.  The kernels store weights, activations and activation gradients
in bfloat16 and accumulate in float.  The comparisons below hand the oracle
exactly the bfloat16 weights and inputs and round the oracle's activations
and gradients to bfloat16 at the same points the kernels do, so what remains
is float-versus-double accumulation (about 1e-6 relative for the fan-ins
here) and the rare element whose rounding lands on the other side of a
bfloat16 boundary (2^-8 relative each, a small fraction of the elements).
2e-3 relative in the 2-norm covers both with margin; a wrong tap, channel,
transpose or mask is an O(1) error.  Without the rounding emulation the
difference is the bfloat16 error itself (about 1e-2), checked separately
against a looser bound.

Gradients meet a second effect.  A one-ulp bf16 flip in an upstream
activation moves a hidden pre-activation by a few 1e-4; where one lies that
close to zero (in the 9 x 19 x 70 volume, -1.1e-4 against a typical 0.64)
its ReLU mask flips, and one element of that layer's gradient changes by
O(1), which moves a parameter gradient by about 1e-2 relative.  The backward
test therefore reads the activations the kernels stored
(mxp_cnn_get_activations): it checks each against the oracle's forward at
2e-3, checks that the stored masks differ from the oracle's only where a
one-ulp bf16 change of every input of that element could move the oracle's
pre-activation across zero,
and then runs the oracle's backward on those activations and masks, so the
gradients are held to 2e-3 at every volume.
"""
import numpy as np
import pytest

import workloads as wl
from oracle import conv, krylov

from gpu_util import announce, rel, to_dev, to_host

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2506_03617_amd as mxp  # noqa: E402

CH = conv.CHANNELS


@pytest.fixture(scope="module")
def ctx():
    c = mxp.Context(0)
    yield c
    c.close()


def bf16_bits(a):
    f = conv.to_bf16(a).astype(np.float32)
    return (f.view(np.uint32) >> 16).astype(np.uint16)


def make_input(shape, seed):
    nb, nz, ny, nx = shape
    rng = np.random.default_rng(seed)
    x = np.zeros((nb, nz, ny, nx, 8))
    x[..., 0:2] = rng.uniform(-1.0, 1.0, (nb, nz, ny, nx, 2))
    x[..., 2] = rng.uniform(1.0 / 9.0, 1.0, (nb, nz, ny, nx))
    x = conv.to_bf16(x)
    return x, bf16_bits(x)


def layers_of(flat):
    out, off = [], 0
    for cin, cout in zip(CH[:-1], CH[1:]):
        nw = cout * cin * 27
        w = flat[off:off + nw].astype(np.float64).reshape(cout, cin, 3, 3, 3)
        off += nw
        b = flat[off:off + cout].astype(np.float64)
        off += cout
        out.append({"w": w, "b": b})
    return out


def flat_of(layers):
    return np.concatenate([np.concatenate([p["w"].ravel(), p["b"].ravel()]) for p in layers]).astype(np.float32)


def emulated_forward(layers, x):
    """Oracle forward on one volume with the kernels' bfloat16 roundings."""
    h = x[..., :3]
    acts = [h]
    for l, p in enumerate(layers):
        y = conv.conv3d(h, conv.to_bf16(p["w"]), p["b"])
        if l < len(layers) - 1:
            y = conv.to_bf16(np.maximum(y, 0.0))
        acts.append(y)
        h = y
    return h, acts


def emulated_backward(layers, acts, gout):
    g = conv.to_bf16(gout)
    grads = [None] * len(layers)
    for l in range(len(layers) - 1, -1, -1):
        gx, gw, gb = conv.conv3d_backward(acts[l], conv.to_bf16(layers[l]["w"]), g)
        grads[l] = {"w": gw, "b": gb}
        if l > 0:
            g = conv.to_bf16(gx * (acts[l] > 0))
    return grads


SHAPE = (2, 5, 7, 45)  # two volumes; x spans two 32-wide tiles, y and z ragged
# one volume over 3 x 3 columns of 32 x 8 voxels (both ragged) and three z segments
SHAPES = [SHAPE, (1, 9, 19, 70)]


def random_params(seed):
    layers = conv.init_params(seed)
    rng = np.random.default_rng(seed + 1)
    for p in layers:
        p["b"] = rng.normal(0.0, 0.05, p["b"].shape)
    return flat_of(layers)


@pytest.mark.parametrize("shape", SHAPES)
def test_forward_matches_oracle(ctx, shape):
    announce("cnn forward", shape)
    net = mxp.Network(ctx, 1)
    flat = random_params(3)
    net.set_params(flat)
    assert np.array_equal(net.get_params(), flat)
    x, bits = make_input(shape, 4)
    xd = torch.from_numpy(bits.view(np.int16)).to("cuda:0")
    out = torch.empty(int(np.prod(shape[:4])) * 2, dtype=torch.float32, device="cuda:0")
    net.forward(shape, xd, out)
    y = out.cpu().numpy().astype(np.float64).reshape(shape + (2,))
    layers = layers_of(flat)
    for b in range(shape[0]):
        ref, _ = emulated_forward(layers, x[b])
        assert rel(y[b], ref) <= 2e-3
        plain, _ = conv.forward(layers, x[b][..., :3])
        assert rel(y[b], plain) <= 3e-2
    net.close()


def bits_to_f64(bits):
    return (bits.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


@pytest.mark.parametrize("shape", SHAPES)
def test_backward_matches_oracle(ctx, shape):
    announce("cnn backward", shape)
    net = mxp.Network(ctx, 1)
    flat = random_params(5)
    net.set_params(flat)
    x, bits = make_input(shape, 6)
    rng = np.random.default_rng(7)
    gout = rng.standard_normal(shape + (2,)).astype(np.float32)
    net.backward(shape, torch.from_numpy(bits.view(np.int16)).to("cuda:0"),
                 torch.from_numpy(gout.ravel()).to("cuda:0"))
    g = layers_of(net.get_grads())
    layers = layers_of(flat)
    V = int(np.prod(shape))
    stored = [bits_to_f64(net.get_activations(l, V)).reshape(shape + (32,)) for l in range(1, len(layers))]
    ref = None
    flips = 0
    for b in range(shape[0]):
        _, acts = emulated_forward(layers, x[b])
        kernel_acts = [acts[0]]
        for l in range(1, len(layers)):
            a_gpu = stored[l - 1][b]
            assert rel(a_gpu, acts[l]) <= 2e-3, (b, l)
            wl_ = conv.to_bf16(layers[l - 1]["w"])
            pre = conv.conv3d(acts[l - 1], wl_, layers[l - 1]["b"])
            # a one-ulp bf16 change of every input moves the pre-activation by
            # at most 2^-7 sum |w| |a| (plus float accumulation): only inside
            # that band may the stored mask differ from the oracle's
            band = 2.0 ** -7 * conv.conv3d(np.abs(acts[l - 1]), np.abs(wl_), np.zeros_like(layers[l - 1]["b"]))
            differ = (a_gpu > 0) != (pre > 0)
            flips += int(differ.sum())
            assert np.all(np.abs(pre[differ]) <= band[differ] + 1e-6), (b, l)
            kernel_acts.append(a_gpu)
        # the oracle's backward on the kernels' activations and ReLU masks
        gb = emulated_backward(layers, kernel_acts, gout[b].astype(np.float64))
        ref = gb if ref is None else [{k: r[k] + q[k] for k in r} for r, q in zip(ref, gb)]
    assert flips <= 1e-4 * V * 32 * (len(layers) - 1)
    for l in range(len(layers)):
        assert rel(g[l]["w"], ref[l]["w"]) <= 2e-3, l
        assert rel(g[l]["b"], ref[l]["b"]) <= 2e-3, l
    net.close()


def test_training_steps_match_oracle_adam(ctx):
    """Three training steps.  The loss and gradients match the oracle's
    float64 network; the Adam update then matches the oracle's Adam (Kingma and
    Ba; pinned at t >= 2 by closed forms in the CPU tests) fed the kernels' own
    gradients, to float rounding, so a wrong moment or bias correction fails."""
    announce("cnn train")
    net = mxp.Network(ctx, 1)
    flat = random_params(8)
    net.set_params(flat)
    x, bits = make_input(SHAPE, 9)
    rng = np.random.default_rng(10)
    target = rng.standard_normal(SHAPE + (2,)).astype(np.float32) * 0.1
    xd = torch.from_numpy(bits.view(np.int16)).to("cuda:0")
    td = torch.from_numpy(target.ravel()).to("cuda:0")
    layers = layers_of(flat)
    state = {}
    lr = 1e-3
    V = int(np.prod(SHAPE))
    for step in range(3):
        loss = net.train_step(SHAPE, xd, td, lr)
        g_gpu = net.get_grads()
        # oracle: the same loss and gradients in float64 from the same parameters
        grads, lsum = None, 0.0
        for b in range(SHAPE[0]):
            y, acts = emulated_forward(layers, x[b])
            d = y - target[b]
            lsum += float(np.sum(d * d))
            gb = emulated_backward(layers, acts, 2.0 * d / (2 * V))
            grads = gb if grads is None else [{k: r[k] + q[k] for k in r} for r, q in zip(grads, gb)]
        assert abs(loss - lsum / (2 * V)) <= 2e-3 * lsum / (2 * V), step
        assert rel(g_gpu.astype(np.float64), flat_of(grads).astype(np.float64)) <= 2e-3, step
        before = flat_of(layers).astype(np.float64)
        conv.adam_step(layers, layers_of(g_gpu), state, lr)
        after_gpu = net.get_params().astype(np.float64)
        delta_ref = flat_of(layers).astype(np.float64) - before
        delta_gpu = after_gpu - before
        # float32 moments and parameters: the step to ~1e-6 relative, plus the
        # rounding of the stored parameter
        bound = 1e-5 * np.abs(delta_ref) + 2.0 ** -23 * np.abs(after_gpu) + 1e-12
        assert np.all(np.abs(delta_gpu - delta_ref) <= bound), (step, np.max(np.abs(delta_gpu - delta_ref) / bound))
        assert np.abs(delta_ref).max() > 0.5 * lr
        layers = layers_of(after_gpu.astype(np.float32))  # continue both from the kernel's parameters
    net.close()


def test_checkpoint_resumes_training_exactly(ctx, tmp_path):
    announce("cnn checkpoint")
    x, bits = make_input(SHAPE, 21)
    rng = np.random.default_rng(22)
    target = rng.standard_normal(SHAPE + (2,)).astype(np.float32) * 0.1
    xd = torch.from_numpy(bits.view(np.int16)).to("cuda:0")
    td = torch.from_numpy(target.ravel()).to("cuda:0")
    a = mxp.Network(ctx, 31)
    for _ in range(2):
        a.train_step(SHAPE, xd, td, 1e-3)
    path = tmp_path / "net.ckpt"
    a.save(path)
    b = mxp.Network(ctx, 32)
    before = b.get_params()
    # damaged files are rejected and leave the network as it was
    raw = path.read_bytes()
    for bad in (raw[:-4], raw + b"\0", b"XXXXXXXX" + raw[8:]):
        (tmp_path / "bad.ckpt").write_bytes(bad)
        with pytest.raises(mxp.MxpError):
            b.load(tmp_path / "bad.ckpt")
    assert np.array_equal(b.get_params(), before)
    with pytest.raises(mxp.MxpError):
        b.load(tmp_path / "missing.ckpt")
    b.load(path)
    assert np.array_equal(b.get_params(), a.get_params())
    # the Adam state travels too: the next steps agree bit for bit
    for _ in range(2):
        la = a.train_step(SHAPE, xd, td, 1e-3)
        lb = b.train_step(SHAPE, xd, td, 1e-3)
        assert la == lb
        assert np.array_equal(a.get_params(), b.get_params())
    a.close()
    b.close()


def test_learned_solve_converges_to_the_solution(ctx):
    # pairs from one source, a short training run, then a solve of another
    # source with the network tried first: the answer must be the FP64 one
    prob = wl.small_problem((28, 26, 24), layer=4, ppw=10, inhomogeneous=True, seed=11, name="learn")
    announce("learned solve")
    P = mxp.Problem(ctx, prob)
    n = prob.npts
    o = P.default_opts()
    o.precision = mxp.MXP_PREC_MIXED
    f1 = to_dev(wl.delta_source(prob, (10, 12, 9)).ravel())
    u1 = torch.zeros_like(f1)
    maxp = 40
    R = torch.zeros(maxp * n, dtype=torch.complex128, device="cuda:0")
    Z = torch.zeros_like(R)
    cnt, rn, zn, st = mxp.mxp_collect_pairs(P, o, f1, u1, R, Z, maxp)
    assert st["status"] == mxp.MXP_OK and cnt == st["outer_its"] and cnt > 3
    kappa = float(np.median(np.array(zn) / np.array(rn)))
    rs = np.sqrt(n)
    crop = (prob.n[0], prob.n[1], prob.n[2])
    X = torch.empty(cnt * n * 8, dtype=torch.int16, device="cuda:0")
    T = torch.empty(cnt * n * 2, dtype=torch.float32, device="cuda:0")
    for k in range(cnt):
        mxp.mxp_cnn_make_sample(P, R[k * n:(k + 1) * n], Z[k * n:(k + 1) * n], (0, 0, 0), crop, rs, rs / kappa,
                                X[k * n * 8:(k + 1) * n * 8], T[k * n * 2:(k + 1) * n * 2])
    net = mxp.Network(ctx, 12)
    shape = (cnt, prob.n[2], prob.n[1], prob.n[0])
    losses = [net.train_step(shape, X, T, 2e-3) for _ in range(60)]
    assert losses[-1] < losses[0]
    mxp.mxp_problem_set_learned(P, net, kappa)
    f2 = wl.delta_source(prob, (17, 13, 14)).ravel()
    f2d = to_dev(f2)
    o.use_learned = 1
    o.stall_ratio = 0.9
    u2 = torch.zeros_like(f2d)
    st = mxp.mxp_solve(P, o, f2d, u2)
    assert st["status"] == mxp.MXP_OK and st["true_relres"] <= o.rtol
    assert st["learned_its"] + st["fallbacks"] >= 1
    # the adaptive acceptance counts work, not time: repeated solves make the
    # same choices and give the same iterate
    o.stall_ratio = 0.0
    runs = []
    for _ in range(2):
        u2.zero_()
        sa = mxp.mxp_solve(P, o, f2d, u2)
        runs.append(({k: sa[k] for k in ("outer_its", "learned_its", "fallbacks", "stencil_steps")}, u2.clone()))
    assert runs[0][0] == runs[1][0] and torch.equal(runs[0][1], runs[1][1])
    assert sa["status"] == mxp.MXP_OK
    # warm start of the inner GMRES (use_learned = 2): an apply solved tightly
    # from the network's start equals the one solved from zero (same system),
    # and solves converge, deterministically
    ow = P.default_opts()
    ow.fprtol = 1e-11
    ow.inner_restart = 60
    ow.max_inner = 200
    rd = to_dev(wl.random_vector(n, 41))
    w_cold, w_warm = torch.empty_like(rd), torch.empty_like(rd)
    mxp.mxp_apply_precond(P, ow, rd, w_cold)
    ow.use_learned = 2
    mxp.mxp_apply_precond(P, ow, rd, w_warm)
    assert rel(to_host(w_warm), to_host(w_cold)) <= 1e-8
    o.use_learned = 2
    warm = []
    for _ in range(2):
        u2.zero_()
        sw = mxp.mxp_solve(P, o, f2d, u2)
        assert sw["status"] == mxp.MXP_OK and sw["true_relres"] <= o.rtol
        warm.append(({k: sw[k] for k in ("outer_its", "learned_its", "fallbacks", "stencil_steps")}, u2.clone()))
    assert warm[0][0] == warm[1][0] and torch.equal(warm[0][1], warm[1][1])
    assert warm[0][0]["learned_its"] + warm[0][0]["fallbacks"] == warm[0][0]["outer_its"]
    o.use_learned = 1
    # the learned form still reaches the complex-double solution
    o.rtol = 1e-12
    o.precision = mxp.MXP_PREC_FP64
    u2.zero_()
    st = mxp.mxp_solve(P, o, f2d, u2)
    assert st["status"] == mxp.MXP_OK
    assert rel(to_host(u2), krylov.direct_solve(prob, f2)) <= 1e-10
    mxp.mxp_problem_set_learned(P, None, 1.0)
    net.close()
    P.close()


def test_learned_gain_on_a_held_out_source(ctx):
    """What the trained network gains over MatExPre alone, on a source it was
    not trained on.  Measured and printed: the network's relative error on the
    held-out source's own (v_j, M(v_j)) pairs, and the stencil steps and outer
    iterations of the plain mixed solve, the learned-direction solve
    (use_learned = 1, counted-work acceptance) and the warm-started solve
    (use_learned = 2).  Asserted: the network predicts M better than zero does
    on held-out pairs; every form reaches the complex-double true residual;
    a learned-direction solve that keeps no proposal is the plain solve, bit
    for bit, at the same stencil-step count (a rejected try changes nothing)."""
    prob = wl.small_problem((28, 26, 24), layer=4, ppw=10, inhomogeneous=True, seed=11, name="gain")
    announce("learned gain")
    P = mxp.Problem(ctx, prob)
    n = prob.npts
    rs = np.sqrt(n)
    crop = (prob.n[0], prob.n[1], prob.n[2])
    o = P.default_opts()
    o.precision = mxp.MXP_PREC_MIXED

    def pairs(node, maxp=40):
        f = to_dev(wl.delta_source(prob, node).ravel())
        u = torch.zeros_like(f)
        R = torch.zeros(maxp * n, dtype=torch.complex128, device="cuda:0")
        Z = torch.zeros_like(R)
        cnt, rn, zn, st = mxp.mxp_collect_pairs(P, o, f, u, R, Z, maxp)
        assert st["status"] == mxp.MXP_OK
        return cnt, R, Z, np.array(zn) / np.array(rn)

    def samples(cnt, R, Z, kappa):
        X = torch.empty(cnt * n * 8, dtype=torch.int16, device="cuda:0")
        T = torch.empty(cnt * n * 2, dtype=torch.float32, device="cuda:0")
        for k in range(cnt):
            mxp.mxp_cnn_make_sample(P, R[k * n:(k + 1) * n], Z[k * n:(k + 1) * n], (0, 0, 0), crop, rs, rs / kappa,
                                    X[k * n * 8:(k + 1) * n * 8], T[k * n * 2:(k + 1) * n * 2])
        return X, T

    train = [pairs(node) for node in ((10, 12, 9), (18, 8, 15), (7, 18, 12))]
    kappa = float(np.median(np.concatenate([t[3] for t in train])))
    data = [samples(c, R, Z, kappa) for (c, R, Z, _) in train]
    net = mxp.Network(ctx, 21)
    rng = np.random.default_rng(3)
    for step in range(150):
        X, T = data[step % len(data)]
        c = train[step % len(data)][0]
        b = int(rng.integers(0, c - 1))
        shape = (2, prob.n[2], prob.n[1], prob.n[0])
        net.train_step(shape, X[b * n * 8:(b + 2) * n * 8], T[b * n * 2:(b + 2) * n * 2], 1e-3)
    # held-out source: prediction error on its own pairs
    held = (17, 13, 14)
    c, R, Z, _ = pairs(held)
    X, T = samples(c, R, Z, kappa)
    errs = []
    for k in range(c):
        out = torch.empty(n * 2, dtype=torch.float32, device="cuda:0")
        net.forward((1, prob.n[2], prob.n[1], prob.n[0]), X[k * n * 8:(k + 1) * n * 8], out)
        t = T[k * n * 2:(k + 1) * n * 2].double()
        errs.append(((out.double() - t).norm() / t.norm()).item())
    assert np.median(errs) < 1.0, errs
    # the three forms on the held-out source
    mxp.mxp_problem_set_learned(P, net, kappa)
    f = to_dev(wl.delta_source(prob, held).ravel())
    res = {}
    for mode in (0, 1, 2):
        o.use_learned = mode
        o.stall_ratio = 0.0
        u = torch.zeros_like(f)
        st = mxp.mxp_solve(P, o, f, u)
        assert st["status"] == mxp.MXP_OK and st["true_relres"] <= o.rtol, (mode, st)
        res[mode] = (st, u)
    plain, learned, warm = (res[m][0] for m in (0, 1, 2))
    if learned["learned_its"] == 0:
        assert learned["stencil_steps"] == plain["stencil_steps"]
        assert learned["outer_its"] == plain["outer_its"]
        assert torch.equal(res[1][1], res[0][1])
    gain = {"held_out_pair_err_median": round(float(np.median(errs)), 3),
            "plain": (plain["outer_its"], plain["stencil_steps"]),
            "learned": (learned["outer_its"], learned["stencil_steps"], learned["learned_its"], learned["fallbacks"]),
            "warm": (warm["outer_its"], warm["stencil_steps"], warm["learned_its"], warm["fallbacks"]),
            "steps_gain_learned": round(plain["stencil_steps"] / learned["stencil_steps"], 4),
            "steps_gain_warm": round(plain["stencil_steps"] / warm["stencil_steps"], 4)}
    announce("learned gain measured", gain)
    mxp.mxp_problem_set_learned(P, None, 1.0)
    net.close()
    P.close()


def test_failure_paths_are_reported_and_recovered(ctx):
    """Forced failures: a network with zero weights proposes z = 0, every try
    is rejected and the solve is MatExPre's (the FP64 true residual judges);
    fprtol = 1 makes Algorithm 1 return w = 0 before its first iteration, and
    FGMRES reports the singular direction as MXP_ERR_BREAKDOWN instead of
    returning a wrong iterate."""
    prob = wl.small_problem((28, 26, 24), layer=4, ppw=10, inhomogeneous=True, seed=11, name="fail")
    announce("failure paths")
    P = mxp.Problem(ctx, prob)
    f = to_dev(wl.delta_source(prob, (17, 13, 14)).ravel())
    o = P.default_opts()
    o.precision = mxp.MXP_PREC_MIXED
    u = torch.zeros_like(f)
    plain = mxp.mxp_solve(P, o, f, u)
    u_plain = u.clone()
    net = mxp.Network(ctx, 5)
    net.set_params(np.zeros(mxp.Network.num_params(), dtype=np.float32))
    mxp.mxp_problem_set_learned(P, net, 1.0)
    o.use_learned = 1
    o.stall_ratio = 0.0
    u.zero_()
    st = mxp.mxp_solve(P, o, f, u)
    assert st["status"] == mxp.MXP_OK and st["true_relres"] <= o.rtol
    assert st["learned_its"] == 0 and st["fallbacks"] >= 1
    assert st["outer_its"] == plain["outer_its"] and torch.equal(u, u_plain)
    mxp.mxp_problem_set_learned(P, None, 1.0)
    net.close()
    ob = P.default_opts()
    ob.fprtol = 1.0
    u.zero_()
    with pytest.raises(mxp.MxpError) as ei:
        mxp.mxp_solve(P, ob, f, u)
    assert ei.value.status == mxp.MXP_ERR_BREAKDOWN
    assert torch.isfinite(u).all()
    P.close()
