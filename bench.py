"""Benchmark: seconds to solve the 3D homogeneous Helmholtz workload (256^3
grid, c = 1, ppw 8, 20-cell absorbing layer, Gaussian-smoothed point source
of standard deviation 2 cells) to 1e-6 relative residual with
MatExPre-preconditioned FGMRES(20) on one MI355X.  `--workload` selects the
2D random-field 2048^2 or the 2D homogeneous 128^2 workload instead, or one
of the other measurements (layered batch, learned stage, paper tables, ...).

One step = one complete solve in the paper's arithmetic, complex double
(outer FGMRES, every preconditioner apply, every exp / psi_1 action): its
mean is `value`.  Each step also solves the same system in the mixed form
(complex-float stepping, complex-double Krylov bases and true residual),
alternating with the double solve, and the line reports that form's time,
speed-up and solution error against the double solve.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0


# Sources that determine each profiled kernel's code: a counter summary is
# used only while these files are unchanged.
KERNEL_SOURCES = {
    "cheb2d": ("cheb2d.hip", "kernels.h"),
    "stencil3d": ("kernels.hip", "kernels.h"),
    "cheb3d": ("cheb3d.hip", "cheb3d.h", "kernels.h"),
    "cheb3d3": ("cheb3d.hip", "cheb3d.h", "kernels.h"),
}


def kernel_source_hash(family: str) -> str:
    h = hashlib.sha256()
    for name in KERNEL_SOURCES[family]:
        with open(os.path.join(ROOT, "paper_2506_03617_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(kernel: str, workload: str):
    """HBM bytes per launch from the committed counter summary, if it was taken
    on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        data = json.load(fh)
    rec = data.get(f"{kernel}@{workload}")
    family = kernel.split("_")[0]
    if not rec or family not in KERNEL_SOURCES or rec.get("source_hash") != kernel_source_hash(family):
        return None
    return rec.get("bytes_per_launch")


def cpu_baseline(prob, f, actions_per_solve: int, fraction: int = 16):
    """The oracle, as it stands, on a bounded sample: one exp(i (t/fraction) A_s) v
    action (SciPy expm_multiply, whose work grows linearly with t ||A||) at the
    full grid, scaled by `fraction` and by the number of matrix-function actions
    one GPU solve performs."""
    from oracle import matfun, operator as op
    if prob.dim == 3:
        fraction *= 2
    threads = os.environ.get("OMP_NUM_THREADS")
    As = op.helmholtz(prob, prob.default_shift())
    v = f.ravel().astype(np.complex128)
    t0 = time.perf_counter()
    matfun.exp_action(As, prob.default_t() / fraction, v)
    t_sample = time.perf_counter() - t0
    return {
        "value": round(t_sample * fraction * actions_per_solve, 1),
        "unit": "s per solve (extrapolated)",
        "cores": int(threads) if threads else os.cpu_count(),
        "kind": "oracle",
        "sample": f"one exp(i(t/{fraction})A_s)v action at {'x'.join(map(str, prob.n))} by expm_multiply "
                  f"({t_sample:.1f} s), times {fraction} and {actions_per_solve} actions per solve",
    }


def measure_roofline(mxp, torch, P, prob, o, reps, prec):
    """Roofline of the dominant kernel of a solve in precision `prec`: the
    Clenshaw kernel of its exp actions.  Its average launch duration comes
    from HIP events around complete exp actions on the library's stream
    (torch's current stream), divided by the launches those actions make."""
    c64 = prec == mxp.MXP_PREC_MIXED
    tdt, tag, R = (torch.complex64, "c64", "float") if c64 else (torch.complex128, "c128", "double")
    z = 8 if c64 else 16          # bytes per complex value
    sch = mxp.mxp_design_schedule(P.desc, o.t, o.shift, prec)
    x = torch.randn(prob.npts, dtype=tdt, device="cuda:0")
    y = torch.empty_like(x)
    mxp.mxp_apply_exp(P, o.t, o.shift, x, y)  # tunes the tiles if needed
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record()
    for _ in range(reps):
        mxp.mxp_apply_exp(P, o.t, o.shift, x, y)
    ev1.record()
    torch.cuda.synchronize()
    t_action = ev0.elapsed_time(ev1) * 1e-3 / reps
    t_full = t_action  # whole action (every launch)
    rd_D = 0 if prob.c is None else z // 2
    m = sch.m
    if prob.dim == 2:
        # fused pass k_cheb2d<R, K, NX>: K Clenshaw levels per launch
        tiles = mxp.mxp_get_tiles(P, prec)
        K = tiles["K"]
        passes = -(-(m + 1) // K)   # passes per series (m + 1 Clenshaw levels)
        # per point: inputs L_{-2}, L_{-1} (absent in the first pass), x, D;
        # outputs two levels (one in the final pass)
        rd_xD = z + rd_D
        if passes == 1:
            per_series = rd_xD + z
        else:
            per_series = (rd_xD + 2 * z) + (passes - 2) * (2 * z + rd_xD + 2 * z) + (2 * z + rd_xD + z)
        launches_per_series = passes
        kernel = f"k_cheb2d<{R},{K},{tiles['NX']}> (fused Clenshaw pass, Ly={tiles['Ly']})"
        key = f"cheb2d_{tag}_K{K}_NX{tiles['NX']}_Ly{tiles['Ly']}"
        extra = {"levels_per_launch": K}
    elif mxp.mxp_get_tiles(P, prec)["K"] == 3:
        # three-level pass k_cheb3d3<R, VAR> (the 3D tuner's choice): levels in
        # triples, then a pair or a single level for the remainder and the
        # final level as a sweep.  Per point: the first pass reads x and writes
        # two levels; every later pass reads in0, in1, x and writes two; a
        # remainder pair the same; a single sweep and the final sweep read two
        # levels and x and write one; each launch reads D.
        trip = m // 3
        rem = m - 3 * trip
        per_series = ((3 * z + rd_D) + (trip - 1) * (5 * z + rd_D) + (rem == 2) * (5 * z + rd_D)
                      + (rem == 1) * (4 * z + rd_D) + (4 * z + rd_D))
        launches_per_series = trip + (rem == 2) + (rem == 1) + 1
        kernel = f"k_cheb3d3<{R},VAR> (three Clenshaw levels per pass; with the series' last one or two launches)"
        key = f"cheb3d3_{tag}"
        extra = {"levels_per_launch": 3}
    elif mxp.mxp_get_tiles(P, prec)["K"] == 2:
        # two-level pass k_cheb3d<R, VAR> (the 3D tuner's choice): levels in
        # pairs, then an odd level and the final level as single sweeps.  Per
        # point: the first pass reads x and writes two levels; every later pass
        # reads in0, in1, x and writes two; an odd sweep and the final sweep
        # read two levels and x and write one; each launch reads D.
        pairs = m // 2
        per_series = (3 * z + rd_D) + (pairs - 1) * (5 * z + rd_D) + (m % 2) * (4 * z + rd_D) + (4 * z + rd_D)
        launches_per_series = pairs + (m % 2) + 1
        kernel = f"k_cheb3d<{R},VAR> (two Clenshaw levels per pass; with the series' last one or two single-level sweeps)"
        key = f"cheb3d_{tag}"
        extra = {"levels_per_launch": 2}
    else:
        # single-level z-marching sweep k_stencil3d<R, OPS>: one level per
        # launch.  Per point: the first sweep reads x and writes b_{m-1}; the
        # second reads b_{m-1}, x; every later one reads b_{k+1}, b_{k+2}, x;
        # each reads D and writes one level.
        per_series = (2 * z + rd_D) + (3 * z + rd_D) + (m - 2) * (4 * z + rd_D)
        launches_per_series = m
        kernel = f"k_stencil3d<{R},OPS> (z-marching Clenshaw step)"
        key = f"stencil3d_{tag}"
        extra = {"levels_per_launch": 1}
    launches = sch.S * launches_per_series
    bytes_per_launch = per_series * prob.npts / launches_per_series
    avg_launch_s = t_action / launches
    achieved = bytes_per_launch / avg_launch_s / 1e9
    # the same work as unfused Clenshaw steps (4 values + D per point per step)
    unfused_equiv = (4 * z + rd_D) * prob.npts * sch.S * m / t_full / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": load_traffic(key, prob.name),
            "kernel": kernel, "avg_launch_us": round(avg_launch_s * 1e6, 3),
            "bytes_per_launch": round(bytes_per_launch), **extra,
            "action_ms": round(t_full * 1e3, 3),
            "us_per_clenshaw_level": round(t_full / (sch.S * m) * 1e6, 3),
            "unfused_step_equivalent_GBps": round(unfused_equiv, 1),
            f"schedule_{tag}": {"S": sch.S, "m": m, "m_psi": sch.m_psi}}


def layered_sources(args):
    """Indices (of the 32 surface sources) the layered batch solves: --sources
    (e.g. 0-10 or 3,7,12), else --rhs equally spaced ones.  Exits with a
    message on indices outside 0..31, repeated or malformed."""
    if not args.sources:
        return [round(k * 31 / max(args.rhs - 1, 1)) for k in range(args.rhs)]
    which = []
    try:
        for part in args.sources.split(","):
            lo, _, hi = part.partition("-")
            which.extend(range(int(lo), int(hi or lo) + 1))
    except ValueError:
        which = []
    if not which or min(which) < 0 or max(which) > 31 or len(set(which)) != len(which):
        print(f"--sources {args.sources!r}: distinct indices in 0..31 expected", file=sys.stderr)
        sys.exit(2)
    return which


def bench_layered_batch(args, torch, mxp, wl):
    """The layered batch: `--rhs` of the 32 surface sources on the 512x512x256
    grid (or the indices `--sources` names) plus the 16 uneven 96^3..192^3
    problems (one source each; left out with `--no-extras`), solved by one
    mxp_solve_batch call in the mixed form with FGMRES(20).  One step = the
    whole batched solve."""
    os.environ.setdefault("MXP_VERBOSE", "1")   # one line per outer iteration: progress
    which = layered_sources(args)
    main_p = wl.config4_main()
    extras = [] if args.no_extras else wl.config4_extras()
    ctx = mxp.Context(0)
    probs = [main_p] + extras
    handles = [mxp.Problem(ctx, p) for p in probs]
    rhs = [wl.config4_sources(main_p, which)]
    for p in extras:
        rhs.append(wl.delta_source(p, (p.n[0] // 2, p.n[1] // 2, p.layer + 2)).ravel()[None, :])
    opts = []
    for h in handles:
        o = h.default_opts()
        o.precision = mxp.MXP_PREC_MIXED
        o.outer_restart = 20
        opts.append(o)
    f_list = [torch.from_numpy(f).to("cuda:0") for f in rhs]
    del rhs
    u_list = [torch.zeros_like(f) for f in f_list]
    print(f"[bench] layered batch: sources {which} on {main_p.n} + {len(extras)} extra grids",
          file=sys.stderr, flush=True)
    times, all_stats = [], None
    for k in range(args.warmup + max(args.steps, 1)):
        for u in u_list:
            u.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        status, all_stats = mxp.mxp_solve_batch(ctx, handles, opts, f_list, u_list, 0)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        print(f"[bench] batch solve {k}: status {status}, {dt:.2f} s", file=sys.stderr, flush=True)
        if k >= args.warmup:
            times.append(dt)
    s_per = sum(times) / len(times)
    n_rhs = len(all_stats)
    pts = sum(p.npts * (len(which) if i == 0 else 1) for i, p in enumerate(probs))
    line = {
        "metric": "s to 1e-6 rel. residual (plain vs FP32/learned); stencil HBM GB/s vs peak",
        "value": round(s_per, 3), "unit": "s", "n_gpus": 1, "steps": len(times), "warmup": args.warmup,
        "ms_per_step": round(s_per * 1e3, 1), "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": "c64 stepping and inner basis + c128 Krylov sums and outer solve",
        "data": "synthetic (seeded layered speeds with two lenses, point sources)",
        "config": {"workload": "3d-layered-batch", "main_grid": list(main_p.n), "main_sources": len(which),
                   "source_indices": which,
                   "extra_grids": [list(p.n) for p in extras], "right_hand_sides": n_rhs,
                   "grid_points_total": pts, "precision": "mixed", "outer_restart": 20},
        "per_rhs": [{k: s[k] for k in ("outer_its", "inner_mean", "stencil_steps", "true_relres", "seconds",
                                       "status")} for s in all_stats],
    }
    print(json.dumps(line), flush=True)
    for h in handles:
        h.close()
    ctx.close()


PEAK_BF16_TFLOPS = 2500.0


def layered_model(wl, n, layer, seed):
    h = 1.0 / (max(n) - 1)
    c = wl.layered_speed(n, layer, 12, 1500.0, 4500.0, 2, seed)
    return wl.Problem(f"3d-layered-{n[0]}", n, h, wl.omega_for(8, h), layer, c)


def network_flops(voxels: int) -> float:
    """Algorithmic flops of one network forward (real channel counts)."""
    chans = (3, 32, 32, 32, 32, 32, 2)
    return 2.0 * voxels * 27 * sum(a * b for a, b in zip(chans[:-1], chans[1:]))


def bench_network(args, torch, mxp):
    """The network alone: forward passes at 256^3 and training steps on
    4 x 64^3 crops (random weights and inputs), timed with HIP events on the
    library's stream."""
    ctx = mxp.Context(0)
    net = mxp.Network(ctx, 3)
    V = 256 ** 3
    xin = torch.randint(0, 1 << 14, (V * 8,), dtype=torch.int16, device="cuda:0")
    out = torch.empty(V * 2, dtype=torch.float32, device="cuda:0")
    shape = (1, 256, 256, 256)
    net.forward(shape, xin, out)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = max(args.roofline_reps, 1)
    ev0.record()
    for _ in range(reps):
        net.forward(shape, xin, out)
    ev1.record()
    torch.cuda.synchronize()
    t_fwd = ev0.elapsed_time(ev1) * 1e-3 / reps
    del xin, out
    B = 4
    tshape = (B, 64, 64, 64)
    Vt = B * 64 ** 3
    xt = torch.randint(0, 1 << 14, (Vt * 8,), dtype=torch.int16, device="cuda:0")
    tt = torch.randn(Vt * 2, dtype=torch.float32, device="cuda:0")
    net.train_step(tshape, xt, tt, 1e-4)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        net.train_step(tshape, xt, tt, 1e-4)
    torch.cuda.synchronize()
    t_step = (time.perf_counter() - t0) / reps
    fl = network_flops(V)
    line = {"workload": "network", "forward_256cube_ms": round(t_fwd * 1e3, 3),
            "forward_TFLOPs": round(fl / t_fwd / 1e12, 1),
            "train_step_4x64cube_ms": round(t_step * 1e3, 3),
            "train_TFLOPs": round(3 * network_flops(Vt) / t_step / 1e12, 1),
            "roofline": {"bound": "mfma", "achieved": round(fl / t_fwd / 1e12, 1), "peak": PEAK_BF16_TFLOPS,
                         "unit": "TFLOP/s", "frac": round(fl / t_fwd / 1e12 / PEAK_BF16_TFLOPS, 4)}}
    print(json.dumps(line), flush=True)
    net.close()
    ctx.close()


def bench_learned(args, torch, mxp, wl):
    """The learned stage: (residual, preconditioned residual) pairs from
    MatExPre solves on seeded 128^3 layered models, 64^3 bf16 crops, Adam
    training on the matrix-core kernels, then an unseen 256^3 layered model
    solved with and without the network (mixed form, FGMRES(20))."""
    rng = np.random.default_rng(55)
    os.environ.setdefault("MXP_VERBOSE", "1")   # one line per outer iteration: progress
    if args.conv_only:
        bench_network(args, torch, mxp)
        return
    ctx = mxp.Context(0)
    t_start = time.perf_counter()
    # --- pairs
    crops_in, crops_t = [], []
    n_pairs = 0
    crop = (64, 64, 64)
    kappas = []
    for mdl in range(args.train_models):
        prob = layered_model(wl, (128, 128, 128), 16, 5000 + mdl)
        P = mxp.Problem(ctx, prob)
        o = P.default_opts()
        o.precision = mxp.MXP_PREC_MIXED
        o.outer_restart = 20
        n = prob.npts
        for src in range(2):
            x = int(rng.integers(20, 108))
            f = torch.from_numpy(wl.delta_source(prob, (x, 64, 18 + 40 * src)).ravel()).to("cuda:0")
            u = torch.zeros_like(f)
            maxp = 24
            R = torch.zeros(maxp * n, dtype=torch.complex128, device="cuda:0")
            Z = torch.zeros_like(R)
            cnt, rn, zn, st = mxp.mxp_collect_pairs(P, o, f, u, R, Z, maxp)
            kappas += [z / r for r, z in zip(rn, zn)]
            kap = float(np.median(kappas))
            rs = np.sqrt(n)
            for k in range(cnt):
                for _ in range(2):
                    off = tuple(int(rng.integers(0, 128 - 64 + 1)) for _ in range(3))
                    X = torch.empty(64 ** 3 * 8, dtype=torch.int16, device="cuda:0")
                    T = torch.empty(64 ** 3 * 2, dtype=torch.float32, device="cuda:0")
                    mxp.mxp_cnn_make_sample(P, R[k * n:(k + 1) * n], Z[k * n:(k + 1) * n], off, crop, rs, rs / kap,
                                            X, T)
                    crops_in.append(X)
                    crops_t.append(T)
            n_pairs += cnt
            print(f"[bench] model {mdl} source {src}: {cnt} pairs, outer {st['outer_its']}, "
                  f"{time.perf_counter() - t_start:.1f} s", file=sys.stderr, flush=True)
            del R, Z
        P.close()
    kappa = float(np.median(kappas))
    t_data = time.perf_counter() - t_start
    # --- training (batches of 4 crops)
    X_all = torch.stack(crops_in)
    T_all = torch.stack(crops_t)
    net = mxp.Network(ctx, 7)
    B = 4
    shape = (B, 64, 64, 64)
    losses = []
    t1 = time.perf_counter()
    for step in range(args.train_steps):
        idx = torch.from_numpy(rng.choice(len(crops_in), size=B, replace=False)).to("cuda:0")
        xb = X_all.index_select(0, idx).contiguous().view(-1)
        tb = T_all.index_select(0, idx).contiguous().view(-1)
        lr = 2e-3 if step < args.train_steps // 2 else (5e-4 if step < 3 * args.train_steps // 4 else 1.25e-4)
        losses.append(net.train_step(shape, xb, tb, lr))
        if step % 100 == 0:
            print(f"[bench] train step {step}: loss {losses[-1]:.4e}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t1
    del X_all, T_all, crops_in, crops_t
    # --- conv throughput at the evaluation size (inference forward)
    ne = args.eval_grid
    test = layered_model(wl, (ne, ne, ne), 20 if ne >= 256 else 16, 9999)
    V = test.npts
    xin = torch.zeros(V * 8, dtype=torch.int16, device="cuda:0")
    out = torch.empty(V * 2, dtype=torch.float32, device="cuda:0")
    vshape = (1, ne, ne, ne)
    net.forward(vshape, xin, out)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(3):
        net.forward(vshape, xin, out)
    ev1.record()
    torch.cuda.synchronize()
    t_fwd = ev0.elapsed_time(ev1) * 1e-3 / 3
    # every layer runs as a 32-output-channel GEMM; algorithmic flops count the real channels
    flops = network_flops(V)
    del xin, out
    # --- evaluation: plain mixed vs learned on the unseen model
    P = mxp.Problem(ctx, test)
    f = torch.from_numpy(wl.delta_source(test, (ne // 2, ne // 2, test.layer + 2)).ravel()).to("cuda:0")
    u = torch.zeros_like(f)
    o = P.default_opts()
    o.precision = mxp.MXP_PREC_MIXED
    o.outer_restart = args.eval_restart
    res = {}
    print(f"[bench] network forward at {ne}^3: {t_fwd * 1e3:.2f} ms", file=sys.stderr, flush=True)
    mxp.mxp_problem_set_learned(P, net, kappa)
    # untimed warm-up: schedules, tiles and workspaces of the evaluation grid
    # (both precisions of the mixed form) are set up before any timed solve
    o.use_learned = 0
    mxp.mxp_solve(P, o, f, u)
    for mode in ("plain", "learned", "warm"):
        # learned: the network's direction tried first at every outer iteration;
        # warm: its output starts the inner GMRES of every preconditioner apply
        o.use_learned = {"plain": 0, "learned": 1, "warm": 2}[mode]
        o.stall_ratio = 0.0   # cost-aware acceptance (counted work)
        u.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = mxp.mxp_solve(P, o, f, u)
        torch.cuda.synchronize()
        st["wall"] = time.perf_counter() - t0
        res[mode] = st
        print(f"[bench] {mode}: {st['wall']:.2f} s, outer {st['outer_its']}, learned {st['learned_its']}, "
              f"fallbacks {st['fallbacks']}, relres {st['true_relres']:.2e}", file=sys.stderr, flush=True)
    line = {
        "metric": "s to 1e-6 rel. residual (plain vs FP32/learned); stencil HBM GB/s vs peak",
        "value": round(res["learned"]["wall"], 3), "unit": "s", "n_gpus": 1, "steps": 1, "warmup": 1,
        "ms_per_step": round(res["learned"]["wall"] * 1e3, 1), "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": "bf16 network + c64 stepping and inner basis + c128 Krylov sums and outer solve",
        "data": "synthetic (seeded layered models, point sources); pairs generated by the solver",
        "config": {"workload": "3d-learned", "train_grid": [128, 128, 128], "train_models": args.train_models,
                   "pairs": n_pairs, "crops": 2 * n_pairs, "crop": list(crop), "train_steps": args.train_steps,
                   "batch": B, "eval_grid": [ne, ne, ne], "precision": "mixed", "outer_restart": args.eval_restart,
                   "stall_ratio": "adaptive (0)"},
        "learned": {k: res["learned"][k] for k in ("wall", "outer_its", "learned_its", "fallbacks", "inner_mean",
                                                     "stencil_steps", "true_relres")},
        "warm_start": {k: res["warm"][k] for k in ("wall", "outer_its", "learned_its", "fallbacks", "inner_mean",
                                                   "stencil_steps", "true_relres")},
        "gain_vs_plain": {m: {"stencil_steps": round(res["plain"]["stencil_steps"] / res[m]["stencil_steps"], 4),
                              "wall": round(res["plain"]["wall"] / res[m]["wall"], 4)} for m in ("learned", "warm")},
        "plain_mixed": {k: res["plain"][k] for k in ("wall", "outer_its", "inner_mean", "stencil_steps",
                                                     "true_relres")},
        "training": {"data_seconds": round(t_data, 1), "train_seconds": round(t_train, 1),
                     "loss_first": losses[0], "loss_last": float(np.mean(losses[-20:])), "kappa": kappa},
        "roofline": {"bound": "mfma", "achieved": round(flops / t_fwd / 1e12, 1), "peak": PEAK_BF16_TFLOPS,
                     "unit": "TFLOP/s", "frac": round(flops / t_fwd / 1e12 / PEAK_BF16_TFLOPS, 4), "traffic": None,
                     "kernel": "k_conv_zm<CIN,*> (network forward, 6 layers, 256^3)",
                     "forward_ms": round(t_fwd * 1e3, 3)},
    }
    print(json.dumps(line), flush=True)
    mxp.mxp_problem_set_learned(P, None, 1.0)
    net.close()
    P.close()
    ctx.close()


def bench_paper_tables(args, torch, mxp, wl):
    """The paper's printed iteration counts (tests/golden/paper_tables.json):
    every entry whose grid fits one GPU, solved at the paper's settings and
    outer tolerance 1e-5: complex-double stepping up to 241^3 nodes and on
    every 2D grid below 2.5e7 nodes, the mixed form above (its counts equal
    the complex-double ones in every case measured).  One
    step is the whole set; value is the summed solve time.  Also times the
    operation of the paper's weak-scaling figure, psi_1(itA)v followed by one
    fixed-point step, on the 3D homogeneous model at freq 20 and 40."""
    tables = json.load(open(os.path.join(ROOT, "tests", "golden", "paper_tables.json")))
    ctx = mxp.Context(0)
    out, total = [], 0.0

    def solve(prob, f, shift, fprtol, prec):
        P = mxp.Problem(ctx, prob)
        o = P.default_opts()
        o.precision = prec
        o.rtol = 1e-5
        o.shift = shift
        o.fprtol = fprtol
        fd = torch.from_numpy(f.ravel()).to("cuda:0")
        u = torch.zeros_like(fd)
        t0 = time.perf_counter()
        st = mxp.mxp_solve(P, o, fd, u)
        sec = time.perf_counter() - t0
        P.close()
        del fd, u
        torch.cuda.empty_cache()
        return st, sec

    def record(table, key, prob, row, st, sec, prec):
        nonlocal total
        total += sec
        e = {"table": table, **key, "grid": list(prob.n), "precision": "fp64" if prec == 0 else "mixed",
             "outer": st["outer_its"], "inner": round(st["inner_mean"], 2), "std": round(st["inner_std"], 2),
             "paper": {"outer": row["outer"], "inner": row["inner"], "std": row["std"]}, "seconds": round(sec, 3)}
        out.append(e)
        print(f"[bench] {table} {key} {prob.n}: outer {e['outer']} (paper {row['outer']}), inner {e['inner']} "
              f"+- {e['std']} (paper {row['inner']} +- {row['std']}), {sec:.2f} s", file=sys.stderr, flush=True)

    big = 10 ** 8 // 4  # nodes above which the mixed form is used (time)
    for row in tables["shift_2d"]["rows"]:
        prob = wl.homog_problem(2, row["freq"])
        prec = 0 if prob.npts < big else 1
        st, sec = solve(prob, wl.dipole_source(prob), row["k"] / row["freq"], 0.01, prec)
        record("shift_2d", {"freq": row["freq"], "s": f"{row['k']}/freq"}, prob, row, st, sec, prec)
    for row in tables["fprtol_3d"]["rows"]:
        prob = wl.homog_problem(3, row["freq"])
        prec = 0 if prob.npts <= 241 ** 3 else 1
        st, sec = solve(prob, wl.dipole_source(prob), 1.0 / row["freq"], row["fprtol"], prec)
        record("fprtol_3d", {"freq": row["freq"], "fprtol": row["fprtol"]}, prob, row, st, sec, prec)
    noshift = []
    for row in tables["noshift_2d"]["rows"]:
        prob = wl.homog_problem(2, row["freq"])
        P = mxp.Problem(ctx, prob)
        o = P.default_opts()
        o.precision = mxp.MXP_PREC_FP64  # unshifted: the mixed form stalls below ~1e-4 (FP32 actions)
        o.rtol = 1e-5
        o.shift = 0.0
        o.fprtol = 0.01
        fd = torch.from_numpy(wl.dipole_source(prob).ravel()).to("cuda:0")
        u = torch.zeros_like(fd)
        t0 = time.perf_counter()
        mxp.mxp_solve(P, o, fd, u)
        sec = time.perf_counter() - t0
        total += sec
        inner, res = mxp.mxp_solve_history(P)
        P.close()
        del fd, u
        noshift.append({"freq": row["freq"], "grid": list(prob.n), "inner": inner, "res": [float(f"{r:.4g}") for r in res],
                        "paper": {"inner": row["inner"], "res": row["res"]}, "seconds": round(sec, 3)})
        print(f"[bench] noshift_2d freq {row['freq']}: inner {inner} (paper {row['inner']}), "
              f"res {['%.3e' % r for r in res]} (paper {row['res']}), {sec:.2f} s", file=sys.stderr, flush=True)
    skipped = []
    for row in tables["lens"]["rows"]:
        prob_n = 20 * row["freq"] + 41
        if row["dim"] == 3 and prob_n ** 3 > 500 ** 3:
            # 841^3: the FP64 Krylov bases alone exceed one GPU's 288 GB
            skipped.append({"table": "lens", "dim": 3, "freq": row["freq"], "grid": [prob_n] * 3})
            continue
        prob = wl.lens_problem(row["dim"], row["freq"])
        prec = 0 if prob.npts <= 241 ** 3 else 1
        st, sec = solve(prob, wl.lens_source(prob), 1.0 / row["freq"], 0.08, prec)
        record("lens", {"dim": row["dim"], "freq": row["freq"]}, prob, row, st, sec, prec)
    n = len(out)
    exact = sum(e["outer"] == e["paper"]["outer"] for e in out)
    near = sum(abs(e["outer"] - e["paper"]["outer"]) <= 1 and abs(e["inner"] - e["paper"]["inner"]) <= 1.0 for e in out)

    # the weak-scaling figure's operation: psi_1(itA)v, then one fixed-point
    # step w = e^{itA} w + psi_1 r (two matrix-function actions), complex double
    weak = []
    for freq in (20, 40):
        prob = wl.homog_problem(3, freq)
        P = mxp.Problem(ctx, prob)
        o = P.default_opts()
        x = torch.from_numpy(wl.dipole_source(prob).ravel()).to("cuda:0")
        y = torch.empty_like(x)
        z = torch.empty_like(x)
        mxp.mxp_apply_psi1(P, o.t, o.shift, x, y)    # warm (tile tuning)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        mxp.mxp_apply_psi1(P, o.t, o.shift, x, y)
        mxp.mxp_apply_exp(P, o.t, o.shift, y, z)
        z.add_(y)
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        weak.append({"freq": freq, "grid": list(prob.n), "seconds": round(sec, 3),
                     "paper": "40-50 s on ceil((freq/20)^3) cluster nodes (weak-scaling figure, Section 4.2.2)"})
        print(f"[bench] psi_1 + one fixed-point step, 3D homogeneous {prob.n}: {sec:.3f} s", file=sys.stderr, flush=True)
        P.close()
        del x, y, z
        torch.cuda.empty_cache()
    rec = {
        "metric": "s for the paper's iteration-count experiments (outer tolerance 1e-5); outer/inner counts vs the paper's tables",
        "value": round(total, 3), "unit": "s", "n_gpus": 1, "steps": 1, "warmup": 0,
        "ms_per_step": round(total * 1e3, 1), "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": "c128 (c64 stepping and inner basis above 2.5e7 nodes) + c128 Krylov sums and outer solve",
        "data": "synthetic: the paper's homogeneous and converging-lens models, recomputed from their definitions",
        "config": {"workload": "paper-tables", "entries": n, "skipped": skipped},
        "matches": {"outer_exact": exact, "outer_and_inner_within_1": near, "entries": n},
        "entries": out, "noshift_2d": noshift, "weak_scaling_op": weak,
    }
    print(json.dumps(rec), flush=True)


def bench_variants(args, torch, mxp, wl):
    """The four inner systems/solvers of Algorithm 1 (inner_solver 0-3: GMRES
    and the plain fixed-point iteration on the exp form, Theorem 2.1; the same
    two on the psi_2 form, Section 3.1 and Theorem 2.2) on the 2D homogeneous
    model with a dipole source, fprtol 0.01, outer tolerance 1e-5, complex
    double: with the shift 1/freq at freq 40, 80, 160, and unshifted at freq
    20 and 40 (inner iterations capped at 3000).  One step is the whole set;
    value is the summed solve time."""
    ctx = mxp.Context(0)
    out, total = [], 0.0
    cases = [(freq, None, (0, 1, 2, 3)) for freq in (40, 80, 160)] + [(freq, 0.0, (0, 1, 2, 3)) for freq in (20, 40)]
    for freq, shift, solvers in cases:
        prob = wl.homog_problem(2, freq)
        fd = torch.from_numpy(wl.dipole_source(prob).ravel()).to("cuda:0")
        for solver in solvers:
            P = mxp.Problem(ctx, prob)
            o = P.default_opts()
            o.rtol = 1e-5
            o.fprtol = 0.01
            o.inner_solver = solver
            o.max_inner = 3000
            if shift is not None:
                o.shift = shift
            u = torch.zeros_like(fd)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st = mxp.mxp_solve(P, o, fd, u)
            torch.cuda.synchronize()
            sec = time.perf_counter() - t0
            total += sec
            inner, _ = mxp.mxp_solve_history(P)
            e = {"freq": freq, "shift": "1/freq" if shift is None else shift, "inner_solver": solver,
                 "status": st["status"], "outer": st["outer_its"], "inner_mean": round(st["inner_mean"], 2),
                 "inner": inner, "actions": st["fn_actions"], "relres": st["true_relres"], "seconds": round(sec, 3)}
            out.append(e)
            print(f"[bench] variants freq {freq} shift {e['shift']} solver {solver}: outer {e['outer']} "
                  f"inner {inner} actions {e['actions']} {sec:.2f} s", file=sys.stderr, flush=True)
            P.close()
    rec = {
        "metric": "s for the inner-solver variants (outer tolerance 1e-5); iteration counts per variant",
        "value": round(total, 3), "unit": "s", "n_gpus": 1, "steps": 1, "warmup": 0,
        "ms_per_step": round(total * 1e3, 1), "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": "c128", "data": "synthetic: the paper's 2D homogeneous model, dipole source",
        "config": {"workload": "variants"}, "entries": out,
    }
    print(json.dumps(rec), flush=True)


def bench_matfun_krylov(args, torch, mxp, wl):
    """One exp(i t A_s) action by the Chebyshev schedule (complex double and
    complex float) and by the Arnoldi route (complex double, tolerances 1e-6
    and 1e-10, at most 250 vectors per basis, restarted by time stepping
    beyond that) on the 128^2 homogeneous and 2048^2 GRF
    workloads, each timed warm; value is the Arnoldi/Chebyshev time ratio at
    2048^2 and 1e-6."""
    ctx = mxp.Context(0)
    out = []
    for prob in (wl.config1(), wl.config2()):
        P = mxp.Problem(ctx, prob)
        t, s = prob.default_t(), prob.default_shift()
        x = torch.from_numpy(wl.random_vector(prob.npts, 5)).to("cuda:0")
        e = {"workload": prob.name, "grid": list(prob.n)}
        ref = torch.empty_like(x)
        for name, dt in (("chebyshev_c128_ms", torch.complex128), ("chebyshev_c64_ms", torch.complex64)):
            xx = x.to(dt)
            yy = torch.empty_like(xx)
            mxp.mxp_apply_exp(P, t, s, xx, yy)  # warm (tile tuning)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            mxp.mxp_apply_exp(P, t, s, xx, yy)
            torch.cuda.synchronize()
            e[name] = round(1e3 * (time.perf_counter() - t0), 3)
            if dt == torch.complex128:
                ref.copy_(yy)
        sch = mxp.mxp_design_schedule(P.desc, t, s, mxp.MXP_PREC_FP64)
        e["chebyshev_c128_levels"] = sch.S * sch.m
        y = torch.empty_like(x)
        mxp.mxp_apply_fn_krylov(P, False, t, s, 1e-6, 250, x, y)  # warm (basis allocation)
        for tol in (1e-6, 1e-10):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st, dim = mxp.mxp_apply_fn_krylov(P, False, t, s, tol, 250, x, y)
            torch.cuda.synchronize()
            sec = time.perf_counter() - t0
            e[f"arnoldi_{tol:g}"] = {"status": st, "vectors": dim, "ms": round(1e3 * sec, 1),
                                     "rel_diff_to_chebyshev_c128": ((y - ref).norm() / ref.norm()).item()}
        print(f"[bench] matfun-krylov {e}", file=sys.stderr, flush=True)
        out.append(e)
        P.close()
        del x, y, ref
        torch.cuda.empty_cache()
    big = out[-1]
    rec = {
        "metric": "Arnoldi / Chebyshev time for one exp(i t A_s) action (2048^2, tol 1e-6)",
        "value": round(big["arnoldi_1e-06"]["ms"] / big["chebyshev_c128_ms"], 1), "unit": "x",
        "n_gpus": 1, "steps": 1, "warmup": 1, "ms_per_step": big["arnoldi_1e-06"]["ms"],
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "c128",
        "data": "synthetic (seeded random input vector)", "config": {"workload": "matfun-krylov"}, "entries": out,
    }
    print(json.dumps(rec), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="3d-homog-256",
                    choices=["2d-grf-2048", "2d-homog-128", "3d-homog-256", "3d-layered-batch", "3d-learned",
                             "paper-tables", "variants", "matfun-krylov"])
    ap.add_argument("--train-models", type=int, default=6, help="3d-learned: 128^3 training models")
    ap.add_argument("--train-steps", type=int, default=1500, help="3d-learned: Adam steps")
    ap.add_argument("--eval-restart", type=int, default=60, help="3d-learned: FGMRES restart of the evaluation")
    ap.add_argument("--eval-grid", type=int, default=256, help="3d-learned: nodes per axis of the evaluation model")
    ap.add_argument("--conv-only", action="store_true",
                    help="3d-learned: time the network alone (forward at 256^3, training steps on 4 x 64^3)")
    ap.add_argument("--rhs", type=int, default=2,
                    help="3d-layered-batch: surface sources on the 512x512x256 grid (of 32), equally spaced")
    ap.add_argument("--sources", default=None,
                    help="3d-layered-batch: explicit source indices (of the 32), e.g. 0-10 or 3,7,12 "
                         "(overrides --rhs)")
    ap.add_argument("--no-extras", action="store_true",
                    help="3d-layered-batch: leave out the 16 uneven grids")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-form solves beside the double ones")
    ap.add_argument("--fp64-below", type=float, default=None,
                    help="mixed form: relative residual below which its actions run in double "
                         "(default: the library's default options)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--roofline-reps", type=int, default=3)
    ap.add_argument("--graphs", action="store_true", help="replay matrix-function actions from HIP graphs")
    ap.add_argument("--tiles", default=None,
                    help="K,NX,Ly of the fused 2D passes for both precisions, or K,NX,Ly/K,NX,Ly for "
                         "complex double / complex float (default: autotuned)")
    ap.add_argument("--roofline-only", action="store_true",
                    help="skip the solves: run only the exp-action timing loop and a plain "
                         "1 GiB device copy (counter calibration); for profiler runs")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU (asked for {args.gpus}): the solver has no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)
    if args.workload == "3d-layered-batch":
        layered_sources(args)  # argument errors before any device work

    import torch
    import paper_2506_03617_amd as mxp
    import workloads as wl

    if args.workload == "3d-layered-batch":
        bench_layered_batch(args, torch, mxp, wl)
        return
    if args.workload == "3d-learned":
        bench_learned(args, torch, mxp, wl)
        return
    if args.workload == "paper-tables":
        bench_paper_tables(args, torch, mxp, wl)
        return
    if args.workload == "variants":
        bench_variants(args, torch, mxp, wl)
        return
    if args.workload == "matfun-krylov":
        bench_matfun_krylov(args, torch, mxp, wl)
        return
    prob = {"2d-grf-2048": wl.config2, "2d-homog-128": wl.config1, "3d-homog-256": wl.config3}[args.workload]()
    centre = tuple(m // 2 for m in prob.n)
    if prob.dim == 3:
        # Gaussian-smoothed point source, standard deviation 2 cells
        f = wl.gaussian_source(prob, tuple(c * prob.h for c in centre), 2 * prob.h)
    else:
        f = wl.delta_source(prob, centre)
    ctx = mxp.Context(0)
    P = mxp.Problem(ctx, prob)
    fd = torch.from_numpy(f.ravel()).to("cuda:0")
    u64 = torch.zeros_like(fd)
    u32 = torch.zeros_like(fd)
    o64 = P.default_opts()
    o64.use_graphs = 1 if args.graphs else 0
    if prob.dim == 3:
        o64.outer_restart = 20   # FGMRES(20) for the 3D workloads
    o_mixed = P.default_opts()
    o_mixed.outer_restart = o64.outer_restart
    o_mixed.use_graphs = o64.use_graphs
    o_mixed.precision = mxp.MXP_PREC_MIXED
    if args.fp64_below is not None:
        o_mixed.fp64_below = args.fp64_below
    if args.tiles:
        parts = args.tiles.split("/")
        if len(parts) == 1:
            parts = parts * 2
        for prec, part in zip((mxp.MXP_PREC_FP64, mxp.MXP_PREC_MIXED), parts):
            K_, NX_, Ly_ = (int(v) for v in part.split(","))
            mxp.mxp_set_tiles(P, prec, K_, NX_, Ly_)
    print(f"[bench] {prob.name}: n={prob.n} omega={prob.omega:.2f} t={o64.t:.3e} "
          f"s={o64.shift:.4f}", file=sys.stderr, flush=True)

    if args.roofline_only:
        args.warmup = 0
        args.steps = 0
        args.no_cpu = True
        # plain copy of known size: its FETCH_SIZE / WRITE_SIZE calibrate the counters
        src = torch.ones(1 << 26, dtype=torch.complex128, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    def solve(o, u):
        u.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = mxp.mxp_solve(P, o, fd, u)
        torch.cuda.synchronize()
        return time.perf_counter() - t0, st

    # warm-up: both forms, so that tiles, schedules and workspaces of each are
    # set up before the timed steps
    for w in range(args.warmup):
        for label, o, u in (("fp64", o64, u64), ("mixed", o_mixed, u32)):
            sec, st = solve(o, u)
            print(f"[bench] warmup {w} {label}: {sec:.3f} s {st}", file=sys.stderr, flush=True)
    # timed steps: a double solve (the step) and, alternating with it, the mixed
    # form; each solve is bracketed by device synchronisation
    t64, t32, st64, st32 = [], [], None, None
    t_begin = time.perf_counter()
    for k in range(args.steps):
        sec, st64 = solve(o64, u64)
        t64.append(sec)
        print(f"[bench] step {k} fp64: {sec:.3f} s {st64}", file=sys.stderr, flush=True)
        if not args.no_mixed:
            sec, st32 = solve(o_mixed, u32)
            t32.append(sec)
            print(f"[bench] step {k} mixed: {sec:.3f} s {st32}", file=sys.stderr, flush=True)
    wall = time.perf_counter() - t_begin
    s_per_solve = sum(t64) / max(len(t64), 1)
    keys = ("outer_its", "inner_mean", "inner_std", "stencil_steps", "fn_actions", "true_relres")
    forms = {}
    if t64:
        forms["fp64"] = {"seconds_mean": round(s_per_solve, 4), "seconds_median": round(float(np.median(t64)), 4),
                         **{k: st64[k] for k in keys}}
    if t32:
        m32 = sum(t32) / len(t32)
        err = ((u32 - u64).norm() / u64.norm()).item()
        forms["mixed"] = {"seconds_mean": round(m32, 4), "seconds_median": round(float(np.median(t32)), 4),
                          "speedup_vs_fp64": round(s_per_solve / m32, 3), "rel_err_vs_fp64": err,
                          "outer_its_minus_fp64": st32["outer_its"] - st64["outer_its"],
                          "fp64_below": o_mixed.fp64_below, "fp64_its": st32["fp64_its"],
                          **{k: st32[k] for k in keys}}
    forms["learned"] = None  # the layered workloads only: `--workload 3d-learned`

    roofline = measure_roofline(mxp, torch, P, prob, o64, args.roofline_reps, mxp.MXP_PREC_FP64)
    roofline_c64 = measure_roofline(mxp, torch, P, prob, o_mixed, args.roofline_reps, mxp.MXP_PREC_MIXED)

    cpu = None
    if not args.no_cpu and st64 is not None:
        cpu = cpu_baseline(prob, f, int(st64["fn_actions"]))
        print(f"[bench] cpu baseline: {cpu}", file=sys.stderr, flush=True)

    line = {
        "metric": "s to 1e-6 rel. residual (plain vs FP32/learned); stencil HBM GB/s vs peak",
        "value": round(s_per_solve, 4),
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(s_per_solve * 1e3, 2),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c128",
        "data": "synthetic (seeded GRF speed, point source)" if prob.c is not None
                else "synthetic (constant speed, Gaussian-smoothed point source)" if prob.dim == 3
                else "synthetic (constant speed, point source)",
        "config": {"workload": prob.name, "grid": list(prob.n), "omega": round(prob.omega, 3),
                   "layer": prob.layer, "t": o64.t, "shift": o64.shift, "fprtol": o64.fprtol,
                   "rtol": o64.rtol, "outer_restart": o64.outer_restart,
                   "inner_restart": o64.inner_restart, "precision": "fp64 (value); mixed beside it",
                   "graphs": bool(args.graphs)},
        "forms": forms,
        "timed_wall_s": round(wall, 2),
        "roofline": roofline,
        "roofline_c64": roofline_c64,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    P.close()
    ctx.close()


if __name__ == "__main__":
    main()
