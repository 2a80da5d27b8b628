// C ABI of the MatExPre library: contexts, problems, the building blocks
// (stencil, matrix-function actions, Algorithm 1) and single solves.  The
// solvers live in krylov.cpp, the actions in action.cpp and batched solves
// in batch.cpp.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdlib>
#include <cstring>

#include "engine.h"

namespace mxp {

thread_local std::string g_last_error;
thread_local const Allocator* t_alloc = nullptr;
thread_local bool t_reserved = false;

template <typename R>
static void upload_tables(mxp_problem* P, DevMem& mem, DevTables<R>& t) {
    const GridInfo& g = P->g;
    size_t total = 0;
    for (int d = 0; d < 3; ++d) total += size_t(g.n[d]) * 3;
    std::vector<cpx<R>> host(total);
    size_t off = 0;
    size_t offs[3][3];
    for (int d = 0; d < 3; ++d) {
        AxisTables at;
        if (d < g.dim) {
            at = build_axis_tables(g.axis(d));
        } else {  // unused third axis in 2D: a single node with zero coefficients
            at.alpha.assign(g.n[d], cd(0, 0));
            at.beta.assign(g.n[d], cd(0, 0));
            at.gamma.assign(g.n[d], cd(0, 0));
        }
        const std::vector<cd>* src[3] = {&at.alpha, &at.beta, &at.gamma};
        for (int q = 0; q < 3; ++q) {
            offs[d][q] = off;
            for (int64_t i = 0; i < g.n[d]; ++i)
                host[off + i] = {R((*src[q])[i].real()), R((*src[q])[i].imag())};
            off += g.n[d];
        }
    }
    mem.ensure(total * sizeof(cpx<R>));
    HIP_CHECK(hipMemcpyAsync(mem.p, host.data(), total * sizeof(cpx<R>), hipMemcpyHostToDevice,
                             P->ctx->stream));
    HIP_CHECK(hipStreamSynchronize(P->ctx->stream));
    cpx<R>* base = mem.as<cpx<R>>();
    for (int d = 0; d < 3; ++d) {
        t.alpha[d] = base + offs[d][0];
        t.beta[d] = base + offs[d][1];
        t.gamma[d] = base + offs[d][2];
    }
    if (!g.abc_per_node()) return;
    // absorbing faces with a varying speed: 2 omega/h at the absorbing end
    // nodes of each axis (the kernels multiply by sqrt(D_p)), and times h^2
    DevMem& am = sizeof(R) == 8 ? P->abc64 : P->abc32;
    const size_t na = size_t(g.n[0] + g.n[1] + g.n[2]);
    std::vector<R> ha(2 * na, R(0));
    size_t o = 0;
    for (int d = 0; d < 3; ++d) {
        if (d < g.dim) {
            const AxisLayer ax = g.axis(d);
            const double wgt = 2.0 * g.omega / g.h;
            if (ax.abs_lo) ha[o] += R(wgt);
            if (ax.abs_hi) ha[o + size_t(g.n[d]) - 1] += R(wgt);
            if (ax.abs_lo) ha[na + o] += R(wgt * g.h * g.h);
            if (ax.abs_hi) ha[na + o + size_t(g.n[d]) - 1] += R(wgt * g.h * g.h);
        }
        o += size_t(g.n[d]);
    }
    am.ensure(ha.size() * sizeof(R));
    HIP_CHECK(hipMemcpy(am.p, ha.data(), ha.size() * sizeof(R), hipMemcpyHostToDevice));
    o = 0;
    for (int d = 0; d < 3; ++d) {
        t.abc[d] = am.as<R>() + o;
        t.abc_h2[d] = am.as<R>() + na + o;
        o += size_t(g.n[d]);
    }
}

void context_info(const mxp_context* ctx, int* device, hipStream_t* stream) {
    *device = ctx->device;
    *stream = ctx->stream;
}

const Allocator& context_alloc(const mxp_context* ctx) { return ctx->alloc; }

}  // namespace mxp

using namespace mxp;

extern "C" {

const char* mxp_last_error(void) { return g_last_error.c_str(); }

// The version is part of the autotuner cache key, so it changes whenever the
// tuner's candidates or the kernels they name do (0.2: three-level 3D passes).
const char* mxp_version(void) { return "matexpre-mi355x 0.2.0 (gfx950)"; }

mxp_status mxp_context_create(int device, void* hip_stream, mxp_alloc_fn alloc, mxp_free_fn release, void* user,
                              mxp_context** out) {
    return guard([&]() {
        if (!out) fail(MXP_ERR_INVALID_ARG, "out is NULL");
        *out = nullptr;
        if ((alloc == nullptr) != (release == nullptr))
            fail(MXP_ERR_INVALID_ARG, "alloc and release hooks must be given together");
        int count = 0;
        const hipError_t ce = hipGetDeviceCount(&count);
        if (ce != hipSuccess || count <= 0) {
            (void)hipGetLastError();
            fail(MXP_ERR_INVALID_ARG, std::string("no HIP device available (") + hipGetErrorString(ce) +
                                          ", count " + std::to_string(count) + ")");
        }
        if (device < 0 || device >= count) fail(MXP_ERR_INVALID_ARG, "no such device");
        HIP_CHECK(hipSetDevice(device));
        const char* v = std::getenv("MXP_VERBOSE");
        auto* c = new mxp_context{device, static_cast<hipStream_t>(hip_stream), (v && *v && *v != '0') ? 1 : 0,
                                  Allocator{alloc, release, user, std::make_shared<AllocStats>()}};
        *out = c;
        return MXP_OK;
    });
}

void mxp_context_destroy(mxp_context* ctx) { delete ctx; }

mxp_status mxp_context_alloc_stats(const mxp_context* ctx, mxp_alloc_stats* out) {
    return guard([&]() {
        if (!ctx || !out) fail(MXP_ERR_INVALID_ARG, "context or out is NULL");
        const AllocStats& a = *ctx->alloc.stats;
        out->allocs = a.allocs.load();
        out->frees = a.frees.load();
        out->bytes_live = a.live.load();
        out->bytes_peak = a.peak.load();
        out->late = a.late.load();
        return MXP_OK;
    });
}

mxp_status mxp_problem_create(mxp_context* ctx, const mxp_grid_desc* desc, mxp_problem** out) {
    return guard([&]() {
        if (!ctx || !out) fail(MXP_ERR_INVALID_ARG, "context or out is NULL");
        *out = nullptr;
        GridInfo g = validate_grid(desc);
        use_device(ctx);
        AllocScope scope(ctx->alloc);
        auto P = std::make_unique<mxp_problem>();
        P->ctx_copy = *ctx;
        P->ctx = &P->ctx_copy;
        const int64_t n = g.npts();
        if (!g.homogeneous) {
            // Copy c to the host (it may live on either side) for validation
            // and its range, and build D = 1/c^2 on the device.
            const size_t esz = desc->c_dtype == MXP_F32 ? 4 : 8;
            std::vector<unsigned char> hostc(size_t(n) * esz);
            hipPointerAttribute_t attr;
            bool on_device = false;
            if (hipPointerGetAttributes(&attr, desc->c) == hipSuccess)
                on_device = (attr.type == hipMemoryTypeDevice);
            else
                (void)hipGetLastError();
            if (on_device)
                HIP_CHECK(hipMemcpy(hostc.data(), desc->c, hostc.size(), hipMemcpyDeviceToHost));
            else
                std::memcpy(hostc.data(), desc->c, hostc.size());
            speed_range_host(hostc.data(), desc->c_dtype, n, &g.dmin, &g.dmax);
            DevMem cdev;
            cdev.ensure(hostc.size());
            HIP_CHECK(hipMemcpy(cdev.p, hostc.data(), hostc.size(), hipMemcpyHostToDevice));
            P->D64.ensure(size_t(n) * 8);
            P->D32.ensure(size_t(n) * 4);
            launch_inv_c2(cdev.p, desc->c_dtype == MXP_F32, P->D64.as<double>(), P->D32.as<float>(), n,
                          P->ctx->stream);
            HIP_CHECK(hipStreamSynchronize(P->ctx->stream));
        }
        P->g = g;
        P->Dref = 0.5 * (g.dmin + g.dmax);
        upload_tables<double>(P.get(), P->tables64, P->t64);
        upload_tables<float>(P.get(), P->tables32, P->t32);
        *out = P.release();
        return MXP_OK;
    });
}

void mxp_problem_destroy(mxp_problem* prob) {
    if (!prob) return;
    (void)hipSetDevice(prob->ctx->device);
    (void)hipStreamSynchronize(prob->ctx->stream);
    delete prob;
}

mxp_status mxp_solve_history(const mxp_problem* prob, int32_t cap, int32_t* inner_its, double* relres,
                             int32_t* count) {
    return guard([&]() {
        if (!prob || !count) fail(MXP_ERR_INVALID_ARG, "problem or count is NULL");
        if (cap < 0 || (cap > 0 && (!inner_its || !relres))) fail(MXP_ERR_INVALID_ARG, "history buffers");
        const int32_t n = int32_t(prob->hist_inner.size());
        *count = n;
        for (int32_t k = 0; k < n && k < cap; ++k) {
            inner_its[k] = prob->hist_inner[size_t(k)];
            relres[k] = prob->hist_res[size_t(k)];
        }
        return MXP_OK;
    });
}

int64_t mxp_problem_size(const mxp_problem* prob) { return prob ? prob->g.npts() : 0; }

mxp_status mxp_solve_opts_default(const mxp_grid_desc* desc, mxp_solve_opts* out) {
    return guard([&]() {
        if (!out) fail(MXP_ERR_INVALID_ARG, "out is NULL");
        GridInfo g = validate_grid(desc);
        std::memset(out, 0, sizeof(*out));
        const double freq = g.omega / (2.0 * M_PI);
        out->t = 40.0 * g.h * g.h;
        out->shift = 1.0 / freq;
        out->fprtol = 0.08;
        out->rtol = 1e-6;
        out->outer_restart = 30;
        out->inner_restart = 30;
        out->max_outer = 500;
        out->max_inner = 300;
        out->precision = MXP_PREC_FP64;
        out->use_learned = 0;
        out->stall_ratio = 0.0;
        out->use_graphs = 0;
        out->inner_solver = 0;
        out->fp64_below = 0.0;
        out->fp64_first = 2;
        return MXP_OK;
    });
}

mxp_status mxp_design_schedule(const mxp_grid_desc* desc, double t, double shift, mxp_precision precision,
                               mxp_schedule* out) {
    return guard([&]() {
        if (!out) fail(MXP_ERR_INVALID_ARG, "out is NULL");
        if (precision != MXP_PREC_FP64 && precision != MXP_PREC_MIXED)
            fail(MXP_ERR_INVALID_ARG, "unknown precision");
        GridInfo g = validate_grid(desc);
        if (!g.homogeneous)
            speed_range_host(desc->c, desc->c_dtype, g.npts(), &g.dmin, &g.dmax);
        design_schedule(g, t, shift, precision, out);
        return MXP_OK;
    });
}

mxp_status mxp_apply_A(mxp_problem* prob, double shift, mxp_dtype dtype, const void* x, void* y) {
    return guard([&]() {
        check_problem(prob);
        AllocScope scope(prob->ctx->alloc);
        if (!x || !y || x == y) fail(MXP_ERR_INVALID_ARG, "x and y must be distinct non-NULL pointers");
        if (!(shift >= 0) || !std::isfinite(shift)) fail(MXP_ERR_INVALID_ARG, "shift must be >= 0");
        apply_A(prob, prob->ctx->stream, shift, dtype, x, y);
        HIP_CHECK(hipStreamSynchronize(prob->ctx->stream));
        return MXP_OK;
    });
}

static mxp_status apply_fn(mxp_problem* prob, double t, double shift, mxp_dtype dtype, const void* x,
                           void* y, int fn) {
    return guard([&]() {
        check_problem(prob);
        AllocScope scope(prob->ctx->alloc);
        if (!x || !y || x == y) fail(MXP_ERR_INVALID_ARG, "x and y must be distinct non-NULL pointers");
        int64_t steps = 0;
        if (dtype != MXP_C128 && dtype != MXP_C64) fail(MXP_ERR_INVALID_ARG, "dtype must be MXP_C64 or MXP_C128");
        const Sched& sc = get_sched(prob, t, shift, dtype == MXP_C128 ? MXP_PREC_FP64 : MXP_PREC_MIXED, 0, 0);
        reserve_action(prob, prob->ws, sc, fn == ACT_PSI2, false, prob->ctx->stream);
        t_reserved = true;
        apply_action(prob, prob->ws, prob->ctx->stream, sc, t, shift, fn, dtype, x, y, &steps);
        HIP_CHECK(hipStreamSynchronize(prob->ctx->stream));
        return MXP_OK;
    });
}

mxp_status mxp_apply_exp(mxp_problem* prob, double t, double shift, mxp_dtype dtype, const void* x,
                         void* y) {
    return apply_fn(prob, t, shift, dtype, x, y, ACT_EXP);
}

mxp_status mxp_apply_psi1(mxp_problem* prob, double t, double shift, mxp_dtype dtype, const void* x,
                          void* y) {
    return apply_fn(prob, t, shift, dtype, x, y, ACT_PSI1);
}

mxp_status mxp_apply_psi2(mxp_problem* prob, double t, double shift, mxp_dtype dtype, const void* x,
                          void* y) {
    return apply_fn(prob, t, shift, dtype, x, y, ACT_PSI2);
}

mxp_status mxp_apply_fn_krylov(mxp_problem* prob, int32_t psi, double t, double shift, double tol,
                               int32_t max_dim, const void* x, void* y, int32_t* dim) {
    return guard([&]() {
        check_problem(prob);
        AllocScope scope(prob->ctx->alloc);
        if (!x || !y || x == y) fail(MXP_ERR_INVALID_ARG, "x and y must be distinct non-NULL pointers");
        if (psi != 0 && psi != 1) fail(MXP_ERR_INVALID_ARG, "psi must be 0 (exp) or 1 (psi_1)");
        if (!(t > 0) || !std::isfinite(t)) fail(MXP_ERR_INVALID_ARG, "t must be positive and finite");
        if (!(shift >= 0) || !std::isfinite(shift)) fail(MXP_ERR_INVALID_ARG, "shift must be >= 0");
        if (!(tol > 0) || !(tol < 1)) fail(MXP_ERR_INVALID_ARG, "tol must be in (0, 1)");
        if (max_dim < 1 || max_dim > 250) fail(MXP_ERR_INVALID_ARG, "max_dim must be in 1..250");
        Run run{prob, &prob->ws, prob->ctx->stream, nullptr, nullptr};
        bool ok = false;
        const int m = krylov_action(run, psi != 0, t, shift, tol, max_dim, static_cast<const cpx<double>*>(x),
                                    static_cast<cpx<double>*>(y), &ok);
        HIP_CHECK(hipStreamSynchronize(prob->ctx->stream));
        if (dim) *dim = m;
        if (!ok) g_last_error = "Krylov basis reached max_dim before the estimate met tol";
        return ok ? MXP_OK : MXP_NOT_CONVERGED;
    });
}

mxp_status mxp_apply_precond(mxp_problem* prob, const mxp_solve_opts* opts, mxp_dtype dtype, const void* r, void* w,
                             int32_t* inner_its) {
    return guard([&]() {
        check_problem(prob);
        AllocScope scope(prob->ctx->alloc);
        check_opts(opts);
        if (!r || !w || r == w) fail(MXP_ERR_INVALID_ARG, "r and w must be distinct non-NULL pointers");
        if (dtype != MXP_C128 && dtype != MXP_C64) fail(MXP_ERR_INVALID_ARG, "dtype must be MXP_C64 or MXP_C128");
        Counters cnt;
        Run run{prob, &prob->ws, prob->ctx->stream, nullptr, nullptr};
        run.graphs = opts->use_graphs != 0;
        const int64_t n = npts(prob);
        hipStream_t s = prob->ctx->stream;
        const cpx<double>* r64 = static_cast<const cpx<double>*>(r);
        cpx<double>* w64 = static_cast<cpx<double>*>(w);
        if (dtype == MXP_C64) {  // complex-double copies of the complex-float arguments
            prob->ws.io[0].ensure(size_t(n) * sizeof(cpx<double>));
            prob->ws.io[1].ensure(size_t(n) * sizeof(cpx<double>));
            r64 = prob->ws.io[0].as<cpx<double>>();
            w64 = prob->ws.io[1].as<cpx<double>>();
        }
        reserve_precond(run, *opts);
        t_reserved = true;
        if (dtype == MXP_C64) launch_to_c128(static_cast<const cpx<float>*>(r), prob->ws.io[0].as<cpx<double>>(), n, s);
        const int its = precond(run, *opts, r64, w64, cnt, opts->precision);
        if (dtype == MXP_C64) launch_to_c64(w64, static_cast<cpx<float>*>(w), n, s);
        HIP_CHECK(hipStreamSynchronize(s));
        if (inner_its) *inner_its = its;
        return MXP_OK;
    });
}

mxp_status mxp_set_tiles(mxp_problem* prob, mxp_precision precision, int32_t K, int32_t NX, int32_t Ly) {
    return guard([&]() {
        if (!prob) fail(MXP_ERR_INVALID_ARG, "problem is NULL");
        if (precision != MXP_PREC_FP64 && precision != MXP_PREC_MIXED) fail(MXP_ERR_INVALID_ARG, "unknown precision");
        // 3D sweeps and two-level passes also take Ly = 0 (automatic z-chunk)
        const bool auto_chunk = prob->g.dim == 3 && (K >= 1 && K <= 3) && Ly == 0;
        if (K < 0 || K > kMaxFused || (NX != 1 && NX != 2) || (Ly < 1 && !auto_chunk) ||
            (K > 0 && NX * 64 - 2 * K <= 0))
            fail(MXP_ERR_INVALID_ARG, "tiles: K in 0..8, NX in {1, 2}, Ly >= 1 (Ly = 0 for 3D K = 1, 2)");
        if ((K == 2 || K == 3) && prob->g.dim == 3 && prob->g.abc_per_node())
            fail(MXP_ERR_UNSUPPORTED, "multi-level 3D passes do not carry the absorbing-face term");
        TileCfg& t = prob->tiles[precision == MXP_PREC_MIXED ? 1 : 0];
        (void)hipStreamSynchronize(prob->ctx->stream);
        prob->ws.drop_graphs();  // captured actions bake in the tile shape
        t.K = K;
        t.NX = NX;
        t.Ly = Ly;
        t.us_per_level = 0.0;
        return MXP_OK;
    });
}

mxp_status mxp_get_tiles(const mxp_problem* prob, mxp_precision precision, int32_t* K, int32_t* NX,
                         int32_t* Ly, double* us_per_level) {
    return guard([&]() {
        if (!prob) fail(MXP_ERR_INVALID_ARG, "problem is NULL");
        if (precision != MXP_PREC_FP64 && precision != MXP_PREC_MIXED) fail(MXP_ERR_INVALID_ARG, "unknown precision");
        const TileCfg& t = prob->tiles[precision == MXP_PREC_MIXED ? 1 : 0];
        if (K) *K = t.K;
        if (NX) *NX = t.NX;
        if (Ly) *Ly = t.Ly;
        if (us_per_level) *us_per_level = t.us_per_level;
        return MXP_OK;
    });
}

mxp_status mxp_solve(mxp_problem* prob, const mxp_solve_opts* opts, mxp_dtype dtype, const void* f, void* u,
                     mxp_solve_stats* stats) {
    return guard([&]() -> mxp_status {
        check_problem(prob);
        AllocScope scope(prob->ctx->alloc);
        check_opts(opts);
        if (!f || !u || f == u) fail(MXP_ERR_INVALID_ARG, "f and u must be distinct non-NULL pointers");
        if (dtype != MXP_C128 && dtype != MXP_C64) fail(MXP_ERR_INVALID_ARG, "dtype must be MXP_C64 or MXP_C128");
        Run run{prob, &prob->ws, prob->ctx->stream, nullptr, nullptr};
        if (dtype == MXP_C128)
            return solve(run, *opts, static_cast<const cpx<double>*>(f), static_cast<cpx<double>*>(u), stats);
        // complex-float data: the solve runs on complex-double copies
        const int64_t n = npts(prob);
        hipStream_t s = prob->ctx->stream;
        prob->ws.io[0].ensure(size_t(n) * sizeof(cpx<double>));
        prob->ws.io[1].ensure(size_t(n) * sizeof(cpx<double>));
        cpx<double>* f64 = prob->ws.io[0].as<cpx<double>>();
        cpx<double>* u64 = prob->ws.io[1].as<cpx<double>>();
        launch_to_c128(static_cast<const cpx<float>*>(f), f64, n, s);
        launch_to_c128(static_cast<const cpx<float>*>(u), u64, n, s);
        const mxp_status st = solve(run, *opts, f64, u64, stats);
        launch_to_c64(u64, static_cast<cpx<float>*>(u), n, s);
        HIP_CHECK(hipStreamSynchronize(s));
        return st;
    });
}

mxp_status mxp_problem_set_learned(mxp_problem* prob, mxp_cnn* net, double out_scale) {
    return guard([&]() {
        check_problem(prob);
        AllocScope scope(prob->ctx->alloc);
        if (net && !(out_scale > 0 && std::isfinite(out_scale)))
            fail(MXP_ERR_INVALID_ARG, "out_scale must be positive");
        prob->net = net;
        prob->net_scale = net ? out_scale : 1.0;
        return MXP_OK;
    });
}

mxp_status mxp_collect_pairs(mxp_problem* prob, const mxp_solve_opts* opts, const void* f, void* u,
                             int32_t max_pairs, void* r_out, void* z_out, double* rnorm, double* znorm,
                             int32_t* npairs, mxp_solve_stats* stats) {
    return guard([&]() {
        check_problem(prob);
        AllocScope scope(prob->ctx->alloc);
        check_opts(opts);
        if (!f || !u || f == u) fail(MXP_ERR_INVALID_ARG, "f and u must be distinct non-NULL pointers");
        if (max_pairs < 0 || (max_pairs > 0 && (!r_out || !z_out || !rnorm || !znorm)))
            fail(MXP_ERR_INVALID_ARG, "pair buffers must be given for max_pairs > 0");
        if (opts->use_learned) fail(MXP_ERR_INVALID_ARG, "pairs come from the MatExPre preconditioner alone");
        PairSink ps{static_cast<cpx<double>*>(r_out), static_cast<cpx<double>*>(z_out), rnorm, znorm, max_pairs, 0};
        Run run{prob, &prob->ws, prob->ctx->stream, nullptr, nullptr, &ps};
        const mxp_status st = solve(run, *opts, static_cast<const cpx<double>*>(f), static_cast<cpx<double>*>(u), stats);
        if (npairs) *npairs = ps.count;
        return st;
    });
}

mxp_status mxp_cnn_make_sample(mxp_problem* prob, const void* r, const void* z, const int32_t offset[3],
                               const int32_t crop[3], double rscale, double zscale, void* in, float* target) {
    return guard([&]() {
        check_problem(prob);
        AllocScope scope(prob->ctx->alloc);
        if (!r || !z || !offset || !crop || !in || !target) fail(MXP_ERR_INVALID_ARG, "NULL argument");
        for (int d = 0; d < 3; ++d)
            if (crop[d] < 1 || offset[d] < 0 || offset[d] + crop[d] > prob->g.n[d])
                fail(MXP_ERR_INVALID_ARG, "crop outside the grid");
        const float* D = prob->g.homogeneous ? nullptr : prob->D32.as<float>();
        launch_cnn_crop(r, z, D, float(prob->Dref), prob->g.n[0], prob->g.n[1], offset[0], offset[1], offset[2],
                        crop[0], crop[1], crop[2], rscale, zscale, static_cast<uint16_t*>(in), target,
                        prob->ctx->stream);
        HIP_CHECK(hipStreamSynchronize(prob->ctx->stream));
        return MXP_OK;
    });
}

}  // extern "C"

