// Algorithm 1 of the paper (Section 3.4, eq. fixed-point): psi_1(i t A_s) r,
// then GMRES on (I - exp(i t A_s)) w = psi_1(i t A_s) r to relative tolerance
// fprtol; its variants (the plain fixed-point iteration of Section 2.1,
// Theorem 2.1, and the second inverse formula of Section 3.1 with the
// time-averaged map of Theorem 2.2); the outer flexible GMRES (Section 3.4,
// constant -i t dropped; restart 30 in Section 4 introduction); and the
// matrix functions by the Arnoldi method (the paper's own route, Section 4
// introduction).  Orthogonalisation is classical Gram--Schmidt with one
// re-orthogonalisation (CGS2: two fused multi-dot / multi-update passes); the
// small least-squares problems use Givens rotations on the host in double.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>

#include "engine.h"

namespace mxp {

// ------------------------------------------------------------ Krylov helpers

struct Small {
    cpx<double>* partial;
    cpx<double>* h1;
    cpx<double>* h2;
    cpx<double>* nrm;
    cpx<double>* y;
};

static Small small_buffers(Run& run) {
    const int64_t n = npts(run.P);
    const int nb = reduce_blocks(n);
    Workspace& W = *run.W;
    W.partial.ensure(size_t(nb) * 256 * sizeof(cpx<double>));
    W.small.ensure(size_t(1024) * sizeof(cpx<double>));
    W.host_small.resize(1024);
    cpx<double>* sm = W.small.as<cpx<double>>();
    return Small{W.partial.as<cpx<double>>(), sm, sm + 256, sm + 512, sm + 768};
}

static double norm2(Run& run, const cpx<double>* v) {
    Small sm = small_buffers(run);
    launch_nrm2sq(v, npts(run.P), sm.partial, sm.nrm, run.s);
    cpx<double> hv;
    HIP_CHECK(hipMemcpyAsync(&hv, sm.nrm, sizeof(hv), hipMemcpyDeviceToHost, run.s));
    HIP_CHECK(hipStreamSynchronize(run.s));
    if (!std::isfinite(hv.re)) fail(MXP_ERR_NONFINITE, "non-finite vector norm");
    return std::sqrt(hv.re);
}

// CGS2: orthogonalise w against V_0..V_{nv-1}; h receives the projection
// coefficients and the returned value is ||w|| afterwards.
template <typename TV>
static double cgs2(Run& run, const TV* V, int64_t ld, int nv, cpx<double>* w, std::vector<cd>& h) {
    const int64_t n = npts(run.P);
    hipStream_t s = run.s;
    Small sm = small_buffers(run);
    Workspace& W = *run.W;
    launch_mdot(V, ld, nv, w, n, sm.partial, sm.h1, s);
    launch_mupdate(w, V, ld, nv, sm.h1, n, s);
    launch_mdot(V, ld, nv, w, n, sm.partial, sm.h2, s);
    launch_mupdate(w, V, ld, nv, sm.h2, n, s);
    launch_nrm2sq(w, n, sm.partial, sm.nrm, s);
    HIP_CHECK(hipMemcpyAsync(W.host_small.data(), W.small.p, 513 * sizeof(cpx<double>),
                             hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipStreamSynchronize(s));
    h.resize(nv);
    for (int i = 0; i < nv; ++i)
        h[i] = cd(W.host_small[i].re + W.host_small[256 + i].re,
                  W.host_small[i].im + W.host_small[256 + i].im);
    const double nn = W.host_small[512].re;
    if (!std::isfinite(nn)) fail(MXP_ERR_NONFINITE, "non-finite value in the Arnoldi process");
    return std::sqrt(nn);
}

// Incremental QR of the Hessenberg matrix by Givens rotations.
struct Givens {
    int m;
    std::vector<cd> H;  // column-major (m+1) x m, rotated in place to R
    std::vector<double> c;
    std::vector<cd> s, g;
    explicit Givens(int m_) : m(m_), H(size_t(m_ + 1) * m_), c(m_), s(m_), g(m_ + 1) {}
    void reset(double beta) {
        std::fill(H.begin(), H.end(), cd(0));
        std::fill(g.begin(), g.end(), cd(0));
        g[0] = beta;
    }
    cd& at(int i, int j) { return H[size_t(j) * (m + 1) + i]; }
    // column j: h[0..j] and subdiagonal beta; returns |g_{j+1}|
    double add_column(int j, const std::vector<cd>& h, double beta) {
        for (int i = 0; i <= j; ++i) at(i, j) = h[i];
        at(j + 1, j) = beta;
        for (int i = 0; i < j; ++i) {
            const cd a = at(i, j), b = at(i + 1, j);
            at(i, j) = c[i] * a + s[i] * b;
            at(i + 1, j) = -std::conj(s[i]) * a + c[i] * b;
        }
        const cd a = at(j, j);
        const double b = std::abs(at(j + 1, j));
        if (b == 0.0) {
            c[j] = 1.0;
            s[j] = 0.0;
        } else if (std::abs(a) == 0.0) {
            c[j] = 0.0;
            s[j] = 1.0;
            at(j, j) = b;
        } else {
            const double r = std::hypot(std::abs(a), b);
            const cd ph = a / std::abs(a);
            c[j] = std::abs(a) / r;
            s[j] = ph * b / r;
            at(j, j) = ph * r;
        }
        at(j + 1, j) = 0.0;
        g[j + 1] = -std::conj(s[j]) * g[j];
        g[j] = c[j] * g[j];
        return std::abs(g[j + 1]);
    }
    std::vector<cd> solve(int k) {
        std::vector<cd> y(k);
        for (int i = k - 1; i >= 0; --i) {
            cd acc = g[i];
            for (int q = i + 1; q < k; ++q) acc -= at(i, q) * y[q];
            if (std::abs(at(i, i)) == 0.0)
                fail(MXP_ERR_BREAKDOWN, "singular Hessenberg factor (the preconditioner returned zero)");
            y[i] = acc / at(i, i);
        }
        return y;
    }
};

static void upload_coeffs(Run& run, const std::vector<cd>& y) {
    Small sm = small_buffers(run);
    std::vector<cpx<double>> tmp(y.size());
    for (size_t i = 0; i < y.size(); ++i) tmp[i] = {y[i].real(), y[i].imag()};
    HIP_CHECK(hipMemcpyAsync(sm.y, tmp.data(), tmp.size() * sizeof(cpx<double>), hipMemcpyHostToDevice, run.s));
    HIP_CHECK(hipStreamSynchronize(run.s));
}

// Work one network try counts for, in stencil steps of the working precision:
// the inference measured 4.5 ms at 256^3 against 0.11 ms per complex-float
// sweep (40 steps), plus A z_j and its Gram-Schmidt pass.  Both scale with the
// grid, so the ratio holds at other sizes.
constexpr double kNetTrySteps = 48.0;

// z = learned network applied to v (unit norm), complex double.
static void learned_apply(Run& run, const cpx<double>* v, double vnorm, cpx<double>* z) {
    Range range("network inference");
    mxp_problem* P = run.P;
    const int64_t n = npts(P);
    const ConvShape sh{1, int(P->g.n[2]), int(P->g.n[1]), int(P->g.n[0])};
    // the network sees the residual at unit root-mean-square value
    const double rs = std::sqrt(double(n)) / vnorm;
    const float* D = P->g.homogeneous ? nullptr : P->D32.as<float>();
    cnn_apply(P->net, sh, v, D, float(P->Dref), rs, P->net_scale / rs, z, run.s);
}

// Algorithm 1.  r, w: complex double device vectors.
int precond(Run& run, const mxp_solve_opts& o, const cpx<double>* r, cpx<double>* w, Counters& cnt,
            mxp_precision ap) {
    Range range("preconditioner apply");
    mxp_problem* P = run.P;
    run.graphs = o.use_graphs != 0 && !run.batch;
    Workspace& WS = *run.W;
    const int64_t n = npts(P);
    hipStream_t s = run.s;
    // ap: precision of the matrix-function actions (the inner basis follows
    // o.precision: complex double only in the FP64 form)
    const Sched& sc = get_sched(P, o.t, o.shift, ap, o.cheb_S, o.cheb_m);
    const int m = o.inner_restart;
    // complex-double basis: GMRES in the FP64 form; otherwise one direction vector
    const bool basis64 = o.precision == MXP_PREC_FP64 && (o.inner_solver == 0 || o.inner_solver == 2);
    WS.innerV.ensure(size_t(basis64 ? m + 1 : 1) * n * sizeof(cpx<double>));
    WS.innerRh.ensure(size_t(n) * sizeof(cpx<double>));
    WS.innerTmp.ensure(size_t(n) * sizeof(cpx<double>));
    WS.innerRr.ensure(size_t(n) * sizeof(cpx<double>));
    cpx<double>* V = WS.innerV.as<cpx<double>>();
    cpx<double>* rhat = WS.innerRh.as<cpx<double>>();
    cpx<double>* tmp = WS.innerTmp.as<cpx<double>>();
    cpx<double>* rr = WS.innerRr.as<cpx<double>>();
    const cpx<double> one{1.0, 0.0}, mone{-1.0, 0.0};

    // The exp form (inner_solver 0, 1) solves (I - exp(i t A_s)) w = psi_1(i t A_s) r;
    // the psi_2 form (2, 3) solves (I - psi_1(i t A_s)) w = psi_2(i t A_s) r, the
    // second inverse formula (Section 3.1), whose fixed-point map is the
    // time-averaged one of Theorem 2.2.  Both return w without the factor -i t.
    const bool form2 = o.inner_solver >= 2;
    const int fn_rhs = form2 ? ACT_PSI2 : ACT_PSI1;
    const int fn_op = form2 ? ACT_PSI1 : ACT_EXP;
    // r_hat = psi_1(i t A_s) r (or psi_2); z = ||r_hat||
    action64(run, sc, o.t, o.shift, fn_rhs, ap, r, rhat, &cnt.steps);
    cnt.actions++;
    const double z = norm2(run, rhat);
    launch_zero<double>(w, n, s);
    const double tol = o.fprtol * z;
    // Algorithm 1 tests the tolerance before the first inner iteration.
    if (z == 0.0 || z <= tol) return 0;
    if (o.inner_solver == 1 || o.inner_solver == 3) {
        // plain fixed-point iteration w <- E w + r_hat from w = 0, E the
        // form's operator (Theorems 2.1 and 2.2).  The residual r_hat - (I - E) w
        // of the current iterate is also the step to the next one; the first
        // iterate whose residual meets the test is returned.  w_1 = r_hat needs
        // no action (w_0 = 0 failed the test above).
        cpx<double>* d = V;
        launch_scale(one, rhat, w, n, s);
        int its = 0;
        while (its < o.max_inner) {
            action64(run, sc, o.t, o.shift, fn_op, ap, w, d, &cnt.steps);
            cnt.actions++;
            ++its;
            launch_axpby(one, rhat, one, d, n, s);  // E w + r_hat
            launch_axpby(mone, w, one, d, n, s);    // minus w: the residual of w
            const double res = norm2(run, d);
            if (!std::isfinite(res)) fail(MXP_ERR_NONFINITE, "non-finite fixed-point residual");
            if (res <= tol) break;
            launch_axpby(one, d, one, w, n, s);     // the next iterate
        }
        return its;
    }
    // The mixed form keeps the inner basis in complex float: the system is
    // only solved to fprtol, and its actions run in complex float anyway.
    // The new direction and the Gram-Schmidt sums stay in complex double; a
    // float basis vector is widened into `rr` (free within a cycle) as the
    // action's input.  It halves the basis traffic of CGS2.
    const bool v32 = !basis64;
    cpx<float>* V32 = nullptr;
    if (v32) {
        WS.innerV32.ensure(size_t(m + 1) * n * sizeof(cpx<float>));
        V32 = WS.innerV32.as<cpx<float>>();
    }
    const cpx<double>* rcur = rhat;
    double beta = z;
    // Learned warm start (use_learned = 2, not in the paper): the network is
    // trained on pairs (r, M(r)), so w_0 = network(r) approximates this
    // apply's answer.  GMRES then works on the residual r_hat - (I - E) w_0,
    // which costs one action; w_0 is kept only if that residual is below
    // ||r_hat||, else the inner solve starts from zero as Algorithm 1 does.
    if (o.use_learned == 2 && P->net && !form2) {
        const double rn = norm2(run, r);
        if (rn > 0) {
            learned_apply(run, r, rn, w);
            action64(run, sc, o.t, o.shift, fn_op, ap, w, tmp, &cnt.steps);
            cnt.actions++;
            launch_scale(one, rhat, rr, n, s);
            launch_axpby(mone, w, one, rr, n, s);
            launch_axpby(one, tmp, one, rr, n, s);
            const double b0 = norm2(run, rr);
            if (std::isfinite(b0) && b0 < z) {
                rcur = rr;
                beta = b0;
                cnt.learned++;
                if (beta <= tol) return 0;
            } else {
                launch_zero<double>(w, n, s);
                cnt.fallbacks++;
            }
        }
    }
    int its = 0;
    Givens gv(m);
    std::vector<cd> h;
    while (true) {
        if (v32) launch_scale_to_c64({1.0 / beta, 0.0}, rcur, V32, n, s);
        else launch_scale({1.0 / beta, 0.0}, rcur, V, n, s);
        gv.reset(beta);
        int k = 0;
        bool conv = false;
        for (int j = 0; j < m; ++j) {
            cpx<double>* vj = V + size_t(j) * n;
            // the new direction: the basis' next slot, or (float basis) V's first
            cpx<double>* vn = v32 ? V : V + size_t(j + 1) * n;
            if (v32) {
                launch_to_c128(V32 + size_t(j) * n, rr, n, s);
                vj = rr;
            }
            action64(run, sc, o.t, o.shift, fn_op, ap, vj, tmp, &cnt.steps);
            cnt.actions++;
            // v_{j+1} <- v_j - E v_j
            launch_scale(one, vj, vn, n, s);
            launch_axpby(mone, tmp, one, vn, n, s);
            const double hn = v32 ? cgs2(run, V32, n, j + 1, vn, h) : cgs2(run, V, n, j + 1, vn, h);
            ++its;
            const double res = gv.add_column(j, h, hn);
            if (!std::isfinite(res)) fail(MXP_ERR_NONFINITE, "non-finite inner residual estimate");
            const bool breakdown = hn <= 1e-14 * beta;
            if (!breakdown) {
                if (v32) launch_scale_to_c64({1.0 / hn, 0.0}, vn, V32 + size_t(j + 1) * n, n, s);
                else launch_scale({1.0 / hn, 0.0}, vn, vn, n, s);
            }
            k = j + 1;
            if (res <= tol || breakdown) {
                conv = true;
                break;
            }
            if (its >= o.max_inner) break;
        }
        const std::vector<cd> y = gv.solve(k);
        upload_coeffs(run, y);
        if (v32) launch_mcombine(w, static_cast<const cpx<float>*>(V32), n, k, small_buffers(run).y, n, s);
        else launch_mcombine(w, static_cast<const cpx<double>*>(V), n, k, small_buffers(run).y, n, s);
        if (conv || its >= o.max_inner) break;
        // restart: r = r_hat - (w - E w)
        action64(run, sc, o.t, o.shift, fn_op, ap, w, tmp, &cnt.steps);
        cnt.actions++;
        launch_scale(one, rhat, rr, n, s);
        launch_axpby(mone, w, one, rr, n, s);
        launch_axpby(one, tmp, one, rr, n, s);
        rcur = rr;
        beta = norm2(run, rr);
        if (beta <= tol) break;
    }
    return its;
}

// Gram-Schmidt with a second pass, complex double), H is the Hessenberg
// matrix of A_s on it, and y = ||x|| V f(i t H) e_1 with the small
// exponential computed densely on the host (psi_1 from the augmented matrix
// [[i t H, e_1], [0, 0]]).  At m = 8, 16, 24, 32 and then every 16 vectors the
// estimate h_{m+1,m} |e_m^T f(i t H_m) e_1| (relative to ||x||) is compared
// with tol.
// x may equal y (the basis holds x before y is written).  Returns the basis
// size; *ok is false if max_dim vectors did not meet tol (y then holds the
// last approximation).
static int arnoldi_action(Run& run, bool psi, double t, double shift, double tol, int max_dim,
                         const cpx<double>* x, cpx<double>* y, bool* ok) {
    mxp_problem* P = run.P;
    Workspace& WS = *run.W;
    const int64_t n = npts(P);
    hipStream_t s = run.s;
    *ok = false;
    const double beta = norm2(run, x);
    if (beta == 0.0) {
        launch_zero<double>(y, n, s);
        *ok = true;
        return 0;
    }
    WS.krylovV.ensure(size_t(max_dim + 1) * n * sizeof(cpx<double>));
    cpx<double>* V = WS.krylovV.as<cpx<double>>();
    launch_scale({1.0 / beta, 0.0}, x, V, n, s);
    const size_t ldh = size_t(max_dim) + 1;
    std::vector<cd> H(ldh * max_dim, cd(0.0, 0.0));  // column j holds A_s v_j
    std::vector<cd> h, f;
    auto small_fn = [&](int k) {
        const int q = psi ? k + 1 : k;
        std::vector<cd> M(size_t(q) * q, cd(0.0, 0.0));
        for (int j = 0; j < k; ++j)
            for (int i = 0; i <= std::min(j + 1, k - 1); ++i) M[size_t(i) * q + j] = cd(0.0, t) * H[i + ldh * j];
        if (psi) M[k] = 1.0;  // row 0, column k: e_1
        expm_dense(q, M);
        f.resize(k);
        for (int i = 0; i < k; ++i) f[i] = M[size_t(i) * q + (psi ? k : 0)] * beta;
    };
    int m = 0;
    for (int j = 0; j < max_dim; ++j) {
        cpx<double>* vj = V + size_t(j) * n;
        cpx<double>* vn = V + size_t(j + 1) * n;
        apply_A64(P, s, shift, vj, vn, 1.0, nullptr, 0.0);
        const double hn = cgs2(run, V, n, j + 1, vn, h);
        double hmax = hn;
        for (int i = 0; i <= j; ++i) {
            H[i + ldh * j] = h[i];
            hmax = std::max(hmax, std::abs(h[i]));
        }
        H[j + 1 + ldh * j] = hn;
        m = j + 1;
        const bool breakdown = hn <= 1e-13 * hmax;  // the space is invariant: f(i t H) is exact
        if (!breakdown) launch_scale({1.0 / hn, 0.0}, vn, vn, n, s);
        if (breakdown || (m % 8 == 0 && (m <= 32 || m % 16 == 0)) || m == max_dim) {
            small_fn(m);
            const double est = breakdown ? 0.0 : hn * std::abs(f[m - 1]) / beta;
            if (!std::isfinite(est)) fail(MXP_ERR_NONFINITE, "non-finite Krylov estimate");
            if (est <= tol) {
                *ok = true;
                break;
            }
        }
    }
    upload_coeffs(run, f);
    launch_zero<double>(y, n, s);  // mcombine accumulates: y += V f
    launch_mcombine(y, V, n, m, small_buffers(run).y, n, s);
    return m;
}

// The Arnoldi route restarted by time stepping: with tau = t/q,
//   exp(i t A_s) x = (exp(i tau A_s))^q x, a fresh basis per substep, and
//   psi_1(i t A_s) x = (1/q) sum_{k<q} exp(i k tau A_s) p, p = psi_1(i tau A_s) x
// (the variation-of-constants split the Chebyshev schedule also uses), by
// y <- exp(i tau A_s) y + p.  q starts at 1 and doubles, up to 64, until every
// substep's basis meets tol / q within max_dim vectors.  Returns the vectors
// built over all attempts; *ok is false if q = 64 did not suffice.
int krylov_action(Run& run, bool psi, double t, double shift, double tol, int max_dim,
                         const cpx<double>* x, cpx<double>* y, bool* ok) {
    Range range("arnoldi action");
    const int64_t n = npts(run.P);
    hipStream_t s = run.s;
    int total = 0;
    *ok = false;
    run.W->krylovV.ensure(size_t(max_dim + 1) * n * sizeof(cpx<double>));
    if (psi) run.W->krylovP.ensure(size_t(n) * sizeof(cpx<double>));
    (void)small_buffers(run);
    (void)plain_diag(run.P, shift);
    t_reserved = true;
    for (int q = 1; q <= 64 && !*ok; q *= 2) {
        const double tau = t / q, tq = tol / q;
        bool all = true, step_ok = false;
        if (!psi) {
            const cpx<double>* cur = x;
            for (int k = 0; k < q && all; ++k) {
                total += arnoldi_action(run, false, tau, shift, tq, max_dim, cur, y, &step_ok);
                all = step_ok;
                cur = y;
            }
        } else {
            run.W->krylovP.ensure(size_t(n) * sizeof(cpx<double>));
            cpx<double>* p = run.W->krylovP.as<cpx<double>>();
            total += arnoldi_action(run, true, tau, shift, tq, max_dim, x, p, &step_ok);
            all = step_ok;
            launch_scale({1.0, 0.0}, p, y, n, s);
            for (int k = 1; k < q && all; ++k) {
                total += arnoldi_action(run, false, tau, shift, tq, max_dim, y, y, &step_ok);
                all = step_ok;
                launch_axpby({1.0, 0.0}, p, {1.0, 0.0}, y, n, s);
            }
            if (q > 1) launch_scale({1.0 / q, 0.0}, y, y, n, s);
        }
        *ok = all;
    }
    return total;
}

void check_opts(const mxp_solve_opts* o) {
    if (!o) fail(MXP_ERR_INVALID_ARG, "options are NULL");
    if (!(o->t > 0) || !std::isfinite(o->t)) fail(MXP_ERR_INVALID_ARG, "t must be positive");
    if (!(o->shift >= 0) || !std::isfinite(o->shift)) fail(MXP_ERR_INVALID_ARG, "shift must be >= 0");
    if (!(o->fprtol > 0) || o->fprtol > 1) fail(MXP_ERR_INVALID_ARG, "fprtol must be in (0, 1]");
    if (!(o->rtol > 0) || o->rtol >= 1) fail(MXP_ERR_INVALID_ARG, "rtol must be in (0, 1)");
    if (o->outer_restart < 1 || o->outer_restart > 200) fail(MXP_ERR_INVALID_ARG, "outer_restart in 1..200");
    if (o->inner_restart < 1 || o->inner_restart > 200) fail(MXP_ERR_INVALID_ARG, "inner_restart in 1..200");
    if (o->max_outer < 1 || o->max_inner < 1) fail(MXP_ERR_INVALID_ARG, "iteration limits must be >= 1");
    if (o->precision != MXP_PREC_FP64 && o->precision != MXP_PREC_MIXED)
        fail(MXP_ERR_INVALID_ARG, "unknown precision");
    if (o->cheb_S < 0 || o->cheb_m < 0) fail(MXP_ERR_INVALID_ARG, "cheb_S, cheb_m must be >= 0");
    if (o->use_learned < 0 || o->use_learned > 2) fail(MXP_ERR_INVALID_ARG, "use_learned must be 0, 1 or 2");
    if (o->use_learned && !(o->stall_ratio >= 0 && o->stall_ratio <= 1))
        fail(MXP_ERR_INVALID_ARG, "stall_ratio must be in [0, 1]");
    if (o->inner_solver < 0 || o->inner_solver > 3) fail(MXP_ERR_INVALID_ARG, "inner_solver must be 0, 1, 2 or 3");
    if (!(o->fp64_below >= 0) || !(o->fp64_below < 1)) fail(MXP_ERR_INVALID_ARG, "fp64_below must be in [0, 1)");
    if (o->fp64_first < 0) fail(MXP_ERR_INVALID_ARG, "fp64_first must be >= 0");
}

void reserve_precond(Run& run, const mxp_solve_opts& o) {
    mxp_problem* P = run.P;
    Workspace& WS = *run.W;
    const size_t n = size_t(npts(P));
    const Sched& sc = get_sched(P, o.t, o.shift, o.precision, o.cheb_S, o.cheb_m);
    reserve_action(P, WS, sc, o.inner_solver >= 2, o.use_graphs != 0 && !run.batch, run.s);
    if (o.precision == MXP_PREC_MIXED && (o.fp64_below > 0 || o.fp64_first > 0)) {
        const Sched& s64 = get_sched(P, o.t, o.shift, MXP_PREC_FP64, o.cheb_S, o.cheb_m);
        reserve_action(P, WS, s64, o.inner_solver >= 2, o.use_graphs != 0 && !run.batch, run.s);
    }
    const int m = o.inner_restart;
    const bool gmres = o.inner_solver == 0 || o.inner_solver == 2;
    const bool basis64 = o.precision == MXP_PREC_FP64 && gmres;
    WS.innerV.ensure(size_t(basis64 ? m + 1 : 1) * n * sizeof(cpx<double>));
    WS.innerRh.ensure(n * sizeof(cpx<double>));
    WS.innerTmp.ensure(n * sizeof(cpx<double>));
    WS.innerRr.ensure(n * sizeof(cpx<double>));
    if (gmres && !basis64) WS.innerV32.ensure(size_t(m + 1) * n * sizeof(cpx<float>));
    (void)small_buffers(run);
    if (o.use_learned && P->net)
        cnn_reserve(P->net, ConvShape{1, int(P->g.n[2]), int(P->g.n[1]), int(P->g.n[0])}, run.s);
}

void reserve_solve(Run& run, const mxp_solve_opts& o) {
    mxp_problem* P = run.P;
    Workspace& WS = *run.W;
    const size_t n = size_t(npts(P));
    const int m = o.outer_restart;
    WS.outerV.ensure(size_t(m + 1) * n * sizeof(cpx<double>));
    WS.outerZ.ensure(size_t(m) * n * sizeof(cpx<double>));
    WS.outerR.ensure(n * sizeof(cpx<double>));
    (void)plain_diag(P, 0.0);  // A itself, for A z_j and the true residual
    reserve_precond(run, o);
}

mxp_status solve(Run& run, const mxp_solve_opts& o, const cpx<double>* f, cpx<double>* u,
                        mxp_solve_stats* st) {
    Range range("mxp solve");
    const auto t0 = std::chrono::steady_clock::now();
    mxp_problem* P = run.P;
    Workspace& WS = *run.W;
    const int64_t n = npts(P);
    hipStream_t s = run.s;
    const int m = o.outer_restart;
    reserve_solve(run, o);
    t_reserved = true;
    cpx<double>* V = WS.outerV.as<cpx<double>>();
    cpx<double>* Z = WS.outerZ.as<cpx<double>>();
    cpx<double>* r = WS.outerR.as<cpx<double>>();
    Counters cnt;
    std::vector<int> inner;
    std::vector<int32_t> hist_inner;
    std::vector<double> hist_res;
    const double bnorm = norm2(run, f);
    // r = -f - A u
    apply_A64(P, s, 0.0, u, r, -1.0, f, -1.0);
    double beta = norm2(run, r);
    int its = 0, cycles = 0;
    double relres = bnorm > 0 ? beta / bnorm : 0.0;
    Givens gv(m);
    std::vector<cd> h;
    if (bnorm == 0.0) {
        launch_zero<double>(u, n, s);
        relres = 0.0;
    }
    if (o.use_learned && !P->net) fail(MXP_ERR_INVALID_ARG, "use_learned needs a network (mxp_problem_set_learned)");
    if (o.use_learned && run.batch) fail(MXP_ERR_UNSUPPORTED, "the learned stage runs in single solves only");
    int misses = 0;
    // cost-aware acceptance in counted work (reproducible): mean log residual
    // reduction and stencil steps of the MatExPre iterations so far; a network
    // try counts as kNetTrySteps steps
    double m_log = 0.0;
    int64_t m_steps = 0;
    int m_count = 0;
    while (bnorm > 0.0 && beta > o.rtol * bnorm) {
        ++cycles;
        launch_scale({1.0 / beta, 0.0}, r, V, n, s);
        gv.reset(beta);
        double prev_res = beta;
        // the network gets a fresh chance in every restart cycle
        bool use_net = o.use_learned == 1;
        misses = 0;
        int k = 0;
        bool est_ok = false;
        for (int j = 0; j < m; ++j) {
            cpx<double>* vj = V + size_t(j) * n;
            cpx<double>* zj = Z + size_t(j) * n;
            cpx<double>* vn = V + size_t(j + 1) * n;
            // Learned stage: try the network's z_j first and keep it when the
            // Arnoldi residual estimate falls below a threshold times the
            // previous one: stall_ratio when it is > 0, else the smaller of
            // the mean reduction of MatExPre's own iterations (a kept
            // direction takes a slot of the restart cycle, so it must do as
            // well as the iteration it displaces) and the reduction they
            // achieve on average in the stencil steps one network try counts
            // for (so it is also at least as cost-effective).  Otherwise the MatExPre
            // preconditioner supplies z_j; after two misses in a row it does
            // so until the next restart cycle.  The first iteration of a
            // solve always uses MatExPre (it calibrates the threshold).
            double hn = 0.0, res = 0.0;
            bool accepted = false;
            const bool calibrated = o.stall_ratio > 0 || m_count > 0;
            if (use_net && calibrated) {
                learned_apply(run, vj, 1.0, zj);
                apply_A64(P, s, 0.0, zj, vn, 1.0, nullptr, 0.0);
                hn = cgs2(run, V, n, j + 1, vn, h);
                Givens trial = gv;
                res = trial.add_column(j, h, hn);
                // a proposal whose column is zero or (nearly) dependent on the
                // earlier ones leaves a singular factor, and its residual
                // estimate (zero after a degenerate rotation) means nothing
                double col = hn * hn;
                for (int i = 0; i <= j; ++i) col += std::norm(h[i]);
                const bool singular = !(std::abs(trial.at(j, j)) > 1e-8 * std::sqrt(col));
                double thr = o.stall_ratio;
                if (thr <= 0) {
                    const double per_it = m_log / m_count;                            // log reduction per iteration
                    const double per_step = m_log / std::max(double(m_steps), 1.0);  // ... per stencil step
                    thr = std::min(1.0, std::min(std::exp(per_it), std::exp(per_step * kNetTrySteps)));
                }
                if (!singular && std::isfinite(res) && res <= thr * prev_res) {
                    gv = trial;
                    accepted = true;
                    cnt.learned++;
                    misses = 0;
                } else {
                    cnt.fallbacks++;
                    if (++misses >= 2) use_net = false;
                }
            }
            if (!accepted) {
                const int64_t steps0 = cnt.steps;
                // mixed form: the first fp64_first outer iterations of the solve
                // (whose directions enter the iterate with the largest
                // coefficients), and those starting below fp64_below, run the
                // preconditioner's actions in double
                const bool dbl = o.precision == MXP_PREC_MIXED &&
                                 (its < o.fp64_first || (o.fp64_below > 0 && prev_res <= o.fp64_below * bnorm));
                if (dbl) cnt.fp64_its++;
                inner.push_back(precond(run, o, vj, zj, cnt, dbl ? MXP_PREC_FP64 : o.precision));
                if (run.pairs && run.pairs->count < run.pairs->max) {
                    PairSink& ps = *run.pairs;
                    HIP_CHECK(hipMemcpyAsync(ps.r + size_t(ps.count) * n, vj, size_t(n) * sizeof(cpx<double>),
                                             hipMemcpyDeviceToDevice, s));
                    HIP_CHECK(hipMemcpyAsync(ps.z + size_t(ps.count) * n, zj, size_t(n) * sizeof(cpx<double>),
                                             hipMemcpyDeviceToDevice, s));
                    ps.rnorm[ps.count] = 1.0;
                    ps.znorm[ps.count] = norm2(run, zj);
                    ps.count++;
                }
                apply_A64(P, s, 0.0, zj, vn, 1.0, nullptr, 0.0);
                hn = cgs2(run, V, n, j + 1, vn, h);
                res = gv.add_column(j, h, hn);
                if (res > 0 && prev_res > 0 && std::isfinite(res)) {
                    m_log += std::log(res / prev_res);
                    m_steps += cnt.steps - steps0;
                    ++m_count;
                }
            }
            ++its;
            prev_res = res;
            hist_inner.push_back(accepted ? -1 : inner.back());
            hist_res.push_back(bnorm > 0 ? res / bnorm : 0.0);
            if (P->ctx->verbose) {
                const double el = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
                std::fprintf(stderr, "[mxp] outer %d: est relres %.3e, %s, steps %lld, %.2f s\n", its,
                             res / bnorm, accepted ? "learned" : ("inner " + std::to_string(inner.back())).c_str(),
                             (long long)cnt.steps, el);
                std::fflush(stderr);
            }
            if (!std::isfinite(res)) fail(MXP_ERR_NONFINITE, "non-finite outer residual estimate");
            const bool breakdown = hn <= 1e-14 * beta;
            if (!breakdown) launch_scale({1.0 / hn, 0.0}, vn, vn, n, s);
            k = j + 1;
            if (res <= o.rtol * bnorm || breakdown) {
                est_ok = true;
                break;
            }
            if (its >= o.max_outer) break;
        }
        const std::vector<cd> y = gv.solve(k);
        upload_coeffs(run, y);
        launch_mcombine(u, Z, n, k, small_buffers(run).y, n, s);
        apply_A64(P, s, 0.0, u, r, -1.0, f, -1.0);
        beta = norm2(run, r);
        relres = beta / bnorm;
        if ((est_ok && relres <= o.rtol) || its >= o.max_outer) break;
        if (relres <= o.rtol) break;
    }
    HIP_CHECK(hipStreamSynchronize(s));
    if (!run.batch) {  // batched right-hand sides run on concurrent host threads
        P->hist_inner = std::move(hist_inner);
        P->hist_res = std::move(hist_res);
    }
    if (st) {
        std::memset(st, 0, sizeof(*st));
        st->outer_its = its;
        int tot = 0;
        for (int v : inner) tot += v;
        st->inner_its_total = tot;
        if (!inner.empty()) {
            const double mean = double(tot) / inner.size();
            double var = 0;
            for (int v : inner) var += (v - mean) * (v - mean);
            st->inner_mean = mean;
            st->inner_std = std::sqrt(var / inner.size());
        }
        st->stencil_steps = cnt.steps;
        st->fn_actions = cnt.actions;
        st->true_relres = relres;
        st->restarts = std::max(0, cycles - 1);
        st->learned_its = cnt.learned;
        st->fp64_its = cnt.fp64_its;
        st->fallbacks = cnt.fallbacks;
        st->status = relres <= o.rtol ? MXP_OK : MXP_NOT_CONVERGED;
        st->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    return relres <= o.rtol ? MXP_OK : MXP_NOT_CONVERGED;
}

}  // namespace mxp
