// C ABI of the MatExPre library: contexts, problems, matrix-function actions,
// the preconditioner of Algorithm 1 and the outer flexible GMRES.
//
// Paper passages implemented here:
//   * Section 3.1 (eq. inverse-1): exp(i t A) and psi_1(i t A) actions;
//     t psi_1(i t A) r = sum_{k<S} exp(i k tau A) tau psi_1(i tau A) r, tau = t/S
//     (semigroup property plus the variation-of-constants integral);
//   * Section 3.4 (eq. fixed-point, Algorithm 1): inner GMRES on
//     (I - exp(i t A_s)) w = psi_1(i t A_s) r to relative tolerance fprtol;
//   * Section 3.4: complex shift A_s = A + i omega^2 s D; outer flexible GMRES
//     (constant -i t dropped);
//   * Section 4 introduction: restart 30 for both solvers;
//   * variants of Algorithm 1: the plain fixed-point iteration (Section 2.1,
//     Theorem 2.1) and the second inverse formula
//     (I - psi_1(i t A_s)) w = psi_2(i t A_s) r (Section 3.1; its fixed-point
//     map is Theorem 2.2's), with the psi_2 action on the exp substeps;
//   * the matrix functions by the Arnoldi method, the paper's own route
//     (Section 4 introduction), as an alternative building block.
// Orthogonalisation is classical Gram--Schmidt with one re-orthogonalisation
// (CGS2: two fused multi-dot / multi-update passes); the small least-squares
// problems use Givens rotations on the host in double.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cmath>
#include <cstring>
#include <condition_variable>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <tuple>
#include <vector>

#include "cheb3d.h"
#include "cnn_net.h"
#include "devmem.h"
#include "kernels.h"
#include "mxp_internal.h"

struct mxp_context {
    int device;
    hipStream_t stream;
    int verbose;  // MXP_VERBOSE=1: one line per outer iteration on stderr
};

namespace mxp {

thread_local std::string g_last_error;

template <typename R>
struct DevTables {
    cpx<R>* alpha[3] = {nullptr, nullptr, nullptr};
    cpx<R>* beta[3] = {nullptr, nullptr, nullptr};
    cpx<R>* gamma[3] = {nullptr, nullptr, nullptr};
};

// Per-axis diagonal tables gamma_d + (kD * Dref - centre)/dim for one
// (shift, centre) pair, in both precisions.
struct DiagTables {
    DevMem mem64, mem32;
    cpx<double>* g64[3] = {nullptr, nullptr, nullptr};
    cpx<float>* g32[3] = {nullptr, nullptr, nullptr};
    // 2D fused passes: h^2-scaled alpha, beta, gamma of the x and y axes
    // ([axis][alpha, beta, gamma]) and the interior box with unit weights
    DevMem fmem64, fmem32;
    cpx<double>* f64[2][3] = {{nullptr, nullptr, nullptr}, {nullptr, nullptr, nullptr}};
    cpx<float>* f32[2][3] = {{nullptr, nullptr, nullptr}, {nullptr, nullptr, nullptr}};
    int64_t ix0 = 0, ix1 = 0, iy0 = 0, iy1 = 0;
};

struct Sched {
    mxp_schedule s;
    DiagTables diag;
    double t = 0.0;
    mxp_precision prec = MXP_PREC_FP64;
    // psi_2 series on the same segment, designed at its first use
    mutable std::vector<double> coef_psi2;
    mutable int m_psi2 = -1;
};

// Which matrix function an action applies.
enum ActFn { ACT_EXP = 0, ACT_PSI1 = 1, ACT_PSI2 = 2 };

// Tile configuration of the temporally blocked 2D Clenshaw pass.
struct TileCfg {
    int K = 0, NX = 1, Ly = 32;
    double us_per_level = 0.0;
};

// Device workspace of one solve: Krylov bases, matrix-function buffers and
// reduction scratch.  A problem owns one for its single-solve calls; a
// batched solve gives every right-hand side its own.
// A matrix-function action captured into a HIP graph (fixed input and
// output buffers of the workspace), replayed on the workspace's own stream.
struct GraphEntry {
    int uses = 0;  // the first use runs eagerly (allocations, tile tuning)
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int64_t steps = 0;  // Clenshaw levels per replay
};

struct Workspace {
    // [0..5] pass/substep buffers, [6] psi addend, (f64) [7..8] graph input /
    // output, (f32) [7..8] casts, [9] the psi_2 action's first-substep term
    DevMem act64[10], act32[10];
    DevMem innerV, innerRh, innerTmp, innerRr;
    DevMem innerV32;  // complex-float inner basis of the mixed form
    DevMem krylovV, krylovP;
    DevMem outerV, outerZ, outerR;
    DevMem partial, small;
    std::vector<cpx<double>> host_small;
    // captured actions, keyed by (schedule, function, precision); the stream they
    // replay on and the events that order it with the solve's stream
    std::map<std::tuple<const void*, int, int>, GraphEntry> graphs;
    hipStream_t gstream = nullptr;
    hipEvent_t gev[2] = {nullptr, nullptr};
    Workspace() = default;
    Workspace(const Workspace&) = delete;
    Workspace& operator=(const Workspace&) = delete;
    void drop_graphs() {
        for (auto& kv : graphs) {
            if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
            if (kv.second.graph) (void)hipGraphDestroy(kv.second.graph);
        }
        graphs.clear();
    }
    ~Workspace() {
        drop_graphs();
        if (gstream) {
            (void)hipStreamSynchronize(gstream);
            (void)hipStreamDestroy(gstream);
        }
        for (hipEvent_t e : gev)
            if (e) (void)hipEventDestroy(e);
    }
};

class Batcher;

// Where a solve copies its (Krylov vector, preconditioned vector) pairs.
struct PairSink {
    cpx<double>* r;
    cpx<double>* z;
    double* rnorm;  // host
    double* znorm;  // host
    int max, count;
};

// One solve in progress: its problem (read-only while solving), workspace,
// the stream its Krylov work runs on, and the batcher its matrix-function
// actions go to (nullptr: run them directly on that stream).
struct Run {
    mxp_problem* P;
    Workspace* W;
    hipStream_t s;
    Batcher* batch;
    hipEvent_t ev;  // batched runs: marks the action input ready on s
    PairSink* pairs = nullptr;
    bool graphs = false;  // replay matrix-function actions from captured HIP graphs
};

}  // namespace mxp

struct mxp_problem {
    mxp_context ctx_copy;  // device, stream, verbosity: the problem outlives nothing it points to
    mxp_context* ctx;      // == &ctx_copy
    mxp::GridInfo g;
    mxp::DevMem tables64, tables32, D64, D32;
    mxp::DevTables<double> t64;
    mxp::DevTables<float> t32;
    std::map<std::tuple<double, double, int, int, int>, std::unique_ptr<mxp::Sched>> scheds;
    std::map<double, std::unique_ptr<mxp::DiagTables>> plain_diag;  // centre 0, keyed by shift
    double Dref = 0.0;  // reference value of D folded into the diagonal tables
    mxp::TileCfg tiles[2];  // per precision (0 = double, 1 = float); K = 0 until tuned
    mxp::Workspace ws;      // workspace of the single-solve calls
    mxp_cnn* net = nullptr; // learned stage (not owned), with its output scale
    double net_scale = 1.0;
    // per outer iteration of the last single solve: inner iterations (-1 for
    // a kept network direction) and the Arnoldi relative residual estimate
    std::vector<int32_t> hist_inner;
    std::vector<double> hist_res;
};

namespace mxp {

static int64_t npts(const mxp_problem* P) { return P->g.npts(); }

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
}

static void build_diag(mxp_problem* P, double shift, cd centre, DiagTables& dt) {
    const GridInfo& g = P->g;
    const cd share = (cd(g.omega * g.omega, g.omega * g.omega * shift) * P->Dref - centre) / double(g.dim);
    size_t total = 0;
    for (int d = 0; d < 3; ++d) total += size_t(g.n[d]);
    std::vector<cpx<double>> h64(total);
    std::vector<cpx<float>> h32(total);
    size_t off = 0, offs[3];
    for (int d = 0; d < 3; ++d) {
        offs[d] = off;
        if (d < g.dim) {
            const AxisTables at = build_axis_tables(g.axis(d));
            for (int64_t i = 0; i < g.n[d]; ++i) {
                const cd v = at.gamma[i] + share;
                h64[off + i] = {v.real(), v.imag()};
                h32[off + i] = {float(v.real()), float(v.imag())};
            }
        } else {
            for (int64_t i = 0; i < g.n[d]; ++i) {
                h64[off + i] = {0.0, 0.0};
                h32[off + i] = {0.0f, 0.0f};
            }
        }
        off += g.n[d];
    }
    // Interior box: a node needs alpha = beta = 1/h^2 on its axis, i.e. the
    // stretch is 1 at the node and both half-nodes (everywhere with the
    // absorbing potential, which sits in the diagonal).  Nodes 0 and n-1 are
    // excluded so that every neighbour read stays inside the grid there.
    auto span = [&](int d, int64_t* lo, int64_t* hi) {
        const AxisLayer ax = g.axis(d);
        int64_t a0 = 1, a1 = g.n[d] - 1;
        while (a0 < a1 && (ax.stretch(a0 * g.h) != 0.0 || ax.stretch((a0 - 0.5) * g.h) != 0.0 ||
                           ax.stretch((a0 + 0.5) * g.h) != 0.0))
            ++a0;
        while (a1 > a0 && (ax.stretch((a1 - 1) * g.h) != 0.0 || ax.stretch((a1 - 0.5) * g.h) != 0.0 ||
                           ax.stretch((a1 - 1.5) * g.h) != 0.0))
            --a1;
        *lo = a0;
        *hi = a1;
    };
    if (g.dim == 2) {
        span(0, &dt.ix0, &dt.ix1);
        span(1, &dt.iy0, &dt.iy1);
        if (!(dt.ix0 < dt.ix1 && dt.iy0 < dt.iy1)) dt.ix0 = dt.ix1 = dt.iy0 = dt.iy1 = 0;
        const double h2 = g.h * g.h;
        const size_t tot2 = 3 * size_t(g.n[0] + g.n[1]);
        std::vector<cpx<double>> s64(tot2);
        std::vector<cpx<float>> s32(tot2);
        size_t o = 0, fo[2][3];
        for (int d = 0; d < 2; ++d) {
            const AxisTables at = build_axis_tables(g.axis(d));
            const std::vector<cd>* src[3] = {&at.alpha, &at.beta, &at.gamma};
            for (int q = 0; q < 3; ++q) {
                fo[d][q] = o;
                for (int64_t i = 0; i < g.n[d]; ++i) {
                    const cd v = ((*src[q])[i] + (q == 2 ? share : cd(0.0, 0.0))) * h2;
                    s64[o + i] = {v.real(), v.imag()};
                    s32[o + i] = {float(v.real()), float(v.imag())};
                }
                o += g.n[d];
            }
        }
        dt.fmem64.ensure(tot2 * sizeof(cpx<double>));
        dt.fmem32.ensure(tot2 * sizeof(cpx<float>));
        HIP_CHECK(hipMemcpy(dt.fmem64.p, s64.data(), tot2 * sizeof(cpx<double>), hipMemcpyHostToDevice));
        HIP_CHECK(hipMemcpy(dt.fmem32.p, s32.data(), tot2 * sizeof(cpx<float>), hipMemcpyHostToDevice));
        for (int d = 0; d < 2; ++d)
            for (int q = 0; q < 3; ++q) {
                dt.f64[d][q] = dt.fmem64.as<cpx<double>>() + fo[d][q];
                dt.f32[d][q] = dt.fmem32.as<cpx<float>>() + fo[d][q];
            }
    }
    dt.mem64.ensure(total * sizeof(cpx<double>));
    dt.mem32.ensure(total * sizeof(cpx<float>));
    HIP_CHECK(hipMemcpy(dt.mem64.p, h64.data(), total * sizeof(cpx<double>), hipMemcpyHostToDevice));
    HIP_CHECK(hipMemcpy(dt.mem32.p, h32.data(), total * sizeof(cpx<float>), hipMemcpyHostToDevice));
    for (int d = 0; d < 3; ++d) {
        dt.g64[d] = dt.mem64.as<cpx<double>>() + offs[d];
        dt.g32[d] = dt.mem32.as<cpx<float>>() + offs[d];
    }
}

static const DiagTables& plain_diag(mxp_problem* P, double shift) {
    auto it = P->plain_diag.find(shift);
    if (it != P->plain_diag.end()) return *it->second;
    auto dt = std::make_unique<DiagTables>();
    build_diag(P, shift, cd(0.0, 0.0), *dt);
    const DiagTables& ref = *dt;
    P->plain_diag.emplace(shift, std::move(dt));
    return ref;
}

static const Sched& get_sched(mxp_problem* P, double t, double shift, mxp_precision prec,
                              int forceS, int forcem) {
    auto key = std::make_tuple(t, shift, int(prec), forceS, forcem);
    auto it = P->scheds.find(key);
    if (it != P->scheds.end()) return *it->second;
    auto sc = std::make_unique<Sched>();
    design_schedule(P->g, t, shift, prec, &sc->s, forceS, forcem);
    build_diag(P, shift, cd(sc->s.centre_re, sc->s.centre_im), sc->diag);
    sc->t = t;
    sc->prec = prec;
    const Sched& ref = *sc;
    P->scheds.emplace(key, std::move(sc));
    return ref;
}

template <typename R>
static StencilArgs<R> base_args(mxp_problem* P, double shift, const DiagTables& diag) {
    StencilArgs<R> a{};
    const GridInfo& g = P->g;
    a.dim = g.dim;
    a.n0 = g.n[0];
    a.n1 = g.n[1];
    a.n2 = g.n[2];
    const DevTables<R>* t;
    if constexpr (sizeof(R) == 8) t = &P->t64; else t = &P->t32;
    for (int d = 0; d < 3; ++d) {
        a.alpha[d] = t->alpha[d];
        a.beta[d] = t->beta[d];
        if constexpr (sizeof(R) == 8) a.gamma[d] = diag.g64[d]; else a.gamma[d] = diag.g32[d];
    }
    if (g.homogeneous) {
        a.D = nullptr;
        a.Dconst = R(P->Dref);  // D - Dref is exactly zero
    } else {
        if constexpr (sizeof(R) == 8) a.D = P->D64.as<double>(); else a.D = P->D32.as<float>();
        a.Dconst = R(0);
    }
    a.Dref = R(P->Dref);
    const double w2 = g.omega * g.omega;
    a.kD = {R(w2), R(w2 * shift)};
    a.g = {R(1), R(0)};
    a.cx = a.e2 = a.e3 = {R(0), R(0)};
    return a;
}

template <typename R>
static cpx<R> to_cpx(cd v) { return {R(v.real()), R(v.imag())}; }

static cd coef_at(const double* c, int k) { return cd(c[2 * k], c[2 * k + 1]); }

// Where the launches of a matrix-function action go: straight onto a stream,
// or into a list that a batched solve replays in lockstep with other actions.
template <typename R>
struct StepRec {
    int kind;  // 0: stencil sweep (st); 1: temporally blocked 2D pass (cp, K, NX); 2: two-level 3D pass (c3)
    StencilArgs<R> st;
    ChebPassArgs<R> cp;
    ChebPass3DArgs<R> c3;
    int K, NX;
};

template <typename R>
struct Emit {
    hipStream_t s;
    std::vector<StepRec<R>>* rec;  // non-null: record instead of launching
    void sweep(const StencilArgs<R>& a) const {
        if (rec) {
            StepRec<R> r{};
            r.kind = 0;
            r.st = a;
            rec->push_back(r);
        } else {
            launch_stencil(a, s);
        }
    }
    void pass(const ChebPassArgs<R>& a, int K, int NX) const {
        if (rec) {
            StepRec<R> r{};
            r.kind = 1;
            r.cp = a;
            r.K = K;
            r.NX = NX;
            rec->push_back(r);
        } else {
            launch_cheb2d<R>(a, K, NX, s);
        }
    }
    void pass3d(const ChebPass3DArgs<R>& a) const {
        if (rec) {
            StepRec<R> r{};
            r.kind = 2;
            r.c3 = a;
            rec->push_back(r);
        } else {
            launch_cheb3d<R>(a, s);
        }
    }
};

// out = post * (sum_{k<=m} c_k T_k(Ahat) x + add), Ahat = (A_s - centre)/hw,
// by the Clenshaw recurrence b_k = c_k x + 2 Ahat b_{k+1} - b_{k+2}.
// bufA, bufB: scratch distinct from x, add and out.  out may equal x.
template <typename R>
static void cheb_series(const Emit<R>& em, const StencilArgs<R>& base, const mxp_schedule& sc,
                        const double* coef, int m, const cpx<R>* x, cpx<R>* out, cpx<R>* bufA,
                        cpx<R>* bufB, cd post, const cpx<R>* add, int64_t* steps) {
    const double hw = sc.half_width;
    StencilArgs<R> a = base;  // the centre is already folded into the diagonal tables
    a.x = x;
    // b_{m-1} = c_{m-1} x + 2 Ahat (c_m x)
    a.b1 = x;
    a.g = to_cpx<R>(coef_at(coef, m) * (2.0 / hw));
    a.cx = to_cpx<R>(coef_at(coef, m - 1));
    a.b2 = nullptr;
    a.b3 = nullptr;
    a.out = bufA;
    em.sweep(a);
    // b_{m-2} = c_{m-2} x + 2 Ahat b_{m-1} - c_m x
    a.b1 = bufA;
    a.g = to_cpx<R>(cd(2.0 / hw, 0.0));
    a.cx = to_cpx<R>(coef_at(coef, m - 2) - coef_at(coef, m));
    a.out = bufB;
    em.sweep(a);
    cpx<R>* cur = bufB;   // b_{k+1}
    cpx<R>* prev = bufA;  // b_{k+2}
    for (int k = m - 3; k >= 1; --k) {
        a.b1 = cur;
        a.b2 = prev;
        a.e2 = {R(-1), R(0)};
        a.cx = to_cpx<R>(coef_at(coef, k));
        a.out = prev;
        em.sweep(a);
        std::swap(cur, prev);
    }
    // out = post * (c_0 x + Ahat b_1 - b_2 + add)
    a.b1 = cur;
    a.b2 = prev;
    a.g = to_cpx<R>(post / hw);
    a.cx = to_cpx<R>(post * coef_at(coef, 0));
    a.e2 = to_cpx<R>(-post);
    a.b3 = add;
    a.e3 = to_cpx<R>(post);
    a.out = out;
    em.sweep(a);
    *steps += m;
}

// The same series on a 3D grid with two Clenshaw levels per pass: levels
// 0 .. m-1 in pairs (level q: c_{m-q} x + (q ? 2/hw : 0) S(L_{q-1}) - L_{q-2}),
// an odd one left over and the final level (post, add) as single sweeps.
// bufs: four scratch vectors distinct from x, add and out.
template <typename R>
static void cheb_series3d(const Emit<R>& em, const StencilArgs<R>& base, const mxp_schedule& sc, const double* coef,
                          int m, const cpx<R>* x, cpx<R>* out, cpx<R>* const bufs[4], cd post, const cpx<R>* add,
                          int64_t* steps) {
    const double hw = sc.half_width;
    ChebPass3DArgs<R> a{};
    a.n0 = base.n0;
    a.n1 = base.n1;
    a.n2 = base.n2;
    for (int d = 0; d < 3; ++d) {
        a.alpha[d] = base.alpha[d];
        a.beta[d] = base.beta[d];
        a.gamma[d] = base.gamma[d];
    }
    a.D = base.D;
    a.Dconst = base.Dconst;
    a.Dref = base.Dref;
    a.kD = base.kD;
    a.x = x;
    cheb3d_geometry<R>(a);
    const cpx<R>* prevA = nullptr;  // L_{q-2}
    const cpx<R>* prevB = nullptr;  // L_{q-1}
    int q = 0, pair = 0;
    while (q + 1 <= m - 1) {
        a.cx[0] = to_cpx<R>(coef_at(coef, m - q));
        a.g[0] = R(q == 0 ? 0.0 : 2.0 / hw);
        a.cx[1] = to_cpx<R>(coef_at(coef, m - q - 1));
        a.g[1] = R(2.0 / hw);
        a.in0 = prevA;
        a.in1 = prevB;
        a.outA = bufs[2 * pair];
        a.outB = bufs[2 * pair + 1];
        em.pass3d(a);
        prevA = a.outA;
        prevB = a.outB;
        pair ^= 1;
        q += 2;
    }
    StencilArgs<R> st = base;
    st.x = x;
    if (q == m - 1) {
        // one more plain level: c_{m-q} x + (q ? 2/hw : 0) S(L_{q-1}) - L_{q-2}
        st.b1 = prevB ? prevB : x;
        st.g = to_cpx<R>(cd(q == 0 ? 0.0 : 2.0 / hw, 0.0));
        st.cx = to_cpx<R>(coef_at(coef, m - q));
        st.b2 = prevA;
        st.e2 = {R(-1), R(0)};
        st.b3 = nullptr;
        st.e3 = {R(0), R(0)};
        st.out = bufs[2 * pair];
        em.sweep(st);
        prevA = prevB;
        prevB = st.out;
    }
    // final level: post * (c_0 x + (1/hw) S(L_{m-1}) - L_{m-2}) + post * add
    st.b1 = prevB ? prevB : x;
    st.g = to_cpx<R>(prevB ? post / hw : cd(0.0, 0.0));
    st.cx = to_cpx<R>(post * coef_at(coef, 0));
    st.b2 = prevA;
    st.e2 = to_cpx<R>(-post);
    st.b3 = add;
    st.e3 = to_cpx<R>(post);
    st.out = out;
    em.sweep(st);
    *steps += m;
}

template <typename R>
static DevMem* act_buffers(Workspace& W) {
    if constexpr (sizeof(R) == 8) return W.act64; else return W.act32;
}

template <typename R>
static ChebPassArgs<R> pass_base(mxp_problem* P, const StencilArgs<R>& st, const DiagTables& dt) {
    ChebPassArgs<R> a{};
    a.n0 = st.n0;
    a.n1 = st.n1;
    cpx<R>* const(*f)[3];
    if constexpr (sizeof(R) == 8) f = dt.f64; else f = dt.f32;
    a.ax = f[0][0];
    a.bx = f[0][1];
    a.gx = f[0][2];
    a.ay = f[1][0];
    a.by = f[1][1];
    a.gy = f[1][2];
    a.D = st.D;
    a.Dconst = st.Dconst;
    a.Dref = st.Dref;
    const double h2 = P->g.h * P->g.h;
    a.kD = {R(double(st.kD.re) * h2), R(double(st.kD.im) * h2)};
    a.ix0 = dt.ix0;
    a.ix1 = dt.ix1;
    a.iy0 = dt.iy0;
    a.iy1 = dt.iy1;
    return a;
}

// out = post * (sum_k c_k T_k(Ahat) x + add) by fused Clenshaw passes (2D).
// bufs: four scratch vectors distinct from x, add and out.
template <typename R>
static void cheb_series_fused(mxp_problem* P, const Emit<R>& em, const StencilArgs<R>& st, const DiagTables& dt,
                              const TileCfg& tc,
                              const mxp_schedule& sc, const double* coef, int m, const cpx<R>* x,
                              cpx<R>* out, cpx<R>* const bufs[4], cd post, const cpx<R>* add,
                              int64_t* steps) {
    ChebPassArgs<R> a = pass_base<R>(P, st, dt);
    a.x = x;
    if (post.imag() != 0.0) fail(MXP_ERR_INVALID_ARG, "series scaling must be real");
    const double inv_h2 = 1.0 / (P->g.h * P->g.h);
    a.post = R(post.real());
    a.e3 = add ? R(post.real()) : R(0);
    const R post_final = a.post, e3_final = a.e3;
    const cpx<R>* prevA = nullptr;
    const cpx<R>* prevB = nullptr;
    int pair = 0;
    int q0 = 0;
    while (q0 <= m) {
        const int nlev = std::min(tc.K, m + 1 - q0);
        const bool last = (q0 + nlev == m + 1);
        for (int l = 0; l < nlev; ++l) {
            // level q: b_{m-q} = c_{m-q} x + (2/hw) A_s-step - b_{m-q+2}; the final
            // level uses c_0 and 1/hw and is scaled by post in the kernel
            const int q = q0 + l;
            const cd cx = coef_at(coef, m - q);
            const double gq = (q == 0) ? 0.0 : (q == m ? 1.0 : 2.0) / sc.half_width;
            a.cx[l] = to_cpx<R>(cx);
            a.g[l] = R(gq * inv_h2);
        }
        a.final_pass = last ? 1 : 0;
        // non-final passes end on a plain level: unit scale, no addend
        a.post = last ? post_final : R(1);
        a.e3 = last ? e3_final : R(0);
        a.in0 = prevA;
        a.in1 = prevB;
        a.add = last ? add : nullptr;
        a.outA = last ? nullptr : bufs[2 * pair];
        a.outB = last ? out : bufs[2 * pair + 1];
        cheb2d_geometry<R>(a, nlev, tc.NX, tc.Ly);
        em.pass(a, nlev, tc.NX);
        prevA = a.outA;
        prevB = a.outB;
        pair ^= 1;
        q0 += nlev;
    }
    *steps += m;
}

template <typename R>
static void tune_tiles(mxp_problem* P, Workspace& ws, const Sched& sd, hipStream_t s);

// y = exp(i t A_s) x, psi_1(i t A_s) x or psi_2(i t A_s) x (fn), precision R.
// x and y distinct device vectors of precision R; buffers from workspace ws.
template <typename R>
static void action(mxp_problem* P, Workspace& ws, const Emit<R>& em, const Sched& sd, double t, double shift,
                   int fn, const cpx<R>* x, cpx<R>* y, int64_t* steps) {
    if (fn < ACT_EXP || fn > ACT_PSI2) fail(MXP_ERR_INVALID_ARG, "unknown matrix function");
    const bool psi = fn == ACT_PSI1;
    const mxp_schedule& sc = sd.s;
    const int64_t n = npts(P);
    DevMem* W = act_buffers<R>(ws);
    for (int q = 0; q < 7; ++q) W[q].ensure(size_t(n) * sizeof(cpx<R>));
    cpx<R>* w[6];
    for (int q = 0; q < 6; ++q) w[q] = W[q].as<cpx<R>>();
    cpx<R>* pbuf = W[6].as<cpx<R>>();
    const StencilArgs<R> base = base_args<R>(P, shift, sd.diag);
    const bool fused = (P->g.dim == 2);
    TileCfg tc;
    if (fused) {
        TileCfg& slot = P->tiles[sizeof(R) == 4 ? 1 : 0];
        if (slot.K == 0) {
            if (em.rec) fail(MXP_ERR_HIP, "tiles must be tuned before a batched action");
            tune_tiles<R>(P, ws, sd, em.s);
        }
        tc = slot;
    }
    const int S = sc.S;
    // Scratch for one series: five buffers other than its input (four for the
    // passes, one for the output); the unfused path uses two of them.
    auto pick = [&](const cpx<R>* cur, cpx<R>** b, cpx<R>** o) {
        int k = 0;
        for (int q = 0; q < 6 && k < 5; ++q)
            if (w[q] != cur) {
                if (k < 4) b[k] = w[q]; else *o = w[q];
                ++k;
            }
    };
    auto series = [&](const double* coef, int m, const cpx<R>* xin, cpx<R>* out, cd post,
                      const cpx<R>* add) {
        cpx<R>* b[4];
        cpx<R>* spare;
        pick(xin, b, &spare);
        if (fused) {
            cheb_series_fused<R>(P, em, base, sd.diag, tc, sc, coef, m, xin, out, b, post, add, steps);
        } else if (P->g.dim == 3 && P->tiles[sizeof(R) == 4 ? 1 : 0].K == 2) {
            cheb_series3d<R>(em, base, sc, coef, m, xin, out, b, post, add, steps);
        } else {
            cheb_series<R>(em, base, sc, coef, m, xin, out, b[0], b[1], post, add, steps);
        }
    };
    auto substep_out = [&](const cpx<R>* xin) {
        cpx<R>* b[4];
        cpx<R>* spare = nullptr;
        pick(xin, b, &spare);
        return spare;
    };
    if (fn == ACT_PSI2) {
        // With tau = t/S, E = exp(i tau A_s) and F = tau psi_1(i tau A_s):
        //   t^2 psi_2(i t A_s) x = S y_1 + F (g_1 + ... + g_{S-1}),
        // y_1 = tau^2 psi_2(i tau A_s) x, g_1 = F x, g_{k+1} = E g_k + g_1
        // (split the double time integral at the substeps).  The running sum
        // G_k = g_1 + ... + g_k obeys G_{k+1} = E G_k + (k+1) g_1, so its mean
        // H_k = G_k / k obeys H_{k+1} = (k/(k+1)) E H_k + g_1: one exp series
        // with scaled coefficients per substep, and no extra vector update.
        if (sd.m_psi2 < 0) design_psi2_series(sc, sd.t, sd.prec, &sd.coef_psi2, &sd.m_psi2);
        const double it2 = 1.0 / (t * t);
        if (S == 1) {
            series(sd.coef_psi2.data(), sd.m_psi2, x, y, cd(it2, 0.0), nullptr);
            return;
        }
        W[9].ensure(size_t(n) * sizeof(cpx<R>));
        cpx<R>* y1 = W[9].as<cpx<R>>();
        series(sd.coef_psi2.data(), sd.m_psi2, x, y1, cd(1.0, 0.0), nullptr);
        series(sc.coef_psi, sc.m_psi, x, pbuf, cd(1.0, 0.0), nullptr);  // g_1 = H_1
        const cpx<R>* hk = pbuf;
        std::vector<double> scaled(2 * size_t(std::max(sc.m, sc.m_psi) + 1));
        for (int k = 1; k <= S - 2; ++k) {
            const double f = double(k) / double(k + 1);
            for (int i = 0; i < 2 * (sc.m + 1); ++i) scaled[i] = f * sc.coef[i];
            cpx<R>* out = substep_out(hk);
            series(scaled.data(), sc.m, hk, out, cd(1.0, 0.0), pbuf);
            hk = out;
        }
        // t^2 psi_2 x = S (((S-1)/S) F H_{S-1} + y_1)
        const double f = double(S - 1) / double(S);
        for (int i = 0; i < 2 * (sc.m_psi + 1); ++i) scaled[i] = f * sc.coef_psi[i];
        series(scaled.data(), sc.m_psi, hk, y, cd(double(S) * it2, 0.0), y1);
        return;
    }
    const cpx<R>* xcur = x;
    int first = 0;
    const cpx<R>* add = nullptr;
    if (psi) {
        // p = tau psi_1(i tau A_s) x; with S == 1 the answer is p / t.
        if (S == 1) {
            series(sc.coef_psi, sc.m_psi, x, y, cd(1.0 / t, 0.0), nullptr);
            return;
        }
        series(sc.coef_psi, sc.m_psi, x, pbuf, cd(1.0, 0.0), nullptr);
        xcur = pbuf;
        add = pbuf;
        first = 1;
    }
    for (int sub = first; sub < S; ++sub) {
        const bool last = (sub == S - 1);
        cpx<R>* out = last ? y : substep_out(xcur);
        const cd post = (psi && last) ? cd(1.0 / t, 0.0) : cd(1.0, 0.0);
        series(sc.coef, sc.m, xcur, out, post, add);
        xcur = out;
    }
}

// Times candidate tile configurations of the fused 2D pass on this problem's
// own buffers (HIP events on the context stream) and keeps the fastest per
// Clenshaw level.
template <typename R>
static void tune_tiles(mxp_problem* P, Workspace& ws, const Sched& sd, hipStream_t s) {
    const int64_t n = npts(P);
    DevMem* W = act_buffers<R>(ws);
    for (int q = 0; q < 7; ++q) {
        W[q].ensure(size_t(n) * sizeof(cpx<R>));
        launch_zero<R>(W[q].as<cpx<R>>(), n, s);
    }
    const StencilArgs<R> st = base_args<R>(P, 0.0, sd.diag);
    ChebPassArgs<R> a = pass_base<R>(P, st, sd.diag);
    a.x = W[0].as<cpx<R>>();
    a.in0 = W[1].as<cpx<R>>();
    a.in1 = W[2].as<cpx<R>>();
    a.outA = W[3].as<cpx<R>>();
    a.outB = W[4].as<cpx<R>>();
    for (int l = 0; l < kMaxFused; ++l) {
        a.cx[l] = {R(0.1), R(0)};
        a.g[l] = R(0.1);
    }
    a.post = R(1);
    a.e3 = R(0);
    a.final_pass = 0;
    TileCfg best;
    best.us_per_level = 1e300;
    hipEvent_t e0, e1;
    HIP_CHECK(hipEventCreate(&e0));
    HIP_CHECK(hipEventCreate(&e1));
    // short segments and single levels give small grids enough wavefronts
    const int Ks[] = {1, 2, 3, 4, 6, 8};
    // Every workgroup (4 wavefronts) is resident at once, so the compute units
    // holding one more of them than the others set the time.  Besides the
    // fixed lengths, each (K, NX) tries the segment lengths whose workgroup
    // count is just below c times the CU count, c = 1..6.
    const int Lys[] = {4, 8, 12, 16, 20, 24, 28, 32, 40, 48, 64, 96, 128};
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
        fail(MXP_ERR_HIP, "cannot query the compute-unit count");
    for (int NX = 1; NX <= 2; ++NX) {
        for (int K : Ks) {
            if (sizeof(R) == 8 && NX == 2 && K > 3) continue;  // register-limited
            const int64_t W = int64_t(NX) * 64 - 2 * K;
            const int64_t strips = (P->g.n[0] + W - 1) / W;
            std::vector<int> lys(std::begin(Lys), std::end(Lys));
            for (int c = 1; c <= 6; ++c) {
                const int64_t segs = (4 * int64_t(c) * cus) / strips;  // waves <= 4 c CUs
                if (segs < 1) continue;
                const int64_t ly = (P->g.n[1] + segs - 1) / segs;
                if (ly >= 2 && ly <= 256) lys.push_back(int(ly));
            }
            std::sort(lys.begin(), lys.end());
            lys.erase(std::unique(lys.begin(), lys.end()), lys.end());
            for (int Ly : lys) {
                // segments longer than the grid only repeat the one-segment case
                if (Ly != lys.front() && Ly / 2 >= P->g.n[1]) continue;
                cheb2d_geometry<R>(a, K, NX, Ly);
                if (a.W <= 0) continue;
                launch_cheb2d<R>(a, K, NX, s);  // warm
                HIP_CHECK(hipEventRecord(e0, s));
                const int reps = 3;
                for (int r = 0; r < reps; ++r) launch_cheb2d<R>(a, K, NX, s);
                HIP_CHECK(hipEventRecord(e1, s));
                HIP_CHECK(hipEventSynchronize(e1));
                float ms = 0;
                HIP_CHECK(hipEventElapsedTime(&ms, e0, e1));
                const double us = 1e3 * ms / (reps * K);
                if (P->ctx->verbose) {
                    std::fprintf(stderr, "[mxp] tune %s K=%d NX=%d Ly=%d: %.3f us/level\n",
                                 sizeof(R) == 4 ? "c64" : "c128", K, NX, Ly, us);
                }
                if (us < best.us_per_level) {
                    best.K = K;
                    best.NX = NX;
                    best.Ly = Ly;
                    best.us_per_level = us;
                }
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (best.K == 0) fail(MXP_ERR_HIP, "tile autotuning measured no candidate");
    P->tiles[sizeof(R) == 4 ? 1 : 0] = best;
}

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

// y = exp, psi_1 or psi_2 action (fn) on complex-double vectors, in the requested
// precision, enqueued on stream s with workspace ws, or recorded into
// rec64 / rec32 when given (the caller then launches the records and, for
// the mixed form, the cast back).  The mixed form casts at the boundary.
static void action64_on(mxp_problem* P, Workspace& ws, hipStream_t s, const Sched& sc, double t, double shift,
                        int fn, mxp_precision prec, const cpx<double>* x, cpx<double>* y, int64_t* steps,
                        std::vector<StepRec<double>>* rec64 = nullptr,
                        std::vector<StepRec<float>>* rec32 = nullptr) {
    if (prec == MXP_PREC_FP64) {
        action<double>(P, ws, Emit<double>{s, rec64}, sc, t, shift, fn, x, y, steps);
        return;
    }
    const int64_t n = npts(P);
    ws.act32[7].ensure(size_t(n) * sizeof(cpx<float>));
    ws.act32[8].ensure(size_t(n) * sizeof(cpx<float>));
    cpx<float>* xs = ws.act32[7].as<cpx<float>>();
    cpx<float>* ys = ws.act32[8].as<cpx<float>>();
    launch_to_c64(x, xs, n, s);
    action<float>(P, ws, Emit<float>{s, rec32}, sc, t, shift, fn, xs, ys, steps);
    if (!rec32) launch_to_c128(ys, y, n, s);
}

static void action64(Run& run, const Sched& sc, double t, double shift, int fn, mxp_precision prec,
                     const cpx<double>* x, cpx<double>* y, int64_t* steps);

// The same action from a captured HIP graph.  The graph reads a fixed input
// buffer and writes a fixed output buffer of the workspace (the mixed form's
// cast buffers, or two complex-double staging buffers), so one capture per
// (schedule, function, precision) serves every call: the input is staged, the
// graph replays on the workspace's stream (ordered after and before the
// caller's stream by events) and the output is copied out.  The first use of
// a key runs eagerly (it allocates the buffers and tunes the tiles), the
// second captures.  Kernels only: nothing in an action is a memset or a copy.
static void action64_graph(mxp_problem* P, Workspace& ws, hipStream_t s, const Sched& sc, double t, double shift,
                           int fn, mxp_precision prec, const cpx<double>* x, cpx<double>* y, int64_t* steps) {
    const int64_t n = npts(P);
    const bool f32 = prec != MXP_PREC_FP64;
    DevMem* in = f32 ? &ws.act32[7] : &ws.act64[7];
    DevMem* out = f32 ? &ws.act32[8] : &ws.act64[8];
    const size_t bytes = size_t(n) * (f32 ? sizeof(cpx<float>) : sizeof(cpx<double>));
    in->ensure(bytes);
    out->ensure(bytes);
    if (f32) launch_to_c64(x, in->as<cpx<float>>(), n, s);
    else launch_scale({1.0, 0.0}, x, in->as<cpx<double>>(), n, s);
    auto run_action = [&](hipStream_t st, int64_t* cnt) {
        if (f32)
            action<float>(P, ws, Emit<float>{st, nullptr}, sc, t, shift, fn, in->as<cpx<float>>(),
                          out->as<cpx<float>>(), cnt);
        else
            action<double>(P, ws, Emit<double>{st, nullptr}, sc, t, shift, fn, in->as<cpx<double>>(),
                           out->as<cpx<double>>(), cnt);
    };
    GraphEntry& ge = ws.graphs[std::make_tuple(static_cast<const void*>(&sc), fn, int(prec))];
    if (ge.uses++ == 0) {
        run_action(s, steps);
    } else {
        if (!ws.gstream) {
            HIP_CHECK(hipStreamCreateWithFlags(&ws.gstream, hipStreamNonBlocking));
            HIP_CHECK(hipEventCreateWithFlags(&ws.gev[0], hipEventDisableTiming));
            HIP_CHECK(hipEventCreateWithFlags(&ws.gev[1], hipEventDisableTiming));
        }
        HIP_CHECK(hipEventRecord(ws.gev[0], s));
        HIP_CHECK(hipStreamWaitEvent(ws.gstream, ws.gev[0], 0));
        if (!ge.exec) {
            int64_t cnt = 0;
            HIP_CHECK(hipStreamBeginCapture(ws.gstream, hipStreamCaptureModeThreadLocal));
            try {
                run_action(ws.gstream, &cnt);
            } catch (...) {
                hipGraph_t g = nullptr;
                (void)hipStreamEndCapture(ws.gstream, &g);
                if (g) (void)hipGraphDestroy(g);
                throw;
            }
            HIP_CHECK(hipStreamEndCapture(ws.gstream, &ge.graph));
            HIP_CHECK(hipGraphInstantiate(&ge.exec, ge.graph, nullptr, nullptr, 0));
            ge.steps = cnt;
        }
        HIP_CHECK(hipGraphLaunch(ge.exec, ws.gstream));
        *steps += ge.steps;
        HIP_CHECK(hipEventRecord(ws.gev[1], ws.gstream));
        HIP_CHECK(hipStreamWaitEvent(s, ws.gev[1], 0));
    }
    if (f32) launch_to_c128(out->as<cpx<float>>(), y, n, s);
    else launch_scale({1.0, 0.0}, out->as<cpx<double>>(), y, n, s);
}

// ------------------------------------------------------------ batched actions
//
// A batched solve runs every right-hand side's FGMRES in its own host thread
// and HIP stream.  Each matrix-function action a thread needs becomes a
// request; when every active thread has one pending, the requests run as one
// lockstep action: step k of every request is launched before step k + 1 of
// any, and the 3D sweeps of one step that share an operand set go out as a
// single launch over all their grids (uneven sizes included).  The 2D
// temporally blocked passes are launched per request within the same step.

struct ActionReq {
    Run* run;
    const Sched* sd;
    double t, shift;
    int fn;  // ActFn
    mxp_precision prec;
    const cpx<double>* x;
    cpx<double>* y;
    int64_t steps = 0;
    bool done = false;
    bool failed = false;
    mxp_status status = MXP_OK;
    std::string msg;
};

class Batcher {
  public:
    Batcher(int device, hipStream_t s) : device_(device), s_(s) {
        HIP_CHECK(hipEventCreateWithFlags(&done_, hipEventDisableTiming));
    }
    ~Batcher() {
        (void)hipEventDestroy(done_);
        if (host_) (void)hipHostFree(host_);
    }
    Batcher(const Batcher&) = delete;
    Batcher& operator=(const Batcher&) = delete;

    // A solve thread starts (before its first request) or ends (after its last).
    void join() {
        std::lock_guard<std::mutex> lk(mu_);
        ++active_;
    }
    void leave() {
        std::unique_lock<std::mutex> lk(mu_);
        --active_;
        maybe_run(lk);
    }
    // Blocks until the lockstep action holding r has been enqueued and has
    // finished on the device.
    void act(ActionReq& r) {
        std::unique_lock<std::mutex> lk(mu_);
        r.done = false;
        pending_.push_back(&r);
        maybe_run(lk);
        cv_.wait(lk, [&] { return r.done; });
        if (r.failed) fail(r.status, r.msg);
    }
    int64_t launches() const { return launches_; }

  private:
    void maybe_run(std::unique_lock<std::mutex>& lk) {
        while (!running_ && active_ > 0 && int(pending_.size()) >= active_) {
            std::vector<ActionReq*> batch;
            batch.swap(pending_);
            running_ = true;
            lk.unlock();
            try {
                execute(batch);
            } catch (const Error& e) {
                for (ActionReq* q : batch) {
                    q->failed = true;
                    q->status = e.status;
                    q->msg = e.what();
                }
            } catch (const std::exception& e) {
                for (ActionReq* q : batch) {
                    q->failed = true;
                    q->status = MXP_ERR_HIP;
                    q->msg = e.what();
                }
            }
            lk.lock();
            running_ = false;
            for (ActionReq* q : batch) q->done = true;
            cv_.notify_all();
        }
    }

    struct Group {  // one batched 3D launch
        int prec;   // 0 double, 1 float
        int kind;   // 0 sweeps, 2 two-level passes
        int ops;    // operand set / variant
        size_t jobs_off, lut_off;
        int64_t blocks;
    };

    // jobs of one batched launch over grids of different sizes: the job
    // array, then the lookup table with one uint32 per 64 workgroups
    template <typename Job>
    static void add_table(std::vector<unsigned char>& buf, Group& g, std::vector<Job>& jobs) {
        auto align = [&](size_t a) { buf.resize((buf.size() + a - 1) / a * a); };
        int64_t b0 = 0;
        for (auto& j : jobs) {
            j.block0 = b0;
            b0 += (j.blocks + 63) / 64 * 64;
        }
        g.blocks = b0;
        align(256);
        g.jobs_off = buf.size();
        const size_t jb = jobs.size() * sizeof(Job);
        buf.resize(buf.size() + jb);
        std::memcpy(buf.data() + g.jobs_off, jobs.data(), jb);
        align(256);
        g.lut_off = buf.size();
        std::vector<uint32_t> lut(size_t(b0 / 64));
        for (size_t q = 0; q < jobs.size(); ++q)
            for (int64_t c = jobs[q].block0 / 64; c < (jobs[q].block0 + jobs[q].blocks + 63) / 64; ++c)
                lut[size_t(c)] = uint32_t(q);
        buf.resize(buf.size() + lut.size() * sizeof(uint32_t));
        std::memcpy(buf.data() + g.lut_off, lut.data(), lut.size() * sizeof(uint32_t));
    }

    template <typename R>
    static void add_passes(std::vector<unsigned char>& buf, Group& g, const std::vector<const ChebPass3DArgs<R>*>& ps) {
        std::vector<Cheb3DJob<R>> jobs(ps.size());
        for (size_t q = 0; q < ps.size(); ++q) {
            jobs[q].a = *ps[q];
            jobs[q].blocks = int64_t(ps[q]->tiles_x) * ps[q]->tiles_y * ps[q]->zchunks;
        }
        add_table(buf, g, jobs);
    }

    template <typename R>
    static void add_jobs(std::vector<unsigned char>& buf, Group& g, const std::vector<const StencilArgs<R>*>& sw) {
        std::vector<Sweep3DJob<R>> jobs(sw.size());
        for (size_t q = 0; q < sw.size(); ++q) {
            jobs[q].a = *sw[q];
            jobs[q].geom = sweep3d_geometry(*sw[q]);
            jobs[q].blocks = int64_t(jobs[q].geom.tiles_x) * jobs[q].geom.tiles_y * jobs[q].geom.zchunks;
        }
        add_table(buf, g, jobs);
    }

    void execute(std::vector<ActionReq*>& reqs) {
        HIP_CHECK(hipSetDevice(device_));
        const size_t nq = reqs.size();
        // inputs are ready once each solve's stream reaches this point
        for (ActionReq* q : reqs) {
            HIP_CHECK(hipEventRecord(q->run->ev, q->run->s));
            HIP_CHECK(hipStreamWaitEvent(s_, q->run->ev, 0));
        }
        std::vector<std::vector<StepRec<double>>> r64(nq);
        std::vector<std::vector<StepRec<float>>> r32(nq);
        size_t L = 0;
        for (size_t i = 0; i < nq; ++i) {
            ActionReq* q = reqs[i];
            action64_on(q->run->P, *q->run->W, s_, *q->sd, q->t, q->shift, q->fn, q->prec, q->x, q->y, &q->steps,
                        &r64[i], &r32[i]);
            L = std::max(L, r64[i].size() + r32[i].size());
        }
        // plan: per step, the 3D sweeps grouped by precision and operand set
        std::vector<unsigned char> buf;
        std::vector<std::vector<Group>> plan(L);
        for (size_t k = 0; k < L; ++k) {
            std::map<int, std::vector<const StencilArgs<double>*>> g64;
            std::map<int, std::vector<const StencilArgs<float>*>> g32;
            std::map<int, std::vector<const ChebPass3DArgs<double>*>> p64;
            std::map<int, std::vector<const ChebPass3DArgs<float>*>> p32;
            for (size_t i = 0; i < nq; ++i) {
                if (k < r64[i].size() && r64[i][k].kind == 0 && r64[i][k].st.dim == 3)
                    g64[sweep_ops(r64[i][k].st)].push_back(&r64[i][k].st);
                if (k < r32[i].size() && r32[i][k].kind == 0 && r32[i][k].st.dim == 3)
                    g32[sweep_ops(r32[i][k].st)].push_back(&r32[i][k].st);
                if (k < r64[i].size() && r64[i][k].kind == 2)
                    p64[cheb3d_variant(r64[i][k].c3)].push_back(&r64[i][k].c3);
                if (k < r32[i].size() && r32[i][k].kind == 2)
                    p32[cheb3d_variant(r32[i][k].c3)].push_back(&r32[i][k].c3);
            }
            for (auto& kv : g64) {
                Group g{0, 0, kv.first, 0, 0, 0};
                add_jobs<double>(buf, g, kv.second);
                plan[k].push_back(g);
            }
            for (auto& kv : g32) {
                Group g{1, 0, kv.first, 0, 0, 0};
                add_jobs<float>(buf, g, kv.second);
                plan[k].push_back(g);
            }
            for (auto& kv : p64) {
                Group g{0, 2, kv.first, 0, 0, 0};
                add_passes<double>(buf, g, kv.second);
                plan[k].push_back(g);
            }
            for (auto& kv : p32) {
                Group g{1, 2, kv.first, 0, 0, 0};
                add_passes<float>(buf, g, kv.second);
                plan[k].push_back(g);
            }
        }
        // one upload of every job table of this action
        if (!buf.empty()) {
            if (host_bytes_ < buf.size()) {
                if (host_) HIP_CHECK(hipHostFree(host_));
                host_ = nullptr;
                host_bytes_ = 0;
                HIP_CHECK(hipHostMalloc(&host_, buf.size()));
                host_bytes_ = buf.size();
            }
            std::memcpy(host_, buf.data(), buf.size());
            table_.ensure(buf.size());
            HIP_CHECK(hipMemcpyAsync(table_.p, host_, buf.size(), hipMemcpyHostToDevice, s_));
        }
        const unsigned char* dev = table_.as<unsigned char>();
        for (size_t k = 0; k < L; ++k) {
            // launches that are not batched: 2D passes and 2D sweeps (3D
            // sweeps and 3D passes go out in the grouped launches below)
            for (size_t i = 0; i < nq; ++i) {
                if (k < r64[i].size()) {
                    const StepRec<double>& r = r64[i][k];
                    if (r.kind == 1) launch_cheb2d<double>(r.cp, r.K, r.NX, s_);
                    else if (r.kind == 0 && r.st.dim != 3) launch_stencil(r.st, s_);
                }
                if (k < r32[i].size()) {
                    const StepRec<float>& r = r32[i][k];
                    if (r.kind == 1) launch_cheb2d<float>(r.cp, r.K, r.NX, s_);
                    else if (r.kind == 0 && r.st.dim != 3) launch_stencil(r.st, s_);
                }
            }
            for (const Group& g : plan[k]) {
                const uint32_t* lut = reinterpret_cast<const uint32_t*>(dev + g.lut_off);
                if (g.kind == 2 && g.prec == 0)
                    launch_cheb3d_batch<double>(reinterpret_cast<const Cheb3DJob<double>*>(dev + g.jobs_off), lut,
                                                g.blocks, g.ops, s_);
                else if (g.kind == 2)
                    launch_cheb3d_batch<float>(reinterpret_cast<const Cheb3DJob<float>*>(dev + g.jobs_off), lut,
                                               g.blocks, g.ops, s_);
                else if (g.prec == 0)
                    launch_stencil3d_batch<double>(reinterpret_cast<const Sweep3DJob<double>*>(dev + g.jobs_off),
                                                   lut, g.blocks, g.ops, s_);
                else
                    launch_stencil3d_batch<float>(reinterpret_cast<const Sweep3DJob<float>*>(dev + g.jobs_off), lut,
                                                  g.blocks, g.ops, s_);
                ++launches_;
            }
        }
        // mixed form: cast the results back
        for (ActionReq* q : reqs)
            if (q->prec != MXP_PREC_FP64)
                launch_to_c128(q->run->W->act32[8].as<cpx<float>>(), q->y, npts(q->run->P), s_);
        HIP_CHECK(hipEventRecord(done_, s_));
        for (ActionReq* q : reqs) HIP_CHECK(hipStreamWaitEvent(q->run->s, done_, 0));
        // the staging buffer and job tables are reused by the next action
        HIP_CHECK(hipStreamSynchronize(s_));
    }

    std::mutex mu_;
    std::condition_variable cv_;
    int active_ = 0;
    bool running_ = false;
    std::vector<ActionReq*> pending_;
    int device_;
    hipStream_t s_;
    hipEvent_t done_ = nullptr;
    DevMem table_;
    void* host_ = nullptr;
    size_t host_bytes_ = 0;
    int64_t launches_ = 0;
};

static void action64(Run& run, const Sched& sc, double t, double shift, int fn, mxp_precision prec,
                     const cpx<double>* x, cpx<double>* y, int64_t* steps) {
    if (!run.batch) {
        if (run.graphs)
            action64_graph(run.P, *run.W, run.s, sc, t, shift, fn, prec, x, y, steps);
        else
            action64_on(run.P, *run.W, run.s, sc, t, shift, fn, prec, x, y, steps);
        return;
    }

    ActionReq r;
    r.run = &run;
    r.sd = &sc;
    r.t = t;
    r.shift = shift;
    r.fn = fn;
    r.prec = prec;
    r.x = x;
    r.y = y;
    run.batch->act(r);
    *steps += r.steps;
}

struct Counters {
    int64_t steps = 0, actions = 0;
    int learned = 0, fallbacks = 0;
};

// z = learned network applied to v (unit norm), complex double.
static void learned_apply(Run& run, const cpx<double>* v, double vnorm, cpx<double>* z) {
    mxp_problem* P = run.P;
    const int64_t n = npts(P);
    const ConvShape sh{1, int(P->g.n[2]), int(P->g.n[1]), int(P->g.n[0])};
    // the network sees the residual at unit root-mean-square value
    const double rs = std::sqrt(double(n)) / vnorm;
    const float* D = P->g.homogeneous ? nullptr : P->D32.as<float>();
    cnn_apply(P->net, sh, v, D, float(P->Dref), rs, P->net_scale / rs, z, run.s);
}

// Algorithm 1.  r, w: complex double device vectors.
static int precond(Run& run, const mxp_solve_opts& o, const cpx<double>* r, cpx<double>* w, Counters& cnt) {
    mxp_problem* P = run.P;
    run.graphs = o.use_graphs != 0 && !run.batch;
    Workspace& WS = *run.W;
    const int64_t n = npts(P);
    hipStream_t s = run.s;
    const Sched& sc = get_sched(P, o.t, o.shift, o.precision, o.cheb_S, o.cheb_m);
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
    action64(run, sc, o.t, o.shift, fn_rhs, o.precision, r, rhat, &cnt.steps);
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
            action64(run, sc, o.t, o.shift, fn_op, o.precision, w, d, &cnt.steps);
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
            action64(run, sc, o.t, o.shift, fn_op, o.precision, vj, tmp, &cnt.steps);
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
        action64(run, sc, o.t, o.shift, fn_op, o.precision, w, tmp, &cnt.steps);
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

static void apply_A64(mxp_problem* P, hipStream_t s, double shift, const cpx<double>* x, cpx<double>* y,
                      double g, const cpx<double>* add, double eadd) {
    StencilArgs<double> a = base_args<double>(P, shift, plain_diag(P, shift));
    a.g = {g, 0.0};
    a.b1 = x;
    a.b2 = add;
    a.e2 = {eadd, 0.0};
    a.out = y;
    launch_stencil(a, s);
}

// f(i t A_s) x with f = exp or psi_1 from one Arnoldi basis, the route the
// paper takes for its matrix functions (a Krylov method, Section 4
// introduction).  V spans the Krylov space of A_s from x (classical
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
static int krylov_action(Run& run, bool psi, double t, double shift, double tol, int max_dim,
                         const cpx<double>* x, cpx<double>* y, bool* ok) {
    const int64_t n = npts(run.P);
    hipStream_t s = run.s;
    int total = 0;
    *ok = false;
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

static void check_opts(const mxp_solve_opts* o) {
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
    if (o->use_learned && !(o->stall_ratio >= 0 && o->stall_ratio <= 1))
        fail(MXP_ERR_INVALID_ARG, "stall_ratio must be in [0, 1]");
    if (o->inner_solver < 0 || o->inner_solver > 3) fail(MXP_ERR_INVALID_ARG, "inner_solver must be 0, 1, 2 or 3");
}

static mxp_status solve(Run& run, const mxp_solve_opts& o, const cpx<double>* f, cpx<double>* u,
                        mxp_solve_stats* st) {
    const auto t0 = std::chrono::steady_clock::now();
    mxp_problem* P = run.P;
    Workspace& WS = *run.W;
    const int64_t n = npts(P);
    hipStream_t s = run.s;
    const int m = o.outer_restart;
    WS.outerV.ensure(size_t(m + 1) * n * sizeof(cpx<double>));
    WS.outerZ.ensure(size_t(m) * n * sizeof(cpx<double>));
    WS.outerR.ensure(size_t(n) * sizeof(cpx<double>));
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
    // cost-aware acceptance: mean log residual reduction and wall time of the
    // MatExPre iterations so far, wall time of the last network try
    double m_log = 0.0, m_sec = 0.0, n_sec = 0.0;
    int m_count = 0;
    auto now = [] { return std::chrono::steady_clock::now(); };
    auto secs = [](std::chrono::steady_clock::time_point a, std::chrono::steady_clock::time_point b) {
        return std::chrono::duration<double>(b - a).count();
    };
    while (bnorm > 0.0 && beta > o.rtol * bnorm) {
        ++cycles;
        launch_scale({1.0 / beta, 0.0}, r, V, n, s);
        gv.reset(beta);
        double prev_res = beta;
        // the network gets a fresh chance in every restart cycle
        bool use_net = o.use_learned != 0;
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
            // achieve on average in the time one network try takes (so it is
            // also at least as cost-effective).  Otherwise the MatExPre
            // preconditioner supplies z_j; after two misses in a row it does
            // so until the next restart cycle.  The first iteration of a
            // solve always uses MatExPre (it calibrates the threshold).
            double hn = 0.0, res = 0.0;
            bool accepted = false;
            const bool calibrated = o.stall_ratio > 0 || m_count > 0;
            if (use_net && calibrated) {
                const auto a0 = now();
                learned_apply(run, vj, 1.0, zj);
                apply_A64(P, s, 0.0, zj, vn, 1.0, nullptr, 0.0);
                hn = cgs2(run, V, n, j + 1, vn, h);
                n_sec = secs(a0, now());
                Givens trial = gv;
                res = trial.add_column(j, h, hn);
                double thr = o.stall_ratio;
                if (thr <= 0) {
                    const double per_it = m_log / m_count;                          // log reduction per iteration
                    const double rate = per_it / std::max(m_sec / m_count, 1e-9);  // ... per second
                    thr = std::min(1.0, std::min(std::exp(per_it), std::exp(rate * n_sec)));
                }
                if (std::isfinite(res) && res <= thr * prev_res) {
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
                const auto a0 = now();
                inner.push_back(precond(run, o, vj, zj, cnt));
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
                    m_sec += secs(a0, now());
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
        st->fallbacks = cnt.fallbacks;
        st->status = relres <= o.rtol ? MXP_OK : MXP_NOT_CONVERGED;
        st->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    return relres <= o.rtol ? MXP_OK : MXP_NOT_CONVERGED;
}

template <class F>
static mxp_status guard(F&& fn) {
    try {
        g_last_error.clear();
        return fn();
    } catch (const Error& e) {
        g_last_error = e.what();
        return e.status;
    } catch (const std::bad_alloc&) {
        g_last_error = "host allocation failed";
        return MXP_ERR_OOM;
    } catch (const std::exception& e) {
        g_last_error = e.what();
        return MXP_ERR_HIP;
    }
}

static void use_device(const mxp_context* ctx) { HIP_CHECK(hipSetDevice(ctx->device)); }

void context_info(const mxp_context* ctx, int* device, hipStream_t* stream) {
    *device = ctx->device;
    *stream = ctx->stream;
}

static void check_problem(const mxp_problem* P) {
    if (!P) fail(MXP_ERR_INVALID_ARG, "problem is NULL");
    use_device(P->ctx);
}

}  // namespace mxp

using namespace mxp;

extern "C" {

const char* mxp_last_error(void) { return g_last_error.c_str(); }

const char* mxp_version(void) { return "matexpre-mi355x 0.1.0 (gfx950)"; }

mxp_status mxp_context_create(int device, void* hip_stream, mxp_context** out) {
    return guard([&]() {
        if (!out) fail(MXP_ERR_INVALID_ARG, "out is NULL");
        *out = nullptr;
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
        auto* c = new mxp_context{device, static_cast<hipStream_t>(hip_stream), (v && *v && *v != '0') ? 1 : 0};
        *out = c;
        return MXP_OK;
    });
}

void mxp_context_destroy(mxp_context* ctx) { delete ctx; }

mxp_status mxp_problem_create(mxp_context* ctx, const mxp_grid_desc* desc, mxp_problem** out) {
    return guard([&]() {
        if (!ctx || !out) fail(MXP_ERR_INVALID_ARG, "context or out is NULL");
        *out = nullptr;
        GridInfo g = validate_grid(desc);
        use_device(ctx);
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
        if (!x || !y || x == y) fail(MXP_ERR_INVALID_ARG, "x and y must be distinct non-NULL pointers");
        if (!(shift >= 0) || !std::isfinite(shift)) fail(MXP_ERR_INVALID_ARG, "shift must be >= 0");
        if (dtype == MXP_C128) {
            apply_A64(prob, prob->ctx->stream, shift, static_cast<const cpx<double>*>(x),
                      static_cast<cpx<double>*>(y), 1.0, nullptr, 0.0);
        } else if (dtype == MXP_C64) {
            StencilArgs<float> a = base_args<float>(prob, shift, plain_diag(prob, shift));
            a.b1 = static_cast<const cpx<float>*>(x);
            a.out = static_cast<cpx<float>*>(y);
            launch_stencil(a, prob->ctx->stream);
        } else {
            fail(MXP_ERR_INVALID_ARG, "dtype must be MXP_C64 or MXP_C128");
        }
        HIP_CHECK(hipStreamSynchronize(prob->ctx->stream));
        return MXP_OK;
    });
}

static mxp_status apply_fn(mxp_problem* prob, double t, double shift, mxp_dtype dtype, const void* x,
                           void* y, int fn) {
    return guard([&]() {
        check_problem(prob);
        if (!x || !y || x == y) fail(MXP_ERR_INVALID_ARG, "x and y must be distinct non-NULL pointers");
        int64_t steps = 0;
        if (dtype == MXP_C128) {
            const Sched& sc = get_sched(prob, t, shift, MXP_PREC_FP64, 0, 0);
            action<double>(prob, prob->ws, Emit<double>{prob->ctx->stream, nullptr}, sc, t, shift, fn,
                           static_cast<const cpx<double>*>(x), static_cast<cpx<double>*>(y), &steps);
        } else if (dtype == MXP_C64) {
            const Sched& sc = get_sched(prob, t, shift, MXP_PREC_MIXED, 0, 0);
            action<float>(prob, prob->ws, Emit<float>{prob->ctx->stream, nullptr}, sc, t, shift, fn,
                          static_cast<const cpx<float>*>(x), static_cast<cpx<float>*>(y), &steps);
        } else {
            fail(MXP_ERR_INVALID_ARG, "dtype must be MXP_C64 or MXP_C128");
        }
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

mxp_status mxp_apply_precond(mxp_problem* prob, const mxp_solve_opts* opts, const void* r, void* w,
                             int32_t* inner_its) {
    return guard([&]() {
        check_problem(prob);
        check_opts(opts);
        if (!r || !w || r == w) fail(MXP_ERR_INVALID_ARG, "r and w must be distinct non-NULL pointers");
        Counters cnt;
        Run run{prob, &prob->ws, prob->ctx->stream, nullptr, nullptr};
        const int its = precond(run, *opts, static_cast<const cpx<double>*>(r), static_cast<cpx<double>*>(w), cnt);
        HIP_CHECK(hipStreamSynchronize(prob->ctx->stream));
        if (inner_its) *inner_its = its;
        return MXP_OK;
    });
}

mxp_status mxp_set_tiles(mxp_problem* prob, mxp_precision precision, int32_t K, int32_t NX, int32_t Ly) {
    return guard([&]() {
        if (!prob) fail(MXP_ERR_INVALID_ARG, "problem is NULL");
        if (precision != MXP_PREC_FP64 && precision != MXP_PREC_MIXED) fail(MXP_ERR_INVALID_ARG, "unknown precision");
        if (K < 0 || K > kMaxFused || (NX != 1 && NX != 2) || Ly < 1 || (K > 0 && NX * 64 - 2 * K <= 0))
            fail(MXP_ERR_INVALID_ARG, "tiles: K in 0..8, NX in {1, 2}, Ly >= 1");
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

mxp_status mxp_solve(mxp_problem* prob, const mxp_solve_opts* opts, const void* f, void* u,
                     mxp_solve_stats* stats) {
    return guard([&]() {
        check_problem(prob);
        check_opts(opts);
        if (!f || !u || f == u) fail(MXP_ERR_INVALID_ARG, "f and u must be distinct non-NULL pointers");
        Run run{prob, &prob->ws, prob->ctx->stream, nullptr, nullptr};
        return solve(run, *opts, static_cast<const cpx<double>*>(f), static_cast<cpx<double>*>(u), stats);
    });
}

mxp_status mxp_solve_batch(mxp_context* ctx, int32_t nprob, mxp_problem* const* problems, const int32_t* nrhs,
                           const void* const* f, void* const* u, const mxp_solve_opts* opts, int32_t max_resident,
                           mxp_solve_stats* stats) {
    return guard([&]() -> mxp_status {
        if (!ctx || nprob < 1 || !problems || !nrhs || !f || !u || !opts)
            fail(MXP_ERR_INVALID_ARG, "batch: context, problem, rhs and option arrays must be given");
        if (max_resident < 0) fail(MXP_ERR_INVALID_ARG, "max_resident must be >= 0");
        use_device(ctx);
        struct Item {
            mxp_problem* P;
            const mxp_solve_opts* o;
            const cpx<double>* f;
            cpx<double>* u;
            size_t bytes;
        };
        std::vector<Item> items;
        for (int q = 0; q < nprob; ++q) {
            mxp_problem* P = problems[q];
            if (!P) fail(MXP_ERR_INVALID_ARG, "batch: problem is NULL");
            if (P->ctx->device != ctx->device) fail(MXP_ERR_INVALID_ARG, "batch: problem on another device");
            check_opts(&opts[q]);
            if (opts[q].use_learned) fail(MXP_ERR_UNSUPPORTED, "batch: the learned stage runs in single solves only");
            if (nrhs[q] < 0) fail(MXP_ERR_INVALID_ARG, "batch: nrhs must be >= 0");
            if (nrhs[q] == 0) continue;
            if (!f[q] || !u[q] || f[q] == u[q]) fail(MXP_ERR_INVALID_ARG, "batch: f and u must be distinct non-NULL");
            const mxp_solve_opts& o = opts[q];
            const int64_t n = npts(P);
            // everything the right-hand side's solve allocates (workspace estimate)
            const size_t vec = size_t(n) * sizeof(cpx<double>);
            size_t bytes = vec * (size_t(2 * o.outer_restart + 2) + size_t(o.inner_restart + 4));
            bytes += o.precision == MXP_PREC_FP64 ? 7 * vec : 9 * vec / 2;
            if (o.inner_solver >= 2) bytes += o.precision == MXP_PREC_FP64 ? vec : vec / 2;  // psi_2's y_1
            bytes += size_t(reduce_blocks(n)) * 256 * sizeof(cpx<double>) + (1 << 20);
            // set up once, outside the threads: schedules, diagonal tables and
            // 2D tiles are shared read-only by every right-hand side of P
            const Sched& sd = get_sched(P, o.t, o.shift, o.precision, o.cheb_S, o.cheb_m);
            if (o.inner_solver >= 2 && sd.m_psi2 < 0)
                design_psi2_series(sd.s, sd.t, sd.prec, &sd.coef_psi2, &sd.m_psi2);
            (void)plain_diag(P, 0.0);
            if (P->g.dim == 2) {
                if (o.precision == MXP_PREC_FP64 && P->tiles[0].K == 0)
                    tune_tiles<double>(P, P->ws, sd, P->ctx->stream);
                if (o.precision == MXP_PREC_MIXED && P->tiles[1].K == 0)
                    tune_tiles<float>(P, P->ws, sd, P->ctx->stream);
            }
            for (int r = 0; r < nrhs[q]; ++r)
                items.push_back({P, &o, static_cast<const cpx<double>*>(f[q]) + size_t(r) * n,
                                 static_cast<cpx<double>*>(u[q]) + size_t(r) * n, bytes});
        }
        HIP_CHECK(hipStreamSynchronize(ctx->stream));
        size_t free_b = 0, total_b = 0;
        HIP_CHECK(hipMemGetInfo(&free_b, &total_b));
        const size_t budget = free_b > (size_t(2) << 30) ? free_b - (size_t(2) << 30) : free_b / 2;
        const int cap = max_resident > 0 ? max_resident : int(items.size());

        Batcher B(ctx->device, ctx->stream);
        std::mutex mu;
        std::condition_variable cv;
        int running = 0;
        size_t running_bytes = 0;
        std::vector<mxp_status> status(items.size(), MXP_OK);
        std::vector<std::string> msgs(items.size());
        std::vector<std::thread> threads;
        const int dev = ctx->device;
        for (size_t k = 0; k < items.size(); ++k) {
            {
                std::unique_lock<std::mutex> lk(mu);
                cv.wait(lk, [&] {
                    return running == 0 || (running < cap && running_bytes + items[k].bytes <= budget);
                });
                ++running;
                running_bytes += items[k].bytes;
            }
            B.join();
            threads.emplace_back([&, k, dev]() {
                const Item& it = items[k];
                try {
                    HIP_CHECK(hipSetDevice(dev));
                    Workspace W;
                    hipStream_t s = nullptr;
                    hipEvent_t ev = nullptr;
                    HIP_CHECK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
                    if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
                        (void)hipStreamDestroy(s);
                        fail(MXP_ERR_HIP, "event creation failed");
                    }
                    Run run{it.P, &W, s, &B, ev};
                    try {
                        status[k] = solve(run, *it.o, it.f, it.u, stats ? &stats[k] : nullptr);
                    } catch (...) {
                        (void)hipStreamSynchronize(s);
                        (void)hipEventDestroy(ev);
                        (void)hipStreamDestroy(s);
                        throw;
                    }
                    (void)hipEventDestroy(ev);
                    (void)hipStreamDestroy(s);
                } catch (const Error& e) {
                    status[k] = e.status;
                    msgs[k] = e.what();
                } catch (const std::exception& e) {
                    status[k] = MXP_ERR_HIP;
                    msgs[k] = e.what();
                }
                if (stats && status[k] < 0) stats[k].status = status[k];
                B.leave();
                {
                    std::lock_guard<std::mutex> lk(mu);
                    --running;
                    running_bytes -= it.bytes;
                }
                cv.notify_all();
            });
        }
        for (auto& th : threads) th.join();
        mxp_status worst = MXP_OK;
        for (size_t k = 0; k < items.size(); ++k) {
            if (status[k] < 0) fail(status[k], "batch right-hand side " + std::to_string(k) + ": " + msgs[k]);
            if (status[k] == MXP_NOT_CONVERGED) worst = MXP_NOT_CONVERGED;
        }
        return worst;
    });
}

mxp_status mxp_problem_set_learned(mxp_problem* prob, mxp_cnn* net, double out_scale) {
    return guard([&]() {
        check_problem(prob);
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
