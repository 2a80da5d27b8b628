// Internal state of contexts and problems, and the functions that the
// library's translation units share (not part of the C ABI):
//   action.cpp  set-up tables, schedules and the matrix-function actions
//   krylov.cpp  Algorithm 1 (inner GMRES), the outer flexible GMRES and the
//               Arnoldi route to the matrix functions
//   batch.cpp   batched solves (lockstep actions over many right-hand sides)
//   api.cpp     the C ABI entry points
#pragma once

#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <complex>
#include <map>
#include <memory>
#include <string>
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
    int verbose;           // MXP_VERBOSE=1: one line per outer iteration on stderr
    mxp::Allocator alloc;  // device memory of the context's problems and networks
};

namespace mxp {

extern thread_local std::string g_last_error;

template <typename R>
struct DevTables {
    cpx<R>* alpha[3] = {nullptr, nullptr, nullptr};
    cpx<R>* beta[3] = {nullptr, nullptr, nullptr};
    cpx<R>* gamma[3] = {nullptr, nullptr, nullptr};
    // first-order absorbing faces with a varying speed: per-axis weights
    // 2 omega/h at absorbing end nodes, and the same times h^2 (2D passes)
    R* abc[3] = {nullptr, nullptr, nullptr};
    R* abc_h2[3] = {nullptr, nullptr, nullptr};
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
    DevMem io[2];  // complex-double copies of complex-float arguments
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
    mxp::DevMem tables64, tables32, D64, D32, abc64, abc32;
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

inline int64_t npts(const mxp_problem* P) { return P->g.npts(); }

struct Counters {
    int64_t steps = 0, actions = 0;
    int learned = 0, fallbacks = 0;
    int fp64_its = 0;  // mixed form: outer iterations whose actions ran in double
};

template <typename R>
inline cpx<R> to_cpx(cd v) { return {R(v.real()), R(v.imag())}; }

// Where the launches of a matrix-function action go: straight onto a stream,
// or into a list that a batched solve replays in lockstep with other actions.
template <typename R>
struct StepRec {
    int kind;  // 0: stencil sweep (st); 1: temporally blocked 2D pass (cp, K, NX); 2 / 3: two- / three-level 3D pass (c3)
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
    void pass3d3(const ChebPass3DArgs<R>& a) const {
        if (rec) {
            StepRec<R> r{};
            r.kind = 3;
            r.c3 = a;
            rec->push_back(r);
        } else {
            launch_cheb3d3<R>(a, s);
        }
    }
};

// out = post * (sum_{k<=m} c_k T_k(Ahat) x + add), Ahat = (A_s - centre)/hw,
// by the Clenshaw recurrence b_k = c_k x + 2 Ahat b_{k+1} - b_{k+2}.

// ---------------------------------------------------------------- action.cpp

// Diagonal tables of A_s itself (segment centre 0) for one shift.
const DiagTables& plain_diag(mxp_problem* P, double shift);
// The schedule of (t, shift, precision, forced S / m), designed at first use.
const Sched& get_sched(mxp_problem* P, double t, double shift, mxp_precision prec, int forceS, int forcem);
// Tunes the 2D pass tiles of the schedule's precision if they are not set.
void ensure_tiles(mxp_problem* P, Workspace& ws, const Sched& sd, hipStream_t s);
// y = A_s x in the precision of dtype.
void apply_A(mxp_problem* P, hipStream_t s, double shift, mxp_dtype dtype, const void* x, void* y);
// y = g A_s x + eadd add in complex double (add may be nullptr).
void apply_A64(mxp_problem* P, hipStream_t s, double shift, const cpx<double>* x, cpx<double>* y, double g,
               const cpx<double>* add, double eadd);
// y = f(i t A_s) x (f by ActFn) on vectors of dtype, in that precision.
void apply_action(mxp_problem* P, Workspace& ws, hipStream_t s, const Sched& sd, double t, double shift, int fn,
                  mxp_dtype dtype, const void* x, void* y, int64_t* steps);
// exp(i t A_s) x on caller-provided buffers: six device vectors of n values of
// dtype (none of them x or y) and the 2D pass tiles tc (K > 0).
void apply_action_on(mxp_problem* P, void* const bufs[6], const TileCfg& tc, hipStream_t s, const Sched& sd,
                     double t, double shift, mxp_dtype dtype, const void* x, void* y, int64_t* steps);
// Bytes of the diagonal tables of one schedule, and building them into buffers
// the tables own (ext == nullptr) or into the caller's device region ext.
size_t diag_table_bytes(const GridInfo& g);
void build_diag(mxp_problem* P, double shift, cd centre, DiagTables& dt, void* ext, hipStream_t s);
void action64_on(mxp_problem* P, Workspace& ws, hipStream_t s, const Sched& sc, double t, double shift, int fn,
                 mxp_precision prec, const cpx<double>* x, cpx<double>* y, int64_t* steps,
                 std::vector<StepRec<double>>* rec64 = nullptr, std::vector<StepRec<float>>* rec32 = nullptr);
void action64_graph(mxp_problem* P, Workspace& ws, hipStream_t s, const Sched& sc, double t, double shift, int fn,
                    mxp_precision prec, const cpx<double>* x, cpx<double>* y, int64_t* steps);

// ----------------------------------------------------------------- batch.cpp

// The action of a solve: direct, from a captured graph, or through its batcher.
void action64(Run& run, const Sched& sc, double t, double shift, int fn, mxp_precision prec,
              const cpx<double>* x, cpx<double>* y, int64_t* steps);

// ---------------------------------------------------------------- krylov.cpp

void check_opts(const mxp_solve_opts* o);
// Everything an action, a preconditioner apply or a solve with these options
// allocates, taken at the entry of the call; afterwards the thread is marked
// reserved, and a later allocation counts as late in the context's statistics.
void reserve_action(mxp_problem* P, Workspace& ws, const Sched& sd, bool psi2, bool graphs, hipStream_t s);
void reserve_precond(Run& run, const mxp_solve_opts& o);
void reserve_solve(Run& run, const mxp_solve_opts& o);
// Algorithm 1 with the matrix-function actions in precision ap.
int precond(Run& run, const mxp_solve_opts& o, const cpx<double>* r, cpx<double>* w, Counters& cnt,
            mxp_precision ap);
int krylov_action(Run& run, bool psi, double t, double shift, double tol, int max_dim, const cpx<double>* x,
                  cpx<double>* y, bool* ok);
mxp_status solve(Run& run, const mxp_solve_opts& o, const cpx<double>* f, cpx<double>* u, mxp_solve_stats* st);

// ------------------------------------------------------------------- api.cpp

template <class F>
inline mxp_status guard(F&& fn) {
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

// A roctx range for the lifetime of a scope (shown by rocprofv3 --marker-trace;
// per host thread, so the ranges of a batched solve's threads nest on their own).
struct Range {
    explicit Range(const char* name) { roctxRangePushA(name); }
    ~Range() { roctxRangePop(); }
    Range(const Range&) = delete;
    Range& operator=(const Range&) = delete;
};

inline void use_device(const mxp_context* ctx) { HIP_CHECK(hipSetDevice(ctx->device)); }

inline void check_problem(const mxp_problem* P) {
    if (!P) fail(MXP_ERR_INVALID_ARG, "problem is NULL");
    use_device(P->ctx);
}

}  // namespace mxp
