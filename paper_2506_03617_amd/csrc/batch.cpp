// Batched solves: many right-hand sides of one or more problems, each with
// its own flexible GMRES (Section 3.4), whose matrix-function actions run in
// lockstep so that the 3D stencil sweeps of one step go out as one launch
// over all grids.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <condition_variable>
#include <cstring>
#include <map>
#include <mutex>
#include <thread>

#include "engine.h"

namespace mxp {

// ------------------------------------------------------------ batched actions
//
// A batched solve runs every right-hand side's FGMRES in its own host thread
// and HIP stream.  Each matrix-function action a thread needs becomes a
// request; when every active thread has one pending, the requests run as one
// lockstep action: step k of every request is launched before step k + 1 of
// any.  The 3D sweeps of one step that share an operand set go out as a
// single launch over all their grids (uneven sizes included), and so do the
// 3D two- and three-level passes and the 2D temporally blocked passes of one
// step that share a shape.  The batched sweep, two-level and 2D kernels are
// persistent (resident workgroups striding over every grid's tiles); the
// three-level pass runs one workgroup per tile.

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
    // Device room for the job tables of one lockstep action, taken before
    // the solves start (a larger action grows it, counted as late).
    void reserve(size_t bytes) { table_.ensure(bytes); }

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

    struct Group {  // one batched launch
        int prec;   // 0 double, 1 float
        int kind;   // 0 3D sweeps, 1 2D passes, 2 / 3 3D two- / three-level passes
        int ops;    // operand set / variant; 2D passes: K * 4 + NX
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
    static void add_passes2d(std::vector<unsigned char>& buf, Group& g, const std::vector<const StepRec<R>*>& ps) {
        std::vector<Cheb2DJob<R>> jobs(ps.size());
        for (size_t q = 0; q < ps.size(); ++q) {
            jobs[q].a = prepare_cheb2d(ps[q]->cp, ps[q]->K, ps[q]->NX);
            jobs[q].blocks = cheb2d_blocks(jobs[q].a);
        }
        add_table(buf, g, jobs);
    }

    template <typename R>
    static void add_jobs(std::vector<unsigned char>& buf, Group& g, const std::vector<const StencilArgs<R>*>& sw) {
        std::vector<Sweep3DJob<R>> jobs(sw.size());
        for (size_t q = 0; q < sw.size(); ++q) {
            jobs[q].a = *sw[q];
            jobs[q].geom = sweep3d_geometry(*sw[q]);
            jobs[q].blocks = jobs[q].geom.blocks;
        }
        add_table(buf, g, jobs);
    }

    void execute(std::vector<ActionReq*>& reqs) {
        Range range("batched lockstep action");
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
            std::map<int, std::vector<const StepRec<double>*>> f64;
            std::map<int, std::vector<const StepRec<float>*>> f32;
            std::map<int, std::vector<const ChebPass3DArgs<double>*>> t64;
            std::map<int, std::vector<const ChebPass3DArgs<float>*>> t32;
            for (size_t i = 0; i < nq; ++i) {
                if (k < r64[i].size() && r64[i][k].kind == 3)
                    t64[cheb3d_variant(r64[i][k].c3)].push_back(&r64[i][k].c3);
                if (k < r32[i].size() && r32[i][k].kind == 3)
                    t32[cheb3d_variant(r32[i][k].c3)].push_back(&r32[i][k].c3);
                if (k < r64[i].size() && r64[i][k].kind == 1)
                    f64[r64[i][k].K * 4 + r64[i][k].NX].push_back(&r64[i][k]);
                if (k < r32[i].size() && r32[i][k].kind == 1)
                    f32[r32[i][k].K * 4 + r32[i][k].NX].push_back(&r32[i][k]);
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
            for (auto& kv : f64) {
                Group g{0, 1, kv.first, 0, 0, 0};
                add_passes2d<double>(buf, g, kv.second);
                plan[k].push_back(g);
            }
            for (auto& kv : f32) {
                Group g{1, 1, kv.first, 0, 0, 0};
                add_passes2d<float>(buf, g, kv.second);
                plan[k].push_back(g);
            }
            for (auto& kv : t64) {
                Group g{0, 3, kv.first, 0, 0, 0};
                add_passes<double>(buf, g, kv.second);
                plan[k].push_back(g);
            }
            for (auto& kv : t32) {
                Group g{1, 3, kv.first, 0, 0, 0};
                add_passes<float>(buf, g, kv.second);
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
            // launches that are not batched: 2D sweeps (the unfused path;
            // every other step goes out in the grouped launches below)
            for (size_t i = 0; i < nq; ++i) {
                if (k < r64[i].size() && r64[i][k].kind == 0 && r64[i][k].st.dim != 3)
                    launch_stencil(r64[i][k].st, s_);
                if (k < r32[i].size() && r32[i][k].kind == 0 && r32[i][k].st.dim != 3)
                    launch_stencil(r32[i][k].st, s_);
            }
            for (const Group& g : plan[k]) {
                const uint32_t* lut = reinterpret_cast<const uint32_t*>(dev + g.lut_off);
                if (g.kind == 1 && g.prec == 0)
                    launch_cheb2d_batch<double>(reinterpret_cast<const Cheb2DJob<double>*>(dev + g.jobs_off), lut,
                                                g.blocks, g.ops / 4, g.ops % 4, s_);
                else if (g.kind == 1)
                    launch_cheb2d_batch<float>(reinterpret_cast<const Cheb2DJob<float>*>(dev + g.jobs_off), lut,
                                               g.blocks, g.ops / 4, g.ops % 4, s_);
                else if (g.kind == 3 && g.prec == 0)
                    launch_cheb3d3_batch<double>(reinterpret_cast<const Cheb3DJob<double>*>(dev + g.jobs_off), lut,
                                                 g.blocks, g.ops, s_);
                else if (g.kind == 3)
                    launch_cheb3d3_batch<float>(reinterpret_cast<const Cheb3DJob<float>*>(dev + g.jobs_off), lut,
                                                g.blocks, g.ops, s_);
                else if (g.kind == 2 && g.prec == 0)
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

void action64(Run& run, const Sched& sc, double t, double shift, int fn, mxp_precision prec,
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

}  // namespace mxp

using namespace mxp;

extern "C" {

mxp_status mxp_solve_batch(mxp_context* ctx, int32_t nprob, mxp_problem* const* problems, const int32_t* nrhs,
                           const void* const* f, void* const* u, const mxp_solve_opts* opts, int32_t max_resident,
                           mxp_solve_stats* stats) {
    return guard([&]() -> mxp_status {
        Range range("mxp solve batch");
        if (!ctx || nprob < 1 || !problems || !nrhs || !f || !u || !opts)
            fail(MXP_ERR_INVALID_ARG, "batch: context, problem, rhs and option arrays must be given");
        if (max_resident < 0) fail(MXP_ERR_INVALID_ARG, "max_resident must be >= 0");
        use_device(ctx);
        AllocScope scope(ctx->alloc);
        struct Item {
            mxp_problem* P;
            const mxp_solve_opts* o;
            const cpx<double>* f;
            cpx<double>* u;
            size_t bytes;
        };
        std::vector<Item> items;
        size_t table_steps = 0, table_per_rhs = 0;
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
            const bool switches = o.precision == MXP_PREC_MIXED && (o.fp64_below > 0 || o.fp64_first > 0);
            if (switches) bytes += (o.inner_solver >= 2 ? 8 : 7) * vec;  // the double actions' buffers
            bytes += size_t(reduce_blocks(n)) * 256 * sizeof(cpx<double>) + (1 << 20);
            // set up once, outside the threads: schedules, diagonal tables and
            // 2D tiles are shared read-only by every right-hand side of P
            const Sched& sd = get_sched(P, o.t, o.shift, o.precision, o.cheb_S, o.cheb_m);
            if (o.inner_solver >= 2 && sd.m_psi2 < 0)
                design_psi2_series(sd.s, sd.t, sd.prec, &sd.coef_psi2, &sd.m_psi2);
            (void)plain_diag(P, 0.0);
            ensure_tiles(P, P->ws, sd, P->ctx->stream);
            if (switches) {  // the double schedule the late outer iterations switch to
                const Sched& s64 = get_sched(P, o.t, o.shift, MXP_PREC_FP64, o.cheb_S, o.cheb_m);
                if (o.inner_solver >= 2 && s64.m_psi2 < 0)
                    design_psi2_series(s64.s, s64.t, s64.prec, &s64.coef_psi2, &s64.m_psi2);
                ensure_tiles(P, P->ws, s64, P->ctx->stream);
            }
            for (int r = 0; r < nrhs[q]; ++r)
                items.push_back({P, &o, static_cast<const cpx<double>*>(f[q]) + size_t(r) * n,
                                 static_cast<cpx<double>*>(u[q]) + size_t(r) * n, bytes});
            // steps of one action: the longest schedule the solve may use
            auto action_steps = [](const Sched& x) {
                const int mmax = std::max(std::max(x.s.m, x.s.m_psi), std::max(x.m_psi2, 0));
                return size_t(x.s.S + 2) * size_t(mmax + 1);
            };
            size_t steps = action_steps(sd);
            if (switches) steps = std::max(steps, action_steps(get_sched(P, o.t, o.shift, MXP_PREC_FP64, o.cheb_S, o.cheb_m)));
            if (P->g.dim == 3) {
                // job-table bytes per right-hand side and step: the job, two
                // alignments and one lookup entry per 64 workgroups (tiles no
                // smaller than 62 x 4 nodes, z segments of at least 8 planes)
                const int64_t blocks = ((P->g.n[0] + 61) / 62) * ((P->g.n[1] + 3) / 4) * ((P->g.n[2] + 7) / 8);
                const size_t per = sizeof(Cheb3DJob<double>) + sizeof(Sweep3DJob<double>) + 1024 +
                                   4 * size_t(blocks / 64 + 1);
                table_steps = std::max(table_steps, steps);
                table_per_rhs = std::max(table_per_rhs, per);
            } else {
                // 2D: one pass job per right-hand side and step (strips at
                // least 48 columns wide, segments of at least one row)
                const int64_t blocks = ((P->g.n[0] + 47) / 48) * P->g.n[1] / 4 + 1;
                const size_t per = sizeof(Cheb2DJob<double>) + 1024 + 4 * size_t(blocks / 64 + 1);
                table_steps = std::max(table_steps, steps);
                table_per_rhs = std::max(table_per_rhs, per);
            }
        }
        HIP_CHECK(hipStreamSynchronize(ctx->stream));
        size_t free_b = 0, total_b = 0;
        HIP_CHECK(hipMemGetInfo(&free_b, &total_b));
        const size_t budget = free_b > (size_t(2) << 30) ? free_b - (size_t(2) << 30) : free_b / 2;
        const int cap = max_resident > 0 ? max_resident : int(items.size());

        Batcher B(ctx->device, ctx->stream);
        if (table_steps > 0) {
            const size_t resident = std::min(size_t(cap), items.size());
            B.reserve(std::min(table_steps * table_per_rhs * resident, size_t(64) << 20));
        }
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
                    AllocScope thread_scope(ctx->alloc);
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

}  // extern "C"
