// Serving: continuous batching of independent Poisson solves on one device.
//
// A request queue in arrival order feeds a fixed pool of worker threads (the
// slots).  Each worker owns one non-blocking HIP stream and one pinned host
// buffer, and runs a whole request on that stream: setup of the handle (its
// level hierarchy and Krylov basis stay resident for the request's lifetime),
// the caller's data or manufactured data, the FGMRES solve, the error against
// the closed-form solution (manufactured data), and stream-ordered teardown.
// Requests on different slots therefore overlap on the device.  Admission is
// FIFO against a byte budget: the head of the queue starts only when a slot is
// free and its estimated peak device bytes fit in what running requests leave
// of the budget.
//
// Cross-request batching: the tail of every V-cycle (the small coarse levels
// and the coarse solve, one workgroup's work) goes through a batcher.  The
// tails of the requests that reach them together (the first to arrive waits at
// most a short window for the others) run as one launch per precision and
// dimension, one workgroup per request, on the first request's stream, ordered
// after each member's finer levels (an event per member) and before each
// member's prolongation (one event per batch).  A workgroup runs exactly the
// request's own tail, so results do not depend on the batch.
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>

#include "core.h"

namespace iim {

struct Job {
    iim_request req{};
    std::vector<double> params;
    iim_result res{};
};

// one V-cycle tail waiting for (or taken by) a batch
struct TailJob {
    Problem* p = nullptr;
    hipEvent_t ready = nullptr;  // the member's: recorded on p's stream after the levels above the tail
    hipEvent_t done = nullptr;   // the member's: recorded on the leader's stream after the batch
    bool launched = false;
    int error = 0;
};

// Batches the V-cycle tails of the requests that reach them together.  The
// first worker to arrive at an open batch leads it: it waits (at most the
// window) until every solving worker has joined or the window has passed,
// closes the batch, makes its own stream wait for the other members' finer
// levels, launches the batch there and records one event that the members'
// streams wait for.  No thread other than the workers is involved.
struct TailBatcher final : TailRunner {
    int window_us = 0;
    std::mutex mu;
    std::condition_variable cv;
    std::vector<TailJob*> open;  // members of the batch being gathered
    bool leader_waiting = false;
    int solving = 0;  // workers inside a solve: the ones whose tails may join a batch
    int64_t batches = 0, jobs = 0;

    explicit TailBatcher(int window) : window_us(window) {}
    void enter() {
        std::lock_guard<std::mutex> lk(mu);
        ++solving;
    }
    void leave() {
        {
            std::lock_guard<std::mutex> lk(mu);
            --solving;
        }
        cv.notify_all();  // a leader waiting for this worker's tail need not wait longer
    }
    void run(Problem& p) override;
    static void launch(const std::vector<TailJob*>& batch, hipStream_t s);
};

struct Server {
    int device = 0;
    int64_t budget = 0;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Job*> queue;
    std::unordered_map<uint64_t, std::unique_ptr<Job>> jobs;
    uint64_t next_ticket = 1;
    int64_t reserved = 0, peak = 0, submitted = 0, completed = 0, failed = 0, running = 0;
    bool stopping = false;
    std::vector<std::thread> workers;
    std::unique_ptr<TailBatcher> engine;  // null: every request launches its own tails
    std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();

    double clock() const {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    void worker();
    void run(Job& j, hipStream_t s, double* hpin);
};

// the calling worker's events: its finer levels done, its tail's batch done
// (each is recorded and waited for only while the worker takes part in one
// batch, so no other batch can record it meanwhile)
struct MemberEvents {
    hipEvent_t ready = nullptr, done = nullptr;
    ~MemberEvents() {
        if (ready) (void)hipEventDestroy(ready);
        if (done) (void)hipEventDestroy(done);
    }
};

void TailBatcher::run(Problem& p) {
    thread_local MemberEvents tl;
    if (!tl.ready) IIM_HIP(hipEventCreateWithFlags(&tl.ready, hipEventDisableTiming));
    if (!tl.done) IIM_HIP(hipEventCreateWithFlags(&tl.done, hipEventDisableTiming));
    TailJob job;
    job.p = &p;
    job.ready = tl.ready;
    job.done = tl.done;
    std::unique_lock<std::mutex> lk(mu);
    const bool lead = open.empty();
    if (!lead) IIM_HIP(hipEventRecord(job.ready, p.stream));  // the leader orders its own stream
    open.push_back(&job);
    if (!lead) {
        cv.notify_all();
        cv.wait(lk, [&] { return job.launched; });
        lk.unlock();
        if (job.error) throw Error(job.error, "batched coarse-level launch failed");
        IIM_HIP(hipStreamWaitEvent(p.stream, job.done, 0));
        return;
    }
    // lead: gather the tails of the other solving workers for at most the window
    if (window_us > 0) {
        const auto deadline = std::chrono::steady_clock::now() + std::chrono::microseconds(window_us);
        cv.wait_until(lk, deadline, [&] { return (int)open.size() >= solving; });
    }
    std::vector<TailJob*> batch;
    batch.swap(open);  // later arrivals open the next batch
    ++batches;
    jobs += (int64_t)batch.size();
    lk.unlock();
    int err = 0;
    try {
        launch(batch, p.stream);
        for (TailJob* j : batch)
            if (j != &job) IIM_HIP(hipEventRecord(j->done, p.stream));
    } catch (const Error& e) {
        err = e.code;
    } catch (...) {
        err = IIM_E_INTERNAL;
    }
    lk.lock();
    for (TailJob* j : batch) {
        j->error = err;
        j->launched = true;
    }
    lk.unlock();
    cv.notify_all();
    if (err) throw Error(err, "batched coarse-level launch failed");
}

// one launch per (precision, dimension) group, at most TAIL_BATCH_MAX tails
// each, on stream s after every member's finer levels
void TailBatcher::launch(const std::vector<TailJob*>& batch, hipStream_t s) {
    for (int prec = 0; prec <= 2; ++prec)
        for (int dim = 2; dim <= 3; ++dim) {
            TailBatch B{};
            auto flush = [&] {
                if (!B.count) return;
                if (prec == IIM_PREC_FP64) run_tail_batch<double, double>(dim, B, s);
                else if (prec == IIM_PREC_MIXED32) run_tail_batch<float, float>(dim, B, s);
                else run_tail_batch<float, __half>(dim, B, s);
                B.count = 0;
            };
            for (TailJob* j : batch) {
                if (j->p->opt.precision != prec || j->p->dim != dim) continue;
                if (j->p->stream != s) IIM_HIP(hipStreamWaitEvent(s, j->ready, 0));
                B.d[B.count] = j->p->d_tail;
                B.lds[B.count] = j->p->tail_lds_bytes;
                if (++B.count == TAIL_BATCH_MAX) flush();
            }
            flush();
        }
}

void Server::run(Job& j, hipStream_t s, double* hpin) {
    iim_result& r = j.res;
    try {
        auto p = make_problem(&j.req.grid, &j.req.geom, &j.req.opt, s, hpin);
        r.n_unknowns = p->levels[0].nunk;
        if (j.req.data_kind == 0) {
            // the caller's problem: data per control point, box faces and f
            const int64_t ncd = p->cp.ncp * (p->bc == IIM_BC_JUMP ? 2 : 1);
            if (j.req.n_cp_data != ncd)
                throw Error(IIM_E_INVALID_ARG, "n_cp_data is " + std::to_string(j.req.n_cp_data) +
                                                   ", the problem's control points need " + std::to_string(ncd));
            p->set_boundary_data(j.req.cp_data, j.req.box_data, j.req.mem_kind);
            p->set_rhs(j.req.f, j.req.mem_kind);
        } else {
            p->synth_data(j.req.data_kind);
        }
        const int64_t n1 = j.req.grid.n + 1;
        const int64_t tot = j.req.grid.dim == 2 ? n1 * n1 : n1 * n1 * n1;
        double* u = j.req.u_out ? j.req.u_out : (double*)p->mem.alloc(tot * sizeof(double));
        iim_stats st{};
        if (engine) {
            p->tail_runner = engine.get();
            engine->enter();
        }
        int status;
        try {
            status = p->solve(u, nullptr, j.req.hist, j.req.hist_cap, &st);
        } catch (...) {
            if (engine) engine->leave();
            p->tail_runner = nullptr;
            throw;
        }
        if (engine) engine->leave();
        p->tail_runner = nullptr;
        r.max_error = j.req.data_kind == 0 ? 0.0 : p->synth_error(j.req.data_kind, u);
        r.status = status;
        r.iterations = st.iterations;
        r.hist_len = st.hist_len;
        r.shift_alpha = st.shift_alpha;
        r.rel_residual = st.final_rel_residual;
        r.device_bytes = (int64_t)p->mem.peak;
        r.t_finish = clock();  // the result is complete; teardown follows
    } catch (const Error& e) {
        r.status = e.code;
        r.t_finish = clock();
    } catch (...) {
        r.status = IIM_E_INTERNAL;
        r.t_finish = clock();
    }
}

void Server::worker() {
    hipStream_t s = nullptr;
    double* hpin = nullptr;
    bool ok = hipSetDevice(device) == hipSuccess && hipStreamCreateWithFlags(&s, hipStreamNonBlocking) == hipSuccess &&
              hipHostMalloc((void**)&hpin, HPIN_DOUBLES * sizeof(double), hipHostMallocCoherent) == hipSuccess;
    while (true) {
        Job* j = nullptr;
        {
            std::unique_lock<std::mutex> lk(mu);
            cv_work.wait(lk, [&] {
                return (stopping && queue.empty()) ||
                       (!queue.empty() && reserved + queue.front()->res.estimated_bytes <= budget);
            });
            if (queue.empty()) break;
            j = queue.front();
            queue.pop_front();
            reserved += j->res.estimated_bytes;
            peak = std::max(peak, reserved);
            ++running;
            j->res.t_start = clock();
        }
        cv_work.notify_all();  // the new head may fit beside this one
        if (ok)
            run(*j, s, hpin);
        else {
            j->res.status = IIM_E_DEVICE;
            j->res.t_finish = clock();
        }
        {
            std::lock_guard<std::mutex> lk(mu);
            reserved -= j->res.estimated_bytes;
            --running;
            if (j->res.status < 0) ++failed; else ++completed;
            j->res.done = 1;
        }
        cv_done.notify_all();
        cv_work.notify_all();
    }
    if (hpin) (void)hipHostFree(hpin);
    if (s) (void)hipStreamDestroy(s);
}

// the parameter checks that must hold before the estimator reads params
static void check_request(const iim_request& q) {
    const iim_grid& g = q.grid;
    const iim_geometry& geo = q.geom;
    if (g.dim != 2 && g.dim != 3) throw Error(IIM_E_INVALID_ARG, "dim must be 2 or 3");
    if (g.n < 8 || g.n > 16384) throw Error(IIM_E_INVALID_ARG, "n out of range");
    if (!(g.hi > g.lo)) throw Error(IIM_E_INVALID_ARG, "empty domain");
    if (!geo.params) throw Error(IIM_E_INVALID_ARG, "null params");
    if (geo.kind == IIM_GEOM_SPHERE && geo.nparams < g.dim + 1)
        throw Error(IIM_E_INVALID_ARG, "sphere needs dim + 1 parameters");
    if (geo.kind == IIM_GEOM_STAR2D && (g.dim != 2 || geo.nparams < 5))
        throw Error(IIM_E_INVALID_ARG, "star needs dim 2 and 5 parameters");
    if (geo.kind == IIM_GEOM_SPHERE_UNION &&
        (geo.nparams < 1 || geo.params[0] < 0 || geo.nparams < 1 + (g.dim + 1) * (int64_t)geo.params[0]))
        throw Error(IIM_E_INVALID_ARG, "sphere union parameter count");
    if (geo.kind < 0 || geo.kind > 3) throw Error(IIM_E_INVALID_ARG, "bad geometry kind");
    if (geo.kind == IIM_GEOM_GYROID && (g.dim != 3 || geo.nparams < 4 || !g.periodic))
        throw Error(IIM_E_INVALID_ARG, "the gyroid needs dim 3, 4 parameters and a periodic grid");
    check_singular_connected(g, geo);
    if (q.data_kind != 0 && q.data_kind != 1) throw Error(IIM_E_INVALID_ARG, "unknown data kind");
    if (q.data_kind == 0) {
        if (!q.f) throw Error(IIM_E_INVALID_ARG, "caller data needs f");
        if (q.n_cp_data < 0 || (q.n_cp_data > 0 && !q.cp_data))
            throw Error(IIM_E_INVALID_ARG, "caller data needs cp_data");
        if (q.mem_kind != IIM_MEM_HOST && q.mem_kind != IIM_MEM_DEVICE) throw Error(IIM_E_INVALID_ARG, "bad mem_kind");
    }
    if (q.hist_cap < 0 || (q.hist_cap > 0 && !q.hist)) throw Error(IIM_E_INVALID_ARG, "bad history buffer");
}

}  // namespace iim

using namespace iim;

struct iim_server {
    Server s;
};

#define SRV_TRY(...)                                               \
    try {                                                          \
        __VA_ARGS__;                                               \
    } catch (const iim::Error& e) {                                \
        iim::set_error(e.what());                                  \
        return e.code;                                             \
    } catch (const std::exception& e) {                            \
        iim::set_error(std::string("internal error: ") + e.what()); \
        return IIM_E_INTERNAL;                                     \
    } catch (...) {                                                \
        iim::set_error("internal error");                          \
        return IIM_E_INTERNAL;                                     \
    }

extern "C" {

int iim_server_create_ex(int64_t budget_bytes, int32_t max_slots, const iim_server_options* opt,
                         iim_server** out) {
    SRV_TRY({
        if (!out) throw Error(IIM_E_INVALID_ARG, "null argument");
        *out = nullptr;
        if (budget_bytes <= 0) throw Error(IIM_E_INVALID_ARG, "budget must be positive");
        if (max_slots < 1 || max_slots > 64) throw Error(IIM_E_INVALID_ARG, "max_slots must be in [1, 64]");
        iim_server_options o{0, 0};
        if (opt) o = *opt;
        if (o.batch_window_us < 0 || o.batch_window_us > 100000)
            throw Error(IIM_E_INVALID_ARG, "batch_window_us must be in [0, 100000]");
        auto srv = std::make_unique<iim_server>();
        IIM_HIP(hipGetDevice(&srv->s.device));
        configure_pool(srv->s.device);
        srv->s.budget = budget_bytes;
        if (o.batch_tails) srv->s.engine = std::make_unique<TailBatcher>(o.batch_window_us);
        for (int i = 0; i < max_slots; ++i) srv->s.workers.emplace_back([p = &srv->s] { p->worker(); });
        *out = srv.release();
        return IIM_OK;
    })
}

int iim_server_create(int64_t budget_bytes, int32_t max_slots, iim_server** out) {
    return iim_server_create_ex(budget_bytes, max_slots, nullptr, out);
}

int iim_server_submit(iim_server* srv, const iim_request* req, uint64_t* ticket) {
    SRV_TRY({
        if (!srv || !req || !ticket) throw Error(IIM_E_INVALID_ARG, "null argument");
        check_request(*req);
        auto j = std::make_unique<Job>();
        j->req = *req;
        j->params.assign(req->geom.params, req->geom.params + req->geom.nparams);
        j->req.geom.params = j->params.data();
        j->res.estimated_bytes = estimate_bytes(j->req.grid, j->req.geom, j->req.opt);
        Server& s = srv->s;
        {
            std::lock_guard<std::mutex> lk(s.mu);
            if (s.stopping) throw Error(IIM_E_INVALID_ARG, "server is shutting down");
            const uint64_t id = s.next_ticket++;
            j->res.t_submit = s.clock();
            ++s.submitted;
            Job* jp = j.get();
            s.jobs.emplace(id, std::move(j));
            if (jp->res.estimated_bytes > s.budget) {  // can never run: fail now, keep the queue moving
                jp->res.status = IIM_E_BUDGET;
                jp->res.t_start = jp->res.t_finish = jp->res.t_submit;
                jp->res.done = 1;
                ++s.failed;
            } else {
                s.queue.push_back(jp);
            }
            *ticket = id;
        }
        s.cv_work.notify_all();
        s.cv_done.notify_all();
        return IIM_OK;
    })
}

int iim_server_poll(iim_server* srv, uint64_t ticket, iim_result* res) {
    SRV_TRY({
        if (!srv || !res) throw Error(IIM_E_INVALID_ARG, "null argument");
        std::lock_guard<std::mutex> lk(srv->s.mu);
        auto it = srv->s.jobs.find(ticket);
        if (it == srv->s.jobs.end()) throw Error(IIM_E_INVALID_ARG, "unknown ticket");
        *res = it->second->res;
        return IIM_OK;
    })
}

int iim_server_wait(iim_server* srv, uint64_t ticket, iim_result* res) {
    SRV_TRY({
        if (!srv || !res) throw Error(IIM_E_INVALID_ARG, "null argument");
        std::unique_lock<std::mutex> lk(srv->s.mu);
        auto it = srv->s.jobs.find(ticket);
        if (it == srv->s.jobs.end()) throw Error(IIM_E_INVALID_ARG, "unknown ticket");
        Job* j = it->second.get();
        srv->s.cv_done.wait(lk, [&] { return j->res.done != 0; });
        *res = j->res;
        return IIM_OK;
    })
}

int iim_server_stats_get(iim_server* srv, iim_server_stats* st) {
    SRV_TRY({
        if (!srv || !st) throw Error(IIM_E_INVALID_ARG, "null argument");
        Server& s = srv->s;
        std::lock_guard<std::mutex> lk(s.mu);
        st->submitted = s.submitted;
        st->completed = s.completed;
        st->failed = s.failed;
        st->running = s.running;
        st->queued = (int64_t)s.queue.size();
        st->bytes_reserved = s.reserved;
        st->bytes_budget = s.budget;
        st->peak_bytes_reserved = s.peak;
        st->tail_batches = st->tail_jobs = 0;
        if (s.engine) {
            std::lock_guard<std::mutex> lk2(s.engine->mu);
            st->tail_batches = s.engine->batches;
            st->tail_jobs = s.engine->jobs;
        }
        return IIM_OK;
    })
}

double iim_server_clock(iim_server* srv) { return srv ? srv->s.clock() : 0.0; }

void iim_server_destroy(iim_server* srv) {
    if (!srv) return;
    {
        std::lock_guard<std::mutex> lk(srv->s.mu);
        srv->s.stopping = true;
    }
    srv->s.cv_work.notify_all();
    for (auto& t : srv->s.workers) t.join();
    delete srv;
    trim_pool();
}

}  // extern "C"
