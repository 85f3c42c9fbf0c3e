// Serving loop: a stream of independent solve requests with continuous
// batching. Requests are copied at submission; a pool of host threads runs
// their setup (validation, local graphs, coarse operator and its inverse);
// one GPU thread admits set-up requests while their device memory fits the
// budget, advances every active problem by a chunk of iterations with one
// launch per kernel (a batch whose per-problem done flags mask finished
// problems), and retires the problems that converged, freeing their memory
// for the next admissions. A problem's arithmetic does not depend on the
// other members of its batch (per-problem reductions in a fixed order), so a
// served result equals the result of solving it alone.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <set>
#include <thread>

#include "runtime.h"

namespace ddmgnn {
namespace {

using Clock = std::chrono::steady_clock;

double ms_between(Clock::time_point a, Clock::time_point b) {
    return std::chrono::duration<double, std::milli>(b - a).count();
}

struct Request {
    uint64_t ticket = 0;
    // owned copy of the descriptor
    std::vector<double> xy, a_val, b, u0, weights;
    std::vector<int32_t> tri, a_rowptr, a_col, sub_nodes;
    std::vector<uint8_t> dirichlet;
    std::vector<int64_t> sub_ptr;
    ddmgnn_problem_desc desc{};
    ddmgnn_solve_opts opts{};
    HostSetup hs;
    int setup_rc = DDMGNN_OK;
    std::string err;
    size_t bytes = 0;
    Clock::time_point t_submit, t_setup0, t_setup1, t_admit, t_created, t_done;
    ddmgnn_problem* prob = nullptr;
    bool fresh = false;  // admitted, not initialised yet
    // result
    std::vector<double> u;
    ddmgnn_stats stats{};
    int status = DDMGNN_E_PENDING;
};

template <typename T>
void copy_in(std::vector<T>& dst, const T* src, int64_t n) {
    if (src && n > 0) dst.assign(src, src + n);
}

// Options that must agree among the problems of one batch.
uint64_t structure_key(const ddmgnn_solve_opts& o) {
    const int m = o.krylov == DDMGNN_FCG ? o.m_max : o.krylov == DDMGNN_FGMRES ? o.restart : 1;
    return ((uint64_t)o.local_solver << 32) | ((uint64_t)o.krylov << 24) | ((uint64_t)m << 16) |
           ((uint64_t)o.precision << 8) | ((uint64_t)o.prolong << 4) | (uint64_t)(o.coarse != 0);
}

// One set-up request waiting for admission.
struct Candidate {
    size_t bytes;
    uint64_t key;  // structure_key of its options
    bool ok;       // setup succeeded
};
enum Decision { ADMIT, REJECT, WAIT };

// The admission rule of the serving loop, over the set-up requests in ticket
// order: one whose setup failed or that is larger than the budget is rejected
// wherever it stands (it could never run); the others are admitted while they
// share the active group's options key (any key when nothing is active), fit
// the budget next to the active bytes and keep at most max_active active; the
// first that does not is WAIT, and so is every later one (no overtaking).
std::vector<Decision> plan_admission(const std::vector<Candidate>& ready, size_t bytes_active, int n_active,
                                     uint64_t group, size_t budget, int max_active) {
    std::vector<Decision> out(ready.size(), WAIT);
    size_t bytes = bytes_active;
    uint64_t g = group;
    bool blocked = false;
    for (size_t i = 0; i < ready.size(); ++i) {
        const Candidate& c = ready[i];
        if (!c.ok || c.bytes > budget) {
            out[i] = REJECT;
            continue;
        }
        if (blocked || (n_active > 0 && c.key != g) || n_active >= max_active || bytes + c.bytes > budget) {
            blocked = true;
            continue;
        }
        g = c.key;
        bytes += c.bytes;
        ++n_active;
        out[i] = ADMIT;
    }
    return out;
}

}  // namespace
}  // namespace ddmgnn

using namespace ddmgnn;

struct ddmgnn_server {
    ddmgnn_ctx* ctx = nullptr;
    std::shared_ptr<ModelDev> model;
    size_t budget = 0;
    int max_active = 0;
    std::mutex mu;
    std::condition_variable cv;        // work for the GPU thread or setup workers
    std::condition_variable cv_done;   // a request finished
    std::deque<Request*> pending;      // submitted, waiting for host setup
    std::map<uint64_t, Request*> ready;  // set up, waiting for admission (ticket order)
    std::map<uint64_t, Request*> finished;
    std::set<uint64_t> live;           // submitted and not collected
    size_t in_flight = 0;              // submitted and not finished
    uint64_t next_ticket = 1;
    bool stop = false;
    std::thread gpu;
    std::vector<std::thread> workers;
    hipStream_t upload = nullptr;      // problem creation, beside the active chunk on ctx's stream
    std::string loop_error;

    void setup_worker();
    void gpu_loop();
    void finish(Request* r);
};

void ddmgnn_server::finish(Request* r) {
    r->t_done = Clock::now();
    r->stats.latency_ms = ms_between(r->t_submit, r->t_done);
    r->stats.status = r->status;
    const Clock::time_point admitted = r->t_admit == Clock::time_point() ? r->t_done : r->t_admit;
    r->stats.setup_ms = ms_between(r->t_setup0, r->t_setup1);
    r->stats.queue_ms = ms_between(r->t_submit, r->t_setup0) + ms_between(r->t_setup1, admitted);
    r->stats.upload_ms = r->t_created == Clock::time_point() ? 0.0 : ms_between(r->t_admit, r->t_created);
    std::lock_guard<std::mutex> lk(mu);
    finished[r->ticket] = r;
    --in_flight;
    cv_done.notify_all();
}

void ddmgnn_server::setup_worker() {
    for (;;) {
        Request* r = nullptr;
        {
            std::unique_lock<std::mutex> lk(mu);
            cv.wait(lk, [&] { return stop || !pending.empty(); });
            if (pending.empty()) return;
            r = pending.front();
            pending.pop_front();
        }
        r->t_setup0 = Clock::now();
        std::string e = validate(r->desc);
        if (e.empty()) e = build_setup(r->desc, r->hs, false);  // coarse level: on the device at admission
        if (e.empty()) e = prepare_upload(r->desc, r->hs);      // admission then only copies
        const bool lu = r->opts.local_solver == DDMGNN_LOCAL_LU && r->opts.krylov != DDMGNN_CG;
        if (e == "NOT_SPD") {
            r->setup_rc = DDMGNN_E_NOT_SPD;
            r->err = "coarse matrix R_0 A R_0^T is not positive definite";
        } else if (!e.empty()) {
            r->setup_rc = DDMGNN_E_INVALID;
            r->err = e;
        } else {
            // DDM-LU requests: the local inverses are formed on the device at the
            // first solve; their bytes count in the admission budget.
            size_t lu_bytes = 0;
            if (lu)
                for (int32_t i = 0; i < r->hs.K; ++i) {
                    const int64_t k = r->hs.sub_ptr[i + 1] - r->hs.sub_ptr[i];
                    lu_bytes += (size_t)(k * lu_ld(k)) * sizeof(double) + sizeof(int64_t);
                }
            r->bytes = problem_device_bytes(r->hs.n, r->hs.nnz, r->hs.K, r->hs.sk, r->hs.n_edges) + lu_bytes +
                       (r->opts.krylov == DDMGNN_FGMRES ? fgmres_bytes(r->hs.n, r->opts.restart) : 0);
        }
        r->t_setup1 = Clock::now();
        std::lock_guard<std::mutex> lk(mu);
        ready[r->ticket] = r;
        cv.notify_all();
    }
}

// One round of the GPU thread: admissions are planned, the active set's
// chunk of iterations is launched, the admitted problems are created on the
// upload stream while it runs, then the chunk is polled, converged problems
// retire and the new ones join the active set (a rebuilt batch next round).
void ddmgnn_server::gpu_loop() {
    (void)hipSetDevice(ctx->device);
    std::vector<Request*> active;
    BatchPtr B;
    bool changed = false;
    size_t bytes_active = 0;
    uint64_t group = 0;
    ddmgnn_solve_opts gopts{};
    auto fail_all = [&](int rc) {
        const std::string msg = "serving loop: " + std::string(ddmgnn_last_error());
        B.reset();
        for (Request* r : active) {
            delete r->prob;
            r->prob = nullptr;
            r->status = rc;
            r->err = msg;
            finish(r);
        }
        active.clear();
        bytes_active = 0;
    };
    for (;;) {
        std::vector<Request*> admit, reject;
        {
            std::unique_lock<std::mutex> lk(mu);
            cv.wait(lk, [&] { return !active.empty() || !ready.empty() || (stop && in_flight == 0); });
            if (active.empty() && ready.empty() && stop && in_flight == 0) return;
            // Admission in ticket order; the first request that does not fit waits (no overtaking).
            std::vector<Candidate> cands;
            std::vector<uint64_t> tickets;
            for (const auto& kv : ready) {
                cands.push_back({kv.second->bytes, structure_key(kv.second->opts), kv.second->setup_rc == DDMGNN_OK});
                tickets.push_back(kv.first);
            }
            const std::vector<Decision> plan = plan_admission(cands, bytes_active, (int)active.size(),
                                                              active.empty() ? 0 : group, budget, max_active);
            for (size_t i = 0; i < plan.size(); ++i) {
                if (plan[i] == WAIT) continue;
                auto it = ready.find(tickets[i]);
                (plan[i] == ADMIT ? admit : reject).push_back(it->second);
                ready.erase(it);
            }
        }
        for (Request* r : reject) {
            if (r->setup_rc == DDMGNN_OK) {
                r->setup_rc = DDMGNN_E_BUDGET;
                r->err = "request needs more device memory than the server budget";
            }
            r->status = r->setup_rc;
            finish(r);
        }
        if (!active.empty() && changed) {
            std::vector<ddmgnn_problem*> probs;
            std::vector<uint8_t> init;
            for (Request* r : active) {
                probs.push_back(r->prob);
                init.push_back(r->fresh ? 1 : 0);
                r->fresh = false;
            }
            B.reset();
            int rc = build_batch(ctx, probs.data(), (int)probs.size(), B);
            if (!rc) rc = batch_begin(*B, gopts, &init);
            if (rc) fail_all(rc);
            changed = false;
        }
        int rc = DDMGNN_OK;
        const bool running = !active.empty();
        if (running) rc = batch_iterate(*B, gopts, std::max(1, gopts.check_every), false);  // asynchronous
        std::vector<Request*> incoming;
        for (Request* r : admit) {
            r->t_admit = Clock::now();
            ddmgnn_problem* P = nullptr;
            const int crc = create_problem(ctx, r->desc, model, std::move(r->hs), &P, upload);
            r->t_created = Clock::now();
            r->hs = HostSetup();
            if (crc) {
                r->status = crc;
                r->err = ddmgnn_last_error();
                finish(r);
                continue;
            }
            P->rtol = r->opts.rtol;
            P->max_it = r->opts.max_it;
            r->prob = P;
            r->fresh = true;
            incoming.push_back(r);
        }
        auto join_incoming = [&] {
            for (Request* r : incoming) {
                if (active.empty()) {
                    group = structure_key(r->opts);
                    gopts = r->opts;
                }
                bytes_active += r->bytes;
                active.push_back(r);
                changed = true;
            }
        };
        if (!running) {
            join_incoming();
            continue;
        }
        if (!rc) rc = batch_poll(*B);
        if (rc) {
            fail_all(rc);
            join_incoming();
            continue;
        }
        std::vector<uint8_t> done(active.size(), 0);
        bool any = false;
        for (size_t i = 0; i < active.size(); ++i) {
            done[i] = batch_state(*B, (int)i).done ? 1 : 0;
            any = any || done[i];
        }
        if (!any) {
            join_incoming();
            continue;
        }
        rc = batch_true_residual(*B, &done);
        if (rc) {
            fail_all(rc);
            join_incoming();
            continue;
        }
        std::vector<Request*> keep;
        for (size_t i = 0; i < active.size(); ++i) {
            Request* r = active[i];
            if (!done[i]) {
                keep.push_back(r);
                continue;
            }
            const KState& k = batch_state(*B, (int)i);
            ddmgnn_problem* P = r->prob;
            r->u.resize(P->hs.n);
            hipError_t e = hipMemcpyAsync(r->u.data(), P->u.p, P->hs.n * sizeof(double), hipMemcpyDeviceToHost,
                                          ctx->stream);
            if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
            const bool converged = k.status == 0 && k.rel <= r->opts.rtol;
            ddmgnn_stats& S = r->stats;
            std::memset(&S, 0, sizeof(S));
            S.iterations = k.it;
            S.converged = converged;
            S.rel_residual = k.rel;
            S.true_rel_residual = k.r0n > 0 ? std::sqrt(k.rr_true) / k.r0n : 0.0;
            S.solve_ms = ms_between(r->t_admit, Clock::now());
            S.dss_kernel = dss_kernel_of(P, gopts);
            if (e != hipSuccess) {
                r->status = DDMGNN_E_HIP;
                r->err = std::string("result copy: ") + hipGetErrorString(e);
            } else {
                r->status = k.status ? k.status : (converged ? DDMGNN_OK : DDMGNN_E_MAXIT);
                if (r->status) r->err = k.status ? "Krylov breakdown or non-finite residual" : "not converged within max_it";
            }
            bytes_active -= r->bytes;
            delete P;
            r->prob = nullptr;
            finish(r);
        }
        active.swap(keep);
        changed = true;
        if (active.empty()) B.reset();
        join_incoming();
    }
}

extern "C" {

int ddmgnn_server_create(ddmgnn_ctx* ctx, const ddmgnn_model* model, int64_t hbm_budget, int32_t max_active,
                         int32_t setup_threads, ddmgnn_server** out) {
    if (!ctx || !model || !out) return fail(DDMGNN_E_INVALID, "null argument");
    if (hbm_budget <= 0 || max_active < 1) return fail(DDMGNN_E_INVALID, "budget and max_active must be positive");
    if (setup_threads < 0 || setup_threads > 64) return fail(DDMGNN_E_INVALID, "setup_threads must be in [0, 64]");
    auto s = std::make_unique<ddmgnn_server>();
    s->ctx = ctx;
    s->model = model->dev;
    s->budget = (size_t)hbm_budget;
    s->max_active = max_active;
    {  // the upload stream lives on the context's device (the caller's current device is restored)
        int prev = 0;
        (void)hipGetDevice(&prev);
        hipError_t e = hipSetDevice(ctx->device);
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->upload, hipStreamNonBlocking);
        (void)hipSetDevice(prev);
        if (e != hipSuccess) return fail(DDMGNN_E_HIP, std::string("server upload stream: ") + hipGetErrorString(e));
    }
    const int nw = setup_threads ? setup_threads : 4;
    for (int i = 0; i < nw; ++i) s->workers.emplace_back(&ddmgnn_server::setup_worker, s.get());
    s->gpu = std::thread(&ddmgnn_server::gpu_loop, s.get());
    *out = s.release();
    return DDMGNN_OK;
}

int ddmgnn_server_submit(ddmgnn_server* srv, const ddmgnn_problem_desc* desc_in, const ddmgnn_solve_opts* opts,
                         uint64_t* ticket) {
    if (!srv || !desc_in || !opts || !ticket) return fail(DDMGNN_E_INVALID, "null argument");
    if (int rc = check_opts(*opts)) return rc;
    HostDesc hd;
    const ddmgnn_problem_desc* desc = nullptr;
    if (int rc = host_desc(desc_in, hd, &desc)) return rc;
    if (desc->n_nodes <= 0 || desc->n_tri <= 0 || desc->n_sub <= 0 || !desc->sub_ptr)
        return fail(DDMGNN_E_INVALID, "empty problem");
    auto r = std::make_unique<Request>();
    const int64_t n = desc->n_nodes, nt = desc->n_tri, K = desc->n_sub;
    const int64_t nnz = desc->a_rowptr ? desc->a_rowptr[n] : 0;
    const int64_t sk = desc->sub_ptr[K];
    if (nnz < 0 || sk < 0) return fail(DDMGNN_E_INVALID, "negative sizes");
    copy_in(r->xy, desc->xy, 2 * n);
    copy_in(r->tri, desc->tri, 3 * nt);
    copy_in(r->dirichlet, desc->dirichlet, n);
    copy_in(r->a_rowptr, desc->a_rowptr, n + 1);
    copy_in(r->a_col, desc->a_col, nnz);
    copy_in(r->a_val, desc->a_val, nnz);
    copy_in(r->b, desc->b, n);
    copy_in(r->u0, desc->u0, n);
    copy_in(r->sub_ptr, desc->sub_ptr, K + 1);
    copy_in(r->sub_nodes, desc->sub_nodes, sk);
    copy_in(r->weights, desc->weights, sk);
    ddmgnn_problem_desc& d = r->desc;
    d.n_nodes = n;
    d.xy = r->xy.empty() ? nullptr : r->xy.data();
    d.n_tri = nt;
    d.tri = r->tri.empty() ? nullptr : r->tri.data();
    d.dirichlet = r->dirichlet.empty() ? nullptr : r->dirichlet.data();
    d.a_rowptr = r->a_rowptr.empty() ? nullptr : r->a_rowptr.data();
    d.a_col = r->a_col.empty() ? nullptr : r->a_col.data();
    d.a_val = r->a_val.empty() ? nullptr : r->a_val.data();
    d.b = r->b.empty() ? nullptr : r->b.data();
    d.u0 = r->u0.empty() ? nullptr : r->u0.data();
    d.n_sub = (int32_t)K;
    d.sub_ptr = r->sub_ptr.data();
    d.sub_nodes = r->sub_nodes.empty() ? nullptr : r->sub_nodes.data();
    d.weights = r->weights.empty() ? nullptr : r->weights.data();
    r->opts = *opts;
    r->t_submit = Clock::now();
    std::lock_guard<std::mutex> lk(srv->mu);
    if (srv->stop) return fail(DDMGNN_E_INVALID, "server is shutting down");
    r->ticket = srv->next_ticket++;
    *ticket = r->ticket;
    ++srv->in_flight;
    srv->live.insert(r->ticket);
    srv->pending.push_back(r.release());
    srv->cv.notify_all();
    return DDMGNN_OK;
}

int ddmgnn_server_poll(ddmgnn_server* srv, uint64_t ticket, double* u_out, ddmgnn_stats* stats) {
    if (!srv) return fail(DDMGNN_E_INVALID, "null server");
    Request* r = nullptr;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        if (!srv->live.count(ticket)) return fail(DDMGNN_E_INVALID, "unknown or already collected ticket");
        auto it = srv->finished.find(ticket);
        if (it == srv->finished.end()) return DDMGNN_E_PENDING;
        r = it->second;
        srv->finished.erase(it);
        srv->live.erase(ticket);
    }
    std::unique_ptr<Request> hold(r);
    if (stats) *stats = r->stats;
    if (u_out && !r->u.empty()) std::memcpy(u_out, r->u.data(), r->u.size() * sizeof(double));
    if (r->status) return fail(r->status, r->err);
    return DDMGNN_OK;
}

int ddmgnn_server_drain(ddmgnn_server* srv) {
    if (!srv) return fail(DDMGNN_E_INVALID, "null server");
    std::unique_lock<std::mutex> lk(srv->mu);
    srv->cv_done.wait(lk, [&] { return srv->in_flight == 0; });
    return DDMGNN_OK;
}

int ddmgnn_server_destroy(ddmgnn_server* srv) {
    if (!srv) return DDMGNN_OK;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stop = true;
        srv->cv.notify_all();
    }
    if (srv->gpu.joinable()) srv->gpu.join();
    for (auto& t : srv->workers)
        if (t.joinable()) t.join();
    for (auto& kv : srv->finished) delete kv.second;
    if (srv->upload) (void)hipStreamDestroy(srv->upload);
    delete srv;
    return DDMGNN_OK;
}

}  // extern "C"

int ddmgnn_server_simulate(const ddmgnn_sim_request* reqs, int32_t n, int64_t hbm_budget, int32_t max_active,
                           int32_t setup_threads, double chunk_s, ddmgnn_sim_result* out) {
    if ((!reqs || !out) && n > 0) return fail(DDMGNN_E_INVALID, "null argument");
    if (n < 0 || hbm_budget <= 0 || max_active < 1 || !(chunk_s > 0.0))
        return fail(DDMGNN_E_INVALID, "n >= 0, hbm_budget > 0, max_active >= 1 and chunk_s > 0 required");
    const int workers = setup_threads > 0 ? setup_threads : 4;
    for (int32_t i = 0; i < n; ++i) {
        if (!(reqs[i].setup_s >= 0.0) || reqs[i].chunks < 1 || reqs[i].bytes < 0)
            return fail(DDMGNN_E_INVALID, "setup_s >= 0, chunks >= 1 and bytes >= 0 required");
        if (i > 0 && reqs[i].arrival < reqs[i - 1].arrival)
            return fail(DDMGNN_E_INVALID, "requests must be in submission order");
    }
    // setup workers take the requests in submission order
    std::vector<double> ready_at(n), free_at(workers, 0.0);
    for (int32_t i = 0; i < n; ++i) {
        auto w = std::min_element(free_at.begin(), free_at.end());
        const double start = std::max(*w, reqs[i].arrival);
        *w = start + reqs[i].setup_s;
        ready_at[i] = *w;
        out[i] = {-1.0, -1.0, DDMGNN_E_PENDING};
    }
    std::vector<int32_t> waiting(n);  // set-up or in setup, not yet decided, in ticket order
    for (int32_t i = 0; i < n; ++i) waiting[i] = i;
    struct Act {
        int32_t i;
        int32_t left;
    };
    std::vector<Act> active;
    size_t bytes_active = 0;
    uint64_t group = 0;
    double t = 0.0;
    while (!waiting.empty() || !active.empty()) {
        std::vector<Candidate> cands;
        std::vector<int32_t> idx;
        for (int32_t i : waiting)
            if (ready_at[i] <= t) {
                cands.push_back({(size_t)reqs[i].bytes, reqs[i].group, reqs[i].setup_ok != 0});
                idx.push_back(i);
            }
        const std::vector<Decision> plan =
            plan_admission(cands, bytes_active, (int)active.size(), active.empty() ? 0 : group, (size_t)hbm_budget,
                           max_active);
        for (size_t q = 0; q < plan.size(); ++q) {
            const int32_t i = idx[q];
            if (plan[q] == WAIT) continue;
            if (plan[q] == REJECT) {
                out[i] = {t, t, reqs[i].setup_ok ? DDMGNN_E_BUDGET : DDMGNN_E_INVALID};
            } else {
                if (active.empty()) group = reqs[i].group;
                active.push_back({i, reqs[i].chunks});
                bytes_active += (size_t)reqs[i].bytes;
                out[i].admitted = t;
            }
            waiting.erase(std::find(waiting.begin(), waiting.end(), i));
        }
        if (active.empty()) {  // idle until the next setup ends
            double next = 1e300;
            for (int32_t i : waiting) next = std::min(next, ready_at[i]);
            if (next == 1e300) break;
            t = std::max(t, next);
            continue;
        }
        t += chunk_s;  // one chunk of every active request (one batched launch sequence)
        for (size_t a = 0; a < active.size();) {
            if (--active[a].left == 0) {
                const int32_t i = active[a].i;
                out[i].finished = t;
                out[i].status = DDMGNN_OK;
                bytes_active -= (size_t)reqs[i].bytes;
                active.erase(active.begin() + (long)a);
            } else {
                ++a;
            }
        }
    }
    return DDMGNN_OK;
}
