// Serving runtime: continuous batching of ADAPT solves on one device.
//
// Requests (a Hamiltonian, a pool, a convergence threshold) are queued by
// gocp_server_submit from any thread.  A worker thread owns the device side:
// it admits queued requests in arrival order while a slot is free and the
// request's device footprint fits the HBM budget, starts each admitted
// request from its Hartree-Fock state, and advances all admitted requests
// together, `iters_per_step` ADAPT iterations per step, with one launch per
// kernel for the whole set (the lock-step group of the batched form).  After
// each step it retires the requests that converged or hit their iteration
// limit, frees their memory, and admits waiting requests into the freed
// room, so requests that arrive while others run join the running set.
// Every request computes exactly what it computes alone.

#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>

#include "adapt.h"

namespace gocp {
namespace {

int64_t now_ns() {
    return std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

struct Request {
    uint64_t ticket = 0;
    const Ham *h = nullptr;
    const Pool *p = nullptr;
    int max_iter = 0;
    double tol = 0.0;
    uint64_t hf = 0;
    size_t footprint = 0;
    int64_t t_submit = 0, t_admit = 0, t_done = 0;
    int status = GOCP_EBUSY;
    bool finished = false;
    std::unique_ptr<Instance> inst;
    // record, copied out of the device when the request finishes
    int n_iter = 0, converged = 0;
    std::vector<double> energies, thetas, gnorms, gmax;
    std::vector<int32_t> ops, substeps;
};

// Device tables of a request (an upper bound: staged tables carry up to
// kStrGroup - 1 zero strings per class or operator).
size_t table_bytes(const Ham *h, const Pool *p) {
    const size_t nc = (size_t)h->n_classes(), m = (size_t)p->n_ops(), ps = p->str_z.size();
    const size_t ham = ((size_t)h->n_terms() + (kStrGroup - 1) * nc) * sizeof(HTerm) +
                       nc * (sizeof(HClass) + sizeof(HSub)) + (nc + 1) * sizeof(int32_t);
    const size_t pool = ps * sizeof(HTerm) + m * sizeof(HClass) +                       // pair tables
                        (ps + (kStrGroup - 1) * m) * sizeof(HTerm) +                      // screen tables
                        m * (sizeof(HClass) + sizeof(HSub)) + (m + 1) * sizeof(int32_t) +
                        m * sizeof(double);
    return ham + pool;
}

}  // namespace
}  // namespace gocp

struct gocp_server {
    gocp_ctx *ctx = nullptr;
    hipStream_t stream = nullptr;
    int dtype = 0, max_slots = 1, iters_per_step = 1;
    int schedule = 1;     // amplitudes per lane, or 0: chosen from the active set
    size_t budget = 0;
    std::mutex mu;
    std::condition_variable cv;
    std::deque<gocp::Request *> queue;
    std::vector<gocp::Request *> active;   // touched by the worker only
    int32_t n_active = 0;                  // size of `active`, guarded by mu
    std::map<uint64_t, std::unique_ptr<gocp::Request>> requests;
    size_t bytes_in_use = 0;
    uint64_t next_ticket = 1;
    int64_t completed = 0, steps = 0;
    bool stop = false;
    std::string worker_error;
    gocp::Group group;
    std::thread worker;
    void choose_schedule();

    void finish(gocp::Request *r, int status) {   // caller holds mu
        r->status = status;
        r->finished = true;
        r->t_done = gocp::now_ns();
        ++completed;
    }

    void run();
};

namespace gocp {
namespace {

void copy_record(Request *r, hipStream_t s) {
    const int n = r->max_iter;
    r->energies.assign(n + 1, 0.0);
    r->thetas.assign(std::max(n, 1), 0.0);
    r->gnorms.assign(n + 1, 0.0);
    r->gmax.assign(n + 1, 0.0);
    r->ops.assign(std::max(n, 1), 0);
    r->substeps.assign(std::max(n, 1), 0);
    gocp_adapt_result res{0, 0, r->energies.data(), r->ops.data(), r->thetas.data(),
                          r->gnorms.data(), r->gmax.data(), r->substeps.data()};
    read_result(r->inst.get(), s, &res, nullptr);
    r->n_iter = res.n_iter;
    r->converged = res.converged;
}

}  // namespace
}  // namespace gocp

// Adaptive schedule: one amplitude per lane while the active set has fewer
// than four tiles of 64 amplitudes per compute unit (the launches are then
// latency-bound and more tiles keep more units busy); otherwise wider blocking,
// which cuts the work per amplitude (2 for complex128 states, whose widest
// blocking runs short of registers; 4 for complex64).
void gocp_server::choose_schedule() {
    if (schedule != 0) return;
    long tiles = 0;
    for (gocp::Request *r : active) tiles += gocp::tiles_for(r->inst->ip.n_qubits, 1);
    group.R = tiles < 4L * ctx->n_cu ? 1 : (dtype == GOCP_C128 ? 2 : 4);
}

void gocp_server::run() {
    using namespace gocp;
    try {
        hip_check(hipSetDevice(ctx->device), "hipSetDevice");
        std::vector<int32_t> done;
        for (;;) {
            std::vector<Request *> admitted;
            {
                std::unique_lock<std::mutex> lk(mu);
                if (stop) break;
                while (!queue.empty() && (int)(active.size() + admitted.size()) < max_slots) {
                    Request *r = queue.front();
                    if (r->footprint > budget) {           // can never fit
                        queue.pop_front();
                        finish(r, GOCP_ENOMEM);
                        continue;
                    }
                    if (bytes_in_use + r->footprint > budget) break;   // wait for room, in order
                    queue.pop_front();
                    bytes_in_use += r->footprint;
                    admitted.push_back(r);
                }
                if (active.empty() && admitted.empty()) {
                    cv.notify_all();
                    cv.wait(lk, [&] { return stop || !queue.empty(); });
                    continue;
                }
            }
            // admit: allocate, start from Hartree-Fock, evaluate E_0 and the first screen
            std::vector<int> fresh;
            for (Request *r : admitted) {
                r->inst.reset(instance_create(ctx, r->h, r->p, nullptr, dtype, r->max_iter, r->tol, r->hf, stream));
                r->t_admit = now_ns();
                fresh.push_back((int)active.size());
                active.push_back(r);
            }
            {
                std::lock_guard<std::mutex> lk(mu);
                n_active = (int32_t)active.size();
            }
            if (!admitted.empty()) {
                group.inst.clear();
                for (Request *r : active) group.inst.push_back(r->inst.get());
                choose_schedule();
                group.rebuild(stream);
                group.start(fresh, stream);
            }
            // one step of every admitted request
            group.step(iters_per_step, stream, false);
            const int n = (int)active.size();
            done.assign(n, 0);
            launch_gather_done(group.desc, n, group.done, stream);
            hip_check(hipMemcpyAsync(done.data(), group.done, sizeof(int32_t) * n, hipMemcpyDeviceToHost, stream), "D2H");
            hip_check(hipStreamSynchronize(stream), "hipStreamSynchronize");
            // retire finished requests
            std::vector<Request *> keep, gone;
            for (int i = 0; i < n; ++i) (done[i] ? gone : keep).push_back(active[i]);
            for (Request *r : gone) {
                int status = GOCP_OK;
                try {
                    copy_record(r, stream);
                } catch (const Error &e) {
                    status = e.code;
                }
                r->inst.reset();   // the stream is idle: the workspace can be freed
                std::lock_guard<std::mutex> lk(mu);
                bytes_in_use -= r->footprint;
                finish(r, status);
            }
            {
                std::lock_guard<std::mutex> lk(mu);
                ++steps;
            }
            if (!gone.empty()) {
                active.swap(keep);
                {
                    std::lock_guard<std::mutex> lk(mu);
                    n_active = (int32_t)active.size();
                }
                group.inst.clear();
                for (Request *r : active) group.inst.push_back(r->inst.get());
                choose_schedule();
                group.rebuild(stream);
                cv.notify_all();
            }
        }
    } catch (const std::exception &e) {
        std::lock_guard<std::mutex> lk(mu);
        worker_error = e.what();
    }
    // cancel whatever is left
    std::lock_guard<std::mutex> lk(mu);
    (void)hipStreamSynchronize(stream);
    for (Request *r : active) {
        r->inst.reset();
        if (!r->finished) finish(r, worker_error.empty() ? GOCP_ECANCELED : GOCP_EDEVICE);
    }
    active.clear();
    n_active = 0;
    for (Request *r : queue)
        if (!r->finished) finish(r, worker_error.empty() ? GOCP_ECANCELED : GOCP_EDEVICE);
    queue.clear();
    bytes_in_use = 0;
    cv.notify_all();
}

using namespace gocp;

extern "C" {

int gocp_request_footprint(int n_qubits, int n_ops, int n_strings, int64_t n_terms, int n_classes,
                           int max_iter, int dtype, int64_t *bytes) {
    GOCP_GUARD_BEGIN
    if (!bytes) throw Error(GOCP_EINVAL, "null output");
    if (n_qubits < 1 || n_qubits > kMaxQubits) throw Error(GOCP_ENOTSUP, "qubit count out of range");
    check_dtype(dtype);
    const InstPlan ip = plan_instance(n_qubits, n_ops, max_iter, dtype, true);
    *bytes = (int64_t)(ip.bytes + (size_t)n_terms * sizeof(HTerm) + (size_t)n_classes * sizeof(HClass) +
                       2 * ((size_t)n_strings * sizeof(HTerm) + (size_t)n_ops * sizeof(HClass)) +
                       (size_t)n_ops * sizeof(double));
    return GOCP_OK;
    GOCP_GUARD_END
}

int gocp_server_create(gocp_ctx *ctx, int64_t hbm_budget_bytes, int32_t max_slots, int dtype,
                       int32_t iters_per_step, int32_t amps_per_lane, gocp_server **out) {
    GOCP_GUARD_BEGIN
    check_ctx(ctx);
    check_dtype(dtype);
    if (!out || hbm_budget_bytes <= 0 || max_slots <= 0 || iters_per_step <= 0)
        throw Error(GOCP_EINVAL, "invalid server parameters");
    if (amps_per_lane != 0 && amps_per_lane != 1 && amps_per_lane != 2 && amps_per_lane != 4)
        throw Error(GOCP_EINVAL, "amps_per_lane must be 0 (adaptive), 1, 2 or 4");
    std::unique_ptr<gocp_server> s(new gocp_server());
    s->ctx = ctx;
    s->dtype = dtype;
    s->budget = (size_t)hbm_budget_bytes;
    s->max_slots = max_slots;
    s->iters_per_step = iters_per_step;
    hip_check(hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking), "hipStreamCreate");
    s->group.ctx = ctx;
    s->group.dtype = dtype;
    s->schedule = amps_per_lane;
    s->group.R = amps_per_lane ? amps_per_lane : 1;
    gocp_server *raw = s.get();
    s->worker = std::thread([raw] { raw->run(); });
    *out = s.release();
    return GOCP_OK;
    GOCP_GUARD_END
}

int gocp_server_submit(gocp_server *s, const gocp_ham *hh, const gocp_pool *pp, int32_t max_iter,
                       double grad_tol, uint64_t *ticket) {
    GOCP_GUARD_BEGIN
    if (!s || !ticket) throw Error(GOCP_EINVAL, "null argument");
    const Ham *h = as_ham(hh);
    const Pool *p = as_pool(pp);
    if (h->n_qubits != p->n_qubits) throw Error(GOCP_ESHAPE, "Hamiltonian and pool act on different qubit counts");
    if (max_iter < 0) throw Error(GOCP_EINVAL, "negative max_iter");
    std::unique_ptr<Request> r(new Request());
    r->h = h;
    r->p = p;
    r->max_iter = max_iter;
    r->tol = grad_tol;
    r->hf = hf_index(p->n_qubits, p->n_electrons, p->mapping);
    r->footprint = plan_instance(h->n_qubits, p->n_ops(), max_iter, s->dtype, true).bytes + table_bytes(h, p);
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) throw Error(GOCP_EINVAL, "server is shutting down");
    if (!s->worker_error.empty()) throw Error(GOCP_EDEVICE, "server worker failed: " + s->worker_error);
    r->ticket = s->next_ticket++;
    r->t_submit = now_ns();
    *ticket = r->ticket;
    s->queue.push_back(r.get());
    s->requests[r->ticket] = std::move(r);
    s->cv.notify_all();
    return GOCP_OK;
    GOCP_GUARD_END
}

int gocp_server_poll(gocp_server *s, uint64_t ticket, gocp_adapt_result *res, gocp_request_info *info) {
    GOCP_GUARD_BEGIN
    if (!s) throw Error(GOCP_EINVAL, "null server");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->requests.find(ticket);
    if (it == s->requests.end()) throw Error(GOCP_EINVAL, "unknown ticket");
    Request *r = it->second.get();
    if (!r->finished) return GOCP_EBUSY;
    if (info) {
        info->status = r->status;
        info->n_qubits = r->h->n_qubits;
        info->t_submit_ns = r->t_submit;
        info->t_admit_ns = r->t_admit;
        info->t_done_ns = r->t_done;
    }
    if (res && r->status == GOCP_OK) {
        if (!res->energies || !res->ops || !res->thetas || !res->gnorms)
            throw Error(GOCP_EINVAL, "null result arrays");
        const int n = r->n_iter, nscr = n + (r->converged ? 1 : 0);
        res->n_iter = n;
        res->converged = r->converged;
        std::copy(r->energies.begin(), r->energies.begin() + n + 1, res->energies);
        std::copy(r->ops.begin(), r->ops.begin() + n, res->ops);
        std::copy(r->thetas.begin(), r->thetas.begin() + n, res->thetas);
        std::copy(r->gnorms.begin(), r->gnorms.begin() + nscr, res->gnorms);
        if (res->gmax) std::copy(r->gmax.begin(), r->gmax.begin() + nscr, res->gmax);
        if (res->substeps) std::copy(r->substeps.begin(), r->substeps.begin() + n, res->substeps);
    }
    const int status = r->status;
    s->requests.erase(it);
    return status;
    GOCP_GUARD_END
}

int gocp_server_stats(gocp_server *s, int32_t *active, int32_t *queued, int64_t *completed,
                      int64_t *bytes_in_use, int64_t *steps) {
    GOCP_GUARD_BEGIN
    if (!s) throw Error(GOCP_EINVAL, "null server");
    std::lock_guard<std::mutex> lk(s->mu);
    if (active) *active = s->n_active;
    if (queued) *queued = (int32_t)s->queue.size();
    if (completed) *completed = s->completed;
    if (bytes_in_use) *bytes_in_use = (int64_t)s->bytes_in_use;
    if (steps) *steps = s->steps;
    if (!s->worker_error.empty()) throw Error(GOCP_EDEVICE, "server worker failed: " + s->worker_error);
    return GOCP_OK;
    GOCP_GUARD_END
}

int gocp_server_destroy(gocp_server *s) {
    GOCP_GUARD_BEGIN
    if (!s) return GOCP_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv.notify_all();
    if (s->worker.joinable()) s->worker.join();
    (void)hipSetDevice(s->ctx->device);
    (void)hipStreamDestroy(s->stream);
    delete s;
    return GOCP_OK;
    GOCP_GUARD_END
}

}  // extern "C"
