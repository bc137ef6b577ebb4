// Serving runtime: continuous batching of ADAPT solves on one device.
//
// Requests (a Hamiltonian, a pool, a convergence threshold) are queued by
// gocp_server_submit from any thread.  A worker thread owns the device side.
//
// * Memory.  The server allocates everything it uses when it is created: one
//   device arena of the HBM budget, two buffers for the lock-step group's
//   descriptor and row tables, and pinned flag buffers.  An admitted request
//   takes one block of the arena holding its workspace and its own copy of
//   its Hamiltonian's and pool's device tables (copied from the handles'
//   pinned table images), so the bytes in use are exactly the blocks of the
//   admitted requests, and the worker loop never calls hipMalloc or hipFree.
// * Admission.  In arrival order, while a slot is free and the request's
//   block fits in the arena (first fit); a request larger than the arena
//   fails with GOCP_ENOMEM at once.
// * Steps.  All admitted requests advance together, `iters_per_step` ADAPT
//   iterations per step, one launch per kernel for the whole set (the
//   lock-step group of the batched form).  Two steps are kept queued on the
//   stream: while the device runs step k + 1, the worker waits for step k's
//   event (polling), reads its done flags, starts the record copies of the
//   requests that finished, admits waiting requests into free blocks and
//   rebuilds the group's tables into the buffer step k + 1 does not use.  A
//   retired request's block is released when its record copy (queued after
//   every step that still lists it) has completed.
// Every request computes exactly what adapt_solve computes for it alone with
// the same schedule.

#include <chrono>
#include <condition_variable>
#include <cstdlib>
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

size_t al256(size_t b) { return (b + 255) & ~(size_t)255; }

// First-fit allocator over the arena's byte range (blocks of 256-byte
// multiples, free neighbours merged).
struct ArenaAlloc {
    size_t cap = 0, used = 0;
    std::map<size_t, size_t> free_;     // offset -> size
    void init(size_t c) {
        cap = c;
        used = 0;
        free_.clear();
        if (c) free_[0] = c;
    }
    bool alloc(size_t n, size_t &off) {
        n = al256(n);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < n) continue;
            off = it->first;
            const size_t rest = it->second - n;
            free_.erase(it);
            if (rest) free_[off + n] = rest;
            used += n;
            return true;
        }
        return false;
    }
    void release(size_t off, size_t n) {
        n = al256(n);
        used -= n;
        auto it = free_.emplace(off, n).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
};

struct Request {
    uint64_t ticket = 0;
    const Ham *h = nullptr;
    const Pool *p = nullptr;
    int max_iter = 0;
    double tol = 0.0;
    uint64_t hf = 0;
    std::shared_ptr<const TableImage> himg, pimg;   // built at submission
    InstPlan ip;                                    // workspace layout (own state buffer)
    size_t footprint = 0;                           // workspace + both table copies
    size_t off = 0;                                 // block in the arena while admitted
    bool placed = false, retiring = false;
    int64_t t_submit = 0, t_admit = 0, t_done = 0;
    int status = GOCP_EBUSY;
    bool finished = false;
    std::unique_ptr<Instance> inst;
    DeviceHam dh;
    DevicePool dp;
    // record: [state | histories] copied to pinned host memory at retirement
    char *rec_host = nullptr;
    size_t rec_bytes = 0;
    hipEvent_t rec_ev = nullptr;
    int n_iter = 0, converged = 0;
    std::vector<double> energies, thetas, gnorms, gmax;
    std::vector<int32_t> ops, substeps;
    ~Request() {
        if (rec_host) (void)hipHostFree(rec_host);
        if (rec_ev) (void)hipEventDestroy(rec_ev);
    }
};

// A queued step: its completion event, the done flags it copies back, and the
// members it advanced (in group order).
struct Flight {
    hipEvent_t ev = nullptr;
    int32_t *flags = nullptr;       // pinned, max_slots entries
    std::vector<Request *> members;
};

}  // namespace
}  // namespace gocp

struct gocp_server {
    gocp_ctx *ctx = nullptr;
    hipStream_t stream = nullptr;
    int dtype = 0, max_slots = 1, iters_per_step = 1;
    int schedule = 1;     // amplitudes per lane, or 0: chosen from the active set
    size_t budget = 0;
    char *arena = nullptr;
    char *tables[2] = {nullptr, nullptr};
    gocp::Flight flight[2];
    std::mutex mu;
    std::condition_variable cv;
    // guarded by mu: the queue, the ticket map, the counters, worker_error,
    // stop, and the arena allocator (read by gocp_server_stats)
    std::deque<gocp::Request *> queue;
    std::map<uint64_t, std::unique_ptr<gocp::Request>> requests;
    gocp::ArenaAlloc alloc;
    int32_t n_active = 0;
    uint64_t next_ticket = 1;
    int64_t completed = 0, steps = 0;
    bool stop = false;
    std::string worker_error;
    int64_t fail_admission_at = 0;    // test hook: the n-th admission fails (0: never)
    int64_t admissions = 0;
    // worker only
    std::vector<gocp::Request *> active;      // members of the group, in group order
    std::vector<gocp::Request *> retiring;    // record copies in flight
    gocp::Group group;
    std::thread worker;

    void finish(gocp::Request *r, int status) {   // caller holds mu
        if (r->finished) return;
        r->status = status;
        r->finished = true;
        r->t_done = gocp::now_ns();
        ++completed;
    }
    void choose_schedule();
    bool admit(std::vector<int> &fresh);
    void enqueue_step(gocp::Flight &f);
    void retire(gocp::Request *r);
    void finish_records(bool wait);
    void run();
    void release_all();
};

namespace gocp {
namespace {

// Parse a finished request's record (state and histories) from its pinned copy.
void parse_record(Request *r) {
    const InstPlan &ip = r->ip;
    const char *b = r->rec_host;
    AdaptState st;
    std::memcpy(&st, b, sizeof(st));
    const int n = r->max_iter, nit = std::min(std::max(st.iter, 0), n);
    const int nscr = std::min(nit + (st.converged ? 1 : 0), n + 1);
    r->n_iter = nit;
    r->converged = st.converged;
    r->energies.assign(n + 1, 0.0);
    r->thetas.assign(std::max(n, 1), 0.0);
    r->gnorms.assign(n + 1, 0.0);
    r->gmax.assign(n + 1, 0.0);
    r->ops.assign(std::max(n, 1), 0);
    r->substeps.assign(std::max(n, 1), 0);
    auto at = [&](size_t o) { return b + (o - ip.o_st); };
    std::memcpy(r->energies.data(), at(ip.o_he), (size_t)(nit + 1) * 8);
    if (nit > 0) {
        std::memcpy(r->ops.data(), at(ip.o_hop), (size_t)nit * 4);
        std::memcpy(r->thetas.data(), at(ip.o_hth), (size_t)nit * 8);
        std::memcpy(r->substeps.data(), at(ip.o_hns), (size_t)nit * 4);
    }
    if (nscr > 0) {
        std::memcpy(r->gnorms.data(), at(ip.o_hgn), (size_t)nscr * 8);
        std::memcpy(r->gmax.data(), at(ip.o_hgm), (size_t)nscr * 8);
    }
    if (st.status) throw Error(st.status, "non-finite value during ADAPT");
}

}  // namespace
}  // namespace gocp

// Adaptive schedule: one amplitude per lane while the active set has fewer
// than four tiles of 64 amplitudes per compute unit (the launches are then
// latency-bound and more tiles keep more units busy); otherwise four, which
// cuts the work per amplitude.  The compacted H v, H w launch's parts follow
// the group's parts rule.
void gocp_server::choose_schedule() {
    if (schedule != 0) return;
    long tiles = 0;
    for (gocp::Request *r : active) tiles += gocp::tiles_for(r->ip.n_qubits, 1);
    group.R = tiles < 4L * ctx->n_cu ? 1 : 4;
    group.P = group.parts_rule();
}

// Admit queued requests in arrival order while a slot is free and a block
// fits; each admitted request's tables are copied into its block and its
// instance initialised there (stream-ordered).  A request whose
// initialisation fails ends with that error and gives its block back.
// Returns whether any request was admitted; fresh gets their group indices.
bool gocp_server::admit(std::vector<int> &fresh) {
    using namespace gocp;
    bool any = false;
    for (;;) {
        Request *r = nullptr;
        int64_t nth = 0;
        {
            std::lock_guard<std::mutex> lk(mu);
            if (stop || queue.empty() || (int)active.size() >= max_slots) break;
            r = queue.front();
            if (r->footprint > alloc.cap) {           // can never fit
                queue.pop_front();
                finish(r, GOCP_ENOMEM);
                continue;
            }
            size_t off = 0;
            if (!alloc.alloc(r->footprint, off)) break;   // wait for room, in order
            queue.pop_front();
            r->off = off;
            r->placed = true;
            nth = ++admissions;
        }
        try {
            if (fail_admission_at > 0 && nth == fail_admission_at)
                throw Error(GOCP_EDEVICE, "admission failure requested by GOCP_TEST_FAIL_ADMISSION");
            char *blk = arena + r->off;
            char *th = blk + al256(r->ip.bytes), *tp = th + r->himg->bytes;
            hip_check(hipMemcpyAsync(th, r->himg->host, r->himg->bytes, hipMemcpyHostToDevice, stream), "H2D tables");
            hip_check(hipMemcpyAsync(tp, r->pimg->host, r->pimg->bytes, hipMemcpyHostToDevice, stream), "H2D tables");
            r->dh = place_ham(*r->himg, th, ctx->device);
            r->dp = place_pool(*r->pimg, tp, ctx->device);
            r->inst.reset(instance_create(ctx, r->h, r->p, nullptr, dtype, r->max_iter, r->tol, r->hf, stream, blk,
                                          &r->dh, &r->dp));
        } catch (const Error &e) {
            r->inst.reset();
            std::lock_guard<std::mutex> lk(mu);
            alloc.release(r->off, r->footprint);
            r->placed = false;
            finish(r, e.code);
            continue;
        }
        r->t_admit = now_ns();
        fresh.push_back((int)active.size());
        active.push_back(r);
        any = true;
    }
    return any;
}

// Queue one step of every active request, then the gather of their done
// flags into the step's pinned buffer and the step's event.
void gocp_server::enqueue_step(gocp::Flight &f) {
    using namespace gocp;
    group.step(iters_per_step, stream, false);
    const int n = (int)active.size();
    launch_gather_done(group.desc, n, group.done, stream);
    hip_check(hipMemcpyAsync(f.flags, group.done, sizeof(int32_t) * n, hipMemcpyDeviceToHost, stream), "D2H flags");
    hip_check(hipEventRecord(f.ev, stream), "hipEventRecord");
    f.members = active;
}

// A request that finished: queue the copy of its state and histories (after
// every step queued so far, which may still list it) and its event.
void gocp_server::retire(gocp::Request *r) {
    using namespace gocp;
    r->retiring = true;
    r->inst->finalized = true;     // served states are not handed back
    hip_check(hipMemcpyAsync(r->rec_host, r->inst->mem + r->ip.o_st, r->rec_bytes, hipMemcpyDeviceToHost, stream),
              "D2H record");
    hip_check(hipEventRecord(r->rec_ev, stream), "hipEventRecord");
    retiring.push_back(r);
}

// Requests whose record copy has completed: parse the record, release the
// block, and mark them finished (all of them, waiting, with `wait`).
void gocp_server::finish_records(bool wait) {
    using namespace gocp;
    std::vector<Request *> keep;
    for (Request *r : retiring) {
        hipError_t q = wait ? hipEventSynchronize(r->rec_ev) : hipEventQuery(r->rec_ev);
        if (q == hipErrorNotReady) {
            keep.push_back(r);
            continue;
        }
        int status = GOCP_OK;
        if (q != hipSuccess) {
            status = GOCP_EDEVICE;
        } else {
            try {
                parse_record(r);
            } catch (const Error &e) {
                status = e.code;
            }
        }
        r->inst.reset();
        std::lock_guard<std::mutex> lk(mu);
        alloc.release(r->off, r->footprint);
        r->placed = false;
        finish(r, status);
        if (q != hipSuccess && q != hipErrorNotReady) hip_check(q, "record copy");
    }
    retiring.swap(keep);
    if (keep.size() != retiring.size()) cv.notify_all();
}

void gocp_server::run() {
    using namespace gocp;
    std::deque<Flight *> inflight;
    try {
        hip_check(hipSetDevice(ctx->device), "hipSetDevice");
        int next = 0;
        bool removed = false;
        for (;;) {
            {
                std::lock_guard<std::mutex> lk(mu);
                if (stop) break;
            }
            finish_records(false);
            // admissions and the group rebuild, with at most one step queued
            // (it reads the current table buffer; the rebuild writes the other)
            if (inflight.size() <= 1) {
                bool changed = removed;
                if (removed) {          // retired members leave the group first, freeing their slots
                    std::vector<Request *> keep;
                    for (Request *r : active)
                        if (!r->retiring) keep.push_back(r);
                    active.swap(keep);
                    removed = false;
                }
                std::vector<int> fresh;
                if (admit(fresh)) changed = true;
                if (changed) {
                    group.inst.clear();
                    for (Request *r : active) group.inst.push_back(r->inst.get());
                    choose_schedule();
                    group.rebuild(stream);
                    if (!fresh.empty()) group.start(fresh, stream);
                    std::lock_guard<std::mutex> lk(mu);
                    n_active = (int32_t)active.size();
                }
            }
            while (inflight.size() < 2 && !active.empty()) {
                Flight &f = flight[next];
                next ^= 1;
                enqueue_step(f);
                inflight.push_back(&f);
            }
            if (inflight.empty()) {
                std::unique_lock<std::mutex> lk(mu);
                if (!retiring.empty()) {
                    lk.unlock();
                    finish_records(true);
                    continue;
                }
                cv.notify_all();
                cv.wait(lk, [&] { return stop || !queue.empty(); });
                continue;
            }
            // wait for the oldest step (polling: records of earlier
            // retirements are finished meanwhile)
            Flight *f = inflight.front();
            hipError_t q;
            while ((q = hipEventQuery(f->ev)) == hipErrorNotReady) {
                finish_records(false);
                std::this_thread::sleep_for(std::chrono::microseconds(20));
            }
            hip_check(q, "step");
            inflight.pop_front();
            for (size_t i = 0; i < f->members.size(); ++i) {
                Request *r = f->members[i];
                if (f->flags[i] && !r->retiring) {
                    retire(r);
                    removed = true;
                }
            }
            std::lock_guard<std::mutex> lk(mu);
            ++steps;
        }
        (void)hipStreamSynchronize(stream);
        finish_records(true);
    } catch (const std::exception &e) {
        std::lock_guard<std::mutex> lk(mu);
        worker_error = e.what();
    }
    release_all();
}

// End every unfinished request (GOCP_ECANCELED on shutdown, GOCP_EDEVICE
// after a worker error) once the stream is idle.
void gocp_server::release_all() {
    using namespace gocp;
    (void)hipStreamSynchronize(stream);
    std::lock_guard<std::mutex> lk(mu);
    const int code = worker_error.empty() ? GOCP_ECANCELED : GOCP_EDEVICE;
    for (Request *r : retiring) {
        r->inst.reset();
        if (r->placed) alloc.release(r->off, r->footprint);
        r->placed = false;
        finish(r, code);
    }
    retiring.clear();
    for (Request *r : active) {
        r->inst.reset();
        if (r->placed) alloc.release(r->off, r->footprint);
        r->placed = false;
        finish(r, code);
    }
    active.clear();
    n_active = 0;
    for (Request *r : queue) finish(r, code);
    queue.clear();
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
    // an estimate from the sizes alone (the exact block, with the tables'
    // padding and stage layout, is known once the handles' images are built)
    const InstPlan ip = plan_instance(n_qubits, n_ops, max_iter, dtype, true);
    *bytes = (int64_t)(ip.bytes + (size_t)n_terms * sizeof(HTerm) + (size_t)n_classes * sizeof(HClass) +
                       2 * ((size_t)n_strings * sizeof(HTerm) + (size_t)n_ops * sizeof(HClass)) +
                       (size_t)n_ops * sizeof(double));
    return GOCP_OK;
    GOCP_GUARD_END
}

int gocp_request_bytes(const gocp_ham *hh, const gocp_pool *pp, int32_t max_iter, int dtype, int64_t *bytes) {
    GOCP_GUARD_BEGIN
    if (!bytes) throw Error(GOCP_EINVAL, "null output");
    const Ham *h = as_ham(hh);
    const Pool *p = as_pool(pp);
    if (h->n_qubits != p->n_qubits) throw Error(GOCP_ESHAPE, "Hamiltonian and pool act on different qubit counts");
    if (max_iter < 0) throw Error(GOCP_EINVAL, "negative max_iter");
    check_dtype(dtype);
    const InstPlan ip = plan_instance(h->n_qubits, p->n_ops(), max_iter, dtype, true);
    *bytes = (int64_t)(al256(ip.bytes) + ham_image(*h)->bytes + pool_image(*p)->bytes);
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
    s->budget = al256((size_t)hbm_budget_bytes);
    s->max_slots = max_slots;
    s->iters_per_step = iters_per_step;
    s->schedule = amps_per_lane;
    if (const char *e = std::getenv("GOCP_TEST_FAIL_ADMISSION")) s->fail_admission_at = std::atoll(e);
    // everything the worker will use, allocated now: the arena, two group
    // table buffers (rows scale with the states' amplitudes, at most about
    // 0.4 bytes per amplitude against at least 40 bytes of workspace, plus
    // a few KiB per member), pinned flag buffers and events
    auto cleanup = [&]() {
        for (int k = 0; k < 2; ++k) {
            if (s->tables[k]) (void)hipFree(s->tables[k]);
            if (s->flight[k].flags) (void)hipHostFree(s->flight[k].flags);
            if (s->flight[k].ev) (void)hipEventDestroy(s->flight[k].ev);
        }
        if (s->arena) (void)hipFree(s->arena);
        if (s->stream) (void)hipStreamDestroy(s->stream);
    };
    try {
        hip_check(hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking), "hipStreamCreate");
        hip_check(hipMalloc(&s->arena, s->budget), "hipMalloc server arena");
        const size_t tcap = al256(s->budget / 64 + (size_t)max_slots * 4096 + ((size_t)1 << 16));
        for (int k = 0; k < 2; ++k) {
            hip_check(hipMalloc(&s->tables[k], tcap), "hipMalloc group tables");
            hip_check(hipHostMalloc(reinterpret_cast<void **>(&s->flight[k].flags), sizeof(int32_t) * max_slots, 0),
                      "hipHostMalloc flags");
            hip_check(hipEventCreateWithFlags(&s->flight[k].ev, hipEventDisableTiming), "hipEventCreate");
        }
        s->group.ext[0] = s->tables[0];
        s->group.ext[1] = s->tables[1];
        s->group.ext_cap = tcap;
    } catch (...) {
        cleanup();
        throw;
    }
    s->alloc.init(s->budget);
    s->group.ctx = ctx;
    s->group.dtype = dtype;
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
    hip_check(hipSetDevice(s->ctx->device), "hipSetDevice");
    std::unique_ptr<Request> r(new Request());
    r->h = h;
    r->p = p;
    r->max_iter = max_iter;
    r->tol = grad_tol;
    r->hf = hf_index(p->n_qubits, p->n_electrons, p->mapping);
    // the table images and the record buffer are made here, in the caller's
    // thread, so that the worker only copies them
    r->himg = ham_image(*h);
    r->pimg = pool_image(*p);
    r->ip = plan_instance(h->n_qubits, p->n_ops(), max_iter, s->dtype, true);
    r->footprint = al256(r->ip.bytes) + r->himg->bytes + r->pimg->bytes;
    r->rec_bytes = r->ip.o_g - r->ip.o_st;
    hip_check(hipHostMalloc(reinterpret_cast<void **>(&r->rec_host), r->rec_bytes, 0), "hipHostMalloc record");
    hip_check(hipEventCreateWithFlags(&r->rec_ev, hipEventDisableTiming), "hipEventCreate");
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
    std::unique_ptr<Request> gone;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->requests.find(ticket);
    if (it == s->requests.end()) throw Error(GOCP_EINVAL, "unknown ticket");
    Request *r = it->second.get();
    if (!r->finished) {
        if (!s->worker_error.empty()) throw Error(GOCP_EDEVICE, "server worker failed: " + s->worker_error);
        return GOCP_EBUSY;
    }
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
    gone = std::move(it->second);
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
    if (bytes_in_use) *bytes_in_use = (int64_t)s->alloc.used;
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
    (void)hipStreamSynchronize(s->stream);
    s->requests.clear();
    for (int k = 0; k < 2; ++k) {
        (void)hipFree(s->tables[k]);
        (void)hipHostFree(s->flight[k].flags);
        (void)hipEventDestroy(s->flight[k].ev);
    }
    s->group.inst.clear();
    (void)hipFree(s->arena);
    (void)hipStreamDestroy(s->stream);
    delete s;
    return GOCP_OK;
    GOCP_GUARD_END
}

}  // extern "C"
