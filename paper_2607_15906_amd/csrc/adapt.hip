// ADAPT runs on the device: single runs, lock-step batches of instances, and
// the building blocks of the serving runtime.
//
// An Instance owns the device workspace of one ADAPT problem (state, sigma,
// line-search vectors, partial sums, iteration state and history).  A Group
// is a set of instances advanced together: every kernel of an iteration is
// launched once for the whole group, over a table of (instance, tile) work
// items, so instances of different sizes share each launch.  A group can
// capture its iteration (and a chunk of eight iterations) into hipGraphs that
// are replayed on the caller's stream.

#include "adapt.h"

#include <map>
#include <mutex>
#include <string>

namespace gocp {

namespace {
std::mutex g_tune_mu;
std::map<std::string, int> g_tune;

std::string tune_key(std::vector<int> q, int dtype) {
    std::sort(q.begin(), q.end());
    std::string k = std::to_string(dtype) + ":";
    for (int v : q) k += std::to_string(v) + ",";
    return k;
}
}  // namespace

int autotune_cached(const std::vector<int> &qubits, int dtype) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find(tune_key(qubits, dtype));
    return it == g_tune.end() ? 0 : it->second;
}

void autotune_store(const std::vector<int> &qubits, int dtype, int R) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[tune_key(qubits, dtype)] = R;
}

void Group::choose_schedule(int schedule, hipStream_t s) {
    const int r = schedule & 0xff, p = schedule >> 8;
    if ((r == 1 || r == 2 || r == 4) && (p == 0 || p == kHvwPartsLo)) {
        R = r;
        P = p ? p : kHvwPartsHi;
        rebuild(s);
        return;
    }
    if (schedule != 0)
        throw Error(GOCP_EINVAL, "schedule must be 0 (autotune) or 1, 2 or 4 amplitudes per lane, plus 256 x 4 for "
                                 "four H v, H w parts");
    P = parts_rule();
    std::vector<int> q;
    for (Instance *in : inst) q.push_back(in->ip.n_qubits);
    int best = autotune_cached(q, dtype);
    if (best == 0) {
        // each candidate: one warm-up pass, then the fastest of three timed
        // passes; a larger blocking must beat the best so far by 2 %
        double best_ms = 0.0;
        for (int cand : {1, 2, 4}) {
            R = cand;
            rebuild(s);
            (void)time_tile_kernels(s, 1);
            double ms = time_tile_kernels(s, 5);
            for (int trial = 1; trial < 3; ++trial) ms = std::min(ms, time_tile_kernels(s, 5));
            if (best == 0 || ms < 0.98 * best_ms) {
                best = cand;
                best_ms = ms;
            }
        }
        autotune_store(q, dtype, best);
    }
    R = best;
    rebuild(s);
}

// Copy one instance's iteration record to the caller's arrays (synchronises).
void read_result(Instance *in, hipStream_t s, gocp_adapt_result *res, AdaptState *out_state) {
    AdaptState st;
    hip_check(hipMemcpyAsync(&st, in->mem + in->ip.o_st, sizeof(st), hipMemcpyDeviceToHost, s), "D2H");
    hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");
    if (out_state) *out_state = st;
    if (st.status) throw Error(st.status, "non-finite value during ADAPT");
    if (!res) return;
    if (!res->energies || !res->ops || !res->thetas || !res->gnorms)
        throw Error(GOCP_EINVAL, "null result arrays");
    const int n = st.iter;
    const int nscr = n + (st.converged ? 1 : 0);
    const InstPlan &ip = in->ip;
    char *b = in->mem;
    res->n_iter = n;
    res->converged = st.converged;
    hip_check(hipMemcpyAsync(res->energies, b + ip.o_he, (size_t)(n + 1) * 8, hipMemcpyDeviceToHost, s), "D2H");
    if (n > 0) {
        hip_check(hipMemcpyAsync(res->ops, b + ip.o_hop, (size_t)n * 4, hipMemcpyDeviceToHost, s), "D2H");
        hip_check(hipMemcpyAsync(res->thetas, b + ip.o_hth, (size_t)n * 8, hipMemcpyDeviceToHost, s), "D2H");
        if (res->substeps)
            hip_check(hipMemcpyAsync(res->substeps, b + ip.o_hns, (size_t)n * 4, hipMemcpyDeviceToHost, s), "D2H");
    }
    if (nscr > 0) {
        hip_check(hipMemcpyAsync(res->gnorms, b + ip.o_hgn, (size_t)nscr * 8, hipMemcpyDeviceToHost, s), "D2H");
        if (res->gmax)
            hip_check(hipMemcpyAsync(res->gmax, b + ip.o_hgm, (size_t)nscr * 8, hipMemcpyDeviceToHost, s), "D2H");
    }
    hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");
}

// Advance a group until every member is done or max_iter iterations have
// been issued.  The done flags are copied back asynchronously after every
// chunk and inspected two chunks later, so the device queue never drains
// while the host checks for convergence.
void run_to_completion(Group &g, int max_iter, bool use_graph, hipStream_t s) {
    const int n = (int)g.inst.size();
    if (n == 0 || max_iter <= 0) return;
    int *flags = nullptr;
    const int ring = 2;
    hip_check(hipHostMalloc(reinterpret_cast<void **>(&flags), sizeof(int) * n * ring, 0), "hipHostMalloc");
    hipEvent_t ev[ring] = {nullptr, nullptr};
    bool pending[ring] = {false, false};
    try {
        for (int k = 0; k < ring; ++k)
            hip_check(hipEventCreateWithFlags(&ev[k], hipEventDisableTiming), "hipEventCreate");
        int issued = 0, chunk = 0;
        while (issued < max_iter) {
            const int slot = chunk % ring;
            if (pending[slot]) {
                hip_check(hipEventSynchronize(ev[slot]), "hipEventSynchronize");
                pending[slot] = false;
                bool all = true;
                for (int i = 0; i < n; ++i) all = all && flags[slot * n + i];
                if (all) break;
            }
            const int m = std::min(Group::kChunk, max_iter - issued);
            g.step(m, s, use_graph);
            issued += m;
            launch_gather_done(g.desc, n, g.done, s);
            hip_check(hipMemcpyAsync(&flags[slot * n], g.done, sizeof(int) * n, hipMemcpyDeviceToHost, s), "D2H");
            hip_check(hipEventRecord(ev[slot], s), "hipEventRecord");
            pending[slot] = true;
            ++chunk;
        }
        hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");
    } catch (...) {
        for (int k = 0; k < ring; ++k)
            if (ev[k]) (void)hipEventDestroy(ev[k]);
        (void)hipHostFree(flags);
        throw;
    }
    for (int k = 0; k < ring; ++k) (void)hipEventDestroy(ev[k]);
    (void)hipHostFree(flags);
}

}  // namespace gocp

struct gocp_batch {
    gocp::Group group;
    std::vector<std::unique_ptr<gocp::Instance>> owned;
    int max_iter = 0;
    bool use_graph = true;
    int issued = 0;
    // events of gocp_batch_step_timed, created with the batch so that a timed
    // call creates and destroys none: two per sampled launch, without the
    // system-scope fence (timing only: no cache writeback and invalidation
    // around the sampled kernel), and the two ends of the timed region
    std::vector<hipEvent_t> tev;
    hipEvent_t tend[2] = {nullptr, nullptr};
    ~gocp_batch() {
        for (hipEvent_t e : tev)
            if (e) (void)hipEventDestroy(e);
        for (hipEvent_t e : tend)
            if (e) (void)hipEventDestroy(e);
    }
};

using namespace gocp;

extern "C" {

int adapt_solve(gocp_ctx *ctx, const gocp_ham *hh, const gocp_pool *pp, void *psi_dev, int dtype,
                const gocp_adapt_params *params, gocp_adapt_result *res) {
    GOCP_GUARD_BEGIN
    check_ctx(ctx);
    if (!params || !res) throw Error(GOCP_EINVAL, "null params or result");
    if (!psi_dev) throw Error(GOCP_EINVAL, "null state pointer");
    hipStream_t s = ctx->user_stream;
    std::unique_ptr<Instance> in(instance_create(ctx, as_ham(hh), as_pool(pp), psi_dev, dtype,
                                                 params->max_iter, params->grad_tol, 0, s));
    Group g;
    g.ctx = ctx;
    g.dtype = dtype;
    g.inst.push_back(in.get());
    g.choose_schedule(params->schedule, s);
    g.start({0}, s);
    run_to_completion(g, params->max_iter, params->use_graph != 0, s);
    g.finalize({0}, s);
    read_result(in.get(), s, res, nullptr);
    return GOCP_OK;
    GOCP_GUARD_END
}

int gocp_batch_create(gocp_ctx *ctx, int32_t n, const gocp_ham *const *hams,
                      const gocp_pool *const *pools, void *const *psi_dev, int dtype,
                      const gocp_adapt_params *params, gocp_batch **out) {
    GOCP_GUARD_BEGIN
    check_ctx(ctx);
    if (!out || !params || n <= 0 || !hams || !pools || !psi_dev)
        throw Error(GOCP_EINVAL, "null argument or empty batch");
    hipStream_t s = ctx->user_stream;
    std::unique_ptr<gocp_batch> b(new gocp_batch());
    b->group.ctx = ctx;
    b->group.dtype = dtype;
    b->max_iter = params->max_iter;
    b->use_graph = params->use_graph != 0;
    b->tev.assign(2 * (size_t)std::min(std::max(params->max_iter, 0), 512), nullptr);
    for (hipEvent_t &e : b->tev) hip_check(hipEventCreateWithFlags(&e, hipEventDisableSystemFence), "hipEventCreate");
    for (hipEvent_t &e : b->tend) hip_check(hipEventCreate(&e), "hipEventCreate");
    for (int i = 0; i < n; ++i) {
        if (!psi_dev[i]) throw Error(GOCP_EINVAL, "null state pointer");
        b->owned.emplace_back(instance_create(ctx, as_ham(hams[i]), as_pool(pools[i]), psi_dev[i],
                                              dtype, params->max_iter, params->grad_tol, 0, s));
        b->group.inst.push_back(b->owned.back().get());
    }
    b->group.choose_schedule(params->schedule, s);
    std::vector<int> all(n);
    for (int i = 0; i < n; ++i) all[i] = i;
    b->group.start(all, s);
    *out = b.release();
    return GOCP_OK;
    GOCP_GUARD_END
}

int gocp_batch_step(gocp_batch *b, int32_t n_iter) {
    GOCP_GUARD_BEGIN
    if (!b) throw Error(GOCP_EINVAL, "null batch");
    check_ctx(b->group.ctx);
    if (n_iter < 0) throw Error(GOCP_EINVAL, "negative iteration count");
    b->group.step(n_iter, b->group.ctx->user_stream, b->use_graph);
    b->issued += n_iter;
    return GOCP_OK;
    GOCP_GUARD_END
}

int gocp_batch_step_timed(gocp_batch *b, int32_t n_iter, int32_t kernel, int32_t every,
                          double *total_ms, double *kernel_ms) {
    GOCP_GUARD_BEGIN
    if (!b || !total_ms || !kernel_ms) throw Error(GOCP_EINVAL, "null argument");
    check_ctx(b->group.ctx);
    if (n_iter <= 0 || every <= 0) throw Error(GOCP_EINVAL, "need at least one iteration and every >= 1");
    static const int kids[5] = {K_LINE_VW, K_LINE_HVW, K_TAYLOR, K_ENERGY_SCREEN, K_SCREEN_SUM1};
    if (kernel < 0 || kernel > 4) throw Error(GOCP_EINVAL, "kernel must be 0..4");
    hipStream_t s = b->group.ctx->user_stream;
    // events for the sampled launches and the two ends, from the batch's set
    // (grown here only for more iterations than the batch was created for)
    const int n_samp = (n_iter + every - 1) / every;
    while (b->tev.size() < 2 * (size_t)n_samp) {
        hipEvent_t e = nullptr;
        hip_check(hipEventCreateWithFlags(&e, hipEventDisableSystemFence), "hipEventCreate");
        b->tev.push_back(e);
    }
    const std::vector<hipEvent_t> &ev = b->tev;
    hip_check(hipEventRecord(b->tend[0], s), "hipEventRecord");
    int sampled = 0;
    for (int i = 0; i < n_iter; ++i) {
        for (Instance *in : b->group.inst) in->finalized = false;
        if (i % every == 0) {
            b->group.enqueue_iteration(s, kids[kernel], &ev[2 * sampled]);
            ++sampled;
        } else {
            b->group.enqueue_iteration(s);
        }
    }
    b->group.select_pending(s);
    hip_check(hipEventRecord(b->tend[1], s), "hipEventRecord");
    hip_check(hipEventSynchronize(b->tend[1]), "hipEventSynchronize");
    double k = 0.0;
    for (int i = 0; i < sampled; ++i) {
        float ms = 0.f;
        hip_check(hipEventElapsedTime(&ms, ev[2 * i], ev[2 * i + 1]), "hipEventElapsedTime");
        k += ms;
    }
    float tot = 0.f;
    hip_check(hipEventElapsedTime(&tot, b->tend[0], b->tend[1]), "hipEventElapsedTime");
    b->issued += n_iter;
    *total_ms = tot;
    *kernel_ms = k / sampled;
    return GOCP_OK;
    GOCP_GUARD_END
}

int gocp_batch_run(gocp_batch *b) {
    GOCP_GUARD_BEGIN
    if (!b) throw Error(GOCP_EINVAL, "null batch");
    check_ctx(b->group.ctx);
    const int left = b->max_iter - b->issued;
    run_to_completion(b->group, left, b->use_graph, b->group.ctx->user_stream);
    b->issued = b->max_iter;
    return GOCP_OK;
    GOCP_GUARD_END
}

int gocp_batch_poll(gocp_batch *b, int32_t *n_active) {
    GOCP_GUARD_BEGIN
    if (!b || !n_active) throw Error(GOCP_EINVAL, "null argument");
    check_ctx(b->group.ctx);
    hipStream_t s = b->group.ctx->user_stream;
    const int n = (int)b->group.inst.size();
    std::vector<int32_t> done(n);
    launch_gather_done(b->group.desc, n, b->group.done, s);
    hip_check(hipMemcpyAsync(done.data(), b->group.done, sizeof(int32_t) * n, hipMemcpyDeviceToHost, s), "D2H");
    hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");
    int act = 0;
    for (int i = 0; i < n; ++i) act += done[i] ? 0 : 1;
    *n_active = act;
    return GOCP_OK;
    GOCP_GUARD_END
}

int gocp_batch_result(gocp_batch *b, int32_t i, gocp_adapt_result *res) {
    GOCP_GUARD_BEGIN
    if (!b || !res) throw Error(GOCP_EINVAL, "null argument");
    check_ctx(b->group.ctx);
    if (i < 0 || i >= (int)b->group.inst.size()) throw Error(GOCP_EINVAL, "instance index out of range");
    hipStream_t s = b->group.ctx->user_stream;
    b->group.finalize({i}, s);
    read_result(b->group.inst[i], s, res, nullptr);
    return GOCP_OK;
    GOCP_GUARD_END
}

int gocp_batch_time_kernel(gocp_batch *b, int32_t which, int32_t n_launch, double *avg_ms) {
    GOCP_GUARD_BEGIN
    if (!b || !avg_ms || n_launch <= 0) throw Error(GOCP_EINVAL, "null argument or no launches");
    if (which < 0 || which > 3) throw Error(GOCP_EINVAL, "kernel id must be 0, 1, 2 or 3");
    check_ctx(b->group.ctx);
    hipStream_t s = b->group.ctx->user_stream;
    Group &g = b->group;
    const int kid = which == 1 ? K_LINE_HVW : g.es_kid();
    const int mode = which == 1 ? 0 : which == 2 ? 4 : 3;                // dry modes
    // which 3: both reduction stages
    auto launch = [&]() {
        if (which == 3) {
            launch_kernel(K_SCREEN_SUM1, g.dtype, g.R, g.desc, g.bgrp, g.ng, mode, s, g.scb);
            launch_kernel(g.sr_kid(), g.dtype, g.R, g.desc, g.binst, (int)g.inst.size(), mode, s);
        } else if (kid == K_LINE_HVW) {
            g.launch_hvw(mode, s);
        } else {
            launch_kernel(kid, g.dtype, g.R, g.desc, g.btile, g.nt, mode, s);
        }
    };
    hipEvent_t e0, e1;
    hip_check(hipEventCreate(&e0), "hipEventCreate");
    hip_check(hipEventCreate(&e1), "hipEventCreate");
    launch();     // warm
    hip_check(hipEventRecord(e0, s), "hipEventRecord");
    for (int i = 0; i < n_launch; ++i) launch();
    hip_check(hipEventRecord(e1, s), "hipEventRecord");
    hip_check(hipEventSynchronize(e1), "hipEventSynchronize");
    float ms = 0.f;
    hip_check(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *avg_ms = (double)ms / n_launch;
    return GOCP_OK;
    GOCP_GUARD_END
}

int gocp_batch_schedule(gocp_batch *b, int32_t *amps_per_lane) {
    GOCP_GUARD_BEGIN
    if (!b || !amps_per_lane) throw Error(GOCP_EINVAL, "null argument");
    *amps_per_lane = b->group.schedule_code();
    return GOCP_OK;
    GOCP_GUARD_END
}

int gocp_batch_destroy(gocp_batch *b) {
    GOCP_GUARD_BEGIN
    if (!b) return GOCP_OK;
    (void)hipSetDevice(b->group.ctx->device);
    (void)hipStreamSynchronize(b->group.ctx->user_stream);
    delete b;
    return GOCP_OK;
    GOCP_GUARD_END
}

}  // extern "C"
