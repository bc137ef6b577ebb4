// Device-resident ADAPT instances and lock-step groups of them (shared by
// the batched form and the serving runtime).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <memory>
#include <vector>

#include "runtime.h"

namespace gocp {

struct Instance {
    const Ham *h = nullptr;
    const Pool *p = nullptr;
    void *psi = nullptr;
    int dtype = 0;
    int max_iter = 0;
    double tol = 0.0;
    InstPlan ip;
    char *mem = nullptr;
    InstDev desc;
    bool finalized = false;
    bool owns_mem = true;
    ~Instance() {
        if (mem && owns_mem) (void)hipFree(mem);
    }
};

// Validate, allocate and initialise one instance (state upload and counter
// reset are stream-ordered on s).  With psi == nullptr the instance holds its
// own state buffer, initialised to the Hartree-Fock basis state `hf`.  With
// `at` the workspace is placed there (ip.bytes, allocated by the caller) and
// the tables `dh`, `dp` are used instead of the handles' device caches: no
// device memory is allocated.
inline Instance *instance_create(gocp_ctx *ctx, const Ham *h, const Pool *p, void *psi, int dtype,
                          int max_iter, double tol, uint64_t hf, hipStream_t s, char *at = nullptr,
                          const DeviceHam *dh = nullptr, const DevicePool *dp = nullptr) {
    if (!h || !p) throw Error(GOCP_EINVAL, "null Hamiltonian or pool");
    if (h->n_qubits != p->n_qubits)
        throw Error(GOCP_ESHAPE, "Hamiltonian and pool act on different qubit counts");
    check_dtype(dtype);
    if (max_iter < 0) throw Error(GOCP_EINVAL, "negative max_iter");
    std::unique_ptr<Instance> in(new Instance());
    in->h = h;
    in->p = p;
    in->dtype = dtype;
    in->max_iter = max_iter;
    in->tol = tol;
    const bool own = psi == nullptr;
    in->ip = plan_instance(h->n_qubits, p->n_ops(), max_iter, dtype, own);
    if (at) {
        in->mem = at;
        in->owns_mem = false;
    } else {
        hip_check(hipMalloc(&in->mem, in->ip.bytes), "hipMalloc instance workspace");
    }
    in->psi = own ? in->mem + in->ip.o_psi : psi;
    in->desc = at ? make_desc_at(in->ip, in->mem, dh, dp, in->psi, nullptr)
                  : make_desc(ctx->device, in->ip, in->mem, h, p, in->psi, nullptr);
    const AdaptState st = make_state(in->ip, in->mem, max_iter, tol, true);
    hip_check(hipMemsetAsync(in->mem + in->ip.o_v, 0, in->ip.o_pe - in->ip.o_v, s), "hipMemsetAsync");
    if (in->ip.o_hv)
        hip_check(hipMemsetAsync(in->mem + in->ip.o_hv, 0, in->ip.bytes - in->ip.o_hv, s), "hipMemsetAsync");
    if (in->ip.o_actn)
        hip_check(hipMemsetAsync(in->mem + in->ip.o_actn, 0, (size_t)in->ip.n_pblk * 4, s), "hipMemsetAsync");
    hip_check(hipMemcpyAsync(in->mem + in->ip.o_st, &st, sizeof(st), hipMemcpyHostToDevice, s), "H2D");
    if (own) launch_basis(dtype, in->psi, 1u << h->n_qubits, (uint32_t)hf, s);
    return in.release();
}

// Tiles of 64 R amplitudes covering a 2^n state.
inline int tiles_for(int n_qubits, int R) {
    const size_t dim = (size_t)1 << n_qubits, t = (size_t)kTile * R;
    return (int)((dim + t - 1) / t);
}

struct Group {
    gocp_ctx *ctx = nullptr;
    int dtype = 0;
    int R = 1;                 // amplitudes per lane of the tile kernels
    int P = kHvwPartsHi;       // workgroups per tile slot of the compacted H v, H w launch
    bool xf = false;           // R = 1 and every member's pool has an X-class screen
    int scb = 1;               // operator column blocks of the first screen reduction stage
    bool wide = false;         // some member's pool has more than kPairBlock operators
    std::vector<int> ntile;    // tiles of each member for R
    std::vector<int> ngroup;   // tile groups of each member (first reduction stage)
    int ng = 0;
    std::vector<Instance *> inst;
    char *meta = nullptr;
    size_t meta_cap = 0;
    InstDev *desc = nullptr;
    int2 *btile = nullptr, *bpair = nullptr, *bsub = nullptr, *binst = nullptr, *bgrp = nullptr;
    int2 *bact = nullptr;      // rows of the compacted H v, H w launch (members with lists)
    int2 *bhvw = nullptr;      // tile rows of the whole-state H v, H w launch (the others)
    int32_t *done = nullptr;   // n flags gathered on the device
    int nt = 0, np = 0, na = 0, nh = 0;
    std::vector<int> tile0, pair0;
    static constexpr int kChunk = 8;
    hipGraph_t graph[2] = {nullptr, nullptr};
    hipGraphExec_t exec[2] = {nullptr, nullptr};
    // Caller-provided table buffers (the server's): each rebuild writes the
    // one the previous rebuild did not, so launches still queued with the
    // previous tables read them intact; rebuild() then never allocates.
    char *ext[2] = {nullptr, nullptr};
    size_t ext_cap = 0;
    int ext_cur = 0;

    ~Group() {
        drop_graphs();
        if (meta && !ext[0]) (void)hipFree(meta);
    }

    void drop_graphs() {
        for (int k = 0; k < 2; ++k) {
            if (exec[k]) (void)hipGraphExecDestroy(exec[k]);
            if (graph[k]) (void)hipGraphDestroy(graph[k]);
            exec[k] = nullptr;
            graph[k] = nullptr;
        }
    }

    // Upload descriptors and work tables of the current members.
    void rebuild(hipStream_t s) {
        drop_graphs();
        std::vector<InstDev> d;
        std::vector<int2> bt, bp, bi, bg, ba, bh;
        tile0.clear();
        pair0.clear();
        ntile.clear();
        ngroup.clear();
        for (size_t i = 0; i < inst.size(); ++i) {
            InstDev di = inst[i]->desc;
            di.n_tiles = tiles_for(di.n_qubits, R);
            di.n_groups = (di.n_tiles + kGroup - 1) / kGroup;
            // members that keep a list of the amplitudes where v or w is
            // nonzero (complex64 states) take the compacted H v, H w launch:
            // one slot per pair block (at most kHvwSlots) of P workgroups, a
            // function of the member and the schedule alone, so its results
            // do not depend on the group it runs in
            di.hvw_parts = P;
            if (P == kHvwPartsLo) di.hsegp = di.hsegp_lo;
            if (di.act) {
                di.n_lpart = std::min(kHvwSlots, inst[i]->ip.n_pblk) * P;
                for (int y = 0; y < di.n_lpart; ++y) ba.push_back(make_int2((int)i, y));
            } else {
                di.n_lpart = di.n_tiles;
                for (int t = 0; t < di.n_tiles; ++t) bh.push_back(make_int2((int)i, t));
            }
            d.push_back(di);
            ntile.push_back(di.n_tiles);
            tile0.push_back((int)bt.size());
            pair0.push_back((int)bp.size());
            for (int t = 0; t < di.n_tiles; ++t) bt.push_back(make_int2((int)i, t));
            for (int t = 0; t < inst[i]->ip.n_pblk; ++t) bp.push_back(make_int2((int)i, t));
            bi.push_back(make_int2((int)i, 0));
            for (int gi = 0; gi < di.n_groups; ++gi) bg.push_back(make_int2((int)i, gi));
            ngroup.push_back(di.n_groups);
        }
        ng = (int)bg.size();
        nt = (int)bt.size();
        xf = R == 1 && !inst.empty();
        scb = 1;
        wide = false;
        for (Instance *in : inst) {
            xf = xf && in->desc.n_xchunks > 0;
            scb = std::max(scb, sum1_blocks(in->ip.M));
            wide = wide || in->ip.M > kPairBlock;
        }
        np = (int)bp.size();
        na = (int)ba.size();
        nh = (int)bh.size();
        const size_t sub = std::max<size_t>({bt.size(), bp.size(), inst.size(), 1});
        auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
        const size_t o_bt = al(d.size() * sizeof(InstDev));
        const size_t o_bp = o_bt + al(bt.size() * sizeof(int2));
        const size_t o_bs = o_bp + al(bp.size() * sizeof(int2));
        const size_t o_bi = o_bs + al(sub * sizeof(int2));
        const size_t o_bg = o_bi + al(std::max<size_t>(inst.size(), 1) * sizeof(int2));
        const size_t o_ba = o_bg + al(std::max<size_t>(bg.size(), 1) * sizeof(int2));
        const size_t o_bh = o_ba + al(std::max<size_t>(ba.size(), 1) * sizeof(int2));
        const size_t o_dn = o_bh + al(std::max<size_t>(bh.size(), 1) * sizeof(int2));
        const size_t need = o_dn + al(std::max<size_t>(inst.size(), 1) * sizeof(int32_t));
        if (ext[0]) {
            if (need > ext_cap) throw Error(GOCP_ENOMEM, "group tables exceed the server's table buffers");
            ext_cur ^= 1;
            meta = ext[ext_cur];
            meta_cap = ext_cap;
        } else if (need > meta_cap) {
            if (meta) {
                hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");
                hip_check(hipFree(meta), "hipFree");
                meta = nullptr;
            }
            meta_cap = std::max(need, (size_t)1 << 16) * 2;
            hip_check(hipMalloc(&meta, meta_cap), "hipMalloc group tables");
        }
        desc = reinterpret_cast<InstDev *>(meta);
        btile = reinterpret_cast<int2 *>(meta + o_bt);
        bpair = reinterpret_cast<int2 *>(meta + o_bp);
        bsub = reinterpret_cast<int2 *>(meta + o_bs);
        binst = reinterpret_cast<int2 *>(meta + o_bi);
        bgrp = reinterpret_cast<int2 *>(meta + o_bg);
        bact = reinterpret_cast<int2 *>(meta + o_ba);
        bhvw = reinterpret_cast<int2 *>(meta + o_bh);
        done = reinterpret_cast<int32_t *>(meta + o_dn);
        if (!d.empty())
            hip_check(hipMemcpyAsync(desc, d.data(), d.size() * sizeof(InstDev), hipMemcpyHostToDevice, s), "H2D");
        if (!bt.empty())
            hip_check(hipMemcpyAsync(btile, bt.data(), bt.size() * sizeof(int2), hipMemcpyHostToDevice, s), "H2D");
        if (!bp.empty())
            hip_check(hipMemcpyAsync(bpair, bp.data(), bp.size() * sizeof(int2), hipMemcpyHostToDevice, s), "H2D");
        if (!bi.empty())
            hip_check(hipMemcpyAsync(binst, bi.data(), bi.size() * sizeof(int2), hipMemcpyHostToDevice, s), "H2D");
        if (!bg.empty())
            hip_check(hipMemcpyAsync(bgrp, bg.data(), bg.size() * sizeof(int2), hipMemcpyHostToDevice, s), "H2D");
        if (!ba.empty())
            hip_check(hipMemcpyAsync(bact, ba.data(), ba.size() * sizeof(int2), hipMemcpyHostToDevice, s), "H2D");
        if (!bh.empty())
            hip_check(hipMemcpyAsync(bhvw, bh.data(), bh.size() * sizeof(int2), hipMemcpyHostToDevice, s), "H2D");
        // a group of one instance launches with null row tables: its rows
        // are (0, workgroup index), which the kernels then form without a load
        if (inst.size() == 1) btile = bpair = binst = bgrp = bact = bhvw = nullptr;
    }

    // One ADAPT iteration of every member: the selection from the pending
    // screen partials (in every workgroup of the line-search-vector launch)
    // and the line-search vectors, H v / H w, the angle and the Taylor update,
    // then the new state's energy and screen partials and their group sums.
    // The new state's selection is pending until the next iteration or
    // select_pending().
    // With `ev` set, the launch of kernel id `timed_kid` records its start in
    // ev[0] and its end in ev[1] (for the H v, H w pair: the first one's start,
    // the second one's end).
    void enqueue_iteration(hipStream_t s, int timed_kid = -1, const hipEvent_t *ev = nullptr) const {
        if (inst.empty()) return;
        const int n = (int)inst.size();
        struct L {
            int kid, mode;
            const int2 *rows;
            int nrows;
        };
        (void)n;
        const L seq[5] = {{lv_kid(), 1, bpair, np},        {K_LINE_HVW, 1, bhvw, nh},
                          {K_TAYLOR, 1, bpair, np},        {es_kid(), 2, btile, nt},
                          {K_SCREEN_SUM1, 2, bgrp, ng}};
        for (const L &l : seq) {
            const bool t = ev && base_kid(l.kid) == timed_kid;
            const hipEvent_t t0 = t ? ev[0] : nullptr, t1 = t ? ev[1] : nullptr;
            if (l.kid == K_LINE_HVW) launch_hvw(l.mode, s, t0, t1);
            else launch_kernel(l.kid, dtype, R, desc, l.rows, l.nrows, l.mode, s, l.kid == K_SCREEN_SUM1 ? scb : 0,
                               0.0, 0, t0, t1);
        }
    }

    // The H v, H w launches over the whole group (mode as k_line_hvw):
    // compacted for members with lists, whole-state for the others; t0 takes
    // the first launch's start, t1 the second one's end.
    void launch_hvw(int mode, hipStream_t s, hipEvent_t t0 = nullptr, hipEvent_t t1 = nullptr) const {
        launch_hvw_act(desc, bact, na, mode, s, t0, nullptr);
        launch_kernel(K_LINE_HVW, dtype, R, desc, bhvw, nh, mode, s, 0, 0.0, 0, nullptr, t1);
    }

    // Selection (energy, gradients, operator, record) of every member's
    // pending partials; selecting them again later writes the same record.
    void select_pending(hipStream_t s) const {
        if (inst.empty()) return;
        launch_kernel(sr_kid(), dtype, R, desc, binst, (int)inst.size(), kModePending, s);
    }

    void capture() {
        hipStream_t cs = ctx->own_stream;
        const int iters[2] = {1, kChunk};
        for (int k = 0; k < 2; ++k) {
            hip_check(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
            for (int i = 0; i < iters[k]; ++i) enqueue_iteration(cs);
            select_pending(cs);
            hip_check(hipStreamEndCapture(cs, &graph[k]), "hipStreamEndCapture");
            hip_check(hipGraphInstantiate(&exec[k], graph[k], nullptr, nullptr, 0), "hipGraphInstantiate");
        }
    }

    // Enqueue n iterations on s (graph replays when use_graph).
    void step(int n, hipStream_t s, bool use_graph) {
        if (inst.empty() || n <= 0) return;
        for (Instance *in : inst) in->finalized = false;
        if (!use_graph) {
            for (int i = 0; i < n; ++i) enqueue_iteration(s);
            select_pending(s);
            return;
        }
        if (!exec[0]) capture();
        for (int i = 0; i < n / kChunk; ++i) hip_check(hipGraphLaunch(exec[1], s), "hipGraphLaunch");
        for (int i = 0; i < n % kChunk; ++i) hip_check(hipGraphLaunch(exec[0], s), "hipGraphLaunch");
    }

    // Launch one kernel over the tile (0), pair (1), instance (2) or tile-group
    // (3) rows of a subset of members.
    void launch_subset(int which, int mode, const std::vector<int> &members, int table, hipStream_t s) {
        std::vector<int2> rows;
        for (int i : members) {
            const int n = table == 0 ? ntile[i] : table == 1 ? inst[i]->ip.n_pblk : table == 3 ? ngroup[i] : 1;
            for (int t = 0; t < n; ++t) rows.push_back(make_int2(i, t));
        }
        if (rows.empty()) return;
        hip_check(hipMemcpyAsync(bsub, rows.data(), rows.size() * sizeof(int2), hipMemcpyHostToDevice, s), "H2D");
        launch_kernel(which, dtype, R, desc, bsub, (int)rows.size(), mode, s, which == K_SCREEN_SUM1 ? scb : 0);
    }

    // Time one energy+screen launch and one line-search launch over the
    // whole group (dry modes: neither sigma nor the iteration record is
    // written); milliseconds.
    double time_tile_kernels(hipStream_t s, int reps) {
        hipEvent_t e0, e1;
        hip_check(hipEventCreate(&e0), "hipEventCreate");
        hip_check(hipEventCreate(&e1), "hipEventCreate");
        const int n = (int)inst.size();
        launch_kernel(es_kid(), dtype, R, desc, btile, nt, 3, s);
        launch_kernel(K_SCREEN_SUM1, dtype, R, desc, bgrp, ng, 3, s, scb);
        launch_kernel(sr_kid(), dtype, R, desc, binst, n, 3, s);
        launch_hvw(0, s);
        hip_check(hipEventRecord(e0, s), "hipEventRecord");
        for (int i = 0; i < reps; ++i) {
            launch_kernel(es_kid(), dtype, R, desc, btile, nt, 3, s);
            launch_kernel(K_SCREEN_SUM1, dtype, R, desc, bgrp, ng, 3, s, scb);
            launch_kernel(sr_kid(), dtype, R, desc, binst, n, 3, s);
            launch_hvw(0, s);
        }
        hip_check(hipEventRecord(e1, s), "hipEventRecord");
        hip_check(hipEventSynchronize(e1), "hipEventSynchronize");
        float ms = 0.f;
        hip_check(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        return (double)ms / reps;
    }

    // Choose the schedule: amplitudes per lane R (1, 2 or 4) in the low byte,
    // the compacted H v, H w launch's parts P in the next (0 for
    // kHvwPartsHi, or kHvwPartsLo); 0 = autotune: R timed on this group's
    // members (the fastest kept, remembered per composition of qubit counts
    // and precision), P by parts_rule().  Call before start(): the trial
    // launches recompute values start() recomputes.
    void choose_schedule(int schedule, hipStream_t s);
    // The schedule in the encoding choose_schedule takes.
    // the energy+screen launch of the group
    int es_kid() const { return xf ? K_ENERGY_SCREEN_X : K_ENERGY_SCREEN; }
    // the selection launches of the group
    int lv_kid() const { return wide ? K_LINE_VW_W : K_LINE_VW; }
    int sr_kid() const { return wide ? K_SCREEN_REDUCE_W : K_SCREEN_REDUCE; }
    int schedule_code() const { return R | (P == kHvwPartsHi ? 0 : P << 8); }
    // kHvwPartsLo when the compacted launch would have more than four
    // workgroups per compute unit with kHvwPartsHi (many instances: fewer,
    // longer runs per workgroup pay there), else kHvwPartsHi.
    int parts_rule() const {
        long rows = 0;
        for (const Instance *in : inst)
            if (in->desc.act) rows += (long)std::min(kHvwSlots, in->ip.n_pblk) * kHvwPartsHi;
        return rows > 4L * ctx->n_cu ? kHvwPartsLo : kHvwPartsHi;
    }

    // Energy, screen and selection of the starting state of the given members.
    void start(const std::vector<int> &members, hipStream_t s) {
        launch_subset(es_kid(), 1, members, 0, s);
        launch_subset(K_SCREEN_SUM1, 1, members, 3, s);
        launch_subset(sr_kid(), kModePending, members, 2, s);
    }

    // Scale the states of the given members to unit norm (their renormalisation
    // is otherwise folded into the next Taylor update).
    void finalize(const std::vector<int> &members, hipStream_t s) {
        std::vector<int> todo;
        for (int i : members)
            if (!inst[i]->finalized) todo.push_back(i);
        if (todo.empty()) return;
        launch_subset(K_NORMALIZE, 1, todo, 1, s);
        launch_subset(K_UNIT_NORM, 0, todo, 2, s);
        for (int i : todo) inst[i]->finalized = true;
    }
};

void read_result(Instance *in, hipStream_t s, gocp_adapt_result *res, AdaptState *out_state);
int autotune_cached(const std::vector<int> &qubits, int dtype);
void autotune_store(const std::vector<int> &qubits, int dtype, int R);
void run_to_completion(Group &g, int max_iter, bool use_graph, hipStream_t s);

}  // namespace gocp
