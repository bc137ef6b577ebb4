// Device runtime of libgocp: contexts, device copies of the term tables,
// per-call workspaces, and the device C ABI entry points.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <string>

#include "device.h"

namespace gocp {

void launch_kernel(int which, int dtype, const InstDev *insts, const int2 *blk, int nblk, int mode,
                   hipStream_t s, int j, double th, int ns);
void launch_basis(int dtype, void *psi, uint32_t dim, uint32_t index, hipStream_t s);

enum { K_APPLY_H = 0, K_GRAD = 1, K_LINE_VW = 2, K_LINE_HVW = 3, K_TAYLOR = 4, K_NORMALIZE = 5 };

void hip_check(hipError_t e, const char *what) {
    if (e != hipSuccess)
        throw Error(e == hipErrorOutOfMemory ? GOCP_ENOMEM : GOCP_EDEVICE,
                    std::string(what) + ": " + hipGetErrorString(e));
}

namespace {

template <typename T>
T *dev_upload(const std::vector<T> &v) {
    T *p = nullptr;
    const size_t bytes = std::max<size_t>(1, v.size()) * sizeof(T);
    hip_check(hipMalloc(&p, bytes), "hipMalloc");
    if (!v.empty()) hip_check(hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice), "hipMemcpy");
    return p;
}

// Contiguous split of `cost` into kNW ranges of about equal total cost.
std::vector<int32_t> balanced_split(const std::vector<double> &cost) {
    double total = 0.0;
    for (double c : cost) total += c;
    std::vector<int32_t> split(kNW + 1, (int32_t)cost.size());
    split[0] = 0;
    double acc = 0.0;
    int w = 1;
    for (size_t i = 0; i < cost.size() && w < kNW; ++i) {
        acc += cost[i];
        while (w < kNW && acc >= total * w / kNW) split[w++] = (int32_t)(i + 1);
    }
    for (int k = 1; k <= kNW; ++k) split[k] = std::max(split[k], split[k - 1]);
    return split;
}

int current_device() {
    int d = 0;
    hip_check(hipGetDevice(&d), "hipGetDevice");
    return d;
}

}  // namespace

void release_device_ham(DeviceHam *d) {
    if (!d) return;
    (void)hipFree(d->hcls);
    (void)hipFree(d->hterm);
    (void)hipFree(d->cls_split);
    delete d;
}

void release_device_pool(DevicePool *d) {
    if (!d) return;
    (void)hipFree(d->pop);
    (void)hipFree(d->pterm);
    (void)hipFree(d->op_norm1);
    (void)hipFree(d->op_sched);
    (void)hipFree(d->op_split);
    delete d;
}

const DeviceHam *device_ham(const Ham &h, int dev) {
    std::lock_guard<std::mutex> lk(h.mu);
    if ((int)h.dev.size() <= dev) h.dev.resize(dev + 1, nullptr);
    if (h.dev[dev]) return h.dev[dev];
    std::unique_ptr<DeviceHam> d(new DeviceHam());
    d->device = dev;
    std::vector<HClass> cls(h.n_classes());
    for (int c = 0; c < h.n_classes(); ++c) cls[c] = HClass{h.cls_x[c], h.cls_off[c], h.cls_off[c + 1], 0};
    std::vector<HTerm> terms(h.str_z.size());
    for (size_t s = 0; s < terms.size(); ++s) terms[s] = HTerm{h.str_c[s], h.str_z[s], 0u};
    d->hcls = dev_upload(cls);
    d->hterm = dev_upload(terms);
    std::vector<double> cost(h.n_classes());
    for (int c = 0; c < h.n_classes(); ++c) cost[c] = 5.0 * (h.cls_off[c + 1] - h.cls_off[c]) + 6.0;
    d->cls_split = dev_upload(balanced_split(cost));
    h.dev[dev] = d.release();
    return h.dev[dev];
}

const DevicePool *device_pool(const Pool &p, int dev) {
    std::lock_guard<std::mutex> lk(p.mu);
    if ((int)p.dev.size() <= dev) p.dev.resize(dev + 1, nullptr);
    if (p.dev[dev]) return p.dev[dev];
    std::unique_ptr<DevicePool> d(new DevicePool());
    d->device = dev;
    std::vector<HClass> ops(p.n_ops());
    for (int k = 0; k < p.n_ops(); ++k) ops[k] = HClass{p.op_x[k], p.op_off[k], p.op_off[k + 1], p.kind[k]};
    std::vector<HTerm> terms(p.str_z.size());
    for (size_t s = 0; s < terms.size(); ++s) terms[s] = HTerm{p.str_c[s], p.str_z[s], 0u};
    d->pop = dev_upload(ops);
    d->pterm = dev_upload(terms);
    d->op_norm1 = dev_upload(p.op_norm1);
    // gradient screen schedule: operators in GOCP family order, families
    // dealt to the waves of a workgroup in contiguous, cost-balanced ranges
    const std::vector<int32_t> &sched = p.fam_members;
    std::vector<double> cost(sched.size());
    for (size_t i = 0; i < sched.size(); ++i)
        cost[i] = 5.0 * (p.op_off[sched[i] + 1] - p.op_off[sched[i]]) + 20.0;
    d->op_sched = dev_upload(sched);
    d->op_split = dev_upload(balanced_split(cost));
    p.dev[dev] = d.release();
    return p.dev[dev];
}

// ---------------------------------------------------------------- workspace

// Device memory for the buffers of a set of instances, carved from one
// allocation that is kept and grown per context.
struct Arena {
    char *base = nullptr;
    size_t cap = 0, used = 0;
    void reset() { used = 0; }
    size_t take(size_t bytes) {
        const size_t off = (used + 255) & ~(size_t)255;
        used = off + bytes;
        return off;
    }
};

struct InstPlan {
    int n_qubits = 0, M = 0, max_iter = 0, dtype = 0;
    int n_tiles = 0, n_pblk = 0;
    size_t o_sigma, o_v, o_w, o_pe, o_pn, o_pg, o_pl, o_pt, o_cnt, o_st, o_he, o_hop, o_hth,
        o_hgn, o_hgm, o_hns, o_hpr, o_g;
};

struct BatchPlan {
    std::vector<InstPlan> inst;
    std::vector<int2> blk_tile, blk_pair;
    size_t o_desc = 0, o_btile = 0, o_bpair = 0;
    size_t bytes = 0;
};

}  // namespace gocp

struct gocp_ctx {
    int device = 0;
    hipStream_t user_stream = nullptr;
    hipStream_t own_stream = nullptr;
    gocp::Arena arena;
    std::string arch;
    int n_cu = 0;
};

namespace gocp {

void plan_instance(InstPlan &ip, Arena &a, int nq, int M, int max_iter, int dtype) {
    ip.n_qubits = nq;
    ip.M = M;
    ip.max_iter = max_iter;
    ip.dtype = dtype;
    const size_t dim = (size_t)1 << nq;
    const size_t es = dtype == GOCP_C64 ? 8 : 16;
    ip.n_tiles = (int)((dim + kTile - 1) / kTile);
    ip.n_pblk = (int)((dim / 2 + kPairBlock - 1) / kPairBlock);
    if (ip.n_pblk < 1) ip.n_pblk = 1;
    const size_t hist = (size_t)max_iter + 1;
    ip.o_sigma = a.take(dim * 16);
    ip.o_v = a.take(dim * es);
    ip.o_w = a.take(dim * es);
    ip.o_pe = a.take(ip.n_tiles * 8);
    ip.o_pn = a.take(ip.n_tiles * 8);
    ip.o_pg = a.take((size_t)ip.n_tiles * std::max(M, 1) * 8);
    ip.o_pl = a.take((3 * (size_t)ip.n_tiles + 2 * (size_t)ip.n_pblk) * 8);
    ip.o_pt = a.take((size_t)ip.n_pblk * 8);
    ip.o_cnt = a.take(4 * sizeof(int32_t));
    ip.o_st = a.take(sizeof(AdaptState));
    ip.o_he = a.take(hist * 8);
    ip.o_hop = a.take(hist * 4);
    ip.o_hth = a.take(hist * 8);
    ip.o_hgn = a.take(hist * 8);
    ip.o_hgm = a.take(hist * 8);
    ip.o_hns = a.take(hist * 4);
    ip.o_hpr = a.take(hist * 8);
    ip.o_g = a.take((size_t)std::max(M, 1) * 8);
}

// Lay out and (re)allocate the workspace for `n` instances; zeroes the
// arrival counters.  Returns the plan; offsets are relative to ctx->arena.base.
BatchPlan make_plan(gocp_ctx *ctx, const std::vector<int> &nq, const std::vector<int> &M,
                    int max_iter, int dtype) {
    BatchPlan bp;
    Arena a;
    const size_t n = nq.size();
    bp.inst.resize(n);
    for (size_t i = 0; i < n; ++i) plan_instance(bp.inst[i], a, nq[i], M[i], max_iter, dtype);
    for (size_t i = 0; i < n; ++i) {
        for (int t = 0; t < bp.inst[i].n_tiles; ++t) bp.blk_tile.push_back(make_int2((int)i, t));
        for (int t = 0; t < bp.inst[i].n_pblk; ++t) bp.blk_pair.push_back(make_int2((int)i, t));
    }
    bp.o_desc = a.take(n * sizeof(InstDev));
    bp.o_btile = a.take(bp.blk_tile.size() * sizeof(int2));
    bp.o_bpair = a.take(bp.blk_pair.size() * sizeof(int2));
    bp.bytes = a.used;
    if (ctx->arena.cap < bp.bytes) {
        if (ctx->arena.base) {
            hip_check(hipStreamSynchronize(ctx->user_stream), "hipStreamSynchronize");
            hip_check(hipFree(ctx->arena.base), "hipFree");
            ctx->arena.base = nullptr;
            ctx->arena.cap = 0;
        }
        const size_t cap = std::max(bp.bytes, (size_t)1 << 20);
        hip_check(hipMalloc(&ctx->arena.base, cap), "hipMalloc workspace");
        ctx->arena.cap = cap;
    }
    for (size_t i = 0; i < n; ++i)
        hip_check(hipMemsetAsync(ctx->arena.base + bp.inst[i].o_cnt, 0, 4 * sizeof(int32_t),
                                 ctx->user_stream),
                  "hipMemsetAsync");
    return bp;
}

InstDev make_desc(gocp_ctx *ctx, const InstPlan &ip, const Ham *h, const Pool *p, void *psi,
                  double2 *sigma_override) {
    char *b = ctx->arena.base;
    InstDev I;
    std::memset(&I, 0, sizeof(I));
    if (h) {
        const DeviceHam *dh = device_ham(*h, ctx->device);
        I.hcls = dh->hcls;
        I.hterm = dh->hterm;
        I.cls_split = dh->cls_split;
    }
    if (p) {
        const DevicePool *dp = device_pool(*p, ctx->device);
        I.pop = dp->pop;
        I.pterm = dp->pterm;
        I.op_norm1 = dp->op_norm1;
        I.op_sched = dp->op_sched;
        I.op_split = dp->op_split;
    }
    I.psi = psi;
    I.sigma = sigma_override ? sigma_override : reinterpret_cast<double2 *>(b + ip.o_sigma);
    I.v = b + ip.o_v;
    I.w = b + ip.o_w;
    I.part_e = reinterpret_cast<double *>(b + ip.o_pe);
    I.part_n = reinterpret_cast<double *>(b + ip.o_pn);
    I.part_g = reinterpret_cast<double *>(b + ip.o_pg);
    I.part_l = reinterpret_cast<double *>(b + ip.o_pl);
    I.part_t = reinterpret_cast<double *>(b + ip.o_pt);
    I.counters = reinterpret_cast<int32_t *>(b + ip.o_cnt);
    I.st = reinterpret_cast<AdaptState *>(b + ip.o_st);
    I.n_qubits = ip.n_qubits;
    I.M = ip.M;
    I.n_tiles = ip.n_tiles;
    I.n_pblk = ip.n_pblk;
    return I;
}

AdaptState make_state(gocp_ctx *ctx, const InstPlan &ip, int max_iter, double grad_tol, bool hist) {
    char *b = ctx->arena.base;
    AdaptState s;
    std::memset(&s, 0, sizeof(s));
    s.max_iter = max_iter;
    s.grad_tol = grad_tol;
    s.nrm = 1.0;
    if (hist) {
        s.hist_e = reinterpret_cast<double *>(b + ip.o_he);
        s.hist_op = reinterpret_cast<int32_t *>(b + ip.o_hop);
        s.hist_theta = reinterpret_cast<double *>(b + ip.o_hth);
        s.hist_gnorm = reinterpret_cast<double *>(b + ip.o_hgn);
        s.hist_gmax = reinterpret_cast<double *>(b + ip.o_hgm);
        s.hist_nsub = reinterpret_cast<int32_t *>(b + ip.o_hns);
        s.hist_pred = reinterpret_cast<double *>(b + ip.o_hpr);
    }
    s.g = reinterpret_cast<double *>(b + ip.o_g);
    return s;
}

void upload(gocp_ctx *ctx, size_t off, const void *src, size_t bytes) {
    hip_check(hipMemcpyAsync(ctx->arena.base + off, src, bytes, hipMemcpyHostToDevice, ctx->user_stream),
              "hipMemcpyAsync H2D");
}

void download(gocp_ctx *ctx, void *dst, size_t off, size_t bytes) {
    hip_check(hipMemcpyAsync(dst, ctx->arena.base + off, bytes, hipMemcpyDeviceToHost, ctx->user_stream),
              "hipMemcpyAsync D2H");
}

void sync(gocp_ctx *ctx) { hip_check(hipStreamSynchronize(ctx->user_stream), "hipStreamSynchronize"); }

const Ham *as_ham(const gocp_ham *h) {
    if (!h) throw Error(GOCP_EINVAL, "null Hamiltonian");
    return reinterpret_cast<const Ham *>(h);
}
const Pool *as_pool(const gocp_pool *p) {
    if (!p) throw Error(GOCP_EINVAL, "null pool");
    return reinterpret_cast<const Pool *>(p);
}
void check_ctx(gocp_ctx *ctx) {
    if (!ctx) throw Error(GOCP_EINVAL, "null context");
    hip_check(hipSetDevice(ctx->device), "hipSetDevice");
}
void check_dtype(int dtype) {
    if (dtype != GOCP_C128 && dtype != GOCP_C64) throw Error(GOCP_EINVAL, "unknown state dtype");
}

// Single-instance setup shared by the one-shot calls.
struct Single {
    BatchPlan bp;
    InstDev I;
    int2 *btile, *bpair;
    InstDev *desc;
};

Single setup_single(gocp_ctx *ctx, const Ham *h, const Pool *p, const void *psi, int dtype,
                    int max_iter, double grad_tol, bool hist, double2 *sigma_override = nullptr) {
    if (!psi) throw Error(GOCP_EINVAL, "null state pointer");
    check_dtype(dtype);
    int nq = h ? h->n_qubits : p->n_qubits;
    if (h && p && h->n_qubits != p->n_qubits)
        throw Error(GOCP_ESHAPE, "Hamiltonian and pool act on different qubit counts");
    Single s;
    s.bp = make_plan(ctx, {nq}, {p ? p->n_ops() : 0}, max_iter, dtype);
    const InstPlan &ip = s.bp.inst[0];
    s.I = make_desc(ctx, ip, h, p, const_cast<void *>(psi), sigma_override);
    AdaptState st = make_state(ctx, ip, max_iter, grad_tol, hist);
    upload(ctx, ip.o_st, &st, sizeof(st));
    upload(ctx, s.bp.o_desc, &s.I, sizeof(InstDev));
    upload(ctx, s.bp.o_btile, s.bp.blk_tile.data(), s.bp.blk_tile.size() * sizeof(int2));
    upload(ctx, s.bp.o_bpair, s.bp.blk_pair.data(), s.bp.blk_pair.size() * sizeof(int2));
    s.desc = reinterpret_cast<InstDev *>(ctx->arena.base + s.bp.o_desc);
    s.btile = reinterpret_cast<int2 *>(ctx->arena.base + s.bp.o_btile);
    s.bpair = reinterpret_cast<int2 *>(ctx->arena.base + s.bp.o_bpair);
    return s;
}

void read_state(gocp_ctx *ctx, const Single &s, AdaptState *out) {
    download(ctx, out, s.bp.inst[0].o_st, sizeof(AdaptState));
    sync(ctx);
}

// One ADAPT iteration for every instance of a batch: screen, line search,
// Taylor update, new energy.  Five launches, all stream-ordered.
void enqueue_iteration(const BatchPlan &bp, InstDev *desc, int2 *btile, int2 *bpair, int dtype,
                       hipStream_t s) {
    const int nt = (int)bp.blk_tile.size(), np = (int)bp.blk_pair.size();
    launch_kernel(K_GRAD, dtype, desc, btile, nt, 1, s, 0, 0.0, 0);
    launch_kernel(K_LINE_VW, dtype, desc, bpair, np, 1, s, 0, 0.0, 0);
    launch_kernel(K_LINE_HVW, dtype, desc, btile, nt, 1, s, 0, 0.0, 0);
    launch_kernel(K_TAYLOR, dtype, desc, bpair, np, 1, s, 0, 0.0, 0);
    launch_kernel(K_APPLY_H, dtype, desc, btile, nt, 2, s, 0, 0.0, 0);
}

}  // namespace gocp

using namespace gocp;

#define GOCP_GUARD_BEGIN try {
#define GOCP_GUARD_END                                   \
    }                                                    \
    catch (const gocp::Error &e) {                       \
        gocp::set_last_error(e.what());                  \
        return e.code;                                   \
    }                                                    \
    catch (const std::bad_alloc &) {                     \
        gocp::set_last_error("host allocation failed");  \
        return GOCP_ENOMEM;                              \
    }                                                    \
    catch (const std::exception &e) {                    \
        gocp::set_last_error(e.what());                  \
        return GOCP_EINVAL;                              \
    }

extern "C" {

int gocp_ctx_create(int device, void *stream, gocp_ctx **out) {
    GOCP_GUARD_BEGIN
    if (!out) throw Error(GOCP_EINVAL, "null output handle");
    int n = 0;
    hip_check(hipGetDeviceCount(&n), "hipGetDeviceCount");
    if (device < 0 || device >= n) throw Error(GOCP_EDEVICE, "no such HIP device");
    hip_check(hipSetDevice(device), "hipSetDevice");
    hipDeviceProp_t prop;
    hip_check(hipGetDeviceProperties(&prop, device), "hipGetDeviceProperties");
    const std::string arch = prop.gcnArchName;
    if (arch.rfind("gfx950", 0) != 0)
        throw Error(GOCP_EDEVICE, "libgocp is built for gfx950 (MI355X); device is " + arch);
    std::unique_ptr<gocp_ctx> c(new gocp_ctx());
    c->device = device;
    c->arch = arch;
    c->n_cu = prop.multiProcessorCount;
    hip_check(hipStreamCreateWithFlags(&c->own_stream, hipStreamNonBlocking), "hipStreamCreate");
    c->user_stream = static_cast<hipStream_t>(stream);   // NULL: the default stream
    *out = c.release();
    return GOCP_OK;
    GOCP_GUARD_END
}

int gocp_ctx_destroy(gocp_ctx *ctx) {
    GOCP_GUARD_BEGIN
    if (!ctx) return GOCP_OK;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->user_stream);
    if (ctx->arena.base) (void)hipFree(ctx->arena.base);
    if (ctx->own_stream) (void)hipStreamDestroy(ctx->own_stream);
    delete ctx;
    return GOCP_OK;
    GOCP_GUARD_END
}

int gocp_ctx_set_stream(gocp_ctx *ctx, void *stream) {
    GOCP_GUARD_BEGIN
    check_ctx(ctx);
    hip_check(hipStreamSynchronize(ctx->user_stream), "hipStreamSynchronize");
    ctx->user_stream = static_cast<hipStream_t>(stream);
    return GOCP_OK;
    GOCP_GUARD_END
}

int gocp_ctx_synchronize(gocp_ctx *ctx) {
    GOCP_GUARD_BEGIN
    check_ctx(ctx);
    sync(ctx);
    return GOCP_OK;
    GOCP_GUARD_END
}

int gocp_state_basis(gocp_ctx *ctx, int n_qubits, uint64_t index, void *psi_dev, int dtype) {
    GOCP_GUARD_BEGIN
    check_ctx(ctx);
    check_dtype(dtype);
    if (!psi_dev) throw Error(GOCP_EINVAL, "null state pointer");
    if (n_qubits < 1 || n_qubits > kMaxQubits) throw Error(GOCP_ENOTSUP, "qubit count out of range");
    if (index >= ((uint64_t)1 << n_qubits)) throw Error(GOCP_EINVAL, "basis index out of range");
    launch_basis(dtype, psi_dev, 1u << n_qubits, (uint32_t)index, ctx->user_stream);
    return GOCP_OK;
    GOCP_GUARD_END
}

int energy(gocp_ctx *ctx, const gocp_ham *hh, const void *psi_dev, int dtype, double *e_out) {
    GOCP_GUARD_BEGIN
    check_ctx(ctx);
    if (!e_out) throw Error(GOCP_EINVAL, "null output");
    Single s = setup_single(ctx, as_ham(hh), nullptr, psi_dev, dtype, 0, 0.0, false);
    launch_kernel(K_APPLY_H, dtype, s.desc, s.btile, (int)s.bp.blk_tile.size(), 0, ctx->user_stream, 0, 0.0, 0);
    AdaptState st;
    read_state(ctx, s, &st);
    if (st.status) throw Error(st.status, "non-finite energy or zero norm");
    *e_out = st.energy;
    return GOCP_OK;
    GOCP_GUARD_END
}

int gocp_apply_hamiltonian(gocp_ctx *ctx, const gocp_ham *hh, const void *psi_dev, int dtype,
                           void *sigma_dev, double *e_out) {
    GOCP_GUARD_BEGIN
    check_ctx(ctx);
    if (!sigma_dev) throw Error(GOCP_EINVAL, "null sigma pointer");
    Single s = setup_single(ctx, as_ham(hh), nullptr, psi_dev, dtype, 0, 0.0, false,
                            static_cast<double2 *>(sigma_dev));
    launch_kernel(K_APPLY_H, dtype, s.desc, s.btile, (int)s.bp.blk_tile.size(), 0, ctx->user_stream, 0, 0.0, 0);
    if (e_out) {
        AdaptState st;
        read_state(ctx, s, &st);
        if (st.status) throw Error(st.status, "non-finite energy or zero norm");
        *e_out = st.energy;
    }
    return GOCP_OK;
    GOCP_GUARD_END
}

int pool_gradients(gocp_ctx *ctx, const gocp_ham *hh, const gocp_pool *pp, const void *psi_dev,
                   int dtype, double *g_out, int g_on_device) {
    GOCP_GUARD_BEGIN
    check_ctx(ctx);
    if (!g_out) throw Error(GOCP_EINVAL, "null output");
    const Ham *h = as_ham(hh);
    const Pool *p = as_pool(pp);
    Single s = setup_single(ctx, h, p, psi_dev, dtype, 0, 0.0, false);
    const int nt = (int)s.bp.blk_tile.size();
    launch_kernel(K_APPLY_H, dtype, s.desc, s.btile, nt, 0, ctx->user_stream, 0, 0.0, 0);
    launch_kernel(K_GRAD, dtype, s.desc, s.btile, nt, 0, ctx->user_stream, 0, 0.0, 0);
    const size_t gbytes = (size_t)p->n_ops() * sizeof(double);
    if (g_on_device) {
        hip_check(hipMemcpyAsync(g_out, ctx->arena.base + s.bp.inst[0].o_g, gbytes,
                                 hipMemcpyDeviceToDevice, ctx->user_stream),
                  "hipMemcpyAsync D2D");
    } else {
        download(ctx, g_out, s.bp.inst[0].o_g, gbytes);
        AdaptState st;
        read_state(ctx, s, &st);
        if (st.status) throw Error(st.status, "non-finite gradient");
    }
    return GOCP_OK;
    GOCP_GUARD_END
}

int taylor5_apply(gocp_ctx *ctx, const gocp_pool *pp, int32_t k, double theta, void *psi_dev,
                  int dtype, int32_t *n_substeps_out) {
    GOCP_GUARD_BEGIN
    check_ctx(ctx);
    const Pool *p = as_pool(pp);
    if (k < 0 || k >= p->n_ops()) throw Error(GOCP_EINVAL, "operator index out of range");
    if (!std::isfinite(theta)) throw Error(GOCP_EINVAL, "non-finite angle");
    if (theta == 0.0) {
        if (n_substeps_out) *n_substeps_out = 0;
        return GOCP_OK;
    }
    const int ns = std::max(1, (int)std::ceil(std::fabs(theta) * p->op_norm1[k] / 0.5));
    Single s = setup_single(ctx, nullptr, p, psi_dev, dtype, 0, 0.0, false);
    const int np = (int)s.bp.blk_pair.size();
    launch_kernel(K_TAYLOR, dtype, s.desc, s.bpair, np, 0, ctx->user_stream, k, theta, ns);
    launch_kernel(K_NORMALIZE, dtype, s.desc, s.bpair, np, 0, ctx->user_stream, 0, 0.0, 0);
    if (n_substeps_out) *n_substeps_out = ns;
    return GOCP_OK;
    GOCP_GUARD_END
}

int adapt_solve(gocp_ctx *ctx, const gocp_ham *hh, const gocp_pool *pp, void *psi_dev, int dtype,
                const gocp_adapt_params *params, gocp_adapt_result *res) {
    GOCP_GUARD_BEGIN
    check_ctx(ctx);
    if (!params || !res) throw Error(GOCP_EINVAL, "null params or result");
    if (params->max_iter < 0) throw Error(GOCP_EINVAL, "negative max_iter");
    if (!res->energies || !res->ops || !res->thetas || !res->gnorms)
        throw Error(GOCP_EINVAL, "null result arrays");
    const Ham *h = as_ham(hh);
    const Pool *p = as_pool(pp);
    const int max_iter = params->max_iter;
    Single s = setup_single(ctx, h, p, psi_dev, dtype, max_iter, params->grad_tol, true);
    hipStream_t st = ctx->user_stream;
    const int nt = (int)s.bp.blk_tile.size();
    launch_kernel(K_APPLY_H, dtype, s.desc, s.btile, nt, 1, st, 0, 0.0, 0);

    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
    hipStream_t cap = st;
    const bool use_graph = params->use_graph != 0 && max_iter > 0;
    if (use_graph) {
        // capture on the context's own stream, ordered after the user stream
        cap = ctx->own_stream;
        if (cap != st) {
            hipEvent_t ev;
            hip_check(hipEventCreateWithFlags(&ev, hipEventDisableTiming), "hipEventCreate");
            hip_check(hipEventRecord(ev, st), "hipEventRecord");
            hip_check(hipStreamWaitEvent(cap, ev, 0), "hipStreamWaitEvent");
            (void)hipEventDestroy(ev);
        }
        hip_check(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
        enqueue_iteration(s.bp, s.desc, s.btile, s.bpair, dtype, cap);
        hip_check(hipStreamEndCapture(cap, &graph), "hipStreamEndCapture");
        hip_check(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0), "hipGraphInstantiate");
    }
    // poll the device-side done flag every few iterations so a converged run
    // stops launching work
    AdaptState *pinned = nullptr;
    hip_check(hipHostMalloc(reinterpret_cast<void **>(&pinned), sizeof(AdaptState), 0), "hipHostMalloc");
    const size_t o_st = s.bp.inst[0].o_st;
    const int poll = 8;
    try {
        for (int it = 0; it < max_iter; ++it) {
            if (use_graph)
                hip_check(hipGraphLaunch(exec, cap), "hipGraphLaunch");
            else
                enqueue_iteration(s.bp, s.desc, s.btile, s.bpair, dtype, st);
            if ((it + 1) % poll == 0 && it + 1 < max_iter) {
                hipStream_t q = use_graph ? cap : st;
                hip_check(hipMemcpyAsync(pinned, ctx->arena.base + o_st, sizeof(AdaptState),
                                         hipMemcpyDeviceToHost, q), "hipMemcpyAsync");
                hip_check(hipStreamSynchronize(q), "hipStreamSynchronize");
                if (pinned->done) break;
            }
        }
        if (use_graph) hip_check(hipStreamSynchronize(cap), "hipStreamSynchronize");
        launch_kernel(K_NORMALIZE, dtype, s.desc, s.bpair, (int)s.bp.blk_pair.size(), 1, st, 0, 0.0, 0);
        hip_check(hipMemcpyAsync(pinned, ctx->arena.base + o_st, sizeof(AdaptState),
                                 hipMemcpyDeviceToHost, st), "hipMemcpyAsync");
        sync(ctx);
    } catch (...) {
        (void)hipHostFree(pinned);
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        throw;
    }
    AdaptState fin = *pinned;
    (void)hipHostFree(pinned);
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (fin.status) throw Error(fin.status, "non-finite value during ADAPT");

    const int n_it = fin.iter;
    const InstPlan &ip = s.bp.inst[0];
    const int n_scr = n_it + (fin.converged ? 1 : 0);
    res->n_iter = n_it;
    res->converged = fin.converged;
    download(ctx, res->energies, ip.o_he, (size_t)(n_it + 1) * 8);
    if (n_it > 0) {
        download(ctx, res->ops, ip.o_hop, (size_t)n_it * 4);
        download(ctx, res->thetas, ip.o_hth, (size_t)n_it * 8);
        if (res->substeps) download(ctx, res->substeps, ip.o_hns, (size_t)n_it * 4);
    }
    if (n_scr > 0) {
        download(ctx, res->gnorms, ip.o_hgn, (size_t)n_scr * 8);
        if (res->gmax) download(ctx, res->gmax, ip.o_hgm, (size_t)n_scr * 8);
    }
    sync(ctx);
    return GOCP_OK;
    GOCP_GUARD_END
}

}  // extern "C"
