// Host-side runtime pieces shared by the device C ABI sources.
#pragma once

#include <hip/hip_runtime.h>

#include <memory>
#include <string>
#include <vector>

#include "device.h"

struct gocp_ctx {
    int device = 0;
    hipStream_t user_stream = nullptr;   // where calls are ordered (NULL: default stream)
    hipStream_t own_stream = nullptr;    // private stream used for graph capture
    char *arena = nullptr;               // workspace of the one-shot calls
    size_t arena_cap = 0;
    // what the arena's descriptor and row tables were last written for
    // (Hamiltonian and pool uids, state, sigma, dtype); cleared when the
    // arena is reallocated (a stream change keeps them: the tables stay valid)
    uint64_t shot_h = 0, shot_p = 0;
    const void *shot_psi = nullptr, *shot_sig = nullptr;
    int shot_dtype = -1;
    std::string arch;
    int n_cu = 0;
};

namespace gocp {

enum {
    K_ENERGY_SCREEN = 0, K_SCREEN_REDUCE = 1, K_LINE_VW = 2, K_LINE_HVW = 3, K_TAYLOR = 4,
    K_NORMALIZE = 5, K_UNIT_NORM = 6, K_SCREEN_SUM1 = 7,
    // the energy+screen launch with the X-class screen (members whose pools
    // are single strings with such tables, one amplitude per lane; any other R
    // launches K_ENERGY_SCREEN)
    K_ENERGY_SCREEN_X = 8,
    // the selection kernels for pools of more than kPairBlock operators (a
    // thread sums several operator columns)
    K_SCREEN_REDUCE_W = 9, K_LINE_VW_W = 10
};

// The kernel a variant id stands for (timing hooks name the plain ids).
inline int base_kid(int kid) {
    return kid == K_ENERGY_SCREEN_X ? K_ENERGY_SCREEN
           : kid == K_SCREEN_REDUCE_W ? K_SCREEN_REDUCE
           : kid == K_LINE_VW_W       ? K_LINE_VW
                                      : kid;
}

// Re-optimisation layers (one block of kPairBlock pairs per 2 kPairBlock
// amplitudes): out = T5(x)^ns in for pool generator j; and the backward step
// (partial[block] of Re <lam | dL phi>, lam <- L^+ lam; lam formed from sigma,
// psi and the state record's energy when sigma is not null).
void launch_layer_fwd(int dtype, const void *in, void *out, const HClass *pop, const HTerm *pterm, int j, int ns,
                      double x, int nq, hipStream_t s);
void launch_layer_adj(int dtype, const void *phi, double2 *lam, double *partial, const HClass *pop,
                      const HTerm *pterm, int j, int ns, double x, int nq, const double2 *sigma, const void *psi,
                      const AdaptState *st, hipStream_t s);

// R = amplitudes per lane of the tile kernels (1, 2 or 4); the pair kernels ignore it.
// For K_SCREEN_SUM1, j is the number of operator column blocks of kPairBlock
// (sum1_blocks; 0 or 1: one block, whose threads loop over further columns).
// t0 / t1, when set, take the dispatch's own start / end timestamps
// (hipExtLaunchKernel), so the span between them holds the kernel alone and not
// the queue's launch latency; with no rows to launch they are recorded at once.
inline int sum1_blocks(int M) { return M > kPairBlock ? (M + kPairBlock - 1) / kPairBlock : 1; }
void launch_kernel(int which, int dtype, int R, const InstDev *insts, const int2 *blk, int nblk, int mode,
                   hipStream_t s, int j = 0, double th = 0.0, int ns = 0, hipEvent_t t0 = nullptr,
                   hipEvent_t t1 = nullptr);
// Compacted H v, H w launch (complex64 states with a compaction list): rows
// (instance, slot P + part), P = hvw_parts; t0 / t1 as for launch_kernel.
void launch_hvw_act(const InstDev *insts, const int2 *blk, int nblk, int mode, hipStream_t s,
                    hipEvent_t t0 = nullptr, hipEvent_t t1 = nullptr);
void launch_basis(int dtype, void *psi, uint32_t dim, uint32_t index, hipStream_t s);
// Copy n values of the phase trace (kPhaseRows x kPhases) from the current
// device; false in builds without GOCP_PHASE_TRACE.
bool phase_trace_read(unsigned long long *out, size_t n);
void launch_scale_copy(int dtype, const void *src, void *dst, uint32_t dim, double scale, hipStream_t s);
void launch_sector_weight(int dtype, const void *psi, uint32_t dim, const SectorRows &rows, double *part, int nblk,
                          hipStream_t s);
// Queue sigma = H psi and the energy of psi (one-shot workspace of ctx) on the
// context stream; returns the device state record holding e_num, nrm, energy.
const AdaptState *enqueue_energy_sigma(gocp_ctx *ctx, const Ham *h, const void *psi, int dtype, double2 *sigma);
// GOCP multi-operator step over the pair-block rows (norm partials in part_t).
void launch_fused(int dtype, int n, const InstDev *insts, const int2 *blk, int nblk, const FuseArgs &fa,
                  hipStream_t s);
void launch_gather_done(const InstDev *insts, int n, int32_t *out, hipStream_t s);

// Byte offsets of one instance's buffers inside its workspace.
struct InstPlan {
    int n_qubits = 0, M = 0, max_iter = 0, dtype = 0;
    int n_tiles = 0, n_pblk = 0;
    int n_groups = 0;
    size_t o_sigma = 0, o_v = 0, o_w = 0, o_pe = 0, o_pn = 0, o_pg = 0, o_pg2 = 0, o_pe2 = 0, o_pn2 = 0, o_pl = 0, o_pt = 0,
           o_st = 0, o_he = 0, o_hop = 0, o_hth = 0, o_hgn = 0, o_hgm = 0, o_hns = 0,
           o_hpr = 0, o_g = 0, o_psi = 0, o_hv = 0, o_hw = 0, o_act = 0, o_actn = 0;
    size_t bytes = 0;
};

// Lay out the workspace of one instance; own_psi reserves room for the state
// too, adapt (FP64 states only) the H v and H w an ADAPT iteration keeps.
InstPlan plan_instance(int nq, int M, int max_iter, int dtype, bool own_psi, bool adapt = true);

// Device copies of a Hamiltonian's / pool's tables on device `dev`, uploaded
// on first use (allocates).  The *_resident forms never upload: they return
// nullptr when the tables are not on the device yet.
const DeviceHam *device_ham(const Ham &h, int dev);
const DevicePool *device_pool(const Pool &p, int dev);
const DeviceHam *device_ham_resident(const Ham &h, int dev);
const DevicePool *device_pool_resident(const Pool &p, int dev);

// Descriptor of an instance whose workspace starts at `base`; with upload
// false the tables must already be resident (else GOCP_EINVAL).
InstDev make_desc(int device, const InstPlan &ip, char *base, const Ham *h, const Pool *p, void *psi,
                  double2 *sigma_override, bool upload = true);
// The same with the tables given (either may be null).
InstDev make_desc_at(const InstPlan &ip, char *base, const DeviceHam *dh, const DevicePool *dp, void *psi,
                     double2 *sigma_override);

// A handle's device tables laid out in one pinned host buffer: `ham` / `pool`
// hold the arrays' byte offsets in the pointer fields, and place_* turns them
// into a DeviceHam / DevicePool for a copy of the image at a device address.
struct TableImage {
    char *host = nullptr;     // pinned (hipHostMalloc)
    size_t bytes = 0;         // a multiple of 256
    DeviceHam ham;
    DevicePool pool;
    ~TableImage();
};
std::shared_ptr<const TableImage> ham_image(const Ham &h);
std::shared_ptr<const TableImage> pool_image(const Pool &p);
DeviceHam place_ham(const TableImage &im, char *base, int device);
DevicePool place_pool(const TableImage &im, char *base, int device);
AdaptState make_state(const InstPlan &ip, char *base, int max_iter, double grad_tol, bool hist);

const Ham *as_ham(const gocp_ham *h);
const Pool *as_pool(const gocp_pool *p);
void check_ctx(gocp_ctx *ctx);
void check_dtype(int dtype);

}  // namespace gocp

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
