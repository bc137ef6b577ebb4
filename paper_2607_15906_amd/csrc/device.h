// Device-side data structures shared by the HIP sources (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "internal.h"

namespace gocp {

// Waves per workgroup of the tile kernels, and lanes per wave on CDNA.
constexpr int kWave = 64;
constexpr int kNW = 16;
constexpr int kTile = kWave;           // amplitudes per tile (one per lane)
constexpr int kPairBlock = 256;        // threads (= amplitude pairs) per pair-kernel block
// Term tables are staged into LDS in chunks of at most this many records.
constexpr int kStageTerms = 4096;      // strings (64 KiB)
constexpr int kStageCls = 1024;        // classes or operators (16 KiB)
// Each class or operator of the staged tables is padded with zero strings to a
// whole number of groups of this many strings (the tile kernels read and sum
// strings a group at a time).
constexpr int kStrGroup = 4;
// Groups of H's strings taken per step by the one-amplitude-per-lane walk, and
// the zero groups that pad H's Z-mask and X-mask tables at their end (a step
// that runs past a wave's last group reads them; its coefficients are zero).
constexpr int kWalkBatch = 2;
constexpr int kTablePadGroups = 16;
static_assert(kTablePadGroups >= 4 * kWalkBatch, "the walk reads up to 4 kWalkBatch - 1 groups past a run");
// Fixed per-record VALU cost estimates used to balance records over the waves
// of a tile block (an H class; a screened operator, which adds a wave sum).
constexpr int kClassCost = 10;
constexpr int kOpCost = 36;
// Strings a pair kernel reads at once; each pool operator's strings are padded
// to a multiple of it (zero strings) in pool order.
constexpr int kPairGroup = 8;
// A screened operator whose strings share their Z bits outside a mask b of at
// most kFactBits bits has f(d) = (-1)^popcount(d & z_b) F(d & b); when F is
// nonzero at no more than two patterns t1, t2 (values v1, v2), the operator is
// stored as one group of parameters {v1, v2, 0, 0 | z_b, b, t1, t2} and its
// X mask carries this flag.
constexpr uint32_t kFactBit = 0x80000000u;
constexpr int kFactBits = 4;
// Phase trace of the energy+screen launch (builds with GOCP_PHASE_TRACE):
// workgroups recorded and points per workgroup.
constexpr int kPhaseRows = 1024;
constexpr int kPhases = 6;
// Tiles per group in the first stage of the screen reduction.
constexpr int kGroup = 16;
// Compacted H v, H w launch (complex64 states): each tile of 64 active
// amplitudes is spread over P workgroups, each applying 1 / P of H's classes,
// with P (the group's schedule) kHvwPartsHi or kHvwPartsLo: at 14 qubits one
// instance runs its launch in 6.1 us with 8 and 7.2 us with 4 or 16, while
// the 64-instance batch runs 8 % faster with 4 (2 is no faster).  An instance
// gets at most kHvwSlots tile slots (its workgroups loop over further tiles),
// and states whose pair blocks number more than kActMaxBlocks use the
// whole-state launch.
constexpr int kHvwPartsHi = 8;
constexpr int kHvwPartsLo = 4;
constexpr int kHvwSlots = 32;
// Class records per batch of the compacted launch's walk (table values read
// through the scalar cache): two measured faster than three or four at 14
// qubits (6.1 against 6.2 and 6.7 us per launch), whose larger batches spill
// scalar registers.
constexpr int kHvwBatch = 2;

// Occupation decoding of a basis index (bit j = parity(r[j] & index)) and the
// electron count of the sector, passed by value to the sector-weight kernel.
struct SectorRows {
    uint32_t r[32];
    int32_t n, ne;
};

// GOCP multi-operator step: at most kFuseMax operators of one family per pass.
constexpr int kFuseMax = 4;
struct FuseArgs {
    int32_t op[kFuseMax];     // pool indices
    int32_t ns[kFuseMax];     // substeps (0: the operator is skipped)
    int32_t piv[kFuseMax];    // echelon pivot bits of the X masks' span, ascending
    double x[kFuseMax];       // substep angle theta / ns
};
constexpr int kActMaxBlocks = 1024;
// Launch mode of k_screen_reduce that selects the pending partials of an
// ADAPT run (the iteration and mode k_energy_screen recorded with them).
constexpr int kModePending = 5;

// A folded Pauli string as the pair kernels read it (16 bytes): the magnitude
// of its coefficient, its Z mask, and the coefficient's sign bit, so that the
// signed term at amplitude d is |c| with sign bit popcount(d & z) + sign.
// The tile kernels read the same data from two arrays instead: the
// magnitudes (FP64; staged in LDS and read by broadcast) and the Z masks with
// the sign in bit 31 (`zs`, read through the scalar cache), so that only
// eight bytes per string cross the LDS into the vector registers.
struct HTerm {
    double c;        // |c|
    uint32_t z;
    uint32_t sign;   // 1 if c < 0
};

// Start offsets (relative to the class's first string, 16 bits each) of the
// eight sub-buckets of a class's strings.  Within a class the strings are
// ordered by key = 4 z_6 + 2 z_7 + z_8 (bits 6-8 of the Z mask, the register
// bits of a lane's amplitudes), so every grouping of the strings by z_6, or by
// (z_6, z_7), is a union of consecutive sub-buckets.
struct HSub {
    uint32_t w[4];
};

// An X-mask class of H (or a pool operator): its mask and string range.
struct HClass {
    uint32_t x;
    int32_t s0, s1;
    int32_t pad;
};

// Per-iteration ADAPT state of one instance, resident in device memory.
struct AdaptState {
    int32_t iter;          // operators appended so far
    int32_t max_iter;
    int32_t done;          // set when converged or max_iter reached
    int32_t converged;
    int32_t jsel;          // operator chosen by the current screen
    int32_t nsub;          // Taylor substeps of the current update
    int32_t status;        // 0 ok, else a GOCP_E* code raised on the device
    int32_t pad0;
    int32_t pend_it;       // iteration and mode of the screen partials awaiting
    int32_t pend_mode;     // selection (written by k_energy_screen)
    int32_t sel_it;        // iteration and mode of the partials the standalone
    int32_t sel_mode;      // selection last recorded (k_screen_reduce)
    double grad_tol;
    double theta;          // angle of the current update
    double e_num;          // sum Re<psi|sigma> of the stored state
    double nrm;            // sum |psi|^2 of the stored state
    double energy;         // e_num / nrm
    double gnorm, gmax;
    double pred;           // line-search landscape value at theta
    // the update as a whole: T5(theta/s)^s = I + upd_alpha A + upd_beta A^2
    // (A^3 = -A), applied to upd_scale * psi
    double upd_alpha, upd_beta, upd_scale;
    // history (device arrays; may be null for one-shot calls)
    double *hist_e;        // max_iter + 1
    int32_t *hist_op;      // max_iter
    double *hist_theta;    // max_iter
    double *hist_gnorm;    // max_iter + 1
    double *hist_gmax;     // max_iter + 1
    int32_t *hist_nsub;    // max_iter
    double *hist_pred;     // max_iter
    double *g;             // M gradients of the latest screen
};

// One instance as the kernels see it.
struct InstDev {
    // Hamiltonian, grouped by X mask
    const HClass *hcls;
    const double *hcoef;        // |c| of H's strings, class by class
    const uint32_t *hzs;        // z | sign << 31 of the same strings
    const HSub *hsub;
    const int4 *hchunk;         // per LDS stage: class range [x, y), string range [z, w)
    const int32_t *hseg;        // n_hchunks x (kNW + 1) class boundaries of the waves
    const int32_t *hsegp;       // n_hchunks x (kNW P + 1): each wave's run cut into P = hvw_parts
    const int32_t *hsegp_lo;    // the same with P = kHvwPartsLo (hsegp holds kHvwPartsHi until a
                                // group schedule selects this one)
    // the grouped walk's table (one amplitude per lane): per chunk, factored
    // classes' parameter groups, then the other classes' groups of strings
    const double *hcoefG;
    const uint32_t *hzsG;
    const int4 *hchunkG;        // per chunk: start, end of the factored groups, end (in strings)
    const uint32_t *hgx;        // X mask of each group of hcoefG / hzsG
    const int32_t *hgseg;       // n_hchunks x 2 (kNW + 1): the waves' runs of each kind (group indices)
    // pool, in pool order (pair kernels)
    const HClass *pop;          // one record per operator
    const HTerm *pterm;
    const double *op_norm1;
    // pool in GOCP family order (gradient screen); HClass.pad = pool index;
    // factored operators have x | kFactBit and one group of parameters
    const HClass *sop;
    const double *scoef;        // |c| and z | sign << 31 of the screen's strings
    const uint32_t *szs;
    const HSub *psub;
    const int4 *pchunk;         // per LDS stage: operator range [x, y), string range [z, w)
    const int32_t *pseg;        // n_pchunks x (kNW + 1) operator boundaries of the waves
    // pools of single-string operators, screen at one amplitude per lane: one
    // record per X mask {x, s0, s1, count} whose strings [s0, s1) are
    // operators (xop: their pool indices), so one gather serves them all;
    // strings packed without padding inside an LDS stage chunk (n_xchunks = 0:
    // not built)
    const HClass *xrec;
    const double *xcoef;
    const uint32_t *xzs;
    const int32_t *xop;
    const int4 *xchunk;         // per LDS stage: record range [x, y), string range [z, w) (w padded)
    const int32_t *xseg;        // n_xchunks x (kNW + 1) record boundaries of the waves
    // buffers (psi, v, w in the state precision; sigma FP64)
    void *psi;
    double2 *sigma;
    void *v;
    void *w;
    double2 *hv;                // H v and H w (FP64), kept by the line search for the
    double2 *hw;                // next sigma; null outside ADAPT runs of FP64 states
    uint32_t *act;              // per pair block, the amplitudes where v or w is nonzero
    int32_t *act_n;             // (compacted by k_line_vw; null unless compacted)
    double *part_e;             // n_tiles
    double *part_n;             // n_tiles
    double *part_g;             // n_tiles * M
    double *part_g2;            // n_groups * M (sums over groups of kGroup tiles)
    double *part_e2;            // n_groups
    double *part_n2;            // n_groups
    double *part_l;             // 2 * n_pblk + 3 * n_lpart (line-search dots)
    double *part_t;             // n_pblk (Taylor norms)
    AdaptState *st;
    int32_t n_qubits;
    int32_t M;
    int32_t n_tiles;
    int32_t n_pblk;
    int32_t n_hchunks;
    int32_t n_pchunks;
    int32_t n_xchunks;
    int32_t n_groups;
    int32_t n_lpart;            // workgroups of the H v, H w launch (partial triples)
    int32_t hvw_parts;          // P of the compacted H v, H w launch (kHvwPartsHi or kHvwPartsLo)
};

// Device tables of a Hamiltonian or pool: every array lies in one block of
// device memory (`base`, laid out as the handle's TableImage), either owned
// by the handle's per-device cache or placed inside a serving request's block.
struct DeviceHam {
    int device = -1;
    char *base = nullptr;
    HClass *hcls = nullptr;
    double *hcoef = nullptr;
    uint32_t *hzs = nullptr;
    HSub *hsub = nullptr;
    int4 *hchunk = nullptr;
    int32_t *hseg = nullptr;     // per chunk, kNW + 1 wave boundaries of its classes
    int32_t *hsegp = nullptr;    // per chunk, kNW kHvwPartsHi + 1 boundaries of the waves' runs
    int32_t *hsegp_lo = nullptr; // per chunk, kNW kHvwPartsLo + 1 boundaries
    double *hcoefG = nullptr;    // the grouped walk's table (see InstDev)
    uint32_t *hzsG = nullptr;
    int4 *hchunkG = nullptr;
    uint32_t *hgx = nullptr;
    int32_t *hgseg = nullptr;
    int n_chunks = 0;
};

struct DevicePool {
    int device = -1;
    char *base = nullptr;
    HClass *pop = nullptr;
    HTerm *pterm = nullptr;
    double *op_norm1 = nullptr;
    HClass *sop = nullptr;
    double *scoef = nullptr;
    uint32_t *szs = nullptr;
    HSub *psub = nullptr;
    int4 *pchunk = nullptr;
    int32_t *pseg = nullptr;     // per chunk, kNW + 1 wave boundaries of its operators
    int n_chunks = 0;
    // X-class screen of a pool of single-string operators (n_xchunks = 0: none)
    HClass *xrec = nullptr;
    double *xcoef = nullptr;
    uint32_t *xzs = nullptr;
    int32_t *xop = nullptr;
    int4 *xchunk = nullptr;
    int32_t *xseg = nullptr;
    int n_xchunks = 0;
};

void hip_check(hipError_t e, const char *what);

}  // namespace gocp
