// HIP kernels of the GOCP ADAPT-VQE hot path for gfx950 (CDNA4).
//
// All statevector work is the application of folded Pauli terms
//   (c Z^z X^x psi)[d] = c (-1)^popcount(d & z) psi[d ^ x]
// to a 2^n statevector.  Two kernel shapes carry it:
//
// * Tile kernels (energy / H apply, gradient screen, the H v / H w products of
//   the line search).  A workgroup owns 64 consecutive amplitudes, one per
//   lane, and its 16 waves split the work items (X-mask classes of H; the
//   pool operators in GOCP family order, or, for pools of single strings,
//   their X masks with the member operators) between them.  For one X mask the 64
//   gathered partners psi[d ^ x] form one aligned 64-amplitude block, so every
//   gather is a fully coalesced, permuted block read.  Term tables are wave
//   uniform and stream through scalar loads.  Per-wave partial results meet
//   in LDS and are summed in a fixed order.
// * Pair kernels (Taylor update, line-search vectors).  A pool generator has
//   one X mask x, so it acts independently on the pairs (d, d ^ x); one lane
//   owns one pair, runs the whole substepped fifth-order chain (Sec. III.B,
//   Eq. 5-6) in FP64 registers and writes the pair back: one read and one
//   write of the state per update instead of five matrix-vector passes.
//
// Reductions are deterministic: wave butterflies, then fixed-order sums over
// waves inside a workgroup.  Every cross-workgroup sum is formed by a later
// launch that reads the plain-stored per-workgroup partials in a fixed order
// (no atomics, no arrival counters, no floating-point atomics), so results are
// bit-reproducible and do not depend on which instances share a launch (one
// exception: a pool of single strings is screened by the X-class launch only
// when every member of the launch has such a pool, and that launch sums a
// record's members over the wave in another order than the per-operator one,
// so such a member's gradients can differ in the last bits between the two).

#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <algorithm>
#include <cmath>

#include "device.h"

namespace gocp {

// ------------------------------------------------------------------ phase trace

// Builds with GOCP_PHASE_TRACE record, for every ADAPT-iteration launch of the
// energy+screen kernel, the device's constant-rate clock (s_memrealtime) at
// kPhases points of each workgroup (kPhaseRows rows; a later launch overwrites
// them): the entry, the end of the prologue, the H stage written, the end of
// the H walk in the last wave, sigma and the energy partials done, the end of
// the screen in the last wave.  Other builds record nothing.
#ifdef GOCP_PHASE_TRACE
__device__ unsigned long long g_phase[kPhaseRows * kPhases];
__device__ __forceinline__ void phase_mark(int slot, int mode) {
    if (mode == 2 && threadIdx.x == 0 && blockIdx.x < kPhaseRows)
        ((volatile unsigned long long *)g_phase)[blockIdx.x * kPhases + slot] = __builtin_amdgcn_s_memrealtime();
}
__device__ __forceinline__ void phase_mark_last(int slot, int mode) {
    if (mode == 2 && (threadIdx.x & (kWave - 1)) == 0 && blockIdx.x < kPhaseRows)
        atomicMax(&g_phase[blockIdx.x * kPhases + slot], __builtin_amdgcn_s_memrealtime());
}
#else
__device__ __forceinline__ void phase_mark(int, int) {}
__device__ __forceinline__ void phase_mark_last(int, int) {}
#endif

// ------------------------------------------------------------------ helpers

// Global-memory loads go through the global address space (not flat), so
// they count only against the vector-memory wait counter and LDS reads do not
// wait for gathers in flight.
#define GOCP_AS1 __attribute__((address_space(1)))
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// State element access: raw() loads the stored bits, cvt() widens to FP64.
// Period (in ADAPT iterations) of the fresh H psi that resets the carried sigma:
// the stored state is rounded to its precision at every update while the
// carried sigma follows the unrounded update, so the energy and gradients
// formed with a carried sigma are off by a term of first order in that
// rounding.  For FP64 states this is ~1e-15 and sigma is carried between
// fresh applications every 32 iterations.  For complex64 states it is ~1e-7 Ha
// at 14 qubits (against ~1e-10 with a fresh H psi, whose Rayleigh quotient is
// second order in the rounding), so complex64 states apply H afresh every
// iteration and do not keep H v, H w.
template <typename T> struct Refresh;
template <> struct Refresh<float2> { static constexpr int kPeriod = 1; };
template <> struct Refresh<double2> { static constexpr int kPeriod = 32; };

template <typename T> struct Amp;
template <> struct Amp<double2> {
    using Raw = u32x4;
    static constexpr int kShift = 4;       // log2 of the element size
    static __device__ __forceinline__ Raw raw(const void *p, uint32_t i) {
        return ((const GOCP_AS1 u32x4 *)(uintptr_t)p)[i];
    }
    // element at byte offset `off` (a multiple of the element size)
    static __device__ __forceinline__ Raw raw_at(const void *p, uint32_t off) {
        return *(const GOCP_AS1 u32x4 *)((const GOCP_AS1 char *)(uintptr_t)p + off);
    }
    static __device__ __forceinline__ double2 cvt(Raw r) {
        return make_double2(__hiloint2double((int)r.y, (int)r.x), __hiloint2double((int)r.w, (int)r.z));
    }
    static __device__ __forceinline__ double2 load(const void *p, uint32_t i) { return cvt(raw(p, i)); }
    static __device__ __forceinline__ void store(void *p, uint32_t i, double2 v) {
        static_cast<double2 *>(p)[i] = v;
    }
    static __device__ __forceinline__ double2 rounded(double2 v) { return v; }
};
template <> struct Amp<float2> {
    using Raw = u32x2;
    static constexpr int kShift = 3;
    static __device__ __forceinline__ Raw raw(const void *p, uint32_t i) {
        return ((const GOCP_AS1 u32x2 *)(uintptr_t)p)[i];
    }
    static __device__ __forceinline__ Raw raw_at(const void *p, uint32_t off) {
        return *(const GOCP_AS1 u32x2 *)((const GOCP_AS1 char *)(uintptr_t)p + off);
    }
    static __device__ __forceinline__ double2 cvt(Raw r) {
        return make_double2((double)__uint_as_float(r.x), (double)__uint_as_float(r.y));
    }
    static __device__ __forceinline__ double2 load(const void *p, uint32_t i) { return cvt(raw(p, i)); }
    static __device__ __forceinline__ void store(void *p, uint32_t i, double2 v) {
        static_cast<float2 *>(p)[i] = make_float2((float)v.x, (float)v.y);
    }
    static __device__ __forceinline__ double2 rounded(double2 v) {
        return make_double2((double)(float)v.x, (double)(float)v.y);
    }
};

// Read-only tables are read through the constant address space: with a wave
// uniform index the load becomes a scalar (SMEM) load broadcast to all lanes.
#define GOCP_AS4 __attribute__((address_space(4)))
// Global-memory view of a pointer (vector loads without the flat path).
template <typename T>
__device__ __forceinline__ const GOCP_AS1 T *gptr(const T *p) {
    return (const GOCP_AS1 T *)(uintptr_t)p;
}

// Writable global-memory view (stores without the flat path: a flat store
// still in flight makes every later wait on vector loads a full wait).
template <typename T>
__device__ __forceinline__ GOCP_AS1 T *gmut(T *p) {
    return (GOCP_AS1 T *)(uintptr_t)p;
}

// Complex128 element i through the global path (one 16-byte access).
__device__ __forceinline__ double2 gload2(const double2 *p, size_t i) {
    typedef double d2v __attribute__((ext_vector_type(2)));
    const d2v v = ((const GOCP_AS1 d2v *)(uintptr_t)p)[i];
    return make_double2(v.x, v.y);
}
__device__ __forceinline__ void gstore2(double2 *p, size_t i, double2 a) {
    typedef double d2v __attribute__((ext_vector_type(2)));
    d2v v;
    v.x = a.x;
    v.y = a.y;
    ((GOCP_AS1 d2v *)(uintptr_t)p)[i] = v;
}

template <typename T>
__device__ __forceinline__ const GOCP_AS4 T *cptr(const T *p) {
    return (const GOCP_AS4 T *)(uintptr_t)p;
}

__device__ __forceinline__ HClass load_rec(const GOCP_AS4 HClass *p, int i) {
    HClass r;
    r.x = p[i].x;
    r.s0 = p[i].s0;
    r.s1 = p[i].s1;
    r.pad = p[i].pad;
    return r;
}
__device__ __forceinline__ int4 load_rec(const GOCP_AS4 int4 *p, int i) {
    return make_int4(p[i].x, p[i].y, p[i].z, p[i].w);
}
__device__ __forceinline__ HTerm load_rec(const GOCP_AS4 HTerm *p, int i) {
    HTerm r;
    r.c = p[i].c;
    r.z = p[i].z;
    r.sign = p[i].sign;
    return r;
}

// c (-1)^popcount(d & z) for c = (-1)^sign |c|: the sign bit of the result is
// the low bit of popcount(d & z) + sign, placed over |c| (popcount-with-add
// and shift-or, two instructions).
__device__ __forceinline__ double signed_coef(const HTerm &t, uint32_t d) {
    const uint32_t bit = ((uint32_t)__popc(d & t.z) + t.sign) << 31;
    return __hiloint2double((int)(bit | (uint32_t)__double2hiint(t.c)), __double2loint(t.c));
}

// The same sum at two amplitudes d and e (the two members of a pair), in
// string order.  A pool operator's strings are padded with zero strings to a
// multiple of kPairGroup, so its scalar loads go out kPairGroup at a time and
// a generator of up to kPairGroup strings waits once.
__device__ __forceinline__ void string_sum2(const GOCP_AS4 HTerm *t, int s0, int s1, uint32_t d,
                                            uint32_t e, double &hd, double &he) {
    hd = 0.0;
    he = 0.0;
    for (int s = s0; s < s1; s += kPairGroup) {
        HTerm a[kPairGroup];
#pragma unroll
        for (int q = 0; q < kPairGroup; ++q) a[q] = load_rec(t, s + q);
#pragma unroll
        for (int q = 0; q < kPairGroup; ++q) {
            hd += signed_coef(a[q], d);
            he += signed_coef(a[q], e);
        }
    }
}

__device__ __forceinline__ int state_done(const AdaptState *st) { return cptr(&st->done)[0]; }

// The workgroup's work row (instance, index).  A null table stands for a
// group of one instance, whose rows are (0, workgroup index): no load.
__device__ __forceinline__ int2 work_row(const int2 *blk) {
    if (!blk) return make_int2(0, (int)blockIdx.x);
    const GOCP_AS4 int32_t *r = cptr(reinterpret_cast<const int32_t *>(blk)) + 2 * blockIdx.x;
    return make_int2(r[0], r[1]);
}

// The leading fields of an instance's state record, read in one scalar load.
struct StHead {
    int32_t iter, max_iter, done, converged, jsel, nsub, status, pad0, pend_it, pend_mode, sel_it, sel_mode;
};
__device__ __forceinline__ StHead load_head(const AdaptState *st) {
    const GOCP_AS4 int32_t *p = cptr(reinterpret_cast<const int32_t *>(st));
    StHead h;
    h.iter = p[0];
    h.max_iter = p[1];
    h.done = p[2];
    h.converged = p[3];
    h.jsel = p[4];
    h.nsub = p[5];
    h.status = p[6];
    h.pad0 = p[7];
    h.pend_it = p[8];
    h.pend_mode = p[9];
    h.sel_it = p[10];
    h.sel_mode = p[11];
    return h;
}

// DPP move of a double (as two 32-bit halves); lanes of rows outside ROW_MASK
// receive 0.  With every row written and a pattern that reads inside the row
// (the quad permutations and mirrors) no lane keeps its old value, so the
// move takes none (no zeroing of the destination first).
template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ double dpp_f64(double v) {
    if constexpr (ROW_MASK == 0xf && (CTRL <= 0xff || CTRL == 0x140 || CTRL == 0x141)) {
        const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xf, 0xf, false);
        const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xf, 0xf, false);
        return __hiloint2double(hi, lo);
    } else {
        const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROW_MASK, 0xf, false);
        const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROW_MASK, 0xf, false);
        return __hiloint2double(hi, lo);
    }
}

__device__ __forceinline__ double read_lane(double v, int l) {
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), l),
                            __builtin_amdgcn_readlane(__double2loint(v), l));
}

// row_sum: sum over each row of 16 lanes, returned to every lane of the row:
// pairs and quads, then halves of a row and whole rows by mirroring.
// wave_sum: sum over the 64 lanes of a full wave: row sums, then rows 0+1 and
// 2+3 by broadcasting lane 15 of a row into the next, and all four by
// broadcasting lane 31 into rows 2 and 3; lane 63 ends with the total.
// Register moves only, no LDS.
__device__ __forceinline__ double row_sum(double v) {
    v += dpp_f64<0xB1>(v);          // quad_perm [1,0,3,2]
    v += dpp_f64<0x4E>(v);          // quad_perm [2,3,0,1]
    v += dpp_f64<0x141>(v);         // row_half_mirror
    v += dpp_f64<0x140>(v);         // row_mirror
    return v;
}

__device__ __forceinline__ double wave_sum(double v) {
    v = row_sum(v);
    v += dpp_f64<0x142, 0xA>(v);    // row_bcast:15 into rows 1 and 3
    v += dpp_f64<0x143, 0xC>(v);    // row_bcast:31 into rows 2 and 3
    return read_lane(v, kWave - 1);
}

// a + b after exchanging halves (W = 32: lanes 32-63 of a with lanes 0-31 of
// b, v_permlane32_swap) or odd and even rows (W = 16: v_permlane16_swap):
// lanes 0-31 (W = 32) or rows 0 and 2 (W = 16) end with the pair sums of a,
// the others with those of b.
template <int W>
__device__ __forceinline__ double swap_add(double a, double b) {
    const unsigned al = (unsigned)__double2loint(a), ah = (unsigned)__double2hiint(a);
    const unsigned bl = (unsigned)__double2loint(b), bh = (unsigned)__double2hiint(b);
    if constexpr (W == 32) {
        const auto l = __builtin_amdgcn_permlane32_swap(al, bl, false, false);
        const auto h = __builtin_amdgcn_permlane32_swap(ah, bh, false, false);
        return __hiloint2double((int)h[0], (int)l[0]) + __hiloint2double((int)h[1], (int)l[1]);
    } else {
        const auto l = __builtin_amdgcn_permlane16_swap(al, bl, false, false);
        const auto h = __builtin_amdgcn_permlane16_swap(ah, bh, false, false);
        return __hiloint2double((int)h[0], (int)l[0]) + __hiloint2double((int)h[1], (int)l[1]);
    }
}

// Sums over the 64 lanes of eight values at once: halves of the wave, then
// rows, then the two halves of each row (row mirror) and the eight lanes of
// each half-row.  Lane l ends with the sum of v[l >> 3].  Register moves
// only; every lane of the wave active.
__device__ __forceinline__ double fold8(const double (&v)[8]) {
    double w[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) w[i] = swap_add<32>(v[i], v[i + 4]);
    const double u0 = swap_add<16>(w[0], w[2]), u1 = swap_add<16>(w[1], w[3]);
    const bool up = threadIdx.x & 8;
    double t = (up ? u1 : u0) + dpp_f64<0x140>(up ? u0 : u1);   // row_mirror
    t += dpp_f64<0xB1>(t);          // quad_perm [1,0,3,2]
    t += dpp_f64<0x4E>(t);          // quad_perm [2,3,0,1]
    t += dpp_f64<0x141>(t);         // row_half_mirror
    return t;
}

__device__ __forceinline__ int wave_id() {
    return __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
}

// Sum of `n` values at stride `stride` from `src`, in index order per thread
// and a fixed tree over threads; the result is returned to every thread.
// Sum of one value per thread over a block of NT threads: per-wave sums, then
// the NT / 64 wave sums in wave order; returned to every thread.
template <int NT>
__device__ __forceinline__ double block_reduce(double acc, double *lds) {
    const double w = wave_sum(acc);
    if ((threadIdx.x & (kWave - 1)) == 0) lds[threadIdx.x >> 6] = w;
    __syncthreads();
    double r = 0.0;
#pragma unroll
    for (int k = 0; k < NT / kWave; ++k) r += lds[k];
    __syncthreads();
    return r;
}

template <int NT>
__device__ double block_sum_strided(const double *src, int n, int stride, double *lds) {
    double acc = 0.0;
    for (int i = threadIdx.x; i < n; i += NT) acc += src[(size_t)i * stride];
    return block_reduce<NT>(acc, lds);
}


// ------------------------------------------------------------------ LDS staging of term tables

// Shared memory of a tile kernel: one chunk of records (classes or
// operators), their sub-bucket offsets and their strings' coefficient
// magnitudes (the strings' Z masks are read through the scalar cache); reused
// for the cross-wave reduction.
struct Stage {
    double coef[kStageTerms + kStrGroup];   // the chunk's magnitudes, then one zero group
    HClass cls[kStageCls];
    HSub sub[kStageCls];
};

// Stage the coefficient magnitudes [sb, se) of a chunk (sb and se are
// multiples of kStrGroup, so whole 16-byte pairs are copied).
__device__ __forceinline__ void stage_coef(Stage &S, const double *co, int sb, int se);

// Copy n 16-byte records from global memory to LDS with the whole workgroup
// (kNW * kWave threads), four loads in flight per thread.
template <typename R>
__device__ __forceinline__ void stage_copy(R *dst, const R *src, int n) {
    static_assert(sizeof(R) == 16, "records are 16 bytes");
    constexpr int NT = kNW * kWave;
    const GOCP_AS1 u32x4 *s = (const GOCP_AS1 u32x4 *)(uintptr_t)src;
    u32x4 *d = reinterpret_cast<u32x4 *>(dst);
    int i = threadIdx.x;
    for (; i + 3 * NT < n; i += 4 * NT) {
        const u32x4 a = s[i], b = s[i + NT], c = s[i + 2 * NT], e = s[i + 3 * NT];
        d[i] = a;
        d[i + NT] = b;
        d[i + 2 * NT] = c;
        d[i + 3 * NT] = e;
    }
    for (; i < n; i += NT) d[i] = s[i];
}

__device__ __forceinline__ void stage_coef(Stage &S, const double *co, int sb, int se) {
    stage_copy(reinterpret_cast<u32x4 *>(S.coef), reinterpret_cast<const u32x4 *>(co + sb), (se - sb) / 2);
    if (threadIdx.x < kStrGroup) S.coef[kStageTerms + threadIdx.x] = 0.0;
}

// |c| with sign bit popcount(d & z) + sign, for zs = z | sign << 31 and
// dz = d | 1 << 31 (d < 2^31): popcount(dz & zs) counts the sign bit with
// the Z bits (and, popcount, shift-or).
__device__ __forceinline__ double signed_cz(double c, uint32_t zs, uint32_t dz) {
    const uint32_t bit = (uint32_t)__popc(dz & zs) << 31;
    return __hiloint2double((int)(bit | (uint32_t)__double2hiint(c)), __double2loint(c));
}
__device__ __forceinline__ uint32_t with_sign_bit(uint32_t d) { return d | 0x80000000u; }

// sum_s c_s (-1)^popcount(d & z_s) over the chunk's strings [s0, s1): every
// lane reads the same magnitude from LDS (a broadcast) and the same Z mask
// through the scalar cache (zs = the chunk's masks), four strings per step;
// d = with_sign_bit(amplitude).
__device__ __forceinline__ double lds_string_sum(const double *co, const GOCP_AS4 uint32_t *zs, int s0, int s1,
                                                 uint32_t d) {
    double f0 = 0.0, f1 = 0.0;
    int s = s0;
    for (; s + 4 <= s1; s += 4) {
        const double a = co[s], b = co[s + 1], c = co[s + 2], e = co[s + 3];
        f0 += signed_cz(a, zs[s], d);
        f1 += signed_cz(b, zs[s + 1], d);
        f0 += signed_cz(c, zs[s + 2], d);
        f1 += signed_cz(e, zs[s + 3], d);
    }
    for (; s < s1; ++s) f0 += signed_cz(co[s], zs[s], d);
    return f0 + f1;
}

__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Register blocking.  A lane of a tile kernel holds R amplitudes
// d_r = d0 + 64 r (r < R, d0 with bits 6.. of r zero), so the sign of a string
// at d_r is (-1)^popcount(d0 & z) times (-1)^popcount(r & u) with u the
// string's register bits (z_6, z_7).  Strings are summed once at d0 into one
// bucket per u, and f_r = sum_u (-1)^popcount(r & u) G_u is a Walsh-Hadamard
// transform of the buckets: one signed term per string for all R amplitudes.
//
// Bucket i of R: value u and the range [k0, k1) of sub-buckets it spans
// (sub-bucket key = 4 z_6 + 2 z_7 + z_8).
template <int R>
__device__ __forceinline__ void bucket(int i, int &u, int &k0, int &k1) {
    if (R == 1) { u = 0; k0 = 0; k1 = 8; }
    else if (R == 2) { u = i; k0 = 4 * i; k1 = 4 * i + 4; }
    else { const int b6 = i >> 1, b7 = i & 1; u = b6 | (b7 << 1); k0 = 2 * i; k1 = 2 * i + 2; }
}

// In-place transform G_u -> f_r = sum_u (-1)^popcount(r & u) G_u.
template <int R>
__device__ __forceinline__ void wht(double *g) {
#pragma unroll
    for (int h = 1; h < R; h <<= 1)
#pragma unroll
        for (int i = 0; i < R; i += 2 * h)
#pragma unroll
            for (int j = i; j < i + h; ++j) {
                const double a = g[j], b = g[j + h];
                g[j] = a + b;
                g[j + h] = a - b;
            }
}

// Class (or operator) c of the staged chunk: f_r for the lane's R amplitudes
// (zs = the chunk's Z masks).
// Flagged records (kFactBit in the X mask) hold one group of parameters:
// factored H classes (FK = kFactH: f = |v| (-1)^popcount(dz & m0) when
// popcount(dz & m1) and popcount(dz & m2) are even, dz = d | 1 << 31) or
// factored pool operators (FK = kFactPool).
constexpr int kFactNone = 0, kFactPool = 1, kFactH = 2;
__device__ __forceinline__ double fact_h(double v, uint32_t m0, uint32_t m1, uint32_t m2, uint32_t dz) {
    const uint32_t off = ((uint32_t)__popc(dz & m1) | (uint32_t)__popc(dz & m2)) & 1u;
    const uint32_t keep = off - 1u;                  // all ones when both are even
    const uint32_t hi = ((uint32_t)__popc(dz & m0) << 31) | (uint32_t)__double2hiint(v);
    return __hiloint2double((int)(hi & keep), (int)((uint32_t)__double2loint(v) & keep));
}

template <int R, int FK = kFactNone>
__device__ __forceinline__ void class_coeffs(const Stage &S, const GOCP_AS4 uint32_t *zs, int c, int sb, uint32_t d0,
                                             double *f) {
    const int s0 = uni(S.cls[c].s0) - sb, s1 = uni(S.cls[c].s1) - sb;
    if constexpr (FK == kFactH) {
        if ((uint32_t)uni((int)S.cls[c].x) & kFactBit) {
            const double v = S.coef[s0];
            const uint32_t m0 = zs[s0], m1 = zs[s0 + 1], m2 = zs[s0 + 2];
#pragma unroll
            for (int r = 0; r < R; ++r) f[r] = fact_h(v, m0, m1, m2, with_sign_bit(d0 | ((uint32_t)r << 6)));
            return;
        }
    }
    if constexpr (FK == kFactPool) {
        // a factored operator, evaluated at each of the lane's amplitudes
        if ((uint32_t)uni((int)S.cls[c].x) & kFactBit) {
            const double v1 = S.coef[s0], v2 = S.coef[s0 + 1];
            const uint32_t zb = zs[s0], bm = zs[s0 + 1], t1 = zs[s0 + 2], t2 = zs[s0 + 3];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const uint32_t d = d0 | ((uint32_t)r << 6), u = d & bm;
                double v = u == t1 ? v1 : 0.0;
                v = u == t2 ? v2 : v;
                const uint32_t bit = (uint32_t)__popc(d & zb) << 31;
                f[r] = __hiloint2double((int)((uint32_t)__double2hiint(v) ^ bit), __double2loint(v));
            }
            return;
        }
    }
    const uint32_t dz = with_sign_bit(d0);
    if (R == 1) {
        f[0] = lds_string_sum(S.coef, zs, s0, s1, dz);
        return;
    }
    uint32_t w[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) w[i] = (uint32_t)uni((int)S.sub[c].w[i]);
    double g[R];
#pragma unroll
    for (int i = 0; i < R; ++i) {
        int u, k0, k1;
        bucket<R>(i, u, k0, k1);
        const int a = (int)((w[k0 >> 1] >> (16 * (k0 & 1))) & 0xffffu);
        const int e = k1 >= 8 ? s1 - s0 : (int)((w[k1 >> 1] >> (16 * (k1 & 1))) & 0xffffu);
        g[u] = lds_string_sum(S.coef, zs, s0 + a, s0 + e, dz);
    }
    wht<R>(g);
#pragma unroll
    for (int r = 0; r < R; ++r) f[r] = g[r];
}

// Byte offsets of the lane's R amplitudes d0 + 64 r in a vector of elements
// of 2^SH bytes, 0 for an amplitude beyond the state; the partner of
// amplitude r under X mask x is then at byte offset off[r] ^ (x << SH)
// (element x, in range, for an amplitude beyond the state).
template <int R, int SH>
__device__ __forceinline__ void lane_offsets(uint32_t d0, uint32_t dim, uint32_t (&off)[R]) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const uint32_t d = d0 | ((uint32_t)r << 6);
        off[r] = d < dim ? d << SH : 0u;
        asm volatile("" : "+v"(off[r]));  // keep the shifted offsets: one XOR per gather
    }
}

// One amplitude per lane: the wave's records [c0, c1) of the staged chunk
// (classes or operators, each padded to whole groups of kStrGroup strings),
// walked as a software pipeline over two register sets.  While record c is
// summed, the first string group of record c + 1 and its gathered amplitudes
// from v0 (and v1) are in flight, and the record after that is being read.
// d must lie in the state (its bits feed the gather index directly).
// fin(c, f_c(d), raw amplitudes at d ^ x_c) is called for every record in order.
// Records flagged kFactBit hold one group of parameters instead of strings:
// factored H classes (FK = kFactH, see fact_h) or factored pool operators
// (FK = kFactPool: f(d) = (-1)^popcount(d & z_b) times v1 or v2 where d & b
// equals t1 or t2, and 0 elsewhere).
template <typename T, int NV, int FK, typename Fin>
__device__ __forceinline__ void walk_classes_r1(const Stage &S, const GOCP_AS4 uint32_t *zs, int c0, int c1, int sb,
                                                uint32_t d, const void *v0, const void *v1, Fin &&fin) {
    using Raw = typename Amp<T>::Raw;
    struct Rec {
        uint32_t x;
        int s0, s1;
    };
    struct Grp {                        // one group of strings: magnitudes and Z masks
        double c[kStrGroup];
        uint32_t z[kStrGroup];
    };
    uint32_t doff = d << Amp<T>::kShift;
    asm volatile("" : "+v"(doff));      // keep the shifted offset: one XOR per gather
    const uint32_t dz = with_sign_bit(d);
    // start reading record r: its first string group and its gathered amplitudes
    auto issue = [&](const HClass &r, Grp &g, Raw (&p)[NV]) {
        const Rec k{(uint32_t)uni((int)r.x), uni(r.s0) - sb, uni(r.s1) - sb};
#pragma unroll
        for (int q = 0; q < kStrGroup; ++q) {
            g.c[q] = S.coef[k.s0 + q];
            g.z[q] = zs[k.s0 + q];
        }
        const uint32_t o = doff ^ (k.x << Amp<T>::kShift);
        p[0] = Amp<T>::raw_at(v0, o);
        if (NV == 2) p[NV - 1] = Amp<T>::raw_at(v1, o);
        return k;
    };
    // f(d) of a record whose first group is in registers; further groups are
    // read here (the string range is uniform: scalar loop bounds)
    auto coef = [&](const Rec &k, const Grp &g) {
        if constexpr (FK == kFactH) {
            if (k.x & kFactBit) return fact_h(g.c[0], g.z[0], g.z[1], g.z[2], dz);
        }
        if constexpr (FK == kFactPool) {
            if (k.x & kFactBit) {
                const uint32_t u = d & g.z[1];
                double v = u == g.z[2] ? g.c[0] : 0.0;
                v = u == g.z[3] ? g.c[1] : v;
                const uint32_t bit = (uint32_t)__popc(d & g.z[0]) << 31;
                return __hiloint2double((int)((uint32_t)__double2hiint(v) ^ bit), __double2loint(v));
            }
        }
        double f0 = signed_cz(g.c[0], g.z[0], dz) + signed_cz(g.c[2], g.z[2], dz);
        double f1 = signed_cz(g.c[1], g.z[1], dz) + signed_cz(g.c[3], g.z[3], dz);
        const int s1 = uni(k.s1);
        for (int s = uni(k.s0) + kStrGroup; s < s1; s += kStrGroup) {
            const double a0 = S.coef[s], a1 = S.coef[s + 1], a2 = S.coef[s + 2], a3 = S.coef[s + 3];
            f0 += signed_cz(a0, zs[s], dz) + signed_cz(a2, zs[s + 2], dz);
            f1 += signed_cz(a1, zs[s + 1], dz) + signed_cz(a3, zs[s + 3], dz);
        }
        return f0 + f1;
    };
    // Reads ahead are issued unconditionally (past the end of the run they
    // re-read its last record, harmlessly), so every pass issues the same
    // loads in the same order.
    if (c0 >= c1) return;
    const int cl = c1 - 1;
    Grp gA, gB;
    Raw pA[NV], pB[NV];
    Rec kA = issue(S.cls[c0], gA, pA);
    HClass rB = S.cls[min(c0 + 1, cl)];
    for (int c = c0;; c += 2) {
        const Rec kB = issue(rB, gB, pB);
        const HClass rA = S.cls[min(c + 2, cl)];
        fin(c, coef(kA, gA), pA);
        if (c + 1 >= c1) break;
        kA = issue(rA, gA, pA);
        rB = S.cls[min(c + 3, cl)];
        fin(c + 1, coef(kB, gB), pB);
        if (c + 2 >= c1) break;
    }
}

// One amplitude per lane, for operators linear in the per-group sums (H
// applied to NV vectors): acc[2 v + {0,1}] += sum over the groups [g0, g1) of
// the staged chunk (chunk-relative) of f_g(d) vec_v[d ^ x_g], with f_g the
// signed sum of group g's kStrGroup strings and x_g its class's X mask.  The
// groups are walked K at a time as a two-stage pipeline, 2 K per pass.  Z masks and X masks
// come through the scalar cache and magnitudes from LDS; scalar loads return
// out of order, so every use of one waits for all outstanding scalar and LDS
// loads.  Each step therefore first waits for the data of its own K groups
// (issued one step earlier), and only then issues the next step's loads:
// Z masks and magnitudes of the next K groups, their gathers (with X masks
// read two steps ahead), and the X masks of the step after.  Groups past g1
// take their magnitudes from the stage's zero group; their Z and X masks are
// read from the tables' zero padding or from the following groups (a run reads
// up to 4 K - 1 groups past its end).
// d must lie in the state.
// With FG the groups are factored classes, one group of parameters each
// {|v|, 0, 0, 0 | m0, m1, m2, 0}: f(d) = |v| (-1)^popcount(dz & m0) when
// popcount(dz & m1) and popcount(dz & m2) are both even (dz = d | 1 << 31),
// else 0; only the first magnitude of a group is read from LDS.
template <typename T, int NV, int K, bool FG>
__device__ __forceinline__ void walk_groups_r1(const Stage &S, const GOCP_AS4 uint32_t *zs,
                                               const GOCP_AS4 uint32_t *gx, int g0, int g1, uint32_t d,
                                               const void *v0, const void *v1, double *acc) {
    using Raw = typename Amp<T>::Raw;
    struct Bat {
        double c[K][kStrGroup];
        uint32_t z[K][kStrGroup];
        Raw p[K][NV];
    };
    if (g0 >= g1) return;
    uint32_t doff = d << Amp<T>::kShift;
    asm volatile("" : "+v"(doff));      // keep the shifted offset: one XOR per gather
    const uint32_t dz = with_sign_bit(d);
    // the pointer and index laundering below ties each load to the wait
    // before it (the loads are not hoisted above it)
    auto load_x = [&](uint32_t (&x)[K], int g) {
        const GOCP_AS4 uint32_t *p = gx + g;
        asm volatile("" : "+s"(p));
#pragma unroll
        for (int k = 0; k < K; ++k) x[k] = p[k];
    };
    auto load_zc = [&](Bat &b, int g) {
        const GOCP_AS4 uint32_t *zp = zs + kStrGroup * g;
        asm volatile("" : "+s"(zp));
#pragma unroll
        for (int k = 0; k < K; ++k)
#pragma unroll
            for (int q = 0; q < kStrGroup; ++q) b.z[k][q] = zp[kStrGroup * k + q];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            int ci = g + k < g1 ? kStrGroup * (g + k) : kStageTerms;
            asm volatile("" : "+s"(ci));
#pragma unroll
            for (int q = 0; q < (FG ? 1 : kStrGroup); ++q) b.c[k][q] = S.coef[ci + q];
        }
    };
    auto gather = [&](Bat &b, const uint32_t (&x)[K]) {
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const uint32_t o = doff ^ (x[k] << Amp<T>::kShift);
            b.p[k][0] = Amp<T>::raw_at(v0, o);
            if (NV == 2) b.p[k][NV - 1] = Amp<T>::raw_at(v1, o);
        }
    };
    // (a use of scalar-loaded data waits for every outstanding scalar and LDS
    // load, so the Z masks and X masks stand for the magnitudes too)
    auto ready = [&](const Bat &b, const uint32_t (&x)[K]) {
#pragma unroll
        for (int k = 0; k < K; ++k) {
#pragma unroll
            for (int q = 0; q < kStrGroup; ++q) asm volatile("" ::"s"(b.z[k][q]));
            asm volatile("" ::"s"(x[k]));
        }
    };
    auto compute = [&](const Bat &b) {
#pragma unroll
        for (int k = 0; k < K; ++k) {
            double f;
            if constexpr (FG) {
                f = fact_h(b.c[k][0], b.z[k][0], b.z[k][1], b.z[k][2], dz);
            } else {
                const double f0 = signed_cz(b.c[k][0], b.z[k][0], dz) + signed_cz(b.c[k][2], b.z[k][2], dz);
                const double f1 = signed_cz(b.c[k][1], b.z[k][1], dz) + signed_cz(b.c[k][3], b.z[k][3], dz);
                f = f0 + f1;
            }
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                const double2 a = Amp<T>::cvt(b.p[k][v]);
                acc[2 * v] = fma(f, a.x, acc[2 * v]);
                acc[2 * v + 1] = fma(f, a.y, acc[2 * v + 1]);
            }
        }
    };
    // The main part: while every group a pass loads lies below g1 the loads
    // need no bounds select, and they use running table pointers (Z masks and
    // X masks through the scalar cache, magnitudes through an LDS address
    // held in a VGPR) with constant offsets, so a pass costs a few scalar
    // instructions instead of an index computation and a select per group.
    typedef __attribute__((address_space(3))) const double lds_f64;
    auto load_zc_at = [&](Bat &b, const GOCP_AS4 uint32_t *zq, lds_f64 *cq, int off) {
#pragma unroll
        for (int k = 0; k < K; ++k)
#pragma unroll
            for (int q = 0; q < kStrGroup; ++q) b.z[k][q] = zq[kStrGroup * (off + k) + q];
#pragma unroll
        for (int k = 0; k < K; ++k)
#pragma unroll
            for (int q = 0; q < (FG ? 1 : kStrGroup); ++q) b.c[k][q] = cq[kStrGroup * (off + k) + q];
    };
    auto load_x_at = [&](uint32_t (&x)[K], const GOCP_AS4 uint32_t *xq, int off) {
#pragma unroll
        for (int k = 0; k < K; ++k) x[k] = xq[off + k];
    };
    Bat A, B;
    uint32_t xa[K], xb[K];
    load_x(xa, g0);
#pragma unroll
    for (int k = 0; k < K; ++k) asm volatile("" ::"s"(xa[k]));
    gather(A, xa);
    load_zc(A, g0);
    load_x(xb, g0 + K);
    int g = g0;
    if (g + 3 * K <= g1) {
        const GOCP_AS4 uint32_t *zq = zs + kStrGroup * g, *xq = gx + g;
        lds_f64 *cq = (lds_f64 *)(S.coef + kStrGroup * g);
        do {
            ready(A, xb);
            __builtin_amdgcn_sched_barrier(0);
            asm volatile("" : "+s"(zq), "+s"(xq), "+v"(cq));
            gather(B, xb);
            load_zc_at(B, zq, cq, K);
            load_x_at(xa, xq, 2 * K);
            __builtin_amdgcn_sched_barrier(0);
            compute(A);
            __builtin_amdgcn_sched_barrier(0);
            ready(B, xa);
            __builtin_amdgcn_sched_barrier(0);
            asm volatile("" : "+s"(zq), "+s"(xq), "+v"(cq));
            gather(A, xa);
            load_zc_at(A, zq, cq, 2 * K);
            load_x_at(xb, xq, 3 * K);
            __builtin_amdgcn_sched_barrier(0);
            compute(B);
            __builtin_amdgcn_sched_barrier(0);
            zq += kStrGroup * 2 * K;
            xq += 2 * K;
            cq += kStrGroup * 2 * K;
            g += 2 * K;
        } while (g + 3 * K <= g1);
    }
    // The rest (at most two passes), with the bounds selects.  One exit,
    // after both steps: every load issued is consumed on every path (a load
    // used only past a branch would be sunk into it, next to its use).  A
    // step that starts past g1 sums zero magnitudes; the last pass reads ahead
    // into the tables' zero padding and leaves those loads unused.
    // Scheduling barriers keep each step in the order wait, issue, compute.
    for (;; g += 2 * K) {
        ready(A, xb);
        __builtin_amdgcn_sched_barrier(0);
        gather(B, xb);
        load_zc(B, g + K);
        load_x(xa, g + 2 * K);
        __builtin_amdgcn_sched_barrier(0);
        compute(A);
        __builtin_amdgcn_sched_barrier(0);
        ready(B, xa);
        __builtin_amdgcn_sched_barrier(0);
        gather(A, xa);
        load_zc(A, g + 2 * K);
        load_x(xb, g + 3 * K);
        __builtin_amdgcn_sched_barrier(0);
        compute(B);
        __builtin_amdgcn_sched_barrier(0);
        if (g + 2 * K >= g1) break;
    }
}

// The wave's records [c0, c1) of stage chunk k (chunk-relative) from a
// kNW + 1 boundary table per chunk.
__device__ __forceinline__ void wave_range(const int32_t *seg, int k, int cb, int &c0, int &c1) {
    const GOCP_AS4 int32_t *t = cptr(seg) + k * (kNW + 1) + wave_id();
    c0 = t[0] - cb;
    c1 = t[1] - cb;
}

// Apply the X-mask classes of H to NV vectors at the lane's R amplitudes:
// acc[(k R + r) 2 + {0,1}] += sum_classes f_class(d_r) vec_k[d_r ^ x_class].
// The table is staged chunk by chunk; wave w takes classes w, w + kNW, ... of
// a chunk, and the gathers of its next class are issued before the current
// class's strings are summed.
template <typename T, int NV, int R>
__device__ __forceinline__ void apply_classes(const InstDev &I, Stage &S, uint32_t d0, uint32_t dim,
                                              const void *v0, const void *v1, double *acc, int trace_mode = 0) {
    const int wv = wave_id();
    const GOCP_AS4 int4 *hch = cptr(I.hchunk);
    for (int k = 0; k < I.n_hchunks; ++k) {
        const int4 bd = load_rec(hch, k);
        const int cb = bd.x, ce = bd.y, sb = bd.z, se = bd.w;
        __syncthreads();
        // one vector at one amplitude per lane: the grouped walk (no class
        // records); two vectors (H v, H w of complex128 states) keep the class
        // walk, which measured faster there (20.7 against 28.2 us at 14 qubits)
        constexpr bool grouped = R == 1 && NV == 1;
        // the grouped walk stages its own table (factored classes first)
        const int4 gbd = grouped ? load_rec(cptr(I.hchunkG), k) : make_int4(0, 0, 0, 0);
        if (!grouped) stage_copy(S.cls, I.hcls + cb, ce - cb);
        if (R > 1) stage_copy(S.sub, I.hsub + cb, ce - cb);
        if (grouped) stage_coef(S, I.hcoefG, gbd.x, gbd.z);
        else stage_coef(S, I.hcoef, sb, se);
        const GOCP_AS4 uint32_t *zs = cptr(I.hzs) + sb;
        __syncthreads();
        if (k == 0) phase_mark(2, trace_mode);
        if constexpr (grouped) {
            // the wave's run of factored classes, then its run of string groups
            const int gb = gbd.x / kStrGroup;
            const GOCP_AS4 uint32_t *zg = cptr(I.hzsG) + gbd.x, *gx = cptr(I.hgx) + gb;
            const GOCP_AS4 int32_t *t = cptr(I.hgseg) + k * 2 * (kNW + 1) + wv;
            const uint32_t dd = d0 < dim ? d0 : 0u;
            walk_groups_r1<T, NV, kWalkBatch, true>(S, zg, gx, t[0] - gb, t[1] - gb, dd, v0, v1, acc);
            walk_groups_r1<T, NV, kWalkBatch, false>(S, zg, gx, t[kNW + 1] - gb, t[kNW + 2] - gb, dd, v0, v1, acc);
            continue;
        }
        int c0, c1;
        wave_range(I.hseg, k, cb, c0, c1);
        if constexpr (R == 1) {
            walk_classes_r1<T, NV, kFactH>(S, zs, c0, c1, sb, d0 < dim ? d0 : 0u, v0, v1,
                                   [&](int, double f, const typename Amp<T>::Raw (&p)[NV]) {
#pragma unroll
                                       for (int v = 0; v < NV; ++v) {
                                           const double2 a = Amp<T>::cvt(p[v]);
                                           acc[2 * v] = fma(f, a.x, acc[2 * v]);
                                           acc[2 * v + 1] = fma(f, a.y, acc[2 * v + 1]);
                                       }
                                   });
            continue;
        }
        int c = c0;
        uint32_t off[R];
        lane_offsets<R, Amp<T>::kShift>(d0, dim, off);
        // Two FP64 vectors at four amplitudes per lane hold 32 VGPRs of
        // gathers per class: they are issued at the start of their own
        // class (their latency passes under its coefficients) instead of a
        // class ahead, which would double that and spill.
        constexpr bool ahead = !(NV == 2 && R == 4 && sizeof(typename Amp<T>::Raw) == 16);
        if constexpr (!ahead) {
            for (; c < c1; ++c) {
                typename Amp<T>::Raw rc[NV][R];
                const uint32_t xc = (uint32_t)uni((int)S.cls[c].x) << Amp<T>::kShift;
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    rc[0][r] = Amp<T>::raw_at(v0, off[r] ^ xc);
                    rc[NV - 1][r] = Amp<T>::raw_at(v1, off[r] ^ xc);
                }
                double f[R];
                class_coeffs<R, kFactH>(S, zs, c, sb, d0, f);
#pragma unroll
                for (int v = 0; v < NV; ++v)
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        const double2 p = Amp<T>::cvt(rc[v][r]);
                        acc[2 * (v * R + r)] = fma(f[r], p.x, acc[2 * (v * R + r)]);
                        acc[2 * (v * R + r) + 1] = fma(f[r], p.y, acc[2 * (v * R + r) + 1]);
                    }
            }
            continue;
        }
        typename Amp<T>::Raw rn[NV][R];
        if (c < c1) {
            const uint32_t xn = (uint32_t)uni((int)S.cls[c].x) << Amp<T>::kShift;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                rn[0][r] = Amp<T>::raw_at(v0, off[r] ^ xn);
                if (NV == 2) rn[NV - 1][r] = Amp<T>::raw_at(v1, off[r] ^ xn);
            }
        }
        for (; c < c1; ++c) {
            typename Amp<T>::Raw rc[NV][R];
#pragma unroll
            for (int v = 0; v < NV; ++v)
#pragma unroll
                for (int r = 0; r < R; ++r) rc[v][r] = rn[v][r];
            const int cn = c + 1;
            if (cn < c1) {
                const uint32_t xn = (uint32_t)uni((int)S.cls[cn].x) << Amp<T>::kShift;
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    rn[0][r] = Amp<T>::raw_at(v0, off[r] ^ xn);
                    if (NV == 2) rn[NV - 1][r] = Amp<T>::raw_at(v1, off[r] ^ xn);
                }
            }
            double f[R];
            class_coeffs<R, kFactH>(S, zs, c, sb, d0, f);
#pragma unroll
            for (int v = 0; v < NV; ++v)
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const double2 p = Amp<T>::cvt(rc[v][r]);
                    acc[2 * (v * R + r)] = fma(f[r], p.x, acc[2 * (v * R + r)]);
                    acc[2 * (v * R + r) + 1] = fma(f[r], p.y, acc[2 * (v * R + r) + 1]);
                }
        }
    }
    __syncthreads();          // the stage may be reused by the caller
}

__device__ __forceinline__ uint32_t insert_zero_bit(uint32_t p, int hb) {
    const uint32_t lo = p & ((1u << hb) - 1u);
    return ((p >> hb) << (hb + 1)) | lo;
}

// ------------------------------------------------------------------ energy + gradient screen

// One launch per state, per tile of 64 R amplitudes (R per lane):
//   1. sigma = H psi on the tile (FP64), and the tile's <psi|sigma>, <psi|psi>;
//   2. when a screen is due, the tile's share of
//      g_j = 2 Re <sigma | A_j psi> / <psi|psi> for every pool operator, with
//      the tile's own sigma values taken from LDS.  Operators are visited in
//      GOCP family order (the family-ordered table is staged in LDS; each wave
//      takes a contiguous, cost-balanced run of each stage's operators);
// and writes the tile's partials; k_screen_reduce, launched next, forms the
// energy, the norm, the gradients, |g|max, ||g||_2 and the selected operator.
// mode 0: one-shot (energy; gradients when the instance has a pool);
// mode 1: starting state of an ADAPT run (E_0 and the first screen);
// mode 2: state after an update: iteration counter + 1, its energy, and the
//         next screen unless the iteration budget is spent;
// mode 3: the work of mode 0 without writing sigma or the state record (kernel
//         timing in the middle of a run); mode 4: likewise for the work of
//         mode 2 when sigma is carried through the update.
template <typename T, int R, bool XF = false>
__global__ __launch_bounds__(kNW *kWave) void k_energy_screen(const InstDev *__restrict__ insts,
                                                             const int2 *__restrict__ blk, int mode) {
    phase_mark(0, mode);
    const int2 b = work_row(blk);
    const InstDev &I = insts[b.x];
    AdaptState *st = I.st;
    // the descriptor fields and the state record's head are each loaded in
    // one batch ahead of every test that uses them (a chain of one load per
    // field otherwise)
    const int M = I.M, nq = I.n_qubits, nhc = I.n_hchunks;
    const double2 *hvp = I.hv;
    const GOCP_AS4 int4 *hch = cptr(I.hchunk);
    asm volatile("" ::"s"(st), "s"(M), "s"(nq), "s"(nhc), "s"(hvp), "s"(hch));
    const StHead h = load_head(st);
    const int4 bd0 = load_rec(hch, 0);
    asm volatile("" ::"s"(h.done), "s"(h.iter), "s"(h.max_iter), "s"(bd0.x), "s"(bd0.y), "s"(bd0.z), "s"(bd0.w));
    const bool oneshot = mode == 0 || mode >= 3, dry = mode >= 3;
    if (!oneshot && h.done) return;
    const int it = mode == 2 ? h.iter + 1 : 0;
    const bool screen = M > 0 && (oneshot || it < h.max_iter);
    const int lane = threadIdx.x & (kWave - 1);
    const int wv = wave_id();
    const uint32_t dim = 1u << nq;
    const uint32_t d0 = (uint32_t)b.y * (kTile * R) + lane;

    __shared__ Stage S;
    __shared__ double2 s_sig[R][kWave];
    __shared__ double opbuf[kNW][4][kWave];   // per wave: lane contributions of up to four operators
    static_assert(!XF || R == 1, "the X-class screen runs at one amplitude per lane");
    __shared__ int32_t s_xop[XF ? kStageTerms : 1];   // X-class screen: the strings' pool indices
    // XF: every member's pool is single strings with an X-class screen (one
    // gather per X mask serves all the operators of that mask)
    constexpr bool xform = XF;

    // Stage chunk k of the screen's tables (operator records, sub-buckets
    // for R > 1, magnitudes) into S; the caller orders it with barriers.
    const GOCP_AS4 int4 *pch = cptr(xform ? I.xchunk : I.pchunk);
    auto stage_screen = [&](int k) {
        const int4 bd = load_rec(pch, k);
        if constexpr (xform) {
            stage_copy(S.cls, I.xrec + bd.x, bd.y - bd.x);
            stage_coef(S, I.xcoef, bd.z, bd.w);
            stage_copy(reinterpret_cast<u32x4 *>(s_xop), reinterpret_cast<const u32x4 *>(I.xop + bd.z),
                       (bd.w - bd.z) / kStrGroup);
            return;
        }
        stage_copy(S.cls, I.sop + bd.x, bd.y - bd.x);
        if (R > 1) stage_copy(S.sub, I.psub + bd.x, bd.y - bd.x);
        stage_coef(S, I.scoef, bd.z, bd.w);
    };
    // 1. sigma on the tile: H psi, or, after an update, sigma carried through
    //    it (the update is I + al A + be A^2 on scale * psi, so
    //    H psi' = scale (sigma + al H w - be H v) with the line search's H v,
    //    H w).  Every Refresh<T>::kPeriod iterations H psi is applied afresh,
    //    which bounds the drift from the rounding of the stored state.
    const bool carry = I.hv != nullptr && (mode == 4 || (mode == 2 && (it % Refresh<T>::kPeriod) != 0));
    if ((mode == 1 || mode == 2) && b.y == 0 && threadIdx.x == 0) {
        GOCP_AS1 AdaptState *gs = gmut(st);
        gs->pend_it = it;
        gs->pend_mode = mode;
    }
    double pe = 0.0, pn = 0.0;
    if (!carry) {
        double acc[2 * R];
#pragma unroll
        for (int i = 0; i < 2 * R; ++i) acc[i] = 0.0;
        phase_mark(1, mode);
        apply_classes<T, 1, R>(I, S, d0, dim, I.psi, nullptr, acc, mode);
        phase_mark_last(3, mode);
        // the cross-wave sums go through the operator buffers, so the screen's
        // first stage chunk is staged meanwhile
        double2 (*red)[kWave] = reinterpret_cast<double2 (*)[kWave]>(&opbuf[0][0][0]);
        if (screen) stage_screen(0);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            red[wv][lane] = make_double2(acc[2 * r], acc[2 * r + 1]);
            __syncthreads();
            if (wv == 0) {
                double ar = 0.0, ai = 0.0;
#pragma unroll
                for (int k = 0; k < kNW; ++k) {
                    ar += red[k][lane].x;
                    ai += red[k][lane].y;
                }
                const uint32_t d = d0 | ((uint32_t)r << 6);
                const bool valid = d < dim;
                const double2 own = valid ? Amp<T>::load(I.psi, d) : make_double2(0.0, 0.0);
                if (valid) {
                    pe += own.x * ar + own.y * ai;
                    pn += own.x * own.x + own.y * own.y;
                    if (!dry) gstore2(I.sigma, d, make_double2(ar, ai));
                }
                s_sig[r][lane] = valid ? make_double2(ar, ai) : make_double2(0.0, 0.0);
            }
            __syncthreads();
        }
    } else {
        if (screen) stage_screen(0);
        if (wv == 0) {
            const double al = cptr(&st->upd_alpha)[0], be = cptr(&st->upd_beta)[0];
            const double sc = cptr(&st->upd_scale)[0];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const uint32_t d = d0 | ((uint32_t)r << 6);
                double2 sg = make_double2(0.0, 0.0);
                if (d < dim) {
                    const double2 s0 = gload2(I.sigma, d), hv = gload2(I.hv, d), hw = gload2(I.hw, d);
                    sg.x = sc * (s0.x + al * hw.x - be * hv.x);
                    sg.y = sc * (s0.y + al * hw.y - be * hv.y);
                    const double2 own = Amp<T>::load(I.psi, d);
                    pe += own.x * sg.x + own.y * sg.y;
                    pn += own.x * own.x + own.y * own.y;
                    if (!dry) gstore2(I.sigma, d, sg);
                }
                s_sig[r][lane] = sg;
            }
        }
        __syncthreads();
    }
    if (wv == 0) {
        pe = wave_sum(pe);
        pn = wave_sum(pn);
        if (lane == 0) {
            gmut(I.part_e)[b.y] = pe;
            gmut(I.part_n)[b.y] = pn;
        }
    }

    phase_mark(4, mode);
    // 2. gradient screen on the tile
    if (screen) {
        double2 sg[R];
#pragma unroll
        for (int r = 0; r < R; ++r) sg[r] = s_sig[r][lane];
        const uint32_t *szs = xform ? I.xzs : I.szs;
        const int32_t *pseg = xform ? I.xseg : I.pseg;
        const int npc = xform ? I.n_xchunks : I.n_pchunks;
        for (int k = 0; k < npc; ++k) {
            const int4 bd = load_rec(pch, k);
            const int ob = bd.x, sb = bd.z;
            // chunk 0 was staged with the sigma sums (the barrier after them
            // ordered it); later chunks after the previous one's walk
            if (k > 0) {
                __syncthreads();
                stage_screen(k);
                __syncthreads();
            }
            const GOCP_AS4 uint32_t *zs = cptr(szs) + sb;
            int o0, o1;
            wave_range(pseg, k, ob, o0, o1);
            // Per-operator sums over the wave's 64 amplitudes, four operators
            // at a time: every lane stores its contribution to the wave's
            // buffer; after every fourth operator of the wave's run (and after
            // its last) row r of the wave adds the buffer's operator r (four
            // contributions per lane, then a 16-lane row sum) -- one row
            // reduction per four operators instead of one wave reduction each.
            // The buffer is private to the wave, whose LDS accesses complete
            // in order.
            int nbuf = 0, obase = 0;
            auto flush = [&]() {
                const int r = lane >> 4, q = (lane & 15) * 4;
                const double t4 = (opbuf[wv][r][q] + opbuf[wv][r][q + 1]) + (opbuf[wv][r][q + 2] + opbuf[wv][r][q + 3]);
                const double t = row_sum(r < nbuf ? t4 : 0.0);
                // the operator's partial goes straight to its pool index
                if ((lane & 15) == 0 && r < nbuf)
                    gmut(I.part_g)[(size_t)b.y * M + (xform ? s_xop[obase + r] : S.cls[obase + r].pad)] = t;
                nbuf = 0;
            };
            auto push = [&](int o, double v) {
                if (nbuf == 0) obase = o;
                opbuf[wv][nbuf][lane] = v;
                if (++nbuf == 4) flush();
            };
            if constexpr (xform) {
                // X-class records: one gather per record serves its member
                // strings, each an operator pushed under its string index
                // (a wave's strings are consecutive, so four pushes in a row
                // are the strings obase .. obase + 3)
                const uint32_t dd = d0 < dim ? d0 : 0u, dz = with_sign_bit(dd);
                uint32_t doff = dd << Amp<T>::kShift;
                asm volatile("" : "+v"(doff));
                typename Amp<T>::Raw pn{};
                if (o0 < o1) pn = Amp<T>::raw_at(I.psi, doff ^ ((uint32_t)uni((int)S.cls[o0].x) << Amp<T>::kShift));
                for (int o = o0; o < o1; ++o) {
                    const int s0 = uni(S.cls[o].s0) - sb, s1 = uni(S.cls[o].s1) - sb;
                    const typename Amp<T>::Raw pc = pn;
                    if (o + 1 < o1)
                        pn = Amp<T>::raw_at(I.psi, doff ^ ((uint32_t)uni((int)S.cls[o + 1].x) << Amp<T>::kShift));
                    const double2 a = Amp<T>::cvt(pc);
                    const double q = sg[0].x * a.x + sg[0].y * a.y;
                    // members eight at a time, their masks in one batch of
                    // scalar loads (reads past s1 stay in the stage and in the
                    // table's padding, and are not used); a full batch of
                    // eight is summed over the wave in registers (fold8) and
                    // stored by one lane per operator, a shorter one goes
                    // through the buffer (emptied first, so that it holds
                    // consecutive strings)
                    for (int t = s0; t < s1; t += 8) {
                        uint32_t z[8];
                        double c[8];
#pragma unroll
                        for (int u = 0; u < 8; ++u) {
                            z[u] = zs[t + u];
                            c[u] = S.coef[t + u];
                        }
                        if (t + 8 <= s1) {
                            if (nbuf > 0) flush();
                            double v[8];
#pragma unroll
                            for (int u = 0; u < 8; ++u) v[u] = q * signed_cz(c[u], z[u], dz);
                            const double r = fold8(v);
                            if ((lane & 7) == 0)
                                gmut(I.part_g)[(size_t)b.y * M + s_xop[t + (lane >> 3)]] = r;
                        } else {
#pragma unroll
                            for (int u = 0; u < 8; ++u)
                                if (t + u < s1) push(t + u, q * signed_cz(c[u], z[u], dz));
                        }
                    }
                }
            } else if constexpr (R == 1) {
                walk_classes_r1<T, 1, kFactPool>(S, zs, o0, o1, sb, d0 < dim ? d0 : 0u, I.psi, nullptr,
                                      [&](int o, double h, const typename Amp<T>::Raw (&p)[1]) {
                                          const double2 a = Amp<T>::cvt(p[0]);
                                          push(o, h * (sg[0].x * a.x + sg[0].y * a.y));
                                      });
            } else {
            int o = o0;
            uint32_t off[R];
            lane_offsets<R, Amp<T>::kShift>(d0, dim, off);
            typename Amp<T>::Raw rn[R];
            if (o < o1) {
                const uint32_t xn = (uint32_t)uni((int)S.cls[o].x) << Amp<T>::kShift;
#pragma unroll
                for (int r = 0; r < R; ++r) rn[r] = Amp<T>::raw_at(I.psi, off[r] ^ xn);
            }
            for (; o < o1; ++o) {
                typename Amp<T>::Raw rc[R];
#pragma unroll
                for (int r = 0; r < R; ++r) rc[r] = rn[r];
                const int on = o + 1;
                if (on < o1) {
                    const uint32_t xn = (uint32_t)uni((int)S.cls[on].x) << Amp<T>::kShift;
#pragma unroll
                    for (int r = 0; r < R; ++r) rn[r] = Amp<T>::raw_at(I.psi, off[r] ^ xn);
                }
                double h[R];
                class_coeffs<R, kFactPool>(S, zs, o, sb, d0, h);
                double val = 0.0;
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const double2 p = Amp<T>::cvt(rc[r]);
                    val += h[r] * (sg[r].x * p.x + sg[r].y * p.y);
                }
                push(o, val);
            }
            }
            if (nbuf > 0) flush();
        }
    }
    phase_mark_last(5, mode);
}

// The screen's partials are summed in two launches that follow
// k_energy_screen on the same stream (each kernel boundary orders the stores
// of one launch before the loads of the next); every sum runs in a fixed
// order, so results do not depend on scheduling.
//
// First stage: workgroup (i, g) adds tiles g kGroup, ..., (g + 1) kGroup - 1
// of instance i in tile order: the energy and norm partials, and every
// operator's partial (thread = operator, all kGroup loads in flight).  The
// grid's second dimension splits the operators into blocks of kPairBlock
// columns (pools with many operators); block 0 also adds energy and norm.
__global__ __launch_bounds__(kPairBlock) void k_screen_sum1(const InstDev *__restrict__ insts,
                                                           const int2 *__restrict__ blk, int mode) {
    const int2 b = work_row(blk);
    const InstDev &I = insts[b.x];
    // The descriptor fields are loaded in one batch; then the state record's
    // head and the group's partials are loaded together: the sums are formed
    // whatever the state says and stored only when it asks for them, so no
    // load waits on the state's test (nor is moved behind it).
    const AdaptState *st = I.st;
    const int M = I.M, n_tiles = I.n_tiles;
    const double *pe = I.part_e, *pn = I.part_n, *pg = I.part_g;
    double *pe2 = I.part_e2, *pn2 = I.part_n2, *pg2 = I.part_g2;
    asm volatile("" ::"s"(st), "s"(M), "s"(n_tiles), "s"(pe), "s"(pn), "s"(pg), "s"(pe2), "s"(pn2), "s"(pg2));
    const StHead h = load_head(st);
    // the group's kGroup loads go out together (indices clamped into the
    // group, surplus values masked), then are added in tile order
    const int t0 = b.y * kGroup, nt = min(kGroup, n_tiles - t0);
    auto group_sum = [&](const GOCP_AS1 double *src, size_t stride) {
        double x[kGroup];
#pragma unroll
        for (int t = 0; t < kGroup; ++t) x[t] = src[(size_t)min(t, nt - 1) * stride];
        double a = 0.0;
#pragma unroll
        for (int t = 0; t < kGroup; ++t) a += t < nt ? x[t] : 0.0;
        return a;
    };
    const bool en = blockIdx.y == 0;              // this block also adds energy and norm
    const int j0 = blockIdx.y * kPairBlock + threadIdx.x;
    // the energy or norm column (threads 0 and 1) and the thread's operator
    // column go out in one batch (every thread loads both, from clamped
    // indices; M = 0 leaves one allocated column)
    const GOCP_AS1 double *se = gptr(j0 == 0 ? pe : pn) + t0;
    const GOCP_AS1 double *sg = gptr(pg) + (size_t)t0 * M + (j0 < M ? j0 : 0);
    double xe[kGroup], xg[kGroup];
#pragma unroll
    for (int t = 0; t < kGroup; ++t) {
        xe[t] = se[min(t, nt - 1)];
        xg[t] = sg[(size_t)min(t, nt - 1) * M];
    }
    double ae = 0.0, ag = 0.0;
#pragma unroll
    for (int t = 0; t < kGroup; ++t) {
        ae += t < nt ? xe[t] : 0.0;
        ag += t < nt ? xg[t] : 0.0;
    }
    const bool oneshot = mode == 0 || mode >= 3;
    const bool live = oneshot || !h.done;
    const int it = mode == 2 ? h.iter + 1 : 0;
    const bool screen = live && M > 0 && (oneshot || it < h.max_iter);
    if (en && live && j0 < 2) (j0 == 0 ? pe2 : pn2)[b.y] = ae;
    if (!screen) return;
    if (j0 < M) pg2[(size_t)b.y * M + j0] = ag;
    for (int j = j0 + (int)gridDim.y * kPairBlock; j < M; j += (int)gridDim.y * kPairBlock)
        pg2[(size_t)b.y * M + j] = group_sum(gptr(pg) + (size_t)t0 * M + j, (size_t)M);
}

// The first kGroup group sums of the energy, the norm and the thread's first
// operator column (indices clamped into range; surplus values are masked
// where they are added).  A kernel issues these loads as early as it can,
// ahead of the state record's test, and select_state adds them.
struct SelPre {
    double xe[kGroup], xn[kGroup], xg[kGroup];
    u32x4 rec;                  // the pool record (pool order) of the thread's first operator
};
__device__ __forceinline__ void sel_load(const InstDev &I, SelPre &p) {
    const int M = I.M, ng = I.n_groups;
    const GOCP_AS1 double *pe2 = gptr(I.part_e2), *pn2 = gptr(I.part_n2), *pg2 = gptr(I.part_g2);
    const int jt = (int)threadIdx.x < M ? (int)threadIdx.x : 0;   // M = 0: one allocated column
    p.rec = ((const GOCP_AS1 u32x4 *)(uintptr_t)I.pop)[jt];
#pragma unroll
    for (int u = 0; u < kGroup; ++u) {
        const int t = min(u, ng - 1);
        p.xe[u] = pe2[t];
        p.xn[u] = pn2[t];
        p.xg[u] = pg2[(size_t)t * M + jt];
    }
}

// Second stage: energy, norm and gradients of an instance from the group sums,
// then the operator selection and whether the run ends (modes as
// k_energy_screen).  Every workgroup that calls it computes the same values in
// the same order: thread k adds operator columns k, k + NT, ... over the groups
// in group order, per-thread results meet by wave sums in wave order, and the
// tie band is searched in a second pass over the same sums.  `writer`
// workgroups also write the record.  pre holds the first batch of the group
// sums (sel_load); max_iter is the state record's.  Returns the selected
// operator and whether the run is over, in every thread; with rec_out (LDS),
// the thread that owns a selected operator below NT also leaves its pool
// record there (visible after the return).  Wide (pools of more than NT
// operators) sums a thread's later operator columns kCols at a time, with
// their loads in flight together, and keeps all the sums it will test again
// in registers; the same sums in the same order, so the same results.
template <int NT, bool Wide = false>
__device__ void select_state(const InstDev &I, AdaptState *st, int mode, int it, int max_iter, bool writer,
                             const SelPre &pre, int &jsel, bool &done, HClass *rec_out = nullptr) {
    __shared__ double red[2][NT / kWave];
    __shared__ int redi[NT / kWave];
    const int lane = threadIdx.x & (kWave - 1);
    const int wv = threadIdx.x >> 6;
    const bool oneshot = mode == 0 || mode >= 3, dry = mode >= 3;
    const int M = I.M, ng = I.n_groups;
    const bool screen = M > 0 && (oneshot || it < max_iter);
    // sums over the groups in group order; loads go out kGroup at a time
    // (indices clamped into range, surplus values masked), so a sum waits
    // once per kGroup groups instead of once per group; the first batch is
    // the preloaded one
    const GOCP_AS1 double *pe2 = gptr(I.part_e2), *pn2 = gptr(I.part_n2), *pg2 = gptr(I.part_g2);
    double e_num = 0.0, nrm = 0.0;
#pragma unroll
    for (int u = 0; u < kGroup; ++u)
        if (u < ng) {
            e_num += pre.xe[u];
            nrm += pre.xn[u];
        }
    for (int t0 = kGroup; t0 < ng; t0 += kGroup) {
        double xe[kGroup], xn[kGroup];
#pragma unroll
        for (int u = 0; u < kGroup; ++u) {
            const int t = min(t0 + u, ng - 1);
            xe[u] = pe2[t];
            xn[u] = pn2[t];
        }
#pragma unroll
        for (int u = 0; u < kGroup; ++u)
            if (t0 + u < ng) {
                e_num += xe[u];
                nrm += xn[u];
            }
    }
    const double inv = 2.0 / nrm;
    auto grad = [&](int j) {
        double a = 0.0;
        int t0 = 0;
        if (j == (int)threadIdx.x) {
#pragma unroll
            for (int u = 0; u < kGroup; ++u)
                if (u < ng) a += pre.xg[u];
            t0 = kGroup;
        }
        for (; t0 < ng; t0 += kGroup) {
            double x[kGroup];
#pragma unroll
            for (int u = 0; u < kGroup; ++u) x[u] = pg2[(size_t)min(t0 + u, ng - 1) * M + j];
#pragma unroll
            for (int u = 0; u < kGroup; ++u)
                if (t0 + u < ng) a += x[u];
        }
        return a * inv;
    };
    // the sums of kCols columns (jb, jb + NT, ...; indices clamped into
    // range, surplus values unused) with all their loads in flight together,
    // each added over the groups in group order as in grad
    constexpr int kCols = 2;
    auto cols = [&](int jb, double (&a)[kCols]) {
        int jc[kCols];
#pragma unroll
        for (int c = 0; c < kCols; ++c) {
            jc[c] = min(jb + c * NT, M - 1);
            a[c] = 0.0;
        }
        for (int t0 = 0; t0 < ng; t0 += kGroup) {
            double x[kCols][kGroup];
#pragma unroll
            for (int c = 0; c < kCols; ++c)
#pragma unroll
                for (int u = 0; u < kGroup; ++u) x[c][u] = pg2[(size_t)min(t0 + u, ng - 1) * M + jc[c]];
#pragma unroll
            for (int c = 0; c < kCols; ++c)
#pragma unroll
                for (int u = 0; u < kGroup; ++u)
                    if (t0 + u < ng) a[c] += x[c][u];
        }
#pragma unroll
        for (int c = 0; c < kCols; ++c) a[c] *= inv;
    };
    double gmax = 0.0, gn = 0.0;
    int jmin = 0x7fffffff;
    if (screen) {
        // a thread's first kCache gradients are kept for the tie-band pass
        // (Wide: its own column, then kBat batches of kCols columns)
        constexpr int kBat = 3, kCache = Wide ? 1 + kBat * kCols : 4;
        const int j0 = threadIdx.x;
        double gc[kCache];
        double amax = 0.0, sq = 0.0;
        GOCP_AS1 double *gout = gmut(cptr(&st->g)[0]);
        auto take = [&](int j, double g) {
            if (writer && !dry) gout[j] = g;
            amax = fmax(amax, fabs(g));
            sq += g * g;
        };
        if constexpr (Wide) {
            gc[0] = j0 < M ? grad(j0) : 0.0;
            if (j0 < M) take(j0, gc[0]);
#pragma unroll
            for (int bt = 0; bt < kBat; ++bt) {
                const int c0 = 1 + bt * kCols;
                double a[kCols];
                if (c0 * NT < M) {
                    cols(j0 + c0 * NT, a);
                } else {
#pragma unroll
                    for (int c = 0; c < kCols; ++c) a[c] = 0.0;
                }
#pragma unroll
                for (int c = 0; c < kCols; ++c) {
                    gc[c0 + c] = a[c];
                    if (j0 + (c0 + c) * NT < M) take(j0 + (c0 + c) * NT, a[c]);
                }
            }
            for (int j = j0 + kCache * NT; j < M; j += NT) take(j, grad(j));
        } else {
            for (int j = j0, i = 0; j < M; j += NT, ++i) {
                const double g = grad(j);
                if (i < kCache) gc[i] = g;
                take(j, g);
            }
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) amax = fmax(amax, __shfl_xor(amax, off, kWave));
        sq = wave_sum(sq);
        if (lane == 0) {
            red[0][wv] = amax;
            red[1][wv] = sq;
        }
        __syncthreads();
        for (int w = 0; w < NT / kWave; ++w) {
            gmax = fmax(gmax, red[0][w]);
            gn += red[1][w];
        }
        gn = sqrt(gn);
        // lowest index within the tie band of the largest magnitude
        const double thresh = gmax * (1.0 - 1e-12);
        int jm = 0x7fffffff;
        if constexpr (Wide) {
#pragma unroll
            for (int c = kCache - 1; c >= 0; --c)     // the lowest cached match wins
                if (j0 + c * NT < M && fabs(gc[c]) >= thresh) jm = j0 + c * NT;
            if (jm == 0x7fffffff)
                for (int j = j0 + kCache * NT; j < M; j += NT)
                    if (fabs(grad(j)) >= thresh) {
                        jm = j;
                        break;
                    }
        } else {
            for (int j = j0, i = 0; j < M; j += NT, ++i)
                if (fabs(i < kCache ? gc[i] : grad(j)) >= thresh) {
                    jm = j;
                    break;
                }
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) jm = min(jm, __shfl_xor(jm, off, kWave));
        if (lane == 0) redi[wv] = jm;
        __syncthreads();
        for (int w = 0; w < NT / kWave; ++w) jmin = min(jmin, redi[w]);
        if (rec_out && (int)threadIdx.x == (jmin < M ? jmin : 0))
            *rec_out = HClass{pre.rec.x, (int32_t)pre.rec.y, (int32_t)pre.rec.z, (int32_t)pre.rec.w};
        __syncthreads();
    }
    const double e = e_num / nrm;
    bool bad = !(nrm > 0.0) || !isfinite(e) || (screen && !isfinite(gn));
    bool end = bad;
    if (mode == 1 && max_iter <= 0) end = true;
    if (mode == 2 && it >= max_iter) end = true;
    const bool conv = screen && mode != 0 && !oneshot && gn < cptr(&st->grad_tol)[0];
    if (conv) end = true;
    jsel = jmin < M ? jmin : 0;
    done = end;
    if (!writer || dry || threadIdx.x != 0) return;
    // the record is written through global (not flat) stores; its history
    // pointers are never written by a kernel
    GOCP_AS1 AdaptState *gs = gmut(st);
    double *hist_e = cptr(&st->hist_e)[0], *hist_gn = cptr(&st->hist_gnorm)[0], *hist_gm = cptr(&st->hist_gmax)[0];
    gs->e_num = e_num;
    gs->nrm = nrm;
    gs->energy = e;
    if (mode == 1) {
        if (hist_e) gmut(hist_e)[0] = e;
    } else if (mode == 2) {
        gs->iter = it;
        if (hist_e) gmut(hist_e)[it] = e;
    }
    if (screen) {
        gs->gmax = gmax;
        gs->gnorm = gn;
        gs->jsel = jsel;
        if (mode != 0) {
            if (hist_gn) gmut(hist_gn)[it] = gn;
            if (hist_gm) gmut(hist_gm)[it] = gmax;
        }
    }
    if (conv) gs->converged = 1;
    if (bad) gs->status = GOCP_ENUMERIC;
    if (end && mode != 0) gs->done = 1;
    if (bad) gs->done = 1;
}

// Standalone selection, one workgroup per instance: modes as k_energy_screen,
// or kModePending to select the partials the last k_energy_screen of an ADAPT
// run left (their iteration and mode recorded by it; selecting the same
// partials again writes the same record).
template <bool Wide>
__global__ __launch_bounds__(kPairBlock) void k_screen_reduce(const InstDev *__restrict__ insts,
                                                             const int2 *__restrict__ blk, int mode) {
    const InstDev &I = insts[work_row(blk).x];
    AdaptState *st = I.st;
    SelPre pre;
    sel_load(I, pre);
    const int max_iter = cptr(&st->max_iter)[0];
    int it = 0;
    if (mode == kModePending) {
        if (state_done(st)) return;
        it = cptr(&st->pend_it)[0];
    }
    int j;
    bool done;
    const bool pending = mode == kModePending;
    if (pending) {
        const int m = cptr(&st->pend_mode)[0];
        select_state<kPairBlock, Wide>(I, st, m, it, max_iter, true, pre, j, done);
        if (threadIdx.x == 0) {
            st->sel_it = it;
            st->sel_mode = m;
        }
    } else {
        select_state<kPairBlock, Wide>(I, st, mode, it, max_iter, true, pre, j, done);
    }
}

// ------------------------------------------------------------------ line search vectors

// Selection of the generator (see select_state; Wide for pools of more than
// kPairBlock operators), then w = A psi and v = -A w on its pairs and the
// partial dot products Re<v|sigma>, Re<sigma|w>.
template <typename T, bool Wide>
__global__ __launch_bounds__(kPairBlock) void k_line_vw(const InstDev *__restrict__ insts,
                                                       const int2 *__restrict__ blk) {
    const int2 b = work_row(blk);
    const InstDev &I = insts[b.x];
    // the descriptor fields used by the selection and the pair work, then the
    // state record's head, are each loaded in one batch ahead of their uses
    // (a chain of one load per field otherwise)
    AdaptState *st = I.st;
    {
        const int M = I.M, ng = I.n_groups, nq = I.n_qubits;
        const double *pe2 = I.part_e2, *pn2 = I.part_n2, *pg2 = I.part_g2;
        const HClass *pop = I.pop;
        const HTerm *pterm = I.pterm;
        const void *psi = I.psi;
        const double2 *sigma = I.sigma;
        asm volatile("" ::"s"(st), "s"(M), "s"(ng), "s"(nq), "s"(pe2), "s"(pn2), "s"(pg2), "s"(pop), "s"(pterm),
                     "s"(psi), "s"(sigma));
    }
    const StHead h = load_head(st);
    // the selection's first group sums go out with the head (vector loads:
    // the head's test does not wait for them)
    SelPre pre;
    sel_load(I, pre);
    asm volatile("" ::"s"(h.done), "s"(h.pend_it), "s"(h.pend_mode), "s"(h.sel_it), "s"(h.sel_mode), "s"(h.jsel),
                 "s"(h.max_iter));
    if (h.done) return;
    // selection of the partials the last k_energy_screen left, done by every
    // workgroup (the same sums in the same order) and recorded by pair block 0,
    // unless a standalone selection already recorded it
    // (the selecting thread hands the operator's pool record over in LDS, so
    // it is not loaded after the selection)
    __shared__ HClass s_rec;
    int j;
    bool have = false;
    if (h.sel_it == h.pend_it && h.sel_mode == h.pend_mode) {
        j = h.jsel;
    } else {
        bool over;
        select_state<kPairBlock, Wide>(I, st, h.pend_mode, h.pend_it, h.max_iter, b.y == 0, pre, j, over, &s_rec);
        if (over) return;
        have = j < kPairBlock && j < I.M;
    }
    HClass C;
    if (have) {
        C.x = (uint32_t)uni((int)s_rec.x);
        C.s0 = uni(s_rec.s0);
        C.s1 = uni(s_rec.s1);
        C.pad = 0;
    } else {
        C = load_rec(cptr(I.pop), j);
    }
    const uint32_t m = C.x;
    const int hb = 31 - __clz(m);
    const uint32_t half = 1u << (I.n_qubits - 1);
    const uint32_t p = (uint32_t)b.y * kPairBlock + threadIdx.x;
    double p2 = 0.0, p7 = 0.0;
    bool fd = false, fe = false;
    uint32_t ad = 0, ae = 0;
    if (p < half) {
        const uint32_t d = insert_zero_bit(p, hb), e = d ^ m;
        const double2 a = Amp<T>::load(I.psi, d), c = Amp<T>::load(I.psi, e);
        const double2 sd = I.sigma[d], se = I.sigma[e];
        double hd, he;
        string_sum2(cptr(I.pterm), C.s0, C.s1, d, e, hd, he);
        const double2 wd = make_double2(hd * c.x, hd * c.y);
        const double2 we = make_double2(he * a.x, he * a.y);
        const double hh = -hd * he;
        const double2 vd = make_double2(hh * a.x, hh * a.y);
        const double2 ve = make_double2(hh * c.x, hh * c.y);
        Amp<T>::store(I.w, d, wd);
        Amp<T>::store(I.w, e, we);
        Amp<T>::store(I.v, d, vd);
        Amp<T>::store(I.v, e, ve);
        p2 = vd.x * sd.x + vd.y * sd.y + ve.x * se.x + ve.y * se.y;
        p7 = sd.x * wd.x + sd.y * wd.y + se.x * we.x + se.y * we.y;
        // the amplitudes where the stored v or w is nonzero
        const double2 rvd = Amp<T>::rounded(vd), rwd = Amp<T>::rounded(wd);
        const double2 rve = Amp<T>::rounded(ve), rwe = Amp<T>::rounded(we);
        fd = rvd.x != 0.0 || rvd.y != 0.0 || rwd.x != 0.0 || rwd.y != 0.0;
        fe = rve.x != 0.0 || rve.y != 0.0 || rwe.x != 0.0 || rwe.y != 0.0;
        ad = d;
        ae = e;
    }
    __shared__ double r2[kPairBlock / kWave], r7[kPairBlock / kWave];
    const int wv = wave_id(), lane = threadIdx.x & (kWave - 1);
    if (I.act) {
        // compaction for the H v, H w launch: this block's active amplitudes
        // in a fixed order (wave by wave; within a wave the first members of
        // the pairs in lane order, then the second members)
        __shared__ int wcnt[kPairBlock / kWave];
        const unsigned long long bd = __ballot(fd), be = __ballot(fe);
        const unsigned long long lt = (1ull << lane) - 1ull;
        const int nd = __popcll(bd), ne = __popcll(be);
        if (lane == 0) wcnt[wv] = nd + ne;
        __syncthreads();
        int base = 0, tot = 0;
        for (int k = 0; k < kPairBlock / kWave; ++k) {
            base += k < wv ? wcnt[k] : 0;
            tot += wcnt[k];
        }
        uint32_t *out = I.act + (size_t)b.y * 2 * kPairBlock;
        if (fd) out[base + __popcll(bd & lt)] = ad;
        if (fe) out[base + nd + __popcll(be & lt)] = ae;
        if (threadIdx.x == 0) I.act_n[b.y] = tot;
    }
    p2 = wave_sum(p2);
    p7 = wave_sum(p7);
    if (lane == 0) {
        r2[wv] = p2;
        r7[wv] = p7;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a2 = 0.0, a7 = 0.0;
        for (int k = 0; k < kPairBlock / kWave; ++k) {
            a2 += r2[k];
            a7 += r7[k];
        }
        I.part_l[2 * b.y] = a2;
        I.part_l[2 * b.y + 1] = a7;
    }
}

// E(theta) = a_uu + 2 a_uv cos + 2 a_uw sin + a_vv cos^2 + 2 a_vw sin cos + a_ww sin^2
struct Landscape {
    double uu, uv, uw, vv, vw, ww;
    __device__ double value(double th) const {
        double s, c;
        sincos(th, &s, &c);
        return value_sc(s, c);
    }
    __device__ double value_sc(double s, double c) const {
        return uu + 2.0 * uv * c + 2.0 * uw * s + vv * c * c + 2.0 * vw * s * c + ww * s * s;
    }
    __device__ double deriv_sc(double s, double c) const {
        return -2.0 * uv * s + 2.0 * uw * c - 2.0 * vv * s * c + 2.0 * vw * (c * c - s * s) +
               2.0 * ww * s * c;
    }
    // the sum of the moduli of E''s terms: E' evaluated in double precision is
    // exact to within a few units of rounding of this
    __device__ double deriv_abs_sc(double s, double c) const {
        return 2.0 * (fabs(uv * s) + fabs(uw * c) + fabs(vv * s * c) + fabs(vw * (c * c - s * s)) +
                      fabs(ww * s * c));
    }
    __device__ double deriv(double th) const {
        double s, c;
        sincos(th, &s, &c);
        return deriv_sc(s, c);
    }
    __device__ double deriv2_sc(double s, double c) const {
        return -2.0 * uv * c - 2.0 * uw * s + 2.0 * (ww - vv) * (c * c - s * s) - 8.0 * vw * s * c;
    }
};

// First local minimum of E from 0 in the descent direction -sign(g), found by
// one wave: 1-degree steps (64 at a time) until d E' >= 0, then inside that
// one-degree bracket Newton steps on E' (E'' analytic) from the secant point
// of the bracket's ends, each kept inside the bracket (a step that would
// leave it goes to the bracket's midpoint instead) until the step no longer
// moves the point or E' there is zero to within its own rounding.  Without a sign change within a full turn, the best
// sampled angle.  Called by all 64 lanes of one wave; returns the angle in
// every lane.
__device__ double line_search_wave(const Landscape &L, double g, double &s_out, double &c_out) {
    s_out = 0.0;
    c_out = 1.0;
    if (g == 0.0) return 0.0;
    const int lane = threadIdx.x & (kWave - 1);
    const double dir = g > 0.0 ? -1.0 : 1.0;
    const double step = M_PI / 180.0;
    int kfirst = 0;
    double s_hi = 0.0, c_hi = 1.0, e_hi = 0.0;
    for (int base = 0; base < 360 && kfirst == 0; base += kWave) {
        const int k = base + lane + 1;
        double sk, ck;
        sincos(dir * k * step, &sk, &ck);
        const double ek = L.deriv_sc(sk, ck);
        const bool hit = k <= 360 && dir * ek >= 0.0;
        const unsigned long long mask = __ballot(hit);
        if (mask) {
            const int l = __ffsll((long long)mask) - 1;
            kfirst = base + l + 1;
            s_hi = read_lane(sk, l);
            c_hi = read_lane(ck, l);
            e_hi = read_lane(ek, l);
        }
    }
    if (kfirst == 0) {
        // no sign change: argmin over the 360 sampled angles (first on ties)
        double best = 0.0;
        int bestk = 0;
        for (int base = 0; base < 360; base += kWave) {
            const int k = base + lane + 1;
            double v = k <= 360 ? L.value(dir * k * step) : INFINITY;
            int kk = k;
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) {
                const double ov = __shfl_xor(v, off, kWave);
                const int ok = __shfl_xor(kk, off, kWave);
                if (ov < v || (ov == v && ok < kk)) {
                    v = ov;
                    kk = ok;
                }
            }
            if (bestk == 0 || v < best) {
                best = v;
                bestk = kk;
            }
        }
        sincos(dir * bestk * step, &s_out, &c_out);
        return dir * bestk * step;
    }
    // bracket: lo (E' not yet past zero) and hi = the first sample that is;
    // sin and cos inside it from those at hi, by the angle-addition formulas
    // with series for the offset (at most one degree, where the series below
    // are exact to rounding: next terms below 1e-20 relative)
    const double ref = dir * kfirst * step;
    double lo = dir * (kfirst - 1) * step, hi = ref;
    auto sc_at = [&](double x, double &st, double &ct) {
        const double dl = x - ref, d2 = dl * dl;
        const double sd = dl * (1.0 - d2 / 6.0 * (1.0 - d2 / 20.0 * (1.0 - d2 / 42.0)));
        const double cd = 1.0 - d2 / 2.0 * (1.0 - d2 / 12.0 * (1.0 - d2 / 30.0 * (1.0 - d2 / 56.0)));
        st = s_hi * cd + c_hi * sd;
        ct = c_hi * cd - s_hi * sd;
    };
    double st, ct;
    sc_at(lo, st, ct);
    const double e_lo = L.deriv_sc(st, ct);
    double x = 0.5 * (lo + hi);
    if (e_lo != e_hi) {
        const double xs = lo + (hi - lo) * (e_lo / (e_lo - e_hi));
        if (xs > fmin(lo, hi) && xs < fmax(lo, hi)) x = xs;
    }
    // (a run of midpoint steps alone halves the bracket each time, so the
    // cap is reached only if Newton keeps failing).  The search ends at a
    // step below 1e-15 of max(|x|, 1 degree), or where |E'| is below four
    // units of rounding of its terms' moduli: there its sign is noise, and
    // further steps (Newton's or the midpoint's) would only wander inside the
    // rounding band around the root.
    const double tol = 1e-15 * fmax(fabs(x), step);
    constexpr double eps = 0x1p-52;   // double's machine epsilon
    for (int it = 0; it < 48; ++it) {
        sc_at(x, st, ct);
        const double d1 = L.deriv_sc(st, ct), d2v = L.deriv2_sc(st, ct);
        if (fabs(d1) <= 4.0 * eps * L.deriv_abs_sc(st, ct)) break;
        if (dir * d1 >= 0.0) hi = x; else lo = x;
        double xn = d2v != 0.0 ? x - d1 / d2v : 0.5 * (lo + hi);
        if (!(xn > fmin(lo, hi) && xn < fmax(lo, hi))) xn = 0.5 * (lo + hi);
        const bool done = fabs(xn - x) <= tol;
        x = xn;
        if (done) break;
    }
    sc_at(x, s_out, c_out);
    return x;
}

// H v, H w with shared class coefficients and the tile's partial Re<v|Hv>,
// Re<w|Hw>, Re<v|Hw> (the angle is chosen from them by the Taylor launch
// that follows).  mode 1: ADAPT iteration (instances already done are
// skipped); mode 0: timing.
template <typename T, int R>
__device__ __forceinline__ void line_hvw(const InstDev *__restrict__ insts, const int2 *__restrict__ blk, int mode) {
    const int2 b = work_row(blk);
    const InstDev &I = insts[b.x];
    AdaptState *st = I.st;
    if (mode != 0 && state_done(st)) return;
    const int lane = threadIdx.x & (kWave - 1);
    const int wv = wave_id();
    const uint32_t dim = 1u << I.n_qubits;
    const uint32_t d0 = (uint32_t)b.y * (kTile * R) + lane;

    // The three dots have v* or w* as left factor, and v, w vanish wherever
    // the selected generator does: a tile with v = w = 0 on all its amplitudes
    // contributes nothing.  Unless H v and H w are kept for the carried sigma
    // (FP64 states), such a tile only writes zero partials.  Every wave reads
    // the same amplitudes, so all waves of the tile take the same branch.
    if (I.hv == nullptr) {
        bool act = false;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint32_t d = d0 | ((uint32_t)r << 6);
            if (d < dim) {
                const double2 a = Amp<T>::load(I.v, d), c = Amp<T>::load(I.w, d);
                act = act || a.x != 0.0 || a.y != 0.0 || c.x != 0.0 || c.y != 0.0;
            }
        }
        if (__ballot(act) == 0ull) {
            if (wv == 0 && lane == 0) {
                double *pl = I.part_l + 2 * I.n_pblk + 3 * b.y;
                pl[0] = 0.0;
                pl[1] = 0.0;
                pl[2] = 0.0;
            }
            return;
        }
    }

    __shared__ Stage S;
    double acc[4 * R];
#pragma unroll
    for (int i = 0; i < 4 * R; ++i) acc[i] = 0.0;
    apply_classes<T, 2, R>(I, S, d0, dim, I.v, I.w, acc);
    double4 (*red)[kWave] = reinterpret_cast<double4 (*)[kWave]>(&S);
    double p3 = 0.0, p5 = 0.0, p6 = 0.0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        red[wv][lane] = make_double4(acc[2 * r], acc[2 * r + 1], acc[2 * (R + r)], acc[2 * (R + r) + 1]);
        __syncthreads();
        if (wv == 0) {
            double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
#pragma unroll
            for (int k = 0; k < kNW; ++k) {
                const double4 q = red[k][lane];
                a0 += q.x;
                a1 += q.y;
                a2 += q.z;
                a3 += q.w;
            }
            const uint32_t d = d0 | ((uint32_t)r << 6);
            if (d < dim) {
                const double2 ov = Amp<T>::load(I.v, d), ow = Amp<T>::load(I.w, d);
                p3 += ov.x * a0 + ov.y * a1;
                p5 += ow.x * a2 + ow.y * a3;
                p6 += ov.x * a2 + ov.y * a3;
                if (I.hv) {
                    I.hv[d] = make_double2(a0, a1);
                    I.hw[d] = make_double2(a2, a3);
                }
            }
        }
        __syncthreads();
    }
    if (wv == 0) {
        p3 = wave_sum(p3);
        p5 = wave_sum(p5);
        p6 = wave_sum(p6);
        if (lane == 0) {
            double *pl = I.part_l + 2 * I.n_pblk + 3 * b.y;
            pl[0] = p3;
            pl[1] = p5;
            pl[2] = p6;
        }
    }
}

template <typename T, int R>
__global__ __launch_bounds__(kNW *kWave) void k_line_hvw(const InstDev *__restrict__ insts,
                                                        const int2 *__restrict__ blk, int mode) {
    line_hvw<T, R>(insts, blk, mode);
}
// one amplitude per lane: at most 64 VGPRs, two workgroups per CU
template <typename T>
__global__ __launch_bounds__(kNW *kWave) __attribute__((amdgpu_waves_per_eu(8))) void k_line_hvw1(
    const InstDev *__restrict__ insts, const int2 *__restrict__ blk, int mode) {
    line_hvw<T, 1>(insts, blk, mode);
}

// H applied to two vectors at the lane's amplitudes d[a], a < C, over the
// records [c0, c1) of H's class table (global indices), every table value
// read through the scalar cache (no LDS staging):
//   acc[a][2 v + {0,1}] += f_c(d[a]) vec_v(d[a] ^ x_c),  v = 0, 1.
// NB records per batch: the batch's records are read in one go, then every
// record's first string group and the gathers of all C amplitudes are issued
// together, then the strings are summed (a record's further groups are read
// where they are used); each record's table values serve all C amplitudes.
// Records past c1 re-read the run's last record and are not summed.
// Factored classes (kFactBit) hold one group of parameters (see fact_h).
template <typename T, int NB, int C>
__device__ __forceinline__ void walk_run_scalar(const HClass *hcls, const double *hcoef, const uint32_t *hzs,
                                                int c0, int c1, const uint32_t (&d)[C], const void *v0,
                                                const void *v1, double (&acc)[C][4]) {
    using Raw = typename Amp<T>::Raw;
    if (c0 >= c1) return;
    uint32_t doff[C], dz[C];
#pragma unroll
    for (int a = 0; a < C; ++a) {
        doff[a] = d[a] << Amp<T>::kShift;
        asm volatile("" : "+v"(doff[a]));      // keep the shifted offset: one XOR per gather
        dz[a] = with_sign_bit(d[a]);
    }
    const GOCP_AS4 HClass *rec = cptr(hcls);
    const GOCP_AS4 double *co = cptr(hcoef);
    const GOCP_AS4 uint32_t *zs = cptr(hzs);
    for (int c = c0; c < c1; c += NB) {
        HClass r[NB];
#pragma unroll
        for (int k = 0; k < NB; ++k) r[k] = load_rec(rec, min(c + k, c1 - 1));
        double cm[NB][kStrGroup];
        uint32_t zm[NB][kStrGroup];
        Raw p[NB][C][2];
#pragma unroll
        for (int k = 0; k < NB; ++k) {
#pragma unroll
            for (int a = 0; a < C; ++a) {
                const uint32_t o = doff[a] ^ (r[k].x << Amp<T>::kShift);
                p[k][a][0] = Amp<T>::raw_at(v0, o);
                p[k][a][1] = Amp<T>::raw_at(v1, o);
            }
#pragma unroll
            for (int q = 0; q < kStrGroup; ++q) {
                cm[k][q] = co[r[k].s0 + q];
                zm[k][q] = zs[r[k].s0 + q];
            }
        }
#pragma unroll
        for (int k = 0; k < NB; ++k) {
            if (c + k >= c1) break;
            double f[C];
            if (r[k].x & kFactBit) {
#pragma unroll
                for (int a = 0; a < C; ++a) f[a] = fact_h(cm[k][0], zm[k][0], zm[k][1], zm[k][2], dz[a]);
            } else {
                double f0[C], f1[C];
#pragma unroll
                for (int a = 0; a < C; ++a) {
                    f0[a] = signed_cz(cm[k][0], zm[k][0], dz[a]) + signed_cz(cm[k][2], zm[k][2], dz[a]);
                    f1[a] = signed_cz(cm[k][1], zm[k][1], dz[a]) + signed_cz(cm[k][3], zm[k][3], dz[a]);
                }
                for (int q = r[k].s0 + kStrGroup; q < r[k].s1; q += kStrGroup) {
#pragma unroll
                    for (int a = 0; a < C; ++a) {
                        f0[a] += signed_cz(co[q], zs[q], dz[a]) + signed_cz(co[q + 2], zs[q + 2], dz[a]);
                        f1[a] += signed_cz(co[q + 1], zs[q + 1], dz[a]) + signed_cz(co[q + 3], zs[q + 3], dz[a]);
                    }
                }
#pragma unroll
                for (int a = 0; a < C; ++a) f[a] = f0[a] + f1[a];
            }
#pragma unroll
            for (int a = 0; a < C; ++a)
#pragma unroll
                for (int v = 0; v < 2; ++v) {
                    const double2 x = Amp<T>::cvt(p[k][a][v]);
                    acc[a][2 * v] = fma(f[a], x.x, acc[a][2 * v]);
                    acc[a][2 * v + 1] = fma(f[a], x.y, acc[a][2 * v + 1]);
                }
        }
    }
}

// H v, H w dots over the listed active amplitudes (complex64 states, whose
// line search keeps no H v, H w).  The three dots have v* or w* as left
// factor, so only amplitudes where v or w is nonzero contribute; k_line_vw
// lists them per pair block (entries [0, count) of the block's list).
// Row (instance, slot P + part), P = hvw_parts (a power of two), slot <
// min(kHvwSlots, pair blocks):
// the workgroup takes the lists of pair blocks slot, slot + slots, ..., 64
// entries at a time (one per lane; two blocks' entries per pass where both
// have some left), and wave w applies run `part` of its
// segment of H's classes (a 1 / (kNW P) share of H) with the table
// read through the scalar cache.  Since the dots are linear in H v and H w,
// each (block, tile, run) adds v* (H_run v) etc. at once; the workgroup writes
// its partial triple to row y of the line-search partials.  The row count is
// a function of the instance alone.  Every table and list value is loaded in
// as few dependent steps as the data allow: the descriptor, then the state's
// flag with the wave's run bounds and the first block's count and entries,
// then the class records, then the strings with the gathers.
// mode 1: ADAPT iteration; mode 0: timing.
template <typename T>
// (at most 64 VGPRs: two workgroups per CU, which the many rows of a batch need)
__global__ __launch_bounds__(kNW *kWave) __attribute__((amdgpu_waves_per_eu(8))) void k_line_hvw_act(
    const InstDev *__restrict__ insts, const int2 *__restrict__ blk, int mode) {
    const int2 b = work_row(blk);
    const InstDev &I = insts[b.x];
    const int lane = threadIdx.x & (kWave - 1);
    const int wv = wave_id();
    const AdaptState *st = I.st;
    const int nq = I.n_qubits, nb = I.n_pblk, nhc = I.n_hchunks, np = I.hvw_parts;
    const int32_t *hsegp = I.hsegp, *act_n = I.act_n;
    const void *vv = I.v, *vw = I.w;
    const uint32_t *act = I.act, *hzs = I.hzs;
    const HClass *hcls = I.hcls;
    const double *hcoef = I.hcoef;
    double *part_l = I.part_l;
    asm volatile("" ::"s"(st), "s"(nq), "s"(nb), "s"(nhc), "s"(np), "s"(hsegp), "s"(act_n), "s"(vv), "s"(vw),
                 "s"(act), "s"(hzs), "s"(hcls), "s"(hcoef), "s"(part_l));
    const int lg = 31 - __clz(np);
    const int slot = b.y >> lg, part = b.y & (np - 1);
    const int nslot = min(kHvwSlots, nb);
    const int r0 = wv * np + part;
    constexpr int kList = 2 * kPairBlock;          // list capacity of a pair block
    const int done = cptr(&st->done)[0];
    const int ra = cptr(hsegp)[r0], rb = cptr(hsegp)[r0 + 1];
    const int cnt0 = cptr(act_n)[slot];
    const uint32_t e0 = gptr(act)[(size_t)slot * kList + lane];
    asm volatile("" ::"s"(done), "s"(ra), "s"(rb), "s"(cnt0));
    if (mode != 0 && done) return;
    const uint32_t dim = 1u << nq;
    __shared__ double rsum[3][kNW];
    double p3 = 0.0, p5 = 0.0, p6 = 0.0;
    // H applied over the wave's run (every stage chunk of H) at C amplitudes
    auto walk = [&](auto cc, const auto &d, auto &acc) {
        constexpr int C = decltype(cc)::value;
        for (int k = 0; k < nhc; ++k) {
            const int r = k * (kNW * np + 1) + r0;
            const int c0 = k == 0 ? ra : cptr(hsegp)[r], c1 = k == 0 ? rb : cptr(hsegp)[r + 1];
            // (records per batch: kHvwBatch for one amplitude, half for two,
            // the same gathers per batch)
            walk_run_scalar<T, (C > 1 ? kHvwBatch / 2 : kHvwBatch), C>(hcls, hcoef, hzs, c0, c1, d, vv, vw, acc);
        }
    };
    auto entry = [&](int bk, int g, bool on, bool first) {
        uint32_t d = first ? e0 : gptr(act)[(size_t)bk * kList + min(g, kList - 1)];
        return on ? d & (dim - 1u) : 0u;
    };
    // (each amplitude's own v, w are loaded before its walk, so their
    // latency passes under it)
    auto add = [&](const double2 &ov, const double2 &ow, bool on, const double (&acc)[4]) {
        if (on) {
            p3 += ov.x * acc[0] + ov.y * acc[1];
            p5 += ow.x * acc[2] + ow.y * acc[3];
            p6 += ov.x * acc[2] + ov.y * acc[3];
        }
    };
    // the slot's blocks two at a time (slot + 2 i nslot and the next one), 64
    // entries of each per pass: one walk over the run serves both
    for (int bk = slot; bk < nb; bk += 2 * nslot) {
        const int bk2 = bk + nslot;
        const int cnt = min(max(bk == slot ? cnt0 : cptr(act_n)[bk], 0), kList);
        const int cnt2 = bk2 < nb ? min(max(cptr(act_n)[bk2], 0), kList) : 0;
        for (int t = 0; t * kWave < max(cnt, cnt2); ++t) {
            const int g = t * kWave + lane;
            const bool on = g < cnt;
            const uint32_t d = entry(bk, g, on, bk == slot && t == 0);
            if (t * kWave < cnt2) {
                const bool on2 = g < cnt2;
                const uint32_t dd[2] = {d, entry(bk2, g, on2, false)};
                const double2 ov = Amp<T>::load(vv, dd[0]), ow = Amp<T>::load(vw, dd[0]);
                const double2 ov2 = Amp<T>::load(vv, dd[1]), ow2 = Amp<T>::load(vw, dd[1]);
                double acc[2][4] = {{0.0, 0.0, 0.0, 0.0}, {0.0, 0.0, 0.0, 0.0}};
                walk(std::integral_constant<int, 2>(), dd, acc);
                add(ov, ow, on, acc[0]);
                add(ov2, ow2, on2, acc[1]);
            } else {
                const uint32_t dd[1] = {d};
                const double2 ov = Amp<T>::load(vv, d), ow = Amp<T>::load(vw, d);
                double acc[1][4] = {{0.0, 0.0, 0.0, 0.0}};
                walk(std::integral_constant<int, 1>(), dd, acc);
                add(ov, ow, on, acc[0]);
            }
        }
    }
    // the workgroup's triple: wave sums, then waves in order
    p3 = wave_sum(p3);
    p5 = wave_sum(p5);
    p6 = wave_sum(p6);
    if (lane == 0) {
        rsum[0][wv] = p3;
        rsum[1][wv] = p5;
        rsum[2][wv] = p6;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        double a = 0.0;
        for (int k = 0; k < kNW; ++k) a += rsum[threadIdx.x][k];
        part_l[2 * nb + 3 * b.y + threadIdx.x] = a;
    }
}

// ------------------------------------------------------------------ K3: O(5) Taylor update

// The angle of an ADAPT iteration, computed by every workgroup of the Taylor
// launch from the line-search partials (so no workgroup waits on another):
// the five dot products, each summed in a fixed order, give the landscape, and
// wave 0 searches it.  Returns theta and the substep count in every thread;
// the workgroup of pair block 0 also writes the iteration record.
// Inputs of the landscape: the state's scalars and the selected operator's
// gradient and norm (scalar loads), and this thread's shares of the five
// line-search dot products (vector loads).  Issued in one batch; the values
// are first used by choose_angle.
struct AngleIn {
    double nrm, e_num, gj, onorm;
    int it;                     // the state record's iteration and history arrays (for the writer)
    int32_t *h_op, *h_ns;
    double *h_th, *h_pr;
    double r[5];                // the thread's first share (masked by use3, use2)
    double q[5];                // the sum of its further shares
    bool use3, use2;
};
__device__ __forceinline__ void angle_loads(const AdaptState *st, const double *g, const double *op_norm1,
                                            const double *part_l, int n_pblk, int n_lpart, int j, AngleIn &in) {
    in.nrm = cptr(&st->nrm)[0];
    in.e_num = cptr(&st->e_num)[0];
    in.gj = cptr(g)[j];
    in.onorm = cptr(op_norm1)[j];
    in.it = cptr(&st->iter)[0];
    in.h_op = cptr(&st->hist_op)[0];
    in.h_ns = cptr(&st->hist_nsub)[0];
    in.h_th = cptr(&st->hist_theta)[0];
    in.h_pr = cptr(&st->hist_pred)[0];
    // a thread's first share is loaded (at a clamped index) and left
    // unused until the angle is chosen, so nothing waits on it here; further
    // shares, for states with more partials than threads, are summed in
    // their loops
    const GOCP_AS1 double *pp = gptr(part_l), *pl = pp + 2 * n_pblk;
    const int i0 = threadIdx.x;
    const int l3 = min(i0, n_lpart - 1), l2 = min(i0, n_pblk - 1);
    in.use3 = i0 < n_lpart;
    in.use2 = i0 < n_pblk;
    in.r[0] = pl[3 * l3];
    in.r[1] = pl[3 * l3 + 1];
    in.r[2] = pl[3 * l3 + 2];
    in.r[3] = pp[2 * l2];
    in.r[4] = pp[2 * l2 + 1];
#pragma unroll
    for (int k = 0; k < 5; ++k) in.q[k] = 0.0;
    for (int i = i0 + kPairBlock; i < n_lpart; i += kPairBlock) {
        in.q[0] += pl[3 * i];
        in.q[1] += pl[3 * i + 1];
        in.q[2] += pl[3 * i + 2];
    }
    for (int i = i0 + kPairBlock; i < n_pblk; i += kPairBlock) {
        in.q[3] += pp[2 * i];
        in.q[4] += pp[2 * i + 1];
    }
}

__device__ void choose_angle(const AngleIn &in, AdaptState *st, int j, bool writer, double &theta, int &ns) {
    __shared__ double red[5][kPairBlock / kWave];
    __shared__ double s_th;
    __shared__ int s_ns;
    const int lane = threadIdx.x & (kWave - 1), wv = wave_id();
    const double nrm = in.nrm, e_num = in.e_num, gj = in.gj, onorm = in.onorm;
    double q[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) q[k] = ((k < 3 ? in.use3 : in.use2) ? in.r[k] : 0.0) + in.q[k];
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        const double v = wave_sum(q[k]);
        if (lane == 0) red[k][wv] = v;
    }
    __syncthreads();
    if (wv == 0) {
        double P[5];
#pragma unroll
        for (int k = 0; k < 5; ++k) {
            P[k] = 0.0;
            for (int w = 0; w < kPairBlock / kWave; ++w) P[k] += red[k][w];
        }
        const double P3 = P[0], P5 = P[1], P6 = P[2], P2 = P[3], P7 = P[4];
        const double inv = 1.0 / nrm;
        Landscape L;
        L.uu = (e_num - 2.0 * P2 + P3) * inv;
        L.uv = (P2 - P3) * inv;
        L.uw = (P7 - P6) * inv;
        L.vv = P3 * inv;
        L.vw = P6 * inv;
        L.ww = P5 * inv;
        double sth, cth;
        const double th = line_search_wave(L, gj, sth, cth);
        if (lane == 0) {
            const int n = th == 0.0 ? 0 : max(1, (int)ceil(fabs(th) * onorm / 0.5));
            s_th = th;
            s_ns = n;
            if (writer) {
                // T5(h) = I + a A + b A^2 once A^3 = -A (and A^4 = -A^2); the product
                // of such factors stays in that span and multiplies like the
                // complex numbers (1 - b) + i a (A acts as i on its +-i
                // eigenspaces), so the chain T5(h)^n is I + al A + be A^2 with
                // (1 - be) + i al = ((1 - b) + i a)^n, formed by squaring
                double al = 0.0, be = 0.0;
                if (n > 0) {
                    const double h = th / n, h2 = h * h;
                    const double a = h * (1.0 - h2 / 6.0 * (1.0 - h2 / 20.0));   // h - h^3/6 + h^5/120
                    const double b = h2 * (0.5 - h2 / 24.0);                     // h^2/2 - h^4/24
                    double zr = 1.0 - b, zi = a, pr = 1.0, pi = 0.0;
                    for (int k = n; k > 0; k >>= 1) {
                        if (k & 1) {
                            const double tr = pr * zr - pi * zi;
                            pi = pr * zi + pi * zr;
                            pr = tr;
                        }
                        const double sr = zr * zr - zi * zi;
                        zi = 2.0 * zr * zi;
                        zr = sr;
                    }
                    al = pi;
                    be = 1.0 - pr;
                }
                // global (not flat) stores; the history pointers are never
                // written by a kernel
                GOCP_AS1 AdaptState *gs = gmut(st);
                const double pred = L.value_sc(sth, cth);
                gs->upd_alpha = al;
                gs->upd_beta = be;
                gs->upd_scale = 1.0 / sqrt(nrm);
                gs->theta = th;
                gs->nsub = n;
                gs->pred = pred;
                if (in.h_op) gmut(in.h_op)[in.it] = j;
                if (in.h_th) gmut(in.h_th)[in.it] = th;
                if (in.h_ns) gmut(in.h_ns)[in.it] = n;
                if (in.h_pr) gmut(in.h_pr)[in.it] = pred;
            }
        }
    }
    __syncthreads();
    theta = s_th;
    ns = s_ns;
}

// psi <- T5(theta/s)^s (scale * psi) on the pairs of generator j.  In an ADAPT
// iteration (adapt != 0) j comes from the device state, theta and s from the
// line search done here, and scale is 1/sqrt(<psi|psi>) of the stored state
// (the renormalisation of the previous update, applied here); one-shot calls
// pass them as arguments.  Writes the per-workgroup |psi|^2 of the result to
// part_t.
template <typename T, bool Adapt>
__global__ __launch_bounds__(kPairBlock) void k_taylor5(const InstDev *__restrict__ insts,
                                                       const int2 *__restrict__ blk, int j_arg, double theta_arg,
                                                       int s_arg) {
    const int2 b = work_row(blk);
    const InstDev &I = insts[b.x];
    // Loads in batches ahead of their uses (a chain of one load per field
    // otherwise): the descriptor fields; the state record's head; then the
    // generator's record, gradient and norm together with the line-search
    // partials; then its strings and the pair's amplitudes.  None of the pair
    // work depends on the angle, so all of it is read before the angle is
    // chosen.
    AdaptState *st = I.st;
    const HClass *pop = I.pop;
    const HTerm *pterm = I.pterm;
    const double *op_norm1 = I.op_norm1, *part_l = I.part_l;
    void *psi = I.psi;
    const int nq = I.n_qubits, npb = I.n_pblk, nlp = I.n_lpart;
    asm volatile("" ::"s"(st), "s"(pop), "s"(pterm), "s"(op_norm1), "s"(part_l), "s"(psi), "s"(nq), "s"(npb),
                 "s"(nlp));
    int j = j_arg;
    const double *gv = nullptr;
    if constexpr (Adapt) {
        const StHead h = load_head(st);
        gv = cptr(&st->g)[0];
        asm volatile("" ::"s"(h.done), "s"(h.jsel), "s"(gv));
        if (h.done) return;
        j = h.jsel;
    }
    const HClass C = load_rec(cptr(pop), j);
    AngleIn in;
    if constexpr (Adapt) angle_loads(st, gv, op_norm1, part_l, npb, nlp, j, in);
    const uint32_t m = C.x;
    const int hb = 31 - __clz(m);
    const uint32_t half = 1u << (nq - 1);
    const uint32_t p = (uint32_t)b.y * kPairBlock + threadIdx.x;
    const bool own = p < half;
    const uint32_t d = own ? insert_zero_bit(p, hb) : 0u, e = d ^ m;
    double hd = 0.0, he = 0.0;
    double2 a = make_double2(0.0, 0.0), c = a;
    if (own) {
        a = Amp<T>::load(psi, d);
        c = Amp<T>::load(psi, e);
        string_sum2(cptr(pterm), C.s0, C.s1, d, e, hd, he);
    }
    double theta = theta_arg;
    int ns = s_arg;
    if constexpr (Adapt) choose_angle(in, st, j, b.y == 0, theta, ns);
    const double scale = Adapt ? 1.0 / sqrt(in.nrm) : 1.0;
    double nn = 0.0;
    if (own) {
        a.x *= scale; a.y *= scale;
        c.x *= scale; c.y *= scale;
        if (ns > 0) {
            const double x = theta / ns;
            for (int sub = 0; sub < ns; ++sub) {
                double2 va = a, vc = c, acca = a, accc = c;
                double coef = 1.0;
#pragma unroll
                for (int n = 1; n <= 5; ++n) {
                    const double2 na = make_double2(hd * vc.x, hd * vc.y);   // (A v)[d] = h(d) v[e]
                    const double2 nc = make_double2(he * va.x, he * va.y);   // (A v)[e] = h(e) v[d]
                    va = na;
                    vc = nc;
                    coef = coef * x / n;
                    acca.x = fma(coef, va.x, acca.x);
                    acca.y = fma(coef, va.y, acca.y);
                    accc.x = fma(coef, vc.x, accc.x);
                    accc.y = fma(coef, vc.y, accc.y);
                }
                a = acca;
                c = accc;
            }
        }
        Amp<T>::store(I.psi, d, a);
        Amp<T>::store(I.psi, e, c);
        const double2 ra = Amp<T>::rounded(a), rc = Amp<T>::rounded(c);
        nn = ra.x * ra.x + ra.y * ra.y + rc.x * rc.x + rc.y * rc.y;
    }
    __shared__ double rn[kPairBlock / kWave];
    nn = wave_sum(nn);
    const int wv = wave_id(), lane = threadIdx.x & (kWave - 1);
    if (lane == 0) rn[wv] = nn;
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0.0;
        for (int k = 0; k < kPairBlock / kWave; ++k) a += rn[k];
        I.part_t[b.y] = a;
    }
}

// ------------------------------------------------------------------ re-optimisation layers

// ADAPT with every angle re-optimised: the ansatz is a chain of layers
// L(theta) = T5(x)^s (Eq. 5-6, x = theta / s), each a pool generator with one
// X mask, so one lane owns one amplitude pair (d, e = d ^ x_A) of the layer's
// generator and applies its polynomials in registers.  On a pair,
// (A v)[d] = h(d) v[e] and (A v)[e] = h(e) v[d].

// sum_{n <= N} x^n A^n / n! on the pair (a at d, c at e), as the power sum of Eq. 6.
template <int N>
__device__ __forceinline__ void pair_series(double hd, double he, double x, double2 &a, double2 &c) {
    double2 va = a, vc = c, acca = a, accc = c;
    double coef = 1.0;
#pragma unroll
    for (int n = 1; n <= N; ++n) {
        const double2 na = make_double2(hd * vc.x, hd * vc.y);
        const double2 nc = make_double2(he * va.x, he * va.y);
        va = na;
        vc = nc;
        coef = coef * x / n;
        acca.x = fma(coef, va.x, acca.x);
        acca.y = fma(coef, va.y, acca.y);
        accc.x = fma(coef, vc.x, accc.x);
        accc.y = fma(coef, vc.y, accc.y);
    }
    a = acca;
    c = accc;
}

// The pair of lane p for generator record C on 2^nq amplitudes: d (bit hb of
// the mask cleared), e = d ^ mask, and whether the lane owns a pair.
__device__ __forceinline__ bool layer_pair(const HClass &C, int nq, uint32_t &d, uint32_t &e) {
    const uint32_t m = C.x;
    const int hb = 31 - __clz(m);
    const uint32_t p = blockIdx.x * kPairBlock + threadIdx.x;
    const bool own = p < (1u << (nq - 1));
    d = own ? insert_zero_bit(p, hb) : 0u;
    e = d ^ m;
    return own;
}

// Forward layer, out of place: out = T5(x)^ns in on every pair of generator j.
template <typename T>
__global__ __launch_bounds__(kPairBlock) void k_layer_fwd(const void *__restrict__ in, void *__restrict__ out,
                                                         const HClass *__restrict__ pop,
                                                         const HTerm *__restrict__ pterm, int j, int ns, double x,
                                                         int nq) {
    const HClass C = load_rec(cptr(pop), j);
    uint32_t d, e;
    if (!layer_pair(C, nq, d, e)) return;
    double2 a = Amp<T>::load(in, d), c = Amp<T>::load(in, e);
    double hd, he;
    string_sum2(cptr(pterm), C.s0, C.s1, d, e, hd, he);
    for (int sub = 0; sub < ns; ++sub) pair_series<5>(hd, he, x, a, c);
    Amp<T>::store(out, d, a);
    Amp<T>::store(out, e, c);
}

// Backward layer: with phi the state before the layer and lam the adjoint
// vector after it (complex128, updated in place),
//   partial[block] = sum over the block's pairs of Re <lam | T5(x)^(ns-1) A T4(x) phi>
//   lam <- T5(-x)^ns lam
// (the layer's derivative and its adjoint: the series in -A, since A^+ = -A).
// When sigma is given this is the last layer: lam is first formed as
// sigma - E psi with psi = the ansatz state (state type T) and E = e_num / nrm
// of the state record st.
template <typename T>
__global__ __launch_bounds__(kPairBlock) void k_layer_adj(const void *__restrict__ phi, double2 *__restrict__ lam,
                                                         double *__restrict__ partial,
                                                         const HClass *__restrict__ pop,
                                                         const HTerm *__restrict__ pterm, int j, int ns, double x,
                                                         int nq, const double2 *__restrict__ sigma,
                                                         const void *__restrict__ psi,
                                                         const AdaptState *__restrict__ st) {
    const HClass C = load_rec(cptr(pop), j);
    uint32_t d, e;
    const bool own = layer_pair(C, nq, d, e);
    double dot = 0.0;
    if (own) {
        double hd, he;
        string_sum2(cptr(pterm), C.s0, C.s1, d, e, hd, he);
        double2 la, lc;
        if (sigma) {
            const double en = cptr(&st->e_num)[0] / cptr(&st->nrm)[0];
            const double2 sa = sigma[d], sc = sigma[e], pa = Amp<T>::load(psi, d), pc = Amp<T>::load(psi, e);
            la = make_double2(sa.x - en * pa.x, sa.y - en * pa.y);
            lc = make_double2(sc.x - en * pc.x, sc.y - en * pc.y);
        } else {
            la = lam[d];
            lc = lam[e];
        }
        double2 a = Amp<T>::load(phi, d), c = Amp<T>::load(phi, e);
        pair_series<4>(hd, he, x, a, c);
        const double2 na = make_double2(hd * c.x, hd * c.y), nc = make_double2(he * a.x, he * a.y);
        a = na;
        c = nc;
        for (int sub = 1; sub < ns; ++sub) pair_series<5>(hd, he, x, a, c);
        dot = (la.x * a.x + la.y * a.y) + (lc.x * c.x + lc.y * c.y);
        for (int sub = 0; sub < ns; ++sub) pair_series<5>(hd, he, -x, la, lc);
        lam[d] = la;
        lam[e] = lc;
    }
    __shared__ double rd[kPairBlock / kWave];
    dot = wave_sum(dot);
    const int wv = wave_id(), lane = threadIdx.x & (kWave - 1);
    if (lane == 0) rd[wv] = dot;
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0.0;
        for (int k = 0; k < kPairBlock / kWave; ++k) a += rd[k];
        partial[blockIdx.x] = a;
    }
}

// GOCP multi-operator step (Sec. III.A families, Eq. 5-6 chains): N pool
// operators of one commuting family, X masks independent over GF(2), applied
// in one pass.  The masks span a group of 2^N bit flips; each operator maps
// every coset (orbit) of it into itself.  An orbit's 2^N amplitudes sit in
// 2^N adjacent lanes: local index m (the lane's low N bits; bit j for
// operator j) holds the representative XOR the masks of m's bits, the
// representative having zero bits at the span's echelon pivots.  Operator j
// pairs m with m ^ 2^j, a lane shuffle, so every operator's substepped O(5)
// chain runs in registers and the state is read and written once.  Each lane
// takes its local index in two orbits (the first and the second half of the
// orbit numbers), so the launch has the pair kernels' workgroups and norm
// partials (part_t).  The operators' polynomials commute: their order is free.
template <typename T, int N>
__global__ __launch_bounds__(kPairBlock) void k_taylor5_fused(const InstDev *__restrict__ insts,
                                                             const int2 *__restrict__ blk, FuseArgs fa) {
    const int2 b = work_row(blk);
    const InstDev &I = insts[b.x];
    const int nq = I.n_qubits;
    const uint32_t gid = (uint32_t)b.y * kPairBlock + threadIdx.x;
    const bool own = gid < (1u << (nq - 1));
    const uint32_t m = gid & ((1u << N) - 1u), o = own ? gid >> N : 0u;
    const uint32_t half_orbits = 1u << (nq - N - 1);      // N < n_qubits
    HClass C[N];
#pragma unroll
    for (int j = 0; j < N; ++j) C[j] = load_rec(cptr(I.pop), fa.op[j]);
    uint32_t d[2];
    double2 a[2];
#pragma unroll
    for (int r = 0; r < 2; ++r) {
        uint32_t v = o + (uint32_t)r * half_orbits;
#pragma unroll
        for (int j = 0; j < N; ++j) v = insert_zero_bit(v, fa.piv[j]);
#pragma unroll
        for (int j = 0; j < N; ++j)
            if ((m >> j) & 1u) v ^= C[j].x;
        d[r] = v;
        a[r] = Amp<T>::load(I.psi, v);
    }
#pragma unroll
    for (int j = 0; j < N; ++j) {
        // (A_j v)[d] = f(d) v[d ^ x_j], and d ^ x_j sits in lane ^ 2^j
        double f0, f1;
        string_sum2(cptr(I.pterm), C[j].s0, C[j].s1, d[0], d[1], f0, f1);
        const double x = fa.x[j];
        for (int sub = 0; sub < fa.ns[j]; ++sub) {
            double2 v0 = a[0], v1 = a[1];
            double coef = 1.0;
#pragma unroll
            for (int n = 1; n <= 5; ++n) {
                const double p0x = __shfl_xor(v0.x, 1 << j), p0y = __shfl_xor(v0.y, 1 << j);
                const double p1x = __shfl_xor(v1.x, 1 << j), p1y = __shfl_xor(v1.y, 1 << j);
                v0 = make_double2(f0 * p0x, f0 * p0y);
                v1 = make_double2(f1 * p1x, f1 * p1y);
                coef = coef * x / n;
                a[0].x = fma(coef, v0.x, a[0].x);
                a[0].y = fma(coef, v0.y, a[0].y);
                a[1].x = fma(coef, v1.x, a[1].x);
                a[1].y = fma(coef, v1.y, a[1].y);
            }
        }
    }
    double nn = 0.0;
    if (own) {
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            Amp<T>::store(I.psi, d[r], a[r]);
            const double2 q = Amp<T>::rounded(a[r]);
            nn += q.x * q.x + q.y * q.y;
        }
    }
    __shared__ double rn[kPairBlock / kWave];
    nn = wave_sum(nn);
    const int wv = wave_id(), lane = threadIdx.x & (kWave - 1);
    if (lane == 0) rn[wv] = nn;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int k = 0; k < kPairBlock / kWave; ++k) t += rn[k];
        I.part_t[b.y] = t;
    }
}

// psi *= 1 / sqrt(sum of part_t)   (from_state: 1 / sqrt(st->nrm) instead)
template <typename T>
__global__ __launch_bounds__(kPairBlock) void k_normalize(const InstDev *__restrict__ insts,
                                                         const int2 *__restrict__ blk,
                                                         int from_state) {
    const int2 b = work_row(blk);
    const InstDev &I = insts[b.x];
    __shared__ double lds[kPairBlock];
    double nrm;
    if (from_state) {
        nrm = I.st->nrm;
    } else {
        nrm = block_sum_strided<kPairBlock>(I.part_t, I.n_pblk, 1, lds);
    }
    const double sc = 1.0 / sqrt(nrm);
    const uint32_t dim = 1u << I.n_qubits;
    for (uint32_t k = (uint32_t)b.y * 2 * kPairBlock + threadIdx.x;
         k < min(dim, (uint32_t)(b.y + 1) * 2 * kPairBlock); k += kPairBlock) {
        double2 a = Amp<T>::load(I.psi, k);
        a.x *= sc;
        a.y *= sc;
        Amp<T>::store(I.psi, k, a);
    }
}

// After psi has been scaled to unit norm from the state's own norm: record it.
__global__ void k_state_unit_norm(const InstDev *__restrict__ insts, const int2 *__restrict__ blk) {
    const int2 b = work_row(blk);
    AdaptState *st = insts[b.x].st;
    if (threadIdx.x == 0) {
        st->e_num = st->energy;
        st->nrm = 1.0;
    }
}

// done flag of every instance into one array (one copy to the host).
__global__ void k_gather_done(const InstDev *__restrict__ insts, int n, int32_t *out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = insts[i].st->done;
}

// psi = |index>
template <typename T>
__global__ void k_basis(void *psi, uint32_t dim, uint32_t index) {
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < dim) Amp<T>::store(psi, k, make_double2(k == index ? 1.0 : 0.0, 0.0));
}

// ------------------------------------------------------------------ launchers

// Launch K over nb workgroups of nt lanes on s; with a timestamp event set, the
// dispatch itself records it (start and / or end of the kernel).
#define GOCP_LAUNCH(K, nb, nt, ...)                                                              \
    do {                                                                                         \
        if (t0 || t1) hipExtLaunchKernelGGL(K, dim3(nb), dim3(nt), 0, s, t0, t1, 0, __VA_ARGS__); \
        else hipLaunchKernelGGL(K, dim3(nb), dim3(nt), 0, s, __VA_ARGS__);                       \
    } while (0)

template <typename T, int R>
static void launch_tile(int which, const InstDev *insts, const int2 *blk, int nblk, int mode, hipStream_t s,
                        hipEvent_t t0, hipEvent_t t1) {
    if (which == 2) {
        if constexpr (R == 1) GOCP_LAUNCH((k_energy_screen<T, 1, true>), nblk, kNW * kWave, insts, blk, mode);
        else GOCP_LAUNCH((k_energy_screen<T, R>), nblk, kNW * kWave, insts, blk, mode);
    } else if (which == 0) {
        GOCP_LAUNCH((k_energy_screen<T, R>), nblk, kNW * kWave, insts, blk, mode);
    } else if constexpr (R == 1) {
        GOCP_LAUNCH((k_line_hvw1<T>), nblk, kNW * kWave, insts, blk, mode);
    } else {
        GOCP_LAUNCH((k_line_hvw<T, R>), nblk, kNW * kWave, insts, blk, mode);
    }
}

template <typename T>
static void launch_all(int which, int R, const InstDev *insts, const int2 *blk, int nblk, int mode,
                       hipStream_t s, int j, double th, int ns, hipEvent_t t0, hipEvent_t t1) {
    switch (which) {
    case 0:
    case 3:
    case 8: {
        const int w = which == 0 ? 0 : which == 8 ? 2 : 1;
        if (R == 4) launch_tile<T, 4>(w, insts, blk, nblk, mode, s, t0, t1);
        else if (R == 2) launch_tile<T, 2>(w, insts, blk, nblk, mode, s, t0, t1);
        else launch_tile<T, 1>(w, insts, blk, nblk, mode, s, t0, t1);
        break;
    }
    case 1: GOCP_LAUNCH(k_screen_reduce<false>, nblk, kPairBlock, insts, blk, mode); break;
    case 9: GOCP_LAUNCH(k_screen_reduce<true>, nblk, kPairBlock, insts, blk, mode); break;
    case 7: {
        // j: the operator column blocks (at least one)
        const dim3 grid(nblk, std::max(1, j));
        if (t0 || t1) hipExtLaunchKernelGGL(k_screen_sum1, grid, dim3(kPairBlock), 0, s, t0, t1, 0, insts, blk, mode);
        else hipLaunchKernelGGL(k_screen_sum1, grid, dim3(kPairBlock), 0, s, insts, blk, mode);
        break;
    }
    case 2: GOCP_LAUNCH((k_line_vw<T, false>), nblk, kPairBlock, insts, blk); break;
    case 10: GOCP_LAUNCH((k_line_vw<T, true>), nblk, kPairBlock, insts, blk); break;
    case 4:
        if (mode) GOCP_LAUNCH((k_taylor5<T, true>), nblk, kPairBlock, insts, blk, j, th, ns);
        else GOCP_LAUNCH((k_taylor5<T, false>), nblk, kPairBlock, insts, blk, j, th, ns);
        break;
    case 5: GOCP_LAUNCH(k_normalize<T>, nblk, kPairBlock, insts, blk, mode); break;
    case 6: GOCP_LAUNCH(k_state_unit_norm, nblk, 64, insts, blk); break;
    default: break;
    }
}

// No rows: the timestamp events, if any, mark the empty launch's place in s.
static void record_empty(hipEvent_t t0, hipEvent_t t1, hipStream_t s) {
    if (t0) hip_check(hipEventRecord(t0, s), "hipEventRecord");
    if (t1) hip_check(hipEventRecord(t1, s), "hipEventRecord");
}

void launch_kernel(int which, int dtype, int R, const InstDev *insts, const int2 *blk, int nblk, int mode,
                   hipStream_t s, int j, double th, int ns, hipEvent_t t0, hipEvent_t t1) {
    if (nblk <= 0) return record_empty(t0, t1, s);
    if (dtype == GOCP_C64)
        launch_all<float2>(which, R, insts, blk, nblk, mode, s, j, th, ns, t0, t1);
    else
        launch_all<double2>(which, R, insts, blk, nblk, mode, s, j, th, ns, t0, t1);
    hip_check(hipGetLastError(), "kernel launch");
}

bool phase_trace_read(unsigned long long *out, size_t n) {
#ifdef GOCP_PHASE_TRACE
    hip_check(hipMemcpyFromSymbol(out, HIP_SYMBOL(g_phase), n * sizeof(unsigned long long), 0,
                                  hipMemcpyDeviceToHost),
              "hipMemcpyFromSymbol(phase trace)");
    return true;
#else
    (void)out;
    (void)n;
    return false;
#endif
}

void launch_hvw_act(const InstDev *insts, const int2 *blk, int nblk, int mode, hipStream_t s, hipEvent_t t0,
                    hipEvent_t t1) {
    if (nblk <= 0) return record_empty(t0, t1, s);
    GOCP_LAUNCH(k_line_hvw_act<float2>, nblk, kNW * kWave, insts, blk, mode);
    hip_check(hipGetLastError(), "kernel launch");
}

#undef GOCP_LAUNCH

template <typename T>
static void launch_fused_t(int n, const InstDev *insts, const int2 *blk, int nblk, const FuseArgs &fa,
                           hipStream_t s) {
    switch (n) {
    case 1: hipLaunchKernelGGL((k_taylor5_fused<T, 1>), dim3(nblk), dim3(kPairBlock), 0, s, insts, blk, fa); break;
    case 2: hipLaunchKernelGGL((k_taylor5_fused<T, 2>), dim3(nblk), dim3(kPairBlock), 0, s, insts, blk, fa); break;
    case 3: hipLaunchKernelGGL((k_taylor5_fused<T, 3>), dim3(nblk), dim3(kPairBlock), 0, s, insts, blk, fa); break;
    case 4: hipLaunchKernelGGL((k_taylor5_fused<T, 4>), dim3(nblk), dim3(kPairBlock), 0, s, insts, blk, fa); break;
    default: break;       // the host entry accepts 1 to kFuseMax operators only
    }
}

void launch_fused(int dtype, int n, const InstDev *insts, const int2 *blk, int nblk, const FuseArgs &fa,
                  hipStream_t s) {
    if (nblk <= 0) return;
    if (dtype == GOCP_C64) launch_fused_t<float2>(n, insts, blk, nblk, fa, s);
    else launch_fused_t<double2>(n, insts, blk, nblk, fa, s);
    hip_check(hipGetLastError(), "kernel launch");
}

void launch_layer_fwd(int dtype, const void *in, void *out, const HClass *pop, const HTerm *pterm, int j, int ns,
                      double x, int nq, hipStream_t s) {
    const int nb = std::max(1, ((1 << (nq - 1)) + kPairBlock - 1) / kPairBlock);
    if (dtype == GOCP_C64)
        hipLaunchKernelGGL(k_layer_fwd<float2>, dim3(nb), dim3(kPairBlock), 0, s, in, out, pop, pterm, j, ns, x, nq);
    else
        hipLaunchKernelGGL(k_layer_fwd<double2>, dim3(nb), dim3(kPairBlock), 0, s, in, out, pop, pterm, j, ns, x, nq);
    hip_check(hipGetLastError(), "kernel launch");
}

void launch_layer_adj(int dtype, const void *phi, double2 *lam, double *partial, const HClass *pop,
                      const HTerm *pterm, int j, int ns, double x, int nq, const double2 *sigma, const void *psi,
                      const AdaptState *st, hipStream_t s) {
    const int nb = std::max(1, ((1 << (nq - 1)) + kPairBlock - 1) / kPairBlock);
    if (dtype == GOCP_C64)
        hipLaunchKernelGGL(k_layer_adj<float2>, dim3(nb), dim3(kPairBlock), 0, s, phi, lam, partial, pop, pterm, j,
                           ns, x, nq, sigma, psi, st);
    else
        hipLaunchKernelGGL(k_layer_adj<double2>, dim3(nb), dim3(kPairBlock), 0, s, phi, lam, partial, pop, pterm,
                           j, ns, x, nq, sigma, psi, st);
    hip_check(hipGetLastError(), "kernel launch");
}

void launch_gather_done(const InstDev *insts, int n, int32_t *out, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_gather_done, dim3((n + 255) / 256), dim3(256), 0, s, insts, n, out);
    hip_check(hipGetLastError(), "kernel launch");
}

// Per block: the weight of the block's amplitudes inside the sector (decoded
// occupation with ne electrons, as many in even as in odd spin-orbitals) and
// their total weight, into part[2 block], part[2 block + 1].
template <typename T>
__global__ __launch_bounds__(256) void k_sector_weight(const void *psi, uint32_t dim, SectorRows rows, double *part) {
    double in = 0.0, all = 0.0;
    for (uint32_t d = blockIdx.x * 256 + threadIdx.x; d < dim; d += gridDim.x * 256) {
        uint32_t occ = 0;
        for (int j = 0; j < rows.n; ++j) occ |= (uint32_t)(__popc(rows.r[j] & d) & 1) << j;
        const double2 a = Amp<T>::load(psi, d);
        const double w = a.x * a.x + a.y * a.y;
        all += w;
        const int ne = __popc(occ), nu = __popc(occ & 0x55555555u);
        if (ne == rows.ne && 2 * nu == ne) in += w;
    }
    __shared__ double r[2][256 / kWave];
    in = wave_sum(in);
    all = wave_sum(all);
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & (kWave - 1);
    if (lane == 0) {
        r[0][wv] = in;
        r[1][wv] = all;
    }
    __syncthreads();
    if (threadIdx.x < 2) {
        double a = 0.0;
        for (int k = 0; k < 256 / kWave; ++k) a += r[threadIdx.x][k];
        part[2 * blockIdx.x + threadIdx.x] = a;
    }
}

void launch_sector_weight(int dtype, const void *psi, uint32_t dim, const SectorRows &rows, double *part, int nblk,
                          hipStream_t s) {
    if (dtype == GOCP_C64)
        hipLaunchKernelGGL(k_sector_weight<float2>, dim3(nblk), dim3(256), 0, s, psi, dim, rows, part);
    else
        hipLaunchKernelGGL(k_sector_weight<double2>, dim3(nblk), dim3(256), 0, s, psi, dim, rows, part);
    hip_check(hipGetLastError(), "kernel launch");
}

// dst[i] = scale * src[i] for a state of dim amplitudes (FP64 product, rounded
// to the state's precision once).
template <typename T>
__global__ void k_scale_copy(const void *src, void *dst, uint32_t dim, double scale) {
    const uint32_t i = blockIdx.x * 256 + threadIdx.x;
    if (i >= dim) return;
    const double2 v = Amp<T>::load(src, i);
    Amp<T>::store(dst, i, make_double2(scale * v.x, scale * v.y));
}

void launch_scale_copy(int dtype, const void *src, void *dst, uint32_t dim, double scale, hipStream_t s) {
    const int nb = (int)((dim + 255) / 256);
    if (dtype == GOCP_C64)
        hipLaunchKernelGGL(k_scale_copy<float2>, dim3(nb), dim3(256), 0, s, src, dst, dim, scale);
    else
        hipLaunchKernelGGL(k_scale_copy<double2>, dim3(nb), dim3(256), 0, s, src, dst, dim, scale);
    hip_check(hipGetLastError(), "kernel launch");
}

void launch_basis(int dtype, void *psi, uint32_t dim, uint32_t index, hipStream_t s) {
    const int nb = (int)((dim + 255) / 256);
    if (dtype == GOCP_C64)
        hipLaunchKernelGGL(k_basis<float2>, dim3(nb), dim3(256), 0, s, psi, dim, index);
    else
        hipLaunchKernelGGL(k_basis<double2>, dim3(nb), dim3(256), 0, s, psi, dim, index);
    hip_check(hipGetLastError(), "kernel launch");
}

}  // namespace gocp
