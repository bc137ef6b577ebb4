// HIP kernels of the GOCP ADAPT-VQE hot path for gfx950 (CDNA4).
//
// All statevector work is the application of folded Pauli terms
//   (c Z^z X^x psi)[d] = c (-1)^popcount(d & z) psi[d ^ x]
// to a 2^n statevector.  Two kernel shapes carry it:
//
// * Tile kernels (energy / H apply, gradient screen, the H v / H w products of
//   the line search).  A workgroup owns 64 consecutive amplitudes, one per
//   lane, and its 16 waves split the work items (X-mask classes of H, or the
//   pool operators in GOCP family order) between them.  For one X mask the 64
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
// waves and over workgroups.  The cross-workgroup step is done by the last
// workgroup to arrive (release/acquire fences at device scope around an
// arrival counter), so a kernel and its reduction are one launch and no
// floating-point atomics are used.

#include <hip/hip_runtime.h>

#include <cmath>

#include "device.h"

namespace gocp {

// ------------------------------------------------------------------ helpers

template <typename T> struct Amp;
template <> struct Amp<double2> {
    static __device__ __forceinline__ double2 load(const void *p, uint32_t i) {
        return static_cast<const double2 *>(p)[i];
    }
    static __device__ __forceinline__ void store(void *p, uint32_t i, double2 v) {
        static_cast<double2 *>(p)[i] = v;
    }
    static __device__ __forceinline__ double2 rounded(double2 v) { return v; }
};
template <> struct Amp<float2> {
    static __device__ __forceinline__ double2 load(const void *p, uint32_t i) {
        const float2 f = static_cast<const float2 *>(p)[i];
        return make_double2((double)f.x, (double)f.y);
    }
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
__device__ __forceinline__ HTerm load_rec(const GOCP_AS4 HTerm *p, int i) {
    HTerm r;
    r.c = p[i].c;
    r.z = p[i].z;
    r.pad = 0;
    return r;
}

// c * (-1)^popcount(d & z): flip the sign bit by the parity of d & z.
__device__ __forceinline__ double signed_coef(double c, uint32_t d, uint32_t z) {
    const int flip = (int)((uint32_t)__popc(d & z) << 31);
    return __hiloint2double(__double2hiint(c) ^ flip, __double2loint(c));
}

// sum_s c_s (-1)^popcount(d & z_s) over the strings [s0, s1) of a table,
// four strings per step with two accumulators.
__device__ __forceinline__ double string_sum(const GOCP_AS4 HTerm *t, int s0, int s1, uint32_t d) {
    double f0 = 0.0, f1 = 0.0;
    int s = s0;
    for (; s + 4 <= s1; s += 4) {
        const HTerm a = load_rec(t, s), b = load_rec(t, s + 1), c = load_rec(t, s + 2), e = load_rec(t, s + 3);
        f0 += signed_coef(a.c, d, a.z);
        f1 += signed_coef(b.c, d, b.z);
        f0 += signed_coef(c.c, d, c.z);
        f1 += signed_coef(e.c, d, e.z);
    }
    for (; s < s1; ++s) {
        const HTerm a = load_rec(t, s);
        f0 += signed_coef(a.c, d, a.z);
    }
    return f0 + f1;
}

// The same sum at two amplitudes d and e (the two members of a pair).
__device__ __forceinline__ void string_sum2(const GOCP_AS4 HTerm *t, int s0, int s1, uint32_t d,
                                            uint32_t e, double &hd, double &he) {
    hd = 0.0;
    he = 0.0;
    for (int s = s0; s < s1; ++s) {
        const HTerm a = load_rec(t, s);
        hd += signed_coef(a.c, d, a.z);
        he += signed_coef(a.c, e, a.z);
    }
}

__device__ __forceinline__ int state_done(const AdaptState *st) { return cptr(&st->done)[0]; }

// Sum over a wave with an xor butterfly: every lane ends with the same value.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

__device__ __forceinline__ int wave_id() {
    return __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
}

// Sum of `n` values at stride `stride` from `src`, in index order per thread
// and a fixed tree over threads; the result is returned to every thread.
template <int NT>
__device__ double block_sum_strided(const double *src, int n, int stride, double *lds) {
    double acc = 0.0;
    for (int i = threadIdx.x; i < n; i += NT) acc += src[(size_t)i * stride];
    lds[threadIdx.x] = acc;
    __syncthreads();
#pragma unroll
    for (int h = NT / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) lds[threadIdx.x] += lds[threadIdx.x + h];
        __syncthreads();
    }
    const double r = lds[0];
    __syncthreads();
    return r;
}

// Arrival of this workgroup at the end of its part of a launch.  Returns true
// (in every thread) in the workgroup that arrives last; that workgroup then
// sees every partial written before the other workgroups arrived.
__device__ bool arrive_last(int32_t *counter, int total) {
    __shared__ int s_last;
    __threadfence();                 // release this workgroup's partial writes
    __syncthreads();
    if (threadIdx.x == 0) {
        const int prev = atomicAdd(counter, 1);
        s_last = (prev == total - 1);
        if (s_last) {
            __threadfence();         // acquire the other workgroups' writes
            *counter = 0;            // ready for the next launch
        }
    }
    __syncthreads();
    if (s_last) __threadfence();
    return s_last != 0;
}

__device__ __forceinline__ uint32_t insert_zero_bit(uint32_t p, int hb) {
    const uint32_t lo = p & ((1u << hb) - 1u);
    return ((p >> hb) << (hb + 1)) | lo;
}

// ------------------------------------------------------------------ K1: sigma = H psi, energy

// mode: 0 one-shot (energy to st), 1 initial state of an ADAPT run (E_0),
//       2 end of an ADAPT iteration (E_{k+1}, iteration counter).
template <typename T>
__global__ __launch_bounds__(kNW *kWave) void k_apply_h(const InstDev *__restrict__ insts,
                                                       const int2 *__restrict__ blk, int mode) {
    const int2 b = blk[blockIdx.x];
    const InstDev &I = insts[b.x];
    AdaptState *st = I.st;
    if (mode != 0 && state_done(st)) return;
    const int lane = threadIdx.x & (kWave - 1);
    const int wv = wave_id();
    const uint32_t dim = 1u << I.n_qubits;
    const uint32_t d = (uint32_t)b.y * kTile + lane;
    const bool valid = d < dim;
    const uint32_t dd = valid ? d : 0u;

    double sr = 0.0, si = 0.0;
    const GOCP_AS4 HClass *cls = cptr(I.hcls);
    const GOCP_AS4 HTerm *trm = cptr(I.hterm);
    const int c0 = cptr(I.cls_split)[wv], c1 = cptr(I.cls_split)[wv + 1];
    for (int c = c0; c < c1; ++c) {
        const HClass C = load_rec(cls, c);
        const double f = string_sum(trm, C.s0, C.s1, dd);
        const double2 p = Amp<T>::load(I.psi, dd ^ C.x);
        sr = fma(f, p.x, sr);
        si = fma(f, p.y, si);
    }
    __shared__ double2 red[kNW][kWave];
    __shared__ double lds[kNW * kWave];
    red[wv][lane] = make_double2(sr, si);
    __syncthreads();
    if (wv == 0) {
        double ar = 0.0, ai = 0.0;
#pragma unroll
        for (int k = 0; k < kNW; ++k) {
            ar += red[k][lane].x;
            ai += red[k][lane].y;
        }
        const double2 own = Amp<T>::load(I.psi, dd);
        double pe = valid ? own.x * ar + own.y * ai : 0.0;
        double pn = valid ? own.x * own.x + own.y * own.y : 0.0;
        if (valid) I.sigma[d] = make_double2(ar, ai);
        pe = wave_sum(pe);
        pn = wave_sum(pn);
        if (lane == 0) {
            I.part_e[b.y] = pe;
            I.part_n[b.y] = pn;
        }
    }
    if (!arrive_last(&I.counters[0], I.n_tiles)) return;
    const double e_num = block_sum_strided<kNW * kWave>(I.part_e, I.n_tiles, 1, lds);
    const double nrm = block_sum_strided<kNW * kWave>(I.part_n, I.n_tiles, 1, lds);
    if (threadIdx.x == 0) {
        const double e = e_num / nrm;
        st->e_num = e_num;
        st->nrm = nrm;
        st->energy = e;
        if (!(nrm > 0.0) || !isfinite(e)) {
            st->status = GOCP_ENUMERIC;
            st->done = 1;
        }
        if (mode == 1) {
            if (st->hist_e) st->hist_e[0] = e;
            if (st->max_iter <= 0) st->done = 1;
        } else if (mode == 2) {
            const int it = st->iter + 1;
            if (st->hist_e) st->hist_e[it] = e;
            st->iter = it;
            if (it >= st->max_iter) st->done = 1;
        }
    }
}

// ------------------------------------------------------------------ K2: gradient screen + selection

// g_j = 2 Re <sigma | A_j psi> / <psi|psi> for every j, then (last workgroup)
// |g|max, ||g||_2 and the selected operator.
template <typename T>
__global__ __launch_bounds__(kNW *kWave) void k_pool_grad(const InstDev *__restrict__ insts,
                                                         const int2 *__restrict__ blk, int mode) {
    const int2 b = blk[blockIdx.x];
    const InstDev &I = insts[b.x];
    AdaptState *st = I.st;
    if (mode != 0 && state_done(st)) return;
    const int lane = threadIdx.x & (kWave - 1);
    const int wv = wave_id();
    const uint32_t dim = 1u << I.n_qubits;
    const uint32_t d = (uint32_t)b.y * kTile + lane;
    const bool valid = d < dim;
    const uint32_t dd = valid ? d : 0u;
    const int M = I.M;
    const double2 sg = valid ? I.sigma[dd] : make_double2(0.0, 0.0);

    const GOCP_AS4 HClass *ops = cptr(I.pop);
    const GOCP_AS4 HTerm *trm = cptr(I.pterm);
    const GOCP_AS4 int32_t *sched = cptr(I.op_sched);
    const int o0 = cptr(I.op_split)[wv], o1 = cptr(I.op_split)[wv + 1];
    for (int o = o0; o < o1; ++o) {
        const int j = sched[o];
        const HClass C = load_rec(ops, j);
        const double h = string_sum(trm, C.s0, C.s1, dd);
        const double2 p = Amp<T>::load(I.psi, dd ^ C.x);
        double val = h * (sg.x * p.x + sg.y * p.y);
        val = wave_sum(val);
        if (lane == 0) I.part_g[(size_t)b.y * M + j] = val;
    }
    if (!arrive_last(&I.counters[1], I.n_tiles)) return;

    __shared__ double lds[kNW * kWave];
    __shared__ int ldsi[kNW * kWave];
    constexpr int NT = kNW * kWave;
    const double inv = 2.0 / st->nrm;
    double amax = 0.0, sq = 0.0;
    for (int j = threadIdx.x; j < M; j += NT) {
        double acc = 0.0;
        for (int t = 0; t < I.n_tiles; ++t) acc += I.part_g[(size_t)t * M + j];
        const double g = acc * inv;
        st->g[j] = g;
        amax = fmax(amax, fabs(g));
        sq += g * g;
    }
    // max |g| (exact, order-free) and sum of squares (fixed tree)
    lds[threadIdx.x] = amax;
    __syncthreads();
    for (int h = NT / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) lds[threadIdx.x] = fmax(lds[threadIdx.x], lds[threadIdx.x + h]);
        __syncthreads();
    }
    const double gmax = lds[0];
    __syncthreads();
    lds[threadIdx.x] = sq;
    __syncthreads();
    for (int h = NT / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) lds[threadIdx.x] += lds[threadIdx.x + h];
        __syncthreads();
    }
    const double gn = sqrt(lds[0]);
    __syncthreads();
    // lowest index within the tie band of the largest magnitude
    const double thresh = gmax * (1.0 - 1e-12);
    int jmin = 0x7fffffff;
    for (int j = threadIdx.x; j < M; j += NT)
        if (fabs(st->g[j]) >= thresh) {
            jmin = j;
            break;
        }
    ldsi[threadIdx.x] = jmin;
    __syncthreads();
    for (int h = NT / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) ldsi[threadIdx.x] = min(ldsi[threadIdx.x], ldsi[threadIdx.x + h]);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        st->gmax = gmax;
        st->gnorm = gn;
        st->jsel = ldsi[0] < M ? ldsi[0] : 0;
        if (!isfinite(gn)) {
            st->status = GOCP_ENUMERIC;
            st->done = 1;
        }
        if (mode != 0) {
            const int it = st->iter;
            if (st->hist_gnorm) st->hist_gnorm[it] = gn;
            if (st->hist_gmax) st->hist_gmax[it] = gmax;
            if (gn < st->grad_tol) {
                st->converged = 1;
                st->done = 1;
            }
        }
    }
}

// ------------------------------------------------------------------ line search vectors

// w = A psi and v = -A w on the pairs of the selected generator, and the
// partial dot products Re<v|sigma>, Re<sigma|w>.
template <typename T>
__global__ __launch_bounds__(kPairBlock) void k_line_vw(const InstDev *__restrict__ insts,
                                                       const int2 *__restrict__ blk) {
    const int2 b = blk[blockIdx.x];
    const InstDev &I = insts[b.x];
    AdaptState *st = I.st;
    if (state_done(st)) return;
    const int j = cptr(&st->jsel)[0];
    const HClass C = load_rec(cptr(I.pop), j);
    const uint32_t m = C.x;
    const int hb = 31 - __clz(m);
    const uint32_t half = 1u << (I.n_qubits - 1);
    const uint32_t p = (uint32_t)b.y * kPairBlock + threadIdx.x;
    double p2 = 0.0, p7 = 0.0;
    if (p < half) {
        const uint32_t d = insert_zero_bit(p, hb), e = d ^ m;
        double hd, he;
        string_sum2(cptr(I.pterm), C.s0, C.s1, d, e, hd, he);
        const double2 a = Amp<T>::load(I.psi, d), c = Amp<T>::load(I.psi, e);
        const double2 wd = make_double2(hd * c.x, hd * c.y);
        const double2 we = make_double2(he * a.x, he * a.y);
        const double hh = -hd * he;
        const double2 vd = make_double2(hh * a.x, hh * a.y);
        const double2 ve = make_double2(hh * c.x, hh * c.y);
        Amp<T>::store(I.w, d, wd);
        Amp<T>::store(I.w, e, we);
        Amp<T>::store(I.v, d, vd);
        Amp<T>::store(I.v, e, ve);
        const double2 sd = I.sigma[d], se = I.sigma[e];
        p2 = vd.x * sd.x + vd.y * sd.y + ve.x * se.x + ve.y * se.y;
        p7 = sd.x * wd.x + sd.y * wd.y + se.x * we.x + se.y * we.y;
    }
    __shared__ double r2[kPairBlock / kWave], r7[kPairBlock / kWave];
    p2 = wave_sum(p2);
    p7 = wave_sum(p7);
    const int wv = wave_id(), lane = threadIdx.x & (kWave - 1);
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
        I.part_l[3 * I.n_tiles + 2 * b.y] = a2;
        I.part_l[3 * I.n_tiles + 2 * b.y + 1] = a7;
    }
}

// E(theta) = a_uu + 2 a_uv cos + 2 a_uw sin + a_vv cos^2 + 2 a_vw sin cos + a_ww sin^2
struct Landscape {
    double uu, uv, uw, vv, vw, ww;
    __device__ double value(double th) const {
        double s, c;
        sincos(th, &s, &c);
        return uu + 2.0 * uv * c + 2.0 * uw * s + vv * c * c + 2.0 * vw * s * c + ww * s * s;
    }
    __device__ double deriv(double th) const {
        double s, c;
        sincos(th, &s, &c);
        return -2.0 * uv * s + 2.0 * uw * c - 2.0 * vv * s * c + 2.0 * vw * (c * c - s * s) +
               2.0 * ww * s * c;
    }
};

// First local minimum of E from 0 in the descent direction -sign(g), found by
// one wave: 1-degree steps (64 at a time) until d E' >= 0, then the bracket is
// cut into 64 parts per round until it stops shrinking.  Without a sign
// change within a full turn, the best sampled angle.  Called by all 64 lanes
// of one wave; returns the angle in every lane.
__device__ double line_search_wave(const Landscape &L, double g) {
    if (g == 0.0) return 0.0;
    const int lane = threadIdx.x & (kWave - 1);
    const double dir = g > 0.0 ? -1.0 : 1.0;
    const double step = M_PI / 180.0;
    int kfirst = 0;
    for (int base = 0; base < 360 && kfirst == 0; base += kWave) {
        const int k = base + lane + 1;
        const bool hit = k <= 360 && dir * L.deriv(dir * k * step) >= 0.0;
        const unsigned long long mask = __ballot(hit);
        if (mask) kfirst = base + __ffsll((long long)mask);
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
        return dir * bestk * step;
    }
    double lo = dir * (kfirst - 1) * step, hi = dir * kfirst * step;
    for (int round = 0; round < 16; ++round) {
        const double t = lo + (hi - lo) * (double)(lane + 1) / (double)kWave;
        const bool hit = lane < kWave - 1 && dir * L.deriv(t) >= 0.0;
        const unsigned long long mask = __ballot(hit);
        double nlo, nhi;
        if (mask) {
            const int l = __ffsll((long long)mask) - 1;
            nhi = lo + (hi - lo) * (double)(l + 1) / (double)kWave;
            nlo = l == 0 ? lo : lo + (hi - lo) * (double)l / (double)kWave;
        } else {
            nlo = lo + (hi - lo) * (double)(kWave - 1) / (double)kWave;
            nhi = hi;
        }
        if (nlo == lo && nhi == hi) break;
        lo = nlo;
        hi = nhi;
    }
    return 0.5 * (lo + hi);
}

// H v, H w with shared class coefficients; partial Re<v|Hv>, Re<w|Hw>,
// Re<v|Hw>; the last workgroup forms the landscape and picks the angle.
template <typename T>
__global__ __launch_bounds__(kNW *kWave) void k_line_hvw(const InstDev *__restrict__ insts,
                                                        const int2 *__restrict__ blk) {
    const int2 b = blk[blockIdx.x];
    const InstDev &I = insts[b.x];
    AdaptState *st = I.st;
    if (state_done(st)) return;
    const int lane = threadIdx.x & (kWave - 1);
    const int wv = wave_id();
    const uint32_t dim = 1u << I.n_qubits;
    const uint32_t d = (uint32_t)b.y * kTile + lane;
    const bool valid = d < dim;
    const uint32_t dd = valid ? d : 0u;

    double vr = 0.0, vi = 0.0, wr = 0.0, wi = 0.0;
    const GOCP_AS4 HClass *cls = cptr(I.hcls);
    const GOCP_AS4 HTerm *trm = cptr(I.hterm);
    const int c0 = cptr(I.cls_split)[wv], c1 = cptr(I.cls_split)[wv + 1];
    for (int c = c0; c < c1; ++c) {
        const HClass C = load_rec(cls, c);
        const double f = string_sum(trm, C.s0, C.s1, dd);
        const double2 pv = Amp<T>::load(I.v, dd ^ C.x);
        const double2 pw = Amp<T>::load(I.w, dd ^ C.x);
        vr = fma(f, pv.x, vr);
        vi = fma(f, pv.y, vi);
        wr = fma(f, pw.x, wr);
        wi = fma(f, pw.y, wi);
    }
    __shared__ double4 red[kNW][kWave];
    __shared__ double lds[kNW * kWave];
    red[wv][lane] = make_double4(vr, vi, wr, wi);
    __syncthreads();
    if (wv == 0) {
        double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
#pragma unroll
        for (int k = 0; k < kNW; ++k) {
            const double4 r = red[k][lane];
            a0 += r.x;
            a1 += r.y;
            a2 += r.z;
            a3 += r.w;
        }
        const double2 ov = Amp<T>::load(I.v, dd), ow = Amp<T>::load(I.w, dd);
        double p3 = valid ? ov.x * a0 + ov.y * a1 : 0.0;
        double p5 = valid ? ow.x * a2 + ow.y * a3 : 0.0;
        double p6 = valid ? ov.x * a2 + ov.y * a3 : 0.0;
        p3 = wave_sum(p3);
        p5 = wave_sum(p5);
        p6 = wave_sum(p6);
        if (lane == 0) {
            I.part_l[3 * b.y] = p3;
            I.part_l[3 * b.y + 1] = p5;
            I.part_l[3 * b.y + 2] = p6;
        }
    }
    if (!arrive_last(&I.counters[2], I.n_tiles)) return;
    constexpr int NT = kNW * kWave;
    const double P3 = block_sum_strided<NT>(I.part_l, I.n_tiles, 3, lds);
    const double P5 = block_sum_strided<NT>(I.part_l + 1, I.n_tiles, 3, lds);
    const double P6 = block_sum_strided<NT>(I.part_l + 2, I.n_tiles, 3, lds);
    const double P2 = block_sum_strided<NT>(I.part_l + 3 * I.n_tiles, I.n_pblk, 2, lds);
    const double P7 = block_sum_strided<NT>(I.part_l + 3 * I.n_tiles + 1, I.n_pblk, 2, lds);
    if (wv != 0) return;
    const double inv = 1.0 / st->nrm;
    Landscape L;
    L.uu = (st->e_num - 2.0 * P2 + P3) * inv;
    L.uv = (P2 - P3) * inv;
    L.uw = (P7 - P6) * inv;
    L.vv = P3 * inv;
    L.vw = P6 * inv;
    L.ww = P5 * inv;
    const int j = st->jsel;
    const double th = line_search_wave(L, st->g[j]);
    if (lane == 0) {
        const int ns = th == 0.0 ? 0 : max(1, (int)ceil(fabs(th) * I.op_norm1[j] / 0.5));
        st->theta = th;
        st->nsub = ns;
        st->pred = L.value(th);
        const int it = st->iter;
        if (st->hist_op) st->hist_op[it] = j;
        if (st->hist_theta) st->hist_theta[it] = th;
        if (st->hist_nsub) st->hist_nsub[it] = ns;
        if (st->hist_pred) st->hist_pred[it] = st->pred;
    }
}

// ------------------------------------------------------------------ K3: O(5) Taylor update

// psi <- T5(theta/s)^s (scale * psi) on the pairs of generator j.  In an ADAPT
// iteration (adapt != 0) j, theta, s come from the device state and scale is
// 1/sqrt(<psi|psi>) of the stored state (the renormalisation of the previous
// update, applied here); one-shot calls pass them as arguments.  Writes the
// per-workgroup |psi|^2 of the result to part_t.
template <typename T>
__global__ __launch_bounds__(kPairBlock) void k_taylor5(const InstDev *__restrict__ insts,
                                                       const int2 *__restrict__ blk, int adapt,
                                                       int j_arg, double theta_arg, int s_arg) {
    const int2 b = blk[blockIdx.x];
    const InstDev &I = insts[b.x];
    AdaptState *st = I.st;
    if (adapt && state_done(st)) return;
    const int j = adapt ? cptr(&st->jsel)[0] : j_arg;
    const double theta = adapt ? cptr(&st->theta)[0] : theta_arg;
    const int ns = adapt ? cptr(&st->nsub)[0] : s_arg;
    const double scale = adapt ? 1.0 / sqrt(cptr(&st->nrm)[0]) : 1.0;
    const HClass C = load_rec(cptr(I.pop), j);
    const uint32_t m = C.x;
    const int hb = 31 - __clz(m);
    const uint32_t half = 1u << (I.n_qubits - 1);
    const uint32_t p = (uint32_t)b.y * kPairBlock + threadIdx.x;
    double nn = 0.0;
    if (p < half) {
        const uint32_t d = insert_zero_bit(p, hb), e = d ^ m;
        double hd, he;
        string_sum2(cptr(I.pterm), C.s0, C.s1, d, e, hd, he);
        double2 a = Amp<T>::load(I.psi, d), c = Amp<T>::load(I.psi, e);
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

// psi *= 1 / sqrt(sum of part_t)   (from_state: 1 / sqrt(st->nrm) instead)
template <typename T>
__global__ __launch_bounds__(kPairBlock) void k_normalize(const InstDev *__restrict__ insts,
                                                         const int2 *__restrict__ blk,
                                                         int from_state) {
    const int2 b = blk[blockIdx.x];
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
    if (b.y == 0 && threadIdx.x == 0 && !from_state) I.st->nrm = 1.0;
}

// psi = |index>
template <typename T>
__global__ void k_basis(void *psi, uint32_t dim, uint32_t index) {
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < dim) Amp<T>::store(psi, k, make_double2(k == index ? 1.0 : 0.0, 0.0));
}

// ------------------------------------------------------------------ launchers

template <typename T>
static void launch_all(int which, const InstDev *insts, const int2 *blk, int nblk, int mode,
                       hipStream_t s, int j = 0, double th = 0.0, int ns = 0) {
    switch (which) {
    case 0: hipLaunchKernelGGL(k_apply_h<T>, dim3(nblk), dim3(kNW * kWave), 0, s, insts, blk, mode); break;
    case 1: hipLaunchKernelGGL(k_pool_grad<T>, dim3(nblk), dim3(kNW * kWave), 0, s, insts, blk, mode); break;
    case 2: hipLaunchKernelGGL(k_line_vw<T>, dim3(nblk), dim3(kPairBlock), 0, s, insts, blk); break;
    case 3: hipLaunchKernelGGL(k_line_hvw<T>, dim3(nblk), dim3(kNW * kWave), 0, s, insts, blk); break;
    case 4: hipLaunchKernelGGL(k_taylor5<T>, dim3(nblk), dim3(kPairBlock), 0, s, insts, blk, mode, j, th, ns); break;
    case 5: hipLaunchKernelGGL(k_normalize<T>, dim3(nblk), dim3(kPairBlock), 0, s, insts, blk, mode); break;
    default: break;
    }
}

void launch_kernel(int which, int dtype, const InstDev *insts, const int2 *blk, int nblk, int mode,
                   hipStream_t s, int j, double th, int ns) {
    if (nblk <= 0) return;
    if (dtype == GOCP_C64)
        launch_all<float2>(which, insts, blk, nblk, mode, s, j, th, ns);
    else
        launch_all<double2>(which, insts, blk, nblk, mode, s, j, th, ns);
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
