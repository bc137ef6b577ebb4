// Device runtime of libgocp: contexts, device copies of the term tables,
// per-call workspaces, and the device C ABI entry points.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "runtime.h"

// Workspace of the allocation-free gradient screen (pool_gradients_noalloc):
// one fixed array per device, held until the process ends.  Host code never
// passes `scratch` itself to a kernel or a copy: it is a host-side stand-in.
// The device address is looked up once per device (hipGetSymbolAddress, at
// context creation) and only that address is used.
static constexpr size_t kNoAllocScratchBytes = (size_t)8 << 20;
static __device__ __align__(256) char scratch[kNoAllocScratchBytes];

namespace gocp {


void hip_check(hipError_t e, const char *what) {
    if (e != hipSuccess)
        throw Error(e == hipErrorOutOfMemory ? GOCP_ENOMEM : GOCP_EDEVICE,
                    std::string(what) + ": " + hipGetErrorString(e));
}

namespace {

// Lays the arrays of one handle's device tables out in one buffer, each at a
// 256-byte aligned offset; add() returns the offset in the pointer's type
// (rebased onto a device address by place_*).
struct ImagePacker {
    std::vector<std::pair<size_t, std::vector<char>>> parts;
    size_t used = 0;
    template <typename T>
    T *add(const std::vector<T> &v) {
        const size_t off = (used + 255) & ~(size_t)255;
        std::vector<char> b(std::max<size_t>(1, v.size()) * sizeof(T), 0);
        if (!v.empty()) std::memcpy(b.data(), v.data(), v.size() * sizeof(T));
        used = off + b.size();
        parts.emplace_back(off, std::move(b));
        return reinterpret_cast<T *>(off);
    }
    void finish(TableImage &im) {
        im.bytes = (used + 255) & ~(size_t)255;
        hip_check(hipHostMalloc(reinterpret_cast<void **>(&im.host), im.bytes, 0), "hipHostMalloc table image");
        std::memset(im.host, 0, im.bytes);
        for (const auto &pr : parts) std::memcpy(im.host + pr.first, pr.second.data(), pr.second.size());
    }
};

template <typename T>
void rebase(T *&p, char *base) {
    p = reinterpret_cast<T *>(base + reinterpret_cast<uintptr_t>(p));
}

HTerm make_term(double c, uint32_t z) { return HTerm{std::fabs(c), z, std::signbit(c) ? 1u : 0u}; }

uint32_t sub_key(uint32_t z) { return ((z >> 6) & 1u) << 2 | ((z >> 7) & 1u) << 1 | ((z >> 8) & 1u); }

// Append the strings [a, b) of (c, z) in sub-bucket order to the magnitude
// and Z-mask-with-sign arrays, then zero strings up to a whole number of
// groups of kStrGroup, and return the sub-bucket record of the group (the
// padding sits after the last sub-bucket).
HSub bucket_strings(const std::vector<double> &c, const std::vector<uint32_t> &z, int a, int b,
                    std::vector<double> &co, std::vector<uint32_t> &zs) {
    std::vector<int> idx;
    for (int s = a; s < b; ++s) idx.push_back(s);
    std::stable_sort(idx.begin(), idx.end(), [&](int p, int q) { return sub_key(z[p]) < sub_key(z[q]); });
    if (b - a > 65535) throw Error(GOCP_ENOTSUP, "a class has more than 65535 strings");
    uint16_t off[8];
    int k = 0;
    for (int key = 0; key < 8; ++key) {
        off[key] = (uint16_t)k;
        while (k < (int)idx.size() && (int)sub_key(z[idx[k]]) == key) ++k;
    }
    const size_t start = co.size();
    for (int s : idx) {
        if (z[s] >> 31) throw Error(GOCP_ENOTSUP, "Z mask beyond 31 qubits");
        co.push_back(std::fabs(c[s]));
        zs.push_back(z[s] | (std::signbit(c[s]) ? 1u << 31 : 0u));
    }
    while ((co.size() - start) % kStrGroup) {
        co.push_back(0.0);
        zs.push_back(0u);
    }
    HSub r;
    for (int i = 0; i < 4; ++i) r.w[i] = (uint32_t)off[2 * i] | ((uint32_t)off[2 * i + 1] << 16);
    return r;
}

// Boundaries of consecutive record groups (classes or operators) such that
// each group has at most kStageCls records and kStageTerms strings.
std::vector<int32_t> stage_chunks(const std::vector<int32_t> &off) {
    std::vector<int32_t> b{0};
    const int n = (int)off.size() - 1;
    int start = 0;
    for (int i = 0; i < n; ++i) {
        if (off[i + 1] - off[i] > kStageTerms)
            throw Error(GOCP_ENOTSUP, "a class or operator has more strings than one LDS stage holds");
        if (i + 1 - start > kStageCls || off[i + 1] - off[start] > kStageTerms) {
            b.push_back(i);
            start = i;
        }
    }
    if (b.back() != n) b.push_back(n);
    return b;
}

// Estimated VALU instructions of one class or operator in a tile kernel: a
// fixed cost per record (gather, conversion, multiply-add; for the screen also
// the wave reduction) plus four per string of its padded group.
int record_cost(int n_strings, int fixed) {
    return fixed + 4 * ((n_strings + kStrGroup - 1) / kStrGroup * kStrGroup);
}

// Order the records [b, e) of one LDS stage chunk for the kNW waves of a tile
// block: each record, most expensive first (ties by position), goes to the
// wave with the least work so far (lowest wave on ties); every wave keeps its
// records in their original relative order.  Appends the records to `order`
// and the kNW + 1 wave boundaries (positions in `order`) to `seg`.
void wave_split(const std::vector<int> &cost, int b, int e, std::vector<int32_t> &order,
                std::vector<int32_t> &seg) {
    std::vector<int> idx;
    for (int i = b; i < e; ++i) idx.push_back(i);
    std::stable_sort(idx.begin(), idx.end(), [&](int u, int v) { return cost[u] > cost[v]; });
    std::vector<std::vector<int>> lists(kNW);
    std::vector<long long> load(kNW, 0);
    for (int i : idx) {
        int w = 0;
        for (int k = 1; k < kNW; ++k)
            if (load[k] < load[w]) w = k;
        lists[w].push_back(i);
        load[w] += cost[i];
    }
    for (int w = 0; w < kNW; ++w) {
        std::sort(lists[w].begin(), lists[w].end());
        seg.push_back((int32_t)order.size());
        for (int i : lists[w]) order.push_back(i);
    }
    seg.push_back((int32_t)order.size());
}

// Cut the records order[a, b) of one wave into `parts` contiguous runs whose
// largest cost is as small as possible (binary search on that cost with
// greedy packing); appends the run starts a = b_0 <= ... <= b_{parts-1}.
void cut_runs(const std::vector<int> &cost, const std::vector<int32_t> &order, int a, int b, int parts,
              std::vector<int32_t> &out) {
    long long lo = 0, hi = 0;
    for (int i = a; i < b; ++i) {
        lo = std::max<long long>(lo, cost[order[i]]);
        hi += cost[order[i]];
    }
    auto pack = [&](long long cap, std::vector<int32_t> *cuts) {
        int runs = 1;
        long long cur = 0;
        if (cuts) cuts->push_back(a);
        for (int i = a; i < b; ++i) {
            const int c = cost[order[i]];
            if (cur + c > cap) {
                ++runs;
                cur = 0;
                if (cuts) cuts->push_back(i);
            }
            cur += c;
        }
        return runs;
    };
    while (lo < hi) {
        const long long mid = (lo + hi) / 2;
        if (pack(mid, nullptr) <= parts) hi = mid; else lo = mid + 1;
    }
    std::vector<int32_t> cuts;
    pack(lo, &cuts);
    while ((int)cuts.size() < parts) cuts.push_back(b);
    for (int k = 0; k < parts; ++k) out.push_back(cuts[k]);
}

// Per LDS stage chunk (record boundaries b): its record range and the string
// range of those records in the laid-out table.
std::vector<int4> stage_bounds(const std::vector<int32_t> &b, const std::vector<HClass> &recs) {
    std::vector<int4> out;
    for (size_t k = 0; k + 1 < b.size(); ++k)
        out.push_back(make_int4(b[k], b[k + 1], recs[b[k]].s0, recs[b[k + 1] - 1].s1));
    return out;
}

// H's class of exactly four strings whose Z masks form an affine set z0 +
// {0, u, v, u + v} (three nonzero offsets, each the XOR of the other two)
// with coefficients c, c (-1)^alpha, c (-1)^beta, c (-1)^(alpha + beta):
// f(d) = 4 c (-1)^popcount(d & z0) [popcount(d & u) = alpha mod 2]
// [popcount(d & v) = beta mod 2], since each of the two sums over a factor of
// the set is 2 or 0.  Fills the group {|4c|, 0, 0, 0 | z0 | sign(c) << 31,
// u | alpha << 31, v | beta << 31, 0}: with d | 1 << 31, the three popcounts
// give the sign and the two conditions (both even).
bool factor_class(const std::vector<double> &c, const std::vector<uint32_t> &z, int a, int b,
                  double (&co)[kStrGroup], uint32_t (&zs)[kStrGroup]) {
    if (b - a != 4) return false;
    const uint32_t z0 = z[a], u = z[a + 1] ^ z0, v = z[a + 2] ^ z0;
    const double c0 = c[a], cu = c[a + 1], cv = c[a + 2], cuv = c[a + 3];
    if (c0 == 0.0 || u == 0 || v == 0 || u == v || (z[a + 3] ^ z0) != (u ^ v) || ((u | v | z0) >> 31)) return false;
    if (std::fabs(cu) != std::fabs(c0) || std::fabs(cv) != std::fabs(c0) || std::fabs(cuv) != std::fabs(c0))
        return false;
    const uint32_t alpha = (cu < 0) != (c0 < 0), beta = (cv < 0) != (c0 < 0);
    if (((cuv < 0) != (c0 < 0)) != ((alpha ^ beta) != 0)) return false;
    co[0] = std::fabs(4.0 * c0);
    co[1] = co[2] = co[3] = 0.0;
    zs[0] = z0 | (c0 < 0 ? 1u << 31 : 0u);
    zs[1] = u | (alpha << 31);
    zs[2] = v | (beta << 31);
    zs[3] = 0u;
    return true;
}

// Operator j as f(d) = (-1)^popcount(d & zb) F(d & bm): its strings' Z masks
// agree outside bm (at most kFactBits bits), F(u) = sum_s c_s
// (-1)^popcount(u & z_s) over the submasks u of bm, and F is nonzero at one
// or two patterns (a single string: bm = 0, one pattern).  Fills the parameter group {v1, v2, 0, 0 | zb, bm, t1, t2}
// (t2 = all ones, never matched, when there is one pattern).
bool factor_op(const Pool &p, int j, double (&co)[kStrGroup], uint32_t (&zs)[kStrGroup]) {
    const int a = p.op_off[j], b = p.op_off[j + 1];
    if (b <= a) return false;
    const uint32_t z0 = p.str_z[a];
    uint32_t bm = 0;
    double scale = 0.0;
    for (int s = a; s < b; ++s) {
        bm |= p.str_z[s] ^ z0;
        scale += std::fabs(p.str_c[s]);
    }
    if (__builtin_popcount(bm) > kFactBits || (bm & kFactBit)) return false;
    // F is taken as zero only where the sum is exactly zero (the coefficients
    // of the fermionic pools are dyadic, so their cancellations are exact); a
    // pattern whose sum merely nearly cancels keeps the operator's strings
    std::vector<std::pair<uint32_t, double>> nz;
    for (uint32_t u = bm;; u = (u - 1) & bm) {
        double f = 0.0;
        for (int s = a; s < b; ++s) f += (__builtin_popcount(u & p.str_z[s]) & 1) ? -p.str_c[s] : p.str_c[s];
        if (f != 0.0) {
            if (std::fabs(f) < 1e-12 * scale) return false;
            nz.emplace_back(u, f);
        }
        if (u == 0) break;
    }
    if (nz.empty() || nz.size() > 2) return false;
    co[0] = nz[0].second;
    co[1] = nz.size() > 1 ? nz[1].second : 0.0;
    co[2] = co[3] = 0.0;
    zs[0] = z0 & ~bm;
    zs[1] = bm;
    zs[2] = nz[0].first;
    zs[3] = nz.size() > 1 ? nz[1].first : 0xffffffffu;
    return true;
}

// Padded string offsets of records taken in the order `rec` with `count(r)` strings.
template <typename F>
std::vector<int32_t> padded_offsets(int n, F count) {
    std::vector<int32_t> off{0};
    for (int r = 0; r < n; ++r) {
        const int c = count(r);
        off.push_back(off.back() + (c + kStrGroup - 1) / kStrGroup * kStrGroup);
    }
    return off;
}

}  // namespace

TableImage::~TableImage() {
    if (host) (void)hipHostFree(host);
}

void release_device_ham(DeviceHam *d) {
    if (!d) return;
    (void)hipFree(d->base);
    delete d;
}

void release_device_pool(DevicePool *d) {
    if (!d) return;
    (void)hipFree(d->base);
    delete d;
}

DeviceHam place_ham(const TableImage &im, char *base, int device) {
    DeviceHam d = im.ham;
    d.device = device;
    d.base = base;
    rebase(d.hcls, base);
    rebase(d.hcoef, base);
    rebase(d.hzs, base);
    rebase(d.hsub, base);
    rebase(d.hchunk, base);
    rebase(d.hseg, base);
    rebase(d.hsegp, base);
    rebase(d.hsegp_lo, base);
    rebase(d.hcoefG, base);
    rebase(d.hzsG, base);
    rebase(d.hchunkG, base);
    rebase(d.hgx, base);
    rebase(d.hgseg, base);
    return d;
}

DevicePool place_pool(const TableImage &im, char *base, int device) {
    DevicePool d = im.pool;
    d.device = device;
    d.base = base;
    rebase(d.pop, base);
    rebase(d.pterm, base);
    rebase(d.op_norm1, base);
    rebase(d.sop, base);
    rebase(d.scoef, base);
    rebase(d.szs, base);
    rebase(d.psub, base);
    rebase(d.pchunk, base);
    rebase(d.pseg, base);
    if (d.n_xchunks > 0) {
        rebase(d.xrec, base);
        rebase(d.xcoef, base);
        rebase(d.xzs, base);
        rebase(d.xop, base);
        rebase(d.xchunk, base);
        rebase(d.xseg, base);
    }
    return d;
}

const DeviceHam *device_ham_resident(const Ham &h, int dev) {
    std::lock_guard<std::mutex> lk(h.mu);
    return (int)h.dev.size() > dev ? h.dev[dev] : nullptr;
}

const DevicePool *device_pool_resident(const Pool &p, int dev) {
    std::lock_guard<std::mutex> lk(p.mu);
    return (int)p.dev.size() > dev ? p.dev[dev] : nullptr;
}

namespace {

// The device tables of H in one pinned host image (caller holds h.mu).
const TableImage &ham_image_locked(const Ham &h) {
    if (h.img) return *h.img;
    std::shared_ptr<TableImage> im = std::make_shared<TableImage>();
    ImagePacker pk;
    DeviceHam *d = &im->ham;
    // LDS stage chunks over the classes, then within each chunk the classes
    // re-laid out wave by wave (a chunk keeps the same classes, so its string
    // total and boundaries are unchanged)
    const int nc = h.n_classes();
    auto count = [&](int c) { return h.cls_off[c + 1] - h.cls_off[c]; };
    const std::vector<int32_t> ch = stage_chunks(padded_offsets(nc, count));
    std::vector<int> cost(nc);
    for (int c = 0; c < nc; ++c) cost[c] = record_cost(count(c), kClassCost);
    // each wave's run is further cut into kHvwPartsHi (and, in a second
    // table, kHvwPartsLo) runs of nearly equal cost (the compacted H v, H w
    // launch spreads a tile's classes over workgroups)
    std::vector<int32_t> order, seg, segp, segp_lo;
    for (size_t k = 0; k + 1 < ch.size(); ++k) {
        const size_t s0 = seg.size();
        wave_split(cost, ch[k], ch[k + 1], order, seg);
        for (int w = 0; w < kNW; ++w) {
            cut_runs(cost, order, seg[s0 + w], seg[s0 + w + 1], kHvwPartsHi, segp);
            cut_runs(cost, order, seg[s0 + w], seg[s0 + w + 1], kHvwPartsLo, segp_lo);
        }
        segp.push_back(seg[s0 + kNW]);
        segp_lo.push_back(seg[s0 + kNW]);
    }
    std::vector<HClass> cls;
    std::vector<HSub> sub;
    std::vector<double> co;
    std::vector<uint32_t> zs;
    for (int32_t c : order) {
        const int32_t s0 = (int32_t)co.size();
        sub.push_back(bucket_strings(h.str_c, h.str_z, h.cls_off[c], h.cls_off[c + 1], co, zs));
        cls.push_back(HClass{h.cls_x[c], s0, (int32_t)co.size(), 0});
    }
    // The grouped walk's table (one amplitude per lane): per chunk, the
    // groups of the factored classes (factor_class: one group of parameters
    // each), then every other class's groups of strings, each kind cut into
    // kNW contiguous runs of equal length, one per wave (the walk is linear
    // in the groups, so their order and a class spanning two waves do not
    // matter); per group its class's X mask.
    // Factored classes (factor_class) keep their single group in the class
    // tables too, holding the parameters instead of the strings, and are
    // flagged kFactBit in their record (every kernel that walks classes
    // evaluates them so; the gathers shift the flag out of the X mask).
    std::vector<char> fac(cls.size(), 0);
    for (size_t i = 0; i < cls.size(); ++i) {
        const int32_t c = order[i];
        double c4[kStrGroup];
        uint32_t z4[kStrGroup];
        if (!factor_class(h.str_c, h.str_z, h.cls_off[c], h.cls_off[c + 1], c4, z4)) continue;
        fac[i] = 1;
        cls[i].x |= kFactBit;
        for (int q = 0; q < kStrGroup; ++q) {
            co[cls[i].s0 + q] = c4[q];
            zs[cls[i].s0 + q] = z4[q];
        }
    }
    std::vector<double> gco;
    std::vector<uint32_t> gzs, gx;
    std::vector<int32_t> gseg;
    std::vector<int4> gchunk;
    for (size_t k = 0; k + 1 < ch.size(); ++k) {
        const int32_t sb = (int32_t)gco.size();
        int32_t fe = sb;
        for (int kind = 0; kind < 2; ++kind) {          // factored classes, then the others
            for (int32_t i = ch[k]; i < ch[k + 1]; ++i) {
                if (fac[i] != (kind == 0)) continue;
                for (int32_t s = cls[i].s0; s < cls[i].s1; ++s) {
                    gco.push_back(co[s]);
                    gzs.push_back(zs[s]);
                    if ((s - cls[i].s0) % kStrGroup == 0) gx.push_back(cls[i].x & ~kFactBit);
                }
            }
            if (kind == 0) fe = (int32_t)gco.size();
        }
        const int32_t se = (int32_t)gco.size();
        const int32_t g0 = sb / kStrGroup, g1 = fe / kStrGroup, g2 = se / kStrGroup;
        for (int w = 0; w <= kNW; ++w) gseg.push_back(g0 + (int32_t)((int64_t)(g1 - g0) * w / kNW));
        for (int w = 0; w <= kNW; ++w) gseg.push_back(g1 + (int32_t)((int64_t)(g2 - g1) * w / kNW));
        gchunk.push_back(make_int4(sb, fe, se, 0));
    }
    // zero groups past the end: the walk's read-ahead stays in the tables
    gzs.resize(gzs.size() + (size_t)kTablePadGroups * kStrGroup, 0u);
    gx.resize(gx.size() + kTablePadGroups, 0u);
    d->hcoefG = pk.add(gco);
    d->hzsG = pk.add(gzs);
    d->hchunkG = pk.add(gchunk);
    d->hgx = pk.add(gx);
    d->hgseg = pk.add(gseg);
    d->hcls = pk.add(cls);
    d->hcoef = pk.add(co);
    d->hzs = pk.add(zs);
    d->hsub = pk.add(sub);
    d->hchunk = pk.add(stage_bounds(ch, cls));
    d->hseg = pk.add(seg);
    d->hsegp = pk.add(segp);
    d->hsegp_lo = pk.add(segp_lo);
    d->n_chunks = (int)ch.size() - 1;
    pk.finish(*im);
    h.img = im;
    return *h.img;
}

// The X-class screen of a pool whose operators are single Pauli strings: the
// operators grouped by X mask (classes in the order of their first member in
// family order, members in family order), one record {x, s0, s1, count} per
// class, its members' strings |c|, z | sign << 31 and pool indices packed
// without padding; LDS stage chunks of at most kStageCls records and
// kStageTerms - 2 kStrGroup strings, each padded to a multiple of kStrGroup
// strings, and eight zero masks after the last (the walk reads members eight
// at a time, up to seven past a record's end); records split over the waves as
// for the other tables.  Nothing is added for other pools.
void add_xclass_screen(const Pool &p, ImagePacker &pk, DevicePool *d) {
    const int m = p.n_ops();
    if (m == 0) return;
    for (int k = 0; k < m; ++k)
        if (p.op_off[k + 1] - p.op_off[k] != 1) return;
    std::vector<uint32_t> xs;
    std::vector<std::vector<int>> mem;
    std::unordered_map<uint32_t, int> where;
    for (int r = 0; r < m; ++r) {
        const int j = p.fam_members[r];
        const uint32_t x = p.op_x[j];
        const auto it = where.emplace(x, (int)xs.size()).first;
        if (it->second == (int)xs.size()) {
            xs.push_back(x);
            mem.emplace_back();
        }
        mem[it->second].push_back(j);
    }
    const int nc = (int)xs.size();
    std::vector<int32_t> ch{0};
    for (int c = 0, start = 0, strings = 0; c < nc; ++c) {
        const int n = (int)mem[c].size();
        if (n > kStageTerms - 2 * kStrGroup)
            throw Error(GOCP_ENOTSUP, "an X class has more operators than one LDS stage holds");
        if (c - start + 1 > kStageCls || strings + n > kStageTerms - 2 * kStrGroup) {
            ch.push_back(c);
            start = c;
            strings = 0;
        }
        strings += n;
    }
    ch.push_back(nc);
    // a record: a gather and its conversion, then a sign, a product and a
    // share of the row reduction per member
    std::vector<int> cost(nc);
    for (int c = 0; c < nc; ++c) cost[c] = kOpCost / 2 + 12 * (int)mem[c].size();
    std::vector<int32_t> order, seg;
    for (size_t k = 0; k + 1 < ch.size(); ++k) wave_split(cost, ch[k], ch[k + 1], order, seg);
    std::vector<HClass> rec;
    std::vector<double> co;
    std::vector<uint32_t> zs;
    std::vector<int32_t> op;
    std::vector<int4> bounds;
    for (size_t k = 0; k + 1 < ch.size(); ++k) {
        const int r0 = (int)rec.size(), s0 = (int)co.size();
        for (int i = ch[k]; i < ch[k + 1]; ++i) {
            const int c = order[i];
            HClass h{xs[c], (int32_t)co.size(), 0, (int32_t)mem[c].size()};
            for (int j : mem[c]) {
                const int s = p.op_off[j];
                if (p.str_z[s] >> 31) throw Error(GOCP_ENOTSUP, "Z mask beyond 31 qubits");
                co.push_back(std::fabs(p.str_c[s]));
                zs.push_back(p.str_z[s] | (std::signbit(p.str_c[s]) ? 1u << 31 : 0u));
                op.push_back(j);
            }
            h.s1 = (int32_t)co.size();
            rec.push_back(h);
        }
        while (co.size() % kStrGroup) {
            co.push_back(0.0);
            zs.push_back(0u);
            op.push_back(-1);
        }
        bounds.push_back(make_int4(r0, (int)rec.size(), s0, (int)co.size()));
    }
    zs.resize(zs.size() + 8, 0u);
    d->xrec = pk.add(rec);
    d->xcoef = pk.add(co);
    d->xzs = pk.add(zs);
    d->xop = pk.add(op);
    d->xchunk = pk.add(bounds);
    d->xseg = pk.add(seg);
    d->n_xchunks = (int)bounds.size();
}

// The device tables of a pool in one pinned host image (caller holds p.mu).
const TableImage &pool_image_locked(const Pool &p) {
    if (p.img) return *p.img;
    std::shared_ptr<TableImage> im = std::make_shared<TableImage>();
    ImagePacker pk;
    DevicePool *d = &im->pool;
    // pool order (pair kernels): each operator's strings padded with zero
    // strings to a multiple of kPairGroup, read kPairGroup at a time
    std::vector<HClass> ops(p.n_ops());
    std::vector<HTerm> terms;
    for (int k = 0; k < p.n_ops(); ++k) {
        const int32_t s0 = (int32_t)terms.size();
        for (int s = p.op_off[k]; s < p.op_off[k + 1]; ++s) terms.push_back(make_term(p.str_c[s], p.str_z[s]));
        while ((terms.size() - s0) % kPairGroup) terms.push_back(HTerm{0.0, 0u, 0u});
        ops[k] = HClass{p.op_x[k], s0, (int32_t)terms.size(), p.kind[k]};
    }
    d->pop = pk.add(ops);
    d->pterm = pk.add(terms);
    d->op_norm1 = pk.add(p.op_norm1);
    // gradient screen schedule: operators and their strings re-laid out in
    // GOCP family order (families in creation order, members in assignment
    // order); each record keeps its pool index
    // (within each LDS stage chunk, re-laid out wave by wave as for H, every
    // wave keeping family order)
    const int m = p.n_ops();
    auto count = [&](int r) { const int j = p.fam_members[r]; return p.op_off[j + 1] - p.op_off[j]; };
    // factored operators (factor_op) take one group of parameters instead of
    // their strings, flagged by kFactBit in the X mask
    std::vector<char> fac(m);
    std::vector<std::array<double, kStrGroup>> fco(m);
    std::vector<std::array<uint32_t, kStrGroup>> fzs(m);
    for (int r = 0; r < m; ++r) {
        double c4[kStrGroup];
        uint32_t z4[kStrGroup];
        fac[r] = factor_op(p, p.fam_members[r], c4, z4);
        for (int q = 0; q < kStrGroup; ++q) {
            fco[r][q] = c4[q];
            fzs[r][q] = z4[q];
        }
    }
    auto count_st = [&](int r) { return fac[r] ? kStrGroup : count(r); };
    const std::vector<int32_t> pch = stage_chunks(padded_offsets(m, count_st));
    std::vector<int> cost(m);
    for (int r = 0; r < m; ++r) cost[r] = fac[r] ? kOpCost + 3 * kStrGroup : record_cost(count(r), kOpCost);
    std::vector<int32_t> order, seg;
    for (size_t k = 0; k + 1 < pch.size(); ++k) wave_split(cost, pch[k], pch[k + 1], order, seg);
    std::vector<HClass> sop;
    std::vector<HSub> psub;
    std::vector<double> co;
    std::vector<uint32_t> zs;
    for (int32_t r : order) {
        const int32_t j = p.fam_members[r];
        HClass rec{p.op_x[j], (int32_t)co.size(), 0, j};
        if (fac[r]) {
            rec.x |= kFactBit;
            for (int q = 0; q < kStrGroup; ++q) {
                co.push_back(fco[r][q]);
                zs.push_back(fzs[r][q]);
            }
            psub.push_back(HSub{});
        } else {
            psub.push_back(bucket_strings(p.str_c, p.str_z, p.op_off[j], p.op_off[j + 1], co, zs));
        }
        rec.s1 = (int32_t)co.size();
        sop.push_back(rec);
    }
    d->sop = pk.add(sop);
    d->scoef = pk.add(co);
    d->szs = pk.add(zs);
    d->psub = pk.add(psub);
    d->pchunk = pk.add(stage_bounds(pch, sop));
    d->pseg = pk.add(seg);
    d->n_chunks = (int)pch.size() - 1;
    add_xclass_screen(p, pk, d);
    pk.finish(*im);
    p.img = im;
    return *p.img;
}

}  // namespace

std::shared_ptr<const TableImage> ham_image(const Ham &h) {
    std::lock_guard<std::mutex> lk(h.mu);
    ham_image_locked(h);
    return h.img;
}

std::shared_ptr<const TableImage> pool_image(const Pool &p) {
    std::lock_guard<std::mutex> lk(p.mu);
    pool_image_locked(p);
    return p.img;
}

const DeviceHam *device_ham(const Ham &h, int dev) {
    std::lock_guard<std::mutex> lk(h.mu);
    if ((int)h.dev.size() <= dev) h.dev.resize(dev + 1, nullptr);
    if (h.dev[dev]) return h.dev[dev];
    const TableImage &im = ham_image_locked(h);
    char *base = nullptr;
    hip_check(hipMalloc(&base, im.bytes), "hipMalloc Hamiltonian tables");
    const hipError_t e = hipMemcpy(base, im.host, im.bytes, hipMemcpyHostToDevice);
    if (e != hipSuccess) (void)hipFree(base);
    hip_check(e, "hipMemcpy Hamiltonian tables");
    h.dev[dev] = new DeviceHam(place_ham(im, base, dev));
    return h.dev[dev];
}

const DevicePool *device_pool(const Pool &p, int dev) {
    std::lock_guard<std::mutex> lk(p.mu);
    if ((int)p.dev.size() <= dev) p.dev.resize(dev + 1, nullptr);
    if (p.dev[dev]) return p.dev[dev];
    const TableImage &im = pool_image_locked(p);
    char *base = nullptr;
    hip_check(hipMalloc(&base, im.bytes), "hipMalloc pool tables");
    const hipError_t e = hipMemcpy(base, im.host, im.bytes, hipMemcpyHostToDevice);
    if (e != hipSuccess) (void)hipFree(base);
    hip_check(e, "hipMemcpy pool tables");
    p.dev[dev] = new DevicePool(place_pool(im, base, dev));
    return p.dev[dev];
}

// ---------------------------------------------------------------- workspace

namespace {
struct Bump {
    size_t used = 0;
    size_t take(size_t bytes) {
        const size_t off = (used + 255) & ~(size_t)255;
        used = off + bytes;
        return off;
    }
};
}  // namespace

InstPlan plan_instance(int nq, int M, int max_iter, int dtype, bool own_psi, bool adapt) {
    InstPlan ip;
    Bump a;
    ip.n_qubits = nq;
    ip.M = M;
    ip.max_iter = max_iter;
    ip.dtype = dtype;
    const size_t dim = (size_t)1 << nq;
    const size_t es = dtype == GOCP_C64 ? 8 : 16;
    ip.n_tiles = (int)((dim + kTile - 1) / kTile);
    ip.n_pblk = (int)std::max<size_t>(1, (dim / 2 + kPairBlock - 1) / kPairBlock);
    const size_t hist = (size_t)max_iter + 1;
    ip.o_sigma = a.take(dim * 16);
    ip.o_v = a.take(dim * es);
    ip.o_w = a.take(dim * es);
    ip.o_pe = a.take(ip.n_tiles * 8);
    ip.o_pn = a.take(ip.n_tiles * 8);
    ip.o_pg = a.take((size_t)ip.n_tiles * std::max(M, 1) * 8);
    ip.n_groups = (ip.n_tiles + kGroup - 1) / kGroup;
    ip.o_pg2 = a.take((size_t)ip.n_groups * std::max(M, 1) * 8);
    ip.o_pe2 = a.take((size_t)ip.n_groups * 8);
    ip.o_pn2 = a.take((size_t)ip.n_groups * 8);
    // line-search partials: two per pair block, then three per H v, H w
    // workgroup (one per tile, or up to kHvwPartsHi per compacted tile slot)
    const size_t n_lpart = std::max<size_t>(ip.n_tiles, (size_t)kHvwSlots * kHvwPartsHi);
    ip.o_pl = a.take((2 * (size_t)ip.n_pblk + 3 * n_lpart) * 8);
    ip.o_pt = a.take((size_t)ip.n_pblk * 8);
    ip.o_st = a.take(sizeof(AdaptState));
    ip.o_he = a.take(hist * 8);
    ip.o_hop = a.take(hist * 4);
    ip.o_hth = a.take(hist * 8);
    ip.o_hgn = a.take(hist * 8);
    ip.o_hgm = a.take(hist * 8);
    ip.o_hns = a.take(hist * 4);
    ip.o_hpr = a.take(hist * 8);
    ip.o_g = a.take((size_t)std::max(M, 1) * 8);
    if (own_psi) ip.o_psi = a.take(dim * es);
    if (adapt && dtype == GOCP_C128) {       // complex64 states never carry sigma
        ip.o_hv = a.take(dim * 16);
        ip.o_hw = a.take(dim * 16);
    }
    if (adapt && dtype == GOCP_C64 && ip.n_pblk <= kActMaxBlocks) {   // compacted H v, H w
        ip.o_act = a.take((size_t)ip.n_pblk * 2 * kPairBlock * 4);
        ip.o_actn = a.take((size_t)ip.n_pblk * 4);
    }
    ip.bytes = a.used;
    return ip;
}

InstDev make_desc(int device, const InstPlan &ip, char *b, const Ham *h, const Pool *p, void *psi,
                  double2 *sigma_override, bool upload) {
    const DeviceHam *dh = nullptr;
    const DevicePool *dp = nullptr;
    if (h) {
        dh = upload ? device_ham(*h, device) : device_ham_resident(*h, device);
        if (!dh)
            throw Error(GOCP_EINVAL, "the Hamiltonian's tables are not on this device yet (a device call "
                                     "that takes the Hamiltonian, e.g. energy, uploads them)");
    }
    if (p) {
        dp = upload ? device_pool(*p, device) : device_pool_resident(*p, device);
        if (!dp)
            throw Error(GOCP_EINVAL, "the pool's tables are not on this device yet (a device call that "
                                     "takes the pool, e.g. pool_gradients, uploads them)");
    }
    return make_desc_at(ip, b, dh, dp, psi, sigma_override);
}

InstDev make_desc_at(const InstPlan &ip, char *b, const DeviceHam *dh, const DevicePool *dp, void *psi,
                     double2 *sigma_override) {
    InstDev I;
    std::memset(&I, 0, sizeof(I));
    if (dh) {
        I.hcls = dh->hcls;
        I.hcoef = dh->hcoef;
        I.hzs = dh->hzs;
        I.hsub = dh->hsub;
        I.hchunk = dh->hchunk;
        I.hseg = dh->hseg;
        I.hsegp = dh->hsegp;
        I.hsegp_lo = dh->hsegp_lo;
        I.hcoefG = dh->hcoefG;
        I.hzsG = dh->hzsG;
        I.hchunkG = dh->hchunkG;
        I.hgx = dh->hgx;
        I.hgseg = dh->hgseg;
        I.n_hchunks = dh->n_chunks;
    }
    if (dp) {
        I.pop = dp->pop;
        I.pterm = dp->pterm;
        I.op_norm1 = dp->op_norm1;
        I.sop = dp->sop;
        I.scoef = dp->scoef;
        I.szs = dp->szs;
        I.psub = dp->psub;
        I.pchunk = dp->pchunk;
        I.pseg = dp->pseg;
        I.n_pchunks = dp->n_chunks;
        I.xrec = dp->xrec;
        I.xcoef = dp->xcoef;
        I.xzs = dp->xzs;
        I.xop = dp->xop;
        I.xchunk = dp->xchunk;
        I.xseg = dp->xseg;
        I.n_xchunks = dp->n_xchunks;
    }
    I.psi = psi;
    I.sigma = sigma_override ? sigma_override : reinterpret_cast<double2 *>(b + ip.o_sigma);
    I.v = b + ip.o_v;
    I.w = b + ip.o_w;
    I.hv = ip.o_hv ? reinterpret_cast<double2 *>(b + ip.o_hv) : nullptr;
    I.hw = ip.o_hw ? reinterpret_cast<double2 *>(b + ip.o_hw) : nullptr;
    I.act = ip.o_act ? reinterpret_cast<uint32_t *>(b + ip.o_act) : nullptr;
    I.act_n = ip.o_actn ? reinterpret_cast<int32_t *>(b + ip.o_actn) : nullptr;
    I.part_e = reinterpret_cast<double *>(b + ip.o_pe);
    I.part_n = reinterpret_cast<double *>(b + ip.o_pn);
    I.part_g = reinterpret_cast<double *>(b + ip.o_pg);
    I.part_g2 = reinterpret_cast<double *>(b + ip.o_pg2);
    I.part_e2 = reinterpret_cast<double *>(b + ip.o_pe2);
    I.part_n2 = reinterpret_cast<double *>(b + ip.o_pn2);
    I.n_groups = ip.n_groups;
    I.part_l = reinterpret_cast<double *>(b + ip.o_pl);
    I.part_t = reinterpret_cast<double *>(b + ip.o_pt);
    I.st = reinterpret_cast<AdaptState *>(b + ip.o_st);
    I.n_qubits = ip.n_qubits;
    I.M = ip.M;
    I.n_tiles = ip.n_tiles;
    I.n_pblk = ip.n_pblk;
    I.n_lpart = ip.n_tiles;
    I.hvw_parts = kHvwPartsHi;
    return I;
}

AdaptState make_state(const InstPlan &ip, char *b, int max_iter, double grad_tol, bool hist) {
    AdaptState s;
    std::memset(&s, 0, sizeof(s));
    s.max_iter = max_iter;
    s.grad_tol = grad_tol;
    s.nrm = 1.0;
    s.pend_it = s.sel_it = -1;
    s.pend_mode = s.sel_mode = -1;
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

namespace {

// Device address of `scratch` on each device, resolved once per device with
// that device current; read under the mutex.
std::mutex scratch_mu;
std::vector<char *> scratch_addr;

void resolve_scratch(int device) {
    std::lock_guard<std::mutex> lk(scratch_mu);
    if ((int)scratch_addr.size() <= device) scratch_addr.resize(device + 1, nullptr);
    if (scratch_addr[device]) return;
    void *ptr = nullptr;
    hip_check(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
    if (!ptr) throw Error(GOCP_EDEVICE, "hipGetSymbolAddress(scratch) returned a null address");
    scratch_addr[device] = static_cast<char *>(ptr);
}

char *scratch_base(int device) {
    std::lock_guard<std::mutex> lk(scratch_mu);
    char *b = (int)scratch_addr.size() > device ? scratch_addr[device] : nullptr;
    if (!b) throw Error(GOCP_EDEVICE, "the allocation-free workspace of this device was not resolved");
    return b;
}

// Workspace of a one-shot call: one instance plus its descriptor and block
// tables, carved from the context's arena (grown on demand).
struct OneShot {
    InstPlan ip;
    size_t o_desc = 0, o_btile = 0, o_bpair = 0;
    int nt = 0, np = 0;
    bool xform = false;          // the pool has an X-class screen
    InstDev *desc = nullptr;
    int2 *btile = nullptr, *bpair = nullptr;
    char *base = nullptr;
};

OneShot one_shot(gocp_ctx *ctx, const Ham *h, const Pool *p, const void *psi, int dtype,
                 double2 *sigma_override = nullptr, bool with_state = true) {
    if (!psi) throw Error(GOCP_EINVAL, "null state pointer");
    check_dtype(dtype);
    const int nq = h ? h->n_qubits : p->n_qubits;
    if (h && p && h->n_qubits != p->n_qubits)
        throw Error(GOCP_ESHAPE, "Hamiltonian and pool act on different qubit counts");
    OneShot o;
    o.ip = plan_instance(nq, p ? p->n_ops() : 0, 0, dtype, false, false);
    Bump a;
    a.used = o.ip.bytes;
    o.o_desc = a.take(sizeof(InstDev));
    o.o_btile = a.take((size_t)o.ip.n_tiles * sizeof(int2));
    o.o_bpair = a.take((size_t)o.ip.n_pblk * sizeof(int2));
    if (ctx->arena_cap < a.used) {
        if (ctx->arena) {
            hip_check(hipStreamSynchronize(ctx->user_stream), "hipStreamSynchronize");
            hip_check(hipFree(ctx->arena), "hipFree");
            ctx->arena = nullptr;
            ctx->arena_cap = 0;
        }
        const size_t cap = std::max(a.used, (size_t)1 << 20);
        hip_check(hipMalloc(&ctx->arena, cap), "hipMalloc workspace");
        ctx->arena_cap = cap;
        ctx->shot_dtype = -1;
    }
    char *b = ctx->arena;
    o.base = b;
    hipStream_t s = ctx->user_stream;
    InstDev I = make_desc(ctx->device, o.ip, b, h, p, const_cast<void *>(psi), sigma_override);
    if (with_state) {   // (the Taylor kernels outside ADAPT never read the record)
        AdaptState st = make_state(o.ip, b, 0, 0.0, false);
        hip_check(hipMemcpyAsync(b + o.ip.o_st, &st, sizeof(st), hipMemcpyHostToDevice, s), "H2D");
    }
    // the descriptor and row tables are a function of the key alone and no
    // kernel writes them: a call with the last call's key finds them in place
    const uint64_t kh = h ? h->uid : 0, kp = p ? p->uid : 0;
    if (ctx->shot_dtype != dtype || ctx->shot_h != kh || ctx->shot_p != kp || ctx->shot_psi != psi ||
        ctx->shot_sig != sigma_override) {
        std::vector<int2> bt, bp;
        for (int t = 0; t < o.ip.n_tiles; ++t) bt.push_back(make_int2(0, t));   // rows (0, g) double as group rows
        for (int t = 0; t < o.ip.n_pblk; ++t) bp.push_back(make_int2(0, t));
        hip_check(hipMemcpyAsync(b + o.o_desc, &I, sizeof(I), hipMemcpyHostToDevice, s), "H2D");
        hip_check(hipMemcpyAsync(b + o.o_btile, bt.data(), bt.size() * sizeof(int2), hipMemcpyHostToDevice, s), "H2D");
        hip_check(hipMemcpyAsync(b + o.o_bpair, bp.data(), bp.size() * sizeof(int2), hipMemcpyHostToDevice, s), "H2D");
        ctx->shot_dtype = dtype;
        ctx->shot_h = kh;
        ctx->shot_p = kp;
        ctx->shot_psi = psi;
        ctx->shot_sig = sigma_override;
    }
    o.desc = reinterpret_cast<InstDev *>(b + o.o_desc);
    o.btile = reinterpret_cast<int2 *>(b + o.o_btile);
    o.bpair = reinterpret_cast<int2 *>(b + o.o_bpair);
    o.nt = o.ip.n_tiles;
    o.np = o.ip.n_pblk;
    o.xform = I.n_xchunks > 0;
    return o;
}

AdaptState read_state(gocp_ctx *ctx, const OneShot &o) {
    AdaptState st;
    hip_check(hipMemcpyAsync(&st, o.base + o.ip.o_st, sizeof(st), hipMemcpyDeviceToHost, ctx->user_stream), "D2H");
    hip_check(hipStreamSynchronize(ctx->user_stream), "hipStreamSynchronize");
    return st;
}

}  // namespace

const AdaptState *enqueue_energy_sigma(gocp_ctx *ctx, const Ham *h, const void *psi, int dtype, double2 *sigma) {
    OneShot o = one_shot(ctx, h, nullptr, psi, dtype, sigma);
    launch_kernel(K_ENERGY_SCREEN, dtype, 1, o.desc, o.btile, o.nt, 0, ctx->user_stream);
    launch_kernel(K_SCREEN_SUM1, dtype, 1, o.desc, o.btile, o.ip.n_groups, 0, ctx->user_stream);
    launch_kernel(K_SCREEN_REDUCE, dtype, 1, o.desc, o.btile, 1, 0, ctx->user_stream);
    return reinterpret_cast<const AdaptState *>(o.base + o.ip.o_st);
}

}  // namespace gocp

using namespace gocp;

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
    resolve_scratch(device);
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
    if (ctx->arena) (void)hipFree(ctx->arena);
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

int gocp_phase_trace(gocp_ctx *ctx, uint64_t *out, int32_t n_rows, int32_t *n_phases) {
    GOCP_GUARD_BEGIN
    check_ctx(ctx);
    if (n_phases) *n_phases = kPhases;
    if (!out || n_rows <= 0 || n_rows > kPhaseRows) throw Error(GOCP_EINVAL, "bad phase trace buffer");
    hip_check(hipStreamSynchronize(ctx->user_stream), "hipStreamSynchronize");
    static_assert(sizeof(uint64_t) == sizeof(unsigned long long), "64-bit clock values");
    if (!phase_trace_read(reinterpret_cast<unsigned long long *>(out), (size_t)n_rows * kPhases))
        throw Error(GOCP_ENOTSUP, "this library records no phase trace (build it with GOCP_PHASE_TRACE)");
    return GOCP_OK;
    GOCP_GUARD_END
}

int gocp_ctx_synchronize(gocp_ctx *ctx) {
    GOCP_GUARD_BEGIN
    check_ctx(ctx);
    hip_check(hipStreamSynchronize(ctx->user_stream), "hipStreamSynchronize");
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

int gocp_state_hf(gocp_ctx *ctx, int n_qubits, int n_electrons, int mapping, void *psi_dev, int dtype) {
    GOCP_GUARD_BEGIN
    check_ctx(ctx);
    check_dtype(dtype);
    if (!psi_dev) throw Error(GOCP_EINVAL, "null state pointer");
    if (n_qubits < 1 || n_qubits > kMaxQubits) throw Error(GOCP_ENOTSUP, "qubit count out of range");
    const uint64_t idx = hf_index(n_qubits, n_electrons, mapping);
    launch_basis(dtype, psi_dev, 1u << n_qubits, (uint32_t)idx, ctx->user_stream);
    return GOCP_OK;
    GOCP_GUARD_END
}

int gocp_sector_weight(gocp_ctx *ctx, int n_qubits, int n_electrons, int mapping, const void *psi_dev, int dtype,
                       double *weight) {
    GOCP_GUARD_BEGIN
    check_ctx(ctx);
    check_dtype(dtype);
    if (!psi_dev || !weight) throw Error(GOCP_EINVAL, "null state or output");
    if (n_qubits < 1 || n_qubits > kMaxQubits) throw Error(GOCP_ENOTSUP, "qubit count out of range");
    if (n_electrons < 0 || n_electrons > n_qubits) throw Error(GOCP_EINVAL, "electron count out of range");
    SectorRows rows{};
    const std::vector<uint32_t> r = occupation_rows(n_qubits, mapping);
    for (int j = 0; j < n_qubits; ++j) rows.r[j] = r[j];
    rows.n = n_qubits;
    rows.ne = n_electrons;
    const uint32_t dim = 1u << n_qubits;
    const int nblk = (int)std::min<uint32_t>(1024, (dim + 255) / 256);
    double *part = nullptr;
    hip_check(hipMalloc(&part, sizeof(double) * 2 * nblk), "hipMalloc");
    std::vector<double> h(2 * nblk);
    hipError_t e = hipSuccess;
    try {
        launch_sector_weight(dtype, psi_dev, dim, rows, part, nblk, ctx->user_stream);
        e = hipMemcpyAsync(h.data(), part, sizeof(double) * 2 * nblk, hipMemcpyDeviceToHost, ctx->user_stream);
        if (e == hipSuccess) e = hipStreamSynchronize(ctx->user_stream);
    } catch (...) {
        (void)hipFree(part);
        throw;
    }
    (void)hipFree(part);
    hip_check(e, "sector weight");
    double in = 0.0, all = 0.0;
    for (int b = 0; b < nblk; ++b) {
        in += h[2 * b];
        all += h[2 * b + 1];
    }
    if (!(all > 0.0)) throw Error(GOCP_ENUMERIC, "zero norm");
    *weight = in / all;
    return GOCP_OK;
    GOCP_GUARD_END
}

int energy(gocp_ctx *ctx, const gocp_ham *hh, const void *psi_dev, int dtype, double *e_out) {
    GOCP_GUARD_BEGIN
    check_ctx(ctx);
    if (!e_out) throw Error(GOCP_EINVAL, "null output");
    OneShot o = one_shot(ctx, as_ham(hh), nullptr, psi_dev, dtype);
    launch_kernel(K_ENERGY_SCREEN, dtype, 1, o.desc, o.btile, o.nt, 0, ctx->user_stream);
    launch_kernel(K_SCREEN_SUM1, dtype, 1, o.desc, o.btile, o.ip.n_groups, 0, ctx->user_stream);
    launch_kernel(K_SCREEN_REDUCE, dtype, 1, o.desc, o.btile, 1, 0, ctx->user_stream);
    const AdaptState st = read_state(ctx, o);
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
    OneShot o = one_shot(ctx, as_ham(hh), nullptr, psi_dev, dtype, static_cast<double2 *>(sigma_dev));
    launch_kernel(K_ENERGY_SCREEN, dtype, 1, o.desc, o.btile, o.nt, 0, ctx->user_stream);
    launch_kernel(K_SCREEN_SUM1, dtype, 1, o.desc, o.btile, o.ip.n_groups, 0, ctx->user_stream);
    launch_kernel(K_SCREEN_REDUCE, dtype, 1, o.desc, o.btile, 1, 0, ctx->user_stream);
    if (e_out) {
        const AdaptState st = read_state(ctx, o);
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
    OneShot o = one_shot(ctx, h, p, psi_dev, dtype);
    launch_kernel(o.xform ? K_ENERGY_SCREEN_X : K_ENERGY_SCREEN, dtype, 1, o.desc, o.btile, o.nt, 0,
                  ctx->user_stream);
    launch_kernel(K_SCREEN_SUM1, dtype, 1, o.desc, o.btile, o.ip.n_groups, 0, ctx->user_stream, sum1_blocks(o.ip.M));
    launch_kernel(o.ip.M > kPairBlock ? K_SCREEN_REDUCE_W : K_SCREEN_REDUCE, dtype, 1, o.desc, o.btile, 1, 0,
                  ctx->user_stream);
    const size_t gbytes = (size_t)p->n_ops() * sizeof(double);
    if (g_on_device) {
        hip_check(hipMemcpyAsync(g_out, o.base + o.ip.o_g, gbytes, hipMemcpyDeviceToDevice,
                                 ctx->user_stream), "hipMemcpyAsync D2D");
    } else {
        hip_check(hipMemcpyAsync(g_out, o.base + o.ip.o_g, gbytes, hipMemcpyDeviceToHost,
                                 ctx->user_stream), "hipMemcpyAsync D2H");
        const AdaptState st = read_state(ctx, o);
        if (st.status) throw Error(st.status, "non-finite gradient");
    }
    return GOCP_OK;
    GOCP_GUARD_END
}

int pool_gradients_noalloc(gocp_ctx *ctx, const gocp_ham *hh, const gocp_pool *pp, const void *psi_dev,
                           int dtype, double *g_dev) {
    GOCP_GUARD_BEGIN
    check_ctx(ctx);
    if (!psi_dev || !g_dev) throw Error(GOCP_EINVAL, "null state or output pointer");
    check_dtype(dtype);
    const Ham *h = as_ham(hh);
    const Pool *p = as_pool(pp);
    if (h->n_qubits != p->n_qubits) throw Error(GOCP_ESHAPE, "Hamiltonian and pool act on different qubit counts");
    // layout inside the scratch: the descriptor, then the one-shot workspace
    const InstPlan ip = plan_instance(h->n_qubits, p->n_ops(), 0, dtype, false, false);
    const size_t o_work = (sizeof(InstDev) + 255) & ~(size_t)255;
    if (o_work + ip.bytes > kNoAllocScratchBytes)
        throw Error(GOCP_ENOTSUP, "pool_gradients_noalloc: the workspace of " + std::to_string(o_work + ip.bytes) +
                                      " bytes exceeds its fixed " + std::to_string(kNoAllocScratchBytes) +
                                      "-byte device scratch (use pool_gradients)");
    char *base = scratch_base(ctx->device);
    char *b = base + o_work;
    const InstDev I = make_desc(ctx->device, ip, b, h, p, const_cast<void *>(psi_dev), nullptr, false);
    AdaptState st = make_state(ip, b, 0, 0.0, false);
    st.g = g_dev;                     // the selection pass writes the gradients straight to the caller
    hipStream_t s = ctx->user_stream;
    hip_check(hipMemcpyAsync(base, &I, sizeof(I), hipMemcpyHostToDevice, s), "H2D");
    hip_check(hipMemcpyAsync(b + ip.o_st, &st, sizeof(st), hipMemcpyHostToDevice, s), "H2D");
    // one instance: null row tables, the kernels take rows (0, workgroup)
    const InstDev *desc = reinterpret_cast<const InstDev *>(base);
    launch_kernel(I.n_xchunks > 0 ? K_ENERGY_SCREEN_X : K_ENERGY_SCREEN, dtype, 1, desc, nullptr, ip.n_tiles, 0, s);
    launch_kernel(K_SCREEN_SUM1, dtype, 1, desc, nullptr, ip.n_groups, 0, s, sum1_blocks(ip.M));
    launch_kernel(ip.M > kPairBlock ? K_SCREEN_REDUCE_W : K_SCREEN_REDUCE, dtype, 1, desc, nullptr, 1, 0, s);
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
    if (!psi_dev) throw Error(GOCP_EINVAL, "null state pointer");
    if (theta == 0.0) {
        if (n_substeps_out) *n_substeps_out = 0;
        return GOCP_OK;
    }
    const int ns = std::max(1, (int)std::ceil(std::fabs(theta) * p->op_norm1[k] / 0.5));
    OneShot o = one_shot(ctx, nullptr, p, psi_dev, dtype, nullptr, false);
    launch_kernel(K_TAYLOR, dtype, 1, o.desc, o.bpair, o.np, 0, ctx->user_stream, k, theta, ns);
    launch_kernel(K_NORMALIZE, dtype, 1, o.desc, o.bpair, o.np, 0, ctx->user_stream);
    if (n_substeps_out) *n_substeps_out = ns;
    return GOCP_OK;
    GOCP_GUARD_END
}

int taylor5_apply_family(gocp_ctx *ctx, const gocp_pool *pp, int32_t n, const int32_t *ops,
                         const double *thetas, void *psi_dev, int dtype, int32_t *n_substeps_out) {
    GOCP_GUARD_BEGIN
    check_ctx(ctx);
    const Pool *p = as_pool(pp);
    if (!ops || !thetas) throw Error(GOCP_EINVAL, "null operator or angle array");
    if (n < 1 || n > kFuseMax) throw Error(GOCP_EINVAL, "a fused step takes 1 to 4 operators");
    if (!psi_dev) throw Error(GOCP_EINVAL, "null state pointer");
    FuseArgs fa{};
    uint32_t basis[32] = {};          // echelon basis of the X masks, by leading bit
    bool any = false;
    for (int i = 0; i < n; ++i) {
        const int k = ops[i];
        if (k < 0 || k >= p->n_ops()) throw Error(GOCP_EINVAL, "operator index out of range");
        if (!std::isfinite(thetas[i])) throw Error(GOCP_EINVAL, "non-finite angle");
        for (int i2 = 0; i2 < i; ++i2)
            if (ops[i2] == k) throw Error(GOCP_EINVAL, "an operator appears twice");
        if (p->family_of[k] != p->family_of[ops[0]]) throw Error(GOCP_EINVAL, "operators of different GOCP families");
        uint32_t v = p->op_x[k];
        for (int bit = 31; bit >= 0; --bit)
            if (((v >> bit) & 1u) && basis[bit]) v ^= basis[bit];
        if (!v) throw Error(GOCP_ENOTSUP, "X masks linearly dependent over GF(2)");
        basis[31 - __builtin_clz(v)] = v;
        const double th = thetas[i];
        const int ns = th == 0.0 ? 0 : std::max(1, (int)std::ceil(std::fabs(th) * p->op_norm1[k] / 0.5));
        fa.op[i] = k;
        fa.ns[i] = ns;
        fa.x[i] = ns ? th / ns : 0.0;
        any = any || ns > 0;
    }
    if (n >= p->n_qubits) throw Error(GOCP_ENOTSUP, "the operators' X masks span every qubit");
    for (int bit = 0, q = 0; bit < 32; ++bit)
        if (basis[bit]) fa.piv[q++] = bit;
    if (n_substeps_out)
        for (int i = 0; i < n; ++i) n_substeps_out[i] = fa.ns[i];
    if (!any) return GOCP_OK;
    OneShot o = one_shot(ctx, nullptr, p, psi_dev, dtype, nullptr, false);
    launch_fused(dtype, n, o.desc, o.bpair, o.np, fa, ctx->user_stream);
    launch_kernel(K_NORMALIZE, dtype, 1, o.desc, o.bpair, o.np, 0, ctx->user_stream);
    return GOCP_OK;
    GOCP_GUARD_END
}

}  // extern "C"
