// Greedy Operator Commutativity Partitioning (Sec. III.A, Algorithm 1).
//
// Conflict graph: operators i and j are joined iff the operator commutator
// [A_i, A_j] is non-zero.  For folded strings S_a = c_a Z^{z_a} X^{x_a},
//   [S_a, S_b] = c_a c_b ((-1)^{popcount(x_a & z_b)} - (-1)^{popcount(x_b & z_a)})
//                Z^{z_a ^ z_b} X^{x_a ^ x_b},
// and all pool coefficients are multiples of 1/8, so the commutator is
// accumulated exactly on integers (coefficients scaled by 8).  Every string
// of A_i A_j shares the X mask x_i ^ x_j, so terms are keyed by z alone.
//
// Colouring: vertices by descending degree (stable: ties by pool index), each
// into the lowest-indexed family (families numbered in creation order) that
// holds no neighbour, else a new family.

#include <algorithm>
#include <cmath>

#include "internal.h"

namespace gocp {
namespace {

bool ops_commute(const Pool &p, int i, int j, std::vector<std::pair<uint32_t, int64_t>> &buf) {
    buf.clear();
    for (int a = p.op_off[i]; a < p.op_off[i + 1]; ++a) {
        const uint32_t xa = p.op_x[i], za = p.str_z[a];
        const int64_t ca = (int64_t)std::llround(p.str_c[a] * 8.0);
        for (int b = p.op_off[j]; b < p.op_off[j + 1]; ++b) {
            const uint32_t xb = p.op_x[j], zb = p.str_z[b];
            const int sab = __builtin_popcount(xa & zb) & 1;
            const int sba = __builtin_popcount(xb & za) & 1;
            if (sab == sba) continue;                         // these two strings commute
            const int64_t cb = (int64_t)std::llround(p.str_c[b] * 8.0);
            const int64_t v = (sab ? -2 : 2) * ca * cb;       // ((-1)^sab - (-1)^sba) ca cb
            buf.emplace_back(za ^ zb, v);
        }
    }
    if (buf.empty()) return true;
    std::sort(buf.begin(), buf.end());
    size_t k = 0;
    while (k < buf.size()) {
        int64_t s = 0;
        size_t e = k;
        while (e < buf.size() && buf[e].first == buf[k].first) s += buf[e++].second;
        if (s != 0) return false;
        k = e;
    }
    return true;
}

}  // namespace

void partition_pool(Pool &p) {
    const int M = p.n_ops();
    for (double c : p.str_c)
        if (c * 8.0 != std::nearbyint(c * 8.0)) throw Error(GOCP_EINVAL, "internal: pool coefficient not a multiple of 1/8");
    const int W = (M + 63) / 64;
    std::vector<uint64_t> adj((size_t)M * W, 0);
    std::vector<std::pair<uint32_t, int64_t>> buf;
    p.degree.assign(M, 0);
    p.n_edges = 0;
    for (int i = 0; i < M; ++i)
        for (int j = i + 1; j < M; ++j)
            if (!ops_commute(p, i, j, buf)) {
                adj[(size_t)i * W + j / 64] |= 1ull << (j % 64);
                adj[(size_t)j * W + i / 64] |= 1ull << (i % 64);
                ++p.degree[i];
                ++p.degree[j];
                ++p.n_edges;
            }
    p.order.resize(M);
    for (int v = 0; v < M; ++v) p.order[v] = v;
    std::stable_sort(p.order.begin(), p.order.end(),
                     [&](int a, int b) { return p.degree[a] > p.degree[b]; });

    std::vector<std::vector<uint64_t>> fam_bits;     // member bitset per family
    std::vector<std::vector<int32_t>> fam_list;
    p.family_of.assign(M, -1);
    for (int v : p.order) {
        const uint64_t *row = &adj[(size_t)v * W];
        int chosen = -1;
        for (size_t k = 0; k < fam_bits.size() && chosen < 0; ++k) {
            bool clash = false;
            for (int w = 0; w < W && !clash; ++w) clash = (fam_bits[k][w] & row[w]) != 0;
            if (!clash) chosen = (int)k;
        }
        if (chosen < 0) {
            fam_bits.emplace_back(W, 0);
            fam_list.emplace_back();
            chosen = (int)fam_bits.size() - 1;
        }
        fam_bits[chosen][v / 64] |= 1ull << (v % 64);
        fam_list[chosen].push_back(v);
        p.family_of[v] = chosen;
    }
    p.fam_off.assign(1, 0);
    p.fam_members.clear();
    for (const auto &f : fam_list) {
        p.fam_members.insert(p.fam_members.end(), f.begin(), f.end());
        p.fam_off.push_back((int32_t)p.fam_members.size());
    }
}

}  // namespace gocp
