// Fermion-to-qubit mapping, Hamiltonian assembly and pool construction.
//
// Everything is carried in the folded form c * Z^z X^x with real c (the form
// the kernels consume).  In this form the Jordan-Wigner ladder operators are
//   a+_j = 1/2 Z^{<j} X^{j} - 1/2 Z^{<=j} X^{j},
//   a_j  = 1/2 Z^{<j} X^{j} + 1/2 Z^{<=j} X^{j},
// and the product of two strings is
//   (Z^{z1} X^{x1})(Z^{z2} X^{x2}) = (-1)^{popcount(x1 & z2)} Z^{z1^z2} X^{x1^x2},
// so Hamiltonians with real integrals (Sec. II.A, Eq. 2) stay in real
// arithmetic throughout.
//
// The Bravyi-Kitaev form (Sec. II.A, binary-tree parity encoding, taken as
// the Fenwick-tree encoding b = beta n over GF(2)) is obtained from the JW
// form by the basis change U|n> = |beta n>, which carries Z^z X^x to
// Z^{beta^{-T} z} X^{beta x} without changing the coefficient.

#include <algorithm>
#include <cmath>
#include <memory>
#include <unordered_map>

#include "internal.h"

namespace gocp {
namespace {

inline int parity32(uint32_t v) { return __builtin_popcount(v) & 1; }

inline Term mul(const Term &a, const Term &b) {
    const double s = parity32(a.x & b.z) ? -1.0 : 1.0;
    return Term{a.x ^ b.x, a.z ^ b.z, s * a.c * b.c};
}

using Sum = std::vector<Term>;

Sum mul(const Sum &a, const Sum &b) {
    Sum out;
    out.reserve(a.size() * b.size());
    for (const Term &s : a)
        for (const Term &t : b) out.push_back(mul(s, t));
    return out;
}

Sum jw_create(int j) {
    const uint32_t low = (1u << j) - 1u, bit = 1u << j;
    return {Term{bit, low, 0.5}, Term{bit, low | bit, -0.5}};
}

Sum jw_annihilate(int j) {
    const uint32_t low = (1u << j) - 1u, bit = 1u << j;
    return {Term{bit, low, 0.5}, Term{bit, low | bit, 0.5}};
}

// ---- GF(2) basis change of the Fenwick (Bravyi-Kitaev) encoding
struct BkBasis {
    int n = 0;
    std::vector<uint32_t> beta_rows;     // (beta x)_j = parity(beta_rows[j] & x)
    std::vector<uint32_t> inv_t_rows;    // (beta^{-T} z)_j = parity(inv_t_rows[j] & z)
    std::vector<uint32_t> inv_rows;      // (beta^{-1} b)_j = parity(inv_rows[j] & b)

    explicit BkBasis(int nq) : n(nq), beta_rows(nq), inv_t_rows(nq), inv_rows(nq) {
        for (int j = 0; j < n; ++j) {
            const int lb = (j + 1) & -(j + 1);
            uint32_t r = 0;
            for (int k = 0; k < n; ++k)
                if (j - lb < k && k <= j) r |= 1u << k;
            beta_rows[j] = r;
        }
        // Gauss-Jordan over GF(2): [beta | I] -> [I | beta^{-1}]
        std::vector<uint32_t> a = beta_rows, inv(n);
        for (int j = 0; j < n; ++j) inv[j] = 1u << j;
        for (int col = 0; col < n; ++col) {
            int piv = -1;
            for (int r = col; r < n; ++r)
                if ((a[r] >> col) & 1u) { piv = r; break; }
            if (piv < 0) throw Error(GOCP_EINVAL, "Bravyi-Kitaev matrix is singular");
            std::swap(a[col], a[piv]);
            std::swap(inv[col], inv[piv]);
            for (int r = 0; r < n; ++r)
                if (r != col && ((a[r] >> col) & 1u)) { a[r] ^= a[col]; inv[r] ^= inv[col]; }
        }
        inv_rows = inv;
        // row j of beta^{-T} = column j of beta^{-1}
        for (int j = 0; j < n; ++j) {
            uint32_t r = 0;
            for (int k = 0; k < n; ++k)
                if ((inv[k] >> j) & 1u) r |= 1u << k;
            inv_t_rows[j] = r;
        }
    }
    uint32_t apply(const std::vector<uint32_t> &rows, uint32_t v) const {
        uint32_t out = 0;
        for (int j = 0; j < n; ++j) out |= (uint32_t)parity32(rows[j] & v) << j;
        return out;
    }
    Term map(const Term &t) const { return Term{apply(beta_rows, t.x), apply(inv_t_rows, t.z), t.c}; }
};

inline uint64_t key_of(uint32_t x, uint32_t z) { return ((uint64_t)x << 32) | z; }

void check_qubits(int nq) {
    if (nq < 1) throw Error(GOCP_EINVAL, "qubit count must be >= 1");
    if (nq > kMaxQubits) throw Error(GOCP_ENOTSUP, "at most 30 qubits are supported");
}

Ham *group_terms(int nq, std::vector<Term> terms) {
    std::sort(terms.begin(), terms.end(), [](const Term &a, const Term &b) {
        return a.x != b.x ? a.x < b.x : a.z < b.z;
    });
    Ham *h = new Ham();
    h->n_qubits = nq;
    for (size_t i = 0; i < terms.size(); ++i) {
        if (i == 0 || terms[i].x != terms[i - 1].x) {
            h->cls_x.push_back(terms[i].x);
            h->cls_off.push_back((int32_t)i);
        }
        h->str_z.push_back(terms[i].z);
        h->str_c.push_back(terms[i].c);
    }
    h->cls_off.push_back((int32_t)terms.size());
    return h;
}

std::vector<Term> drain(const std::unordered_map<uint64_t, double> &acc, double tol) {
    std::vector<Term> out;
    out.reserve(acc.size());
    for (const auto &kv : acc)
        if (std::fabs(kv.second) >= tol)
            out.push_back(Term{(uint32_t)(kv.first >> 32), (uint32_t)kv.first, kv.second});
    return out;
}

}  // namespace

Ham *build_hamiltonian(int n_spatial, const double *h1, const double *eri, double e_core,
                       int mapping) {
    if (!h1 || !eri) throw Error(GOCP_EINVAL, "null integral array");
    if (n_spatial < 1) throw Error(GOCP_EINVAL, "n_spatial must be >= 1");
    const int n = n_spatial, N = 2 * n;
    check_qubits(N);
    if (mapping != GOCP_JW && mapping != GOCP_BK) throw Error(GOCP_EINVAL, "unknown mapping");
    for (int64_t i = 0; i < (int64_t)n * n; ++i)
        if (!std::isfinite(h1[i])) throw Error(GOCP_EINVAL, "non-finite one-electron integral");
    for (int64_t i = 0; i < (int64_t)n * n * n * n; ++i)
        if (!std::isfinite(eri[i])) throw Error(GOCP_EINVAL, "non-finite two-electron integral");

    std::vector<Sum> cre(N), ann(N);
    for (int j = 0; j < N; ++j) { cre[j] = jw_create(j); ann[j] = jw_annihilate(j); }

    std::unordered_map<uint64_t, double> acc;
    acc.reserve(1 << 16);
    auto add = [&](const Sum &s, double scale) {
        for (const Term &t : s) acc[key_of(t.x, t.z)] += scale * t.c;
    };
    add(Sum{Term{0u, 0u, 1.0}}, e_core);

    // one-body: h_PQ a+_P a_Q, equal spins
    for (int P = 0; P < N; ++P)
        for (int Q = 0; Q < N; ++Q) {
            if ((P & 1) != (Q & 1)) continue;
            const double v = h1[(P / 2) * n + Q / 2];
            if (v == 0.0) continue;
            add(mul(cre[P], ann[Q]), v);
        }
    // two-body: 1/2 <PQ|RS> a+_P a+_Q a_S a_R, <PQ|RS> = (pr|qs), spins P=R, Q=S
    std::vector<Sum> cc((size_t)N * N), aa((size_t)N * N);
    for (int P = 0; P < N; ++P)
        for (int Q = 0; Q < N; ++Q) {
            cc[(size_t)P * N + Q] = mul(cre[P], cre[Q]);
            aa[(size_t)P * N + Q] = mul(ann[P], ann[Q]);
        }
    for (int P = 0; P < N; ++P)
        for (int Q = 0; Q < N; ++Q) {
            if (P == Q) continue;
            for (int R = 0; R < N; ++R) {
                if ((R & 1) != (P & 1)) continue;
                for (int S = 0; S < N; ++S) {
                    if (S == R || (S & 1) != (Q & 1)) continue;
                    const int p = P / 2, q = Q / 2, r = R / 2, s = S / 2;
                    const double v = eri[(((size_t)p * n + r) * n + q) * n + s];
                    if (v == 0.0) continue;
                    add(mul(cc[(size_t)P * N + Q], aa[(size_t)S * N + R]), 0.5 * v);
                }
            }
        }

    std::vector<Term> terms = drain(acc, kDropTol);
    if (mapping == GOCP_BK) {
        BkBasis bk(N);
        for (Term &t : terms) t = bk.map(t);
    }
    return group_terms(N, std::move(terms));
}

Ham *hamiltonian_from_terms(int nq, const std::vector<Term> &in) {
    check_qubits(nq);
    const uint32_t lim = nq == 32 ? 0xffffffffu : ((1u << nq) - 1u);
    std::unordered_map<uint64_t, double> acc;
    for (const Term &t : in) {
        if ((t.x & ~lim) || (t.z & ~lim)) throw Error(GOCP_EINVAL, "term acts outside the register");
        if (parity32(t.x & t.z)) throw Error(GOCP_EINVAL, "term with an odd number of Y factors: not a real symmetric Hamiltonian");
        if (!std::isfinite(t.c)) throw Error(GOCP_EINVAL, "non-finite coefficient");
        acc[key_of(t.x, t.z)] += t.c;
    }
    return group_terms(nq, drain(acc, kDropTol));
}

uint64_t hf_index(int nq, int ne, int mapping) {
    check_qubits(nq);
    if (ne < 0 || ne > nq) throw Error(GOCP_EINVAL, "electron count out of range");
    const uint32_t occ = ne == 32 ? 0xffffffffu : ((1u << ne) - 1u);
    if (mapping == GOCP_JW) return occ;
    if (mapping != GOCP_BK) throw Error(GOCP_EINVAL, "unknown mapping");
    BkBasis bk(nq);
    return bk.apply(bk.beta_rows, occ);
}

std::vector<uint32_t> occupation_rows(int nq, int mapping) {
    check_qubits(nq);
    std::vector<uint32_t> rows(nq);
    if (mapping == GOCP_JW) {
        for (int j = 0; j < nq; ++j) rows[j] = 1u << j;
        return rows;
    }
    if (mapping != GOCP_BK) throw Error(GOCP_EINVAL, "unknown mapping");
    return BkBasis(nq).inv_rows;
}

uint64_t basis_occupation(int nq, int mapping, uint64_t index) {
    const std::vector<uint32_t> rows = occupation_rows(nq, mapping);
    if (index >> nq) throw Error(GOCP_EINVAL, "basis index out of range");
    uint64_t occ = 0;
    for (int j = 0; j < nq; ++j) occ |= (uint64_t)(__builtin_popcount(rows[j] & (uint32_t)index) & 1) << j;
    return occ;
}

Pool *build_pool(int nq, int ne, int mapping, bool pauli) {
    check_qubits(nq);
    if (ne <= 0 || ne >= nq || (ne & 1)) throw Error(GOCP_EINVAL, "electron count must be even and in (0, n_qubits)");
    if (mapping != GOCP_JW && mapping != GOCP_BK) throw Error(GOCP_EINVAL, "unknown mapping");
    std::vector<Sum> cre(nq), ann(nq);
    for (int j = 0; j < nq; ++j) { cre[j] = jw_create(j); ann[j] = jw_annihilate(j); }
    std::unique_ptr<BkBasis> bk;
    if (mapping == GOCP_BK) bk.reset(new BkBasis(nq));

    Pool *p = new Pool();
    p->n_qubits = nq;
    p->n_electrons = ne;
    p->mapping = mapping;
    p->op_off.push_back(0);

    auto emit = [&](int kind, int i, int j, int a, int b, const Sum &tau) {
        // A = tau - tau^+ ; (c Z^z X^x)^+ = c (-1)^{popcount(x&z)} Z^z X^x
        std::unordered_map<uint64_t, double> acc;
        for (const Term &t : tau) {
            acc[key_of(t.x, t.z)] += t.c;
            acc[key_of(t.x, t.z)] -= (parity32(t.x & t.z) ? -t.c : t.c);
        }
        std::vector<Term> ts = drain(acc, kDropTol);
        if (bk) for (Term &t : ts) t = bk->map(t);
        std::sort(ts.begin(), ts.end(), [](const Term &u, const Term &v) { return u.z < v.z; });
        const size_t want = kind == 1 ? 2 : 8;
        if (ts.size() != want) throw Error(GOCP_EINVAL, "internal: unexpected generator string count");
        for (const Term &t : ts)
            if (t.x != ts[0].x) throw Error(GOCP_EINVAL, "internal: generator with several X masks");
        if (pauli) {
            // one operator per string, its coefficient scaled to unit
            // magnitude: each string of an anti-Hermitian generator is
            // anti-Hermitian by itself and squares to -1
            for (const Term &t : ts) {
                p->str_z.push_back(t.z);
                p->str_c.push_back(t.c > 0.0 ? 1.0 : -1.0);
                p->op_x.push_back(t.x);
                p->op_off.push_back((int32_t)p->str_z.size());
                p->op_norm1.push_back(1.0);
                p->kind.push_back(kind + 2);
                p->idx.insert(p->idx.end(), {i, j, a, b});
            }
            return;
        }
        double n1 = 0.0;
        for (const Term &t : ts) {
            p->str_z.push_back(t.z);
            p->str_c.push_back(t.c);
            n1 += std::fabs(t.c);
        }
        p->op_x.push_back(ts[0].x);
        p->op_off.push_back((int32_t)p->str_z.size());
        p->op_norm1.push_back(n1);
        p->kind.push_back(kind);
        p->idx.insert(p->idx.end(), {i, j, a, b});
    };

    for (int i = 0; i < ne; ++i)
        for (int a = ne; a < nq; ++a)
            if ((i & 1) == (a & 1)) emit(1, i, a, -1, -1, mul(cre[a], ann[i]));
    for (int i = 0; i < ne; ++i)
        for (int j = i + 1; j < ne; ++j)
            for (int a = ne; a < nq; ++a)
                for (int b = a + 1; b < nq; ++b) {
                    if ((i & 1) + (j & 1) != (a & 1) + (b & 1)) continue;
                    emit(2, i, j, a, b, mul(mul(mul(cre[a], cre[b]), ann[j]), ann[i]));
                }
    partition_pool(*p);
    return p;
}

}  // namespace gocp
