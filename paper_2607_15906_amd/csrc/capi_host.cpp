// Host-only C ABI entry points: Hamiltonian load, pool build, partition and
// queries.  None of them touches the GPU.

#include <cstring>
#include <exception>
#include <new>

#include "internal.h"

namespace gocp {
namespace {
thread_local std::string g_last_error;
}
void set_last_error(const std::string &msg) { g_last_error = msg; }
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

const char *gocp_last_error(void) { return g_last_error.c_str(); }

int gocp_version(void) { return 10000; }

int pauli_hamiltonian_load(int n_spatial, const double *h1, const double *eri, double e_core,
                           int mapping, gocp_ham **out) {
    GOCP_GUARD_BEGIN
    if (!out) throw Error(GOCP_EINVAL, "null output handle");
    *out = reinterpret_cast<gocp_ham *>(build_hamiltonian(n_spatial, h1, eri, e_core, mapping));
    return GOCP_OK;
    GOCP_GUARD_END
}

int pauli_hamiltonian_load_terms(int n_qubits, int64_t n_terms, const uint32_t *x,
                                 const uint32_t *z, const double *c, gocp_ham **out) {
    GOCP_GUARD_BEGIN
    if (!out || n_terms < 0 || (n_terms > 0 && (!x || !z || !c)))
        throw Error(GOCP_EINVAL, "null pointer or negative term count");
    std::vector<Term> t((size_t)n_terms);
    for (int64_t i = 0; i < n_terms; ++i) t[i] = Term{x[i], z[i], c[i]};
    *out = reinterpret_cast<gocp_ham *>(hamiltonian_from_terms(n_qubits, t));
    return GOCP_OK;
    GOCP_GUARD_END
}

int gocp_ham_info(const gocp_ham *hh, int32_t *n_qubits, int64_t *n_terms, int32_t *n_classes) {
    GOCP_GUARD_BEGIN
    if (!hh) throw Error(GOCP_EINVAL, "null Hamiltonian");
    const Ham *h = reinterpret_cast<const Ham *>(hh);
    if (n_qubits) *n_qubits = h->n_qubits;
    if (n_terms) *n_terms = h->n_terms();
    if (n_classes) *n_classes = h->n_classes();
    return GOCP_OK;
    GOCP_GUARD_END
}

int gocp_ham_terms(const gocp_ham *hh, int64_t capacity, uint32_t *x, uint32_t *z, double *c) {
    GOCP_GUARD_BEGIN
    if (!hh || !x || !z || !c) throw Error(GOCP_EINVAL, "null pointer");
    const Ham *h = reinterpret_cast<const Ham *>(hh);
    if (capacity < h->n_terms()) throw Error(GOCP_EINVAL, "output capacity below the term count");
    for (int k = 0; k < h->n_classes(); ++k)
        for (int s = h->cls_off[k]; s < h->cls_off[k + 1]; ++s) {
            x[s] = h->cls_x[k];
            z[s] = h->str_z[s];
            c[s] = h->str_c[s];
        }
    return GOCP_OK;
    GOCP_GUARD_END
}

int gocp_ham_free(gocp_ham *hh) {
    GOCP_GUARD_BEGIN
    Ham *h = reinterpret_cast<Ham *>(hh);
    if (h) {
        for (DeviceHam *d : h->dev)
            if (d) release_device_ham(d);
        delete h;
    }
    return GOCP_OK;
    GOCP_GUARD_END
}

int pool_build(int n_qubits, int n_electrons, int mapping, gocp_pool **out) {
    GOCP_GUARD_BEGIN
    if (!out) throw Error(GOCP_EINVAL, "null output handle");
    *out = reinterpret_cast<gocp_pool *>(build_pool(n_qubits, n_electrons, mapping));
    return GOCP_OK;
    GOCP_GUARD_END
}

int pool_build_pauli(int n_qubits, int n_electrons, int mapping, gocp_pool **out) {
    GOCP_GUARD_BEGIN
    if (!out) throw Error(GOCP_EINVAL, "null output handle");
    *out = reinterpret_cast<gocp_pool *>(build_pool(n_qubits, n_electrons, mapping, true));
    return GOCP_OK;
    GOCP_GUARD_END
}

int gocp_pool_info(const gocp_pool *pp, int32_t *n_qubits, int32_t *n_ops, int32_t *n_strings) {
    GOCP_GUARD_BEGIN
    if (!pp) throw Error(GOCP_EINVAL, "null pool");
    const Pool *p = reinterpret_cast<const Pool *>(pp);
    if (n_qubits) *n_qubits = p->n_qubits;
    if (n_ops) *n_ops = p->n_ops();
    if (n_strings) *n_strings = (int32_t)p->str_z.size();
    return GOCP_OK;
    GOCP_GUARD_END
}

int gocp_pool_op(const gocp_pool *pp, int32_t k, int32_t *kind, int32_t idx[4], uint32_t *xmask) {
    GOCP_GUARD_BEGIN
    if (!pp) throw Error(GOCP_EINVAL, "null pool");
    const Pool *p = reinterpret_cast<const Pool *>(pp);
    if (k < 0 || k >= p->n_ops()) throw Error(GOCP_EINVAL, "operator index out of range");
    if (kind) *kind = p->kind[k];
    if (idx) std::memcpy(idx, &p->idx[(size_t)4 * k], 4 * sizeof(int32_t));
    if (xmask) *xmask = p->op_x[k];
    return GOCP_OK;
    GOCP_GUARD_END
}

int gocp_pool_strings(const gocp_pool *pp, int32_t *op_offsets, uint32_t *z, double *c) {
    GOCP_GUARD_BEGIN
    if (!pp || !op_offsets || !z || !c) throw Error(GOCP_EINVAL, "null pointer");
    const Pool *p = reinterpret_cast<const Pool *>(pp);
    std::memcpy(op_offsets, p->op_off.data(), p->op_off.size() * sizeof(int32_t));
    std::memcpy(z, p->str_z.data(), p->str_z.size() * sizeof(uint32_t));
    std::memcpy(c, p->str_c.data(), p->str_c.size() * sizeof(double));
    return GOCP_OK;
    GOCP_GUARD_END
}

int gocp_pool_free(gocp_pool *pp) {
    GOCP_GUARD_BEGIN
    Pool *p = reinterpret_cast<Pool *>(pp);
    if (p) {
        for (DevicePool *d : p->dev)
            if (d) release_device_pool(d);
        delete p;
    }
    return GOCP_OK;
    GOCP_GUARD_END
}

int gocp_partition(const gocp_pool *pp, int32_t *family_of, int32_t *n_families, int32_t *order) {
    GOCP_GUARD_BEGIN
    if (!pp || !family_of || !n_families) throw Error(GOCP_EINVAL, "null pointer");
    const Pool *p = reinterpret_cast<const Pool *>(pp);
    std::memcpy(family_of, p->family_of.data(), p->family_of.size() * sizeof(int32_t));
    *n_families = (int32_t)p->fam_off.size() - 1;
    if (order) std::memcpy(order, p->order.data(), p->order.size() * sizeof(int32_t));
    return GOCP_OK;
    GOCP_GUARD_END
}

int gocp_conflict_degrees(const gocp_pool *pp, int64_t *n_edges, int32_t *deg) {
    GOCP_GUARD_BEGIN
    if (!pp) throw Error(GOCP_EINVAL, "null pool");
    const Pool *p = reinterpret_cast<const Pool *>(pp);
    if (n_edges) *n_edges = p->n_edges;
    if (deg) std::memcpy(deg, p->degree.data(), p->degree.size() * sizeof(int32_t));
    return GOCP_OK;
    GOCP_GUARD_END
}

int gocp_basis_occupation(int n_qubits, int mapping, uint64_t index, uint64_t *occupation) {
    GOCP_GUARD_BEGIN
    if (!occupation) throw Error(GOCP_EINVAL, "null output");
    *occupation = basis_occupation(n_qubits, mapping, index);
    return GOCP_OK;
    GOCP_GUARD_END
}

int gocp_hf_index(int n_qubits, int n_electrons, int mapping, uint64_t *index) {
    GOCP_GUARD_BEGIN
    if (!index) throw Error(GOCP_EINVAL, "null output");
    *index = hf_index(n_qubits, n_electrons, mapping);
    return GOCP_OK;
    GOCP_GUARD_END
}

}  // extern "C"
