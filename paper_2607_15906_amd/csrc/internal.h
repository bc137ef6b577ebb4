// Internal types of libgocp (host side).  Not part of the C ABI.
#pragma once

#include <cstdint>
#include <atomic>
#include <memory>
#include <mutex>
#include <stdexcept>
#include <string>
#include <vector>

#include "gocp.h"

namespace gocp {

constexpr int kMaxQubits = 30;
constexpr double kDropTol = 1e-12;

// Error carrying a C-ABI status code; converted at the ABI boundary.
struct Error : std::runtime_error {
    int code;
    Error(int c, const std::string &m) : std::runtime_error(m), code(c) {}
};

void set_last_error(const std::string &msg);

// A folded Pauli term c * Z^z X^x (see gocp.h).
struct Term {
    uint32_t x, z;
    double c;
};

struct DeviceHam;    // device copy of a Hamiltonian, defined in the HIP sources
struct DevicePool;   // device copy of a pool
struct TableImage;   // a handle's device tables laid out in one pinned host buffer

// Hamiltonian grouped by X mask.  Classes are sorted by x; strings within a
// class by z.  cls_off is CSR into str_z / str_c.
// Identity of a Hamiltonian or pool for caches keyed across calls (addresses
// can be reused after a free; these numbers are not).
inline uint64_t next_uid() {
    static std::atomic<uint64_t> n{0};
    return ++n;
}

struct Ham {
    uint64_t uid = next_uid();
    int n_qubits = 0;
    std::vector<uint32_t> cls_x;
    std::vector<int32_t> cls_off;
    std::vector<uint32_t> str_z;
    std::vector<double> str_c;
    // device copies, one per device ordinal (lazy, guarded by mu)
    mutable std::mutex mu;
    mutable std::vector<DeviceHam *> dev;
    mutable std::shared_ptr<TableImage> img;   // built on first device use (guarded by mu)
    int64_t n_terms() const { return (int64_t)str_z.size(); }
    int n_classes() const { return (int)cls_x.size(); }
};

struct Pool {
    uint64_t uid = next_uid();
    int n_qubits = 0, n_electrons = 0, mapping = 0;
    std::vector<int32_t> kind;            // 1 single, 2 double; 3, 4 one string of either
    std::vector<int32_t> idx;             // 4 per op (-1 padded)
    std::vector<uint32_t> op_x;           // X mask per op
    std::vector<int32_t> op_off;          // CSR into str_z / str_c
    std::vector<uint32_t> str_z;
    std::vector<double> str_c;
    std::vector<double> op_norm1;         // sum |c| per op
    // GOCP partition (computed at build time; immutable)
    std::vector<int32_t> family_of;
    std::vector<int32_t> order;
    std::vector<int32_t> fam_off;         // CSR over families
    std::vector<int32_t> fam_members;     // members in assignment order
    std::vector<int32_t> degree;
    int64_t n_edges = 0;
    mutable std::mutex mu;
    mutable std::vector<DevicePool *> dev;
    mutable std::shared_ptr<TableImage> img;   // built on first device use (guarded by mu)
    int n_ops() const { return (int)op_x.size(); }
};

// ---- host algorithms (host_mapping.cpp, host_gocp.cpp)
Ham *build_hamiltonian(int n_spatial, const double *h1, const double *eri, double e_core,
                       int mapping);
Ham *hamiltonian_from_terms(int n_qubits, const std::vector<Term> &terms);
// pauli: one operator per string of the generators (unit coefficients)
Pool *build_pool(int n_qubits, int n_electrons, int mapping, bool pauli = false);
uint64_t hf_index(int n_qubits, int n_electrons, int mapping);
// Decoding a basis index into spin-orbital occupations under an encoding:
// occupation bit j = parity(rows[j] & index) (JW: the index itself; BK: the
// rows of beta^{-1}, a non-local parity of several qubits).
std::vector<uint32_t> occupation_rows(int n_qubits, int mapping);
uint64_t basis_occupation(int n_qubits, int mapping, uint64_t index);
void partition_pool(Pool &p);   // fills family_of, order, fam_off, fam_members, degree

// device-side release hooks (defined in the HIP sources)
void release_device_ham(DeviceHam *d);
void release_device_pool(DevicePool *d);

}  // namespace gocp
