"""Pins of the oracle's Pauli algebra and fermion-to-qubit mappings (Sec. II.A)."""

import itertools
import json
import math
import os

import numpy as np
import pytest

from oracle.pauli import (string_matrix, string_product, string_products, apply_string,
                          psum_matrix, to_folded, _IPOW)
from oracle.mapping import (ladder_ops, hamiltonian, bk_matrix, hf_index,
                            dense_ladder_occupation, update_set, parity_set, flip_set)
from workloads import molecular_integrals, electron_count

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rng(seed=0):
    return np.random.default_rng(seed)


# ---------------------------------------------------------------- Pauli algebra

def test_string_product_matches_kronecker_matrices():
    rng = _rng(1)
    n = 4
    for _ in range(200):
        x1, z1, x2, z2 = (int(v) for v in rng.integers(0, 1 << n, size=4))
        k, x, z = string_product(x1, z1, x2, z2, n)
        lhs = string_matrix(x1, z1, n) @ string_matrix(x2, z2, n)
        rhs = _IPOW[k] * string_matrix(x, z, n)
        assert np.array_equal(lhs, rhs)


def test_vectorised_products_equal_scalar_products():
    rng = _rng(2)
    n = 9
    a = rng.integers(0, 1 << n, size=(4, 300))
    k, x, z = string_products(a[0], a[1], a[2], a[3], n)
    for i in range(300):
        assert (k[i], x[i], z[i]) == string_product(*(int(v) for v in a[:, i]), n)


def test_apply_string_matches_dense_matrix():
    rng = _rng(3)
    n = 5
    for _ in range(50):
        x, z = (int(v) for v in rng.integers(0, 1 << n, size=2))
        c = complex(rng.standard_normal(), rng.standard_normal())
        psi = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
        ref = c * (string_matrix(x, z, n) @ psi)
        assert np.allclose(apply_string(x, z, c, psi), ref, atol=1e-14)


# ---------------------------------------------------------------- ladder operators

@pytest.mark.parametrize("N", [1, 2, 3, 4, 5, 6])
def test_jw_ladder_equals_occupation_definition(N):
    cre, ann = ladder_ops(N, "jw")
    dense = dense_ladder_occupation(N)
    for p in range(N):
        assert np.allclose(psum_matrix(ann[p], N), dense[p], atol=1e-15)
        assert np.allclose(psum_matrix(cre[p], N), dense[p].conj().T, atol=1e-15)


def _bk_permutation(N):
    beta = bk_matrix(N)
    dim = 1 << N
    U = np.zeros((dim, dim))
    for n_ in range(dim):
        nv = np.array([(n_ >> k) & 1 for k in range(N)])
        b = beta.dot(nv) & 1
        U[int(sum(int(b[j]) << j for j in range(N))), n_] = 1.0
    return U


@pytest.mark.parametrize("N", [2, 3, 4, 5, 6, 7, 8])
def test_bk_ladder_equals_conjugated_occupation_definition(N):
    """BK operators are the occupation-basis ones carried to |beta n>."""
    U = _bk_permutation(N)
    cre, ann = ladder_ops(N, "bk")
    dense = dense_ladder_occupation(N)
    for p in range(N):
        assert np.allclose(psum_matrix(ann[p], N), U @ dense[p] @ U.T, atol=1e-15)


def test_bk_matrix_is_textbook_for_power_of_two():
    # the textbook 8-mode Bravyi-Kitaev matrix, lower-triangular with qubit 0 first
    ref = np.array([[1, 0, 0, 0, 0, 0, 0, 0],
                    [1, 1, 0, 0, 0, 0, 0, 0],
                    [0, 0, 1, 0, 0, 0, 0, 0],
                    [1, 1, 1, 1, 0, 0, 0, 0],
                    [0, 0, 0, 0, 1, 0, 0, 0],
                    [0, 0, 0, 0, 1, 1, 0, 0],
                    [0, 0, 0, 0, 0, 0, 1, 0],
                    [1, 1, 1, 1, 1, 1, 1, 1]])
    assert np.array_equal(bk_matrix(8), ref)
    # update / parity / flip sets of the 8-mode Fenwick tree
    assert update_set(4, 8) == [5, 7]
    assert parity_set(4, 8) == [3]
    assert flip_set(4, 8) == []
    assert flip_set(7, 8) == [6, 5, 3]


@pytest.mark.parametrize("N", [4, 6])
def test_canonical_anticommutation_bk(N):
    cre, ann = ladder_ops(N, "bk")
    A = [psum_matrix(a, N) for a in ann]
    for i in range(N):
        for j in range(N):
            ac = A[i] @ A[j].conj().T + A[j].conj().T @ A[i]
            assert np.allclose(ac, np.eye(1 << N) * (i == j), atol=1e-14)
            assert np.allclose(A[i] @ A[j] + A[j] @ A[i], 0, atol=1e-14)


# ---------------------------------------------------------------- Hamiltonian

def _dense_fermionic_h(h1, eri, e_core, N):
    """Eq. 2 from dense occupation-basis ladder matrices (no Pauli algebra)."""
    a = dense_ladder_occupation(N)
    ad = [m.conj().T for m in a]
    H = e_core * np.eye(1 << N, dtype=np.complex128)
    for P in range(N):
        for Q in range(N):
            if P % 2 == Q % 2:
                H += h1[P // 2, Q // 2] * ad[P] @ a[Q]
    for P, Q, R, S in itertools.product(range(N), repeat=4):
        if P % 2 == R % 2 and Q % 2 == S % 2:
            H += 0.5 * eri[P // 2, R // 2, Q // 2, S // 2] * ad[P] @ ad[Q] @ a[S] @ a[R]
    return H


@pytest.mark.parametrize("nq", [4, 6])
def test_jw_hamiltonian_equals_dense_fermionic_hamiltonian(nq):
    h1, eri, ec = molecular_integrals(nq // 2, 100 + nq)
    ec = 0.7
    Hp = psum_matrix(hamiltonian(h1, eri, ec, "jw"), nq)
    Hf = _dense_fermionic_h(h1, eri, ec, nq)
    assert np.allclose(Hp, Hf, atol=1e-13)


def test_bk_hamiltonian_is_conjugated_jw_and_isospectral():
    nq = 8
    h1, eri, ec = molecular_integrals(nq // 2, 8)
    Hj = psum_matrix(hamiltonian(h1, eri, ec, "jw"), nq)
    Hb = psum_matrix(hamiltonian(h1, eri, ec, "bk"), nq)
    U = _bk_permutation(nq)
    assert np.allclose(Hb, U @ Hj @ U.T, atol=1e-13)
    assert np.allclose(np.linalg.eigvalsh(Hj), np.linalg.eigvalsh(Hb), atol=1e-10)


@pytest.mark.parametrize("nq", [8, 12, 14])
def test_jw_bk_same_term_count_and_coefficient_multiset(nq):
    h1, eri, ec = molecular_integrals(nq // 2, nq)
    Hj = hamiltonian(h1, eri, ec, "jw")
    Hb = hamiltonian(h1, eri, ec, "bk")
    assert len(Hj) == len(Hb)
    cj = np.sort(np.round(np.abs(np.array(list(Hj.values()))), 12))
    cb = np.sort(np.round(np.abs(np.array(list(Hb.values()))), 12))
    assert np.allclose(cj, cb, atol=1e-12)
    # X-mask classes: same count
    assert len({k[0] for k in Hj}) == len({k[0] for k in Hb})


@pytest.mark.parametrize("mapping", ["jw", "bk"])
def test_hamiltonian_is_real_symmetric_in_folded_form(mapping):
    nq = 12
    h1, eri, ec = molecular_integrals(nq // 2, nq)
    x, z, c = to_folded(hamiltonian(h1, eri, ec, mapping))
    assert np.all(np.abs(c.imag) == 0.0)
    # real symmetric matrix => only strings with an even number of Y factors
    assert np.all((np.bitwise_count(x & z) & 1) == 0)


def test_hamiltonian_conserves_particle_number_and_sz():
    nq = 8
    h1, eri, ec = molecular_integrals(nq // 2, 8)
    H = psum_matrix(hamiltonian(h1, eri, ec, "jw"), nq)
    d = np.arange(1 << nq)
    Nop = np.diag(np.bitwise_count(d).astype(float))
    Sz = np.diag(0.5 * (np.bitwise_count(d & 0x55) - np.bitwise_count(d & 0xAA)).astype(float))
    assert np.abs(H @ Nop - Nop @ H).max() < 1e-13
    assert np.abs(H @ Sz - Sz @ H).max() < 1e-13


def _slater_condon_hf(h1, eri, e_core, n_e):
    occ = list(range(n_e))
    e = e_core + sum(h1[i // 2, i // 2] for i in occ)
    for i in occ:
        for j in occ:
            e += 0.5 * eri[i // 2, i // 2, j // 2, j // 2]
            if i % 2 == j % 2:
                e -= 0.5 * eri[i // 2, j // 2, j // 2, i // 2]
    return e


@pytest.mark.parametrize("nq", [4, 8, 12, 14])
@pytest.mark.parametrize("mapping", ["jw", "bk"])
def test_hf_energy_matches_slater_condon(nq, mapping):
    n = nq // 2
    ne = electron_count(n)
    h1, eri, ec = molecular_integrals(n, nq)
    H = hamiltonian(h1, eri, ec, mapping)
    hf = hf_index(nq, ne, mapping)
    # <hf|H|hf> = sum over diagonal (x = 0) strings of c * (-1)^{popcount(hf & z)}
    e = sum(c.real * (-1) ** bin(hf & z).count("1") for (x, z), c in H.items() if x == 0)
    assert abs(e - _slater_condon_hf(h1, eri, ec, ne)) < 1e-12


def test_table1_dense_arithmetic():
    with open(os.path.join(GOLDEN, "paper_values.json")) as f:
        gold = json.load(f)
    elems = (1 << 14) ** 2
    assert elems == 268435456
    assert abs(elems - gold["dense_elements_14q"]["value"]) / elems < gold["dense_elements_14q"]["rel_tol"]
    gb = elems * gold["dense_storage_gb_14q"]["bytes_per_element"] / 1e9
    assert abs(gb - gold["dense_storage_gb_14q"]["value"]) / gb < gold["dense_storage_gb_14q"]["rel_tol"]
    r = gold["rss_reduction_14q"]
    factor = gb * 1e3 / r["rss_mb"]
    assert abs(factor - r["factor"]) / r["factor"] < 0.05


def test_integral_fixture_symmetry():
    h1, eri, _ = molecular_integrals(5, 3)
    assert np.array_equal(h1, h1.T)
    for perm in [(1, 0, 2, 3), (0, 1, 3, 2), (2, 3, 0, 1), (3, 2, 1, 0)]:
        assert np.array_equal(eri, eri.transpose(perm))
    w = np.linalg.eigvalsh(eri.reshape(25, 25))
    assert w.min() > -1e-12
