"""Oracle pins of the Pauli (qubit) pool: every string of every fermionic
generator as an operator of its own, with unit coefficient.

The paper's pool is the fermionic one (Sec. II.B, Table II); the Pauli pool is
the widening its gradient screen and Taylor chain take unchanged, because each
string of an anti-Hermitian generator is anti-Hermitian by itself and squares
to -1 (so the A^3 = -A identity of the line search holds).  The pins below tie
it to the fermionic pool (linearity of Eq. 4 in the operator), to dense
matrices, to the exact rotation cos(theta) + sin(theta) B, and to the textbook
commutation rule of two Pauli strings.
"""

import math

import numpy as np
import pytest
from scipy.linalg import expm

from oracle.pauli import psum_matrix, apply_psum
from oracle.mapping import hamiltonian, hf_index
from oracle.pool import pool_operators, pool_excitations, pauli_pool_operators
from oracle.gocp import conflict_graph
from oracle.statevec import apply_h, energy, gradients, taylor5, substeps, hf_state
from oracle.adapt import adapt_run
from workloads import molecular_integrals, electron_count


def _sector_state(nq, ne, rng):
    d = np.arange(1 << nq)
    mask = (np.bitwise_count(d) == ne) & (np.bitwise_count(d & 0x5555) == ne // 2)
    psi = np.where(mask, rng.standard_normal(1 << nq) + 1j * rng.standard_normal(1 << nq), 0.0)
    return psi / np.linalg.norm(psi)


@pytest.mark.parametrize("nq,ne", [(4, 2), (8, 4), (12, 6), (14, 6)])
@pytest.mark.parametrize("mapping", ["jw", "bk"])
def test_pauli_pool_is_the_split_fermionic_pool(nq, ne, mapping):
    fops = pool_operators(nq, ne, mapping)
    pops = pauli_pool_operators(nq, ne, mapping)
    n1 = sum(1 for k, _ in pool_excitations(nq, ne) if k == 1)
    n2 = len(fops) - n1
    assert len(pops) == 2 * n1 + 8 * n2
    i = 0
    for kind, idx, A in fops:
        # a single's strings carry |c| = 1/2, a double's 1/8 (JW; BK conjugates
        # by a Clifford map, which keeps magnitudes)
        mag = 0.5 if kind == 1 else 0.125
        kids = pops[i:i + len(A)]
        assert sorted(A) == [next(iter(B)) for _, _, B in kids]
        for (pk, pidx, B) in kids:
            (key, b), = B.items()
            assert pk == kind + 2 and pidx == idx
            assert abs(abs(A[key]) - mag) < 1e-15
            assert abs(b - A[key] / mag) < 1e-15
        i += len(A)
    assert i == len(pops)


@pytest.mark.parametrize("mapping", ["jw", "bk"])
def test_pauli_pool_operators_are_anti_hermitian_involutions(mapping):
    for nq, ne in [(4, 2), (6, 2)]:
        for _, _, B in pauli_pool_operators(nq, ne, mapping):
            m = psum_matrix(B, nq)
            assert np.abs(m + m.conj().T).max() < 1e-15
            assert np.abs(m @ m + np.eye(1 << nq)).max() < 1e-15


@pytest.mark.parametrize("mapping", ["jw", "bk"])
def test_fermionic_gradient_is_the_weighted_sum_of_string_gradients(mapping):
    """Eq. 4 is linear in the operator: g(A_k) = sum_s |c_s| g(B_s)."""
    nq = 8
    n = nq // 2
    ne = electron_count(n)
    h1, eri, ec = molecular_integrals(n, 8)
    H = hamiltonian(h1, eri, ec, mapping)
    psi = _sector_state(nq, ne, np.random.default_rng(5))
    sigma = apply_h(H, psi)
    fops = pool_operators(nq, ne, mapping)
    pops = pauli_pool_operators(nq, ne, mapping)
    gf = gradients([A for _, _, A in fops], psi, sigma)
    gp = gradients([B for _, _, B in pops], psi, sigma)
    i = 0
    for k, (_, _, A) in enumerate(fops):
        s = sum(abs(A[key]) * gp[i + t] for t, key in enumerate(sorted(A)))
        assert abs(s - gf[k]) < 1e-13
        i += len(A)
    # and the string gradients are the derivative of the exact rotation
    Hd = psum_matrix(H, nq)
    h = 1e-5
    for j in (0, 7, 40, len(pops) - 1):
        Bd = psum_matrix(pops[j][2], nq)
        e = lambda t: (lambda p: (p.conj() @ Hd @ p).real)(expm(t * Bd) @ psi)
        assert abs((e(h) - e(-h)) / (2 * h) - gp[j]) < 1e-8


@pytest.mark.parametrize("theta", [0.4, -1.3, 2.9])
def test_pauli_taylor_chain_within_its_bound_of_the_exact_rotation(theta):
    """B^2 = -1, so exp(theta B) = cos(theta) + sin(theta) B; each O(5) substep
    of x = theta / s misses the tail of the exponential series, at most
    e^|x| |x|^6 / 6! per substep."""
    nq, ne = 10, 4
    pops = pauli_pool_operators(nq, ne, "jw")
    psi = _sector_state(nq, ne, np.random.default_rng(11))
    for j in (3, 100, len(pops) - 1):
        B = pops[j][2]
        out, s = taylor5(B, theta, psi, renormalize=False)
        assert s == substeps(theta, 1.0) == max(1, math.ceil(abs(theta) / 0.5))
        ref = math.cos(theta) * psi + math.sin(theta) * apply_psum(B, psi)
        x = abs(theta) / s
        bound = s * math.exp(x) * x ** 6 / 720.0
        err = np.abs(out - ref).max()
        assert err <= bound
        assert err > 1e-3 * bound          # the truncation is there, not hidden


@pytest.mark.parametrize("mapping", ["jw", "bk"])
def test_pauli_conflict_graph_is_the_symplectic_form(mapping):
    """Two Pauli strings commute iff popcount(x1 & z2) + popcount(z1 & x2) is even."""
    nq, ne = 8, 4
    pops = pauli_pool_operators(nq, ne, mapping)
    adj = conflict_graph([B for _, _, B in pops], nq)
    keys = [next(iter(B)) for _, _, B in pops]
    for a, (x1, z1) in enumerate(keys):
        for b, (x2, z2) in enumerate(keys):
            anti = (bin(x1 & z2).count("1") + bin(z1 & x2).count("1")) & 1
            assert bool(adj[a, b]) == (a != b and bool(anti))


def test_pauli_pool_adapt_is_variational_and_descends():
    """ADAPT over the Pauli pool: energies fall monotonically and stay above
    the lowest eigenvalue of H over the whole Fock space (the strings need not
    conserve the particle number)."""
    nq = 4
    n = nq // 2
    ne = electron_count(n)
    h1, eri, ec = molecular_integrals(n, 4)
    H = hamiltonian(h1, eri, ec, "jw")
    pops = [B for _, _, B in pauli_pool_operators(nq, ne, "jw")]
    psi0 = hf_state(nq, hf_index(nq, ne, "jw"))
    r = adapt_run(H, pops, psi0, max_iter=8)
    e = np.asarray(r["energies"])
    assert np.all(np.diff(e) <= 1e-12)
    emin = np.linalg.eigvalsh(psum_matrix(H, nq)).min()
    assert e.min() >= emin - 1e-12
    assert e[-1] < energy(H, psi0) - 1e-4
