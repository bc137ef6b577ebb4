"""Oracle pins of the GOCP multi-operator step: members of one commuting family
(Sec. III.A, Algorithm 1), each advanced by its own substepped O(5) chain
(Eq. 5-6), then one renormalisation.  Pinned to the exact exponential of the
sum of the members (they commute), to order independence, and to the single
operator chain."""

import math

import numpy as np
import pytest
from scipy.linalg import expm

from oracle.pauli import psum_matrix
from oracle.pool import pool_operators
from oracle.gocp import gocp_partition
from oracle.statevec import taylor5, taylor5_family, substeps


def _family_members(ops, nq, want):
    fam, fams, order, adj = gocp_partition(ops, nq)
    for F in fams:
        if len(F) >= want:
            return list(F[:want])
    pytest.skip("no family that large")


@pytest.mark.parametrize("mapping", ["jw", "bk"])
@pytest.mark.parametrize("n", [2, 3, 4])
def test_family_step_matches_exponential_of_the_sum(mapping, n):
    nq, ne = 8, 4
    ops = [A for _, _, A in pool_operators(nq, ne, mapping)]
    mem = _family_members(ops, nq, n)
    rng = np.random.default_rng(40 + n)
    thetas = list(rng.uniform(-1.4, 1.4, n))
    psi = rng.standard_normal(1 << nq) + 1j * rng.standard_normal(1 << nq)
    psi /= np.linalg.norm(psi)
    mats = [psum_matrix(ops[j], nq) for j in mem]
    for a in mats:
        for b in mats:
            assert np.abs(a @ b - b @ a).max() < 1e-14       # one family commutes
    out, subs = taylor5_family([ops[j] for j in mem], thetas, psi)
    assert subs == [substeps(t, sum(abs(c) for c in ops[j].values())) for t, j in zip(thetas, mem)]
    ref = expm(sum(t * m for t, m in zip(thetas, mats))) @ psi
    ref /= np.linalg.norm(ref)
    # each chain misses at most s e^x x^6 / 6! of its exponential (||A|| = 1
    # for a generator with A^3 = -A); the renormalisation at most doubles it
    bound = 2 * sum(s * math.exp(abs(t) / s) * (abs(t) / s) ** 6 / 720 for t, s in zip(thetas, subs))
    err = np.abs(out - ref).max()
    assert err <= bound
    assert err > 1e-4 * bound


def test_family_step_is_order_free_and_reduces_to_one_chain():
    nq, ne = 8, 4
    ops = [A for _, _, A in pool_operators(nq, ne, "jw")]
    mem = _family_members(ops, nq, 3)
    rng = np.random.default_rng(3)
    psi = rng.standard_normal(1 << nq) + 1j * rng.standard_normal(1 << nq)
    thetas = [0.7, -1.9, 0.25]
    a, _ = taylor5_family([ops[j] for j in mem], thetas, psi)
    b, _ = taylor5_family([ops[j] for j in mem[::-1]], thetas[::-1], psi)
    assert np.abs(a - b).max() < 1e-14
    one, s = taylor5_family([ops[mem[0]]], [thetas[0]], psi)
    ref, s2 = taylor5(ops[mem[0]], thetas[0], psi)
    assert s == [s2] and np.abs(one - ref).max() < 1e-15
