"""The sparse-matrix CPU baseline (oracle/sparse.py) against the plain oracle:
each Pauli sum's CSR matrix equals the string-by-string application and the
dense Kronecker matrix, and the ADAPT run on the matrices follows the oracle's
run (same operators, energies to rounding)."""

import numpy as np
import pytest

from oracle.pauli import apply_psum, psum_matrix
from oracle.mapping import hamiltonian, hf_index
from oracle.pool import pool_operators
from oracle.statevec import hf_state
from oracle.adapt import adapt_run
from oracle.sparse import psum_csr, adapt_run_csr
from workloads import molecular_integrals, electron_count


def _system(nq, mapping):
    n = nq // 2
    ne = electron_count(n)
    h1, eri, ec = molecular_integrals(n, nq)
    H = hamiltonian(h1, eri, ec, mapping)
    ops = [A for _, _, A in pool_operators(nq, ne, mapping)]
    return H, ops, hf_state(nq, hf_index(nq, ne, mapping))


@pytest.mark.parametrize("mapping", ["jw", "bk"])
def test_csr_matrices_equal_string_application_and_dense(mapping):
    nq = 6
    H, ops, _ = _system(nq, mapping)
    rng = np.random.default_rng(3)
    psi = rng.standard_normal(1 << nq) + 1j * rng.standard_normal(1 << nq)
    for ps in [H] + ops[:5]:
        M = psum_csr(ps, nq)
        assert np.abs(M @ psi - apply_psum(ps, psi)).max() < 1e-12
        assert np.abs(M.toarray() - psum_matrix(ps, nq)).max() < 1e-12
    # one nonzero per row and X mask at most
    xs = {x for (x, _) in H}
    assert psum_csr(H, nq).nnz <= len(xs) << nq


@pytest.mark.parametrize("nq,mapping", [(8, "jw"), (8, "bk")])
def test_sparse_adapt_follows_the_oracle(nq, mapping):
    H, ops, hf = _system(nq, mapping)
    o = adapt_run(H, ops, hf, 10)
    Hm = psum_csr(H, nq)
    r = adapt_run_csr(Hm, [psum_csr(A, nq) for A in ops], [sum(abs(c) for c in A.values()) for A in ops], hf, 10)
    assert r["ops"] == o["ops"]
    assert r["substeps"] == o["substeps"]
    assert np.abs(np.array(r["energies"]) - np.array(o["energies"])).max() < 1e-12
    assert np.abs(np.array(r["thetas"]) - np.array(o["thetas"])).max() < 1e-10
    assert abs(abs(np.vdot(r["psi"], o["psi"])) - 1.0) < 1e-12
