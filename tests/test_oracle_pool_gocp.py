"""Pins of the oracle's pool (Table II) and GOCP partition (Sec. III.A, Algorithm 1)."""

import json
import os

import networkx as nx
import numpy as np
import pytest

from oracle.pauli import psum_matrix, to_folded
from oracle.pool import pool_excitations, pool_operators
from oracle.gocp import (gocp_partition, conflict_graph, commutes_slow,
                         largest_first_order, greedy_families)
from oracle.mapping import bk_matrix

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _gold(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def test_table2_pool_sizes():
    g = _gold("paper_values.json")
    for key in ("pool_size_h2o_12q", "pool_size_beh2_14q"):
        e = g[key]
        assert len(pool_excitations(e["n_qubits"], e["n_electrons"])) == e["value"]


@pytest.mark.parametrize("nq,ne,M", [(4, 2, 3), (8, 4, 26), (10, 4, 54), (12, 6, 117),
                                     (14, 6, 204), (16, 8, 360)])
def test_pool_size_closed_form(nq, ne, M):
    o, v = ne // 2, (nq - ne) // 2          # spatial occupied / virtual per spin
    closed = 2 * o * v + 2 * (o * (o - 1) // 2) * (v * (v - 1) // 2) + (o * v) ** 2
    assert len(pool_excitations(nq, ne)) == closed == M


@pytest.mark.parametrize("mapping", ["jw", "bk"])
def test_pool_string_structure(mapping):
    nq, ne = 12, 6
    for kind, idx, A in pool_operators(nq, ne, mapping):
        x, z, c = to_folded(A)
        assert len(x) == (2 if kind == 1 else 8)
        assert len(set(x.tolist())) == 1                      # one X-mask per operator
        assert np.all(c.imag == 0.0)                          # real folded coefficients
        assert np.all(np.abs(c.real) == (0.5 if kind == 1 else 0.125))
        assert abs(np.abs(c).sum() - 1.0) == 0.0              # ||A||_1 = 1
        assert np.all((np.bitwise_count(x & z) & 1) == 1)    # odd Y count: antisymmetric
        if mapping == "jw":
            assert int(x[0]) == sum(1 << q for q in idx)


def test_pool_generators_dense_properties():
    nq, ne = 8, 4
    d = np.arange(1 << nq)
    Nop = np.diag(np.bitwise_count(d).astype(float))
    Sz = np.diag((np.bitwise_count(d & 0x55) - np.bitwise_count(d & 0xAA)).astype(float))
    for kind, idx, A in pool_operators(nq, ne, "jw"):
        Ad = psum_matrix(A, nq)
        assert np.array_equal(Ad, -Ad.conj().T)               # anti-Hermitian
        assert np.abs(Ad @ Ad @ Ad + Ad).max() == 0.0          # A^3 = -A
        assert np.abs(Ad @ Nop - Nop @ Ad).max() == 0.0
        assert np.abs(Ad @ Sz - Sz @ Ad).max() == 0.0


def test_bk_pool_is_conjugated_jw_pool():
    nq, ne = 6, 2
    beta = bk_matrix(nq)
    dim = 1 << nq
    U = np.zeros((dim, dim))
    for n_ in range(dim):
        b = beta.dot(np.array([(n_ >> k) & 1 for k in range(nq)])) & 1
        U[int(sum(int(b[j]) << j for j in range(nq))), n_] = 1.0
    pj = pool_operators(nq, ne, "jw")
    pb = pool_operators(nq, ne, "bk")
    for (_, _, Aj), (_, _, Ab) in zip(pj, pb):
        assert np.allclose(psum_matrix(Ab, nq), U @ psum_matrix(Aj, nq) @ U.T, atol=0)


# ---------------------------------------------------------------- GOCP

def test_gocp_worked_example_4q():
    g = _gold("gocp_4q_worked_example.json")
    ex = pool_excitations(4, 2)
    assert [[k, list(i)] for k, i in ex] == g["pool"]
    ops = [A for _, _, A in pool_operators(4, 2, "jw")]
    family_of, families, order, adj = gocp_partition(ops, 4)
    edges = sorted([i, j] for i in range(3) for j in range(i + 1, 3) if adj[i, j])
    assert edges == g["edges"]
    assert adj.sum(axis=1).tolist() == g["degrees"]
    assert order == g["largest_first_order"]
    assert family_of == g["family_of"]
    assert len(families) == g["n_families"]


@pytest.mark.parametrize("mapping", ["jw", "bk"])
def test_conflict_graph_equals_stringwise_expansion(mapping):
    ops = [A for _, _, A in pool_operators(8, 4, mapping)]
    adj = conflict_graph(ops, 8)
    for i in range(len(ops)):
        for j in range(i + 1, len(ops)):
            assert adj[i, j] == (not commutes_slow(ops[i], ops[j], 8))


def test_conflict_graph_equals_dense_commutators():
    nq = 8
    ops = [A for _, _, A in pool_operators(nq, 4, "jw")]
    mats = [np.rint(8 * psum_matrix(A, nq).real).astype(np.int64) for A in ops]
    for A, m in zip(ops, mats):
        assert np.array_equal(8 * psum_matrix(A, nq).real, m)   # exact integer matrices
    adj = conflict_graph(ops, nq)
    for i in range(len(ops)):
        for j in range(i + 1, len(ops)):
            comm = mats[i] @ mats[j] - mats[j] @ mats[i]
            assert adj[i, j] == bool(np.any(comm != 0))


@pytest.mark.parametrize("nq,ne", [(8, 4), (12, 6), (14, 6)])
def test_partition_matches_networkx_largest_first(nq, ne):
    ops = [A for _, _, A in pool_operators(nq, ne, "jw")]
    family_of, families, order, adj = gocp_partition(ops, nq)
    G = nx.Graph()
    G.add_nodes_from(range(len(ops)))              # insertion order = pool order
    G.add_edges_from((i, j) for i in range(len(ops)) for j in range(i + 1, len(ops)) if adj[i, j])
    col = nx.greedy_color(G, strategy="largest_first")
    assert [col[v] for v in range(len(ops))] == family_of


@pytest.mark.parametrize("nq,ne", [(8, 4), (12, 6), (14, 6)])
def test_partition_valid_and_bounded(nq, ne):
    ops = [A for _, _, A in pool_operators(nq, ne, "jw")]
    family_of, families, order, adj = gocp_partition(ops, nq)
    K = len(families)
    for fam in families:
        for a in fam:
            for b in fam:
                assert not adj[a, b]
    # Welsh-Powell bound for Largest-First colourings
    deg = adj.sum(axis=1)
    ds = sorted(deg.tolist(), reverse=True)
    assert K <= max(min(d + 1, i + 1) for i, d in enumerate(ds))
    # operators sharing a spin-orbital pairwise fail to commute: a clique
    ex = pool_excitations(nq, ne)
    for q in range(nq):
        members = [k for k, (_, idx) in enumerate(ex) if q in idx]
        for a in members:
            for b in members:
                if a != b:
                    assert adj[a, b]
        assert K >= len(members)


@pytest.mark.parametrize("nq,ne", [(8, 4), (12, 6), (14, 6)])
def test_partition_mapping_invariant(nq, ne):
    pj = gocp_partition([A for _, _, A in pool_operators(nq, ne, "jw")], nq)
    pb = gocp_partition([A for _, _, A in pool_operators(nq, ne, "bk")], nq)
    assert pj[0] == pb[0]
    assert np.array_equal(pj[3], pb[3])


def test_greedy_families_on_textbook_graph():
    # a 5-cycle needs 3 colours; Largest-First with ties by index gives 0,1,0,1,2
    adj = np.zeros((5, 5), dtype=bool)
    for i in range(5):
        adj[i, (i + 1) % 5] = adj[(i + 1) % 5, i] = True
    order = largest_first_order(adj)
    assert order == [0, 1, 2, 3, 4]
    fo, fams = greedy_families(adj, order)
    assert fo == [0, 1, 0, 1, 2]
