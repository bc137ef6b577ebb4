"""Greedy Operator Commutativity Partitioning (Sec. III.A, Algorithm 1).

Test infrastructure only.

Algorithm 1 first builds the non-commutativity graph: vertex j is pool
operator A_j and an edge joins i and j iff the operator commutator [A_i, A_j]
is not zero.  It then orders vertices by descending degree (Largest-First) and
puts each vertex, in that order, into the lowest-indexed family holding none
of its neighbours, opening a new family when none qualifies.

Readings where the paper is silent:

* the commutator is the exact operator commutator, evaluated in Pauli algebra
  with integer arithmetic: every pool coefficient is a multiple of i/8, so
  coefficients scaled by 8 are Gaussian integers and cancellation is exact;
* ties in degree keep ascending pool index (a stable sort);
* families are numbered in creation order.
"""

from __future__ import annotations

import numpy as np

from .pauli import string_products, string_product

__all__ = ["scaled_integer_terms", "commutes_slow", "conflict_graph",
           "largest_first_order", "greedy_families", "gocp_partition"]

_IPOW_INT = [(1, 0), (0, 1), (-1, 0), (0, -1)]   # i^k as (re, im)


def scaled_integer_terms(A: dict):
    """Strings of A with coefficients * 8 as exact integer pairs (re, im)."""
    out = []
    for (x, z), c in A.items():
        re, im = c.real * 8.0, c.imag * 8.0
        if re != round(re) or im != round(im):
            raise ValueError("pool coefficient is not a multiple of 1/8")
        out.append((x, z, int(round(re)), int(round(im))))
    return out


def _gmul(a, b):
    return (a[0] * b[0] - a[1] * b[1], a[0] * b[1] + a[1] * b[0])


def commutes_slow(A: dict, B: dict, N: int) -> bool:
    """[A, B] == 0 by expanding AB - BA string by string (small cases)."""
    acc = {}
    for (xa, za, ra, ia) in scaled_integer_terms(A):
        for (xb, zb, rb, ib) in scaled_integer_terms(B):
            c = _gmul((ra, ia), (rb, ib))
            k1, x, z = string_product(xa, za, xb, zb, N)
            k2, _, _ = string_product(xb, zb, xa, za, N)
            t1 = _gmul(c, _IPOW_INT[k1])
            t2 = _gmul(c, _IPOW_INT[k2])
            r, i = acc.get((x, z), (0, 0))
            acc[(x, z)] = (r + t1[0] - t2[0], i + t1[1] - t2[1])
    return all(v == (0, 0) for v in acc.values())


def conflict_graph(ops, N: int) -> np.ndarray:
    """Boolean adjacency matrix: adj[i, j] iff [A_i, A_j] != 0 (i != j).

    Same expansion as ``commutes_slow`` (every string pair, both orders, exact
    Gaussian-integer coefficients, like strings combined), evaluated for
    operator i against all operators j > i at once.
    """
    if N > 16:
        raise ValueError("oracle conflict graph supports up to 16 qubits")
    M = len(ops)
    terms = [scaled_integer_terms(A) for A in ops]
    op_id = np.concatenate([np.full(len(t), j, dtype=np.int64) for j, t in enumerate(terms)])
    tx = np.array([s[0] for t in terms for s in t], dtype=np.int64)
    tz = np.array([s[1] for t in terms for s in t], dtype=np.int64)
    tr = np.array([s[2] for t in terms for s in t], dtype=np.int64)
    ti = np.array([s[3] for t in terms for s in t], dtype=np.int64)
    pr = np.array([p[0] for p in _IPOW_INT], dtype=np.int64)
    pi = np.array([p[1] for p in _IPOW_INT], dtype=np.int64)
    adj = np.zeros((M, M), dtype=bool)
    for i in range(M - 1):
        a_idx = np.nonzero(op_id == i)[0]
        b_idx = np.nonzero(op_id > i)[0]
        ia = np.repeat(a_idx, len(b_idx))
        ib = np.tile(b_idx, len(a_idx))
        k1, x, z = string_products(tx[ia], tz[ia], tx[ib], tz[ib], N)   # A_i A_j
        k2, _, _ = string_products(tx[ib], tz[ib], tx[ia], tz[ia], N)   # A_j A_i
        cr = tr[ia] * tr[ib] - ti[ia] * ti[ib]
        ci = tr[ia] * ti[ib] + ti[ia] * tr[ib]
        dr = pr[k1] - pr[k2]                     # i^k1 - i^k2
        di = pi[k1] - pi[k2]
        vr = cr * dr - ci * di
        vi = cr * di + ci * dr
        key = (op_id[ib] << 32) | (x << 16) | z
        uniq, inv = np.unique(key, return_inverse=True)
        sr = np.zeros(len(uniq), dtype=np.int64)
        si = np.zeros(len(uniq), dtype=np.int64)
        np.add.at(sr, inv, vr)
        np.add.at(si, inv, vi)
        nz = (sr != 0) | (si != 0)
        js = np.unique(uniq[nz] >> 32)
        adj[i, js] = True
        adj[js, i] = True
    return adj


def largest_first_order(adj: np.ndarray):
    """Vertices by descending degree, ties by ascending index (Largest-First, Algorithm 1)."""
    deg = adj.sum(axis=1)
    return sorted(range(adj.shape[0]), key=lambda v: (-int(deg[v]), v))


def greedy_families(adj: np.ndarray, order):
    """Algorithm 1 assignment: lowest-indexed family with no neighbour, else a new one."""
    families = []            # list of member lists, in creation order
    family_of = [-1] * adj.shape[0]
    for v in order:
        placed = False
        for k, fam in enumerate(families):
            if not any(adj[v, u] for u in fam):
                fam.append(v)
                family_of[v] = k
                placed = True
                break
        if not placed:
            families.append([v])
            family_of[v] = len(families) - 1
    return family_of, families


def gocp_partition(ops, N: int):
    """Returns (family_of, families, order, adjacency) for a list of Pauli sums."""
    adj = conflict_graph(ops, N)
    order = largest_first_order(adj)
    family_of, families = greedy_families(adj, order)
    return family_of, families, order, adj
