"""Fermion-to-qubit mappings and the qubit Hamiltonian (Sec. II.A, Eq. 2-3).

Test infrastructure only.

Readings where the paper is silent:

* Spin-orbitals are interleaved: spin-orbital / qubit ``2p + s`` is spatial
  orbital ``p`` with spin ``s`` (0 = alpha, 1 = beta).
* Jordan-Wigner: ``a_j^dagger = (X_j - i Y_j)/2 * Z_0 ... Z_{j-1}`` (Sec. II.A,
  first bullet: local occupation plus a parity string of weight O(N)).
* Bravyi-Kitaev (Sec. II.A, second bullet: a binary-tree parity encoding of
  weight O(log N)) is taken as the Fenwick-tree encoding, which for N = 2^k is
  the textbook BK transform and for other N its truncation.  Qubit ``j``
  stores the parity of occupations ``n_k`` with ``j - lowbit(j+1) < k <= j``.
  The ladder operators are written with the update, parity and flip sets of
  that tree; ``a_j^dagger = (X_U X_j Z_P - i X_U Y_j Z_R) / 2`` with
  ``R = P minus F``.
* Eq. 2 is in physicist notation, ``h_ijkl a_i^+ a_j^+ a_l a_k`` with
  ``h_ijkl = <ij|kl>``; integrals arrive in chemist notation ``(pq|rs)``, so
  ``<PQ|RS> = (pr|qs)`` when the spins of P, R and of Q, S agree, else 0.
* Terms whose accumulated coefficient has modulus below 1e-12 are dropped.
"""

from __future__ import annotations

import numpy as np

from .pauli import string_products, _IPOW

__all__ = ["lowbit", "update_set", "parity_set", "flip_set", "bk_matrix",
           "ladder_ops", "hamiltonian", "hf_occupation", "hf_index",
           "dense_ladder_occupation"]


def lowbit(i: int) -> int:
    return i & (-i)


def update_set(j: int, N: int):
    """Qubits k > j whose stored parity includes occupation n_j."""
    out = []
    i = j + 1 + lowbit(j + 1)          # 1-based Fenwick ancestors of node j+1
    while i <= N:
        out.append(i - 1)
        i += lowbit(i)
    return out


def parity_set(j: int, N: int):
    """Qubits whose stored parities sum to n_0 + ... + n_{j-1}."""
    out = []
    i = j                              # 1-based prefix [1..j]
    while i > 0:
        out.append(i - 1)
        i -= lowbit(i)
    return out


def flip_set(j: int, N: int):
    """Qubits k < j whose parities, added to qubit j's, give n_j (tree children)."""
    out = []
    node = j + 1
    c = node - 1
    while c > node - lowbit(node):
        out.append(c - 1)
        c -= lowbit(c)
    return out


def bk_matrix(N: int) -> np.ndarray:
    """beta[j, k] = 1 iff j - lowbit(j+1) < k <= j (b = beta n mod 2)."""
    beta = np.zeros((N, N), dtype=np.int64)
    for j in range(N):
        for k in range(N):
            if j - lowbit(j + 1) < k <= j:
                beta[j, k] = 1
    return beta


def _mask(bits) -> int:
    m = 0
    for b in bits:
        m |= 1 << b
    return m


def ladder_ops(N: int, mapping: str):
    """Return (create, annihilate): lists of Pauli sums, one per qubit."""
    create, annih = [], []
    for j in range(N):
        if mapping == "jw":
            low = (1 << j) - 1
            xs, zs_x, zs_y = 1 << j, low, low | (1 << j)
        elif mapping == "bk":
            U = _mask(update_set(j, N))
            P = _mask(parity_set(j, N))
            F = _mask(flip_set(j, N))
            R = P & ~F
            xs, zs_x, zs_y = U | (1 << j), P, R | (1 << j)
        else:
            raise ValueError(f"unknown mapping {mapping!r}")
        create.append({(xs, zs_x): 0.5 + 0j, (xs, zs_y): -0.5j})
        annih.append({(xs, zs_x): 0.5 + 0j, (xs, zs_y): 0.5j})
    return create, annih


def _products_of_sums(factor_lists, coefs, N):
    """Sum over rows r of coefs[r] * prod_f factor_lists[f][r] (Pauli sums).

    Each factor is a two-string Pauli sum; the product over F factors is expanded
    into all 2^F string products with the single-qubit phase table.
    Returns arrays (x, z, c) of all expanded terms (not yet combined).
    """
    rows = len(coefs)
    F = len(factor_lists)
    # per factor: arrays of shape (2, rows) for the two strings of each sum
    tabs = []
    for fl in factor_lists:
        items = [list(s.items()) for s in fl]
        fx = np.array([[it[p][0][0] for it in items] for p in (0, 1)], dtype=np.int64)
        fz = np.array([[it[p][0][1] for it in items] for p in (0, 1)], dtype=np.int64)
        fc = np.array([[it[p][1] for it in items] for p in (0, 1)], dtype=np.complex128)
        tabs.append((fx, fz, fc))
    xs_all, zs_all, cs_all = [], [], []
    for combo in range(1 << F):
        x = np.zeros(rows, dtype=np.int64)
        z = np.zeros(rows, dtype=np.int64)
        k = np.zeros(rows, dtype=np.int64)
        c = np.asarray(coefs, dtype=np.complex128).copy()
        for f in range(F):
            pick = (combo >> f) & 1
            fx, fz, fc = tabs[f][0][pick], tabs[f][1][pick], tabs[f][2][pick]
            kk, x, z = string_products(x, z, fx, fz, N)
            k = k + kk
            c = c * fc
        xs_all.append(x)
        zs_all.append(z)
        cs_all.append(c * _IPOW[k & 3])
    return np.concatenate(xs_all), np.concatenate(zs_all), np.concatenate(cs_all)


def _combine(x, z, c, tol):
    key = (x << 32) | z
    uniq, inv = np.unique(key, return_inverse=True)
    re = np.bincount(inv, weights=c.real, minlength=len(uniq))
    im = np.bincount(inv, weights=c.imag, minlength=len(uniq))
    out = {}
    for u, a, b in zip(uniq.tolist(), re.tolist(), im.tolist()):
        if abs(complex(a, b)) >= tol:
            out[(u >> 32, u & 0xFFFFFFFF)] = complex(a, b)
    return out


def hamiltonian(h1: np.ndarray, eri: np.ndarray, e_core: float, mapping: str,
                tol: float = 1e-12) -> dict:
    """Qubit Hamiltonian of Eq. 2 under JW or BK, as a Pauli sum (Eq. 3).

    ``H = e_core + sum_{PQ} h_PQ a_P^+ a_Q + 1/2 sum_{PQRS} <PQ|RS> a_P^+ a_Q^+ a_S a_R``
    over spin-orbitals, with ``h_PQ = h1[p, q]`` for equal spins.
    """
    n = h1.shape[0]
    N = 2 * n
    cre, ann = ladder_ops(N, mapping)
    xs, zs, cs = [], [], []

    # one-body
    f1, f2, co = [], [], []
    for P in range(N):
        for Q in range(N):
            if P % 2 != Q % 2:
                continue
            v = h1[P // 2, Q // 2]
            if v == 0.0:
                continue
            f1.append(cre[P]); f2.append(ann[Q]); co.append(v)
    if co:
        x, z, c = _products_of_sums([f1, f2], co, N)
        xs.append(x); zs.append(z); cs.append(c)

    # two-body
    g1, g2, g3, g4, co = [], [], [], [], []
    for P in range(N):
        for Q in range(N):
            if P == Q:
                continue
            for R in range(N):
                if R % 2 != P % 2:
                    continue
                for S in range(N):
                    if S == R or S % 2 != Q % 2:
                        continue
                    v = eri[P // 2, R // 2, Q // 2, S // 2]   # <PQ|RS> = (pr|qs)
                    if v == 0.0:
                        continue
                    g1.append(cre[P]); g2.append(cre[Q]); g3.append(ann[S]); g4.append(ann[R])
                    co.append(0.5 * v)
    if co:
        x, z, c = _products_of_sums([g1, g2, g3, g4], co, N)
        xs.append(x); zs.append(z); cs.append(c)

    xs.append(np.array([0], dtype=np.int64))
    zs.append(np.array([0], dtype=np.int64))
    cs.append(np.array([e_core], dtype=np.complex128))
    return _combine(np.concatenate(xs), np.concatenate(zs), np.concatenate(cs), tol)


def hf_occupation(N: int, n_electrons: int) -> int:
    """Occupation bitstring of the reference state: lowest n_e spin-orbitals."""
    return (1 << n_electrons) - 1


def hf_index(N: int, n_electrons: int, mapping: str) -> int:
    """Basis index of the Hartree-Fock reference (Sec. II, reference state)."""
    occ = hf_occupation(N, n_electrons)
    if mapping == "jw":
        return occ
    beta = bk_matrix(N)
    nvec = np.array([(occ >> k) & 1 for k in range(N)], dtype=np.int64)
    b = beta.dot(nvec) & 1
    return int(sum(int(b[j]) << j for j in range(N)))


def dense_ladder_occupation(N: int):
    """Dense annihilation matrices from the occupation-number definition.

    ``a_p |n> = n_p (-1)^{n_0+...+n_{p-1}} |n - e_p>`` on the 2^N occupation basis.
    Used only to pin the Pauli forms on small registers.
    """
    dim = 1 << N
    out = []
    for p in range(N):
        a = np.zeros((dim, dim), dtype=np.complex128)
        for n_ in range(dim):
            if (n_ >> p) & 1:
                sign = -1.0 if bin(n_ & ((1 << p) - 1)).count("1") % 2 else 1.0
                a[n_ ^ (1 << p), n_] = sign
        out.append(a)
    return out
