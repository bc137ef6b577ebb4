"""Synthetic molecular integrals standing in for the paper's molecules.

The paper's systems (BeH2 at 14 qubits, H2O at 12 qubits, LiH; Sec. IV, Tables
II-III) need electronic-structure integrals and geometries that are not
available here.  This module draws seeded real integrals with the structure a
molecular Hamiltonian has (Sec. II.A, Eq. 2):

* ``h1[p, q]``: real symmetric one-electron integrals over ``n`` spatial
  orbitals.  The diagonal is ``-1.5 + 0.5 p`` Ha, so the lowest orbitals are
  the occupied ones; off-diagonal couplings are ``0.1 * N(0,1) * d(p, q)`` with
  ``d(p, q) = 1 / (1 + |p - q|)``.
* ``eri[p, q, r, s] = (pq|rs)`` in chemist notation, built as a sum of ``n``
  symmetric rank-one factors ``(pq|rs) = sum_L B^L_pq B^L_rs`` with
  ``B^L_pq = 0.15 * N(0,1) * d(p, q)``.  The result has the eight-fold
  permutational symmetry of real orbitals and is positive semidefinite as an
  ``n^2 x n^2`` matrix, like a true Coulomb kernel.
* The core energy is 0.

With these constants the Hartree-Fock determinant is the lowest diagonal
element of the (N_e, S_z = 0) block and carries 0.90-0.99 of the weight of its
ground state, with correlation energies of 5-75 mHa at 4-14 qubits: the regime
of a molecule near equilibrium.

Each symmetry-equivalent entry of ``eri`` holds the very same double (it is
computed once per canonical quadruple and copied), so exact algebraic
cancellations stay exact in floating point.

Random draws are taken in a fixed documented order: ``h1`` off-diagonals for
``p < q`` in row-major order, then ``B^L_pq`` for ``L = 0..n-1`` and ``p <= q``
in row-major order.
"""

from __future__ import annotations

import numpy as np

__all__ = ["molecular_integrals", "electron_count"]


def _decay(n: int) -> np.ndarray:
    p = np.arange(n)
    return 1.0 / (1.0 + np.abs(p[:, None] - p[None, :]))


def molecular_integrals(n_spatial: int, seed: int):
    """Return ``(h1, eri, e_core)`` for ``n_spatial`` orbitals and ``seed``.

    ``h1`` has shape (n, n), ``eri`` has shape (n, n, n, n) in chemist order
    ``(pq|rs)``; both are float64 and C-contiguous.
    """
    n = int(n_spatial)
    if n < 1:
        raise ValueError("n_spatial must be >= 1")
    rng = np.random.default_rng(seed)
    d = _decay(n)

    h1 = np.zeros((n, n), dtype=np.float64)
    for p in range(n):
        h1[p, p] = -1.5 + 0.5 * p
    for p in range(n):
        for q in range(p + 1, n):
            v = 0.1 * rng.standard_normal() * d[p, q]
            h1[p, q] = v
            h1[q, p] = v

    B = np.zeros((n, n, n), dtype=np.float64)
    for L in range(n):
        for p in range(n):
            for q in range(p, n):
                v = 0.15 * rng.standard_normal() * d[p, q]
                B[L, p, q] = v
                B[L, q, p] = v

    eri = np.zeros((n, n, n, n), dtype=np.float64)
    pairs = [(p, q) for p in range(n) for q in range(p, n)]
    for a, (p, q) in enumerate(pairs):
        for (r, s) in pairs[a:]:
            v = float(np.dot(B[:, p, q], B[:, r, s]))
            for (i, j, k, l) in ((p, q, r, s), (q, p, r, s), (p, q, s, r), (q, p, s, r),
                                 (r, s, p, q), (s, r, p, q), (r, s, q, p), (s, r, q, p)):
                eri[i, j, k, l] = v
    return h1, eri, 0.0


def electron_count(n_spatial: int) -> int:
    """Closed-shell electron count used by every workload: ``2 * floor(n/2)``."""
    return 2 * (int(n_spatial) // 2)
