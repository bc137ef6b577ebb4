"""Operator pool: spin-conserving occupied-to-virtual singles and doubles.

Test infrastructure only.

The paper's pool sizes (Table II: 92 operators for the 12-qubit water register,
204 for the 14-qubit BeH2 register) are reproduced by spin-orbital,
spin-conserving, occupied -> virtual singles and doubles that are neither spin
adapted nor generalised (92 = 8 electrons in 12 spin-orbitals, 204 = 6
electrons in 14).  Readings where the paper is silent:

* occupied spin-orbitals are 0 .. n_e-1 (interleaved spins), virtuals the rest;
* singles ``tau = a_a^+ a_i`` (same spin), doubles
  ``tau = a_a^+ a_b^+ a_j a_i`` with ``i < j`` occupied, ``a < b`` virtual and
  equal total S_z; the generator is ``A = tau - tau^+`` (anti-Hermitian, so
  ``exp(theta A)`` is the unitary rotation of Sec. III.B);
* order: all singles by ``(i, a)``, then all doubles by ``(i, j, a, b)``; the
  pool index is the position in that order.
"""

from __future__ import annotations

from .pauli import psum_mul, psum_add, psum_dagger, psum_clean
from .mapping import ladder_ops

__all__ = ["pool_excitations", "pool_operators", "pauli_pool_operators"]


def pool_excitations(N: int, n_electrons: int):
    """List of (kind, indices): kind 1 = single (i, a), 2 = double (i, j, a, b)."""
    occ = list(range(n_electrons))
    vir = list(range(n_electrons, N))
    out = []
    for i in occ:
        for a in vir:
            if i % 2 == a % 2:
                out.append((1, (i, a)))
    for i in occ:
        for j in occ:
            if j <= i:
                continue
            for a in vir:
                for b in vir:
                    if b <= a:
                        continue
                    if (i % 2) + (j % 2) == (a % 2) + (b % 2):
                        out.append((2, (i, j, a, b)))
    return out


def pool_operators(N: int, n_electrons: int, mapping: str):
    """Pauli sums of ``A_k = tau_k - tau_k^+`` in pool order."""
    cre, ann = ladder_ops(N, mapping)
    ops = []
    for kind, idx in pool_excitations(N, n_electrons):
        if kind == 1:
            i, a = idx
            tau = psum_mul(cre[a], ann[i], N)
        else:
            i, j, a, b = idx
            tau = psum_mul(psum_mul(psum_mul(cre[a], cre[b], N), ann[j], N), ann[i], N)
        A = psum_clean(psum_add(tau, psum_dagger(tau), -1.0))
        ops.append((kind, idx, A))
    return ops


def pauli_pool_operators(N: int, n_electrons: int, mapping: str):
    """Pauli (qubit) pool: every string of every generator as its own operator.

    Not in the paper (its pool is the fermionic one of Table II); the reading
    here: the string ``c P(x, z)`` of ``A_k`` becomes ``B = (c / |c|) P(x, z)``.
    ``c`` is purely imaginary for an anti-Hermitian ``A_k`` and ``P`` is
    Hermitian, so ``B`` is anti-Hermitian and ``B^2 = -1``.  Order: generators
    in pool order, each one's strings by ascending ``(x, z)`` (one ``x`` per
    generator).  Entries ``(kind + 2, indices, B)``.
    """
    out = []
    for kind, idx, A in pool_operators(N, n_electrons, mapping):
        for (x, z) in sorted(A):
            c = A[(x, z)]
            out.append((kind + 2, idx, {(x, z): c / abs(c)}))
    return out

