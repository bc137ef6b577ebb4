"""Pauli strings and Pauli sums (Sec. II.A, Eq. 3).  Test infrastructure only.

Conventions (the paper fixes none of them):

* Qubit ``q`` is bit ``q`` of a basis index; ``|1>`` means "occupied".
* A string is a pair of integer bit masks ``(x, z)``; on qubit ``q`` it acts as
  I, X, Z or Y for ``(x_q, z_q)`` = (0,0), (1,0), (0,1), (1,1).  Y is the usual
  ``[[0, -i], [i, 0]]`` and equals ``i X Z``.
* A Pauli sum is a dict ``{(x, z): complex coefficient}``.
* Dense matrices put qubit 0 rightmost: ``kron(P_{N-1}, ..., P_0)``.

Acting on a basis vector, ``P(x, z)`` sends ``|c>`` to
``i^{popcount(x&z)} (-1)^{popcount(c&z)} |c ^ x>``, so
``(P psi)[d] = (-i)^{popcount(x&z)} (-1)^{popcount(d&z)} psi[d ^ x]``.
"""

from __future__ import annotations

import numpy as np

__all__ = [
    "single_qubit_matrix", "string_matrix", "psum_matrix",
    "string_product", "string_products", "psum_mul", "psum_add", "psum_scale",
    "psum_clean", "psum_dagger", "apply_string", "apply_psum", "to_folded",
]

_I = np.eye(2, dtype=np.complex128)
_X = np.array([[0, 1], [1, 0]], dtype=np.complex128)
_Y = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
_Z = np.array([[1, 0], [0, -1]], dtype=np.complex128)

# code = x_bit | (z_bit << 1): 0 = I, 1 = X, 2 = Z, 3 = Y
_MATS = {0: _I, 1: _X, 2: _Z, 3: _Y}

# Single-qubit products sigma_a * sigma_b = i^k * sigma_c, tabulated as k.
# XY = iZ, YZ = iX, ZX = iY and the reversed orders carry -i (k = 3).
_PHASE = np.zeros((4, 4), dtype=np.int64)
for _a, _b, _k in ((1, 3, 1), (3, 1, 3),    # X Y = iZ,  Y X = -iZ
                   (3, 2, 1), (2, 3, 3),    # Y Z = iX,  Z Y = -iX
                   (2, 1, 1), (1, 2, 3)):   # Z X = iY,  X Z = -iY
    _PHASE[_a, _b] = _k
_IPOW = np.array([1, 1j, -1, -1j], dtype=np.complex128)


def single_qubit_matrix(code: int) -> np.ndarray:
    return _MATS[code]


def string_matrix(x: int, z: int, n: int) -> np.ndarray:
    """Dense 2^n x 2^n matrix of ``P(x, z)`` by Kronecker products."""
    m = np.ones((1, 1), dtype=np.complex128)
    for q in reversed(range(n)):
        code = ((x >> q) & 1) | (((z >> q) & 1) << 1)
        m = np.kron(m, _MATS[code])
    return m


def psum_matrix(ps: dict, n: int) -> np.ndarray:
    out = np.zeros((1 << n, 1 << n), dtype=np.complex128)
    for (x, z), c in ps.items():
        out += c * string_matrix(x, z, n)
    return out


def string_product(x1: int, z1: int, x2: int, z2: int, n: int):
    """``P(x1,z1) P(x2,z2) = i^k P(x1^x2, z1^z2)``; returns ``(k mod 4, x, z)``.

    Computed qubit by qubit from the single-qubit multiplication table.
    """
    k = 0
    for q in range(n):
        a = ((x1 >> q) & 1) | (((z1 >> q) & 1) << 1)
        b = ((x2 >> q) & 1) | (((z2 >> q) & 1) << 1)
        k += int(_PHASE[a, b])
    return k & 3, x1 ^ x2, z1 ^ z2


def string_products(x1, z1, x2, z2, n: int):
    """Element-wise ``string_product`` over integer arrays (same table)."""
    x1 = np.asarray(x1, dtype=np.int64)
    z1 = np.asarray(z1, dtype=np.int64)
    x2 = np.asarray(x2, dtype=np.int64)
    z2 = np.asarray(z2, dtype=np.int64)
    k = np.zeros(np.broadcast(x1, x2).shape, dtype=np.int64)
    for q in range(n):
        a = ((x1 >> q) & 1) | (((z1 >> q) & 1) << 1)
        b = ((x2 >> q) & 1) | (((z2 >> q) & 1) << 1)
        k += _PHASE[a, b]
    return k & 3, x1 ^ x2, z1 ^ z2


def psum_mul(A: dict, B: dict, n: int) -> dict:
    """Product of two Pauli sums, like terms combined (no dropping)."""
    out: dict = {}
    for (xa, za), ca in A.items():
        for (xb, zb), cb in B.items():
            k, x, z = string_product(xa, za, xb, zb, n)
            key = (x, z)
            out[key] = out.get(key, 0.0) + ca * cb * _IPOW[k]
    return out


def psum_add(A: dict, B: dict, scale_b: complex = 1.0) -> dict:
    out = dict(A)
    for key, c in B.items():
        out[key] = out.get(key, 0.0) + scale_b * c
    return out


def psum_scale(A: dict, s: complex) -> dict:
    return {k: s * c for k, c in A.items()}


def psum_dagger(A: dict) -> dict:
    """Hermitian conjugate: Pauli strings are Hermitian, so conjugate coefficients."""
    return {k: np.conj(c) for k, c in A.items()}


def psum_clean(A: dict, tol: float = 1e-12) -> dict:
    """Drop terms with ``|c| < tol`` (reading for exact cancellations in FP64)."""
    return {k: complex(c) for k, c in A.items() if abs(c) >= tol}


def apply_string(x: int, z: int, c: complex, psi: np.ndarray) -> np.ndarray:
    """``c * P(x, z) @ psi`` from the basis action stated in the module header."""
    d = np.arange(psi.shape[0], dtype=np.int64)
    y = bin(x & z).count("1")
    sign = 1.0 - 2.0 * (np.bitwise_count(d & z) & 1)
    return c * _IPOW[(-y) & 3] * sign * psi[d ^ x]


def apply_psum(ps: dict, psi: np.ndarray) -> np.ndarray:
    out = np.zeros_like(psi, dtype=np.complex128)
    for (x, z), c in ps.items():
        out += apply_string(x, z, c, psi)
    return out


def to_folded(ps: dict):
    """Arrays ``(x, z, c_folded)`` with ``c_folded = c * (-i)^{popcount(x&z)}``.

    ``c P(x, z) = c_folded * Z^z X^x``: the folded coefficient is the one that
    multiplies ``(-1)^{popcount(d&z)} psi[d ^ x]``.  Sorted by ``(x, z)``.
    """
    keys = sorted(ps.keys())
    x = np.array([k[0] for k in keys], dtype=np.int64)
    z = np.array([k[1] for k in keys], dtype=np.int64)
    c = np.array([ps[k] * _IPOW[(-bin(k[0] & k[1]).count("1")) & 3] for k in keys],
                 dtype=np.complex128)
    return x, z, c
