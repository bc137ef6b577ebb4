"""ADAPT on precomputed sparse matrices: the CPU baseline in the style of the
paper's own engine (Sec. IV.C, which keeps the Hamiltonian and the pool as
sparse matrices and advances the state by sparse matrix-vector products).

Test and measurement infrastructure only (the bench's CPU baseline); checked
against the plain oracle.

Every Pauli sum becomes one CSR matrix over the 2^n basis: a string with X
mask x and Z mask z maps amplitude d ^ x into row d with the folded
coefficient times (-1)^popcount(d & z), and strings that share an X mask share
their nonzeros (one per row and X mask).  The iteration is the oracle's
(``adapt.py``): screen, selection, line search, substepped Taylor chain,
renormalisation, new energy, with every Pauli-sum application replaced by a
product with the corresponding matrix.
"""

from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp

from .pauli import to_folded
from .statevec import select, line_search, substeps

__all__ = ["psum_csr", "adapt_run_csr"]


def psum_csr(ps: dict, n_qubits: int) -> sp.csr_matrix:
    """The Pauli sum ``ps`` as a CSR matrix of size 2^n."""
    dim = 1 << n_qubits
    d = np.arange(dim, dtype=np.int64)
    x, z, c = to_folded(ps)
    rows, cols, vals = [], [], []
    for xv in np.unique(x):
        sel = x == xv
        f = np.zeros(dim, dtype=np.complex128)
        for zv, cv in zip(z[sel], c[sel]):
            f += cv * (1.0 - 2.0 * (np.bitwise_count(d & zv) & 1))
        keep = f != 0
        rows.append(d[keep])
        cols.append((d ^ xv)[keep])
        vals.append(f[keep])
    if not rows:
        return sp.csr_matrix((dim, dim), dtype=np.complex128)
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(dim, dim))


def _taylor5(Am: sp.csr_matrix, norm1: float, theta: float, psi: np.ndarray):
    """The oracle's substepped O(5) chain with matrix products; (psi, s)."""
    if theta == 0.0:
        return psi.copy(), 0
    s = substeps(theta, norm1)
    x = theta / s
    for _ in range(s):
        v = psi
        acc = psi.copy()
        c = 1.0
        for k in range(1, 6):
            v = Am @ v
            c = c * x / k
            acc = acc + c * v
        psi = acc
    return psi / math.sqrt(np.vdot(psi, psi).real), s


def adapt_run_csr(Hm: sp.csr_matrix, Ams, norms1, psi0: np.ndarray, max_iter: int, grad_tol: float = 0.0):
    """ADAPT with the Hamiltonian ``Hm`` and the pool ``Ams`` as sparse
    matrices (``norms1``: each generator's sum of string coefficient moduli,
    for the substep rule).  Returns the record of ``adapt.adapt_run``
    (energies, ops, thetas, gnorms, substeps, converged, psi)."""
    psi = psi0 / math.sqrt(np.vdot(psi0, psi0).real)
    sigma = Hm @ psi
    nrm = np.vdot(psi, psi).real
    out = dict(energies=[float(np.vdot(psi, sigma).real / nrm)], ops=[], thetas=[], gnorms=[], substeps=[],
               converged=False)
    for _ in range(max_iter):
        nrm = np.vdot(psi, psi).real
        g = np.array([2.0 * np.vdot(sigma, Am @ psi).real / nrm for Am in Ams])
        j, _, gn = select(g)
        out["gnorms"].append(gn)
        if gn < grad_tol:
            out["converged"] = True
            break
        Am = Ams[j]
        w = Am @ psi
        v = -(Am @ w)
        u = psi - v
        Hv = Hm @ v
        Hw = Hm @ w
        Hu = sigma - Hv
        re = lambda a, b: float(np.vdot(a, b).real)
        coef = (re(u, Hu), re(u, Hv), re(u, Hw), re(v, Hv), re(v, Hw), re(w, Hw))
        theta = line_search(coef, float(g[j]))
        psi, s = _taylor5(Am, norms1[j], theta, psi)
        sigma = Hm @ psi
        out["ops"].append(j)
        out["thetas"].append(theta)
        out["substeps"].append(s)
        out["energies"].append(float(np.vdot(psi, sigma).real / np.vdot(psi, psi).real))
    out["psi"] = psi
    return out
