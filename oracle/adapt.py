"""The ADAPT growth loop (Sec. II.B, Eq. 4; state update Sec. III.B).

Test infrastructure only.

One iteration: gradients of every pool operator at the current state (Eq. 4),
selection by largest magnitude, convergence test, line search for the new
angle, the O(5) Taylor update of the state (Eq. 5-6), and the new energy
(Eq. 1).  The loop starts from the Hartree-Fock reference.

Readings where the paper is silent: convergence when ``||g||_2 < grad_tol``
(checked before an operator is appended), otherwise stop after ``max_iter``
appended operators; an operator may be selected again (it then adds a layer).
"""

from __future__ import annotations

import math

import numpy as np

from .statevec import (apply_h, energy, gradients, select, line_coefficients,
                       line_search, taylor5, landscape)

__all__ = ["adapt_run"]


def adapt_run(H: dict, ops, psi0: np.ndarray, max_iter: int, grad_tol: float = 0.0,
              forced_ops=None, keep_gradients: bool = False):
    """Run ADAPT; ``ops`` is the list of pool Pauli sums in pool order.

    ``forced_ops`` (optional list of pool indices) overrides the selection at
    each iteration, for comparisons that must follow another run's choices.
    Returns a dict with ``energies`` (E_0 .. E_n), ``ops``, ``thetas``,
    ``gnorms`` (one per gradient screen), ``substeps``, ``predicted`` (the
    exact-exponential energy at the chosen angle), ``converged`` and ``psi``.
    """
    psi = psi0 / math.sqrt(np.vdot(psi0, psi0).real)
    sigma = apply_h(H, psi)
    out = dict(energies=[energy(H, psi, sigma)], ops=[], thetas=[], gnorms=[],
               gmax=[], substeps=[], predicted=[], converged=False, grads=[])
    for it in range(max_iter):
        g = gradients(ops, psi, sigma)
        j, gmax, gn = select(g)
        out["gnorms"].append(gn)
        out["gmax"].append(gmax)
        if keep_gradients:
            out["grads"].append(g)
        if gn < grad_tol:
            out["converged"] = True
            break
        if forced_ops is not None:
            j = int(forced_ops[it])
        A = ops[j]
        coef = line_coefficients(H, A, psi, sigma)
        theta = line_search(coef, float(g[j]))
        psi, s = taylor5(A, theta, psi)
        sigma = apply_h(H, psi)
        out["ops"].append(j)
        out["thetas"].append(theta)
        out["substeps"].append(s)
        out["predicted"].append(landscape(coef, theta))
        out["energies"].append(energy(H, psi, sigma))
    out["psi"] = psi
    return out
