"""ADAPT with full re-optimisation of every angle (textbook ADAPT; Sec. II.B).

Test infrastructure only.

After each operator is appended, all angles of the ansatz are optimised
together, instead of freezing the earlier ones (the reading of the frozen-angle
path in ``adapt.py``).  The ansatz state is the chain of layers of Eq. 5
applied to the reference,

    psi(theta) = L_k(theta_k) ... L_1(theta_1) psi_0,

each layer the substepped O(5) Taylor propagator of Eq. 6,
``L(A, theta) = T5(theta / s)^s`` with ``T5(x) = sum_{n<=5} x^n A^n / n!``.
The objective is the Rayleigh quotient of Eq. 1 of that state.

Readings where the paper is silent (it names neither the optimiser nor the
substep rule of a re-optimised layer):

* Substeps of a re-optimised layer: ``s = max(1, ceil(max(|theta|, pi) *
  ||A||_1 / 0.5))``.  The count is then constant for |theta| <= pi, so the
  energy is a smooth function of the angles there (with the frozen path's rule
  s would jump with |theta| and the energy with it, by the truncation error);
  every substep still has ``|x| ||A||_1 <= 0.5``.
* Gradient: the derivative of the energy, ``dE/dtheta_i = 2 Re <(H - E) psi |
  d psi / d theta_i> / <psi|psi>``, with ``d L / d theta = T5(x)^(s-1) A T4(x)``
  (the derivative of the truncated series itself, for constant s), so it is
  exact for the objective above and reduces to Eq. 4 for a new layer at 0.
* Optimiser: BFGS (inverse-Hessian form) from the previous angles and 0 for
  the new one; the search direction ``p = -Hinv g`` (reset to ``-g`` when it is
  not a descent direction), a backtracking line search from step 1 halving
  until ``E(x + t p) <= E(x) + 1e-4 t g.p + 1e-14 (1 + |E(x)|)`` (sufficient
  decrease, up to the rounding of E itself, which near the minimum is larger
  than the decrease a tiny gradient promises; at most 30 halvings), the
  update skipped when ``s.y <= 1e-12 |s| |y|``; stop when ``max |g| < gtol`` or
  after ``maxiter`` steps or when the line search fails.
* ADAPT loop: the screen (Eq. 4), the selection and the convergence test of
  ``adapt.py``, applied to the optimised state.
"""

from __future__ import annotations

import math

import numpy as np

from .pauli import apply_psum
from .statevec import apply_h, gradients, select

__all__ = ["reopt_substeps", "layer", "layer_derivative", "ansatz_state", "energy_and_gradient", "bfgs",
           "adapt_reopt_run", "BFGS_C1", "BFGS_FTOL", "BFGS_HALVINGS"]

BFGS_C1 = 1e-4
BFGS_FTOL = 1e-14       # relative rounding allowance of the sufficient-decrease test
BFGS_HALVINGS = 30


def reopt_substeps(theta: float, norm1: float) -> int:
    return max(1, int(math.ceil(max(abs(theta), math.pi) * norm1 / 0.5)))


def _norm1(A: dict) -> float:
    return sum(abs(c) for c in A.values())


def _t_series(A: dict, x: float, psi: np.ndarray, order: int) -> np.ndarray:
    """sum_{n <= order} x^n A^n psi / n!, as the power sum of Eq. 6."""
    v = psi
    acc = psi.copy()
    c = 1.0
    for n in range(1, order + 1):
        v = apply_psum(A, v)
        c = c * x / n
        acc = acc + c * v
    return acc


def layer(A: dict, theta: float, psi: np.ndarray) -> np.ndarray:
    """L(A, theta) psi = T5(theta/s)^s psi (no renormalisation)."""
    s = reopt_substeps(theta, _norm1(A))
    x = theta / s
    for _ in range(s):
        psi = _t_series(A, x, psi, 5)
    return psi


def layer_derivative(A: dict, theta: float, psi: np.ndarray) -> np.ndarray:
    """dL/dtheta psi = T5(x)^(s-1) A T4(x) psi, x = theta / s."""
    s = reopt_substeps(theta, _norm1(A))
    x = theta / s
    v = apply_psum(A, _t_series(A, x, psi, 4))
    for _ in range(s - 1):
        v = _t_series(A, x, v, 5)
    return v


def ansatz_state(layers, thetas, psi0: np.ndarray) -> np.ndarray:
    psi = psi0
    for A, th in zip(layers, thetas):
        psi = layer(A, th, psi)
    return psi


def energy_and_gradient(H: dict, layers, thetas, psi0: np.ndarray):
    """E(theta) and dE/dtheta_i for every layer, each derivative formed by the
    product rule on its own (the layers before i, the derivative of layer i,
    the layers after it)."""
    psi = ansatz_state(layers, thetas, psi0)
    sigma = apply_h(H, psi)
    nrm = np.vdot(psi, psi).real
    e = np.vdot(psi, sigma).real / nrm
    lam = sigma - e * psi
    grad = np.zeros(len(layers))
    for i in range(len(layers)):
        v = ansatz_state(layers[:i], thetas[:i], psi0)
        v = layer_derivative(layers[i], thetas[i], v)
        for A, th in zip(layers[i + 1:], thetas[i + 1:]):
            v = layer(A, th, v)
        grad[i] = 2.0 * np.vdot(lam, v).real / nrm
    return float(e), grad, psi


def bfgs(fg, x0, gtol: float = 1e-8, maxiter: int = 200):
    """Minimise f from x0 with the BFGS reading of the module header; fg(x)
    returns (f, grad).  Returns (x, f, grad, steps, evaluations)."""
    x = np.array(x0, dtype=np.float64)
    n = len(x)
    f, g = fg(x)
    nev = 1
    hinv = np.eye(n)
    it = 0
    while it < maxiter and np.max(np.abs(g)) >= gtol:
        p = -hinv @ g
        gp = float(g @ p)
        if not gp < 0.0:
            hinv = np.eye(n)
            p = -g
            gp = float(g @ p)
        t = 1.0
        ok = False
        for _ in range(BFGS_HALVINGS + 1):
            xn = x + t * p
            fn, gn = fg(xn)
            nev += 1
            if fn <= f + BFGS_C1 * t * gp + BFGS_FTOL * (1.0 + abs(f)):
                ok = True
                break
            t *= 0.5
        if not ok:
            break
        s = xn - x
        y = gn - g
        sy = float(s @ y)
        if sy > 1e-12 * math.sqrt(float(s @ s)) * math.sqrt(float(y @ y)):
            rho = 1.0 / sy
            i_n = np.eye(n)
            hinv = (i_n - rho * np.outer(s, y)) @ hinv @ (i_n - rho * np.outer(y, s)) + rho * np.outer(s, s)
        x, f, g = xn, fn, gn
        it += 1
    return x, float(f), g, it, nev


def adapt_reopt_run(H: dict, ops, psi0: np.ndarray, max_iter: int, grad_tol: float = 0.0,
                    bfgs_gtol: float = 1e-8, bfgs_maxiter: int = 200, forced_ops=None):
    """ADAPT with every angle re-optimised after each appended operator.

    Returns a dict with ``energies`` (E_0 .. E_n, each at the optimised
    angles), ``ops``, ``thetas`` (the final angles, one per layer),
    ``gnorms`` / ``gmax`` (one per screen), ``grads`` (the screens),
    ``bfgs_steps``, ``bfgs_evals``, ``converged`` and ``psi`` (normalised).
    """
    psi0 = psi0 / math.sqrt(np.vdot(psi0, psi0).real)
    psi = psi0
    sigma = apply_h(H, psi)
    e = float(np.vdot(psi, sigma).real)
    out = dict(energies=[e], ops=[], thetas=[], gnorms=[], gmax=[], grads=[], bfgs_steps=[], bfgs_evals=[],
               converged=False)
    layers, thetas = [], []
    for it in range(max_iter):
        g = gradients(ops, psi, sigma)
        j, gmax, gn = select(g)
        out["gnorms"].append(gn)
        out["gmax"].append(gmax)
        out["grads"].append(g)
        if gn < grad_tol:
            out["converged"] = True
            break
        if forced_ops is not None:
            j = int(forced_ops[it])
        layers.append(ops[j])
        out["ops"].append(j)
        x0 = list(thetas) + [0.0]

        def fg(x):
            ee, gg, _ = energy_and_gradient(H, layers, list(x), psi0)
            return ee, gg
        x, e, _, steps, nev = bfgs(fg, x0, bfgs_gtol, bfgs_maxiter)
        thetas = [float(t) for t in x]
        psi = ansatz_state(layers, thetas, psi0)
        psi = psi / math.sqrt(np.vdot(psi, psi).real)
        sigma = apply_h(H, psi)
        out["energies"].append(float(np.vdot(psi, sigma).real))
        out["bfgs_steps"].append(steps)
        out["bfgs_evals"].append(nev)
    out["thetas"] = thetas
    out["psi"] = psi
    return out
