"""Statevector operations of the hot path.  Test infrastructure only.

* ``apply_h`` / ``energy``: the Rayleigh quotient of Eq. 1, with ``H psi`` taken
  as the Pauli sum of Eq. 3 applied string by string.
* ``gradients``: Eq. 4, ``g_j = <psi|[H, A_j]|psi> / <psi|psi>``.  For an
  anti-Hermitian generator this equals ``2 Re <H psi | A_j psi> / <psi|psi>``,
  which is what is evaluated (the two forms are pinned against each other).
* ``select``: the operator with the largest gradient magnitude (Sec. II.B).
* ``taylor5``: the fifth-order Taylor propagator of Eq. 5-6, accumulated as a
  power sum over the chain ``v_n = A v_{n-1}``.
* ``line_search``: the step length for the newly appended operator.

Readings where the paper is silent:

* Selection ties: gradients whose magnitudes lie within a relative 1e-12 of the
  largest are tied (operators related by spin flip have equal gradients in
  exact arithmetic), and the lowest pool index among them wins.
* Substeps: ``s = max(1, ceil(|theta| * ||A||_1 / 0.5))`` Taylor steps of
  ``theta / s`` each, where ``||A||_1`` is the sum of the string coefficient
  moduli, so every step has ``|x| ||A|| <= 0.5``.  The state is renormalised
  once, after the whole chain.
* Line search: earlier parameters stay frozen and the new angle minimises the
  energy along ``exp(theta A)`` exactly.  Pool generators obey ``A^3 = -A``,
  so ``exp(theta A) psi = u + cos(theta) v + sin(theta) w`` with ``w = A psi``,
  ``v = -A w`` and ``u = psi - v``, which makes ``E(theta)`` a trigonometric
  polynomial in six real numbers ``a_xy = Re <x|H|y>``.  The angle is the first
  local minimum met when walking from 0 in the descent direction ``-sign(g)``:
  1-degree steps until the derivative changes sign, then 60 bisections; if no
  sign change is met within a full turn, the best of the sampled angles.
"""

from __future__ import annotations

import math

import numpy as np

from .pauli import apply_psum

__all__ = ["apply_h", "energy", "gradients", "gradients_commutator", "select",
           "substeps", "taylor5", "line_coefficients", "landscape",
           "landscape_derivative", "line_search", "hf_state", "TIE_RTOL", "taylor5_family"]

TIE_RTOL = 1e-12


def hf_state(n_qubits: int, index: int) -> np.ndarray:
    psi = np.zeros(1 << n_qubits, dtype=np.complex128)
    psi[index] = 1.0
    return psi


def apply_h(H: dict, psi: np.ndarray) -> np.ndarray:
    return apply_psum(H, psi)


def energy(H: dict, psi: np.ndarray, sigma: np.ndarray | None = None) -> float:
    """Eq. 1: ``<psi|H|psi> / <psi|psi>`` (real part; H is Hermitian)."""
    if sigma is None:
        sigma = apply_h(H, psi)
    return float(np.vdot(psi, sigma).real / np.vdot(psi, psi).real)


def gradients(ops, psi: np.ndarray, sigma: np.ndarray) -> np.ndarray:
    """``g_j = 2 Re <sigma | A_j psi> / <psi|psi>`` for every pool operator."""
    nrm = np.vdot(psi, psi).real
    return np.array([2.0 * np.vdot(sigma, apply_psum(A, psi)).real / nrm for A in ops])


def gradients_commutator(H: dict, ops, psi: np.ndarray) -> np.ndarray:
    """Eq. 4 literally: ``<psi|(H A_j - A_j H)|psi> / <psi|psi>``."""
    nrm = np.vdot(psi, psi).real
    hpsi = apply_psum(H, psi)
    out = []
    for A in ops:
        hapsi = apply_psum(H, apply_psum(A, psi))
        ahpsi = apply_psum(A, hpsi)
        out.append(np.vdot(psi, hapsi - ahpsi).real / nrm)
    return np.array(out)


def select(g: np.ndarray):
    """Returns (j*, |g|max, ||g||_2) with the tie reading of the module header."""
    a = np.abs(np.asarray(g, dtype=np.float64))
    gmax = float(a.max())
    thresh = gmax * (1.0 - TIE_RTOL)
    j = int(np.nonzero(a >= thresh)[0][0])
    return j, gmax, float(np.sqrt(np.sum(a * a)))


def substeps(theta: float, norm1: float) -> int:
    return max(1, int(math.ceil(abs(theta) * norm1 / 0.5)))


def taylor5(A: dict, theta: float, psi: np.ndarray, renormalize: bool = True):
    """Eq. 5-6 with the substep reading; returns (new psi, s)."""
    if theta == 0.0:
        return psi.copy(), 0
    norm1 = sum(abs(c) for c in A.values())
    s = substeps(theta, norm1)
    x = theta / s
    for _ in range(s):
        v = psi
        acc = psi.copy()
        c = 1.0
        for n in range(1, 6):
            v = apply_psum(A, v)          # v_n = A v_{n-1}
            c = c * x / n                 # x^n / n!
            acc = acc + c * v
        psi = acc
    if renormalize:
        psi = psi / math.sqrt(np.vdot(psi, psi).real)
    return psi, s


def taylor5_family(As, thetas, psi: np.ndarray):
    """GOCP multi-operator step: members of one commuting family (Sec. III.A)
    each advanced by its own substepped chain (Eq. 5-6) in the given order,
    then one renormalisation.  Returns (new psi, substeps per operator)."""
    subs = []
    for A, th in zip(As, thetas):
        psi, s = taylor5(A, th, psi, renormalize=False)
        subs.append(s)
    return psi / math.sqrt(np.vdot(psi, psi).real), subs


def line_coefficients(H: dict, A: dict, psi: np.ndarray, sigma: np.ndarray):
    """The six numbers ``a_uu, a_uv, a_uw, a_vv, a_vw, a_ww`` of the line search."""
    w = apply_psum(A, psi)
    v = -apply_psum(A, w)
    u = psi - v
    Hv = apply_h(H, v)
    Hw = apply_h(H, w)
    Hu = sigma - Hv
    re = lambda a, b: float(np.vdot(a, b).real)
    return (re(u, Hu), re(u, Hv), re(u, Hw), re(v, Hv), re(v, Hw), re(w, Hw))


def landscape(coef, theta: float) -> float:
    auu, auv, auw, avv, avw, aww = coef
    c, s = math.cos(theta), math.sin(theta)
    return (auu + 2.0 * auv * c + 2.0 * auw * s + avv * c * c
            + 2.0 * avw * s * c + aww * s * s)


def landscape_derivative(coef, theta: float) -> float:
    auu, auv, auw, avv, avw, aww = coef
    c, s = math.cos(theta), math.sin(theta)
    return (-2.0 * auv * s + 2.0 * auw * c - 2.0 * avv * s * c
            + 2.0 * avw * (c * c - s * s) + 2.0 * aww * s * c)


def line_search(coef, g: float) -> float:
    """First local minimum of E(theta) from 0 in the direction -sign(g)."""
    if g == 0.0:
        return 0.0
    d = -1.0 if g > 0 else 1.0
    step = math.pi / 180.0
    prev = 0.0
    for k in range(1, 361):
        th = d * k * step
        if d * landscape_derivative(coef, th) >= 0.0:
            lo, hi = prev, th
            for _ in range(60):
                mid = 0.5 * (lo + hi)
                if d * landscape_derivative(coef, mid) >= 0.0:
                    hi = mid
                else:
                    lo = mid
            return 0.5 * (lo + hi)
        prev = th
    ks = np.arange(1, 361)
    vals = [landscape(coef, d * k * step) for k in ks]
    return float(d * int(ks[int(np.argmin(vals))]) * step)
