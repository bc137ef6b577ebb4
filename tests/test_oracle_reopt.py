"""Pins of the re-optimisation oracle (ADAPT with every angle optimised by
BFGS; oracle/reopt.py): the layer against its closed form and the exact
exponential, its derivative and the energy gradient against central
differences, the gradient of a new layer at zero against Eq. 4, BFGS against
closed-form minima and scipy's BFGS, and the loop against exact
diagonalisation and the JW/BK equivalence."""

import math

import numpy as np
import pytest
from scipy.linalg import expm
from scipy.optimize import minimize

from oracle.pauli import psum_matrix, apply_psum
from oracle.mapping import hamiltonian, hf_index
from oracle.pool import pool_operators
from oracle.statevec import apply_h, gradients, hf_state
from oracle.adapt import adapt_run
from oracle.reopt import (reopt_substeps, layer, layer_derivative, ansatz_state, energy_and_gradient, bfgs,
                          adapt_reopt_run)
from workloads import molecular_integrals, electron_count


def _system(nq, mapping="jw"):
    n = nq // 2
    ne = electron_count(n)
    h1, eri, ec = molecular_integrals(n, nq)
    H = hamiltonian(h1, eri, ec, mapping)
    ops = [A for _, _, A in pool_operators(nq, ne, mapping)]
    return H, ops, hf_state(nq, hf_index(nq, ne, mapping)), ne


def _sector_state(nq, ne, seed):
    rng = np.random.default_rng(seed)
    d = np.arange(1 << nq)
    mask = (np.bitwise_count(d) == ne) & (np.bitwise_count(d & 0x5555) == ne // 2)
    psi = np.where(mask, rng.standard_normal(1 << nq), 0.0).astype(np.complex128)
    return psi / np.linalg.norm(psi)


def _sector_fci(H, nq, ne):
    d = np.arange(1 << nq)
    idx = np.nonzero((np.bitwise_count(d) == ne) & (np.bitwise_count(d & 0x5555) == ne // 2))[0]
    Hd = psum_matrix(H, nq)
    return np.linalg.eigvalsh(Hd[np.ix_(idx, idx)].real)[0]


@pytest.mark.parametrize("theta", [0.3, -1.1, 2.9, -3.7, 5.0])
def test_layer_matches_closed_form_and_exponential(theta):
    """With A^3 = -A, T5(x) = I + b(x) A + c(x) A^2 with b = x - x^3/6 +
    x^5/120 and c = x^2/2 - x^4/24, so the s-fold chain is I + Im(z^s) A +
    (1 - Re z^s) A^2 with z = 1 - c + i b; it is within |z^s - e^(i theta)| of
    exp(theta A)."""
    H, ops, hf, ne = _system(8)
    psi = _sector_state(8, ne, 3)
    A = ops[13]
    Ad = psum_matrix(A, 8)
    s = reopt_substeps(theta, sum(abs(c) for c in A.values()))
    assert s == max(1, math.ceil(max(abs(theta), math.pi) / 0.5))
    x = theta / s
    z = complex(1 - (x * x / 2 - x ** 4 / 24), x - x ** 3 / 6 + x ** 5 / 120) ** s
    closed = psi + z.imag * (Ad @ psi) + (1 - z.real) * (Ad @ (Ad @ psi))
    got = layer(A, theta, psi)
    assert np.abs(got - closed).max() < 1e-13
    assert np.linalg.norm(got - expm(theta * Ad) @ psi) <= abs(z - complex(math.cos(theta), math.sin(theta))) + 1e-13


@pytest.mark.parametrize("theta", [0.0, 0.4, -2.2, 3.0])
def test_layer_derivative_matches_central_difference(theta):
    H, ops, hf, ne = _system(8)
    psi = _sector_state(8, ne, 4)
    A = ops[20]
    h = 1e-5
    fd = (layer(A, theta + h, psi) - layer(A, theta - h, psi)) / (2 * h)
    assert np.abs(layer_derivative(A, theta, psi) - fd).max() < 1e-9


def test_energy_gradient_matches_central_differences():
    H, ops, hf, ne = _system(8)
    rng = np.random.default_rng(9)
    layers = [ops[j] for j in (2, 13, 20, 5)]
    thetas = list(rng.uniform(-2.5, 2.5, size=4))
    e, g, _ = energy_and_gradient(H, layers, thetas, hf)
    h = 1e-5
    for i in range(4):
        tp, tm = list(thetas), list(thetas)
        tp[i] += h
        tm[i] -= h
        fd = (energy_and_gradient(H, layers, tp, hf)[0] - energy_and_gradient(H, layers, tm, hf)[0]) / (2 * h)
        assert abs(g[i] - fd) < 1e-8, (i, g[i], fd)


def test_gradient_of_a_new_layer_at_zero_is_eq4():
    """L(A, 0) = I and dL/dtheta(0) = A, so appending a layer at angle 0 gives
    the gradient of Eq. 4, 2 Re <H psi|A psi> / <psi|psi>."""
    H, ops, hf, ne = _system(8)
    psi = _sector_state(8, ne, 5) * 1.3
    g_ref = gradients(ops, psi, apply_h(H, psi))
    for j in (0, 7, 22):
        e, g, _ = energy_and_gradient(H, [ops[j]], [0.0], psi)
        assert abs(g[0] - g_ref[j]) < 1e-13


def test_bfgs_minimises_quadratic_and_rosenbrock():
    rng = np.random.default_rng(1)
    B = rng.standard_normal((6, 6))
    Q = B @ B.T + 6 * np.eye(6)
    b = rng.standard_normal(6)
    x, f, g, steps, nev = bfgs(lambda x: (0.5 * x @ Q @ x - b @ x, Q @ x - b), np.zeros(6), gtol=1e-12)
    assert np.abs(x - np.linalg.solve(Q, b)).max() < 1e-10
    rb = lambda x: ((1 - x[0]) ** 2 + 100 * (x[1] - x[0] ** 2) ** 2,
                    np.array([-2 * (1 - x[0]) - 400 * x[0] * (x[1] - x[0] ** 2), 200 * (x[1] - x[0] ** 2)]))
    x, f, g, steps, nev = bfgs(rb, np.array([-1.2, 1.0]), gtol=1e-9, maxiter=500)
    assert np.abs(x - 1.0).max() < 1e-6


def test_bfgs_matches_scipy_on_the_ansatz_energy():
    H, ops, hf, ne = _system(8)
    seq = adapt_run(H, ops, hf, 4)["ops"]
    layers = [ops[j] for j in seq]
    fg = lambda x: energy_and_gradient(H, layers, list(x), hf)[:2]
    x, f, g, steps, nev = bfgs(fg, np.zeros(len(layers)) + 0.01, gtol=1e-9)
    ref = minimize(fg, np.zeros(len(layers)) + 0.01, jac=True, method="BFGS",
                   options={"gtol": 1e-9, "maxiter": 200})
    assert abs(f - ref.fun) < 1e-11
    assert np.abs(x - ref.x).max() < 1e-5


def test_adapt_reopt_4q_reaches_sector_ground_state():
    H, ops, hf, ne = _system(4)
    r = adapt_reopt_run(H, ops, hf, 20, grad_tol=1e-7, bfgs_gtol=1e-10)
    assert r["converged"]
    assert abs(r["energies"][-1] - _sector_fci(H, 4, ne)) < 1e-9


def test_adapt_reopt_8q_descends_and_beats_frozen_angles():
    """Energies fall with every layer, stay above the sector ground state, and
    with the same operators the optimised angles are at least as good as the
    frozen ones (up to the two substep rules' truncation difference)."""
    H, ops, hf, ne = _system(8)
    fr = adapt_run(H, ops, hf, 6)
    r = adapt_reopt_run(H, ops, hf, 6, forced_ops=fr["ops"] + [0])
    e = np.array(r["energies"])
    assert np.all(np.diff(e) <= 1e-12)
    assert e[-1] >= _sector_fci(H, 8, ne) - 1e-12
    assert np.all(e <= np.array(fr["energies"]) + 1e-6)
    assert e[-1] < fr["energies"][-1] - 1e-6


def test_adapt_reopt_jw_and_bk_trajectories_identical():
    rj = adapt_reopt_run(*_system(8, "jw")[:3], 5)
    rb = adapt_reopt_run(*_system(8, "bk")[:3], 5)
    assert rj["ops"] == rb["ops"]
    assert np.abs(np.array(rj["energies"]) - np.array(rb["energies"])).max() < 1e-10
    assert np.abs(np.array(rj["thetas"]) - np.array(rb["thetas"])).max() < 1e-6
