"""Pins of the oracle's energy (Eq. 1), gradients (Eq. 4), O(5) chain (Eq. 5-6),
line search and ADAPT loop."""

import json
import math
import os

import numpy as np
import pytest
from scipy.linalg import expm
from scipy.optimize import brentq

from oracle.pauli import psum_matrix, apply_psum
from oracle.mapping import hamiltonian, hf_index
from oracle.pool import pool_operators, pool_excitations
from oracle.statevec import (apply_h, energy, gradients, gradients_commutator, select,
                             taylor5, substeps, line_coefficients, landscape,
                             landscape_derivative, line_search, hf_state, TIE_RTOL)
from oracle.adapt import adapt_run
from workloads import molecular_integrals, electron_count

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _system(nq, mapping="jw", seed=None):
    n = nq // 2
    ne = electron_count(n)
    h1, eri, ec = molecular_integrals(n, nq if seed is None else seed)
    H = hamiltonian(h1, eri, ec, mapping)
    ops = [A for _, _, A in pool_operators(nq, ne, mapping)]
    return h1, eri, ec, H, ops, hf_state(nq, hf_index(nq, ne, mapping)), ne


def _sector_state(nq, ne, rng, mapping="jw"):
    """Random real normalised state inside the (N_e, S_z = 0) sector (JW basis)."""
    d = np.arange(1 << nq)
    mask = (np.bitwise_count(d) == ne) & (np.bitwise_count(d & 0x5555) == ne // 2)
    psi = np.where(mask, rng.standard_normal(1 << nq), 0.0).astype(np.complex128)
    return psi / np.linalg.norm(psi)


def test_energy_matches_dense_rayleigh_quotient():
    h1, eri, ec, H, ops, hf, ne = _system(8)
    Hd = psum_matrix(H, 8)
    rng = np.random.default_rng(0)
    psi = rng.standard_normal(256) + 1j * rng.standard_normal(256)
    ref = (psi.conj() @ Hd @ psi).real / (psi.conj() @ psi).real
    assert abs(energy(H, psi) - ref) < 1e-12
    assert abs(energy(H, 3.0 * psi) - ref) < 1e-12


def test_gradient_forms_agree_and_match_dense_commutator():
    h1, eri, ec, H, ops, hf, ne = _system(8)
    rng = np.random.default_rng(1)
    psi = _sector_state(8, ne, rng)
    sigma = apply_h(H, psi)
    g = gradients(ops, psi, sigma)
    g2 = gradients_commutator(H, ops, psi)
    Hd = psum_matrix(H, 8)
    g3 = np.array([(psi.conj() @ (Hd @ psum_matrix(A, 8) - psum_matrix(A, 8) @ Hd) @ psi).real
                   for A in ops])
    assert np.abs(g - g2).max() < 1e-12
    assert np.abs(g - g3).max() < 1e-12


def test_gradient_matches_finite_difference_of_exact_rotation():
    h1, eri, ec, H, ops, hf, ne = _system(8)
    rng = np.random.default_rng(2)
    psi = _sector_state(8, ne, rng)
    g = gradients(ops, psi, apply_h(H, psi))
    Hd = psum_matrix(H, 8)
    h = 1e-5
    for j in (0, 3, 11, 25):
        Ad = psum_matrix(ops[j], 8)
        ep = (lambda t: (lambda p: (p.conj() @ Hd @ p).real)(expm(t * Ad) @ psi))
        fd = (ep(h) - ep(-h)) / (2 * h)
        assert abs(fd - g[j]) < 1e-8


def _fock_ov(h1, eri, ne, i, a):
    """Spin-orbital Fock element f_ai over the HF occupation."""
    f = h1[a // 2, i // 2] if a % 2 == i % 2 else 0.0
    if a % 2 != i % 2:
        return 0.0
    for j in range(ne):
        f += eri[a // 2, i // 2, j // 2, j // 2]
        if j % 2 == a % 2:
            f -= eri[a // 2, j // 2, j // 2, i // 2]
    return f


def _antisym(eri, a, b, i, j):
    """<ab||ij> = <ab|ij> - <ab|ji> with <pq|rs> = (pr|qs) and spin deltas."""
    def phys(p, q, r, s):
        if p % 2 != r % 2 or q % 2 != s % 2:
            return 0.0
        return eri[p // 2, r // 2, q // 2, s // 2]
    return phys(a, b, i, j) - phys(a, b, j, i)


@pytest.mark.parametrize("nq", [4, 8, 12, 14])
@pytest.mark.parametrize("mapping", ["jw", "bk"])
def test_iteration0_gradients_match_slater_condon(nq, mapping):
    h1, eri, ec, H, ops, hf, ne = _system(nq, mapping)
    g = gradients(ops, hf, apply_h(H, hf))
    for k, (kind, idx) in enumerate(pool_excitations(nq, ne)):
        if kind == 1:
            i, a = idx
            ref = 2.0 * abs(_fock_ov(h1, eri, ne, i, a))
        else:
            i, j, a, b = idx
            ref = 2.0 * abs(_antisym(eri, a, b, i, j))
        assert abs(abs(g[k]) - ref) < 1e-12, (k, kind, idx)


def test_select_ties_take_lowest_index():
    g = np.array([0.1, -0.3, 0.3 * (1 - 1e-14), -0.3, 0.2])
    j, gmax, gn = select(g)
    assert j == 1
    assert gmax == 0.3
    assert abs(gn - math.sqrt(0.01 + 3 * 0.09 + 0.04)) < 1e-14
    g2 = np.array([0.1, -0.3, 0.3 * (1 + 1e-9)])
    assert select(g2)[0] == 2


# ---------------------------------------------------------------- O(5) Taylor chain

def test_taylor_coefficients_of_eq6():
    with open(os.path.join(GOLDEN, "paper_values.json")) as f:
        ref = json.load(f)["taylor_coefficients"]["value"]
    c, out = 1.0, [1.0]
    for n in range(1, 6):
        c = c * 1.0 / n
        out.append(c)
    assert out == ref


def _closed_form_chain(A, theta, psi):
    """T5(x)^s = I + (1 - Re z^s) A^2 + Im(z^s) A with z = 1 - gamma + i beta."""
    s = substeps(theta, sum(abs(c) for c in A.values()))
    x = theta / s
    beta = x - x ** 3 / 6 + x ** 5 / 120
    gamma = x ** 2 / 2 - x ** 4 / 24
    zs = complex(1 - gamma, beta) ** s
    w = apply_psum(A, psi)
    a2 = apply_psum(A, w)
    return psi + (1 - zs.real) * a2 + zs.imag * w, s, zs


@pytest.mark.parametrize("nq,j,theta", [(8, 3, 0.3), (8, 20, -1.7), (12, 5, 2.9), (14, 150, -0.8)])
def test_taylor_chain_matches_closed_form(nq, j, theta):
    h1, eri, ec, H, ops, hf, ne = _system(nq)
    psi = _sector_state(nq, ne, np.random.default_rng(nq + j))
    out, s = taylor5(ops[j], theta, psi, renormalize=False)
    ref, s2, zs = _closed_form_chain(ops[j], theta, psi)
    assert s == s2 == max(1, math.ceil(abs(theta) / 0.5))
    assert np.abs(out - ref).max() < 1e-14
    # pre-renormalisation norm: 1 + (|z|^{2s} - 1) ||P psi||^2, P = -A^2
    ppsi = -apply_psum(ops[j], apply_psum(ops[j], psi))
    pn = np.vdot(ppsi, ppsi).real
    assert abs(np.vdot(out, out).real - (1 + (abs(zs) ** 2 - 1) * pn)) < 1e-14


@pytest.mark.parametrize("theta", [0.3, -1.7, 2.9])
def test_sigma_carried_through_the_update(theta):
    """With A^3 = -A each substep is I + a A + b A^2 and products of such stay
    in that span: (a1, b1) * (a2, b2) = (a1 + a2 - a1 b2 - b1 a2,
    b1 + b2 + a1 a2 - b1 b2).  s such products give the closed form's
    (Im z^s, 1 - Re z^s), and H psi' = sigma + al H w - be H v with
    w = A psi, v = -A w (the sigma an ADAPT iteration carries forward)."""
    nq = 10
    h1, eri, ec, H, ops, hf, ne = _system(nq)
    psi = _sector_state(nq, ne, np.random.default_rng(29))
    A = ops[11]
    out, s = taylor5(A, theta, psi, renormalize=False)
    x = theta / s
    a = x - x ** 3 / 6 + x ** 5 / 120
    b = x ** 2 / 2 - x ** 4 / 24
    al = be = 0.0
    for _ in range(s):
        al, be = al + a - al * b - be * a, be + b + al * a - be * b
    _, _, zs = _closed_form_chain(A, theta, psi)
    assert abs(al - zs.imag) < 1e-14 and abs(be - (1 - zs.real)) < 1e-14
    w = apply_psum(A, psi)
    v = -apply_psum(A, w)
    sigma = apply_h(H, psi)
    carried = sigma + al * apply_h(H, w) - be * apply_h(H, v)
    assert np.abs(carried - apply_h(H, out)).max() < 1e-12


@pytest.mark.parametrize("theta", [0.05, 0.5, -1.3, 3.0])
def test_taylor_chain_versus_expm_within_truncation_bound(theta):
    h1, eri, ec, H, ops, hf, ne = _system(8)
    psi = _sector_state(8, ne, np.random.default_rng(5))
    A = ops[17]
    out, s = taylor5(A, theta, psi, renormalize=False)
    exact = expm(theta * psum_matrix(A, 8)) @ psi
    _, _, zs = _closed_form_chain(A, theta, psi)
    bound = abs(zs - complex(math.cos(theta), math.sin(theta)))
    assert np.linalg.norm(out - exact) <= bound + 1e-14
    # per-substep truncation ~ x^6/720: fidelity beyond 1 - 1e-6 (Sec. IV.C)
    out_n, _ = taylor5(A, theta, psi)
    fid = abs(np.vdot(exact, out_n)) ** 2
    assert fid > 1 - 1e-6


@pytest.mark.parametrize("mapping", ["jw", "bk"])
def test_taylor_preserves_sector_and_reality(mapping):
    from oracle.mapping import bk_matrix
    nq = 12
    h1, eri, ec, H, ops, hf, ne = _system(nq, mapping)
    psi = hf.copy()
    for j, th in ((3, 0.4), (60, -0.9), (100, 1.7)):
        psi, _ = taylor5(ops[j], th, psi)
        assert np.all(psi.imag == 0.0)
        assert abs(np.vdot(psi, psi).real - 1.0) < 1e-15
    # occupations of every basis index (BK indices decoded through beta^-1)
    d = np.arange(1 << nq)
    if mapping == "jw":
        occ = d
    else:
        beta = bk_matrix(nq)
        enc = np.array([int(sum(int(b) << q for q, b in enumerate(beta.dot([(n_ >> k) & 1 for k in range(nq)]) & 1)))
                        for n_ in d])
        occ = np.empty_like(d)
        occ[enc] = d
    inside = (np.bitwise_count(occ) == ne) & (np.bitwise_count(occ & 0x5555) == ne // 2)
    # string-by-string sums of equal-magnitude terms cancel only up to rounding
    assert np.abs(psi[~inside]).max() < 1e-15
    assert np.count_nonzero(psi[inside]) > 1


def test_theta_zero_is_noop():
    h1, eri, ec, H, ops, hf, ne = _system(4)
    out, s = taylor5(ops[0], 0.0, hf)
    assert s == 0 and np.array_equal(out, hf)


# ---------------------------------------------------------------- line search

def test_landscape_matches_dense_exponential_scan():
    h1, eri, ec, H, ops, hf, ne = _system(8)
    psi = _sector_state(8, ne, np.random.default_rng(7))
    sigma = apply_h(H, psi)
    Hd = psum_matrix(H, 8)
    for j in (2, 13):
        A = ops[j]
        coef = line_coefficients(H, A, psi, sigma)
        Ad = psum_matrix(A, 8)
        for th in np.linspace(-math.pi, math.pi, 64):
            p = expm(th * Ad) @ psi
            assert abs(landscape(coef, th) - (p.conj() @ Hd @ p).real) < 1e-12
        assert abs(landscape(coef, 0.0) - energy(H, psi, sigma)) < 1e-12
        g = gradients([A], psi, sigma)[0]
        assert abs(landscape_derivative(coef, 0.0) - g) < 1e-12


def _dense_line(H, A, psi, nq):
    """E(theta) = <e^{theta A} psi|H|e^{theta A} psi> from dense matrices (no
    oracle line-search arithmetic involved)."""
    Hd = psum_matrix(H, nq)
    Ad = psum_matrix(A, nq)
    # A is anti-Hermitian: A = -i K with K Hermitian, so exp(theta A) =
    # V diag(exp(-i theta lam)) V^+ from the eigenpairs of K (checked against
    # expm at one angle)
    lam, V = np.linalg.eigh(1j * Ad)
    c = V.conj().T @ psi
    assert np.abs(V @ (np.exp(-0.7j * lam) * c) - expm(0.7 * Ad) @ psi).max() < 1e-12
    def e(th):
        p = V @ (np.exp(-1j * th * lam) * c)
        return float((p.conj() @ Hd @ p).real)
    return e


def _derivative_pin_error(deriv, coef, e_dense, thetas, h=1e-5):
    """Largest gap between deriv(coef, theta) and the central difference of the
    dense energy at the given angles."""
    return max(abs(deriv(coef, th) - (e_dense(th + h) - e_dense(th - h)) / (2 * h)) for th in thetas)


def test_landscape_derivative_matches_dense_central_differences_away_from_zero():
    """E'(theta) at angles away from 0, where every term of the derivative
    contributes (at theta = 0 the sin-theta terms vanish and the pin against g
    cannot see them): central differences of the dense exponential's energy.
    A sign error in any single term of the derivative is caught."""
    h1, eri, ec, H, ops, hf, ne = _system(8)
    psi = _sector_state(8, ne, np.random.default_rng(11))
    sigma = apply_h(H, psi)
    thetas = [-2.7, -1.3, -0.4, 0.25, 0.9, 1.7, 2.9]
    for j in (1, 13, 25):
        coef = line_coefficients(H, ops[j], psi, sigma)
        e_dense = _dense_line(H, ops[j], psi, 8)
        assert _derivative_pin_error(landscape_derivative, coef, e_dense, thetas) < 1e-8
        # each term of E'(theta) flipped in sign in turn must fail the pin
        auu, auv, auw, avv, avw, aww = coef
        def term(k):
            def f(c, th):
                cs, sn = math.cos(th), math.sin(th)
                parts = [-2.0 * auv * sn, 2.0 * auw * cs, -2.0 * avv * sn * cs,
                         2.0 * avw * (cs * cs - sn * sn), 2.0 * aww * sn * cs]
                parts[k] = -parts[k]
                return sum(parts)
            return f
        for k in range(5):
            assert _derivative_pin_error(term(k), coef, e_dense, thetas) > 1e-4, k


def test_line_search_angle_is_first_minimum_of_dense_energy_scan():
    """theta* against the dense exponential alone: walking from 0 downhill on a
    0.05-degree grid of dense energies, the first grid minimum lies next to
    theta*, and a bounded minimisation of the dense energy around it lands on
    theta* to the precision a minimum allows (~sqrt(machine epsilon))."""
    from scipy.optimize import minimize_scalar
    h1, eri, ec, H, ops, hf, ne = _system(8)
    psi = _sector_state(8, ne, np.random.default_rng(12))
    sigma = apply_h(H, psi)
    g = gradients(ops, psi, sigma)
    step = math.pi / 3600
    for j in (0, 7, 13, 25):
        coef = line_coefficients(H, ops[j], psi, sigma)
        th = line_search(coef, g[j])
        d = -np.sign(g[j])
        e_dense = _dense_line(H, ops[j], psi, 8)
        prev = e_dense(0.0)
        k = 1
        while True:
            cur = e_dense(d * k * step)
            if cur > prev:
                break
            prev = cur
            k += 1
            assert k < 7200
        t_grid = d * (k - 1) * step
        assert abs(t_grid - th) <= step
        lo, hi = sorted((t_grid - 2 * step, t_grid + 2 * step))
        t_min = minimize_scalar(e_dense, bounds=(lo, hi), method="bounded",
                                options={"xatol": 1e-10}).x
        assert abs(t_min - th) < 1e-6
        assert e_dense(th) <= e_dense(t_min) + 1e-13


def test_line_search_matches_brentq():
    h1, eri, ec, H, ops, hf, ne = _system(8)
    psi = _sector_state(8, ne, np.random.default_rng(8))
    sigma = apply_h(H, psi)
    g = gradients(ops, psi, sigma)
    for j in range(0, len(ops), 5):
        coef = line_coefficients(H, ops[j], psi, sigma)
        th = line_search(coef, g[j])
        d = -np.sign(g[j])
        grid = d * np.arange(0, 361) * math.pi / 180
        vals = [d * landscape_derivative(coef, t) for t in grid]
        k = next(i for i in range(1, 361) if vals[i] >= 0)
        ref = brentq(lambda t: landscape_derivative(coef, t), grid[k - 1], grid[k], xtol=1e-15)
        assert abs(th - ref) < 1e-12
        assert landscape(coef, th) <= landscape(coef, 0.0)


# ---------------------------------------------------------------- ADAPT loop

def _sector_fci(H, nq, ne):
    d = np.arange(1 << nq)
    idx = np.nonzero((np.bitwise_count(d) == ne) & (np.bitwise_count(d & 0x5555) == ne // 2))[0]
    cols = []
    for k in idx:
        e = np.zeros(1 << nq, dtype=np.complex128)
        e[k] = 1
        cols.append(apply_h(H, e)[idx].real)
    return np.linalg.eigvalsh(np.array(cols).T)[0]


def test_adapt_4q_reaches_sector_ground_state():
    h1, eri, ec, H, ops, hf, ne = _system(4)
    r = adapt_run(H, ops, hf, 100, grad_tol=1e-7)
    assert r["converged"]
    assert abs(r["energies"][-1] - _sector_fci(H, 4, ne)) < 1e-9


def test_adapt_energy_monotone_and_prediction_within_taylor_error():
    h1, eri, ec, H, ops, hf, ne = _system(8)
    r = adapt_run(H, ops, hf, 25)
    e = np.array(r["energies"])
    assert np.all(np.diff(e) <= 1e-12)
    assert np.all(np.abs(np.array(r["predicted"]) - e[1:]) < 1e-6)
    assert e[-1] >= _sector_fci(H, 8, ne) - 1e-12


def test_adapt_jw_and_bk_trajectories_identical():
    rj = adapt_run(*_system(8, "jw")[3:6], 15)
    rb = adapt_run(*_system(8, "bk")[3:6], 15)
    assert rj["ops"] == rb["ops"]
    assert np.abs(np.array(rj["energies"]) - np.array(rb["energies"])).max() < 1e-10
    assert np.abs(np.array(rj["thetas"]) - np.array(rb["thetas"])).max() < 1e-9
