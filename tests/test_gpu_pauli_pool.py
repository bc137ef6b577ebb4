"""GPU parity of the Pauli (qubit) pool against the FP64 oracle, through the C ABI.

The pool holds every string of every fermionic generator as its own operator
(unit coefficient), so the screen runs over M = S operators of one string
each (14 qubits: 1488) and the Taylor chain over single strings.  Sizes: 4
qubits (ragged tile), 8, 12 and 14 qubits.  Tolerances as for the fermionic
pool: FP64 path 1e-12 relative on gradients, 1e-13 on Taylor states, 1e-10 Ha
on ADAPT energies; complex64 states 1e-6 Ha against the FP64 path.
"""

import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle.mapping import hamiltonian, hf_index
from oracle.pool import pauli_pool_operators
from oracle.statevec import apply_h, gradients as o_gradients, taylor5 as o_taylor5
from oracle.adapt import adapt_run
from workloads import molecular_integrals, electron_count


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def g():
    import paper_2607_15906_amd as g
    return g


@pytest.fixture(scope="module")
def ctx(g):
    return g.Context(0)


_cache = {}


def system(g, nq, mapping):
    key = (nq, mapping)
    if key not in _cache:
        n = nq // 2
        ne = electron_count(n)
        h1, eri, ec = molecular_integrals(n, nq)
        _cache[key] = dict(H=hamiltonian(h1, eri, ec, mapping),
                           ops=[B for _, _, B in pauli_pool_operators(nq, ne, mapping)],
                           hf=hf_index(nq, ne, mapping),
                           gH=g.pauli_hamiltonian_load(h1, eri, ec, mapping),
                           gP=g.pool_build_pauli(nq, ne, mapping))
    return _cache[key]


def rand_state(nq, seed):
    rng = np.random.default_rng(seed)
    psi = rng.standard_normal(1 << nq) + 1j * rng.standard_normal(1 << nq)
    return psi / np.linalg.norm(psi)


def to_dev(psi, dtype="c128"):
    t = torch.from_numpy(np.ascontiguousarray(psi))
    if dtype == "c64":
        t = t.to(torch.complex64)
    return t.to("cuda")


def hf_dev(s, nq, dtype):
    psi = np.zeros(1 << nq, dtype=np.complex128)
    psi[s["hf"]] = 1.0
    return to_dev(psi, dtype)


@pytest.mark.parametrize("nq", [4, 8, 12, 14, 16])
@pytest.mark.parametrize("mapping", ["jw", "bk"])
def test_pauli_pool_gradients(g, ctx, nq, mapping):
    _say(f"[pauli grad] nq={nq} {mapping}")
    s = system(g, nq, mapping)
    psi = rand_state(nq, 60 + nq) * 1.3
    g_ref = o_gradients(s["ops"], psi, apply_h(s["H"], psi))
    gg = g.pool_gradients(ctx, s["gH"], s["gP"], to_dev(psi))
    assert gg.shape == (len(s["ops"]),)
    assert np.abs(gg - g_ref).max() <= 1e-12 * max(1.0, np.abs(g_ref).max())


@pytest.mark.parametrize("nq,j,theta", [(4, 0, 0.3), (4, 11, -2.2), (8, 70, 1.1), (14, 5, -1.6),
                                        (14, 1487, 2.9)])
@pytest.mark.parametrize("mapping", ["jw", "bk"])
def test_pauli_pool_taylor5(g, ctx, nq, j, theta, mapping):
    _say(f"[pauli taylor] nq={nq} j={j} theta={theta} {mapping}")
    s = system(g, nq, mapping)
    psi = rand_state(nq, 70 + nq + j)
    ref, s_ref = o_taylor5(s["ops"][j], theta, psi)
    d = to_dev(psi)
    ns = g.taylor5_apply(ctx, s["gP"], j, theta, d)
    assert ns == s_ref
    assert np.abs(d.cpu().numpy() - ref).max() <= 1e-13


@pytest.mark.parametrize("nq,iters,mapping", [(4, 8, "jw"), (12, 20, "jw"), (12, 20, "bk")])
def test_pauli_pool_adapt_matches_oracle(g, ctx, nq, iters, mapping):
    """Follow the GPU's choices in the oracle: each must be a valid selection
    there (equal-magnitude string gradients tie), and energies, angles,
    substeps and the final state must agree."""
    _say(f"[pauli adapt] nq={nq} {mapping} iters={iters}")
    s = system(g, nq, mapping)
    d = hf_dev(s, nq, "c128")
    r = g.adapt_solve(ctx, s["gH"], s["gP"], d, iters, grad_tol=0.0, schedule=1)
    psi_gpu = d.cpu().numpy()
    hf = np.zeros(1 << nq, dtype=np.complex128)
    hf[s["hf"]] = 1.0
    o = adapt_run(s["H"], s["ops"], hf, iters, grad_tol=0.0, forced_ops=r["ops"] + [0], keep_gradients=True)
    assert len(o["ops"]) == r["n_iter"] == iters
    for k, j in enumerate(r["ops"]):
        a = np.abs(o["grads"][k])
        assert a[j] >= a.max() * (1 - 1e-9), (k, j, a[j], a.max())
    assert np.abs(np.array(o["energies"]) - r["energies"]).max() <= 1e-10
    assert np.abs(np.array(o["thetas"]) - r["thetas"]).max() <= 1e-8
    assert o["substeps"] == r["substeps"]
    assert abs(np.vdot(o["psi"], psi_gpu)) ** 2 >= 1 - 1e-12
    assert r["energies"][-1] < r["energies"][0] - 1e-3


def test_pauli_pool_wide_selection_16q(g, ctx):
    """A 16-qubit pool of 2688 operators, more than the selection caches per
    thread: two ADAPT iterations from a random state (the first selection in
    the start-up reduction, the second in the line-search launch), each
    choice a valid one in the oracle, with its max |g| and ||g||."""
    _say("[pauli wide selection] nq=16 jw")
    s = system(g, 16, "jw")
    assert len(s["ops"]) > 7 * 256
    psi = rand_state(16, 91)
    d = to_dev(psi)
    r = g.adapt_solve(ctx, s["gH"], s["gP"], d, 2, grad_tol=0.0, schedule=1)
    o = adapt_run(s["H"], s["ops"], psi, 2, grad_tol=0.0, forced_ops=r["ops"] + [0], keep_gradients=True)
    assert len(o["ops"]) == r["n_iter"] == 2
    for k, j in enumerate(r["ops"]):
        a = np.abs(o["grads"][k])
        assert a[j] >= a.max() * (1 - 1e-9), (k, j, a[j], a.max())
        assert abs(r["gmax"][k] - a.max()) <= 1e-12 * a.max()
        assert abs(r["gnorms"][k] - np.linalg.norm(a)) <= 1e-12 * np.linalg.norm(a)
    assert np.abs(np.array(o["energies"]) - r["energies"]).max() <= 1e-10
    assert np.abs(np.array(o["thetas"]) - r["thetas"]).max() <= 1e-8


@pytest.mark.parametrize("schedule", [2, 4])
def test_pauli_pool_adapt_register_blocking(g, ctx, schedule):
    """Two and four amplitudes per lane screen the per-operator table (one
    amplitude per lane takes the X-class screen); both against the oracle."""
    _say(f"[pauli adapt] 12q jw schedule={schedule}")
    nq, iters = 12, 10
    s = system(g, nq, "jw")
    d = hf_dev(s, nq, "c128")
    r = g.adapt_solve(ctx, s["gH"], s["gP"], d, iters, grad_tol=0.0, schedule=schedule)
    psi_gpu = d.cpu().numpy()
    hf = np.zeros(1 << nq, dtype=np.complex128)
    hf[s["hf"]] = 1.0
    o = adapt_run(s["H"], s["ops"], hf, iters, grad_tol=0.0, forced_ops=r["ops"] + [0], keep_gradients=True)
    for k, j in enumerate(r["ops"]):
        a = np.abs(o["grads"][k])
        assert a[j] >= a.max() * (1 - 1e-9), (k, j, a[j], a.max())
    assert np.abs(np.array(o["energies"]) - r["energies"]).max() <= 1e-10
    assert np.abs(np.array(o["thetas"]) - r["thetas"]).max() <= 1e-8
    assert abs(np.vdot(o["psi"], psi_gpu)) ** 2 >= 1 - 1e-12


def test_pauli_pool_complex64_14q(g, ctx):
    """complex64 state with FP64 accumulation against the FP64 path, 14 qubits."""
    _say("[pauli c64] 14q jw")
    s = system(g, 14, "jw")
    runs = {}
    for dtype in ("c128", "c64"):
        d = hf_dev(s, 14, dtype)
        runs[dtype] = (g.adapt_solve(ctx, s["gH"], s["gP"], d, 20, grad_tol=0.0, schedule=1),
                       d.cpu().numpy().astype(np.complex128))
    (r64, p64), (r32, p32) = runs["c128"], runs["c64"]
    assert r32["ops"] == r64["ops"]
    assert np.abs(r32["energies"] - r64["energies"]).max() <= 1e-6
    assert abs(np.vdot(p64, p32)) ** 2 / np.vdot(p32, p32).real >= 1 - 1e-6


def test_pauli_and_fermionic_pools_in_one_batch(g, ctx):
    """Members with either pool in one batch give their solo results."""
    _say("[pauli batch] mixed pools")
    specs = [(10, "jw", True), (10, "bk", False), (12, "jw", True), (8, "bk", True)]
    Hs, Ps, hfs, psis = [], [], [], []
    for nq, mapping, pauli in specs:
        n = nq // 2
        ne = electron_count(n)
        h1, eri, ec = molecular_integrals(n, 100 + nq)
        Hs.append(g.pauli_hamiltonian_load(h1, eri, ec, mapping))
        Ps.append((g.pool_build_pauli if pauli else g.pool_build)(nq, ne, mapping))
        hfs.append(hf_index(nq, ne, mapping))
    for (nq, _, _), hf in zip(specs, hfs):
        p = torch.zeros(1 << nq, dtype=torch.complex64, device="cuda")
        g.state_basis(ctx, nq, hf, p)
        psis.append(p)
    iters = 10
    b = g.Batch(ctx, Hs, Ps, psis, max_iter=iters, schedule=1)
    b.run()
    assert b.poll() == 0
    for k, (nq, _, _) in enumerate(specs):
        solo = torch.zeros(1 << nq, dtype=torch.complex64, device="cuda")
        g.state_basis(ctx, nq, hfs[k], solo)
        rs = g.adapt_solve(ctx, Hs[k], Ps[k], solo, iters, schedule=1)
        rb = b.result(k)
        assert rb["ops"] == rs["ops"]
        assert np.array_equal(rb["energies"], rs["energies"])
        assert torch.equal(psis[k], solo)
    b.close()
