"""The configurations the benchmark runs, checked against the FP64 oracle.

* 14 qubits / 6 electrons under Jordan-Wigner and Bravyi-Kitaev: 30 ADAPT
  iterations with complex128 and with complex64 states, each against the
  oracle's own run (Eq. 1, Eq. 4, Eq. 5-6).  Bounds: complex128 energies within
  1e-10 Ha, angles 1e-8, gradient norms 1e-9 (the bar of the FP64 path);
  complex64 energies within 1e-6 Ha, fidelity with the oracle state at least
  1 - 1e-6 (Sec. IV.C), gradient norms and largest gradients within 1e-6, and
  every gradient of the final state within 1e-6 of the oracle's.
* 16 qubits (65536 amplitudes, the serving stream's largest requests; several
  LDS stage chunks of H): energy, sigma, every pool gradient and a Taylor
  update on a random state, and two complex128 ADAPT iterations.
* Members of a mixed batch and requests served in a mix, against the oracle.

Operator choices: where the GPU and the oracle pick different operators the
oracle is re-run with the GPU's choices, and each GPU choice must be a valid
selection there (its gradient within 1e-9 relative of the largest).
"""

import sys
import time

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle.mapping import hamiltonian, hf_index
from oracle.pool import pool_operators
from oracle.statevec import apply_h, energy as o_energy, gradients as o_gradients, taylor5 as o_taylor5
from oracle.adapt import adapt_run
from workloads import molecular_integrals, electron_count, CONFIGS


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


_systems = {}
_oracle_runs = {}


def system(g, nq, mapping, seed):
    key = (nq, mapping, seed)
    if key not in _systems:
        ne = electron_count(nq // 2)
        h1, eri, ec = molecular_integrals(nq // 2, seed)
        _systems[key] = dict(
            nq=nq, ne=ne, H=hamiltonian(h1, eri, ec, mapping),
            ops=[A for _, _, A in pool_operators(nq, ne, mapping)], hf=hf_index(nq, ne, mapping),
            gH=g.pauli_hamiltonian_load(h1, eri, ec, mapping), gP=g.pool_build(nq, ne, mapping))
    return _systems[key]


def hf_vec(s):
    v = np.zeros(1 << s["nq"], dtype=np.complex128)
    v[s["hf"]] = 1.0
    return v


def oracle_run(s, iters, tol=0.0, forced=None):
    key = (id(s), iters, tol, None if forced is None else tuple(forced))
    if key not in _oracle_runs:
        t0 = time.time()
        _oracle_runs[key] = adapt_run(s["H"], s["ops"], hf_vec(s), iters, grad_tol=tol,
                                      forced_ops=None if forced is None else list(forced) + [0],
                                      keep_gradients=True)
        _say(f"  oracle {s['nq']}q {iters} iterations: {time.time() - t0:.1f} s")
    return _oracle_runs[key]


def oracle_following(s, r, iters, tol=0.0):
    """The oracle's run with the GPU record's operator choices (its own run if
    they agree); asserts each GPU choice is a valid selection in the oracle."""
    o = oracle_run(s, iters, tol)
    if o["ops"] != r["ops"]:
        o = oracle_run(s, iters, tol, forced=r["ops"])
    assert len(o["ops"]) == r["n_iter"]
    for k, j in enumerate(r["ops"]):
        a = np.abs(o["grads"][k])
        assert a[j] >= a.max() * (1 - 1e-9), (k, j, a[j], a.max())
    return o


def compare_record(o, r, psi_gpu, dtype):
    """Energies, angles, gradient norms, largest gradients, substeps and the
    fidelity of the final state; returns the measured errors."""
    de = float(np.abs(np.array(o["energies"]) - r["energies"]).max())
    dth = float(np.abs(np.array(o["thetas"]) - np.array(r["thetas"])).max()) if r["n_iter"] else 0.0
    dgn = float(np.abs(np.array(o["gnorms"]) - r["gnorms"]).max())
    dgm = float(np.abs(np.array(o["gmax"]) - r["gmax"]).max())
    out = dict(dE=de, dtheta=dth, dgnorm=dgn, dgmax=dgm)
    if psi_gpu is not None:
        p = psi_gpu / np.linalg.norm(psi_gpu)
        out["infidelity"] = float(1.0 - abs(np.vdot(o["psi"], p)) ** 2)
    _say("  " + ", ".join(f"{k} {v:.2e}" for k, v in out.items()))
    if dtype == "c128":
        assert de <= 1e-10 and dth <= 1e-8 and dgn <= 1e-9 and dgm <= 1e-9
        assert o["substeps"] == r["substeps"]
        if psi_gpu is not None:
            assert out["infidelity"] <= 1e-12
    else:
        assert de <= 1e-6 and dgn <= 1e-6 and dgm <= 1e-6
        if psi_gpu is not None:
            assert out["infidelity"] <= 1e-6
    return out


def run_gpu(g, ctx, s, iters, dtype, tol=0.0, schedule=1):
    t = torch.zeros(1 << s["nq"], dtype=torch.complex128 if dtype == "c128" else torch.complex64,
                    device="cuda")
    g.state_basis(ctx, s["nq"], s["hf"], t)
    r = g.adapt_solve(ctx, s["gH"], s["gP"], t, iters, grad_tol=tol, schedule=schedule)
    return r, t


# --------------------------------------------------------------- 14 qubits

@pytest.mark.timeout(600)
@pytest.mark.parametrize("mapping", ["jw", "bk"])
def test_14q_30_iterations_complex128_and_complex64_against_oracle(g, ctx, mapping):
    cfg = CONFIGS["c3_14q"]
    nq, iters = cfg["n_qubits"], cfg["iters"]
    _say(f"[oracle-workload] {nq}q {mapping} {iters} iterations, complex128 and complex64")
    s = system(g, nq, mapping, cfg["seed"])
    for dtype in ("c128", "c64"):
        r, t = run_gpu(g, ctx, s, iters, dtype)
        assert r["n_iter"] == iters
        o = oracle_following(s, r, iters)
        compare_record(o, r, t.cpu().numpy().astype(np.complex128), dtype)
        # every pool gradient of the final state (Eq. 4), FP64 reductions on
        # the stored state against the oracle's at its own final state
        gg = g.pool_gradients(ctx, s["gH"], s["gP"], t)
        go = o_gradients(s["ops"], o["psi"], apply_h(s["H"], o["psi"]))
        dg = float(np.abs(gg - go).max())
        _say(f"  {dtype}: max |dg| of the final state {dg:.2e}")
        assert dg <= (1e-10 if dtype == "c128" else 1e-6)


# --------------------------------------------------------------- 16 qubits

def _rand_state(nq, seed):
    rng = np.random.default_rng(seed)
    psi = rng.standard_normal(1 << nq) + 1j * rng.standard_normal(1 << nq)
    return psi / np.linalg.norm(psi)


@pytest.mark.timeout(300)
@pytest.mark.parametrize("mapping", ["jw", "bk"])
def test_16q_energy_sigma_gradients_taylor_against_oracle(g, ctx, mapping):
    _say(f"[oracle-workload] 16q {mapping} single-shot")
    s = system(g, 16, mapping, 16)
    assert s["gH"].n_terms > 4096          # several LDS stage chunks
    psi = _rand_state(16, 161)
    d = torch.from_numpy(psi).to("cuda")
    sig_ref = apply_h(s["H"], psi)
    e_ref = o_energy(s["H"], psi, sig_ref)
    sig = torch.zeros(1 << 16, dtype=torch.complex128, device="cuda")
    e = g.apply_hamiltonian(ctx, s["gH"], d, sig)
    assert abs(e - e_ref) <= 1e-12 * max(1.0, abs(e_ref))
    assert np.abs(sig.cpu().numpy() - sig_ref).max() <= 1e-12 * max(1.0, np.abs(sig_ref).max())
    g_ref = o_gradients(s["ops"], psi, sig_ref)
    gg = g.pool_gradients(ctx, s["gH"], s["gP"], d)
    assert np.abs(gg - g_ref).max() <= 1e-12 * max(1.0, np.abs(g_ref).max())
    # complex64 storage of the same state: FP64 reductions of the rounded state
    p32 = psi.astype(np.complex64).astype(np.complex128)
    g32 = g.pool_gradients(ctx, s["gH"], s["gP"], torch.from_numpy(p32).to(torch.complex64).to("cuda"))
    g32_ref = o_gradients(s["ops"], p32, apply_h(s["H"], p32))
    assert np.abs(g32 - g32_ref).max() <= 1e-12 * max(1.0, np.abs(g32_ref).max())
    for j, theta in ((7, 0.8), (300, -2.4)):
        ref, ns_ref = o_taylor5(s["ops"][j], theta, psi)
        dj = torch.from_numpy(psi).to("cuda")
        assert g.taylor5_apply(ctx, s["gP"], j, theta, dj) == ns_ref
        assert np.abs(dj.cpu().numpy() - ref).max() <= 1e-13


@pytest.mark.timeout(300)
@pytest.mark.parametrize("mapping", ["jw", "bk"])
def test_16q_two_adapt_iterations_against_oracle(g, ctx, mapping):
    _say(f"[oracle-workload] 16q {mapping} 2 ADAPT iterations")
    s = system(g, 16, mapping, 16)
    r, t = run_gpu(g, ctx, s, 2, "c128")
    o = oracle_following(s, r, 2)
    compare_record(o, r, t.cpu().numpy(), "c128")


@pytest.mark.timeout(300)
@pytest.mark.parametrize("schedule", [1, 1 + 4 * 256])
def test_16q_complex64_compacted_line_search_against_oracle(g, ctx, schedule):
    """Complex64 at 16 qubits: H spans two LDS stage chunks, so the compacted
    H v / H w launch walks the run tables of both chunks (8 or 4 parts)."""
    _say(f"[oracle-workload] 16q c64 schedule {schedule}")
    s = system(g, 16, "jw", 16)
    r, t = run_gpu(g, ctx, s, 3, "c64", schedule=schedule)
    o = oracle_following(s, r, 3)
    compare_record(o, r, t.cpu().numpy().astype(np.complex128), "c64")


# --------------------------------------------------------------- batch and serving members

@pytest.mark.timeout(300)
@pytest.mark.parametrize("dtype,schedule", [("c128", 0), ("c64", 0), ("c64", 4 + 4 * 256)])
def test_batch_members_against_oracle(g, ctx, dtype, schedule):
    """A mixed batch (the batched workload's sizes, both mappings) at its
    autotuned schedule, and for complex64 also at four amplitudes per lane
    with four H v / H w parts (the batched workload's choice); two members
    followed through 30 iterations."""
    _say(f"[oracle-workload] batch members {dtype} schedule {schedule}")
    specs = [(10, "jw", 1000), (10, "bk", 1001), (12, "jw", 1024), (12, "bk", 1025),
             (14, "jw", 1048), (14, "bk", 1049)]
    ss = [system(g, nq, m, seed) for (nq, m, seed) in specs]
    tdt = torch.complex128 if dtype == "c128" else torch.complex64
    psis = []
    for s in ss:
        t = torch.zeros(1 << s["nq"], dtype=tdt, device="cuda")
        g.state_basis(ctx, s["nq"], s["hf"], t)
        psis.append(t)
    iters = 30
    b = g.Batch(ctx, [s["gH"] for s in ss], [s["gP"] for s in ss], psis, max_iter=iters, schedule=schedule)
    b.run()
    assert b.poll() == 0
    for k in (1, 2):
        r = b.result(k)
        assert r["n_iter"] == iters
        o = oracle_following(ss[k], r, iters)
        compare_record(o, r, psis[k].cpu().numpy().astype(np.complex128), dtype)
    b.close()


@pytest.mark.timeout(300)
@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_served_requests_against_oracle(g, ctx, dtype):
    """Requests of mixed size served together (adaptive schedule), stopping at
    ||g|| < 1e-3 or 120 iterations: two of them against the oracle's run with
    the same threshold and limit (the same number of iterations and the same
    convergence flag)."""
    _say(f"[oracle-workload] served requests {dtype}")
    specs = [(8, "jw", 2000), (10, "bk", 2001), (12, "jw", 2002), (8, "bk", 2003), (10, "jw", 2004)]
    ss = [system(g, nq, m, seed) for (nq, m, seed) in specs]
    tol, max_iter = 1e-3, 120
    srv = g.Server(ctx, 1 << 30, 8, dtype=0 if dtype == "c128" else 1, iters_per_step=4, amps_per_lane=0)
    tickets = [srv.submit(s["gH"], s["gP"], max_iter, tol) for s in ss]
    out = {}
    t0 = time.time()
    while len(out) < len(tickets):
        for t in tickets:
            if t not in out:
                res = srv.poll(t)
                if res is not None:
                    out[t] = res
        assert time.time() - t0 < 120, "served requests did not finish"
        time.sleep(0.001)
    srv.close()
    for k in (1, 2):
        st, r, info = out[tickets[k]]
        assert st == 0
        o = oracle_following(ss[k], r, max_iter, tol)
        assert o["converged"] == r["converged"] and len(o["ops"]) == r["n_iter"]
        compare_record(o, r, None, dtype)
