"""GPU parity of the HIP path against the FP64 oracle, through the C ABI.

Sizes: 4 qubits (one partial tile and a partial pair block: the ragged case),
8 qubits (several tiles), 12 and 14 qubits (the paper's register sizes,
hundreds of tiles); 16 qubits and the benchmarked 14-qubit runs are in
test_gpu_oracle_workloads.py.  Tolerances: FP64 path
1e-12 relative on energies and gradients (rounding of sums of a few thousand
terms), 1e-10 Ha on ADAPT energies; complex64 states: 1e-6 Ha and fidelity
1 - 1e-6.
"""

import math
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle.mapping import hamiltonian, hf_index
from oracle.pool import pool_operators
from oracle.statevec import apply_h, energy as o_energy, gradients as o_gradients, taylor5 as o_taylor5, select
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


def system(g, nq, mapping, seed=None):
    key = (nq, mapping, seed)
    if key not in _cache:
        n = nq // 2
        ne = electron_count(n)
        h1, eri, ec = molecular_integrals(n, nq if seed is None else seed)
        H = hamiltonian(h1, eri, ec, mapping)
        ops = [A for _, _, A in pool_operators(nq, ne, mapping)]
        _cache[key] = dict(H=H, ops=ops, ne=ne, hf=hf_index(nq, ne, mapping),
                           gH=g.pauli_hamiltonian_load(h1, eri, ec, mapping),
                           gP=g.pool_build(nq, ne, mapping))
    return _cache[key]


def rand_state(nq, seed, complex_=True):
    rng = np.random.default_rng(seed)
    psi = rng.standard_normal(1 << nq) + (1j * rng.standard_normal(1 << nq) if complex_ else 0)
    return (psi / np.linalg.norm(psi)).astype(np.complex128)


def to_dev(psi, dtype="c128"):
    t = torch.from_numpy(np.ascontiguousarray(psi))
    if dtype == "c64":
        t = t.to(torch.complex64)
    return t.to("cuda")


@pytest.mark.parametrize("nq", [4, 8, 12, 14])
@pytest.mark.parametrize("mapping", ["jw", "bk"])
def test_energy_and_sigma(g, ctx, nq, mapping):
    _say(f"[energy] nq={nq} {mapping}")
    s = system(g, nq, mapping)
    psi = rand_state(nq, 10 + nq)
    sig_ref = apply_h(s["H"], psi)
    e_ref = o_energy(s["H"], psi, sig_ref)
    d = to_dev(psi)
    e = g.energy(ctx, s["gH"], d)
    assert abs(e - e_ref) <= 1e-12 * max(1.0, abs(e_ref))
    sig = torch.zeros(1 << nq, dtype=torch.complex128, device="cuda")
    e2 = g.apply_hamiltonian(ctx, s["gH"], d, sig)
    assert e2 == e                                           # deterministic
    err = np.abs(sig.cpu().numpy() - sig_ref).max()
    assert err <= 1e-12 * max(1.0, np.abs(sig_ref).max())


@pytest.mark.parametrize("nq", [4, 8, 12, 14])
@pytest.mark.parametrize("mapping", ["jw", "bk"])
def test_pool_gradients(g, ctx, nq, mapping):
    _say(f"[grad] nq={nq} {mapping}")
    s = system(g, nq, mapping)
    psi = rand_state(nq, 20 + nq) * 1.7          # unnormalised on purpose
    g_ref = o_gradients(s["ops"], psi, apply_h(s["H"], psi))
    gg = g.pool_gradients(ctx, s["gH"], s["gP"], to_dev(psi))
    assert np.abs(gg - g_ref).max() <= 1e-12 * max(1.0, np.abs(g_ref).max())
    # device output variant
    out = torch.zeros(s["gP"].n_ops, dtype=torch.float64, device="cuda")
    g.pool_gradients(ctx, s["gH"], s["gP"], to_dev(psi), out=out)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), gg)


def test_gradients_at_hf_full_14q(g, ctx):
    _say("[grad] hf 14q")
    s = system(g, 14, "jw")
    psi = np.zeros(1 << 14, dtype=np.complex128)
    psi[s["hf"]] = 1.0
    g_ref = o_gradients(s["ops"], psi, apply_h(s["H"], psi))
    gg = g.pool_gradients(ctx, s["gH"], s["gP"], to_dev(psi))
    assert np.abs(gg - g_ref).max() <= 1e-13
    assert select(gg)[0] == select(g_ref)[0]


@pytest.mark.parametrize("nq,j,theta", [(4, 0, 0.3), (4, 2, -2.2), (8, 5, 1.1), (8, 20, -0.05),
                                        (12, 40, 0.9), (14, 3, -1.6), (14, 150, 2.9)])
@pytest.mark.parametrize("mapping", ["jw", "bk"])
def test_taylor5(g, ctx, nq, j, theta, mapping):
    _say(f"[taylor] nq={nq} j={j} theta={theta} {mapping}")
    s = system(g, nq, mapping)
    psi = rand_state(nq, 30 + nq + j)
    ref, s_ref = o_taylor5(s["ops"][j], theta, psi)
    d = to_dev(psi)
    ns = g.taylor5_apply(ctx, s["gP"], j, theta, d)
    assert ns == s_ref
    assert np.abs(d.cpu().numpy() - ref).max() <= 1e-13


def test_taylor5_theta_zero_is_noop(g, ctx):
    s = system(g, 8, "jw")
    psi = rand_state(8, 5)
    d = to_dev(psi)
    assert g.taylor5_apply(ctx, s["gP"], 3, 0.0, d) == 0
    assert np.array_equal(d.cpu().numpy(), psi)


def test_state_basis_and_hf_energy(g, ctx):
    s = system(g, 12, "bk")
    d = torch.empty(1 << 12, dtype=torch.complex128, device="cuda")
    g.state_basis(ctx, 12, s["hf"], d)
    torch.cuda.synchronize()
    ref = np.zeros(1 << 12, dtype=np.complex128)
    ref[s["hf"]] = 1.0
    assert np.array_equal(d.cpu().numpy(), ref)
    assert abs(g.energy(ctx, s["gH"], d) - o_energy(s["H"], ref)) < 1e-12


def test_shape_errors(g, ctx):
    s12 = system(g, 12, "jw")
    s14 = system(g, 14, "jw")
    d = to_dev(rand_state(12, 1))
    with pytest.raises(ValueError):
        g.pool_gradients(ctx, s12["gH"], s14["gP"], d)
    # the C ABI itself reports ESHAPE for handles of different qubit counts
    import ctypes as C
    from paper_2607_15906_amd._lib import load
    gout = np.zeros(s14["gP"].n_ops)
    rc = load().pool_gradients(ctx.handle, s12["gH"].handle, s14["gP"].handle, C.c_void_p(d.data_ptr()),
                               0, gout.ctypes.data_as(C.POINTER(C.c_double)), 0)
    assert rc == -4
    with pytest.raises(g.GocpError):
        g.taylor5_apply(ctx, s12["gP"], s12["gP"].n_ops, 0.1, d)


def test_binding_rejects_buffers_of_the_wrong_size_before_any_launch(g, ctx):
    """The C ABI takes bare device pointers; the binding checks every buffer's
    length, dtype and device against the handles, and raises before calling."""
    s12 = system(g, 12, "jw")
    s14 = system(g, 14, "jw")
    d12 = to_dev(rand_state(12, 2))
    before = d12.clone()
    n14 = s14["gP"].n_ops
    bad = [
        lambda: g.energy(ctx, s14["gH"], d12),
        lambda: g.apply_hamiltonian(ctx, s14["gH"], d12, torch.zeros(1 << 14, dtype=torch.complex128, device="cuda")),
        lambda: g.apply_hamiltonian(ctx, s12["gH"], d12, torch.zeros(1 << 11, dtype=torch.complex128, device="cuda")),
        lambda: g.apply_hamiltonian(ctx, s12["gH"], d12, torch.zeros(1 << 12, dtype=torch.complex64, device="cuda")),
        lambda: g.pool_gradients(ctx, s14["gH"], s14["gP"], d12),
        lambda: g.pool_gradients(ctx, s12["gH"], s12["gP"], d12,
                                 out=torch.zeros(s12["gP"].n_ops - 1, dtype=torch.float64, device="cuda")),
        lambda: g.pool_gradients(ctx, s12["gH"], s12["gP"], d12,
                                 out=torch.zeros(s12["gP"].n_ops, dtype=torch.float32, device="cuda")),
        lambda: g.pool_gradients(ctx, s12["gH"], s12["gP"], d12, out=torch.zeros(s12["gP"].n_ops, dtype=torch.float64)),
        lambda: g.taylor5_apply(ctx, s14["gP"], 3, 0.2, d12),
        lambda: g.taylor5_apply_family(ctx, s14["gP"], [0], [0.1], d12),
        lambda: g.adapt_solve(ctx, s14["gH"], s14["gP"], d12, 2),
        lambda: g.adapt_solve(ctx, s12["gH"], s14["gP"], d12, 2),
        lambda: g.state_basis(ctx, 14, 0, d12),
        lambda: g.Batch(ctx, [s14["gH"]], [s14["gP"]], [d12], max_iter=2),
        lambda: g.energy(ctx, s12["gH"], d12.cpu()),
        lambda: g.energy(ctx, s12["gH"], torch.zeros(1 << 12, dtype=torch.float64, device="cuda")),
    ]
    for k, f in enumerate(bad):
        with pytest.raises(ValueError):
            f()
    torch.cuda.synchronize()
    assert torch.equal(d12, before)
    assert n14 > 0


def _adapt_gpu(g, ctx, s, nq, iters, dtype="c128", tol=0.0, use_graph=True, schedule=1):
    psi = np.zeros(1 << nq, dtype=np.complex128)
    psi[s["hf"]] = 1.0
    d = to_dev(psi, dtype)
    r = g.adapt_solve(ctx, s["gH"], s["gP"], d, iters, grad_tol=tol, use_graph=use_graph,
                      schedule=schedule)
    return r, d.cpu().numpy().astype(np.complex128)


def _check_against_oracle(s, r, psi_gpu, iters, tol=0.0, etol=1e-10):
    """Follow the GPU's operator choices in the oracle; each choice must be a
    valid selection there, and energies, angles and the state must agree."""
    hf = np.zeros_like(psi_gpu)
    hf[s["hf"]] = 1.0
    o = adapt_run(s["H"], s["ops"], hf, iters, grad_tol=tol, forced_ops=r["ops"] + [0],
                  keep_gradients=True)
    assert len(o["ops"]) == r["n_iter"]
    for k, j in enumerate(r["ops"]):
        a = np.abs(o["grads"][k])
        assert a[j] >= a.max() * (1 - 1e-9), (k, j, a[j], a.max())
    assert np.abs(np.array(o["energies"]) - r["energies"]).max() <= etol
    assert np.abs(np.array(o["thetas"]) - r["thetas"]).max() <= 1e-8
    assert np.abs(np.array(o["gnorms"]) - r["gnorms"]).max() <= 1e-9
    assert o["substeps"] == r["substeps"]
    fid = abs(np.vdot(o["psi"], psi_gpu)) ** 2
    assert fid >= 1 - 1e-12
    return o


@pytest.mark.parametrize("use_graph", [True, False])
def test_adapt_4q_10_iterations(g, ctx, use_graph):
    _say(f"[adapt] 4q graph={use_graph}")
    s = system(g, 4, "jw")
    r, psi = _adapt_gpu(g, ctx, s, 4, 10, use_graph=use_graph)
    _check_against_oracle(s, r, psi, 10)


@pytest.mark.parametrize("mapping", ["jw", "bk"])
def test_adapt_12q_30_iterations(g, ctx, mapping):
    _say(f"[adapt] 12q {mapping}")
    s = system(g, 12, mapping)
    r, psi = _adapt_gpu(g, ctx, s, 12, 30)
    assert r["n_iter"] == 30
    _check_against_oracle(s, r, psi, 30)


@pytest.mark.parametrize("schedule", [2, 4])
@pytest.mark.parametrize("nq,mapping", [(12, "bk"), (6, "jw"), (4, "jw")])
def test_adapt_register_blocked_schedules(g, ctx, schedule, nq, mapping):
    """2 or 4 amplitudes per lane (tiles of 128 or 256, ragged when the state
    is smaller than a tile) must follow the oracle like the 1-per-lane path."""
    _say(f"[adapt] {nq}q {mapping} schedule={schedule}")
    s = system(g, nq, mapping)
    iters = 12 if nq >= 6 else 6
    r, psi = _adapt_gpu(g, ctx, s, nq, iters, schedule=schedule)
    _check_against_oracle(s, r, psi, iters)


def test_phase_trace_only_in_the_measurement_build(g, ctx):
    """The product library records no phase trace: a valid request is
    ENOTSUP, a bad row count EINVAL."""
    with pytest.raises(g.GocpError) as e:
        g.phase_trace(ctx, 0)
    assert e.value.code == -1
    with pytest.raises(g.GocpError) as e:
        g.phase_trace(ctx, 4)
    assert e.value.code == -5


def test_adapt_bad_schedule_rejected(g, ctx):
    s = system(g, 4, "jw")
    with pytest.raises(g.GocpError) as e:
        _adapt_gpu(g, ctx, s, 4, 2, schedule=3)
    assert e.value.code == -1


def test_adapt_12q_jw_equals_bk(g, ctx):
    rj, _ = _adapt_gpu(g, ctx, system(g, 12, "jw"), 12, 30)
    rb, _ = _adapt_gpu(g, ctx, system(g, 12, "bk"), 12, 30)
    assert rj["ops"] == rb["ops"]
    assert np.abs(rj["energies"] - rb["energies"]).max() <= 1e-10


def test_adapt_convergence_stop(g, ctx):
    s = system(g, 4, "jw")
    r, psi = _adapt_gpu(g, ctx, s, 4, 50, tol=1e-6)
    assert r["converged"] and r["n_iter"] < 50
    assert len(r["gnorms"]) == r["n_iter"] + 1 and r["gnorms"][-1] < 1e-6
    _check_against_oracle(s, r, psi, 50, tol=1e-6)


def test_adapt_14q_first_iterations(g, ctx):
    _say("[adapt] 14q 4 iterations")
    s = system(g, 14, "jw")
    r, psi = _adapt_gpu(g, ctx, s, 14, 4)
    _check_against_oracle(s, r, psi, 4)


@pytest.mark.parametrize("dtype,tol", [("c128", 1e-12), ("c64", 1e-12)])
@pytest.mark.parametrize("iters", [61, 64])
def test_carried_sigma_energy_matches_fresh_energy(g, ctx, dtype, tol, iters):
    """FP64 states carry sigma through each update between fresh H psi
    applications (complex64 states apply H afresh every iteration); the energy
    reported for the last iteration must match a fresh H psi on the stored
    state (61: carried since the last refresh; 64: refreshed)."""
    _say(f"[carry] 12q {dtype} {iters} iterations")
    s = system(g, 12, "bk")
    r, psi = _adapt_gpu(g, ctx, s, 12, iters, dtype)
    e_fresh = g.energy(ctx, s["gH"], to_dev(psi, dtype))
    assert r["n_iter"] == iters
    assert abs(r["energies"][-1] - e_fresh) <= tol


def test_complex64_form_long_run_stays_second_order(g, ctx):
    """Over 120 iterations the complex64 energies track the FP64 ones to
    ~1e-10 (Rayleigh quotients of the stored state are second order in its
    rounding); a scheme first order in the rounding shows ~1e-7 here."""
    _say("[c64] 12q 120 iterations")
    s = system(g, 12, "jw")
    r64, _ = _adapt_gpu(g, ctx, s, 12, 120, "c128")
    r32, _ = _adapt_gpu(g, ctx, s, 12, 120, "c64")
    k = 0
    while k < 120 and r32["ops"][k] == r64["ops"][k]:
        k += 1
    assert k >= 60
    assert np.abs(r32["energies"][:k + 1] - r64["energies"][:k + 1]).max() <= 1e-8


@pytest.mark.parametrize("mapping", ["jw", "bk"])
def test_complex64_form_14q(g, ctx, mapping):
    """complex64 statevector with FP64 accumulation against the FP64 path."""
    _say(f"[c64] 14q {mapping}")
    s = system(g, 14, mapping)
    r64, psi64 = _adapt_gpu(g, ctx, s, 14, 30, "c128")
    r32, psi32 = _adapt_gpu(g, ctx, s, 14, 30, "c64")
    assert np.abs(r32["energies"] - r64["energies"]).max() <= 1e-6
    fid = abs(np.vdot(psi64, psi32)) ** 2 / (np.vdot(psi32, psi32).real)
    assert fid >= 1 - 1e-6
    assert r32["ops"] == r64["ops"]


def test_complex64_compacted_line_search_dense_state(g, ctx):
    """From a dense random state every amplitude is active in the line search,
    so the compacted H v / H w dots of complex64 states run two 64-amplitude
    tiles per workgroup slot at 12 qubits; the trajectory must follow the
    FP64 path (whole-state H v / H w) from the same starting state."""
    _say("[c64] 12q dense start, compacted line search")
    s = system(g, 12, "jw")
    start = rand_state(12, 77).astype(np.complex64).astype(np.complex128)
    start /= np.linalg.norm(start)
    runs = {}
    for dtype in ("c128", "c64"):
        d = to_dev(start, dtype)
        runs[dtype] = g.adapt_solve(ctx, s["gH"], s["gP"], d, 10, grad_tol=0.0, schedule=1)
    r64, r32 = runs["c128"], runs["c64"]
    assert r32["ops"] == r64["ops"]
    assert np.abs(r32["energies"] - r64["energies"]).max() <= 1e-6
    assert np.abs(np.array(r32["thetas"]) - np.array(r64["thetas"])).max() <= 1e-5


def test_complex64_compacted_line_search_large_class(g, ctx):
    """A Hamiltonian with one X-mask class longer than a wave's share of the
    compacted H v / H w launch's stage (the diagonal class, 400 extra Z
    strings at 12 qubits): that launch stages whole chunks instead of each
    wave's own run.  The complex64 trajectory must follow the FP64 path."""
    _say("[c64] 12q large diagonal class, compacted line search with full staging")
    s = system(g, 12, "jw")
    x, z, c = s["gH"].terms()
    rng = np.random.default_rng(5)
    present = {int(zz) for xx, zz in zip(x, z) if int(xx) == 0}
    extra = [m for m in rng.permutation(np.arange(1, 1 << 12)) if int(m) not in present][:400]
    xs = np.concatenate([x, np.zeros(len(extra), dtype=x.dtype)])
    zs = np.concatenate([z, np.array(extra, dtype=z.dtype)])
    cs = np.concatenate([c, rng.uniform(-0.01, 0.01, len(extra))])
    H = g.pauli_hamiltonian_load_terms(12, xs, zs, cs)
    assert int(np.sum(H.terms()[0] == 0)) > 256
    runs = {}
    for dtype in ("c128", "c64"):
        psi = torch.zeros(1 << 12, dtype=torch.complex128 if dtype == "c128" else torch.complex64, device="cuda")
        g.state_basis(ctx, 12, s["hf"], psi)
        runs[dtype] = g.adapt_solve(ctx, H, s["gP"], psi, 12, grad_tol=0.0, schedule=1)
    r64, r32 = runs["c128"], runs["c64"]
    assert r32["ops"] == r64["ops"]
    assert np.abs(r32["energies"] - r64["energies"]).max() <= 1e-6


def _multichunk_12q(g, s, n_extra=3000, seed=9):
    """The 12-qubit Hamiltonian plus n_extra random Hermitian strings (an even
    number of Y factors, real folded coefficients): more strings and X-mask
    classes than one LDS stage chunk holds, so the tile kernels walk several
    chunks.  Returns the oracle Pauli sum and the library Hamiltonian."""
    x, z, c = s["gH"].terms()
    rng = np.random.default_rng(seed)
    have = set(zip(x.tolist(), z.tolist()))
    ex, ez, ec = [], [], []
    while len(ex) < n_extra:
        xx, zz = int(rng.integers(0, 1 << 12)), int(rng.integers(0, 1 << 12))
        if bin(xx & zz).count("1") % 2 or (xx, zz) in have:
            continue
        have.add((xx, zz))
        ex.append(xx); ez.append(zz); ec.append(float(rng.choice([-1, 1]) * rng.uniform(1e-3, 1e-2)))
    H = dict(s["H"])
    for xx, zz, cc in zip(ex, ez, ec):
        H[(xx, zz)] = cc * (1j ** bin(xx & zz).count("1"))   # unfold: c = c_folded i^y
    gH = g.pauli_hamiltonian_load_terms(12, np.concatenate([x, np.array(ex, dtype=x.dtype)]),
                                        np.concatenate([z, np.array(ez, dtype=z.dtype)]),
                                        np.concatenate([c, np.array(ec)]))
    assert gH.n_terms > 4096 and gH.n_classes > 1024
    return H, gH


def test_multichunk_energy_gradients_and_adapt(g, ctx):
    """H split over several LDS stage chunks (by strings and by classes):
    energy, sigma and pool gradients against the oracle, and a complex64
    ADAPT run against the FP64 path (grouped walk, compacted line search)."""
    _say("[multichunk] 12q + 3000 random strings")
    s = system(g, 12, "jw")
    H, gH = _multichunk_12q(g, s)
    psi = rand_state(12, 31)
    sig_ref = apply_h(H, psi)
    e_ref = o_energy(H, psi, sig_ref)
    sig = torch.zeros(1 << 12, dtype=torch.complex128, device="cuda")
    e = g.apply_hamiltonian(ctx, gH, to_dev(psi), sig)
    assert abs(e - e_ref) <= 1e-12 * max(1.0, abs(e_ref))
    assert np.abs(sig.cpu().numpy() - sig_ref).max() <= 1e-12 * max(1.0, np.abs(sig_ref).max())
    g_ref = o_gradients(s["ops"], psi, sig_ref)
    gg = g.pool_gradients(ctx, gH, s["gP"], to_dev(psi))
    assert np.abs(gg - g_ref).max() <= 1e-12 * max(1.0, np.abs(g_ref).max())
    runs = {}
    for dtype in ("c128", "c64"):
        d = torch.zeros(1 << 12, dtype=torch.complex128 if dtype == "c128" else torch.complex64, device="cuda")
        g.state_basis(ctx, 12, s["hf"], d)
        runs[dtype] = g.adapt_solve(ctx, gH, s["gP"], d, 8, grad_tol=0.0, schedule=1)
    assert runs["c64"]["ops"] == runs["c128"]["ops"]
    assert np.abs(runs["c64"]["energies"] - runs["c128"]["energies"]).max() <= 1e-6
