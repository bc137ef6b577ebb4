"""pool_gradients_noalloc: the allocation-free variant of pool_gradients.

Called through the C ABI and checked against pool_gradients (the same kernels
in the same order, so the values must agree bit for bit, well inside the
1e-12 relative bar of the FP64 path) on two calls in a row, the second with a
smaller problem and the other precision, so that the fixed workspace holds the
first call's contents when the second starts.  Also: the rejections (tables
not yet on the device, a workspace larger than the fixed array, bad
pointers), which return before any launch.
"""

import ctypes as C

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from workloads import molecular_integrals, electron_count


@pytest.fixture(scope="module")
def g():
    import paper_2607_15906_amd as g
    return g


@pytest.fixture(scope="module")
def ctx(g):
    return g.Context(0)


def _system(g, nq, mapping, seed):
    ne = electron_count(nq // 2)
    h1, eri, ec = molecular_integrals(nq // 2, seed)
    return g.pauli_hamiltonian_load(h1, eri, ec, mapping), g.pool_build(nq, ne, mapping)


def _state(nq, seed, dtype):
    rng = np.random.default_rng(seed)
    psi = rng.standard_normal(1 << nq) + 1j * rng.standard_normal(1 << nq)
    t = torch.from_numpy(psi / np.linalg.norm(psi) * 1.3).to("cuda")
    return t.to(dtype)


def _noalloc_raw(ctx, H, P, psi, out):
    from paper_2607_15906_amd._lib import load
    code = 0 if psi.dtype == torch.complex128 else 1
    return load().pool_gradients_noalloc(ctx.handle, H.handle, P.handle, C.c_void_p(psi.data_ptr()), code,
                                         C.cast(C.c_void_p(out.data_ptr()), C.POINTER(C.c_double)))


def test_noalloc_matches_pool_gradients_on_two_calls_second_smaller(g, ctx):
    cases = [(14, "jw", 14, torch.complex128), (12, "bk", 12, torch.complex64)]
    for k, (nq, mapping, seed, dt) in enumerate(cases):
        print(f"[noalloc] call {k}: {nq}q {mapping} {dt}", flush=True)
        H, P = _system(g, nq, mapping, seed)
        psi = _state(nq, 100 + nq, dt)
        ref = g.pool_gradients(ctx, H, P, psi)          # uploads the tables
        out = torch.full((P.n_ops,), float("nan"), dtype=torch.float64, device="cuda")
        assert _noalloc_raw(ctx, H, P, psi, out) == 0
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        assert np.abs(got - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max())
        assert np.array_equal(got, ref)
        # again on the same state: the workspace keeps the last call's contents
        out2 = torch.zeros_like(out)
        assert _noalloc_raw(ctx, H, P, psi, out2) == 0
        torch.cuda.synchronize()
        assert torch.equal(out, out2)


def test_noalloc_rejections(g, ctx):
    from paper_2607_15906_amd._lib import load
    # tables not on the device yet: a fresh Hamiltonian and pool
    H, P = _system(g, 10, "jw", 77)
    psi = _state(10, 3, torch.complex128)
    out = torch.zeros(P.n_ops, dtype=torch.float64, device="cuda")
    assert _noalloc_raw(ctx, H, P, psi, out) == -1
    assert b"not on this device" in load().gocp_last_error()
    g.pool_gradients(ctx, H, P, psi)
    assert _noalloc_raw(ctx, H, P, psi, out) == 0
    # a workspace beyond the fixed array: the 16-qubit Pauli pool (M = 2688)
    H16, _ = _system(g, 16, "jw", 16)
    P16 = g.pool_build_pauli(16, 8, "jw")
    psi16 = torch.zeros(1 << 16, dtype=torch.complex128, device="cuda")
    out16 = torch.zeros(P16.n_ops, dtype=torch.float64, device="cuda")
    assert _noalloc_raw(ctx, H16, P16, psi16, out16) == -5
    assert b"exceeds" in load().gocp_last_error()
    # null pointers
    rc = load().pool_gradients_noalloc(ctx.handle, H.handle, P.handle, None, 0,
                                       C.cast(C.c_void_p(out.data_ptr()), C.POINTER(C.c_double)))
    assert rc == -1
    rc = load().pool_gradients_noalloc(ctx.handle, H.handle, P.handle, C.c_void_p(psi.data_ptr()), 0, None)
    assert rc == -1
    torch.cuda.synchronize()


def test_noalloc_binding_checks_sizes(g, ctx):
    H, P = _system(g, 8, "bk", 8)
    psi = _state(8, 5, torch.complex64)
    ref = g.pool_gradients(ctx, H, P, psi)
    out = torch.zeros(P.n_ops, dtype=torch.float64, device="cuda")
    g.pool_gradients_noalloc(ctx, H, P, psi, out)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), ref)
    with pytest.raises(ValueError):
        g.pool_gradients_noalloc(ctx, H, P, psi, torch.zeros(P.n_ops - 1, dtype=torch.float64, device="cuda"))
    with pytest.raises(ValueError):
        g.pool_gradients_noalloc(ctx, H, P, _state(10, 5, torch.complex64), out)
