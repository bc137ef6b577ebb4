"""The one-shot calls reuse the descriptor and row tables left in the
context's workspace by the previous call with the same Hamiltonian, pool,
state, sigma and precision.  Alternating keys, freed and rebuilt objects and
repeated keys must all give the oracle's results."""

import gc
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle.mapping import hamiltonian
from oracle.pool import pool_operators, pauli_pool_operators
from oracle.statevec import apply_h, energy as o_energy, gradients as o_gradients, taylor5 as o_taylor5
from workloads import molecular_integrals, electron_count


def test_one_shot_workspace_reuse_follows_every_key():
    import paper_2607_15906_amd as g
    print("[oneshot] alternating keys", flush=True)
    sys.stdout.flush()
    ctx = g.Context(0)
    nq = 10
    ne = electron_count(nq // 2)
    h1, eri, ec = molecular_integrals(nq // 2, 3)
    Hs = {m: (g.pauli_hamiltonian_load(h1, eri, ec, m), hamiltonian(h1, eri, ec, m)) for m in ("jw", "bk")}
    rng = np.random.default_rng(12)
    states = [rng.standard_normal(1 << nq) + 1j * rng.standard_normal(1 << nq) for _ in range(2)]
    states = [s / np.linalg.norm(s) for s in states]
    devs = [torch.from_numpy(s).to("cuda") for s in states]
    fer = [A for _, _, A in pool_operators(nq, ne, "jw")]
    pau = [B for _, _, B in pauli_pool_operators(nq, ne, "jw")]
    for rep in range(3):
        for m in ("jw", "bk"):
            gH, oH = Hs[m]
            for k in (0, 1, 1, 0):
                e = g.energy(ctx, gH, devs[k])
                assert abs(e - o_energy(oH, states[k])) <= 1e-12 * max(1.0, abs(e))
        # a pool freed and another built (possibly at the same address)
        P = g.pool_build(nq, ne, "jw") if rep % 2 == 0 else g.pool_build_pauli(nq, ne, "jw")
        ops = fer if rep % 2 == 0 else pau
        gH, oH = Hs["jw"]
        for k in (1, 1, 0):
            gg = g.pool_gradients(ctx, gH, P, devs[k])
            ref = o_gradients(ops, states[k], apply_h(oH, states[k]))
            assert np.abs(gg - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max())
        # Taylor calls on a pool alone, then on the same state in complex64
        psi = torch.from_numpy(states[0]).to("cuda")
        g.taylor5_apply(ctx, P, 3, 0.4, psi)
        ref, _ = o_taylor5(ops[3], 0.4, states[0])
        assert np.abs(psi.cpu().numpy() - ref).max() <= 1e-13
        p32 = torch.from_numpy(states[0]).to(torch.complex64).to("cuda")
        r32 = p32.cpu().numpy().astype(np.complex128)
        g.taylor5_apply(ctx, P, 3, 0.4, p32)
        ref32, _ = o_taylor5(ops[3], 0.4, r32 / np.linalg.norm(r32))
        assert np.abs(p32.cpu().numpy().astype(np.complex128) - ref32).max() <= 1e-6
        del P
        gc.collect()


def test_one_shot_taylor_calls_between_state_calls():
    """Taylor calls upload no state record (their kernels read none); energy
    and gradient calls around them, with the descriptor of the same key in
    place or not, still start from a fresh record and follow the oracle."""
    import paper_2607_15906_amd as g
    print("[oneshot] Taylor calls between energy and gradient calls", flush=True)
    ctx = g.Context(0)
    nq = 10
    ne = electron_count(nq // 2)
    h1, eri, ec = molecular_integrals(nq // 2, 5)
    gH, oH = g.pauli_hamiltonian_load(h1, eri, ec, "jw"), hamiltonian(h1, eri, ec, "jw")
    P = g.pool_build(nq, ne, "jw")
    ops = [A for _, _, A in pool_operators(nq, ne, "jw")]
    rng = np.random.default_rng(21)
    s = rng.standard_normal(1 << nq) + 1j * rng.standard_normal(1 << nq)
    s /= np.linalg.norm(s)
    psi = torch.from_numpy(s.copy()).to("cuda")
    for j, th in ((5, 0.7), (5, -0.2), (17, 1.3)):
        for _ in range(2):                         # the second time with every key already in place
            gg = g.pool_gradients(ctx, gH, P, psi)
            ref = o_gradients(ops, s, apply_h(oH, s))
            assert np.abs(gg - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max())
            e = g.energy(ctx, gH, psi)
            assert abs(e - o_energy(oH, s)) <= 1e-12 * max(1.0, abs(e))
        g.taylor5_apply(ctx, P, j, th, psi)
        s, _ = o_taylor5(ops[j], th, s)
        assert np.abs(psi.cpu().numpy() - s).max() <= 1e-13
