"""GPU parity of the GOCP multi-operator step (taylor5_apply_family) against
the FP64 oracle, through the C ABI.

1-4 members of one GOCP family (X masks independent over GF(2)) applied in one
pass; 4 qubits (one partial workgroup), 8, 12 and 14 qubits, JW and BK.
Tolerances: FP64 states 1e-13 per amplitude; complex64 states 1e-6 against the
oracle on the same (rounded) input.
"""

import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle.pool import pool_operators
from oracle.statevec import taylor5_family
from workloads import electron_count


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


def pools(g, nq, mapping):
    key = (nq, mapping)
    if key not in _cache:
        ne = electron_count(nq // 2)
        P = g.pool_build(nq, ne, mapping)
        fam, K, _ = g.gocp_partition(P)
        _cache[key] = (P, fam, [A for _, _, A in pool_operators(nq, ne, mapping)])
    return _cache[key]


def independent_members(P, fam, n):
    """The first family (creation order) holding n members whose X masks are
    independent over GF(2); those members in pool order."""
    for f in range(int(fam.max()) + 1):
        basis, pick = {}, []
        for k in np.flatnonzero(fam == f):
            v = P.op(int(k))[2]
            for bit in sorted(basis, reverse=True):
                if (v >> bit) & 1:
                    v ^= basis[bit]
            if v:
                basis[v.bit_length() - 1] = v
                pick.append(int(k))
            if len(pick) == n:
                return pick
    return None


def rand_state(nq, seed):
    rng = np.random.default_rng(seed)
    psi = rng.standard_normal(1 << nq) + 1j * rng.standard_normal(1 << nq)
    return psi / np.linalg.norm(psi)


@pytest.mark.parametrize("nq", [4, 8, 12, 14])
@pytest.mark.parametrize("n", [1, 2, 3, 4])
@pytest.mark.parametrize("mapping", ["jw", "bk"])
def test_family_step_matches_oracle(g, ctx, nq, n, mapping):
    P, fam, ops = pools(g, nq, mapping)
    mem = independent_members(P, fam, n)
    if mem is None:
        pytest.skip(f"no family with {n} independent members at {nq} qubits")
    _say(f"[fused] nq={nq} n={n} {mapping} ops={mem}")
    rng = np.random.default_rng(nq * 10 + n)
    thetas = rng.uniform(-2.5, 2.5, n)
    psi = rand_state(nq, 80 + nq + n)
    ref, subs = taylor5_family([ops[j] for j in mem], thetas, psi)
    d = torch.from_numpy(psi).to("cuda")
    ns = g.taylor5_apply_family(ctx, P, mem, thetas, d)
    assert ns.tolist() == subs
    assert np.abs(d.cpu().numpy() - ref).max() <= 1e-13
    # complex64 storage, FP64 arithmetic
    d32 = torch.from_numpy(psi).to(torch.complex64).to("cuda")
    p32 = d32.cpu().numpy().astype(np.complex128)
    ref32, _ = taylor5_family([ops[j] for j in mem], thetas, p32 / np.linalg.norm(p32))
    g.taylor5_apply_family(ctx, P, mem, thetas, d32)
    assert np.abs(d32.cpu().numpy().astype(np.complex128) - ref32).max() <= 1e-6


@pytest.mark.parametrize("nq,mapping", [(12, "jw"), (14, "bk")])
def test_family_step_equals_sequential_single_chains(g, ctx, nq, mapping):
    P, fam, _ = pools(g, nq, mapping)
    mem = independent_members(P, fam, 4) or independent_members(P, fam, 3)
    thetas = np.linspace(-1.3, 2.2, len(mem))
    psi = rand_state(nq, 7)
    a = torch.from_numpy(psi).to("cuda")
    b = a.clone()
    g.taylor5_apply_family(ctx, P, mem, thetas, a)
    for j, t in zip(mem, thetas):
        g.taylor5_apply(ctx, P, j, float(t), b)
    assert torch.abs(a - b).max().item() <= 1e-13


def test_family_step_zero_angles_and_errors(g, ctx):
    P, fam, _ = pools(g, 8, "jw")
    mem = independent_members(P, fam, 2)
    psi = torch.from_numpy(rand_state(8, 1)).to("cuda")
    keep = psi.clone()
    ns = g.taylor5_apply_family(ctx, P, mem, [0.0, 0.0], psi)
    assert ns.tolist() == [0, 0] and torch.equal(psi, keep)
    other = [k for k in range(P.n_ops) if fam[k] != fam[mem[0]]][0]
    for bad, why in (([mem[0], other], "families"), ([mem[0], mem[0]], "twice"),
                     (mem * 3 if len(mem) * 3 > 4 else mem + mem + mem, "1 to 4"),
                     ([P.n_ops], "range")):
        with pytest.raises(g.GocpError):
            g.taylor5_apply_family(ctx, P, bad, [0.1] * len(bad), psi)
    assert torch.equal(psi, keep)
    # two strings of one double that commute share their X mask: dependent
    Q = g.pool_build_pauli(8, 4, "jw")
    qf, _, _ = g.gocp_partition(Q)
    pair = next(((a, b) for a in range(Q.n_ops) for b in range(a + 1, Q.n_ops)
                 if qf[a] == qf[b] and Q.op(a)[2] == Q.op(b)[2]), None)
    if pair is not None:
        with pytest.raises(g.GocpError):
            g.taylor5_apply_family(ctx, Q, list(pair), [0.1, 0.2], psi)
    assert torch.equal(psi, keep)
