"""GPU tests of the serving form (continuous batching, through the C ABI).

Each request must compute exactly what adapt_solve computes for it alone,
whether it runs alone, in a mix, or joins a running set; admission must keep
the admitted device footprint within the budget.
"""

import time

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from workloads import molecular_integrals, electron_count


def _say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def g():
    import paper_2607_15906_amd as g
    return g


@pytest.fixture(scope="module")
def ctx(g):
    return g.Context(0)


def _req(g, nq, mapping, seed):
    ne = electron_count(nq // 2)
    h1, eri, ec = molecular_integrals(nq // 2, seed)
    return dict(H=g.pauli_hamiltonian_load(h1, eri, ec, mapping), P=g.pool_build(nq, ne, mapping),
                hf=g.hf_index(nq, ne, mapping), nq=nq)


def _solo(g, ctx, r, max_iter, tol, dtype, schedule=1):
    psi = torch.zeros(1 << r["nq"], dtype=dtype, device="cuda")
    psi[r["hf"]] = 1.0
    return g.adapt_solve(ctx, r["H"], r["P"], psi, max_iter, grad_tol=tol, schedule=schedule)


def _drain(srv, tickets, timeout_s=60.0, watch=None):
    out = {}
    t0 = time.time()
    while len(out) < len(tickets):
        for t in tickets:
            if t not in out:
                r = srv.poll(t)
                if r is not None:
                    out[t] = r
        if watch:
            watch(srv.stats())
        if time.time() - t0 > timeout_s:
            raise TimeoutError("serving requests did not finish")
        time.sleep(0.001)
    return out


def _same(a, b):
    assert a["ops"] == b["ops"]
    assert a["n_iter"] == b["n_iter"] and a["converged"] == b["converged"]
    assert np.array_equal(a["energies"], b["energies"])
    assert np.array_equal(a["gnorms"], b["gnorms"])
    assert np.array_equal(a["thetas"], b["thetas"])


@pytest.mark.parametrize("dtype,code,R", [(torch.complex64, 1, 1), (torch.complex128, 0, 1),
                                          (torch.complex64, 1, 4)])
def test_mix_equals_solo(g, ctx, dtype, code, R):
    _say(f"[serve] mix {dtype} R={R}")
    reqs = [_req(g, *s) for s in [(8, "jw", 1), (10, "bk", 2), (12, "jw", 3), (8, "bk", 4),
                                  (10, "jw", 5), (12, "bk", 6)]]
    srv = g.Server(ctx, hbm_budget_bytes=1 << 30, max_slots=16, dtype=code, iters_per_step=3,
                   amps_per_lane=R)
    tickets = [srv.submit(r["H"], r["P"], 60, 1e-3) for r in reqs]
    res = _drain(srv, tickets)
    srv.close()
    for r, t in zip(reqs, tickets):
        st, rec, info = res[t]
        assert st == 0 and info["status"] == 0 and info["n_qubits"] == r["nq"]
        assert info["t_submit_ns"] <= info["t_admit_ns"] <= info["t_done_ns"]
        _same(rec, _solo(g, ctx, r, 60, 1e-3, dtype, schedule=R))


def test_budget_forces_queueing_and_is_respected(g, ctx):
    _say("[serve] budget")
    reqs = [_req(g, 12, "jw" if i % 2 else "bk", 40 + i) for i in range(6)]
    fp = max(g.request_footprint(r["H"], r["P"], 40) for r in reqs)
    budget = int(2.5 * fp)                          # at most two admitted at once
    srv = g.Server(ctx, hbm_budget_bytes=budget, max_slots=8, dtype=1, iters_per_step=2)
    seen = {"max_bytes": 0, "max_active": 0, "queued": 0}

    def watch(st):
        seen["max_bytes"] = max(seen["max_bytes"], st["bytes_in_use"])
        seen["max_active"] = max(seen["max_active"], st["active"])
        seen["queued"] = max(seen["queued"], st["queued"])

    tickets = [srv.submit(r["H"], r["P"], 40, 1e-3) for r in reqs]
    res = _drain(srv, tickets, watch=watch)
    srv.close()
    assert seen["max_bytes"] <= budget
    assert seen["max_active"] <= 2
    assert seen["queued"] >= 1
    admits = sorted(res[t][2]["t_admit_ns"] for t in tickets)
    assert admits[-1] > min(res[t][2]["t_done_ns"] for t in tickets)   # later ones waited for room
    for r, t in zip(reqs, tickets):
        _same(res[t][1], _solo(g, ctx, r, 40, 1e-3, torch.complex64))


def test_late_arrivals_join_running_set(g, ctx):
    _say("[serve] late arrivals")
    first = [_req(g, 12, "jw", 60), _req(g, 12, "bk", 61)]
    late = [_req(g, 10, "jw", 62), _req(g, 8, "bk", 63)]
    srv = g.Server(ctx, hbm_budget_bytes=1 << 30, max_slots=8, dtype=1, iters_per_step=1)
    t_first = [srv.submit(r["H"], r["P"], 200, 1e-6) for r in first]
    t0 = time.time()
    while srv.stats()["active"] < 2 and time.time() - t0 < 30:
        time.sleep(0.0005)
    t_late = [srv.submit(r["H"], r["P"], 200, 1e-3) for r in late]
    res = _drain(srv, t_first + t_late)
    srv.close()
    done_first = min(res[t][2]["t_done_ns"] for t in t_first)
    assert any(res[t][2]["t_admit_ns"] < done_first for t in t_late)   # overlapped on the device
    for r, t in zip(first, t_first):
        _same(res[t][1], _solo(g, ctx, r, 200, 1e-6, torch.complex64))
    for r, t in zip(late, t_late):
        _same(res[t][1], _solo(g, ctx, r, 200, 1e-3, torch.complex64))


def test_adaptive_schedule_agrees_with_solo(g, ctx):
    """amps_per_lane=0 picks the blocking from the active set (six 14-qubit
    requests give 1536 tiles: wider blocking); results agree with solo runs to
    rounding."""
    _say("[serve] adaptive schedule")
    reqs = [_req(g, 14, "jw" if i % 2 else "bk", 90 + i) for i in range(6)] + [_req(g, 8, "jw", 96)]
    srv = g.Server(ctx, hbm_budget_bytes=1 << 31, max_slots=16, dtype=0, iters_per_step=4, amps_per_lane=0)
    tickets = [srv.submit(r["H"], r["P"], 24, 1e-4) for r in reqs]
    res = _drain(srv, tickets)
    srv.close()
    for r, t in zip(reqs, tickets):
        st, rec, info = res[t]
        assert st == 0
        solo = _solo(g, ctx, r, 24, 1e-4, torch.complex128)
        assert rec["ops"] == solo["ops"] and rec["n_iter"] == solo["n_iter"]
        assert np.abs(rec["energies"] - solo["energies"]).max() <= 1e-10
        assert np.abs(rec["gnorms"] - solo["gnorms"]).max() <= 1e-9


def test_bad_server_schedule_rejected(g, ctx):
    with pytest.raises(g.GocpError):
        g.Server(ctx, hbm_budget_bytes=1 << 30, max_slots=4, dtype=1, amps_per_lane=3)


def test_request_larger_than_budget_is_rejected(g, ctx):
    r = _req(g, 12, "jw", 70)
    small = _req(g, 8, "jw", 71)
    fp = g.request_footprint(r["H"], r["P"], 20)
    srv = g.Server(ctx, hbm_budget_bytes=fp // 2, max_slots=4, dtype=1)
    t_big = srv.submit(r["H"], r["P"], 20, 1e-3)
    t_ok = srv.submit(small["H"], small["P"], 20, 1e-3)
    res = _drain(srv, [t_big, t_ok])
    srv.close()
    assert res[t_big][0] == -2 and res[t_big][1] is None
    assert res[t_ok][0] == 0


def test_shutdown_with_requests_in_flight(g, ctx):
    reqs = [_req(g, 12, "jw", 80 + i) for i in range(3)]
    srv = g.Server(ctx, hbm_budget_bytes=1 << 30, max_slots=1, dtype=1)
    for r in reqs:
        srv.submit(r["H"], r["P"], 300, 0.0)
    time.sleep(0.01)
    srv.close()                                   # cancels; must not hang or fault
    assert True


def test_admission_failure_ends_that_request_only(g, ctx, monkeypatch):
    """The server's second admission is made to fail from the host (the test
    hook GOCP_TEST_FAIL_ADMISSION): that request ends with GOCP_EDEVICE, every
    other request completes normally, and no poll waits forever."""
    _say("[serve] admission failure")
    reqs = [_req(g, 8, "jw" if i % 2 else "bk", 110 + i) for i in range(4)]
    monkeypatch.setenv("GOCP_TEST_FAIL_ADMISSION", "2")
    srv = g.Server(ctx, hbm_budget_bytes=1 << 28, max_slots=8, dtype=1, iters_per_step=2)
    monkeypatch.delenv("GOCP_TEST_FAIL_ADMISSION")
    tickets = [srv.submit(r["H"], r["P"], 30, 1e-3) for r in reqs]
    res = _drain(srv, tickets)
    st = srv.stats()
    srv.close()
    codes = [res[t][0] for t in tickets]
    assert codes.count(-3) == 1 and codes.count(0) == 3, codes
    assert st["bytes_in_use"] == 0
    for r, t in zip(reqs, tickets):
        if res[t][0] == 0:
            _same(res[t][1], _solo(g, ctx, r, 30, 1e-3, torch.complex64))


def test_bytes_in_use_is_the_admitted_blocks(g, ctx):
    """bytes_in_use counts each admitted request's arena block (its workspace
    and its own copy of the Hamiltonian's and pool's device tables) and drops
    to zero once the requests have finished."""
    _say("[serve] bytes in use")
    r = _req(g, 12, "jw", 120)
    block = g.request_footprint(r["H"], r["P"], 400, 1)
    srv = g.Server(ctx, hbm_budget_bytes=1 << 28, max_slots=4, dtype=1, iters_per_step=1)
    t = srv.submit(r["H"], r["P"], 400, 0.0)
    seen = set()
    t0 = time.time()
    while srv.poll(t) is None:
        seen.add(srv.stats()["bytes_in_use"])
        assert time.time() - t0 < 60
    st = srv.stats()
    srv.close()
    assert block in seen
    assert max(seen) == block
    assert st["bytes_in_use"] == 0 and st["completed"] == 1
