#!/usr/bin/env python3
"""Benchmark of the GOCP ADAPT-VQE hot path on one MI355X.

A step is one ADAPT iteration of the 14-qubit, 6-electron (BeH2-sized,
Tables I-II) synthetic system under Jordan-Wigner: gradient screen of the
whole pool, selection, line search, fifth-order Taylor update and the new
energy, with a complex64 statevector and FP64 accumulation.  W untimed
iterations (captured-graph replays) precede exactly K timed iterations,
launched directly so that the dominant kernel can be bracketed by its own
dispatch timestamps (HIP events) in every n-th iteration.  Prints one JSON
line.

Also reported: the precision form against the FP64 oracle, the complex128
path, the Bravyi-Kitaev mapping and a later window of the same run, the Pauli
pool, the GOCP multi-operator step, the 64-instance batched form (with its
roofline and an oracle baseline over worker processes) and the serving stream
(512 requests after 32 warm-up ones, at 0.7x and 1.2x of capacity).  The CPU
legs (the oracle) run first, before the GPU is touched.
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "ADAPT iters/s + Pauli-term amp-updates/s at 14q; p50/p99 solve latency"
FP64_PEAK_TFLOPS = 78.6       # MI355X FP64 vector peak (FMA = 2 flops)
# VALU issue peak: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz lane operations per
# second (a wave64 instruction occupies a SIMD for four cycles; FP64 adds and
# FMAs issue at this rate too)
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
# algorithmic lane operations per string-amplitude of a Pauli-string
# application: AND with the Z mask, popcount, sign, accumulate, and the
# multiply-add by the gathered amplitude
LANE_OPS_PER_STRING_AMP = 5
# HBM bytes per launch of the dominant kernel (FETCH_SIZE and WRITE_SIZE,
# scaled by a 256 MiB copy), from the rocprofv3 counter runs summarised under
# profiles/; keyed by (kernel, amplitudes per lane).  An entry is removed when
# the kernel changes, until the counters are taken again.
TRAFFIC_BYTES = {("k_energy_screen", 1): 2592552}


def _schedule_fields(code):
    """A batch's schedule code as its two parts: amplitudes per lane and the
    compacted H v, H w launch's workgroups per tile slot."""
    return {"amps_per_lane": code & 0xFF, "hvw_parts": (code >> 8) or 8}


def _say(msg):
    print(msg, file=sys.stderr, flush=True)


def _pct(x, q):
    import numpy as np
    return round(float(np.percentile(np.asarray(x), q)), 3) if len(x) else None


# ---------------------------------------------------------------- CPU legs (oracle)

def _oracle_system(nq, ne, mapping, seed):
    from oracle.mapping import hamiltonian, hf_index
    from oracle.pool import pool_operators
    from workloads import molecular_integrals
    h1, eri, ec = molecular_integrals(nq // 2, seed)
    return hamiltonian(h1, eri, ec, mapping), [A for _, _, A in pool_operators(nq, ne, mapping)], \
        hf_index(nq, ne, mapping)


def oracle_headline(nq, ne, mapping, seed, iters):
    """The oracle on the first `iters` iterations of the headline system, one
    host thread: the CPU baseline, and the reference of the precision form."""
    import numpy as np
    from threadpoolctl import threadpool_limits
    from oracle.adapt import adapt_run
    from oracle.statevec import apply_h, gradients
    H, ops, hf = _oracle_system(nq, ne, mapping, seed)
    psi0 = np.zeros(1 << nq, dtype=np.complex128)
    psi0[hf] = 1.0
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        o = adapt_run(H, ops, psi0, iters, keep_gradients=True)
        dt = time.perf_counter() - t0
        g_final = gradients(ops, o["psi"], apply_h(H, o["psi"]))
    return dict(run=o, seconds=dt, g_final=g_final, H=H, ops=ops, psi0=psi0)


def _oracle_task(spec):
    """One worker's share of the batched baseline: one instance, `iters`
    oracle iterations, one thread."""
    import numpy as np
    from threadpoolctl import threadpool_limits
    from oracle.adapt import adapt_run
    nq, ne, mapping, seed, iters = spec
    with threadpool_limits(limits=1):
        H, ops, hf = _oracle_system(nq, ne, mapping, seed)
        psi0 = np.zeros(1 << nq, dtype=np.complex128)
        psi0[hf] = 1.0
        t0 = time.perf_counter()
        adapt_run(H, ops, psi0, iters)
        return time.perf_counter() - t0


def sparse_headline(nq, ne, mapping, seed, iters):
    """The sparse-matrix CPU baseline (the paper's own engine's approach: H and
    the pool as precomputed CSR matrices) on the first `iters` iterations of
    the headline system, one host thread."""
    import numpy as np
    from threadpoolctl import threadpool_limits
    from oracle.sparse import psum_csr, adapt_run_csr
    H, ops, hf = _oracle_system(nq, ne, mapping, seed)
    psi0 = np.zeros(1 << nq, dtype=np.complex128)
    psi0[hf] = 1.0
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        Hm = psum_csr(H, nq)
        Ams = [psum_csr(A, nq) for A in ops]
        norms = [sum(abs(c) for c in A.values()) for A in ops]
        t1 = time.perf_counter()
        adapt_run_csr(Hm, Ams, norms, psi0, iters)
        t2 = time.perf_counter()
    return {"value": round(iters / (t2 - t1), 3), "unit": "iters/s", "cores": 1, "kind": "sparse matrices",
            "sample": f"first {iters} ADAPT iterations of the same 14q JW system from Hartree-Fock with H "
                      f"({Hm.nnz} nonzeros) and the pool as scipy CSR matrices, one thread, {t2 - t1:.2f} s; "
                      f"building the matrices took {t1 - t0:.2f} s more"}


def _oracle_solve_task(spec):
    """One served request solved by the oracle (one thread): seconds, iterations."""
    import numpy as np
    from threadpoolctl import threadpool_limits
    from oracle.adapt import adapt_run
    nq, ne, mapping, seed, max_iter, tol = spec
    with threadpool_limits(limits=1):
        H, ops, hf = _oracle_system(nq, ne, mapping, seed)
        psi0 = np.zeros(1 << nq, dtype=np.complex128)
        psi0[hf] = 1.0
        t0 = time.perf_counter()
        r = adapt_run(H, ops, psi0, max_iter, grad_tol=tol)
        return time.perf_counter() - t0, len(r["ops"])


def oracle_serving_baseline(n_req, workers, nq=8):
    """The oracle solving the first `n_req` `nq`-qubit requests of the serving
    stream (||g|| < 1e-3, at most 300 iterations) on `workers` processes
    (forked before the GPU is touched); larger requests take the oracle
    minutes each."""
    import multiprocessing as mp
    from workloads import serving_requests
    specs = [(d["n_qubits"], d["n_electrons"], d["mapping"], d["seed"], 300, 1e-3)
             for d in serving_requests(64 * n_req, rate_hz=1.0) if d["n_qubits"] == nq][:n_req]
    ctx = mp.get_context("fork")
    t0 = time.perf_counter()
    with ctx.Pool(workers) as pool:
        per = pool.map(_oracle_solve_task, specs, chunksize=1)
    wall = time.perf_counter() - t0
    return specs, {"value": round(len(specs) / wall, 3), "unit": "solves/s", "cores": workers, "kind": "oracle",
                   "sample": f"the first {len(specs)} {nq}-qubit requests of the serving stream, FP64 NumPy "
                             f"oracle on {workers} worker processes (one thread each); {wall:.1f} s wall, "
                             f"{sum(t for t, _ in per):.1f} s of solves, {sum(k for _, k in per)} iterations"}


def oracle_batch_baseline(iters, workers):
    """The oracle over the 64 batched instances, `iters` iterations each, on
    `workers` processes (forked before the GPU is touched)."""
    import multiprocessing as mp
    from workloads import batched_instances
    specs = [(d["n_qubits"], d["n_electrons"], d["mapping"], d["seed"], iters) for d in batched_instances()]
    ctx = mp.get_context("fork")
    t0 = time.perf_counter()
    with ctx.Pool(workers) as pool:
        per = pool.map(_oracle_task, specs, chunksize=1)
    wall = time.perf_counter() - t0
    return {"value": round(len(specs) * iters / wall, 4), "unit": "instance-iters/s", "cores": workers,
            "kind": "oracle", "sample": f"{iters} ADAPT iterations of each of the 64 batched instances, FP64 "
                                        f"NumPy oracle on {workers} worker processes (one thread each); "
                                        f"{wall:.1f} s wall, {sum(per):.1f} s of iterations (Hamiltonian and "
                                        f"pool construction inside the wall time)"}


# ---------------------------------------------------------------- GPU legs

def _system(g, nq, ne, mapping, seed):
    from workloads import molecular_integrals
    h1, eri, ec = molecular_integrals(nq // 2, seed)
    return g.pauli_hamiltonian_load(h1, eri, ec, mapping), g.pool_build(nq, ne, mapping)


def _hf_state(g, ctx, nq, ne, mapping, dtype):
    import torch
    t = torch.zeros(1 << nq, dtype=dtype, device="cuda")
    g.state_basis(ctx, nq, g.hf_index(nq, ne, mapping), t)
    return t


def _string_amps(nq, T, S, off, ops, subs):
    """Algorithmic Pauli-term amplitude updates of the given iterations:
    2^n (3T + S + 2k + 5 k s) per iteration, k = strings of the chosen
    operator (every string applied to every amplitude counts once, whatever
    the kernels skip, fuse or factor)."""
    tot = 0
    for j, s in zip(ops, subs):
        k = int(off[j + 1] - off[j])
        tot += 3 * T + S + 2 * k + 5 * k * s
    return tot * (1 << nq)


def run_adapt_timed(g, ctx, H, P, nq, ne, mapping, dtype, steps, warmup, schedule=0, timed_kernel=3,
                    sample_every=2):
    """Warm-up iterations (graph replays), then `steps` timed iterations
    launched directly, with dispatch-timestamp events around the launch of
    Batch.STEP_KERNELS[timed_kernel] in every sample_every-th of them.
    Returns (batch, record, seconds, mean kernel ms, launches sampled)."""
    import torch
    psi = _hf_state(g, ctx, nq, ne, mapping, dtype)
    b = g.Batch(ctx, [H], [P], [psi], max_iter=warmup + steps, use_graph=True, schedule=schedule)
    if warmup:
        b.step(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, kms = b.step_timed(steps, timed_kernel, sample_every)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    r = b.result(0)
    r["psi"] = psi
    return b, r, dt, kms, (steps + sample_every - 1) // sample_every


def _fused_step_timing(g, ctx, P, nq, reps=200):
    """One GOCP multi-operator step (four members of one family, X masks
    independent) against the same four operators applied one call each,
    on complex64 and complex128 states; mean microseconds per step over
    back-to-back steps on the context's stream (torch's current one): the
    median over five batches of reps / 5 steps, after 20 untimed steps."""
    import numpy as np
    import torch
    fam, _, _ = g.gocp_partition(P)
    mem = None
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
            if len(pick) == 4:
                mem = pick
                break
        if mem:
            break
    thetas = [0.3, -0.2, 0.45, -0.1]
    res = {"ops": mem, "thetas": thetas, "reps": reps}
    for name, dt in (("c64", torch.complex64), ("c128", torch.complex128)):
        psi = torch.zeros(1 << nq, dtype=dt, device="cuda")
        psi[0] = 1.0
        psi += 1e-3
        times = {}
        for mode in ("fused", "sequential"):
            def step():
                if mode == "fused":
                    g.taylor5_apply_family(ctx, P, mem, thetas, psi)
                else:
                    for j, t in zip(mem, thetas):
                        g.taylor5_apply(ctx, P, j, t, psi)
            for _ in range(20):
                step()
            per = []
            for _ in range(5):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                torch.cuda.synchronize()
                e0.record()
                for _ in range(max(1, reps // 5)):
                    step()
                e1.record()
                torch.cuda.synchronize()
                per.append(e0.elapsed_time(e1) * 1e3 / max(1, reps // 5))
            times[mode] = float(np.median(per))
        res[name] = {"fused_us": round(times["fused"], 3), "sequential_us": round(times["sequential"], 3),
                     "speedup": round(times["sequential"] / times["fused"], 3)}
    return res


def precision_block(g, ctx, H, P, nq, ne, mapping, oracle):
    """The precision form against the FP64 oracle on the oracle's iterations:
    the complex64 run free-running (its own selections) and operator-forced
    (the oracle re-run with the complex64 run's selections when they differ);
    energy error per iteration, infidelity of the final state, gradient error
    of every pool operator at the final state, and the same for the complex128
    GPU path."""
    import numpy as np
    import torch
    from oracle.adapt import adapt_run
    o = oracle["run"]
    iters = len(o["ops"])
    out = {"reference": f"FP64 NumPy oracle, first {iters} iterations from Hartree-Fock"}
    for name, dt in (("complex64", torch.complex64), ("complex128", torch.complex128)):
        psi = _hf_state(g, ctx, nq, ne, mapping, dt)
        r = g.adapt_solve(ctx, H, P, psi, iters, schedule=1)
        gg = g.pool_gradients(ctx, H, P, psi)
        p = psi.to(torch.complex128).cpu().numpy()
        p = p / np.linalg.norm(p)
        same = r["ops"] == o["ops"]
        blk = {"same_operator_sequence": same,
               "max_abs_dE_ha": float(np.abs(np.asarray(o["energies"]) - r["energies"]).max()),
               "infidelity_final": float(1.0 - abs(np.vdot(o["psi"], p)) ** 2),
               "max_abs_dg_final": float(np.abs(oracle["g_final"] - gg).max()),
               "max_abs_dgnorm": float(np.abs(np.asarray(o["gnorms"]) - r["gnorms"]).max())}
        if same:
            blk["operator_forced"] = "identical to free-running (same selections)"
        else:
            of = adapt_run(oracle["H"], oracle["ops"], oracle["psi0"], iters, forced_ops=list(r["ops"]) + [0])
            blk["operator_forced"] = {"max_abs_dE_ha": float(np.abs(np.asarray(of["energies"]) - r["energies"]).max()),
                                      "infidelity_final": float(1.0 - abs(np.vdot(of["psi"], p)) ** 2)}
        out[name] = blk
    out["targets"] = {"complex64_dE_ha": 1e-6, "complex64_fidelity": 1 - 1e-6, "complex128_dE_ha": 1e-10}
    return out


def reopt_block(g, ctx, H, P, nq, ne, mapping, iters=8):
    """ADAPT with every angle re-optimised (BFGS over adjoint gradients through
    the Taylor layers), complex128 state, from Hartree-Fock: wall time per
    ADAPT iteration and per energy+gradient evaluation (forward pass, H psi,
    backward pass and the copy of the partials), against the frozen-angle run
    with the same budget of operators."""
    import torch
    psi = _hf_state(g, ctx, nq, ne, mapping, torch.complex128)
    g.adapt_reopt_solve(ctx, H, P, psi, 1)          # warm-up (table uploads, code load)
    psi = _hf_state(g, ctx, nq, ne, mapping, torch.complex128)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = g.adapt_reopt_solve(ctx, H, P, psi, iters)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    psi = _hf_state(g, ctx, nq, ne, mapping, torch.complex128)
    fr = g.adapt_solve(ctx, H, P, psi, iters)
    nev = sum(r["bfgs_evals"])
    layers = sum(2 * (k + 1) for k, e in enumerate(r["bfgs_evals"]) for _ in range(e))
    return {"iterations": iters, "state": "complex128", "seconds": round(dt, 4),
            "adapt_iters_per_s": round(iters / dt, 2), "evaluations": nev,
            "evaluations_per_s": round(nev / dt, 1), "layer_launches": layers,
            "bfgs_steps": r["bfgs_steps"], "final_energy": float(r["energies"][-1]),
            "frozen_final_energy": float(fr["energies"][-1]),
            "energy_gain_over_frozen_ha": float(fr["energies"][-1] - r["energies"][-1])}


def batched_block(g, ctx, schedule, oracle_baseline):
    """The 64-instance batch (24 x 10q, 24 x 12q, 16 x 14q, JW/BK alternating),
    30 iterations each, launched directly with the energy+screen launch timed
    by its dispatch timestamps in every other iteration; its algorithmic lane
    operations over that mean give the batch's roofline fraction."""
    import torch
    from workloads import batched_instances
    insts = batched_instances()
    hams, pools, psis, meta = [], [], [], []
    for d in insts:
        Hi, Pi = _system(g, d["n_qubits"], d["n_electrons"], d["mapping"], d["seed"])
        hams.append(Hi)
        pools.append(Pi)
        psis.append(_hf_state(g, ctx, d["n_qubits"], d["n_electrons"], d["mapping"], torch.complex64))
        meta.append((d["n_qubits"], Hi.n_terms, Pi.n_strings, Pi.strings()[0]))
    iters_b = 30
    bb = g.Batch(ctx, hams, pools, psis, max_iter=iters_b, use_graph=True, schedule=schedule)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, kms = bb.step_timed(iters_b, 3, 2)
    torch.cuda.synchronize()
    dtb = time.perf_counter() - t0
    sched_b = bb.schedule
    ub = 0
    for i in range(len(insts)):
        ri = bb.result(i)
        nqi, Ti, Si, offi = meta[i]
        ub += _string_amps(nqi, Ti, Si, offi, ri["ops"], ri["substeps"])
    bb.close()
    sa = sum((1 << nqi) * (Ti + Si) for (nqi, Ti, Si, _) in meta)
    lane_ops = LANE_OPS_PER_STRING_AMP * sa
    achieved = lane_ops / (kms * 1e-3) / 1e12
    ips = len(insts) * iters_b / dtb
    out = {"instances": len(insts), "mix": "24x10q + 24x12q + 16x14q, JW/BK alternating",
           "iterations_each": iters_b, **_schedule_fields(sched_b), "state": "complex64",
           "seconds": round(dtb, 6), "instance_iters_per_s": round(ips, 2),
           "algorithmic_amp_updates_per_s": float(f"{ub / dtb:.6g}"),
           "roofline": {"bound": "alu", "kernel": "k_energy_screen (all 64 instances per launch)",
                        "achieved": round(achieved, 4), "peak": round(VALU_PEAK_TOPS, 4), "unit": "Tlane-op/s",
                        "frac": round(achieved / VALU_PEAK_TOPS, 5), "avg_launch_us": round(kms * 1e3, 3),
                        "launches_sampled": (iters_b + 1) // 2,
                        "algorithmic_lane_ops_per_launch": int(lane_ops)}}
    if oracle_baseline:
        out["cpu_baseline"] = oracle_baseline
        out["vs_cpu_oracle"] = round(ips / oracle_baseline["value"], 1)
    return out


def serving_block(g, ctx, n_req, warm, max_slots=32, iters_per_step=4, loads=(0.7, 1.2), amps_per_lane=0,
                  state="complex128", deadline_s=600.0, oracle_baseline=None):
    """The serving workload: a Poisson stream of ADAPT solves (8-16 qubits,
    ||g|| < 1e-3, at most 300 iterations).  Capacity is measured first with
    every request submitted at once; the stream then arrives at each `load`
    times that capacity, `warm` warm-up requests first (excluded from the
    figures), then `n_req` measured ones.  Latency is submission to
    completion on the library's clock; the baseline is sequential plain FP64
    adapt_solve on the same device, each solve at its autotuned schedule.  A second capacity run serves the same
    requests with the other state precision.  With `oracle_baseline` (the
    oracle's requests and its solves/s on them) the server also solves those
    requests alone, for the comparison."""
    import numpy as np
    import torch
    from workloads import serving_requests
    specs = serving_requests(n_req + warm, rate_hz=1.0)
    reqs = []
    for d in specs:
        H, P = _system(g, d["n_qubits"], d["n_electrons"], d["mapping"], d["seed"])
        reqs.append((d, H, P, P.strings()[0]))
    tol, max_iter = 1e-3, 300
    budget = 8 << 30
    code = 1 if state == "complex64" else 0

    def drain(srv, tickets, done, t_end=None):
        for t in list(tickets):
            r = srv.poll(t)
            if r is not None:
                done[t] = r
                tickets.remove(t)
        if t_end is not None and time.perf_counter() > t_end:
            raise TimeoutError(f"serving: {len(tickets)} requests unfinished at the deadline")

    def new_server(c=code):
        return g.Server(ctx, budget, max_slots, dtype=c, iters_per_step=iters_per_step,
                        amps_per_lane=amps_per_lane)

    def capacity(c):
        """Every measured request submitted at once; solves/s and the results."""
        srv = new_server(c)
        t0 = time.perf_counter()
        pend = [srv.submit(H, P, max_iter, tol) for (_, H, P, _) in reqs[warm:]]
        done = {}
        while pend:
            drain(srv, pend, done, t0 + deadline_s)
            time.sleep(0.0005)
        rate = n_req / (time.perf_counter() - t0)
        srv.close()
        return rate, done

    cap, done = capacity(code)
    # the gradient screen of every served iteration (all M operators over
    # all 2^n amplitudes, S strings): work every iteration of either
    # precision performs in full, whatever else it carries or compacts
    screen_sa = 0
    for (d, H, P, off), t in zip(reqs[warm:], [k for k in sorted(done)]):
        rec = done[t][1]
        if rec is not None:
            screen_sa += (1 << d["n_qubits"]) * P.n_strings * (rec["n_iter"] + (1 if rec["converged"] else 0))

    runs = {}
    for load in loads:
        rate = load * cap
        srv = new_server()
        arrivals = [d["arrival_s"] / rate for (d, _, _, _) in reqs]
        pend, done, meas = [], {}, []
        t0 = time.perf_counter()
        t_end = t0 + deadline_s
        for k, (d, H, P, _) in enumerate(reqs):
            while time.perf_counter() - t0 < arrivals[k]:
                drain(srv, pend, done, t_end)
                time.sleep(0.0002)
            t = srv.submit(H, P, max_iter, tol)
            pend.append(t)
            if k >= warm:
                meas.append((t, d["n_qubits"]))
        while pend:
            drain(srv, pend, done, t_end)
            time.sleep(0.0005)
        st = srv.stats()
        srv.close()
        lat = {t: (done[t][2]["t_done_ns"] - done[t][2]["t_submit_ns"]) * 1e-6 for t, _ in meas}
        t_sub = min(done[t][2]["t_submit_ns"] for t, _ in meas)
        t_fin = max(done[t][2]["t_done_ns"] for t, _ in meas)
        per_q = {}
        for nq in sorted({q for _, q in meas}):
            ls = [lat[t] for t, q in meas if q == nq]
            per_q[str(nq)] = {"requests": len(ls), "p50_ms": _pct(ls, 50), "p99_ms": _pct(ls, 99)}
        runs[f"{load:g}x"] = {
            "offered_rate_hz": round(rate, 2),
            "solves_per_s": round(n_req / ((t_fin - t_sub) * 1e-9), 2),
            "p50_ms": _pct(list(lat.values()), 50), "p99_ms": _pct(list(lat.values()), 99),
            "per_qubit_count": per_q,
            "completed_ok": sum(1 for t, _ in meas if done[t][0] == 0),
            "converged": sum(1 for t, _ in meas if done[t][1] is not None and done[t][1]["converged"]),
            "server_steps": st["steps"]}

    # the same capacity run with the other state precision (complex64 storage,
    # FP64 arithmetic, or the reverse)
    other = 1 - code
    cap_other, done_other = capacity(other)

    # sequential plain FP64: one adapt_solve at a time, complex128, each at
    # the schedule the autotuner picks for its size (chosen during the
    # warm-up requests, which cover every size, and remembered)
    for (d, H, P, _) in reqs[:warm]:
        psi = _hf_state(g, ctx, d["n_qubits"], d["n_electrons"], d["mapping"], torch.complex128)
        g.adapt_solve(ctx, H, P, psi, max_iter, grad_tol=tol, schedule=0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for (d, H, P, _) in reqs[warm:]:
        psi = _hf_state(g, ctx, d["n_qubits"], d["n_electrons"], d["mapping"], torch.complex128)
        g.adapt_solve(ctx, H, P, psi, max_iter, grad_tol=tol, schedule=0)
    torch.cuda.synchronize()
    seq = n_req / (time.perf_counter() - t0)
    cap_dt = n_req / cap
    achieved = LANE_OPS_PER_STRING_AMP * screen_sa / cap_dt / 1e12
    cpu = None
    if oracle_baseline is not None:
        ospecs, obase = oracle_baseline
        sub = []
        for (nqs, nes, ms, seeds, mi, tl) in ospecs:
            Hs, Ps = _system(g, nqs, nes, ms, seeds)
            sub.append((Hs, Ps))
        srv = g.Server(ctx, budget, max_slots, dtype=code, iters_per_step=iters_per_step, amps_per_lane=amps_per_lane)
        t0 = time.perf_counter()
        pend, done_s = [srv.submit(Hs, Ps, max_iter, tol) for (Hs, Ps) in sub], {}
        while pend:
            drain(srv, pend, done_s, t0 + deadline_s)
            time.sleep(0.0005)
        same = len(sub) / (time.perf_counter() - t0)
        srv.close()
        cpu = dict(obase)
        cpu["gpu_same_requests_solves_per_s"] = round(same, 2)
        cpu["gpu_vs_cpu"] = round(same / obase["value"], 1)
    return {"requests": n_req, "warmup_requests": warm, "qubits": "uniform over {8,10,12,14,16}",
            "grad_tol": tol, "max_iter": max_iter, "state": state, "max_slots": max_slots,
            "iters_per_step": iters_per_step, "amps_per_lane": amps_per_lane if amps_per_lane else "adaptive",
            "hbm_budget_bytes": budget, "capacity_solves_per_s": round(cap, 2),
            "loads": runs, "sequential_fp64_solves_per_s": round(seq, 2),
            "capacity_vs_sequential_fp64": round(cap / seq, 3),
            **({"cpu_baseline": cpu} if cpu else {}),
            "other_state": {"state": "complex64" if other == 1 else "complex128",
                            "capacity_solves_per_s": round(cap_other, 2),
                            "capacity_vs_sequential_fp64": round(cap_other / seq, 3),
                            "completed_ok": sum(1 for r in done_other.values() if r[0] == 0),
                            "converged": sum(1 for r in done_other.values()
                                             if r[1] is not None and r[1]["converged"])},
            "capacity_screen_roofline": {"bound": "alu", "what": "algorithmic lane operations of the gradient "
                                  "screens of every served iteration (5 per string-amplitude, S strings x 2^n "
                                  "amplitudes per screen) over the capacity run's wall time; every other kernel "
                                  "and idle gap counts as time, so this bounds the fraction from below",
                                  "achieved": round(achieved, 4), "peak": round(VALU_PEAK_TOPS, 4),
                                  "unit": "Tlane-op/s", "frac": round(achieved / VALU_PEAK_TOPS, 5)}}


def _phase_trace(g, ctx, H, P, nq, ne, mapping, warm, iters):
    """Phase durations of the energy+screen launch (one amplitude per lane),
    from the measurement build's per-workgroup clock values (100 MHz): for
    each of `iters` ADAPT iterations after `warm`, the median over workgroups
    of each phase, then the median over iterations, in us."""
    import numpy as np
    import torch
    names = ["launch ramp (first entry to workgroup entry)", "prologue (descriptor, state record)",
             "H stage (first chunk of magnitudes into LDS)", "H walk (to the last wave's end)",
             "sigma, energy partials, screen stage", "screen walk (to the last wave's end)"]
    psi = _hf_state(g, ctx, nq, ne, mapping, torch.complex64)
    b = g.Batch(ctx, [H], [P], [psi], max_iter=warm + iters, use_graph=False, schedule=1)
    tiles = (1 << nq) // 64
    b.step(warm)
    per = []
    for _ in range(iters):
        b.step(1)
        t = g.phase_trace(ctx, tiles).astype(np.int64)
        t0 = t[:, 0].min()
        edges = np.concatenate([np.full((tiles, 1), t0), t], axis=1)
        per.append(np.median(np.diff(edges, axis=1), axis=0) * 0.01)
        per[-1] = np.append(per[-1], (t[:, 5].max() - t0) * 0.01)
    b.close()
    med = np.median(np.array(per), axis=0)
    out = {n: round(float(v), 3) for n, v in zip(names, med[:6])}
    out["first entry to the last workgroup's end"] = round(float(med[6]), 3)
    out["iterations"] = f"{warm}..{warm + iters - 1} from Hartree-Fock"
    out["workgroups"] = tiles
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--cpu-sample-iters", type=int, default=12,
                    help="oracle iterations of the headline system: the CPU baseline and the precision "
                         "form's reference (0 disables both)")
    ap.add_argument("--no-forms", action="store_true", help="only the headline (and the CPU legs)")
    ap.add_argument("--serve-requests", type=int, default=512, help="measured requests of the serving stream")
    ap.add_argument("--serve-warmup", type=int, default=32, help="warm-up requests before the measured ones")
    ap.add_argument("--sample-every", type=int, default=0,
                    help="dispatch-timestamp events around every n-th launch of the dominant kernel in the "
                         "timed region (0: every 4th up to 100 steps, else every 8th; each sample costs the "
                         "loop a few microseconds)")
    ap.add_argument("--schedule", type=int, default=0, choices=(0, 1, 2, 4),
                    help="amplitudes per lane of the tile kernels (0: autotune)")
    ap.add_argument("--serve-amps-per-lane", type=int, default=0, choices=(0, 1, 2, 4),
                    help="server schedule (0: chosen from the active set)")
    ap.add_argument("--serve-state", default="complex128", choices=("complex64", "complex128"))
    ap.add_argument("--sparse-sample-iters", type=int, default=60,
                    help="iterations of the sparse-matrix CPU baseline on the headline system (0 disables it)")
    ap.add_argument("--oracle-workers", type=int, default=0,
                    help="worker processes of the batched oracle baseline (0: min(16, CPUs))")
    ap.add_argument("--batch-oracle-iters", type=int, default=4)
    ap.add_argument("--phase-trace", type=int, default=0, metavar="ITERS",
                    help="only the energy+screen launch's phase trace over ITERS iterations of the headline "
                         "system (needs the measurement build: GOCP_PHASE_TRACE=1 after "
                         "python -m paper_2607_15906_amd.build --phase-trace)")
    ap.add_argument("--fused-step-only", action="store_true",
                    help="time only the GOCP multi-operator step against single chains (kernel profiling)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="first run a plain device-to-device copy of this many MiB (a known-size "
                         "kernel that calibrates memory-traffic counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the batched and "
              "serving forms shard by instance across GPUs, which this build does not run.",
              file=sys.stderr)
        sys.exit(2)
    if args.steps <= 0 or args.warmup < 0:
        print("need --steps > 0 and --warmup >= 0", file=sys.stderr)
        sys.exit(2)
    # every 4th launch up to 100 steps (5 samples at 20), every 8th beyond
    every = args.sample_every or (4 if args.steps <= 100 else 8)

    from workloads import CONFIGS
    cfg = CONFIGS["c3_14q"]
    nq, ne, seed = cfg["n_qubits"], cfg["n_electrons"], cfg["seed"]
    mapping = "jw"

    # CPU legs first: nothing has touched the GPU yet, so the oracle worker
    # processes can be forked safely
    oracle = None
    if args.cpu_sample_iters > 0 and not args.fused_step_only and not args.phase_trace:
        _say(f"[bench] CPU oracle: {args.cpu_sample_iters} iterations at 14q (one thread)")
        oracle = oracle_headline(nq, ne, mapping, seed, args.cpu_sample_iters)
    sparse = None
    if args.sparse_sample_iters > 0 and not args.fused_step_only and not args.phase_trace:
        _say(f"[bench] CPU sparse matrices: {args.sparse_sample_iters} iterations at 14q (one thread)")
        sparse = sparse_headline(nq, ne, mapping, seed, args.sparse_sample_iters)
    batch_oracle = serve_oracle = None
    if not args.no_forms and not args.fused_step_only and not args.phase_trace and args.batch_oracle_iters > 0:
        workers = args.oracle_workers or min(16, os.cpu_count() or 1)
        _say(f"[bench] CPU oracle: batched instances on {workers} workers")
        batch_oracle = oracle_batch_baseline(args.batch_oracle_iters, workers)
        _say(f"[bench] CPU oracle: 8-qubit serving requests on {workers} workers")
        serve_oracle = oracle_serving_baseline(32, workers)

    import numpy as np
    import torch
    import paper_2607_15906_amd as g

    if args.copy_probe_mib > 0:
        n = args.copy_probe_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    ctx = g.Context(0)
    H, P = _system(g, nq, ne, mapping, seed)
    if args.fused_step_only:
        print(json.dumps({"gocp_fused_step": _fused_step_timing(g, ctx, P, nq, reps=50)}))
        return
    if args.phase_trace:
        print(json.dumps({"phase_trace": _phase_trace(g, ctx, H, P, nq, ne, mapping, args.warmup,
                                                      args.phase_trace)}))
        return
    off = P.strings()[0]
    T, C, S, M = H.n_terms, H.n_classes, P.n_strings, P.n_ops

    _say(f"[bench] 14q c64: {args.warmup} warmup + {args.steps} timed ADAPT iterations")
    # which tile kernel dominates, from dry timing-hook launches on a scratch batch
    psi_d = _hf_state(g, ctx, nq, ne, mapping, torch.complex64)
    bd = g.Batch(ctx, [H], [P], [psi_d], max_iter=1, schedule=args.schedule)
    pre = {w: bd.time_kernel(w, 20) for w in (0, 1)}
    sched = bd.schedule
    bd.close()
    dom = 3 if pre[0] >= pre[1] else 1
    b, r, dt, kms, nsamp = run_adapt_timed(g, ctx, H, P, nq, ne, mapping, torch.complex64, args.steps,
                                           args.warmup, schedule=sched, timed_kernel=dom, sample_every=every)
    w0, w1 = args.warmup, args.warmup + args.steps
    if r["n_iter"] != w1:
        raise RuntimeError(f"expected {w1} iterations, ran {r['n_iter']}")
    ips = args.steps / dt
    upd = _string_amps(nq, T, S, off, r["ops"][w0:w1], r["substeps"][w0:w1])

    # roofline of the dominant kernel, which is bound by VALU issue: the
    # algorithmic lane operations per launch (LANE_OPS_PER_STRING_AMP per
    # string-amplitude: H psi and the screen for k_energy_screen, two H
    # applications for k_line_hvw) over its mean launch duration, measured
    # live over the timed region; beside it the FP64 view (one signed add per
    # string-amplitude, a real-by-complex multiply-add (4 flops) per (class or
    # operator, amplitude), and the dot products)
    dim = 1 << nq
    string_amps = {3: dim * (T + S), 1: 2 * dim * T}
    flops = {3: dim * (T + 4 * C + 4) + dim * (S + 4 * M), 1: dim * (T + 8 * C + 12)}
    name = g.Batch.STEP_KERNELS[dom]
    lane_ops = LANE_OPS_PER_STRING_AMP * string_amps[dom]
    achieved = lane_ops / (kms * 1e-3) / 1e12
    achieved_fp64 = flops[dom] / (kms * 1e-3) / 1e12
    traffic = TRAFFIC_BYTES.get((name, sched))
    hook = {"k_energy_screen (fresh H psi)": b.time_kernel(0, 50), "k_line_hvw": b.time_kernel(1, 50),
            "k_screen_sum1 + k_screen_reduce": b.time_kernel(3, 50)}
    roofline = {"bound": "alu", "kernel": name, "achieved": round(achieved, 4),
                "peak": round(VALU_PEAK_TOPS, 4), "unit": "Tlane-op/s",
                "frac": round(achieved / VALU_PEAK_TOPS, 5), "traffic": traffic,
                "avg_launch_us": round(kms * 1e3, 3), "launches_sampled": nsamp,
                "algorithmic_string_amps_per_launch": int(string_amps[dom]),
                "algorithmic_lane_ops_per_launch": int(lane_ops),
                "fp64_view": {"achieved_tflops": round(achieved_fp64, 4), "peak_tflops": FP64_PEAK_TFLOPS,
                              "frac": round(achieved_fp64 / FP64_PEAK_TFLOPS, 5),
                              "algorithmic_flops_per_launch": int(flops[dom])},
                "dry_launch_avg_us": {k: round(v * 1e3, 3) for k, v in hook.items()}}
    b.close()

    out = {
        "metric": METRIC, "value": round(ips, 3), "unit": "iters/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(1e3 * dt / args.steps, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "ADAPT iteration, 14 qubits / 6 electrons, Jordan-Wigner, "
                               "complex64 state storage with FP64 arithmetic and reductions",
                   "n_qubits": nq, "n_electrons": ne, "mapping": mapping, "integral_seed": seed,
                   "pauli_terms": T, "xmask_classes": C, "pool_ops": M, "pool_strings": S,
                   "state": "complex64", "timed_iterations": f"{w0}..{w1 - 1} from Hartree-Fock",
                   "launch": "warm-up as captured hipGraph replays, timed iterations as direct launches",
                   **_schedule_fields(sched)},
        "algorithmic_amp_updates_per_s": float(f"{upd / dt:.6g}"),
        "algorithmic_amp_updates_note": "2^n (3T + S + 2k + 5ks) string-amplitudes per iteration, whether or "
                                        "not the kernels skip, fuse or factor them",
        "final_energy": float(r["energies"][-1]),
        "roofline": roofline,
    }

    if oracle is not None:
        _say("[bench] precision form against the oracle")
        out["precision"] = precision_block(g, ctx, H, P, nq, ne, mapping, oracle)

    if not args.no_forms:
        _say("[bench] 14q c128 path")
        b2, r2, dt2, _, _ = run_adapt_timed(g, ctx, H, P, nq, ne, mapping, torch.complex128,
                                            args.steps, args.warmup, schedule=sched, sample_every=every)
        b2.close()
        u2 = _string_amps(nq, T, S, off, r2["ops"][w0:w1], r2["substeps"][w0:w1])
        out["complex128_state"] = {"iters_per_s": round(args.steps / dt2, 3),
                                   "algorithmic_amp_updates_per_s": float(f"{u2 / dt2:.6g}"),
                                   "same_operator_sequence_as_c64": r2["ops"] == r["ops"],
                                   "max_abs_dE_vs_c64": float(np.abs(r2["energies"] - r["energies"]).max())}

        _say("[bench] 14q c64 under Bravyi-Kitaev")
        Hb, Pb = _system(g, nq, ne, "bk", seed)
        b4, r4, dt4, _, _ = run_adapt_timed(g, ctx, Hb, Pb, nq, ne, "bk", torch.complex64, args.steps,
                                            args.warmup, schedule=sched, sample_every=every)
        b4.close()
        out["bravyi_kitaev_14q"] = {"iters_per_s": round(args.steps / dt4, 3), "state": "complex64",
                                    "same_operator_sequence_as_jw": r4["ops"] == r["ops"],
                                    "max_abs_dE_vs_jw": float(np.abs(r4["energies"] - r["energies"]).max())}

        _say("[bench] later window: iterations 30-59")
        b5, r5, dt5, _, _ = run_adapt_timed(g, ctx, H, P, nq, ne, mapping, torch.complex64, 30, 30,
                                            schedule=sched, sample_every=every)
        b5.close()
        out["later_window_14q"] = {"iterations": "30..59 from Hartree-Fock", "state": "complex64",
                                   "iters_per_s": round(30 / dt5, 3)}

        _say("[bench] Pauli pool: 14q c64")
        PP = g.pool_build_pauli(nq, ne, mapping)
        offp = PP.strings()[0]
        b3, r3, dt3, _, _ = run_adapt_timed(g, ctx, H, PP, nq, ne, mapping, torch.complex64, args.steps,
                                            args.warmup, schedule=0, sample_every=every)
        out["pauli_pool"] = {"pool_ops": PP.n_ops, "pool_strings": PP.n_strings, "state": "complex64",
                             **_schedule_fields(b3.schedule), "iters_per_s": round(args.steps / dt3, 3),
                             "algorithmic_amp_updates_per_s": float(
                                 f"{_string_amps(nq, T, PP.n_strings, offp, r3['ops'][w0:w1], r3['substeps'][w0:w1]) / dt3:.6g}"),
                             "final_energy": float(r3["energies"][-1])}
        b3.close()

        _say("[bench] ADAPT with full re-optimisation: 14q, 8 iterations")
        out["reoptimised_adapt_14q"] = reopt_block(g, ctx, H, P, nq, ne, mapping)

        _say("[bench] GOCP multi-operator step: 14q, 4 members of one family")
        out["gocp_fused_step"] = _fused_step_timing(g, ctx, P, nq)

        _say("[bench] batched form: 64 instances x 30 iterations")
        out["batched"] = batched_block(g, ctx, args.schedule, batch_oracle)

        _say(f"[bench] serving form: {args.serve_warmup} + {args.serve_requests} requests")
        out["serving"] = serving_block(g, ctx, n_req=args.serve_requests, warm=args.serve_warmup,
                                       amps_per_lane=args.serve_amps_per_lane, state=args.serve_state,
                                       oracle_baseline=serve_oracle)

    if oracle is not None:
        n_it = args.cpu_sample_iters
        out["cpu_baseline"] = {"value": round(n_it / oracle["seconds"], 5), "unit": "iters/s", "cores": 1,
                               "kind": "oracle",
                               "sample": f"first {n_it} ADAPT iterations of the same 14q JW system from "
                                         f"Hartree-Fock, FP64 NumPy oracle, {oracle['seconds']:.1f} s on one of "
                                         f"{os.cpu_count()} host CPUs"}
        out["vs_cpu_oracle"] = round(ips / out["cpu_baseline"]["value"], 1)
    if sparse is not None:
        out["cpu_sparse_baseline"] = sparse
        out["vs_cpu_sparse"] = round(ips / sparse["value"], 1)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
