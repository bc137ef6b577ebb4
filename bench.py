#!/usr/bin/env python3
"""Benchmark of the GOCP ADAPT-VQE hot path on one MI355X.

A step is one ADAPT iteration of the 14-qubit, 6-electron (BeH2-sized,
Tables I-II) synthetic system under Jordan-Wigner: gradient screen of the
whole pool, selection, line search, fifth-order Taylor update and the new
energy, with a complex64 statevector and FP64 accumulation.  The iteration
runs device-resident as captured hipGraphs; W untimed steps precede exactly K
timed steps.  Prints one JSON line.

Also reported: the complex128 path on the same workload, the 64-instance
batched form, the roofline of the dominant kernel (HIP-event timed), and the
FP64 CPU oracle on a bounded sample of the same iterations.
"""

from __future__ import annotations

import argparse
import json
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
TRAFFIC_BYTES = {("k_energy_screen", 1): 2553596}
# the dominant kernel is bracketed by HIP events in every 8th timed iteration
# (events around every launch would slow the loop by several per cent)
LIVE_SAMPLE_EVERY = 8


def _say(msg):
    print(msg, file=sys.stderr, flush=True)


def _system(g, nq, ne, mapping, seed):
    from workloads import molecular_integrals
    h1, eri, ec = molecular_integrals(nq // 2, seed)
    H = g.pauli_hamiltonian_load(h1, eri, ec, mapping)
    P = g.pool_build(nq, ne, mapping)
    return H, P


def _hf_state(g, ctx, nq, ne, mapping, dtype):
    import torch
    t = torch.zeros(1 << nq, dtype=dtype, device="cuda")
    g.state_basis(ctx, nq, g.hf_index(nq, ne, mapping), t)
    return t


def _amp_updates(nq, T, S, off, ops, subs):
    """Algorithmic Pauli-term amplitude updates of the given iterations:
    2^n (3T + S + 2k + 5 k s) per iteration, k = strings of the chosen operator."""
    tot = 0
    for j, s in zip(ops, subs):
        k = int(off[j + 1] - off[j])
        tot += 3 * T + S + 2 * k + 5 * k * s
    return tot * (1 << nq)


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
            # median of five batches of reps / 5 steps
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


def run_adapt_timed(g, ctx, H, P, nq, ne, mapping, dtype, steps, warmup, schedule=0, timed_kernel=None,
                    sample_every=LIVE_SAMPLE_EVERY):
    """Warm-up iterations (graph replays), then the timed iterations.  With
    timed_kernel (an index of Batch.STEP_KERNELS) the timed iterations are
    launched directly with HIP events around every launch of that kernel, and
    its mean duration over the timed region is returned as well."""
    import torch
    psi = _hf_state(g, ctx, nq, ne, mapping, dtype)
    b = g.Batch(ctx, [H], [P], [psi], max_iter=warmup + steps, use_graph=True, schedule=schedule)
    pre = {w: b.time_kernel(w, 20) for w in (0, 1)}   # dry launches: which tile kernel dominates
    b.step(warmup)
    torch.cuda.synchronize()
    kernel_ms = None
    t0 = time.perf_counter()
    if timed_kernel is None:
        b.step(steps)
    else:
        k = timed_kernel(pre) if callable(timed_kernel) else timed_kernel
        _, kernel_ms = b.step_timed(steps, k, sample_every)
        kernel_ms = (k, kernel_ms)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    r = b.result(0)
    r["psi"] = psi
    return b, r, dt, kernel_ms


def serving_bench(g, ctx, n_req, warm, max_slots=32, iters_per_step=4, load=0.7, amps_per_lane=0,
                  state="complex128"):
    """Poisson stream of ADAPT solves (8-16 qubits, ||g|| < 1e-3, at most 300
    iterations), states of the given precision.  Capacity is measured first with all
    requests submitted at once; the timed stream then arrives at `load` times
    that capacity.  Latency is submission to completion (library clock)."""
    import numpy as np
    import torch
    from workloads import serving_requests
    specs = serving_requests(n_req + warm, rate_hz=1.0)
    reqs = []
    for d in specs:
        H, P = _system(g, d["n_qubits"], d["n_electrons"], d["mapping"], d["seed"])
        reqs.append((d, H, P))
    tol, max_iter = 1e-3, 300
    budget = 8 << 30

    def drain(srv, tickets, done):
        for t in list(tickets):
            r = srv.poll(t)
            if r is not None:
                done[t] = r
                tickets.remove(t)

    # capacity: everything at once
    code = 1 if state == "complex64" else 0
    srv = g.Server(ctx, budget, max_slots, dtype=code, iters_per_step=iters_per_step,
                   amps_per_lane=amps_per_lane)
    t0 = time.perf_counter()
    pend = [srv.submit(H, P, max_iter, tol) for (_, H, P) in reqs[warm:]]
    done = {}
    while pend:
        drain(srv, pend, done)
        time.sleep(0.0005)
    cap = n_req / (time.perf_counter() - t0)
    srv.close()

    # timed Poisson stream at `load` x capacity (warm-up requests first)
    rate = load * cap
    srv = g.Server(ctx, budget, max_slots, dtype=code, iters_per_step=iters_per_step,
                   amps_per_lane=amps_per_lane)
    arrivals = [d["arrival_s"] / rate for (d, _, _) in reqs]
    pend, done, meas = [], {}, []
    t0 = time.perf_counter()
    for k, (d, H, P) in enumerate(reqs):
        while time.perf_counter() - t0 < arrivals[k]:
            drain(srv, pend, done)
            time.sleep(0.0002)
        t = srv.submit(H, P, max_iter, tol)
        pend.append(t)
        if k >= warm:
            meas.append(t)
    t_first = None
    while pend:
        drain(srv, pend, done)
        time.sleep(0.0005)
    st = srv.stats()
    srv.close()
    lat = np.array([(done[t][2]["t_done_ns"] - done[t][2]["t_submit_ns"]) * 1e-6 for t in meas])
    t_sub = min(done[t][2]["t_submit_ns"] for t in meas)
    t_end = max(done[t][2]["t_done_ns"] for t in meas)
    ok = sum(1 for t in meas if done[t][0] == 0)
    conv = sum(1 for t in meas if done[t][1] is not None and done[t][1]["converged"])

    # sequential plain FP64: one adapt_solve at a time, complex128
    t0 = time.perf_counter()
    nseq = 0
    for (d, H, P) in reqs[warm:]:
        psi = _hf_state(g, ctx, d["n_qubits"], d["n_electrons"], d["mapping"], torch.complex128)
        g.adapt_solve(ctx, H, P, psi, max_iter, grad_tol=tol)
        nseq += 1
    torch.cuda.synchronize()
    seq = nseq / (time.perf_counter() - t0)
    return {"requests": n_req, "warmup_requests": warm, "qubits": "uniform over {8,10,12,14,16}",
            "grad_tol": tol, "max_iter": max_iter, "state": state, "max_slots": max_slots,
            "iters_per_step": iters_per_step,
            "amps_per_lane": amps_per_lane if amps_per_lane else "adaptive",
            "hbm_budget_bytes": budget,
            "capacity_solves_per_s": round(cap, 2), "offered_rate_hz": round(rate, 2),
            "solves_per_s": round(n_req / ((t_end - t_sub) * 1e-9), 2),
            "p50_ms": round(float(np.percentile(lat, 50)), 3),
            "p99_ms": round(float(np.percentile(lat, 99)), 3),
            "completed_ok": ok, "converged": conv, "server_steps": st["steps"],
            "sequential_fp64_solves_per_s": round(seq, 2)}


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--cpu-sample-iters", type=int, default=8,
                    help="oracle iterations timed for the CPU baseline (0 disables it)")
    ap.add_argument("--no-forms", action="store_true", help="skip the c128 and batched extras")
    ap.add_argument("--serve-requests", type=int, default=96,
                    help="measured requests of the serving stream (after 16 warm-up requests)")
    ap.add_argument("--sample-every", type=int, default=LIVE_SAMPLE_EVERY,
                    help="HIP events around every n-th launch of the dominant kernel in the timed region")
    ap.add_argument("--schedule", type=int, default=0, choices=(0, 1, 2, 4),
                    help="amplitudes per lane of the tile kernels (0: autotune)")
    ap.add_argument("--serve-amps-per-lane", type=int, default=0, choices=(0, 1, 2, 4),
                    help="server schedule (0: chosen from the active set)")
    ap.add_argument("--serve-state", default="complex128", choices=("complex64", "complex128"))
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

    import numpy as np
    import torch
    import paper_2607_15906_amd as g
    from workloads import CONFIGS, batched_instances

    if args.copy_probe_mib > 0:
        n = args.copy_probe_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    cfg = CONFIGS["c3_14q"]
    nq, ne, seed = cfg["n_qubits"], cfg["n_electrons"], cfg["seed"]
    mapping = "jw"
    ctx = g.Context(0)
    H, P = _system(g, nq, ne, mapping, seed)
    if args.fused_step_only:
        print(json.dumps({"gocp_fused_step": _fused_step_timing(g, ctx, P, nq, reps=50)}))
        return
    off = P.strings()[0]
    T, C, S, M = H.n_terms, H.n_classes, P.n_strings, P.n_ops

    _say(f"[bench] 14q c64: {args.warmup} warmup + {args.steps} timed ADAPT iterations")
    # the dominant tile kernel (k_energy_screen: STEP_KERNELS[3], or k_line_hvw:
    # [1]) from dry timing-hook launches; its live duration over the timed
    # region then feeds the roofline
    b, r, dt, live = run_adapt_timed(g, ctx, H, P, nq, ne, mapping, torch.complex64, args.steps,
                                     args.warmup, schedule=args.schedule,
                                     timed_kernel=lambda pre: 3 if pre[0] >= pre[1] else 1,
                                     sample_every=args.sample_every)
    sched = b.schedule
    w0, w1 = args.warmup, args.warmup + args.steps
    iters = r["n_iter"]
    if iters != w1:
        raise RuntimeError(f"expected {w1} iterations, ran {iters}")
    ips = args.steps / dt
    upd = _amp_updates(nq, T, S, off, r["ops"][w0:w1], r["substeps"][w0:w1])

    # roofline of the dominant kernel, which is bound by VALU issue: the
    # algorithmic lane operations per launch (LANE_OPS_PER_STRING_AMP per
    # string-amplitude: H psi and the screen for k_energy_screen, two H
    # applications for k_line_hvw) over its mean launch duration, measured
    # live with HIP events over the timed region; beside it the FP64 view (one
    # signed add per string-amplitude, a real-by-complex multiply-add (4
    # flops) per (class or operator, amplitude), and the dot products)
    dim = 1 << nq
    string_amps = {3: dim * (T + S), 1: 2 * dim * T}
    flops = {3: dim * (T + 4 * C + 4) + dim * (S + 4 * M),   # H psi + energy + screen partials
             1: dim * (T + 8 * C + 12)}                      # H v and H w + three dots
    dom, kms = live
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
                "avg_launch_us": round(kms * 1e3, 3),
                "launches_sampled": (args.steps + args.sample_every - 1) // args.sample_every,
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
                               "complex64 state with FP64 accumulation",
                   "n_qubits": nq, "n_electrons": ne, "mapping": mapping, "integral_seed": seed,
                   "pauli_terms": T, "xmask_classes": C, "pool_ops": M, "pool_strings": S,
                   "state": "complex64", "graph_replay": True, "amps_per_lane": sched},
        "amp_updates_per_s": float(f"{upd / dt:.6g}"),
        "final_energy": float(r["energies"][-1]),
        "roofline": roofline,
    }

    if not args.no_forms:
        _say("[bench] 14q c128 path")
        b2, r2, dt2, _ = run_adapt_timed(g, ctx, H, P, nq, ne, mapping, torch.complex128,
                                         args.steps, args.warmup, schedule=sched)
        b2.close()
        u2 = _amp_updates(nq, T, S, off, r2["ops"][w0:w1], r2["substeps"][w0:w1])
        same_ops = r2["ops"] == r["ops"]
        p64 = r["psi"].to(torch.complex128)
        fid = float(torch.abs(torch.vdot(r2["psi"], p64)) ** 2 /
                    (torch.vdot(p64, p64).real * torch.vdot(r2["psi"], r2["psi"]).real))
        # precision form: gradients of the final complex64 state against those of
        # the complex128 state, both on the device with FP64 accumulation
        g64 = g.pool_gradients(ctx, H, P, r["psi"])
        g128 = g.pool_gradients(ctx, H, P, r2["psi"])
        out["complex128_state"] = {"iters_per_s": round(args.steps / dt2, 3),
                                   "amp_updates_per_s": float(f"{u2 / dt2:.6g}"),
                                   "same_operator_sequence": same_ops,
                                   "max_abs_dE_vs_c64": float(np.abs(r2["energies"] - r["energies"]).max()),
                                   "final_state_fidelity_c64": fid,
                                   "max_abs_dg_final_c64": float(np.abs(g64 - g128).max())}

        _say("[bench] Pauli pool: 14q c64")
        PP = g.pool_build_pauli(nq, ne, mapping)
        offp = PP.strings()[0]
        b3, r3, dt3, _ = run_adapt_timed(g, ctx, H, PP, nq, ne, mapping, torch.complex64, args.steps,
                                         args.warmup, schedule=0)
        out["pauli_pool"] = {"pool_ops": PP.n_ops, "pool_strings": PP.n_strings, "state": "complex64",
                             "amps_per_lane": b3.schedule, "iters_per_s": round(args.steps / dt3, 3),
                             "amp_updates_per_s": float(f"{_amp_updates(nq, T, PP.n_strings, offp, r3['ops'][w0:w1], r3['substeps'][w0:w1]) / dt3:.6g}"),
                             "final_energy": float(r3["energies"][-1])}
        b3.close()

        _say("[bench] GOCP multi-operator step: 14q, 4 members of one family")
        out["gocp_fused_step"] = _fused_step_timing(g, ctx, P, nq)

        _say("[bench] batched form: 64 instances x 30 iterations")
        insts = batched_instances()
        hams, pools, psis, meta = [], [], [], []
        for d in insts:
            Hi, Pi = _system(g, d["n_qubits"], d["n_electrons"], d["mapping"], d["seed"])
            hams.append(Hi); pools.append(Pi)
            psis.append(_hf_state(g, ctx, d["n_qubits"], d["n_electrons"], d["mapping"], torch.complex64))
            meta.append((d["n_qubits"], Hi.n_terms, Pi.n_strings, Pi.strings()[0]))
        iters_b = 30
        bb = g.Batch(ctx, hams, pools, psis, max_iter=iters_b, use_graph=True, schedule=args.schedule)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        bb.step(iters_b)
        torch.cuda.synchronize()
        dtb = time.perf_counter() - t0
        sched_b = bb.schedule
        ub = 0
        for i in range(len(insts)):
            ri = bb.result(i)
            nqi, Ti, Si, offi = meta[i]
            ub += _amp_updates(nqi, Ti, Si, offi, ri["ops"], ri["substeps"])
        bb.close()
        out["batched"] = {"instances": len(insts), "mix": "24x10q + 24x12q + 16x14q, JW/BK alternating",
                          "iterations_each": iters_b, "amps_per_lane": sched_b,
                          "seconds": round(dtb, 6),
                          "instance_iters_per_s": round(len(insts) * iters_b / dtb, 2),
                          "amp_updates_per_s": float(f"{ub / dtb:.6g}")}

        _say("[bench] serving form: Poisson stream of ADAPT solves")
        out["serving"] = serving_bench(g, ctx, n_req=args.serve_requests, warm=16,
                                       amps_per_lane=args.serve_amps_per_lane, state=args.serve_state)

    if args.cpu_sample_iters > 0:
        _say(f"[bench] CPU oracle baseline: {args.cpu_sample_iters} iterations at 14q")
        from threadpoolctl import threadpool_limits
        from oracle.mapping import hamiltonian, hf_index
        from oracle.pool import pool_operators
        from oracle.adapt import adapt_run
        from workloads import molecular_integrals
        h1, eri, ec = molecular_integrals(nq // 2, seed)
        Ho = hamiltonian(h1, eri, ec, mapping)
        ops = [A for _, _, A in pool_operators(nq, ne, mapping)]
        psi0 = np.zeros(1 << nq, dtype=np.complex128)
        psi0[hf_index(nq, ne, mapping)] = 1.0
        with threadpool_limits(limits=1):
            t0 = time.perf_counter()
            adapt_run(Ho, ops, psi0, args.cpu_sample_iters)
            dto = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": round(args.cpu_sample_iters / dto, 5), "unit": "iters/s",
                               "cores": 1, "kind": "oracle",
                               "sample": f"first {args.cpu_sample_iters} ADAPT iterations of the same "
                                         f"14q JW system from Hartree-Fock, FP64 NumPy oracle, "
                                         f"{dto:.1f} s on {os.cpu_count()} host CPUs (1 thread used)"}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
