"""The five seeded workloads (sizes follow the paper's 12- and 14-qubit systems).

Each entry describes inputs only: qubit count, electron count, mapping,
integral seed, iteration budget, state precision.  Nothing here computes.
"""

from __future__ import annotations

import numpy as np

from .integrals import electron_count

__all__ = ["CONFIGS", "batched_instances", "serving_requests"]

# name -> dict(n_qubits, n_electrons, mappings, seed, iters, dtype)
CONFIGS = {
    # 4 qubits / 2 electrons, H2-like; 10 ADAPT iterations, complex128.
    "c1_4q": dict(n_qubits=4, n_electrons=2, mappings=("jw",), seed=4,
                  iters=10, dtype="c128"),
    # 12 qubits / 6 electrons (H2O-sized register, Table II), JW and BK,
    # 30 ADAPT iterations, complex128.
    "c2_12q": dict(n_qubits=12, n_electrons=6, mappings=("jw", "bk"), seed=12,
                   iters=30, dtype="c128"),
    # 14 qubits / 6 electrons (BeH2-sized register, Tables I-II), JW and BK,
    # complex64 statevector with FP64 reductions beside the FP64 path.
    "c3_14q": dict(n_qubits=14, n_electrons=6, mappings=("jw", "bk"), seed=14,
                   iters=30, dtype="c64"),
}


def batched_instances():
    """64 instances: 24 x 10q, 24 x 12q, 16 x 14q; JW for even i, BK for odd.

    Returns a list of dicts(n_qubits, n_electrons, mapping, seed).
    """
    sizes = [10] * 24 + [12] * 24 + [14] * 16
    out = []
    for i, nq in enumerate(sizes):
        n = nq // 2
        out.append(dict(n_qubits=nq, n_electrons=electron_count(n),
                        mapping="jw" if i % 2 == 0 else "bk", seed=1000 + i))
    return out


def serving_requests(n_requests: int, rate_hz: float, seed: int = 7,
                     qubits=(8, 10, 12, 14, 16)):
    """A Poisson stream of ADAPT solve requests of mixed size.

    Request ``r`` uses integral seed ``2000 + r``; its qubit count is drawn
    uniformly from ``qubits`` and its mapping alternates JW/BK.  Returns a list
    of dicts(arrival_s, n_qubits, n_electrons, mapping, seed).
    """
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_hz, size=n_requests)
    arrivals = np.cumsum(gaps) - gaps[0]
    nqs = rng.choice(np.asarray(qubits), size=n_requests)
    out = []
    for r in range(n_requests):
        nq = int(nqs[r])
        out.append(dict(arrival_s=float(arrivals[r]), n_qubits=nq,
                        n_electrons=electron_count(nq // 2),
                        mapping="jw" if r % 2 == 0 else "bk", seed=2000 + r))
    return out
