"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package only draws random numbers and arranges them into arrays.  It holds
none of the method's arithmetic (no mapping, no Pauli algebra, no state
evolution), so both the CPU oracle and the HIP path may consume it without
sharing any computation.
"""

from .integrals import molecular_integrals, electron_count
from .configs import CONFIGS, batched_instances, serving_requests

__all__ = ["molecular_integrals", "electron_count", "CONFIGS",
           "batched_instances", "serving_requests"]
