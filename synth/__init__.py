"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package holds only input generation: random matrices with the value
distributions of the GEMM workloads, random quantum circuits with their gate
matrices, random bitstrings and random tensor networks.  It contains none of
the method's arithmetic (no splitting, statistics, mode selection or
contraction), so the FP64 oracle and the GPU path can both consume it without
sharing any computation.
"""
from .gemm_inputs import gemm_operands, random_matrix, DISTRIBUTIONS  # noqa: F401
from .circuits import (  # noqa: F401
    grid_circuit, ghz_circuit, identity_circuit, product_circuit,
    random_bitstrings, gate_matrix, GRID_53, with_thetas, coupler_thetas,
)
from .tn_random import random_network, random_closed_network, random_tn_tensor, TN_TYPES  # noqa: F401
