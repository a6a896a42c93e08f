"""Random complex64 matrices for the standalone CGEMM workload.

Value distributions (applied to the real and imaginary component of every
element independently):

* ``"a"``   complex Gaussian, each component N(0, 1);
* ``"b"``   random sign times 2**U with U ~ Uniform(-40, 0) (log-uniform
            magnitudes over [2^-40, 1]);
* ``"c"``   exactly zero with probability 1/8, otherwise random sign times
            2**U with U ~ Uniform(-120, 0);
* ``"u"``   Uniform(-1, 1), the distribution of the paper's CGEMM unit test
            (Sec. 3, the accuracy/throughput test around Eq. 3);
* ``"int"`` integers in [-8, 8]: every product and partial sum is exact in
            FP32 for k <= 2^15, so every GEMM mode must agree bit for bit.

Matrices are returned as numpy complex64 arrays in Fortran (column-major)
order, matching the BLAS convention of the C-ABI: element (i, j) of an
``rows x cols`` matrix sits at ``i + j * rows``.
"""
import numpy as np

DISTRIBUTIONS = ("a", "b", "c", "u", "int")


def _component(rng, dist, size):
    if dist == "a":
        return rng.standard_normal(size)
    if dist == "b":
        sign = np.where(rng.random(size) < 0.5, -1.0, 1.0)
        return sign * np.exp2(rng.uniform(-40.0, 0.0, size))
    if dist == "c":
        sign = np.where(rng.random(size) < 0.5, -1.0, 1.0)
        mag = np.exp2(rng.uniform(-120.0, 0.0, size))
        zero = rng.random(size) < 0.125
        return np.where(zero, 0.0, sign * mag)
    if dist == "u":
        return rng.uniform(-1.0, 1.0, size)
    if dist == "int":
        return rng.integers(-8, 9, size).astype(np.float64)
    raise ValueError(f"unknown distribution {dist!r}")


def random_matrix(rows, cols, dist, rng):
    """rows x cols complex64 matrix, column-major, drawn from ``dist``."""
    n = rows * cols
    re = _component(rng, dist, n).astype(np.float32)
    im = _component(rng, dist, n).astype(np.float32)
    out = np.empty(n, dtype=np.complex64)
    out.real = re
    out.imag = im
    return out.reshape((rows, cols), order="F")


def gemm_operands(m, n, k, dist, seed):
    """Operands A (m x k) and B (k x n) of one CGEMM, column-major complex64."""
    rng = np.random.default_rng(seed)
    a = random_matrix(m, k, dist, rng)
    b = random_matrix(k, n, dist, rng)
    return a, b


def case_seed(dist, shape_index, rep):
    """Seed of one (distribution, shape, repetition) case: 1000*d + 10*s + r."""
    d = DISTRIBUTIONS.index(dist)
    return 1000 * d + 10 * shape_index + rep
