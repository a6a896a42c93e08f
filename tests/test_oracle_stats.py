"""Pins of the exponent statistics and the two-stage selection rule
(Sec. 4.1; AUTO-t of Sec. 5.2) against hand-counted cases, closed-form
expectations for the workload distributions and the paper's stated
property that t = 0 admits no underflow."""
import json
import os

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

import oracle
import synth

F16, F16S, B3, F32 = (oracle.MODE_FP16X2, oracle.MODE_FP16X2_SCALED,
                      oracle.MODE_BF16X3, oracle.MODE_FP32)


def test_hand_counted_stats():
    v = np.array([1.0, 2.0 ** -14, np.nextafter(np.float32(2.0 ** -14), np.float32(0)),
                  0.0, -0.0, -1.5 * 2.0 ** 14, 2.0 ** -110, 2.0 ** -111, 1e-45], dtype=np.float32)
    s = oracle.exp_stats(v)
    # nonzero: 1, 2^-14, below(2^-14), -1.5*2^14, 2^-110, 2^-111, 1e-45 (subnormal)
    assert s["nnz"] == 7 and s["nonfinite"] == 0
    assert s["emax"] == 14
    assert s["n1"] == 3                      # 1, 2^-14, 1.5*2^14
    assert s["n3"] == 5                      # all but 2^-111 and the subnormal
    assert s["n2"] == 3                      # e >= emax - 28 = -14: same three as n1
    s2 = oracle.exp_stats(np.array([np.inf, 1.0, np.nan], dtype=np.float32))
    assert s2["nonfinite"] == 2 and s2["nnz"] == 1


def test_complex_components_are_separate_elements():
    # Sec. 4.1 counts elements; real and imaginary parts are separate FP32 values
    z = np.array([1 + 0j, 0 + 2.0 ** -20 * 1j], dtype=np.complex64)
    s = oracle.exp_stats(z)
    assert s["nnz"] == 2 and s["n1"] == 1


def test_subnormal_exponents_exact():
    tiny = np.array([1e-45], dtype=np.float32)     # 2^-149
    assert oracle.exp_stats(tiny)["emax"] == -149
    big_sub = np.array([np.float32(2.0 ** -127)], dtype=np.float32)
    assert oracle.exp_stats(big_sub)["emax"] == -127


def _st(nnz, emax, n1, n2, n3, nonfinite=0):
    return {"nnz": nnz, "emax": emax, "n1": n1, "n2": n2, "n3": n3, "nonfinite": nonfinite}


def test_rule_levels():
    t = 0.1
    assert oracle.select_level(_st(100, 2, 100, 100, 100), t) == F16
    assert oracle.select_level(_st(100, 2, 91, 100, 100), t) == F16         # 9% underflow tolerated
    assert oracle.select_level(_st(100, 2, 89, 100, 100), t) == F16S        # 11% -> scaling
    assert oracle.select_level(_st(100, 15, 100, 100, 100), t) == F16S      # overflow guard
    assert oracle.select_level(_st(100, -1, 0, 95, 100), t) == F16S
    assert oracle.select_level(_st(100, -1, 0, 80, 100), t) == B3
    assert oracle.select_level(_st(100, -1, 0, 80, 99), t) == F32           # t3 = 0
    assert oracle.select_level(_st(100, -1, 0, 80, 99), t, t3=0.05) == B3
    assert oracle.select_level(_st(0, None, 0, 0, 0), t) == F16             # all zero
    assert oracle.select_level(_st(100, 2, 100, 100, 100, nonfinite=1), t) == F32


def test_rule_combines_both_operands():
    # Sec. 4.1: either operand failing a stage decides the mode
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_examples.json")))
    top = g["selection_rule"]["scaled_max_exponent"]
    good = oracle.exp_stats(np.ones(8, dtype=np.float32))
    small = oracle.exp_stats(np.full(8, 2.0 ** -30, dtype=np.float32))
    wide = oracle.exp_stats(np.array([1.0] * 4 + [2.0 ** -60] * 4, dtype=np.float32))
    assert oracle.select_mode(good, good) == (F16, 0, 0)
    mode, sA, sB = oracle.select_mode(good, small)
    assert mode == F16S and sA == top - 0 and sB == top + 30
    assert oracle.select_mode(small, wide)[0] == B3
    assert oracle.select_mode(wide, good)[0] == B3


def test_workload_distributions_closed_form():
    """(a) complex Gaussian: P(|x| < 2^-14) ~ 2^-13 * 0.4 ~ 5e-5 and
    emax ~ 2 -> FP16X2.  (b) 2^U, U ~ U(-40, 0): 65% below 2^-14, 27.5% below
    2^(emax-28) = 2^-29 -> neither FP16 stage; all above 2^-110 -> BF16X3.
    (c) 2^U, U ~ U(-120, 0) with zeros: 10/120 of the nonzeros below 2^-110
    -> FP32."""
    n = 1 << 17
    a, b = synth.gemm_operands(n // 64, 64, 64, "a", 0)
    sa = oracle.exp_stats(a)
    assert (sa["nnz"] - sa["n1"]) / sa["nnz"] < 4e-4 and sa["emax"] in (1, 2, 3)
    assert oracle.select_mode(sa, oracle.exp_stats(b))[0] == F16
    a, b = synth.gemm_operands(n // 64, 64, 64, "b", 0)
    sa = oracle.exp_stats(a)
    assert abs((sa["nnz"] - sa["n1"]) / sa["nnz"] - 26 / 40) < 0.01
    assert sa["emax"] == -1
    assert abs((sa["nnz"] - sa["n2"]) / sa["nnz"] - 11 / 40) < 0.01
    assert oracle.select_mode(sa, oracle.exp_stats(b))[0] == B3
    a, b = synth.gemm_operands(n // 64, 64, 64, "c", 0)
    sa = oracle.exp_stats(a)
    assert abs(sa["nnz"] / (2 * a.size) - 7 / 8) < 0.01
    assert abs((sa["nnz"] - sa["n3"]) / sa["nnz"] - 10 / 120) < 0.01
    assert oracle.select_mode(sa, oracle.exp_stats(b))[0] == F32


@settings(max_examples=200, deadline=None)
@given(st.lists(st.one_of(st.floats(min_value=-1.0, max_value=1.0, width=32),
                          st.sampled_from([0.0, 2.0 ** -14, 2.0 ** -40, 2.0 ** -29, 3e-39])),
                min_size=1, max_size=40))
def test_auto_zero_admits_no_underflow(values):
    """Sec. 5.2: with t = 0 the selected FP16 mode underflows no element: after
    the shift every nonzero element lies in [2^-14, 2^15)."""
    x = np.array(values, dtype=np.float32)
    s = oracle.exp_stats(x)
    mode, sx, _ = oracle.select_mode(s, s, t=0.0)
    if mode in (F16, F16S):
        nz = x[x != 0].astype(np.float64) * 2.0 ** sx
        assert np.all(np.abs(nz) >= 2.0 ** -14) and np.all(np.abs(nz) < 2.0 ** 15)
        # and the split then represents every element to 22 bits
        hi, lo = oracle.split_fp16x2(x, sx)
        recon = hi.astype(np.float64) + lo.astype(np.float64) / 2048.0
        xs = x.astype(np.float64) * 2.0 ** sx
        assert np.all(np.abs(recon - xs) <= 2.0 ** -22 * np.abs(xs))


def test_amplitude_exponent_golden():
    """Sec. 2.2: an n-qubit amplitude of size 2^-(n-1)/2 must be representable."""
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_examples.json")))
    for case in g["amplitude_exponent"]["cases"]:
        amp = np.float32(2.0 ** (-(case["n"] - 1) / 2))
        s = oracle.exp_stats(np.array([amp], dtype=np.float32))
        fits = oracle.select_level(s, t=0.0) == F16
        assert fits == case["fits_fp16_normal"]
