"""Pins of the oracle's splits (Sec. 2.1, Eq. 2; BF16 three-term split) and of
its emulated-product model, against rounding facts checked independently of
the conversion routines the oracle calls."""
import numpy as np
import pytest
import torch

import oracle
import synth


def _all_mantissas(exponent, signs=(1.0, -1.0), stride=1):
    m = np.arange(0, 1 << 23, stride, dtype=np.uint32)
    out = []
    for s in signs:
        bits = ((np.uint32(exponent + 127) << np.uint32(23)) | m)
        v = bits.view(np.float32)
        out.append(v if s > 0 else -v)
    return np.concatenate(out)


def _is_nearest_even_fp16(x64, h16):
    """Check h16 is a correctly rounded (ties-to-even) FP16 of x64, by
    comparing against the two FP16 neighbours of h16."""
    h = h16.astype(np.float64)
    up = np.nextafter(h16, np.float16(np.inf)).astype(np.float64)
    dn = np.nextafter(h16, np.float16(-np.inf)).astype(np.float64)
    d = np.abs(x64 - h)
    ok = (d <= np.abs(x64 - up)) & (d <= np.abs(x64 - dn))
    tie = (d == np.abs(x64 - up)) | (d == np.abs(x64 - dn))
    even = (h16.view(np.uint16) & 1) == 0
    return bool(np.all(ok & (~tie | even)))


@pytest.mark.parametrize("e,stride", [(0, 1), (-14, 3), (14, 3), (-20, 5), (7, 5)])
def test_fp16x2_exhaustive_binade(e, stride):
    # every mantissa of binade 2^0; every stride-th mantissa of the others
    x = _all_mantissas(e, stride=stride)
    hi, lo = oracle.split_fp16x2(x)
    x64 = x.astype(np.float64)
    # hi is the nearest-even FP16 of x
    assert _is_nearest_even_fp16(x64, hi)
    r64 = x64 - hi.astype(np.float64)
    # the FP32 residual is exact, so lo is the nearest-even FP16 of r * 2^11
    assert _is_nearest_even_fp16(r64 * 2048.0, lo)
    recon = hi.astype(np.float64) + lo.astype(np.float64) / 2048.0
    if -14 <= e <= 14:
        # hi and lo normal or tiny: two 11-bit digits -> 22 correct bits
        nz = r64 != 0
        assert np.all(np.abs(recon - x64) <= 2.0 ** -22 * np.abs(x64))
        assert np.any(nz)


def test_fp16x2_worked_ties():
    # 1 + 2^-11 lies halfway between 1 and 1 + 2^-10: ties to even -> 1,
    # residual 2^-11, scaled by 2^11 -> lo = 1.
    hi, lo = oracle.split_fp16x2(np.array([1 + 2.0 ** -11], dtype=np.float32))
    assert hi[0] == 1.0 and lo[0] == 1.0
    # 1 + 3*2^-11: halfway between 1+2^-10 (odd) and 1+2^-9 (even) -> 1+2^-9
    hi, lo = oracle.split_fp16x2(np.array([1 + 3 * 2.0 ** -11], dtype=np.float32))
    assert hi[0] == 1 + 2.0 ** -9 and lo[0] == -1.0
    # values exactly representable in FP16 have a zero residual
    hi, lo = oracle.split_fp16x2(np.array([0.375, -1024.0, 2.0 ** -14], dtype=np.float32))
    assert np.array_equal(hi.astype(np.float32), [0.375, -1024.0, 2.0 ** -14]) and not lo.any()


def test_fp16x2_scaling_is_a_shift():
    rng = np.random.default_rng(0)
    x = (rng.standard_normal(10000) * 2.0 ** -30).astype(np.float32)
    for s in (20, 30, 40):
        h1, l1 = oracle.split_fp16x2(x, s)
        h2, l2 = oracle.split_fp16x2((x.astype(np.float64) * 2.0 ** s).astype(np.float32), 0)
        assert np.array_equal(h1.view(np.uint16), h2.view(np.uint16))
        assert np.array_equal(l1.view(np.uint16), l2.view(np.uint16))


def test_bf16_rne_matches_torch():
    rng = np.random.default_rng(1)
    x = np.concatenate([
        rng.standard_normal(200000).astype(np.float32),
        (rng.standard_normal(20000) * 1e-38).astype(np.float32),
        np.array([1 + 2.0 ** -8, 1 + 3 * 2.0 ** -8, -(1 + 2.0 ** -8), 3.0e38, 0.0, -0.0], dtype=np.float32),
        _all_mantissas(-3)[::7],
    ])
    ours = oracle.bf16_rne(x)
    ref = torch.from_numpy(x).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(ours, ref)


@pytest.mark.parametrize("e,stride", [(0, 1), (-40, 3), (-100, 3), (100, 3)])
def test_bf16x3_exact_reconstruction(e, stride):
    x = _all_mantissas(e, stride=stride)
    b0, b1, b2 = oracle.split_bf16x3(x)
    f = oracle.bf16_to_f32
    s = f(b0).astype(np.float64) + f(b1).astype(np.float64) + f(b2).astype(np.float64)
    assert np.array_equal(s, x.astype(np.float64))
    ax = np.abs(x.astype(np.float64))
    assert np.all(np.abs(f(b1).astype(np.float64)) <= 2.0 ** -8 * ax)
    assert np.all(np.abs(f(b2).astype(np.float64)) <= 2.0 ** -16 * ax)


@pytest.mark.parametrize("mode", [oracle.MODE_FP16X2, oracle.MODE_FP16X2_SCALED,
                                  oracle.MODE_BF16X3, oracle.MODE_FP32])
def test_emulation_exact_on_integers(mode):
    a, b = synth.gemm_operands(19, 23, 31, "int", 4)
    exact = oracle.cgemm(a, b)
    s = 3 if mode == oracle.MODE_FP16X2_SCALED else 0
    got = oracle.emulated_cgemm(a, b, mode, s, -s)
    assert np.array_equal(got, exact)


def test_emulation_drops_only_the_residual_product():
    # Eq. 2 keeps hi*hi and the two cross terms; the elementwise deviation from
    # the exact product is bounded by the split's 2^-22 representation error
    # of each factor plus the dropped residual product.
    a, b = synth.gemm_operands(40, 30, 50, "u", 9)
    exact = oracle.cgemm(a, b)
    absab = np.abs(a).astype(np.float64) @ np.abs(b).astype(np.float64)
    got = oracle.emulated_cgemm(a, b, oracle.MODE_FP16X2)
    assert np.all(np.abs(got - exact) <= 8 * 2.0 ** -22 * absab)
    # and it is far better than FP16 alone: the correction terms are present
    assert oracle.rel_fro(got, exact) < 2.0 ** -20
    # BF16X3 keeps six products; the dropped ones are below 2^-24 relative
    got3 = oracle.emulated_cgemm(a, b, oracle.MODE_BF16X3)
    assert np.all(np.abs(got3 - exact) <= 8 * 2.0 ** -24 * absab)


def test_emulation_power_of_two_invariance():
    a, b = synth.gemm_operands(16, 16, 16, "a", 2)
    base = oracle.emulated_cgemm(a, b, oracle.MODE_FP16X2)
    a2 = (a * np.float32(2.0 ** -5)).astype(np.complex64)
    b2 = (b * np.float32(2.0 ** 3)).astype(np.complex64)
    scaled = oracle.emulated_cgemm(a2, b2, oracle.MODE_FP16X2_SCALED, 5, -3)
    assert np.array_equal(scaled * 2.0 ** 2, base)


def test_golden_residual_scale():
    import json, os
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_examples.json")))
    sc = g["tcec_split_scale"]["residual_scale_log2"]
    x = np.array([1 + 2.0 ** -11 + 2.0 ** -20], dtype=np.float32)
    hi, lo = oracle.split_fp16x2(x)
    r = float(x[0]) - float(hi[0])
    assert float(lo[0]) == pytest.approx(r * 2.0 ** sc, rel=2.0 ** -10)
