"""GPU parity of the edge branches of the AUTO path and of the production
panel writer, through the C-ABI, against the FP64 oracle.

* Device decisions on inputs that reach every branch of the rule (Sec. 4.1
  stages, the overflow guard e_max <= 14, the BF16X3 floor 2^-110 and
  ceiling e_max <= 126, the all-zero operand): the decision record equals
  ``oracle.select_mode`` on the same FP32 values, and the product meets the
  bar of its mode (exact zeros, <= 2x the FP32 error against the exact
  product, the emulated value of the selected mode to accumulation
  accuracy).
* The panel writer every GEMM runs (rows-contiguous, k-contiguous with and
  without conjugation, and the transpose-fused bit-map layout), unpacked
  from its swizzled chunks on the host and compared bit for bit with the
  oracle's splits (Eq. 2; the BF16 three-term split; FP32 de-interleave),
  padding included.
* The environment variables read at handle creation (Sec. 3).
"""
import math
import os

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

U = 2.0 ** -24


@pytest.fixture(scope="module")
def qce():
    import paper_2303_08989_amd as q
    return q


@pytest.fixture(scope="module")
def handle(qce):
    h = qce.Handle(0)
    yield h
    h.set_tolerance(0.1, 0.0)
    h.close()


def dev(a):
    return torch.from_numpy(np.asfortranarray(a).ravel(order="F").copy()).to("cuda")


def host(t, rows, cols):
    return t.cpu().numpy().reshape((cols, rows)).T


def run(qce, h, A, B, mode="auto", alpha=1.0, beta=0.0, C0=None):
    m, k = A.shape
    n = B.shape[1]
    h.set_mode(mode)
    dC = dev(C0) if C0 is not None else torch.zeros(m * n, dtype=torch.complex64, device="cuda")
    qce.cgemm(h, "N", "N", m, n, k, dev(A), m, dev(B), k, dC, m, alpha, beta)
    torch.cuda.synchronize()
    return host(dC, m, n), h.last_decision()


def _complex(re, im):
    out = np.empty(re.shape, dtype=np.complex64)
    out.real = re
    out.imag = im
    return np.asfortranarray(out)


def _pow2_magnitudes(rng, shape, lo, hi):
    """+-2^U with U uniform in [lo, hi), per real component."""
    re = np.exp2(rng.uniform(lo, hi, shape)) * rng.choice([-1.0, 1.0], shape)
    im = np.exp2(rng.uniform(lo, hi, shape)) * rng.choice([-1.0, 1.0], shape)
    return _complex(re.astype(np.float32), im.astype(np.float32))


def _gauss(rng, shape, scale=1.0):
    return _complex((rng.standard_normal(shape) * scale).astype(np.float32),
                    (rng.standard_normal(shape) * scale).astype(np.float32))


def _check_decision(dec, A, B, t, t3):
    sa, sb = oracle.exp_stats(A), oracle.exp_stats(B)
    mode, s_a, s_b = oracle.select_mode(sa, sb, t, t3)
    assert (dec["mode"], dec["sA"], dec["sB"]) == (mode, s_a, s_b), (dec, mode, s_a, s_b)
    for o, st in enumerate((sa, sb)):
        assert dec["nnz"][o] == st["nnz"] and dec["n1"][o] == st["n1"], o
        assert dec["n3"][o] == st["n3"] and dec["nonfinite"][o] == st["nonfinite"], o
        if st["nnz"]:
            assert dec["emax"][o] == st["emax"], o
        else:
            assert dec["emax"][o] == -2 ** 31, o
        if dec["n2"][o] >= 0:
            assert dec["n2"][o] == st["n2"], o
    return mode


def _check_product(qce, h, A, B, C, dec):
    """C within 2x the FP32 error of the exact product, and within the
    accumulation bound of the oracle's value of the selected mode."""
    m, k = A.shape
    n = B.shape[1]
    exact = oracle.cgemm(A, B)
    C32, _ = run(qce, h, A, B, mode="fp32")
    tA = torch.from_numpy(np.ascontiguousarray(A)).to("cuda")
    tB = torch.from_numpy(np.ascontiguousarray(B)).to("cuda")
    Ct = torch.matmul(tA, tB).cpu().numpy()
    e_fp32 = min(oracle.rel_fro(C32, exact), oracle.rel_fro(Ct, exact))
    e = oracle.rel_fro(C, exact)
    assert e <= 2.0 * e_fp32, (dec["mode_name"], e, e_fp32)
    model = oracle.emulated_cgemm(A, B, dec["mode"], dec["sA"], dec["sB"])
    assert oracle.rel_fro(C, model) <= 4 * U * math.sqrt(k), dec["mode_name"]
    h.set_mode("auto")
    return C32


# ---------------------------------------------------------------------------
# Branches of the device decision
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("scale_exp", [15, 17, 20])
def test_overflow_guard_selects_scaled_with_negative_shift(qce, handle, scale_exp):
    # e_max > 14: stage 1 fails on the overflow guard although nothing
    # underflows; the narrow Gaussian passes stage 2, so the GEMM runs
    # FP16X2_SCALED with a negative shift for A
    rng = np.random.default_rng(scale_exp)
    m, n, k = 96, 80, 72
    A = _gauss(rng, (m, k), 2.0 ** scale_exp)
    B = _gauss(rng, (k, n))
    handle.set_tolerance(0.1, 0.0)
    C, dec = run(qce, handle, A, B)
    mode = _check_decision(dec, A, B, 0.1, 0.0)
    assert mode == oracle.MODE_FP16X2_SCALED
    assert dec["emax"][0] > 14 and dec["sA"] == 14 - dec["emax"][0] < 0
    _check_product(qce, handle, A, B, C, dec)


def test_wide_range_above_fp16_selects_bf16x3(qce, handle):
    # magnitudes 2^-30 .. 2^20: outside FP16's window even after the shift
    rng = np.random.default_rng(3)
    m, n, k = 70, 64, 50
    A = _pow2_magnitudes(rng, (m, k), -30, 20)
    B = _gauss(rng, (k, n))
    handle.set_tolerance(0.1, 0.0)
    C, dec = run(qce, handle, A, B)
    assert _check_decision(dec, A, B, 0.1, 0.0) == oracle.MODE_BF16X3
    assert dec["emax"][0] >= 15
    _check_product(qce, handle, A, B, C, dec)


@pytest.mark.parametrize("top,expect", [(126, oracle.MODE_BF16X3), (127, oracle.MODE_FP32)])
def test_bf16x3_ceiling(qce, handle, top, expect):
    # one component of magnitude 1.5 * 2^top, the rest spread over 2^-30 ..
    # 2^0: stage 2 fails (the window ends 28 binades below the top); the
    # BF16X3 level needs e_max <= 126, so 2^127 falls through to FP32
    rng = np.random.default_rng(top)
    m, n, k = 64, 40, 48
    A = _pow2_magnitudes(rng, (m, k), -30, 0)
    A[5, 7] = np.complex64(complex(1.5 * 2.0 ** top, -0.25))
    B = _gauss(rng, (k, n), 2.0 ** -20)
    handle.set_tolerance(0.1, 0.0)
    C, dec = run(qce, handle, A, B)
    assert _check_decision(dec, A, B, 0.1, 0.0) == expect
    assert dec["emax"][0] == top
    assert np.isfinite(C).all()
    C32 = _check_product(qce, handle, A, B, C, dec)
    if expect == oracle.MODE_FP32:
        assert np.array_equal(C, C32)      # the AUTO-selected FP32 is the forced FP32 kernel


@pytest.mark.parametrize("t3,expect", [(0.0, oracle.MODE_FP32), (0.25, oracle.MODE_BF16X3)])
def test_bf16x3_floor_and_its_tolerance(qce, handle, t3, expect):
    # about 10 % of A's components lie below 2^-110: FP32 at t3 = 0, BF16X3
    # once t3 admits them (the rule's third level, with its own tolerance)
    rng = np.random.default_rng(11)
    m, n, k = 64, 64, 64
    A = _pow2_magnitudes(rng, (m, k), -100, 0)
    low = rng.random((m, k)) < 0.1
    A.real[low] = np.float32(2.0 ** -115)
    B = _gauss(rng, (k, n))
    handle.set_tolerance(0.1, t3)
    try:
        C, dec = run(qce, handle, A, B)
        assert _check_decision(dec, A, B, 0.1, t3) == expect
    finally:
        handle.set_tolerance(0.1, 0.0)
    _check_product(qce, handle, A, B, C, dec)


@pytest.mark.parametrize("b_scale_exp,expect", [(0, oracle.MODE_FP16X2), (-30, oracle.MODE_FP16X2_SCALED)])
def test_all_zero_operand(qce, handle, b_scale_exp, expect):
    # an all-zero A is neutral (level FP16X2, shift 0); the product is an
    # exact zero, and with beta != 0 exactly beta * C0
    rng = np.random.default_rng(5)
    m, n, k = 64, 48, 32
    A = np.zeros((m, k), dtype=np.complex64, order="F")
    B = _gauss(rng, (k, n), 2.0 ** b_scale_exp)
    handle.set_tolerance(0.1, 0.0)
    C, dec = run(qce, handle, A, B)
    assert _check_decision(dec, A, B, 0.1, 0.0) == expect
    assert dec["nnz"][0] == 0 and dec["sA"] == 0 and dec["n1"][0] == 0
    assert dec["stats_taken"] == 1
    assert np.array_equal(C, np.zeros((m, n), np.complex64))
    C0 = synth.random_matrix(m, n, "int", rng)
    beta = complex(-2, 1)
    C, dec = run(qce, handle, A, B, beta=beta, C0=C0)
    assert np.array_equal(C.astype(np.complex128), beta * C0.astype(np.complex128))


def test_both_operands_zero(qce, handle):
    m, n, k = 40, 36, 20
    A = np.zeros((m, k), dtype=np.complex64, order="F")
    B = np.zeros((k, n), dtype=np.complex64, order="F")
    C, dec = run(qce, handle, A, B)
    assert (dec["mode"], dec["sA"], dec["sB"]) == (oracle.MODE_FP16X2, 0, 0)
    assert dec["nnz"] == [0, 0]
    assert np.array_equal(C, np.zeros((m, n), np.complex64))


# ---------------------------------------------------------------------------
# The production panel writer, bit for bit
# ---------------------------------------------------------------------------

_FMT = {"fp16x2": (4, 2), "fp16x2_scaled": (4, 2), "bf16x3": (6, 2), "fp32": (2, 4)}


def _swz(rows, granules):
    r = np.arange(rows)
    if granules == 4:
        return ((r >> 2) & 1) | ((((r >> 1) ^ (r >> 3)) & 1) << 1)
    return ((r >> 2) ^ (r >> 3)) & 1


def decode_panels(buf, mode, rows, k):
    """Unpack the panel format (the layout the header states) into
    (planes, rows_pad, k_pad) arrays of uint16 or uint32 bit patterns."""
    planes, esz = _FMT[mode]
    row_bytes = 16 * esz
    gran = row_bytes // 16
    rows_pad = -(-rows // 128) * 128
    nch = -(-k // 16)
    b = np.asarray(buf, dtype=np.uint8).reshape(rows_pad // 128, nch, planes, 128, gran, 16)
    idx = np.arange(gran)[None, :] ^ _swz(128, gran)[:, None]          # [row, logical g] -> stored g
    b = np.take_along_axis(b, idx[None, None, None, :, :, None], axis=4)
    dt = np.uint16 if esz == 2 else np.uint32
    vals = np.ascontiguousarray(b).view(dt).reshape(rows_pad // 128, nch, planes, 128, 16)
    return vals.transpose(2, 0, 3, 1, 4).reshape(planes, rows_pad, nch * 16)


def expected_planes(P, mode, shift):
    """The oracle's split of the operand P (rows x k), as planes."""
    re = np.ascontiguousarray(P.real, dtype=np.float32)
    im = np.ascontiguousarray(P.imag, dtype=np.float32)
    if mode in ("fp16x2", "fp16x2_scaled"):
        hr, lr = oracle.split_fp16x2(re, shift)
        hi_, li = oracle.split_fp16x2(im, shift)
        return [x.view(np.uint16) for x in (hr, lr, hi_, li)]
    if mode == "bf16x3":
        return list(oracle.split_bf16x3(re)) + list(oracle.split_bf16x3(im))
    return [re.view(np.uint32), im.view(np.uint32)]


def _assert_panels(buf, mode, shift, P):
    rows, k = P.shape
    got = decode_panels(buf.cpu().numpy(), mode, rows, k)
    want = expected_planes(P, mode, shift)
    assert got.shape[0] == len(want)
    for p, ref in enumerate(want):
        assert np.array_equal(got[p, :rows, :k], ref), (mode, shift, p)
        assert not got[p, rows:, :].any() and not got[p, :, k:].any(), (mode, p, "padding")


def _split_values(rng, shape):
    """Components that reach the split's rounding cases: Gaussians, values
    below FP16's normal range, wide exponents, ties of the FP16 and BF16
    conversions, signed zeros."""
    n = int(np.prod(shape))
    pool = np.concatenate([
        rng.standard_normal(n), rng.uniform(-1, 1, n) * 2.0 ** -14, np.exp2(rng.uniform(-40, 10, n)),
        [1 + 2 ** -11, 1 + 3 * 2 ** -11, 1 + 2 ** -8, 1 + 3 * 2 ** -8, 2 ** -14, 2 ** -24, 0.0, -0.0],
    ]).astype(np.float32)
    re = rng.choice(pool, n).reshape(shape)
    im = rng.choice(pool, n).reshape(shape)
    return _complex(re, im)


@pytest.mark.parametrize("mode,shift", [("fp16x2", 0), ("fp16x2_scaled", 5), ("fp16x2_scaled", -3),
                                        ("bf16x3", 0), ("fp32", 0)])
@pytest.mark.parametrize("layout,conj", [(0, False), (0, True), (1, False), (1, True)])
def test_split_panels_bit_exact(qce, handle, mode, shift, layout, conj):
    rng = np.random.default_rng(7 + layout + 3 * (shift + 8))
    rows, k = 200, 70                       # two row blocks, five chunks, ragged tails
    stored = (rows, k) if layout == 0 else (k, rows)
    ld = stored[0] + 9
    X = _split_values(rng, (ld, stored[1]))
    buf = qce.split_panels(handle, mode, shift, dev(X), rows, k, ld, layout=layout, conj=conj)
    torch.cuda.synchronize()
    S = X[:stored[0], :]
    P = S if layout == 0 else S.T
    if conj:
        P = np.conj(P)
    _assert_panels(buf, mode, shift, np.asarray(P, dtype=np.complex64))


@pytest.mark.parametrize("mode,shift", [("fp16x2", 0), ("fp16x2_scaled", 4), ("bf16x3", 0), ("fp32", 0)])
@pytest.mark.parametrize("nr,nk,seed", [(7, 6, 0), (8, 7, 1), (5, 4, 2), (9, 5, 3)])
def test_split_panels_bitmap_bit_exact(qce, handle, mode, shift, nr, nk, seed):
    # the transpose-fused operand: P[r][l] = X[sum bit_t(r) 2^rsh[t] + sum bit_t(l) 2^ksh[t]]
    rng = np.random.default_rng(100 + seed)
    nb = nr + nk
    perm = rng.permutation(nb)
    rsh, ksh = [int(v) for v in perm[:nr]], [int(v) for v in perm[nr:]]
    X = _split_values(rng, (1 << nb,)).reshape(-1)
    r = np.arange(1 << nr)
    l = np.arange(1 << nk)
    roff = sum(((r >> t) & 1) << rsh[t] for t in range(nr))
    koff = sum(((l >> t) & 1) << ksh[t] for t in range(nk))
    P = X[roff[:, None] + koff[None, :]]
    buf = qce.split_panels_bitmap(handle, mode, shift, torch.from_numpy(X).to("cuda"), rsh, ksh)
    torch.cuda.synchronize()
    _assert_panels(buf, mode, shift, P)


def test_split_panels_argument_errors(qce, handle):
    t = torch.zeros(64, dtype=torch.complex64, device="cuda")
    with pytest.raises(qce.QceError):
        qce.split_panels(handle, "fp16x2", 3, t, 8, 8, 8)          # shift without the scaled mode
    with pytest.raises(qce.QceError):
        qce.split_panels(handle, "auto", 0, t, 8, 8, 8)
    with pytest.raises(qce.QceError):
        qce.split_panels(handle, "fp32", 0, t, 8, 8, 4)            # ld < rows
    with pytest.raises(qce.QceError):
        qce.split_panels_bitmap(handle, "fp32", 0, t, [0, 1, 2, 3, 4], [5, 6, 7, 7])   # not a permutation


# ---------------------------------------------------------------------------
# Environment read at handle creation (Sec. 3)
# ---------------------------------------------------------------------------

def _with_env(env, fn):
    saved = {k: os.environ.get(k) for k in env}
    os.environ.update(env)
    try:
        return fn()
    finally:
        for k, v in saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v


def test_environment_selects_mode_and_tolerance(qce):
    import paper_2303_08989_amd._lib as L

    def make():
        return qce.Handle(0)

    h = _with_env({"QCE_MODE": "bf16x3"}, make)
    assert h.get_mode() == L.MODE_BF16X3
    rng = np.random.default_rng(2)
    A = _gauss(rng, (64, 32))
    B = _gauss(rng, (32, 48))
    dC = torch.zeros(64 * 48, dtype=torch.complex64, device="cuda")
    qce.cgemm(h, "N", "N", 64, 48, 32, dev(A), 64, dev(B), 32, dC, 64)
    assert h.last_decision()["mode"] == oracle.MODE_BF16X3
    h.close()
    # 30 % of A below 2^-14 (but inside the shifted window): stage 1 passes
    # only when the tolerance admits them
    A = _gauss(rng, (64, 32))
    low = rng.random((64, 32)) < 0.3
    A.real[low] = np.float32(2.0 ** -20)
    for tol, expect in (("0.5", oracle.MODE_FP16X2), ("0.1", oracle.MODE_FP16X2_SCALED)):
        h = _with_env({"QCE_MODE": "auto", "QCE_UNDERFLOW_TOL": tol}, make)
        assert h.get_mode() == L.MODE_AUTO
        qce.cgemm(h, "N", "N", 64, 48, 32, dev(A), 64, dev(B), 32, dC, 64)
        dec = h.last_decision()
        want = oracle.select_mode(oracle.exp_stats(A), oracle.exp_stats(B), float(tol), 0.0)
        assert (dec["mode"], dec["sA"], dec["sB"]) == want and want[0] == expect
        h.close()
    for bad in ({"QCE_MODE": "fp8"}, {"QCE_UNDERFLOW_TOL": "1.5"}, {"QCE_BF16X3_TOL": "x"}):
        with pytest.raises(qce.QceError) as e:
            _with_env(bad, make)
        assert e.value.status == 1
