"""GPU parity of the emulated CGEMM path (stats -> select -> split -> MFMA
GEMM) against the FP64 oracle, through the C-ABI.

Bars:
* integer-valued inputs: every mode exact, bit for bit (all products and
  partial sums are exact in FP32);
* statistics and decisions: exact integers equal to the oracle's;
* splits: bit-exact against the oracle's splits;
* floating point: relative Frobenius error of the emulated result at most
  twice that of a plain FP32 CGEMM on the same inputs (the smaller of the
  library's FP32 mode and rocBLAS through torch), and within an
  accumulation-level bound of the oracle's FP64 value of the emulated
  product.
"""
import math

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
    h.close()


def dev(a):
    """column-major complex64 numpy matrix -> flat device tensor"""
    flat = np.asfortranarray(a).ravel(order="F")
    return torch.from_numpy(flat.copy()).to("cuda")


def host(t, rows, cols, ld=None):
    ld = ld or rows
    flat = t.cpu().numpy()
    out = np.empty((rows, cols), dtype=np.complex64, order="F")
    for j in range(cols):
        out[:, j] = flat[j * ld:j * ld + rows]
    return out


def run(qce, h, A, B, m, n, k, opA="N", opB="N", alpha=1.0, beta=0.0, C0=None, mode="auto"):
    h.set_mode(mode)
    lda = A.shape[0]
    ldb = B.shape[0]
    dA, dB = dev(A), dev(B)
    dC = dev(C0) if C0 is not None else torch.zeros(m * n, dtype=torch.complex64, device="cuda")
    qce.cgemm(h, opA, opB, m, n, k, dA, lda, dB, ldb, dC, m, alpha, beta)
    torch.cuda.synchronize()
    return host(dC, m, n), h.last_decision()


def shapes_of(m, n, k, opA, opB):
    sa = (m, k) if opA == "N" else (k, m)
    sb = (k, n) if opB == "N" else (n, k)
    return sa, sb


MODES = ["fp16x2", "fp16x2_scaled", "bf16x3", "fp32", "auto"]


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("m,n,k", [(1, 1, 1), (200, 150, 70), (128, 256, 64), (33, 300, 257)])
def test_integer_inputs_bit_exact(qce, handle, mode, m, n, k):
    rng = np.random.default_rng(m * 7 + n * 3 + k)
    A = synth.random_matrix(m, k, "int", rng)
    B = synth.random_matrix(k, n, "int", rng)
    C, dec = run(qce, handle, A, B, m, n, k, mode=mode)
    want = oracle.cgemm(A, B)
    assert np.array_equal(C.astype(np.complex128), want)


@pytest.mark.parametrize("opA,opB", [("N", "T"), ("T", "N"), ("C", "N"), ("N", "C"), ("C", "T"), ("T", "C")])
@pytest.mark.parametrize("mode", ["fp16x2", "bf16x3", "fp32"])
def test_ops_integer_exact(qce, handle, opA, opB, mode):
    m, n, k = 77, 140, 45
    rng = np.random.default_rng(5)
    sa, sb = shapes_of(m, n, k, opA, opB)
    A = synth.random_matrix(*sa, "int", rng)
    B = synth.random_matrix(*sb, "int", rng)
    C, _ = run(qce, handle, A, B, m, n, k, opA, opB, mode=mode)
    assert np.array_equal(C.astype(np.complex128), oracle.cgemm(A, B, opA, opB))


def test_alpha_beta_exact(qce, handle):
    m, n, k = 60, 50, 40
    rng = np.random.default_rng(9)
    A = synth.random_matrix(m, k, "int", rng)
    B = synth.random_matrix(k, n, "int", rng)
    C0 = synth.random_matrix(m, n, "int", rng)
    alpha, beta = complex(2, -1), complex(-3, 0.5)
    for mode in ("fp16x2", "bf16x3", "fp32", "auto"):
        C, _ = run(qce, handle, A, B, m, n, k, alpha=alpha, beta=beta, C0=C0, mode=mode)
        want = oracle.cgemm(A, B, alpha=alpha, beta=beta, C0=C0)
        assert np.array_equal(C.astype(np.complex128), want), mode


def test_beta_zero_ignores_nan_in_c(qce, handle):
    m, n, k = 20, 20, 20
    rng = np.random.default_rng(1)
    A = synth.random_matrix(m, k, "int", rng)
    B = synth.random_matrix(k, n, "int", rng)
    C0 = np.full((m, n), np.nan + 1j * np.nan, dtype=np.complex64, order="F")
    C, _ = run(qce, handle, A, B, m, n, k, C0=C0, mode="auto")
    assert np.array_equal(C.astype(np.complex128), oracle.cgemm(A, B))


def test_k_zero_scales_c(qce, handle):
    m, n = 30, 20
    rng = np.random.default_rng(2)
    C0 = synth.random_matrix(m, n, "int", rng)
    A = np.zeros((m, 1), dtype=np.complex64, order="F")
    B = np.zeros((1, n), dtype=np.complex64, order="F")
    handle.set_mode("auto")
    dA, dB, dC = dev(A), dev(B), dev(C0)
    qce.cgemm(handle, "N", "N", m, n, 0, dA, m, dB, 1, dC, m, 1.0, 2.0)
    assert np.array_equal(host(dC, m, n), 2 * C0)


def test_argument_errors(qce, handle):
    t = torch.zeros(16, dtype=torch.complex64, device="cuda")
    with pytest.raises(qce.QceError) as e:
        qce.cgemm(handle, "N", "N", 4, 4, 4, t, 3, t, 4, t, 4)   # lda < m
    assert e.value.status == 1
    with pytest.raises(qce.QceError):
        qce.cgemm(handle, "N", "N", -1, 4, 4, t, 4, t, 4, t, 4)
    # m == 0 is a successful no-op
    qce.cgemm(handle, "N", "N", 0, 4, 4, t, 1, t, 4, t, 1)


@pytest.mark.parametrize("dist,expect", [("a", oracle.MODE_FP16X2), ("u", oracle.MODE_FP16X2),
                                         ("b", oracle.MODE_BF16X3), ("c", oracle.MODE_FP32)])
def test_auto_decision_matches_oracle(qce, handle, dist, expect):
    m, n, k = 300, 260, 190
    A, B = synth.gemm_operands(m, n, k, dist, seed=17)
    handle.set_tolerance(0.1, 0.0)
    C, dec = run(qce, handle, A, B, m, n, k, mode="auto")
    sa, sb = oracle.exp_stats(A), oracle.exp_stats(B)
    mode, s_a, s_b = oracle.select_mode(sa, sb, 0.1, 0.0)
    assert mode == expect
    assert dec["mode"] == mode and dec["sA"] == s_a and dec["sB"] == s_b
    for o, st in enumerate((sa, sb)):
        assert dec["nnz"][o] == st["nnz"] and dec["n1"][o] == st["n1"]
        assert dec["n3"][o] == st["n3"] and dec["nonfinite"][o] == st["nonfinite"]
        assert dec["emax"][o] == st["emax"]
        if dec["n2"][o] >= 0:
            assert dec["n2"][o] == st["n2"]


def _fp32_refs(qce, h, A, B, m, n, k):
    C32, _ = run(qce, h, A, B, m, n, k, mode="fp32")
    tA = torch.from_numpy(np.ascontiguousarray(A)).to("cuda")
    tB = torch.from_numpy(np.ascontiguousarray(B)).to("cuda")
    Ct = torch.matmul(tA, tB).cpu().numpy()
    return C32, Ct


@pytest.mark.parametrize("dist", ["a", "u", "b", "c"])
@pytest.mark.parametrize("m,n,k", [(384, 320, 512), (257, 129, 1000)])
def test_error_at_most_twice_fp32(qce, handle, dist, m, n, k):
    A, B = synth.gemm_operands(m, n, k, dist, seed=100 + m)
    exact = oracle.cgemm(A, B)
    C, dec = run(qce, handle, A, B, m, n, k, mode="auto")
    C32, Ct = _fp32_refs(qce, handle, A, B, m, n, k)
    e_emul = oracle.rel_fro(C, exact)
    e_fp32 = min(oracle.rel_fro(C32, exact), oracle.rel_fro(Ct, exact))
    assert e_emul <= 2.0 * e_fp32, (dist, dec["mode_name"], e_emul, e_fp32)
    # the emulated value of the selected mode, to accumulation accuracy
    model = oracle.emulated_cgemm(A, B, dec["mode"], dec["sA"], dec["sB"])
    assert oracle.rel_fro(C, model) <= 4 * U * math.sqrt(k) + 1e-30


@pytest.mark.parametrize("mode", ["fp16x2", "fp16x2_scaled", "bf16x3", "fp32"])
def test_forced_modes_match_emulation_model(qce, handle, mode):
    m, n, k = 256, 192, 320
    A, B = synth.gemm_operands(m, n, k, "u", seed=3)
    C, dec = run(qce, handle, A, B, m, n, k, mode=mode)
    model = oracle.emulated_cgemm(A, B, dec["mode"], dec["sA"], dec["sB"])
    assert oracle.rel_fro(C, model) <= 4 * U * math.sqrt(k)
    assert oracle.rel_fro(C, oracle.cgemm(A, B)) < 1e-6


def test_scaled_equals_unscaled_on_prescaled_inputs(qce, handle):
    # FP16X2_SCALED(A, B) == 2^-(sA+sB) FP16X2(A 2^sA, B 2^sB), bit for bit
    m, n, k = 130, 140, 150
    A, B = synth.gemm_operands(m, n, k, "a", seed=8)
    A = (A * np.float32(2.0 ** -30)).astype(np.complex64)
    C1, dec = run(qce, handle, A, B, m, n, k, mode="fp16x2_scaled")
    sA, sB = dec["sA"], dec["sB"]
    As = (A.astype(np.complex128) * 2.0 ** sA).astype(np.complex64)
    Bs = (B.astype(np.complex128) * 2.0 ** sB).astype(np.complex64)
    C2, _ = run(qce, handle, As, Bs, m, n, k, mode="fp16x2")
    assert np.array_equal(C1, (C2.astype(np.complex128) * 2.0 ** -(sA + sB)).astype(np.complex64))


def test_power_of_two_invariance_auto(qce, handle):
    # both calls select FP16X2_SCALED and shift to the same operands, so the
    # results differ by exactly the power of two
    m, n, k = 140, 100, 90
    A, B = synth.gemm_operands(m, n, k, "a", seed=12)
    A1 = (A * np.float32(2.0 ** -20)).astype(np.complex64)
    B1 = (B * np.float32(2.0 ** -19)).astype(np.complex64)
    A2 = (A * np.float32(2.0 ** -27)).astype(np.complex64)
    B2 = (B * np.float32(2.0 ** -25)).astype(np.complex64)
    C1, d1 = run(qce, handle, A1, B1, m, n, k, mode="auto")
    C2, d2 = run(qce, handle, A2, B2, m, n, k, mode="auto")
    assert d1["mode"] == d2["mode"] == oracle.MODE_FP16X2_SCALED
    assert np.array_equal(C2.astype(np.complex128) * 2.0 ** 13, C1.astype(np.complex128))


def test_nonfinite_forces_fp32_and_propagates(qce, handle):
    m, n, k = 64, 48, 40
    A, B = synth.gemm_operands(m, n, k, "a", seed=4)
    A[3, 5] = np.complex64(complex(np.inf, 0))
    C, dec = run(qce, handle, A, B, m, n, k, mode="auto")
    assert dec["mode"] == oracle.MODE_FP32 and dec["nonfinite"][0] == 1
    assert not np.isfinite(C[3, :]).all()
    assert np.isfinite(np.delete(C, 3, axis=0)).all()


def test_split_kernel_bit_exact(qce, handle):
    rng = np.random.default_rng(21)
    vals = np.concatenate([
        rng.standard_normal(5000), rng.uniform(-1, 1, 5000) * 2.0 ** -14,
        np.exp2(rng.uniform(-40, 10, 5000)), [1 + 2 ** -11, 1 + 3 * 2 ** -11, 2 ** -14, 0.0, -0.0],
    ]).astype(np.float32)
    x = np.empty(len(vals) // 2, dtype=np.complex64)
    x.real = vals[: len(x)]
    x.imag = vals[len(x): 2 * len(x)]
    t = torch.from_numpy(x).to("cuda")
    for shift in (0, 5, -3):
        planes = qce.split(handle, "fp16x2", shift, t).cpu().numpy().view(np.uint16)
        hr, lr = oracle.split_fp16x2(x.real, shift)
        hi_, li = oracle.split_fp16x2(x.imag, shift)
        for p, ref in enumerate((hr, lr, hi_, li)):
            assert np.array_equal(planes[p], ref.view(np.uint16)), (shift, p)
    planes = qce.split(handle, "bf16x3", 0, t).cpu().numpy().view(np.uint16)
    refs = list(oracle.split_bf16x3(x.real)) + list(oracle.split_bf16x3(x.imag))
    for p, ref in enumerate(refs):
        assert np.array_equal(planes[p], ref), p


def test_expstats_exact(qce, handle):
    rng = np.random.default_rng(6)
    rows, cols, ld = 300, 70, 310
    M = synth.random_matrix(ld, cols, "c", rng)
    M[5, 3] = np.complex64(complex(1e-45, 3e-39))   # FP32 subnormals
    M[7, 9] = np.complex64(complex(np.nan, 1.0))
    t = dev(M)
    got = qce.expstats(handle, t, rows, cols, ld)
    ref = oracle.exp_stats(M[:rows, :])
    for key in ("nnz", "n1", "n2", "n3", "nonfinite", "emax"):
        assert got[key] == ref[key], key
    # contiguous path with a subnormal maximum
    tiny = np.full((64, 3), np.complex64(complex(3e-40, -1e-42)), order="F")
    got = qce.expstats(handle, dev(tiny), 64, 3, 64)
    ref = oracle.exp_stats(tiny)
    assert got["emax"] == ref["emax"] == -132 and got["n2"] == ref["n2"]


IRREGULAR = [(1, 1, 5), (1, 1, 100000), (100000, 2, 2), (2, 70000, 2), (300, 400, 3),
             (31, 500, 600), (500, 31, 600), (64, 64, 15), (1, 300, 4000), (5, 7, 3),
             (33, 5, 16), (31, 3000, 16), (4000, 1000, 1), (32, 9, 17)]


@pytest.mark.parametrize("m,n,k", IRREGULAR)
@pytest.mark.parametrize("mode", ["auto", "fp16x2", "fp32"])
def test_irregular_shapes_integer_exact(qce, handle, m, n, k, mode):
    rng = np.random.default_rng(m + 3 * n + 7 * k)
    A = synth.random_matrix(m, k, "int", rng)
    B = synth.random_matrix(k, n, "int", rng)
    C, dec = run(qce, handle, A, B, m, n, k, mode=mode)
    assert np.array_equal(C.astype(np.complex128), oracle.cgemm(A, B))
    assert dec["mode"] == oracle.MODE_FP32 and dec["stats_taken"] == 0


@pytest.mark.parametrize("opA,opB", [("T", "N"), ("C", "T"), ("N", "C")])
def test_irregular_ops_alpha_beta(qce, handle, opA, opB):
    m, n, k = 3, 2, 50000          # small output, long k: split over k
    rng = np.random.default_rng(11)
    sa, sb = shapes_of(m, n, k, opA, opB)
    A = synth.random_matrix(*sa, "int", rng)
    B = synth.random_matrix(*sb, "int", rng)
    C0 = synth.random_matrix(m, n, "int", rng)
    C, _ = run(qce, handle, A, B, m, n, k, opA, opB, alpha=complex(1, 2), beta=complex(0, -1), C0=C0)
    want = oracle.cgemm(A, B, opA, opB, alpha=complex(1, 2), beta=complex(0, -1), C0=C0)
    assert np.array_equal(C.astype(np.complex128), want)


@pytest.mark.parametrize("opA,opB", [("T", "N"), ("C", "T"), ("N", "C")])
@pytest.mark.parametrize("m,n,k", [(300, 7, 9), (7, 300, 9), (257, 300, 2)])
def test_short_k_ops_alpha_beta(qce, handle, opA, opB, m, n, k):
    # short k: row-tile and column-tile kernels, every operand layout
    rng = np.random.default_rng(m + n + k)
    sa, sb = shapes_of(m, n, k, opA, opB)
    A = synth.random_matrix(*sa, "int", rng)
    B = synth.random_matrix(*sb, "int", rng)
    C0 = synth.random_matrix(m, n, "int", rng)
    C, _ = run(qce, handle, A, B, m, n, k, opA, opB, alpha=complex(-1, 2), beta=complex(1, 1), C0=C0)
    want = oracle.cgemm(A, B, opA, opB, alpha=complex(-1, 2), beta=complex(1, 1), C0=C0)
    assert np.array_equal(C.astype(np.complex128), want)


@pytest.mark.parametrize("beta", [complex(-1, 1), 0j])
@pytest.mark.parametrize("shift", [0, 1])
@pytest.mark.parametrize("m,n,k", [(2, 5000, 2), (6, 3000, 8), (16, 777, 16), (30, 513, 10),
                                   (7, 300, 8), (6, 300, 5), (64, 300, 8), (1000, 5, 16), (34, 100, 3),
                                   (33, 70, 2), (3, 1000, 7), (8, 257, 16)])
def test_short_k_columns_alpha_beta(qce, handle, m, n, k, shift, beta):
    # short k: one output column per thread below 32 rows, one or two rows
    # per thread from 32.  Even sizes with the operands read whole and C
    # 16-byte aligned move two complex values per load and store; odd
    # sizes, or B and C one element off that alignment (shift), go element
    # by element; with beta = 0, up to 8 rows and C aligned, a block's
    # columns are staged in LDS and stored as one run.  Integer inputs:
    # exact either way.
    rng = np.random.default_rng(7 * m + n + k)
    A = synth.random_matrix(m, k, "int", rng)
    B = synth.random_matrix(k, n, "int", rng)
    C0 = synth.random_matrix(m, n, "int", rng)
    alpha = complex(2, -1)
    pad = torch.zeros(shift, dtype=torch.complex64, device="cuda")
    dB = torch.cat([pad, dev(B)])[shift:]
    dC = torch.cat([pad, dev(C0)])[shift:]
    assert (dB.data_ptr() % 16 == 0) == (shift == 0)
    handle.set_mode("auto")
    qce.cgemm(handle, "N", "N", m, n, k, dev(A), m, dB, k, dC, m, alpha, beta)
    torch.cuda.synchronize()
    want = oracle.cgemm(A, B, alpha=alpha, beta=beta, C0=C0)
    assert np.array_equal(host(dC, m, n).astype(np.complex128), want)


@pytest.mark.parametrize("opA", ["N", "T"])
@pytest.mark.parametrize("m,n,k", [(8, 1, 70000), (24, 1, 5000), (100, 1, 3000), (500, 31, 600)])
def test_long_k_thin_outputs_alpha_beta(qce, handle, opA, m, n, k):
    # long k, thin outputs (GEMV-like, as the root of a batched slice pass),
    # A stored both ways: integer inputs exact with alpha and beta
    rng = np.random.default_rng(m + n + k)
    sa, sb = shapes_of(m, n, k, opA, "N")
    A = synth.random_matrix(*sa, "int", rng)
    B = synth.random_matrix(*sb, "int", rng)
    C0 = synth.random_matrix(m, n, "int", rng)
    C, _ = run(qce, handle, A, B, m, n, k, opA, "N", alpha=complex(1, -1), beta=complex(2, 0), C0=C0)
    want = oracle.cgemm(A, B, opA, "N", alpha=complex(1, -1), beta=complex(2, 0), C0=C0)
    assert np.array_equal(C.astype(np.complex128), want)


@pytest.mark.parametrize("opA,opB", [("N", "N"), ("T", "C"), ("C", "T")])
@pytest.mark.parametrize("m,n,k", [(1, 1, 1024), (2, 3, 5000), (4, 4, 262144), (8, 8, 1 << 20), (16, 16, 70000),
                                   (32, 8, 65536), (8, 32, 4096), (24, 5, 3000), (7, 13, 100000), (4, 64, 70000),
                                   (64, 4, 5000), (3, 40, 3000), (50, 2, 2000), (1, 8, 5000), (6, 2, 3000)])
def test_small_output_long_k_alpha_beta(qce, handle, opA, opB, m, n, k):
    # outputs of up to four 8 x 8, 4 x 16 or 16 x 4 tiles with a long k:
    # each thread adds a whole tile over its own k-values, then the lanes,
    # waves and k ranges are added up; with and without a split of k, rows
    # and columns of a tile past the output, every operand layout; integer
    # inputs exact
    rng = np.random.default_rng(m + 5 * n + k)
    sa, sb = shapes_of(m, n, k, opA, opB)
    A = synth.random_matrix(*sa, "int", rng)
    B = synth.random_matrix(*sb, "int", rng)
    C0 = synth.random_matrix(m, n, "int", rng)
    C, _ = run(qce, handle, A, B, m, n, k, opA, opB, alpha=complex(1, -1), beta=complex(-2, 1), C0=C0)
    want = oracle.cgemm(A, B, opA, opB, alpha=complex(1, -1), beta=complex(-2, 1), C0=C0)
    assert np.array_equal(C.astype(np.complex128), want)


@pytest.mark.parametrize("opB", ["T", "C"])
@pytest.mark.parametrize("m,n,k", [(8, 8, 1 << 20), (2, 4, 5000), (7, 5, 70000), (16, 16, 70000), (24, 7, 3000),
                                   (1, 1, 4096), (4, 64, 70000), (3, 40, 3000), (50, 2, 2000), (16, 16, 1 << 20),
                                   (5, 7, 1 << 20), (24, 3, 1 << 20)])
def test_small_output_long_k_paired_loads(qce, handle, opB, m, n, k):
    # the same kernel with op(A) = A and op(B) = B^T or B^H stored with even
    # leading dimensions (rows padded to an even count): a k-value's values
    # are read two at a time, and an odd m or n ends in a single value; from
    # k = 2^20 the 8 x 8 tiles take four lanes per k-value
    rng = np.random.default_rng(3 * m + n + k)
    A = synth.random_matrix(m + m % 2, k, "int", rng)
    B = synth.random_matrix(n + n % 2, k, "int", rng)
    C0 = synth.random_matrix(m, n, "int", rng)
    C, _ = run(qce, handle, A, B, m, n, k, "N", opB, alpha=complex(0, 1), beta=complex(1, 1), C0=C0)
    want = oracle.cgemm(A[:m], B[:n], "N", opB, alpha=complex(0, 1), beta=complex(1, 1), C0=C0)
    assert np.array_equal(C.astype(np.complex128), want)


@pytest.mark.parametrize("m,n,k", [(1, 1, 1 << 22), (20000, 3, 5), (8, 9, 300000), (8, 8, 1 << 22),
                                   (16, 16, 1 << 20)])
def test_irregular_float_accuracy(qce, handle, m, n, k):
    A, B = synth.gemm_operands(m, n, k, "a", seed=31)
    exact = oracle.cgemm(A, B)
    C, _ = run(qce, handle, A, B, m, n, k, mode="auto")
    tA = torch.from_numpy(np.ascontiguousarray(A)).to("cuda")
    tB = torch.from_numpy(np.ascontiguousarray(B)).to("cuda")
    Ct = torch.matmul(tA, tB).cpu().numpy()
    e = oracle.rel_fro(C, exact)
    assert e <= max(2 * oracle.rel_fro(Ct, exact), 4 * U * math.sqrt(k))


@pytest.mark.parametrize("mode", ["auto", "fp16x2", "fp16x2_scaled", "bf16x3", "fp32"])
@pytest.mark.parametrize("m,n,k", [(200, 150, 5000), (256, 256, 8192), (130, 1000, 3000)])
def test_split_k_integer_exact(qce, handle, mode, m, n, k):
    # few output tiles and a long k: the k range is split over workgroups
    rng = np.random.default_rng(m + n + k)
    A = synth.random_matrix(m, k, "int", rng)
    B = synth.random_matrix(k, n, "int", rng)
    C0 = synth.random_matrix(m, n, "int", rng)
    C, _ = run(qce, handle, A, B, m, n, k, alpha=complex(1, -1), beta=complex(2, 0), C0=C0, mode=mode)
    want = oracle.cgemm(A, B, alpha=complex(1, -1), beta=complex(2, 0), C0=C0)
    assert np.array_equal(C.astype(np.complex128), want)


@pytest.mark.parametrize("dist", ["a", "b", "c"])
def test_split_k_float_accuracy(qce, handle, dist):
    m, n, k = 300, 200, 20000
    A, B = synth.gemm_operands(m, n, k, dist, seed=77)
    A = (A * np.float32(2.0 ** -20)).astype(np.complex64)   # scaled mode for dist a
    exact = oracle.cgemm(A, B)
    C, dec = run(qce, handle, A, B, m, n, k, mode="auto")
    C32, Ct = _fp32_refs(qce, handle, A, B, m, n, k)
    e_fp32 = min(oracle.rel_fro(C32, exact), oracle.rel_fro(Ct, exact))
    assert oracle.rel_fro(C, exact) <= 2.0 * e_fp32, (dec["mode_name"],)
