"""GPU parity at the benchmark's full sizes, in its launch configuration.

Shapes 8192 x 8192 x 8192 and 65536 x 64 x 64, column-major "N", "N"
operands generated exactly as the benchmark generates them, AUTO mode with
t = 0.1 through ``qce_cgemm_emulated``.  The oracle computes sampled
outputs one by one:

* the device's decision equals the closed form for each input distribution
  (complex Gaussian -> FP16X2; log-uniform over [2^-40, 1] -> BF16X3;
  [2^-120, 1] with zeros -> FP32), the Sec. 4.1 rule whose statistics the
  smaller tests pin against the oracle count for count;
* every sampled output lies within the FP32 accumulation bound of the
  oracle's value of the products the selected mode keeps (Eq. 2; the six
  BF16 products), and the sampled Frobenius distance to that value is at
  FP32 accumulation level, so a dropped or mis-signed term would show;
* the sampled error against the exact FP64 product is at most twice that
  of the plain FP32 path on the same inputs (the Eq. 3 gate), and where
  AUTO selects FP32 its result equals the forced FP32 run bit for bit;
* integer inputs give the exact product in every mode at 8192^3.
"""
import numpy as np
import pytest

import oracle
import synth
from synth.gemm_inputs import case_seed

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

U = 2.0 ** -24
NSAMPLES = 256
# (m, n, k, index of the shape in the benchmark's seed formula)
SHAPES = [(8192, 8192, 8192, 2), (65536, 64, 64, 3)]
EXPECTED = {"a": oracle.MODE_FP16X2, "b": oracle.MODE_BF16X3, "c": oracle.MODE_FP32}


@pytest.fixture(scope="module")
def qce():
    import paper_2303_08989_amd as q
    return q


@pytest.fixture(scope="module")
def h(qce):
    hh = qce.Handle(0)
    yield hh
    hh.close()


def _device(M):
    return torch.from_numpy(np.asfortranarray(M).ravel(order="F")).to("cuda")


def _run(qce, h, dA, dB, m, n, k, mode):
    h.set_mode(mode)
    h.set_tolerance(0.1, 0.0)
    dC = torch.empty(m * n, dtype=torch.complex64, device="cuda")
    qce.cgemm(h, "N", "N", m, n, k, dA, m, dB, k, dC, m)
    torch.cuda.synchronize()
    dec = h.last_decision()
    h.set_mode("auto")
    return dC, dec


def _sample(dC, m, ii, jj):
    idx = torch.from_numpy((ii + jj * m).astype(np.int64)).to("cuda")
    return dC[idx].cpu().numpy().astype(np.complex128)


def _rel_fro(x, ref):
    den = np.sqrt(np.sum(np.abs(ref) ** 2))
    return float(np.sqrt(np.sum(np.abs(x - ref) ** 2)) / den)


def _samples(m, n, seed):
    rng = np.random.default_rng(seed)
    return rng.integers(0, m, NSAMPLES), rng.integers(0, n, NSAMPLES)


@pytest.mark.parametrize("m,n,k,si", SHAPES)
@pytest.mark.parametrize("dist", ["a", "b", "c"])
def test_full_size_auto(qce, h, dist, m, n, k, si):
    print(f"full-size AUTO {m}x{n}x{k} dist {dist}", flush=True)
    A, B = synth.gemm_operands(m, n, k, dist, case_seed(dist, si, 0))
    dA, dB = _device(A), _device(B)
    dC, dec = _run(qce, h, dA, dB, m, n, k, "auto")
    assert dec["mode"] == EXPECTED[dist], dec
    assert dec["sA"] == 0 and dec["sB"] == 0
    ii, jj = _samples(m, n, 17 + si)
    got = _sample(dC, m, ii, jj)
    exact = np.array([oracle.cgemm(A[i:i + 1, :], B[:, j:j + 1])[0, 0] for i, j in zip(ii, jj)])
    model = np.array([oracle.emulated_cgemm(A[i:i + 1, :], B[:, j:j + 1], dec["mode"])[0, 0]
                      for i, j in zip(ii, jj)])
    # sum over l of |A_il| |B_lj| with |z| = |re| + |im|: bounds every partial sum
    absA = np.abs(A.real) + np.abs(A.imag)
    absB = np.abs(B.real) + np.abs(B.imag)
    S = np.array([float(absA[i, :].astype(np.float64) @ absB[:, j].astype(np.float64))
                  for i, j in zip(ii, jj)])
    # FP32 accumulation: at most one rounding per MFMA step (k/2 for the
    # FP32 instruction, k/16 for the f16/bf16 one) plus the epilogue
    bound = 2.0 * (k / 2 + 8) * U * S
    assert np.all(np.abs(got - model) <= bound)
    assert _rel_fro(got, model) <= 2e-5
    # the plain FP32 path on the same inputs
    dC32, dec32 = _run(qce, h, dA, dB, m, n, k, "fp32")
    assert dec32["mode"] == oracle.MODE_FP32
    got32 = _sample(dC32, m, ii, jj)
    e_mode, e_32 = _rel_fro(got, exact), _rel_fro(got32, exact)
    assert e_mode <= 2.0 * e_32, (e_mode, e_32)
    if EXPECTED[dist] == oracle.MODE_FP32:
        assert torch.equal(dC, dC32)
    del dA, dB, dC, dC32
    torch.cuda.empty_cache()


@pytest.fixture(scope="module")
def int_operands():
    return synth.gemm_operands(8192, 8192, 8192, "int", case_seed("int", 2, 0))


@pytest.mark.parametrize("mode", ["auto", "fp16x2", "fp16x2_scaled", "bf16x3", "fp32"])
def test_full_size_integer_exact(qce, h, int_operands, mode):
    print(f"full-size integer 8192^3 mode {mode}", flush=True)
    A, B = int_operands
    m = n = k = 8192
    dA, dB = _device(A), _device(B)
    dC, _ = _run(qce, h, dA, dB, m, n, k, mode)
    ii, jj = _samples(m, n, 5)
    got = _sample(dC, m, ii, jj)
    exact = np.array([oracle.cgemm(A[i:i + 1, :], B[:, j:j + 1])[0, 0] for i, j in zip(ii, jj)])
    assert np.array_equal(got, exact)
    del dA, dB, dC
    torch.cuda.empty_cache()
