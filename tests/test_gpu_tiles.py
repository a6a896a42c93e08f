"""GPU parity of the 64 x 64 tile of the panel GEMM (the tile the tuned
table picks for outputs too small to occupy the device), through the C-ABI:
integer inputs exact against the FP64 oracle in every mode and op pair,
ragged tails, split-k, batched entries; and, where k is not split, the same
bits as the 128 x 128 tile on float inputs (each output's k-sum runs chunk
by chunk in the same order)."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def qce():
    import paper_2303_08989_amd as q
    return q


@pytest.fixture(scope="module")
def h(qce):
    hh = qce.Handle(0)
    yield hh
    hh.set_gemm_tile(0)
    hh.close()


def dev(a):
    return torch.from_numpy(np.asfortranarray(a).ravel(order="F").copy()).to("cuda")


def host(t, rows, cols):
    return t.cpu().numpy().reshape((cols, rows)).T


def shapes_of(m, n, k, opA, opB):
    return ((m, k) if opA == "N" else (k, m)), ((k, n) if opB == "N" else (n, k))


def run(qce, h, A, B, m, n, k, tile, mode, opA="N", opB="N", alpha=1.0, beta=0.0, C0=None):
    h.set_mode(mode)
    h.set_gemm_tile(tile)
    dC = dev(C0) if C0 is not None else torch.zeros(m * n, dtype=torch.complex64, device="cuda")
    qce.cgemm(h, opA, opB, m, n, k, dev(A), A.shape[0], dev(B), B.shape[0], dC, m, alpha, beta)
    torch.cuda.synchronize()
    h.set_gemm_tile(0)
    return host(dC, m, n), h.last_decision()


MODES = ["fp16x2", "fp16x2_scaled", "bf16x3", "fp32", "auto"]


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("m,n,k", [(200, 150, 70), (64, 64, 200), (130, 97, 300), (512, 512, 512), (100, 300, 4000)])
def test_tile64_integer_exact(qce, h, mode, m, n, k):
    rng = np.random.default_rng(m + 2 * n + 3 * k)
    A = synth.random_matrix(m, k, "int", rng)
    B = synth.random_matrix(k, n, "int", rng)
    C0 = synth.random_matrix(m, n, "int", rng)
    C, _ = run(qce, h, A, B, m, n, k, 64, mode, alpha=complex(1, 1), beta=complex(0, -2), C0=C0)
    want = oracle.cgemm(A, B, alpha=complex(1, 1), beta=complex(0, -2), C0=C0)
    assert np.array_equal(C.astype(np.complex128), want)


@pytest.mark.parametrize("opA,opB", [("T", "N"), ("C", "T"), ("N", "C")])
@pytest.mark.parametrize("mode", ["fp16x2", "bf16x3", "fp32"])
def test_tile64_ops_exact(qce, h, opA, opB, mode):
    m, n, k = 150, 170, 90
    rng = np.random.default_rng(4)
    sa, sb = shapes_of(m, n, k, opA, opB)
    A = synth.random_matrix(*sa, "int", rng)
    B = synth.random_matrix(*sb, "int", rng)
    C, _ = run(qce, h, A, B, m, n, k, 64, mode, opA, opB)
    assert np.array_equal(C.astype(np.complex128), oracle.cgemm(A, B, opA, opB))


@pytest.mark.parametrize("dist", ["a", "b", "c"])
@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("m,n,k", [(300, 200, 100), (700, 260, 33), (1024, 1024, 256)])
def test_tile64_equals_tile128_bits(qce, h, dist, mode, m, n, k):
    # no k split at these sizes for either tile: identical sums
    rng = np.random.default_rng(7 + m)
    A = synth.random_matrix(m, k, dist, rng)
    B = synth.random_matrix(k, n, dist, rng)
    C64, d64 = run(qce, h, A, B, m, n, k, 64, mode)
    C128, d128 = run(qce, h, A, B, m, n, k, 128, mode)
    assert d64 == d128
    assert np.array_equal(np.ascontiguousarray(C64).view(np.uint32),
                          np.ascontiguousarray(C128).view(np.uint32)), (dist, mode)


def test_tile64_batched_entries(qce, h):
    m, n, k, batch = 96, 80, 200, 6
    rng = np.random.default_rng(9)
    A = [synth.random_matrix(m, k, "int", rng) for _ in range(batch)]
    B = [synth.random_matrix(k, n, "int", rng) for _ in range(batch)]
    dA = torch.cat([dev(a) for a in A])
    dB = torch.cat([dev(b) for b in B])
    dC = torch.zeros(batch * m * n, dtype=torch.complex64, device="cuda")
    h.set_mode("auto")
    h.set_gemm_tile(64)
    qce.cgemm_strided_batched(h, "N", "N", m, n, k, dA, m, m * k, dB, k, k * n, dC, m, m * n, batch)
    torch.cuda.synchronize()
    h.set_gemm_tile(0)
    out = dC.cpu().numpy()
    for z in range(batch):
        Cz = out[z * m * n:(z + 1) * m * n].reshape((n, m)).T
        assert np.array_equal(Cz.astype(np.complex128), oracle.cgemm(A[z], B[z])), z


def test_tile_argument_errors(qce, h):
    with pytest.raises(qce.QceError):
        h.set_gemm_tile(96)
