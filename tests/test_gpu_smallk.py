"""GPU parity of the short-k, narrow-output GEMM (k <= 128, n <= 64), which
splits its operands as it loads them instead of writing panels: against
the FP64 oracle (integer inputs exact in every mode, every op pair, alpha
and beta, batched entries), and bit for bit against the panel path on the
same inputs (the same fragments meet the same MFMA sequence), which a
handle created with QCE_SMALLK=0 still runs."""
import os

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
def handles(qce):
    h = qce.Handle(0)
    saved = os.environ.get("QCE_SMALLK")
    os.environ["QCE_SMALLK"] = "0"
    try:
        hp = qce.Handle(0)
    finally:
        if saved is None:
            os.environ.pop("QCE_SMALLK", None)
        else:
            os.environ["QCE_SMALLK"] = saved
    yield h, hp
    h.close()
    hp.close()


def dev(a):
    return torch.from_numpy(np.asfortranarray(a).ravel(order="F").copy()).to("cuda")


def host(t, rows, cols):
    return t.cpu().numpy().reshape((cols, rows)).T


def shapes_of(m, n, k, opA, opB):
    return ((m, k) if opA == "N" else (k, m)), ((k, n) if opB == "N" else (n, k))


def run(qce, h, A, B, m, n, k, opA="N", opB="N", mode="auto", alpha=1.0, beta=0.0, C0=None):
    h.set_mode(mode)
    dC = dev(C0) if C0 is not None else torch.zeros(m * n, dtype=torch.complex64, device="cuda")
    qce.cgemm(h, opA, opB, m, n, k, dev(A), A.shape[0], dev(B), B.shape[0], dC, m, alpha, beta)
    torch.cuda.synchronize()
    return host(dC, m, n), h.last_decision()


MODES = ["fp16x2", "fp16x2_scaled", "bf16x3", "fp32", "auto"]
SHAPES = [(300, 64, 64), (1000, 40, 100), (130, 33, 17), (4000, 64, 128), (257, 50, 31)]


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("m,n,k", SHAPES)
def test_integer_exact(qce, handles, mode, m, n, k):
    h, _ = handles
    rng = np.random.default_rng(m + n + k)
    A = synth.random_matrix(m, k, "int", rng)
    B = synth.random_matrix(k, n, "int", rng)
    C, _ = run(qce, h, A, B, m, n, k, mode=mode)
    assert np.array_equal(C.astype(np.complex128), oracle.cgemm(A, B))


@pytest.mark.parametrize("opA,opB", [("N", "N"), ("T", "N"), ("C", "N"), ("N", "T"), ("N", "C"), ("C", "C")])
@pytest.mark.parametrize("mode", ["fp16x2", "bf16x3", "fp32", "auto"])
def test_ops_alpha_beta_exact(qce, handles, opA, opB, mode):
    h, _ = handles
    m, n, k = 333, 57, 45
    rng = np.random.default_rng(17)
    sa, sb = shapes_of(m, n, k, opA, opB)
    A = synth.random_matrix(*sa, "int", rng)
    B = synth.random_matrix(*sb, "int", rng)
    C0 = synth.random_matrix(m, n, "int", rng)
    alpha, beta = complex(1, -2), complex(-1, 0.5)
    C, _ = run(qce, h, A, B, m, n, k, opA, opB, mode=mode, alpha=alpha, beta=beta, C0=C0)
    want = oracle.cgemm(A, B, opA, opB, alpha=alpha, beta=beta, C0=C0)
    assert np.array_equal(C.astype(np.complex128), want)


@pytest.mark.parametrize("dist", ["a", "b", "c", "u"])
@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("m,n,k,opA,opB", [(2000, 64, 64, "N", "N"), (513, 48, 100, "T", "C"), (640, 33, 128, "N", "T")])
def test_bit_equal_to_panel_path(qce, handles, dist, mode, m, n, k, opA, opB):
    h, hp = handles
    rng = np.random.default_rng(len(dist) + m)
    sa, sb = shapes_of(m, n, k, opA, opB)
    A = synth.random_matrix(*sa, dist, rng)
    B = synth.random_matrix(*sb, dist, rng)
    if dist == "a" and mode in ("auto", "fp16x2_scaled"):
        A = (A * np.float32(2.0 ** -20)).astype(np.complex64)     # exercise the shifts
    C0 = synth.random_matrix(m, n, "a", rng)
    beta = complex(0.5, -0.25)
    C1, d1 = run(qce, h, A, B, m, n, k, opA, opB, mode=mode, beta=beta, C0=C0)
    C2, d2 = run(qce, hp, A, B, m, n, k, opA, opB, mode=mode, beta=beta, C0=C0)
    assert d1 == d2
    assert np.array_equal(np.ascontiguousarray(C1).view(np.uint32), np.ascontiguousarray(C2).view(np.uint32)), \
        (dist, mode, d1["mode_name"])
    # the value of the mode that ran, to accumulation accuracy; and, where the
    # mode suits the data (AUTO's choice, or a wide-range mode), the exact product
    opa = A if opA == "N" else (A.T if opA == "T" else A.conj().T)
    opb = B if opB == "N" else (B.T if opB == "T" else B.conj().T)
    model = oracle.emulated_cgemm(np.asarray(opa), np.asarray(opb), d1["mode"], d1["sA"], d1["sB"])
    model = model + beta * C0.astype(np.complex128)
    assert oracle.rel_fro(C1, model) <= 4 * 2.0 ** -24 * np.sqrt(k)
    if mode in ("auto", "bf16x3", "fp32"):
        assert oracle.rel_fro(C1, oracle.cgemm(A, B, opA, opB, beta=beta, C0=C0)) < 1e-5


def test_batched_entries_exact(qce, handles):
    h, _ = handles
    m, n, k, batch = 260, 64, 80, 5
    rng = np.random.default_rng(3)
    A = [synth.random_matrix(m, k, "int", rng) for _ in range(batch)]
    B = [synth.random_matrix(k, n, "int", rng) for _ in range(batch)]
    dA = torch.cat([dev(a) for a in A])
    dB = torch.cat([dev(b) for b in B])
    dC = torch.zeros(batch * m * n, dtype=torch.complex64, device="cuda")
    h.set_mode("auto")
    qce.cgemm_strided_batched(h, "N", "N", m, n, k, dA, m, m * k, dB, k, k * n, dC, m, m * n, batch)
    torch.cuda.synchronize()
    out = dC.cpu().numpy()
    for z in range(batch):
        Cz = out[z * m * n:(z + 1) * m * n].reshape((n, m)).T
        assert np.array_equal(Cz.astype(np.complex128), oracle.cgemm(A[z], B[z])), z
        assert h.batch_decision(z)["mode"] == oracle.MODE_FP16X2
