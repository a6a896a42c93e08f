"""GPU parity of the strided batched CGEMM (one launch per phase, entry in
blockIdx.z, per-entry device-side mode selection) through the C-ABI:
integer inputs bit-exact against the FP64 oracle, float entries bit-equal
to the same GEMM run alone (same kernels, same per-entry decision), and
per-entry decisions equal to the oracle's rule."""
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
    hh.close()


def shapes_of(m, n, k, opA, opB):
    sa = (m, k) if opA == "N" else (k, m)
    sb = (k, n) if opB == "N" else (n, k)
    return sa, sb


def pack(mats, stride):
    """column-major matrices -> one flat device buffer, entry z at z*stride"""
    buf = np.zeros(stride * (len(mats) - 1) + mats[-1].size, dtype=np.complex64)
    for z, a in enumerate(mats):
        flat = np.asfortranarray(a).ravel(order="F")
        buf[z * stride:z * stride + flat.size] = flat
    return torch.from_numpy(buf).to("cuda")


def unpack(t, z, stride, rows, cols, ld):
    flat = t.cpu().numpy()[z * stride:]
    out = np.empty((rows, cols), dtype=np.complex64, order="F")
    for j in range(cols):
        out[:, j] = flat[j * ld:j * ld + rows]
    return out


def run_batched(qce, h, As, Bs, m, n, k, opA="N", opB="N", alpha=1.0, beta=0.0, C0s=None,
                mode="auto", share_a=False, pad=0):
    h.set_mode(mode)
    sa, sb = shapes_of(m, n, k, opA, opB)
    lda, ldb, ldc = sa[0], sb[0], m + pad
    strideA = 0 if share_a else sa[0] * sa[1] + 3
    strideB = sb[0] * sb[1] + 5
    strideC = ldc * n + 7
    batch = len(Bs)
    dA = pack(As[:1] if share_a else As, max(strideA, 1))
    dB = pack(Bs, strideB)
    if C0s is None:
        dC = torch.zeros(strideC * batch, dtype=torch.complex64, device="cuda")
    else:
        padded = [np.vstack([c, np.zeros((pad, n), np.complex64)]) for c in C0s]
        dC = pack(padded, strideC)
        dC = torch.cat([dC, torch.zeros(strideC * batch - dC.numel(), dtype=torch.complex64, device="cuda")])
    qce.cgemm_strided_batched(h, opA, opB, m, n, k, dA, lda, strideA, dB, ldb, strideB, dC, ldc, strideC,
                              batch, alpha, beta)
    torch.cuda.synchronize()
    out = [unpack(dC, z, strideC, m, n, ldc) for z in range(batch)]
    decs = [h.batch_decision(z) for z in range(batch)]
    h.set_mode("auto")
    return out, decs


def run_single(qce, h, A, B, m, n, k, opA="N", opB="N", mode="auto"):
    h.set_mode(mode)
    sa, sb = shapes_of(m, n, k, opA, opB)
    dA = torch.from_numpy(np.asfortranarray(A).ravel(order="F").copy()).to("cuda")
    dB = torch.from_numpy(np.asfortranarray(B).ravel(order="F").copy()).to("cuda")
    dC = torch.zeros(m * n, dtype=torch.complex64, device="cuda")
    qce.cgemm(h, opA, opB, m, n, k, dA, sa[0], dB, sb[0], dC, m)
    torch.cuda.synchronize()
    h.set_mode("auto")
    return unpack(dC, 0, 0, m, n, m)


@pytest.mark.parametrize("mode", ["auto", "fp16x2", "fp16x2_scaled", "bf16x3", "fp32"])
@pytest.mark.parametrize("m,n,k", [(200, 150, 96), (130, 100, 3000), (40, 3000, 5), (5, 7, 300), (8, 1, 20000),
                                   (16, 16, 5000)])
def test_integer_exact(qce, h, mode, m, n, k):
    # regular tiles, split-k (few tiles, long k), short k, and dot-like
    # irregular shapes with a split k (one and four tiles of outputs)
    rng = np.random.default_rng(m + n + k)
    batch = 3
    As = [synth.random_matrix(m, k, "int", rng) for _ in range(batch)]
    Bs = [synth.random_matrix(k, n, "int", rng) for _ in range(batch)]
    out, _ = run_batched(qce, h, As, Bs, m, n, k, mode=mode)
    for z in range(batch):
        assert np.array_equal(out[z].astype(np.complex128), oracle.cgemm(As[z], Bs[z])), z


@pytest.mark.parametrize("m,n,k", [(6, 2000, 4), (5, 2000, 4), (64, 50, 4), (66, 9, 3), (33, 9, 3)])
def test_short_k_columns_even_strides(qce, h, m, n, k):
    # short k, entry strides that keep every entry's operands and C 16-byte
    # aligned (even m: two complex values per load and store, in the
    # column kernel below 32 rows and the row kernel from 32)
    rng = np.random.default_rng(m * n + k)
    batch = 3
    As = [synth.random_matrix(m, k, "int", rng) for _ in range(batch)]
    Bs = [synth.random_matrix(k, n, "int", rng) for _ in range(batch)]
    C0s = [synth.random_matrix(m, n, "int", rng) for _ in range(batch)]
    sA, sB, sC = m * k + 4, k * n + 2, m * n + 6
    dA, dB, dC = pack(As, sA), pack(Bs, sB), pack(C0s, sC)
    qce.cgemm_strided_batched(h, "N", "N", m, n, k, dA, m, sA, dB, k, sB, dC, m, sC, batch,
                              complex(0, 1), complex(1, -1))
    torch.cuda.synchronize()
    for z in range(batch):
        want = oracle.cgemm(As[z], Bs[z], alpha=complex(0, 1), beta=complex(1, -1), C0=C0s[z])
        assert np.array_equal(unpack(dC, z, sC, m, n, m).astype(np.complex128), want), z


@pytest.mark.parametrize("opA,opB", [("T", "N"), ("C", "T"), ("N", "C")])
def test_ops_alpha_beta_shared_a(qce, h, opA, opB):
    m, n, k = 160, 140, 80
    rng = np.random.default_rng(3)
    sa, sb = shapes_of(m, n, k, opA, opB)
    A = synth.random_matrix(*sa, "int", rng)
    Bs = [synth.random_matrix(*sb, "int", rng) for _ in range(4)]
    C0s = [synth.random_matrix(m, n, "int", rng) for _ in range(4)]
    out, _ = run_batched(qce, h, [A], Bs, m, n, k, opA, opB, alpha=complex(1, -2), beta=complex(0, 1),
                         C0s=C0s, share_a=True, pad=3)
    for z in range(4):
        want = oracle.cgemm(A, Bs[z], opA, opB, alpha=complex(1, -2), beta=complex(0, 1), C0=C0s[z])
        assert np.array_equal(out[z].astype(np.complex128), want), z


def test_per_entry_decisions_and_bits(qce, h):
    # entries of different distributions take different modes in one launch;
    # each entry equals the same GEMM run alone, bit for bit
    m, n, k = 192, 160, 128
    dists = ["a", "b", "c", "a", "u"]
    ops = [synth.gemm_operands(m, n, k, d, seed=40 + i) for i, d in enumerate(dists)]
    As, Bs = [o[0] for o in ops], [o[1] for o in ops]
    out, decs = run_batched(qce, h, As, Bs, m, n, k, mode="auto")
    for z in range(len(dists)):
        mode, s_a, s_b = oracle.select_mode(oracle.exp_stats(As[z]), oracle.exp_stats(Bs[z]), 0.1, 0.0)
        assert (decs[z]["mode"], decs[z]["sA"], decs[z]["sB"]) == (mode, s_a, s_b), z
        single = run_single(qce, h, As[z], Bs[z], m, n, k)
        assert np.array_equal(out[z], single), z
    assert len({d["mode"] for d in decs}) >= 3


def test_batch_of_one_and_zero(qce, h):
    m, n, k = 64, 64, 64
    A, B = synth.gemm_operands(m, n, k, "a", seed=9)
    out, _ = run_batched(qce, h, [A], [B], m, n, k)
    assert np.array_equal(out[0], run_single(qce, h, A, B, m, n, k))
    d = torch.zeros(8, dtype=torch.complex64, device="cuda")
    qce.cgemm_strided_batched(h, "N", "N", 4, 4, 4, d, 4, 0, d, 4, 0, d, 4, 16, 0)


def test_errors(qce, h):
    d = torch.zeros(64, dtype=torch.complex64, device="cuda")
    with pytest.raises(qce.QceError):
        qce.cgemm_strided_batched(h, "N", "N", 4, 4, 4, d, 4, 16, d, 4, 16, d, 4, 15, 2)   # C overlap
    with pytest.raises(qce.QceError):
        qce.cgemm_strided_batched(h, "N", "N", 4, 4, 4, d, 4, -1, d, 4, 16, d, 4, 16, 2)   # stride
    with pytest.raises(qce.QceError):
        qce.cgemm_strided_batched(h, "N", "N", 4, 4, 4, d, 4, 0, d, 4, 0, d, 4, 16, 70000)  # batch
    with pytest.raises(qce.QceError):
        h.batch_decision(5)
