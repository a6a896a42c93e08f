"""The size policy on the CGEMM entry points (Sec. 4.3: statistics only
above a size, the wide emulation or plain FP32 below it), switched on with
qce_set_gemm_size_policy: each shape runs in the mode the policy gives it,
with the same kernels as that mode called directly, so single and batched
calls are equal bit for bit (grouped entries to accumulation order); with
the switch off AUTO takes statistics on every shape."""
import ctypes

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def qce():
    import paper_2303_08989_amd as q
    return q


@pytest.fixture()
def h(qce):
    hh = qce.Handle(0)
    yield hh
    hh.close()


def operands(m, n, k, seed):
    A, B = synth.gemm_operands(m, n, k, "a", seed)
    dA = torch.from_numpy(np.asfortranarray(A).ravel(order="F").copy()).to("cuda")
    dB = torch.from_numpy(np.asfortranarray(B).ravel(order="F").copy()).to("cuda")
    return dA, dB


def call(qce, h, mode, m, n, k, dA, dB):
    h.set_mode(mode)
    C = torch.zeros(m * n, dtype=torch.complex64, device="cuda")
    qce.cgemm(h, "N", "N", m, n, k, dA, m, dB, k, C, m)
    torch.cuda.synchronize()
    return C, h.last_decision()


@pytest.mark.parametrize("m,n,k,policy,expect", [
    (8192, 64, 64, (512, 512), "fp32"),       # min dim 64 < emul_min: plain FP32
    (600, 520, 530, (512, 512), "auto"),      # min dim >= auto_min: statistics
    (600, 520, 530, (2048, 512), "bf16x3"),   # the paper's tiers: emulation without statistics
    (300, 200, 100, (2048, 512), "fp32"),
])
def test_policy_mode_and_bits(qce, h, m, n, k, policy, expect):
    dA, dB = operands(m, n, k, seed=m + n + k)
    h.set_size_policy(*policy)
    h.set_gemm_size_policy(True)
    C_pol, d_pol = call(qce, h, "auto", m, n, k, dA, dB)
    h.set_gemm_size_policy(False)
    if expect == "auto":
        assert d_pol["stats_taken"] == 1
        C_ref, d_ref = call(qce, h, "auto", m, n, k, dA, dB)
        assert d_ref["mode"] == d_pol["mode"]
    else:
        assert d_pol["stats_taken"] == 0 and d_pol["mode_name"] == expect
        C_ref, _ = call(qce, h, expect, m, n, k, dA, dB)
    assert torch.equal(C_pol.view(torch.int64), C_ref.view(torch.int64))
    # switched off: AUTO takes statistics on any shape
    _, d_off = call(qce, h, "auto", m, n, k, dA, dB)
    assert d_off["stats_taken"] == 1


def test_policy_in_batched_and_grouped(qce, h):
    h.set_size_policy(2048, 512)
    h.set_gemm_size_policy(True)
    h.set_mode("auto")
    m, n, k, batch = 520, 512, 512, 3
    dA, dB = operands(m, n, k * batch, seed=5)
    C = torch.zeros(m * n * batch, dtype=torch.complex64, device="cuda")
    qce.cgemm_strided_batched(h, "N", "N", m, n, k, dA, m, m * k, dB, k, k * n, C, m, m * n, batch)
    torch.cuda.synchronize()
    for z in range(batch):
        d = h.batch_decision(z)
        assert d["mode_name"] == "bf16x3" and d["stats_taken"] == 0
    h.set_mode("bf16x3")
    C2 = torch.zeros_like(C)
    qce.cgemm_strided_batched(h, "N", "N", m, n, k, dA, m, m * k, dB, k, k * n, C2, m, m * n, batch)
    torch.cuda.synchronize()
    assert torch.equal(C.view(torch.int64), C2.view(torch.int64))
    # grouped: one entry per tier
    h.set_mode("auto")
    shapes = [(2048, 2048, 2048), (600, 520, 530), (256, 64, 64)]
    bufs, descs = [], []
    for i, (mm, nn, kk) in enumerate(shapes):
        a, b = operands(mm, nn, kk, seed=20 + i)
        c = torch.zeros(mm * nn, dtype=torch.complex64, device="cuda")
        bufs.append((a, b, c))
        descs.append({"m": mm, "n": nn, "k": kk, "A": a, "lda": mm, "B": b, "ldb": kk, "C": c, "ldc": mm})
    qce.cgemm_grouped(h, descs)
    torch.cuda.synchronize()
    modes = [h.batch_decision(i) for i in range(len(shapes))]
    assert modes[0]["stats_taken"] == 1
    assert modes[1]["mode_name"] == "bf16x3" and modes[1]["stats_taken"] == 0
    assert modes[2]["mode_name"] == "fp32" and modes[2]["stats_taken"] == 0
    # the grouped launch runs its own tile and k-split plan (and the panel
    # path where a single call would take the short-k kernel), so it agrees
    # with a single call of the same mode to accumulation order, not bit
    # for bit
    for i, (mm, nn, kk) in enumerate(shapes[1:], start=1):
        a, b, c = bufs[i]
        ref, _ = call(qce, h, modes[i]["mode_name"], mm, nn, kk, a, b)
        err = torch.linalg.vector_norm(c - ref) / torch.linalg.vector_norm(ref)
        assert float(err) < 1e-5, (shapes[i], float(err))
    h.set_gemm_size_policy(False)


def test_policy_switch_errors(qce, h):
    from paper_2303_08989_amd import _lib
    lib = _lib.load()
    assert lib.qce_set_gemm_size_policy(h._h, 2) == 1        # INVALID_VALUE
    assert lib.qce_set_gemm_size_policy(None, 1) == 1
    assert lib.qce_set_gemm_size_policy(h._h, 1) == 0
    assert lib.qce_set_gemm_size_policy(h._h, 0) == 0
