"""GPU parity on the 53-qubit network the benchmark runs (6 x 9 grid minus a
corner, depth 12, ABCDCDAB; the benchmark's plan parameters), through the
C-ABI contraction in AUTO mode with the size policy (Sec. 4.3):

* one slice contracted step by step; every contraction with k <= 2^20
  (all but the final full contraction) is checked on 16 x 16 sampled output
  entries against FP64 products the oracle computes from the same FP32
  inputs (gathered from the device), within the bound of the mode that ran:
  FP32 accumulation plus the split's representation error (Eq. 2 or the
  six BF16 products) and the FP16 underflow floor after scaling (Sec. 4.2);
* per-slice values of AUTO against the forced-FP32 path over 8 slices:
  fidelity (the reading in the oracle: |<b|a>|^2 / (<a|a><b|b>)) >= 1 - 1e-6.
"""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

U = 2.0 ** -24
NS_SIDE = 16          # sampled rows and columns per contraction (256 outputs)


@pytest.fixture(scope="module")
def qce():
    import paper_2303_08989_amd as q
    return q


@pytest.fixture(scope="module")
def h(qce):
    hh = qce.Handle(0)
    yield hh
    hh.close()


@pytest.fixture(scope="module")
def plan():
    from paper_2303_08989_amd.executor import CircuitPlan
    c = synth.grid_circuit(pattern="ABCDCDAB", depth=12, seed=1, **synth.GRID_53)
    return CircuitPlan(c, max_log2=28, restarts=8, varied=6)


def _offsets(labels, sub, idx):
    """Flat offsets, in a row-major tensor whose axes are the extent-2
    ``labels``, of the indices ``idx`` over the labels ``sub`` (sub[0] the
    most significant bit)."""
    r = len(labels)
    stride = {lab: 1 << (r - 1 - i) for i, lab in enumerate(labels)}
    idx = np.asarray(idx, dtype=np.int64)
    off = np.zeros(idx.shape, dtype=np.int64)
    for t, lab in enumerate(sub):
        off += ((idx >> (len(sub) - 1 - t)) & 1) * stride[lab]
    return off


def _gather(T, offs):
    return T.reshape(-1)[torch.from_numpy(offs).to(T.device)].cpu().numpy()


def _bound(mode, kk, S, sum_a, sum_b, s_min):
    """Per-entry error bound of one sampled output (see the module doc)."""
    acc = 2.0 * (kk / 2 + 8) * U * S
    if mode == oracle.MODE_FP32:
        return acc
    if mode == oracle.MODE_BF16X3:
        return acc + 4.0 * U * S
    # FP16X2 (scaled or not): relative 2^-22 per part, the dropped residual
    # product, and residuals below FP16's normal range after the shift
    return acc + 2.0 ** -20 * S + 2.0 ** (-36 - s_min) * (sum_a + sum_b)


def test_config3_slice_gemms_sampled(qce, h, plan):
    # every contraction of the slice up to k = 2^20 (long split-k steps
    # included) on 16 sampled rows x 16 sampled columns; a final full
    # contraction of two 2^28-element tensors (the fused permuted dot) has
    # its own oracle test at 2^26 elements in tests/test_gpu_contract.py
    from paper_2303_08989_amd import tn
    c = plan.circuit
    x = synth.random_bitstrings(53, 1, seed=5)[0]
    S = set(plan.sliced)
    leaves = tn.circuit_network(c, x)
    vals = {}
    for i, (arr, labels) in enumerate(leaves):
        sub = tn.fix_labels(arr, labels, {lab: 0 for lab in labels if lab in S})
        vals[i] = (torch.from_numpy(sub).to("cuda"), [lab for lab in labels if lab not in S])
    L = len(leaves)
    h.set_mode("auto")
    h.set_tolerance(0.1, 0.0)
    rng = np.random.default_rng(11)
    checked = {}
    longest_k = 0
    for s, (a, b) in enumerate(plan.path):
        A, la = vals.pop(a)
        B, lb = vals.pop(b)
        shared = set(la) & set(lb)
        lc = [lab for lab in lb if lab not in shared] + [lab for lab in la if lab not in shared]
        C = qce.contract(h, A, la, B, lb, lc)
        vals[L + s] = (C, lc)
        K = [lab for lab in la if lab in shared]
        fa = [lab for lab in la if lab not in shared]
        fb = [lab for lab in lb if lab not in shared]
        mA, nB, kk = 2 ** len(fa), 2 ** len(fb), 2 ** len(K)
        if kk > 2 ** 20:
            continue
        torch.cuda.synchronize()
        if min(mA, nB) < 32 or kk < 16:
            mode, sA, sB, name = oracle.MODE_FP32, 0, 0, "fp32"   # bandwidth-bound kernels
        else:
            d = h.last_decision()
            mode, sA, sB, name = d["mode"], d["sA"], d["sB"], d["mode_name"]
        rows = rng.choice(mA, min(mA, NS_SIDE), replace=False)
        cols = rng.choice(nB, min(nB, NS_SIDE), replace=False)
        q = np.arange(kk)
        a_s = _gather(A, _offsets(la, fa, rows)[:, None] + _offsets(la, K, q)[None, :])
        b_s = _gather(B, _offsets(lb, fb, cols)[:, None] + _offsets(lb, K, q)[None, :])
        got = _gather(C, _offsets(lc, fa, rows)[:, None] + _offsets(lc, fb, cols)[None, :])
        got = got.astype(np.complex128)
        exact = oracle.cgemm(a_s, np.asfortranarray(b_s.T))
        abs_a = np.abs(a_s.real).astype(np.float64) + np.abs(a_s.imag)
        abs_b = np.abs(b_s.real).astype(np.float64) + np.abs(b_s.imag)
        Ssum = abs_a @ abs_b.T
        s_min = min(sA, sB, 0) if mode == oracle.MODE_FP16X2_SCALED else 0
        bound = _bound(mode, kk, Ssum, abs_a.sum(axis=1)[:, None], abs_b.sum(axis=1)[None, :], s_min)
        err = np.abs(got - exact)
        assert np.all(err <= bound), (s, name, kk, float(np.max(err / np.maximum(bound, 1e-300))))
        den = np.sqrt(np.sum(np.abs(exact) ** 2))
        if den > 0:
            assert np.sqrt(np.sum(err ** 2)) / den <= 1e-5, (s, name)
        checked[name] = checked.get(name, 0) + 1
        longest_k = max(longest_k, kk)
    print("checked contractions by mode:", checked, "longest k:", longest_k, flush=True)
    # the big GEMMs of a slice take the emulated modes
    assert checked.get("bf16x3", 0) + checked.get("fp16x2", 0) + checked.get("fp16x2_scaled", 0) >= 1
    assert sum(checked.values()) == sum(1 for (_, _, k2) in plan.gemm_shapes if k2 <= 20)
    assert longest_k == 2 ** max(k2 for (_, _, k2) in plan.gemm_shapes if k2 <= 20)


def test_config3_auto_vs_fp32_fidelity(qce, h, plan):
    from paper_2303_08989_amd.executor import Executor
    x = synth.random_bitstrings(53, 1, seed=5)[0]
    ids = range(8)
    vecs = {}
    for mode in ("auto", "fp32"):
        h.set_mode(mode)
        h.set_tolerance(0.1, 0.0)
        vec = torch.empty(len(ids), dtype=torch.complex64, device="cuda")
        Executor(h, plan).amplitude(x, ids, slice_out=vec)
        torch.cuda.synchronize()
        vecs[mode] = vec.cpu().numpy().astype(np.complex128)
    h.set_mode("auto")
    a, b = vecs["auto"], vecs["fp32"]
    assert np.all(np.abs(b) > 0)
    assert oracle.fidelity(a, b) >= 1 - 1e-6
    assert np.max(np.abs(a - b) / np.abs(b)) <= 1e-4
