"""The paper's exploratory random tensor network (Sec. 5.2): 10 nodes with 2
to 4 legs of dimension 32 (reduced from 128), element types 1-3, contracted
pairwise; every GEMM of the chain is run in every mode on the same FP32
inputs and compared with the FP64 oracle of those inputs.

Reading: a closed network of type-2/3 magnitudes underflows FP32 after a few
contractions in any mode, so the chain's intermediates are rescaled by a
power of two (exact) to the type's element scale before the next step; each
GEMM then sees inputs of its type.  The checks restate the paper's findings:
AUTO-t selects a mode that avoids underflow and stays at FP32 accuracy, plain
FP16 loses type 2 and 3 to underflow, FP16 with scaling loses type 3."""
import math

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

DIM = 32
U = 2.0 ** -24
TYPE_RMS = {1: 1e-2, 2: 1e-8, 3: 1e-8}
MODES = [("fp32", None), ("fp16x2", None), ("fp16x2_scaled", None), ("bf16x3", None),
         ("auto", 0.0), ("auto", 0.1), ("auto", 0.5)]


@pytest.fixture(scope="module")
def qce():
    import paper_2303_08989_amd as q
    return q


@pytest.fixture(scope="module")
def h(qce):
    hh = qce.Handle(0)
    yield hh
    hh.close()


def _mat(T, labels, rows, cols):
    perm = [labels.index(x) for x in rows + cols]
    return np.ascontiguousarray(np.transpose(T, perm)).reshape(DIM ** len(rows), DIM ** len(cols))


def _oracle_step(A, la, B, lb, lc):
    K = [x for x in la if x in lb]
    FA = [x for x in la if x not in lb]
    FB = [x for x in lb if x not in la]
    Cm = oracle.cgemm(np.asfortranarray(_mat(A, la, FA, K)), np.asfortranarray(_mat(B, lb, K, FB)))
    C = Cm.reshape([DIM] * (len(FA) + len(FB)))
    tl = FA + FB
    return np.transpose(C, [tl.index(x) for x in lc])


@pytest.fixture(scope="module")
def results(qce, h):
    from paper_2303_08989_amd import tn
    out = {}
    try:
        for tn_type in synth.TN_TYPES:
            labels = synth.random_closed_network(7)
            rng = np.random.default_rng(100 + tn_type)
            tens = {i: (synth.random_tn_tensor((DIM,) * len(l), tn_type, rng), list(l))
                    for i, l in enumerate(labels)}
            L = len(labels)
            steps = []
            for s, (a, b) in enumerate(tn.greedy_path(labels)):
                A, la = tens.pop(a)
                B, lb = tens.pop(b)
                shared = set(la) & set(lb)
                lc = [x for x in lb if x not in shared] + [x for x in la if x not in shared]
                m = DIM ** sum(x not in shared for x in la)
                n = DIM ** sum(x not in shared for x in lb)
                k = DIM ** len(shared)
                C64 = _oracle_step(A, la, B, lb, lc)
                rec = {"regular": min(m, n) >= 32 and k >= 16}
                for mode, t in MODES:
                    h.set_mode(mode)
                    h.set_tolerance(0.1 if t is None else t, 0.0)
                    h.set_size_policy(0, 0)
                    C = qce.contract(h, torch.from_numpy(A).to("cuda"), la, torch.from_numpy(B).to("cuda"),
                                     lb, lc).cpu().numpy()
                    key = mode if t is None else f"auto-{t}"
                    rec[key] = (oracle.rel_fro(C, C64), h.last_decision()["mode"])
                steps.append(rec)
                rms = float(np.sqrt(np.mean(np.abs(C64) ** 2)))
                sc = 2.0 ** round(math.log2(TYPE_RMS[tn_type] / rms)) if rms > 0 else 1.0
                tens[L + s] = ((C64 * sc).astype(np.complex64), lc)
            out[tn_type] = steps
    finally:
        h.set_tolerance(0.1, 0.0)
        h.set_mode("auto")
        h.set_size_policy(*h.default_size_policy)
    return out


def _bound(rec):
    return max(2.0 * rec["fp32"][0], 4 * U)


@pytest.mark.parametrize("tn_type", [1, 2, 3])
def test_auto_modes_stay_at_fp32_accuracy(results, tn_type):
    regular = [r for r in results[tn_type] if r["regular"]]
    assert len(regular) >= 5
    for r in regular:
        for key in ("auto-0.0", "auto-0.1", "auto-0.5", "bf16x3"):
            assert r[key][0] <= _bound(r), (key, r[key], r["fp32"])


def test_type1_every_mode_accurate(results):
    for r in results[1]:
        if r["regular"]:
            assert r["fp16x2"][0] <= _bound(r) and r["fp16x2_scaled"][0] <= _bound(r)
            assert r["auto-0.1"][1] == oracle.MODE_FP16X2


def test_type2_plain_fp16_underflows_scaling_recovers(results):
    for r in results[2]:
        if r["regular"]:
            assert r["fp16x2"][0] > 0.5                       # inputs below FP16's range
            assert r["fp16x2_scaled"][0] <= _bound(r)
            for key in ("auto-0.0", "auto-0.1", "auto-0.5"):
                assert r[key][1] == oracle.MODE_FP16X2_SCALED


def test_type3_needs_the_wide_exponent_modes(results):
    regular = [r for r in results[3] if r["regular"]]
    assert sum(r["fp16x2"][0] > 1e-4 for r in regular) >= len(regular) // 2
    assert any(r["fp16x2_scaled"][0] > _bound(r) for r in regular)   # scaling is not enough
    for r in regular:
        assert r["auto-0.1"][1] in (oracle.MODE_BF16X3, oracle.MODE_FP32)
