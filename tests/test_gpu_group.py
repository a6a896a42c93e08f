"""GPU: grouped small contractions (qce_group_begin / qce_group_end): many
independent small contractions in one launch, against the FP64 oracle;
larger contractions inside a group run at once and stay correct."""
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


def _case(rng, ext, la, lb):
    def t(ls):
        shape = tuple(ext[x] for x in ls)
        n = int(np.prod(shape)) if shape else 1
        return synth.random_matrix(1, n, "int", rng).reshape(shape)
    return t(la), t(lb)


CASES = [
    ({0: 2, 1: 2, 2: 2, 3: 2}, [0, 1, 2], [2, 3], [3, 0, 1]),                 # gate-like, k = 2
    ({0: 8, 1: 4, 2: 3}, [0, 1], [1, 2], [2, 0]),                              # tiny GEMM
    ({0: 5, 1: 7}, [0, 1], [1, 0], []),                                        # full contraction
    ({0: 3, 1: 4}, [0], [1], [1, 0]),                                          # outer product
    ({0: 4, 1: 2, 2: 3, 5: 2}, [5, 0, 1], [1, 5, 2], [5, 2, 0]),              # batch label 5
    ({0: 2, 1: 2, 2: 2, 3: 2, 4: 2, 6: 2, 7: 2}, [7, 0, 1, 2, 3], [3, 2, 4, 6], [6, 7, 4, 0, 1]),
    ({0: 600, 1: 3, 2: 5}, [0, 1], [1, 2], [0, 2]),                            # tall, k = 3
    ({0: 40, 1: 1000, 2: 9}, [0, 1], [1, 2], [2, 0]),                          # k = 1000 (limit 1024)
]


def test_group_exact_against_oracle(qce, h):
    rng = np.random.default_rng(17)
    data = [_case(rng, *c[:3]) for c in CASES]
    outs = []
    with qce.group(h):
        for (ext, la, lb, lc), (A, B) in zip(CASES, data):
            outs.append(qce.contract(h, torch.from_numpy(A).to("cuda"), la, torch.from_numpy(B).to("cuda"), lb, lc))
    for (ext, la, lb, lc), (A, B), C in zip(CASES, data, outs):
        want = oracle.zcontract(A, la, B, lb, lc)
        assert np.array_equal(C.cpu().numpy().astype(np.complex128), want), (la, lb, lc)


def test_group_mixed_with_large_and_float(qce, h):
    # a large contraction inside the group runs at once; float data stays at
    # FP32 accuracy
    rng = np.random.default_rng(3)
    big = synth.random_network(1, 2, 2, 2, max_extent=12, dist="a", extents=[12, 11, 13, 10, 9, 8])
    small = []
    for i in range(30):
        ext = {0: 2, 1: 2, 2: 2, 3: 2}
        A = synth.random_matrix(1, 8, "a", rng).reshape(2, 2, 2)
        B = synth.random_matrix(1, 4, "a", rng).reshape(2, 2)
        small.append((A, B))
    with qce.group(h):
        Cb = qce.contract(h, torch.from_numpy(big["A"]).to("cuda"), big["la"], torch.from_numpy(big["B"]).to("cuda"),
                          big["lb"], big["lc"])
        Cs = [qce.contract(h, torch.from_numpy(A).to("cuda"), [0, 1, 2], torch.from_numpy(B).to("cuda"), [2, 3],
                           [3, 0, 1]) for A, B in small]
    wb = oracle.zcontract(big["A"], big["la"], big["B"], big["lb"], big["lc"])
    assert oracle.rel_fro(Cb.cpu().numpy(), wb) < 1e-6
    for (A, B), C in zip(small, Cs):
        w = oracle.zcontract(A, [0, 1, 2], B, [2, 3], [3, 0, 1])
        assert oracle.rel_fro(C.cpu().numpy(), w) < 1e-6


def test_group_errors(qce, h):
    hh = h._bind_stream()
    assert h.lib.qce_group_end(hh) == 1             # no group open
    assert h.lib.qce_group_begin(hh) == 0
    assert h.lib.qce_group_begin(hh) == 1           # already open
    assert h.lib.qce_group_reset(hh, 0) == 1        # reset with a group open
    assert h.lib.qce_group_end(hh) == 0
    qce.group_reset(h, 1 << 20)


def test_many_groups_reuse_the_descriptor_area(qce, h):
    # more descriptors over many groups than the area holds: it is reused
    rng = np.random.default_rng(5)
    A = synth.random_matrix(1, 16, "int", rng).reshape(2, 2, 2, 2)
    B = synth.random_matrix(1, 4, "int", rng).reshape(2, 2)
    dA, dB = torch.from_numpy(A).to("cuda"), torch.from_numpy(B).to("cuda")
    want = oracle.zcontract(A, [0, 1, 2, 3], B, [3, 4], [4, 0, 1, 2])
    last = None
    for g in range(400):
        with qce.group(h):
            outs = [qce.contract(h, dA, [0, 1, 2, 3], dB, [3, 4], [4, 0, 1, 2]) for _ in range(16)]
        last = outs
        if g % 97 == 0:
            for C in outs:
                assert np.array_equal(C.cpu().numpy().astype(np.complex128), want)
    for C in last:
        assert np.array_equal(C.cpu().numpy().astype(np.complex128), want)
