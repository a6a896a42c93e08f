"""GPU parity of the TTGT contraction path (permute -> emulated CGEMM ->
permute), the FP64 reductions and circuit amplitudes, through the C-ABI,
against the FP64 oracle."""
import math

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


def rounded(circuit):
    out = dict(circuit)
    out["gates"] = [dict(g, matrix=np.asarray(g["matrix"]).astype(np.complex64).astype(np.complex128))
                    for g in circuit["gates"]]
    return out


@pytest.mark.parametrize("seed", range(8))
def test_permute_exact(qce, h, seed):
    rng = np.random.default_rng(seed)
    rank = int(rng.integers(1, 7))
    shape = tuple(int(x) for x in rng.integers(1, 5, rank))
    x = (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)).astype(np.complex64)
    perm = [int(p) for p in rng.permutation(rank)]
    y = qce.permute(h, torch.from_numpy(x).to("cuda"), perm).cpu().numpy()
    assert np.array_equal(y, np.transpose(x, perm))


def test_permute_rank20_pow2(qce, h):
    rng = np.random.default_rng(1)
    shape = (2,) * 20
    x = (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)).astype(np.complex64)
    perm = [int(p) for p in rng.permutation(20)]
    y = qce.permute(h, torch.from_numpy(x).to("cuda"), perm).cpu().numpy()
    assert np.array_equal(y, np.transpose(x, perm))


@pytest.mark.parametrize("seed", range(10))
def test_permute_pow2_tiled(qce, h, seed):
    # power-of-two extents: the tiled bit-permutation path (2^8 .. 2^22
    # elements), including permutations that keep the lowest bits in place
    rng = np.random.default_rng(100 + seed)
    n_bits = int(rng.integers(8, 23))
    exts = []
    while sum(exts) < n_bits:
        exts.append(int(min(rng.integers(1, 5), n_bits - sum(exts))))
    shape = tuple(1 << e for e in exts)
    x = (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)).astype(np.complex64)
    rank = len(shape)
    perm = [int(p) for p in rng.permutation(rank)]
    if seed % 3 == 0 and rank > 1:            # innermost axis stays innermost
        perm = [p for p in perm if p != rank - 1] + [rank - 1]
    y = qce.permute(h, torch.from_numpy(x).to("cuda"), perm).cpu().numpy()
    assert np.array_equal(y, np.transpose(x, perm))


def test_permute_rank28_bits(qce, h):
    # a 2^24-element tensor with every extent 2 and a random axis order, as
    # the circuit intermediates
    rng = np.random.default_rng(5)
    shape = (2,) * 24
    x = (np.arange(1 << 24, dtype=np.float32) + 1j * np.float32(0.5)).astype(np.complex64).reshape(shape)
    perm = [int(p) for p in rng.permutation(24)]
    y = qce.permute(h, torch.from_numpy(x).to("cuda"), perm).cpu().numpy()
    assert np.array_equal(y, np.transpose(x, perm))


@pytest.mark.parametrize("mode", ["fp32", "auto_emulated", "fp16x2", "bf16x3"])
@pytest.mark.parametrize("seed", range(6))
def test_contract_integer_exact(qce, h, mode, seed):
    net = synth.random_network(seed, n_contracted=1 + seed % 3, n_free_a=1 + seed % 2,
                               n_free_b=2 - seed % 2, max_extent=5, dist="int",
                               shuffle_output=True)
    if mode == "auto_emulated":
        h.set_mode("auto")
        h.set_size_policy(0, 0)      # statistics + selection on every GEMM
    else:
        h.set_mode(mode)
    try:
        C = qce.contract(h, torch.from_numpy(net["A"]).to("cuda"), net["la"],
                         torch.from_numpy(net["B"]).to("cuda"), net["lb"], net["lc"]).cpu().numpy()
    finally:
        h.set_size_policy(*h.default_size_policy)
        h.set_mode("auto")
    want = oracle.zcontract(net["A"], net["la"], net["B"], net["lb"], net["lc"])
    assert np.array_equal(C.astype(np.complex128), want)


def _bits_network(rng, nk, nfa, nfb, ints, natural_out=True, swapped_out=False):
    """Every extent 2; K and free labels interleaved at random in A and B.
    Output order: B's free labels then A's (the GEMM's own order), A's then
    B's (swapped_out: the GEMM runs with the operands' roles exchanged), or
    a random order (natural_out False: an output permute)."""
    K = list(range(nk))
    FA = list(range(100, 100 + nfa))
    FB = list(range(200, 200 + nfb))
    la = [int(v) for v in rng.permutation(K + FA)]
    lb = [int(v) for v in rng.permutation(K + FB)]
    lc = [v for v in lb if v in FB] + [v for v in la if v in FA]
    if swapped_out:
        lc = [v for v in la if v in FA] + [v for v in lb if v in FB]
    if not natural_out:
        lc = [int(v) for v in rng.permutation(lc)]

    def t(r):
        if ints:
            return (rng.integers(-3, 4, (2,) * r) + 1j * rng.integers(-3, 4, (2,) * r)).astype(np.complex64)
        return (rng.standard_normal((2,) * r) + 1j * rng.standard_normal((2,) * r)).astype(np.complex64)
    return t(len(la)), la, t(len(lb)), lb, lc


def _contract_counted(qce, hh, A, la, B, lb, lc, mode):
    if mode == "auto_emulated":
        hh.set_mode("auto")
        hh.set_size_policy(0, 0)
    else:
        hh.set_mode(mode)
    hh.set_timing(True)
    hh.reset_timing()
    try:
        C = qce.contract(hh, torch.from_numpy(A).to("cuda"), la, torch.from_numpy(B).to("cuda"), lb, lc)
        t = hh.timing()
        dec = hh.last_decision()
    finally:
        hh.set_timing(False)
        hh.set_size_policy(*hh.default_size_policy)
        hh.set_mode("auto")
    return C.cpu().numpy(), t["permute"][1], dec


@pytest.fixture(scope="module")
def h_unfused(qce):
    import os
    old = os.environ.get("QCE_FUSED_GATHER")
    os.environ["QCE_FUSED_GATHER"] = "0"
    try:
        hh = qce.Handle(0)
    finally:
        if old is None:
            del os.environ["QCE_FUSED_GATHER"]
        else:
            os.environ["QCE_FUSED_GATHER"] = old
    yield hh
    hh.close()


@pytest.mark.parametrize("mode", ["fp32", "auto_emulated", "fp16x2", "bf16x3"])
@pytest.mark.parametrize("seed", range(6))
def test_contract_fused_gather_integer_exact(qce, h, h_unfused, mode, seed):
    # interleaved K and free labels (every extent 2): the split reads each
    # operand through its bit permutation (no permute launched when every
    # label lies in the split's 64 x 64 tile); exact, and equal to the
    # permute-then-split path
    rng = np.random.default_rng(300 + seed)
    nk, nfa, nfb = 4 + seed % 3, 5 + seed % 2, 6 - seed % 2
    A, la, B, lb, lc = _bits_network(rng, nk, nfa, nfb, ints=True, swapped_out=seed >= 4)
    want = oracle.zcontract(A, la, B, lb, lc)
    got, n_perm, _ = _contract_counted(qce, h, A, la, B, lb, lc, mode)
    assert np.array_equal(got.astype(np.complex128), want)
    assert n_perm == 0
    ref, n_perm_ref, _ = _contract_counted(qce, h_unfused, A, la, B, lb, lc, mode)
    assert n_perm_ref >= 1
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("mode", ["fp32", "auto_emulated", "bf16x3"])
@pytest.mark.parametrize("seed", range(4))
def test_contract_fused_gather_many_tiles(qce, h, h_unfused, mode, seed):
    # more labels than the tile holds (several 64 x 64 tiles per operand,
    # tile bases from the high bits), float inputs: both paths against the
    # FP64 oracle, and the same device decision (the statistics of a tensor
    # do not depend on its element order)
    rng = np.random.default_rng(400 + seed)
    nk, nfa, nfb = 7 + seed % 3, 8 + seed % 2, 9 - seed % 2
    A, la, B, lb, lc = _bits_network(rng, nk, nfa, nfb, ints=False, natural_out=seed % 2 == 0)
    want = oracle.zcontract(A, la, B, lb, lc)
    got, _, dec = _contract_counted(qce, h, A, la, B, lb, lc, mode)
    ref, _, dec_ref = _contract_counted(qce, h_unfused, A, la, B, lb, lc, mode)
    bound = 2e-6 if mode in ("fp32", "bf16x3") else 4e-6
    assert oracle.rel_fro(got, want) < bound
    assert oracle.rel_fro(ref, want) < bound
    assert (dec["mode"], dec["sA"], dec["sB"]) == (dec_ref["mode"], dec_ref["sA"], dec_ref["sB"])


@pytest.mark.parametrize("rank", [8, 11, 16, 22, 26])
def test_contract_full_permuted_dot(qce, h, h_unfused, rank):
    # every label summed, the two operands in different label orders: one
    # pass reads one operand through its bit permutation (no permute
    # launched).  Integer inputs: exact, equal to the permute-then-dot path;
    # float inputs: FP32 accuracy against the FP64 oracle.
    rng = np.random.default_rng(500 + rank)
    la = list(range(rank))
    lb = [int(v) for v in rng.permutation(rank)]
    while lb == la:
        lb = [int(v) for v in rng.permutation(rank)]
    # integer sums stay exact in FP32 up to rank 22; rank 26 (the size of
    # the last step of a 53-qubit slice) checks floats only
    for ints in ((True, False) if rank <= 22 else (False,)):
        if ints:
            A = (rng.integers(-3, 4, (2,) * rank) + 1j * rng.integers(-3, 4, (2,) * rank)).astype(np.complex64)
            B = (rng.integers(-3, 4, (2,) * rank) + 1j * rng.integers(-3, 4, (2,) * rank)).astype(np.complex64)
        else:
            A = (rng.standard_normal((2,) * rank) + 1j * rng.standard_normal((2,) * rank)).astype(np.complex64)
            B = (rng.standard_normal((2,) * rank) + 1j * rng.standard_normal((2,) * rank)).astype(np.complex64)
        want = oracle.zcontract(A, la, B, lb, [])
        got, n_perm, dec = _contract_counted(qce, h, A, la, B, lb, [], "auto")
        ref, n_perm_ref, _ = _contract_counted(qce, h_unfused, A, la, B, lb, [], "auto")
        assert dec["mode"] == oracle.MODE_FP32
        assert n_perm == 0 and n_perm_ref == 1
        if ints:
            assert complex(got) == complex(want) == complex(ref)
        else:
            scale = float(np.sum(np.abs(A.astype(np.complex128)) * np.abs(np.transpose(B, np.argsort(lb)))))
            assert abs(complex(got) - complex(want)) <= 4 * rank * 2.0 ** -24 * scale
            assert abs(complex(ref) - complex(want)) <= 4 * rank * 2.0 ** -24 * scale


@pytest.mark.parametrize("layout", ["natural", "swapped", "interleaved", "scalar", "outer"])
def test_contract_layouts_float(qce, h, layout):
    rng = np.random.default_rng(7)
    ext = {0: 3, 1: 4, 2: 5, 3: 2, 4: 6}
    if layout == "scalar":
        la, lb, lc = [0, 1], [1, 0], []
    elif layout == "outer":
        la, lb, lc = [0, 1], [2], [2, 0, 1]
    else:
        la, lb = [2, 0, 1], [3, 1, 4, 2]
        lc = {"natural": [3, 4, 0], "swapped": [0, 3, 4], "interleaved": [3, 0, 4]}[layout]

    def t(ls):
        shape = tuple(ext[x] for x in ls)
        return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)).astype(np.complex64)
    A, B = t(la), t(lb)
    h.set_mode("fp32")
    C = qce.contract(h, torch.from_numpy(A).to("cuda"), la, torch.from_numpy(B).to("cuda"), lb, lc)
    h.set_mode("auto")
    want = oracle.zcontract(A, la, B, lb, lc)
    assert oracle.rel_fro(C.cpu().numpy(), want) < 1e-6


def test_contract_errors(qce, h):
    a = torch.zeros((2, 2), dtype=torch.complex64, device="cuda")
    with pytest.raises(qce.QceError) as e:
        qce.contract(h, a, [0, 3], a, [1, 2], [1, 2])        # trace over one input
    assert e.value.status == 2
    b = torch.zeros((2, 3), dtype=torch.complex64, device="cuda")
    with pytest.raises(qce.QceError) as e:
        qce.contract(h, a, [0, 1], b, [2, 1], [0, 2])        # label 1: extent 2 vs 3
    assert e.value.status == 1


def test_accumulate_f64_exact(qce, h):
    vals = np.array([1e8 + 1j, 3.25 - 2j, -1e8 + 0.5j, 1e-3 + 1e-3j], dtype=np.complex64)
    acc = torch.zeros(2, dtype=torch.float64, device="cuda")
    src = torch.from_numpy(vals).to("cuda")
    for i in range(len(vals)):
        qce.accumulate_f64(h, src[i:i + 1], acc)
    re = im = 0.0
    for v in vals:
        re += float(v.real)
        im += float(v.imag)
    got = acc.cpu().numpy()
    assert got[0] == re and got[1] == im


def test_fidelity_terms(qce, h):
    rng = np.random.default_rng(3)
    a = (rng.standard_normal(10000) + 1j * rng.standard_normal(10000)).astype(np.complex64)
    b = (a + 1e-3 * rng.standard_normal(10000)).astype(np.complex64)
    out = qce.fidelity_terms(h, torch.from_numpy(a).to("cuda"), torch.from_numpy(b).to("cuda")).cpu().numpy()
    a64, b64 = a.astype(np.complex128), b.astype(np.complex128)
    ov = np.vdot(b64, a64)
    assert abs(out[0] - ov.real) <= 1e-12 * abs(ov) and abs(out[1] - ov.imag) <= 1e-12 * abs(ov)
    assert out[2] == pytest.approx(np.vdot(a64, a64).real, rel=1e-13)
    assert out[3] == pytest.approx(np.vdot(b64, b64).real, rel=1e-13)
    fid = (out[0] ** 2 + out[1] ** 2) / (out[2] * out[3])
    assert fid == pytest.approx(oracle.fidelity(a, b), rel=1e-12)


# --- circuits ------------------------------------------------------------

def _amplitudes(qce, h, circuit, xs, max_log2=30, mode="fp32", slice_ids=None, varied=6, policy=None):
    from paper_2303_08989_amd.executor import CircuitPlan, Executor
    plan = CircuitPlan(circuit, max_log2=max_log2, restarts=2, varied=varied)
    h.set_mode(mode)
    if policy:
        h.set_size_policy(*policy)
    try:
        ex = Executor(h, plan)
        out = []
        for x in xs:
            acc = ex.amplitude(x, slice_ids)
            v = acc.cpu().numpy()
            out.append(complex(v[0], v[1]))
    finally:
        h.set_size_policy(*h.default_size_policy)
        h.set_mode("auto")
    return np.array(out), plan


def test_config1_amplitudes_fp32(qce, h):
    # 12-qubit 3x4 grid, depth 8, ABCD layering, plain FP32 path
    c = synth.grid_circuit(3, 4, 8, seed=0)
    xs = synth.random_bitstrings(12, 10, seed=1)
    got, plan = _amplitudes(qce, h, c, xs)
    want = oracle.statevector_amplitudes(rounded(c), xs)
    assert oracle.fidelity(got, want) >= 1 - 1e-6
    assert np.max(np.abs(got - want) / np.abs(want)) < 1e-4
    tn_want = np.array([oracle.tn_amplitude(rounded(c), x) for x in xs[:3]])
    assert np.max(np.abs(got[:3] - tn_want)) < 1e-6 * np.max(np.abs(tn_want)) * 100


def test_executor_grouped_levels_match_path_order(qce, h):
    # a sliced 20-qubit network: the slices' recomputed steps run level by
    # level with small contractions grouped, or one by one in path order;
    # both against the FP64 state vector and each other, every slice value
    from paper_2303_08989_amd.executor import CircuitPlan, Executor
    c = synth.grid_circuit(4, 5, 10, seed=4, pattern="ABCDCDAB")
    plan = CircuitPlan(c, max_log2=12, restarts=2, varied=4)
    assert len(plan.sliced) >= 2
    xs = synth.random_bitstrings(20, 3, seed=8)
    ex = Executor(h, plan)
    ids = range(min(plan.n_slices, 16))
    h.set_mode("fp32")
    try:
        for x in xs:
            v = {}
            for grouped in (True, False):
                out = torch.empty(len(ids), dtype=torch.complex64, device="cuda")
                ex.amplitude(x, ids, slice_out=out, grouped=grouped)
                v[grouped] = out.cpu().numpy().astype(np.complex128)
            scale = np.max(np.abs(v[False]))
            assert np.max(np.abs(v[True] - v[False])) <= 1e-5 * scale
    finally:
        h.set_mode("auto")
    got = []
    for x in xs:
        got.append(complex(*Executor(h, plan).amplitude(x).cpu().numpy()))
    want = oracle.statevector_amplitudes(rounded(c), xs)
    assert oracle.fidelity(np.array(got), want) >= 1 - 1e-6


def test_ghz_and_identity_closed_forms(qce, h):
    n = 8
    got, _ = _amplitudes(qce, h, synth.ghz_circuit(n), [0, (1 << n) - 1, 5])
    assert abs(got[0] - 1 / math.sqrt(2)) < 1e-6 and abs(got[1] - 1 / math.sqrt(2)) < 1e-6
    assert abs(got[2]) < 1e-7
    got, _ = _amplitudes(qce, h, synth.identity_circuit(6, seed=3), [0, 9])
    assert abs(got[0] - 1) < 1e-6 and abs(got[1]) < 1e-6


def test_sliced_amplitude_all_slices(qce, h):
    c = synth.grid_circuit(3, 4, 8, seed=2, pattern="ABCDCDAB")
    x = 1234
    got, plan = _amplitudes(qce, h, c, [x], max_log2=5, varied=3)
    assert len(plan.sliced) >= 2
    want = oracle.statevector_amplitudes(rounded(c), [x])[0]
    assert abs(got[0] - want) < 1e-6 * max(abs(want), 1e-3)


def test_emulated_amplitudes_auto_everywhere(qce, h):
    # every GEMM through statistics + selection (size policy thresholds 0)
    c = synth.grid_circuit(3, 4, 8, seed=5, pattern="ABCDCDAB")
    xs = synth.random_bitstrings(12, 6, seed=2)
    got, _ = _amplitudes(qce, h, c, xs, mode="auto", policy=(0, 0))
    want = oracle.statevector_amplitudes(rounded(c), xs)
    assert oracle.fidelity(got, want) >= 1 - 1e-6


def test_reduced_config3_sliced(qce, h):
    # the 53-qubit generator at reduced size: 4x5 grid, depth 12, ABCDCDAB,
    # sliced, AUTO with the paper's size policy
    c = synth.grid_circuit(4, 5, 12, seed=1, pattern="ABCDCDAB")
    xs = synth.random_bitstrings(20, 2, seed=3)
    got, plan = _amplitudes(qce, h, c, xs, max_log2=12, mode="auto", varied=4)
    assert len(plan.sliced) >= 1
    want = oracle.statevector_amplitudes(rounded(c), xs)
    assert oracle.fidelity(got, want) >= 1 - 1e-6


# --- batch labels (in both inputs and the output) ------------------------

def _batch_case(rng, ext, la, lb, lc):
    def t(ls):
        shape = tuple(ext[x] for x in ls)
        n = int(np.prod(shape)) if shape else 1
        return synth.random_matrix(1, n, "int", rng).reshape(shape)
    return t(la), t(lb)


BATCH_CASES = [
    # (extents, la, lb, lc)
    ({0: 3, 1: 40, 2: 48, 3: 36}, [0, 1, 2], [0, 2, 3], [0, 3, 1]),          # batch in front everywhere
    ({0: 3, 1: 40, 2: 48, 3: 36}, [1, 0, 2], [2, 3, 0], [3, 0, 1]),          # batch in the middle: permutes
    ({0: 2, 5: 3, 1: 64, 2: 64, 3: 64}, [5, 0, 1, 2], [0, 5, 2, 3], [0, 5, 3, 1]),  # two batch labels
    ({0: 4, 1: 2, 2: 2, 3: 2}, [0, 1, 2], [0, 2, 3], [1, 0, 3]),             # irregular entries
    ({0: 5, 1: 33, 3: 40}, [0, 1], [0, 3], [0, 1, 3]),                       # no summed label
    ({0: 7, 2: 300}, [0, 2], [2, 0], [0]),                                   # batched dot products
]


@pytest.mark.parametrize("mode", ["fp32", "auto_emulated", "fp16x2", "bf16x3"])
@pytest.mark.parametrize("case", range(len(BATCH_CASES)))
def test_contract_batch_labels_integer_exact(qce, h, mode, case):
    ext, la, lb, lc = BATCH_CASES[case]
    rng = np.random.default_rng(50 + case)
    A, B = _batch_case(rng, ext, la, lb, lc)
    if mode == "auto_emulated":
        h.set_mode("auto")
        h.set_size_policy(0, 0)
    else:
        h.set_mode(mode)
    try:
        C = qce.contract(h, torch.from_numpy(A).to("cuda"), la, torch.from_numpy(B).to("cuda"), lb, lc)
        C = C.cpu().numpy()
    finally:
        h.set_size_policy(*h.default_size_policy)
        h.set_mode("auto")
    assert np.array_equal(C.astype(np.complex128), oracle.zcontract(A, la, B, lb, lc))


def test_contract_batch_more_than_one_launch(qce, h):
    # 2^17 batch entries (more than one launch of at most 65535)
    rng = np.random.default_rng(8)
    nb = 17
    bl = list(range(10, 10 + nb))
    ext = {x: 2 for x in bl}
    ext.update({0: 2, 1: 2, 2: 2})
    la, lb, lc = bl + [0, 1], bl + [1, 2], bl + [0, 2]
    A, B = _batch_case(rng, ext, la, lb, lc)
    C = qce.contract(h, torch.from_numpy(A).to("cuda"), la, torch.from_numpy(B).to("cuda"), lb, lc).cpu().numpy()
    want = np.matmul(A.reshape(-1, 2, 2).astype(np.complex128), B.reshape(-1, 2, 2).astype(np.complex128))
    assert np.array_equal(C.reshape(-1, 2, 2).astype(np.complex128), want)


def test_size_policy_default_and_roundtrip(qce, h):
    # AUTO from min(m, n, k) >= 512 by default (gfx950 calibration of the
    # Sec. 4.3 thresholds), settable and readable; invalid orders rejected
    fresh = qce.Handle(0)
    try:
        assert fresh.size_policy() == (512, 512) == fresh.default_size_policy
    finally:
        fresh.close()
    prev = h.size_policy()
    try:
        h.set_size_policy(2048, 512)
        assert h.size_policy() == (2048, 512)
        with pytest.raises(qce.QceError):
            h.set_size_policy(256, 512)
        assert h.size_policy() == (2048, 512)
    finally:
        h.set_size_policy(*prev)
