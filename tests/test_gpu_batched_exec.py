"""GPU: batched slices (sliced labels kept as batch labels, one batched GEMM
per contraction step), the FP64 sum of a pass's slice values, and the pass
captured in a HIP graph and replayed per bitstring."""
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


def _rounded(c):
    out = dict(c)
    out["gates"] = [dict(g, matrix=np.asarray(g["matrix"]).astype(np.complex64).astype(np.complex128))
                    for g in c["gates"]]
    return out


def test_accumulate_n_f64(qce, h):
    ints = np.arange(-500, 1500, dtype=np.float32)
    src = torch.from_numpy((ints + 1j * (2 * ints)).astype(np.complex64)).to("cuda")
    acc = torch.tensor([0.5, -1.0], dtype=torch.float64, device="cuda")
    qce.accumulate_n_f64(h, src, acc)
    got = acc.cpu().numpy()
    assert got[0] == 0.5 + float(ints.sum()) and got[1] == -1.0 + 2 * float(ints.sum())
    rng = np.random.default_rng(2)
    v = (rng.standard_normal(1 << 20) + 1j * rng.standard_normal(1 << 20)).astype(np.complex64)
    acc = torch.zeros(2, dtype=torch.float64, device="cuda")
    qce.accumulate_n_f64(h, torch.from_numpy(v).to("cuda"), acc)
    ref = v.astype(np.complex128).sum()
    assert abs(complex(*acc.cpu().numpy()) - ref) < 1e-9


@pytest.mark.parametrize("n_batch", [2, 99])
@pytest.mark.parametrize("mode", ["fp32", "auto_emulated"])
def test_batched_equals_looped_and_oracle(qce, h, n_batch, mode):
    from paper_2303_08989_amd.executor import BatchedExecutor, CircuitPlan, Executor
    c = synth.grid_circuit(3, 4, 8, seed=2, pattern="ABCDCDAB")
    plan = CircuitPlan(c, max_log2=5, restarts=2, varied=3)
    assert len(plan.sliced) >= 3
    xs = synth.random_bitstrings(12, 4, seed=6)
    if mode == "auto_emulated":
        h.set_mode("auto")
        h.set_size_policy(0, 0)
    else:
        h.set_mode(mode)
    try:
        bx = BatchedExecutor(h, plan, n_batch)
        ex = Executor(h, plan)
        got = np.array([complex(*bx.amplitude(x).cpu().numpy()) for x in xs])
        loop = np.array([complex(*ex.amplitude(x).cpu().numpy()) for x in xs])
    finally:
        h.set_size_policy(*h.default_size_policy)
        h.set_mode("auto")
    want = oracle.statevector_amplitudes(_rounded(c), xs)
    assert oracle.fidelity(got, want) >= 1 - 1e-6
    assert np.max(np.abs(got - loop)) <= 1e-5 * np.max(np.abs(want))


def test_reduced_config3_batched_auto(qce, h):
    from paper_2303_08989_amd.executor import BatchedExecutor, CircuitPlan
    c = synth.grid_circuit(4, 5, 12, seed=1, pattern="ABCDCDAB")
    plan = CircuitPlan(c, max_log2=12, restarts=2, varied=4)
    xs = synth.random_bitstrings(20, 2, seed=3)
    bx = BatchedExecutor(h, plan, 8)
    assert bx.n_outer <= 64 and bx.max_intermediate() <= 22
    got = np.array([complex(*bx.amplitude(x).cpu().numpy()) for x in xs])
    want = oracle.statevector_amplitudes(_rounded(c), xs)
    assert oracle.fidelity(got, want) >= 1 - 1e-6


def test_graph_replay_matches_eager(qce, h):
    from paper_2303_08989_amd.executor import BatchedExecutor, CircuitPlan, GraphPass
    c = synth.grid_circuit(3, 4, 8, seed=7, pattern="ABCDCDAB")
    plan = CircuitPlan(c, max_log2=5, restarts=2, varied=3)
    gp = GraphPass(plan, n_batch=3, outer=1)
    bx = BatchedExecutor(h, plan, 3)
    try:
        for x in synth.random_bitstrings(12, 4, seed=8):
            eager = bx.amplitude(x, [1]).cpu().numpy()
            torch.cuda.synchronize()
            replay = gp.amplitude(x).cpu().numpy()
            assert np.array_equal(replay, eager), x
            # eager work between replays
            torch.cuda.synchronize()
    finally:
        gp.close()


def test_graph_replay_sliced_output_wires_back_to_back(qce, h):
    # two final wires sliced as outer labels (their <x| leaves become
    # scalars fixed by the outer value), replays issued back to back with
    # no synchronisation in between: each replay's result must still equal
    # the eager pass for its own bitstring
    from paper_2303_08989_amd import tn
    from paper_2303_08989_amd.executor import BatchedExecutor, CircuitPlan, GraphPass
    c = synth.grid_circuit(3, 4, 8, seed=7, pattern="ABCDCDAB")
    base = CircuitPlan(c, max_log2=5, restarts=2, varied=3, reconfigure=False)   # batch labels enter after the wires
    wires = [labels[0] for _, labels in tn.circuit_network(c, 0)[-c["n"]:]]
    plan = CircuitPlan(c, path=base.path, sliced=list(base.sliced) + wires[:2])
    bx = BatchedExecutor(h, plan, 3)
    pos = [bx.outer_labels.index(w) for w in wires[:2]]
    outer = 1 << pos[0]                      # wire of qubit 0 fixed to 1, qubit 1 to 0
    gp = GraphPass(plan, n_batch=3, outer=outer)
    try:
        assert sorted(b for _, b in gp.xslots if b is not None) == sorted(pos)
        n = c["n"]
        xs = [int(x) for x in synth.random_bitstrings(n, 6, seed=9)]
        xs += [(1 << (n - 1)) | 0b1011, (1 << (n - 1)) | (1 << (n - 2)) | 0b11]
        replays = [gp.amplitude(x).clone() for x in xs]
        for x, r in zip(xs, replays):
            eager = bx.amplitude(x, [outer]).cpu().numpy()
            assert np.array_equal(r.cpu().numpy(), eager), x
        # the bitstring whose two leading bits match the fixed values has a
        # nonzero partial amplitude; a mismatch gives exact zero
        assert np.any(replays[-2].cpu().numpy() != 0)
        assert not np.any(replays[-1].cpu().numpy() != 0)
    finally:
        gp.close()


def test_graph_pass_config1_matches_oracle(qce, h):
    # the 12-qubit workload (3x4 grid, depth 8, ABCD, no slicing) as one
    # captured pass in FP32, replayed per bitstring, against the FP64 state
    # vector
    from paper_2303_08989_amd.executor import CircuitPlan, GraphPass
    c = synth.grid_circuit(3, 4, 8, seed=0)
    plan = CircuitPlan(c, max_log2=30, restarts=2)
    assert not plan.sliced
    xs = synth.random_bitstrings(12, 10, seed=1)
    gp = GraphPass(plan, n_batch=0, mode="fp32")
    try:
        got = np.array([complex(*gp.amplitude(x).cpu().numpy()) for x in xs])
    finally:
        gp.close()
    rounded = dict(c)
    rounded["gates"] = [dict(g, matrix=np.asarray(g["matrix"]).astype(np.complex64).astype(np.complex128))
                        for g in c["gates"]]
    want = oracle.statevector_amplitudes(rounded, xs)
    assert oracle.fidelity(got, want) >= 1 - 1e-6
    assert np.max(np.abs(got - want) / np.abs(want)) <= 1e-4


def test_graph_pass_every_outer_value(qce, h):
    # one captured pass switched over every outer value (the leaves carrying
    # outer labels re-uploaded, including <x| leaves fixed by outer bits):
    # each replay equals the eager pass for that outer value bit for bit, and
    # their sum is the amplitude over all slices
    from paper_2303_08989_amd import tn
    from paper_2303_08989_amd.executor import BatchedExecutor, CircuitPlan, GraphPass
    c = synth.grid_circuit(3, 4, 8, seed=7, pattern="ABCDCDAB")
    base = CircuitPlan(c, max_log2=6, restarts=2, varied=3, reconfigure=False)   # batch labels enter after the wire
    wires = [labels[0] for _, labels in tn.circuit_network(c, 0)[-c["n"]:]]
    plan = CircuitPlan(c, path=base.path, sliced=list(base.sliced) + wires[:1])
    bx = BatchedExecutor(h, plan, 3)
    assert 2 <= bx.n_outer <= 64 and wires[0] in bx.outer_labels
    gp = GraphPass(plan, n_batch=3, outer=0)
    try:
        for x in [int(v) for v in synth.random_bitstrings(12, 2, seed=13)]:
            total = 0j
            for o in range(bx.n_outer):
                got = gp.amplitude(x, outer=o).cpu().numpy()
                want = bx.amplitude(x, [o]).cpu().numpy()
                assert np.array_equal(got, want), (x, o)
                total += complex(*got)
            # and back to the first outer value
            assert np.array_equal(gp.amplitude(x, outer=0).cpu().numpy(), bx.amplitude(x, [0]).cpu().numpy())
            whole = complex(*bx.amplitude(x).cpu().numpy())
            assert abs(total - whole) <= 1e-12 * max(abs(whole), 1e-30)
    finally:
        gp.close()
