"""Host logic of the batched slice executor (batch labels, outer loop,
label bookkeeping) driven by a complex128 einsum stand-in for the library's
contraction, against the FP64 oracle amplitude.  No GPU."""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")


def _einsum(A, la, B, lb, lc):
    letters = {l: chr(97 + i) for i, l in enumerate(sorted(set(la) | set(lb)))}
    expr = "".join(letters[l] for l in la) + "," + "".join(letters[l] for l in lb) + "->" + \
        "".join(letters[l] for l in lc)
    return torch.from_numpy(np.asarray(np.einsum(expr, A.numpy().astype(np.complex128),
                                                 B.numpy().astype(np.complex128))))


@pytest.fixture()
def standin(monkeypatch):
    import paper_2303_08989_amd as qce
    monkeypatch.setattr(qce, "contract", lambda h, A, la, B, lb, lc, out=None: _einsum(A, la, B, lb, lc))

    def acc_n(h, src, dst):
        v = src.numpy().astype(np.complex128).sum()
        dst[0] += v.real
        dst[1] += v.imag
    monkeypatch.setattr(qce, "accumulate_n_f64", acc_n)
    return qce


def _rounded(c):
    out = dict(c)
    out["gates"] = [dict(g, matrix=np.asarray(g["matrix"]).astype(np.complex64).astype(np.complex128))
                    for g in c["gates"]]
    return out


@pytest.mark.parametrize("n_batch", [0, 2, 4, 99])
def test_batched_pass_matches_oracle(standin, n_batch):
    from paper_2303_08989_amd.executor import BatchedExecutor, CircuitPlan
    c = synth.grid_circuit(3, 4, 6, seed=3, pattern="ABCDCDAB")
    plan = CircuitPlan(c, max_log2=3, restarts=1, varied=3)
    assert len(plan.sliced) >= 3
    bx = BatchedExecutor(None, plan, n_batch, device="cpu")
    xs = synth.random_bitstrings(12, 3, seed=4)
    want = oracle.statevector_amplitudes(_rounded(c), xs)
    for x, w in zip(xs, want):
        acc = bx.amplitude(x).numpy()
        assert abs(complex(acc[0], acc[1]) - w) < 1e-6 * max(abs(w), 1e-3)
    assert bx.max_intermediate() >= plan.max_log2


def test_outer_ids_partition_the_slices(standin):
    # outer value o covers slice ids [o 2^b, (o+1) 2^b): partial sums add up
    from paper_2303_08989_amd.executor import BatchedExecutor, CircuitPlan
    c = synth.grid_circuit(3, 4, 6, seed=5, pattern="ABCD")
    plan = CircuitPlan(c, max_log2=3, restarts=1, varied=3)
    assert len(plan.sliced) >= 3
    bx = BatchedExecutor(None, plan, 2, device="cpu")
    x = 77
    parts = [complex(*bx.amplitude(x, [o]).numpy()) for o in range(bx.n_outer)]
    whole = complex(*bx.amplitude(x).numpy())
    assert abs(sum(parts) - whole) < 1e-12


def test_level_batches_order_operands_first():
    # every step's operands computed among the steps come from an earlier
    # level; the levels partition the steps, each level in path order
    from paper_2303_08989_amd.executor import CircuitPlan, level_batches
    c = synth.grid_circuit(3, 4, 6, seed=2, pattern="ABCDCDAB")
    plan = CircuitPlan(c, max_log2=30, restarts=1)
    L = len(plan.label_sets)
    rng = np.random.default_rng(0)
    for steps in (list(range(len(plan.path))),
                  sorted(int(s) for s in rng.choice(len(plan.path), len(plan.path) // 2, replace=False))):
        levels = level_batches(plan.path, L, steps)
        assert sorted(s for lev in levels for s in lev) == steps
        where = {L + s: k for k, lev in enumerate(levels) for s in lev}
        for k, lev in enumerate(levels):
            assert lev == sorted(lev)
            for s in lev:
                for ch in plan.path[s]:
                    if ch in where:
                        assert where[ch] < k


@pytest.mark.parametrize("grouped", [True, False])
def test_executor_memoized_slices_match_oracle(standin, monkeypatch, grouped):
    # the sliced executor (subtrees cached across slices while their labels
    # keep their values) with level order or path order, summed over every
    # slice, against the FP64 state vector; and the per-slice values add up
    import paper_2303_08989_amd as qce
    from paper_2303_08989_amd.executor import CircuitPlan, Executor

    def acc1(h, src, dst):
        v = complex(src.numpy().astype(np.complex128).reshape(-1)[0])
        dst[0] += v.real
        dst[1] += v.imag
    monkeypatch.setattr(qce, "accumulate_f64", acc1)
    c = synth.grid_circuit(3, 4, 6, seed=3, pattern="ABCDCDAB")
    plan = CircuitPlan(c, max_log2=3, restarts=1, varied=3)
    assert len(plan.sliced) >= 3 and plan.varied
    ex = Executor(None, plan, device="cpu")
    xs = synth.random_bitstrings(12, 3, seed=4)
    want = oracle.statevector_amplitudes(_rounded(c), xs)
    for x, w in zip(xs, want):
        out = torch.zeros(plan.n_slices, dtype=torch.complex128)
        acc = ex.amplitude(x, slice_out=out, grouped=grouped).numpy()
        assert abs(complex(acc[0], acc[1]) - w) < 1e-6 * max(abs(w), 1e-3)
        assert abs(complex(out.sum()) - complex(acc[0], acc[1])) < 1e-9


def test_fix_labels_keeps_rank():
    from paper_2303_08989_amd import tn
    arr = np.arange(8, dtype=np.complex64).reshape(2, 2, 2)
    assert tn.fix_labels(arr, [5, 6, 7], {6: 1}).shape == (2, 2)
    assert np.array_equal(tn.fix_labels(arr, [5, 6, 7], {6: 1}), arr[:, 1, :])
    v = tn.fix_labels(arr[0, 0], [9], {9: 1})           # every label fixed: 0-d
    assert v.shape == () and v == arr[0, 0, 1]
    assert tn.fix_labels(arr, [5, 6, 7], {5: 0, 6: 1, 7: 0}).shape == ()


def test_sliced_output_wires_give_scalar_leaves(standin):
    # slicing final wires (labels of <x| leaves) leaves 0-d leaves: the sum
    # over all outer values still equals the oracle's amplitude
    from paper_2303_08989_amd import tn
    from paper_2303_08989_amd.executor import BatchedExecutor, CircuitPlan
    c = synth.grid_circuit(3, 4, 6, seed=3, pattern="ABCDCDAB")
    # the plain greedy path, whose batch labels enter the tree after these wires
    base = CircuitPlan(c, max_log2=5, restarts=1, varied=3, reconfigure=False)
    wires = [labels[0] for _, labels in tn.circuit_network(c, 0)[-c["n"]:]]
    plan = CircuitPlan(c, path=base.path, sliced=list(base.sliced) + wires[:2])
    bx = BatchedExecutor(None, plan, len(base.sliced), device="cpu")
    assert all(w in bx.outer_labels for w in wires[:2]) and bx.n_outer <= 64
    for x in (1234, 4095):
        want = oracle.statevector_amplitudes(_rounded(c), [x])[0]
        acc = bx.amplitude(x).numpy()
        assert abs(complex(acc[0], acc[1]) - want) < 1e-6 * max(abs(want), 1e-3)


def test_batched_pass_estimate_matches_the_pass(monkeypatch):
    # the estimate's per-step shapes are those of the contractions a batched
    # pass actually issues (recorded from the stand-in's calls)
    import paper_2303_08989_amd as qce
    from paper_2303_08989_amd.executor import BatchedExecutor, CircuitPlan, batched_pass_estimate
    calls = []

    def record(h, A, la, B, lb, lc, out=None):
        calls.append((A.numel(), list(la), B.numel(), list(lb), list(lc)))
        return _einsum(A, la, B, lb, lc)
    monkeypatch.setattr(qce, "contract", record)
    c = synth.grid_circuit(3, 4, 6, seed=3, pattern="ABCDCDAB")
    plan = CircuitPlan(c, max_log2=3, restarts=1, varied=3)
    nb = 2
    bx = BatchedExecutor(None, plan, nb, device="cpu")
    bx.run_pass(bx._leaves(0, 0), grouped=False)
    assert len(calls) == len(plan.path)
    fl_rate, by_rate, launch = 1e12, 1e11, 1e-6
    want = 0.0
    for na, la, nb_, lb, lc in calls:
        shared = set(la) & set(lb)
        batch = shared & set(lc)
        m = na // 2 ** len(shared)
        n = nb_ // 2 ** len(shared)
        k = 2 ** len(shared - batch)
        count = 2 ** len(batch)
        flops = 8.0 * m * n * k * count
        nbytes = 8.0 * (na + nb_ + 2 ** len(lc))
        want += max(flops / fl_rate, nbytes / by_rate) + launch
    got = batched_pass_estimate(plan, nb, flops_per_s=fl_rate, bytes_per_s=by_rate, launch_s=launch)
    assert got == pytest.approx(want, rel=1e-12)


def test_plan_for_batching_takes_the_cheaper_order():
    from paper_2303_08989_amd.executor import batched_pass_estimate, plan_for_batching
    c = synth.grid_circuit(3, 4, 8, seed=1, pattern="ABCDCDAB")
    p = plan_for_batching(c, max_log2=4, n_batch=3, restarts=2)
    assert p.batched_estimate == batched_pass_estimate(p, 3)
    assert p.batched_estimate > 0
