"""Host planning (circuit -> network -> greedy path -> slices): structural
checks, and the plan executed by a plain numpy stand-in for the GPU (one
einsum per pairwise step) against the FP64 oracle amplitudes."""
import itertools

import numpy as np
import pytest

import oracle
import synth
from paper_2303_08989_amd import tn
from paper_2303_08989_amd.executor import CircuitPlan


def rounded(circuit):
    """The same circuit with gate matrices rounded to complex64, the values
    the GPU path receives."""
    out = dict(circuit)
    out["gates"] = [dict(g, matrix=np.asarray(g["matrix"]).astype(np.complex64).astype(np.complex128))
                    for g in circuit["gates"]]
    return out


def _numpy_execute(plan, x, slice_ids=None):
    leaves = tn.circuit_network(plan.circuit, x)
    L = len(leaves)
    S = plan.sliced
    total = 0.0 + 0.0j
    ids = range(plan.n_slices) if slice_ids is None else slice_ids
    for sigma in ids:
        val = {lab: (sigma >> i) & 1 for i, lab in enumerate(S)}
        tens = {}
        for i, (arr, labels) in enumerate(leaves):
            idx = tuple(val[l] if l in val else slice(None) for l in labels)
            tens[i] = (arr[idx].astype(np.complex128), [l for l in labels if l not in val])
        for s, (a, b) in enumerate(plan.path):
            ta, la = tens.pop(a)
            tb, lb = tens.pop(b)
            shared = set(la) & set(lb)
            lc = [l for l in lb if l not in shared] + [l for l in la if l not in shared]
            letters = {l: chr(97 + i) if i < 26 else chr(65 + i - 26)
                       for i, l in enumerate(sorted(set(la) | set(lb)))}
            expr = "".join(letters[l] for l in la) + "," + "".join(letters[l] for l in lb) + \
                "->" + "".join(letters[l] for l in lc)
            tens[L + s] = (np.einsum(expr, ta, tb), lc)
        (t, _), = tens.values()
        total += complex(t)
    return total


def test_network_structure():
    c = synth.grid_circuit(3, 4, 8, seed=0)
    leaves = tn.circuit_network(c, 5)
    counts = {}
    for arr, labels in leaves:
        assert arr.shape == (2,) * len(labels)
        for l in labels:
            counts[l] = counts.get(l, 0) + 1
    assert set(counts.values()) == {2}        # every wire joins two tensors
    assert len(leaves) == 2 * c["n"] + len(c["gates"])


def test_greedy_path_is_a_valid_tree():
    c = synth.grid_circuit(3, 4, 8, seed=0)
    ls = [l for _, l in tn.circuit_network(c, 0)]
    for seed, noise in [(None, 0.0), (3, 0.3)]:
        p = tn.greedy_path(ls, seed=seed, noise=noise)
        L = len(ls)
        assert len(p) == L - 1
        used = [x for pair in p for x in pair]
        assert sorted(used) == list(range(2 * L - 2))   # every tensor consumed once
        labs = tn.tree_labels(ls, p)
        assert labs[-1] == frozenset()                 # full contraction -> scalar


def test_config1_plan_numpy_matches_oracle():
    c = synth.grid_circuit(3, 4, 8, seed=0)
    plan = CircuitPlan(c, max_log2=30, restarts=2)
    assert plan.sliced == []
    for x in synth.random_bitstrings(12, 4, seed=1):
        assert abs(_numpy_execute(plan, x) - oracle.tn_amplitude(rounded(c), x)) < 1e-12


def test_sliced_plan_numpy_matches_oracle():
    c = synth.grid_circuit(3, 4, 8, seed=2, pattern="ABCDCDAB")
    plan = CircuitPlan(c, max_log2=5, restarts=2, varied=2)
    assert len(plan.sliced) >= 2 and plan.max_log2 <= 5
    x = 1234
    want = oracle.statevector_amplitudes(rounded(c), [x])[0]
    assert abs(_numpy_execute(plan, x) - want) < 1e-12
    # partial sums over disjoint slice ranges add up
    half = plan.n_slices // 2
    s1 = _numpy_execute(plan, x, range(half))
    s2 = _numpy_execute(plan, x, range(half, plan.n_slices))
    assert abs(s1 + s2 - want) < 1e-12


def test_slicing_reduces_intermediates():
    c = synth.grid_circuit(4, 5, 10, seed=3, pattern="ABCDCDAB")
    ls = [l for _, l in tn.circuit_network(c, 0)]
    p = tn.greedy_path(ls)
    ml, fl, _ = tn.path_cost(ls, p)
    sl = tn.choose_slices(ls, p, ml - 3)
    ml2, fl2, _ = tn.path_cost(ls, p, frozenset(sl))
    assert ml2 <= ml - 3 and len(sl) >= 3


def test_subtree_reconfigure_keeps_a_valid_cheaper_tree():
    c = synth.grid_circuit(4, 5, 10, seed=3, pattern="ABCDCDAB")
    ls = [l for _, l in tn.circuit_network(c, 0)]
    L = len(ls)
    for seed, noise in [(None, 0.0), (1, 0.3)]:
        p = tn.greedy_path(ls, seed=seed, noise=noise)
        q = tn.subtree_reconfigure(ls, p)
        assert len(q) == L - 1
        assert sorted(x for pair in q for x in pair) == list(range(2 * L - 2))
        assert tn.tree_labels(ls, q)[-1] == frozenset()
        ml, fl, _ = tn.path_cost(ls, p)
        ml2, fl2, _ = tn.path_cost(ls, q)
        assert (ml2, fl2) <= (ml, fl)


def test_reconfigured_sliced_plan_numpy_matches_oracle():
    c = synth.grid_circuit(3, 4, 8, seed=5, pattern="ABCDCDAB")
    plan = CircuitPlan(c, max_log2=6, restarts=1, varied=2, reconfigure=True)
    assert plan.max_log2 <= 6
    x = 777
    want = oracle.statevector_amplitudes(rounded(c), [x])[0]
    assert abs(_numpy_execute(plan, x) - want) < 1e-12


def test_autotune_table_rules():
    # cells (power-of-two bucket of 128 x 128 tiles, k class) take the
    # faster tile; every bucket gets a rule for both k classes, in ascending
    # order from zero tiles; the library's lookup (last rule whose
    # thresholds are reached) then lands in a GEMM's own cell
    from paper_2303_08989_amd import autotune
    rows = [dict(m=512, n=512, k=512, batch=1, ms_64=1.0, ms_128=2.0),      # 16 tiles, long k -> 64
            dict(m=1024, n=1024, k=512, batch=1, ms_64=3.0, ms_128=2.0),    # 64 tiles, long k -> 128
            dict(m=256, n=256, k=64, batch=16, ms_64=1.0, ms_128=1.5),      # 64 tiles, short k -> 64
            dict(m=4096, n=4096, k=64, batch=1, ms_64=5.0, ms_128=4.0),     # 1024 tiles, short k -> 128
            dict(m=4096, n=4096, k=4096, batch=1, ms_64=9.0, ms_128=4.0)]   # 1024 tiles, long k -> 128
    for r in rows:
        r["tiles128"] = autotune._tiles128([(r["m"], r["n"], r["k"], r["batch"])])
        r["chunks"] = -(-r["k"] // 16)
    # a grouped launch counts the tiles of all its entries (32 + 32) and its
    # longest k
    rows.append(dict(tiles128=autotune._tiles128([(512, 1024, 64, 1), (1024, 512, 64, 1)]), chunks=4,
                     ms_64=0.5, ms_128=1.0))
    assert rows[-1]["tiles128"] == 64
    rules, sums = autotune.table(rows)
    assert sums["6/0"] == [1.5, 2.5] and sums["6/16"] == [3.0, 2.0]

    def lookup(tiles, chunks):
        tile = 128
        for t0, c0, t in rules:
            if tiles >= t0 and chunks >= c0:
                tile = t
        return tile
    assert lookup(16, 32) == 64 and lookup(16, 1) == 64     # only long k measured: both classes
    assert lookup(64, 32) == 128 and lookup(64, 4) == 64
    assert lookup(100, 4) == 64 and lookup(100, 100) == 128
    assert lookup(1024, 4) == 128 and lookup(5000, 256) == 128
    assert rules[0][0] == 0 and rules == sorted(rules)