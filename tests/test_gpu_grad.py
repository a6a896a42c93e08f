"""GPU adjoint gradients of |<x|U|0>|^2 with respect to per-coupler fSim
angles (reverse pass through the contraction tree on the emulated GEMM)
against the FP64 oracle gradient, central finite differences and a closed
form."""
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


def _runner(qce, h, circuit, max_log2=30, varied=4):
    from paper_2303_08989_amd.executor import CircuitPlan
    from paper_2303_08989_amd.grad import GradientRunner
    # the plain greedy path (the sliced-wire cases rely on its label order)
    plan = CircuitPlan(circuit, max_log2=max_log2, restarts=2, varied=varied, reconfigure=False)
    return GradientRunner(h, plan), plan


def _rounded(circuit):
    out = dict(circuit)
    out["gates"] = [dict(g, matrix=np.asarray(g["matrix"]).astype(np.complex64).astype(np.complex128))
                    for g in circuit["gates"]]
    return out


def _with_mode(h, mode, fn):
    if mode == "auto_emulated":
        h.set_mode("auto")
        h.set_size_policy(0, 0)
    else:
        h.set_mode(mode)
    try:
        return fn()
    finally:
        h.set_size_policy(*h.default_size_policy)
        h.set_mode("auto")


def test_closed_form_two_qubits(qce, h):
    theta = 0.8
    g = {"name": "fsim", "qubits": [0, 1], "matrix": synth.gate_matrix("fsim", theta, 0.5),
         "coupler": 0, "theta": theta, "phi": 0.5}
    c = {"n": 2, "n_couplers": 1,
         "gates": [{"name": "X", "qubits": [1], "matrix": synth.gate_matrix("X")}, g]}
    run, _ = _runner(qce, h, c)
    p, amps, J = run.probabilities_and_jacobian(np.array([theta], np.float32), [0b10, 0b01, 0b00])
    th = float(np.float32(theta))
    assert J[0, 0] == pytest.approx(math.sin(2 * th), abs=1e-6)
    assert J[1, 0] == pytest.approx(-math.sin(2 * th), abs=1e-6)
    assert J[2, 0] == 0.0
    assert p[0] == pytest.approx(math.sin(th) ** 2, abs=1e-6)


@pytest.mark.parametrize("mode", ["fp32", "auto_emulated"])
def test_grid12_matches_oracle_gradient(qce, h, mode):
    base = synth.grid_circuit(3, 4, 8, seed=4, pattern="ABCD")
    th = synth.coupler_thetas(base["n_couplers"], seed=4)
    c = synth.with_thetas(base, th)
    xs = synth.random_bitstrings(12, 6, seed=9)
    run, _ = _runner(qce, h, c)
    p, amps, J = _with_mode(h, mode, lambda: run.probabilities_and_jacobian(th, xs))
    a_ref, J_ref = oracle.probability_theta_gradient(_rounded(c), xs, base["n_couplers"])
    scale = np.max(np.abs(J_ref))
    assert np.max(np.abs(J - J_ref)) <= 2e-5 * scale
    assert oracle.fidelity(amps, a_ref) >= 1 - 1e-6


@pytest.mark.parametrize("mode", ["fp32", "auto_emulated"])
def test_grid20_sliced_matches_oracle_gradient(qce, h, mode):
    # 4 x 5 grid (20 qubits), depth 14, the network sliced (intermediates
    # capped at 2^16 elements: 4 sliced labels): the adjoint Jacobian against the FP64
    # product-rule gradient of the state vector on four couplers spread over
    # the grid (each differentiated occurrence is one 2^20 state vector)
    base = synth.grid_circuit(4, 5, 14, seed=4, pattern="ABCDCDAB")
    ne = base["n_couplers"]
    th = synth.coupler_thetas(ne, seed=5)
    c = synth.with_thetas(base, th)
    xs = synth.random_bitstrings(20, 4, seed=13)
    run, plan = _runner(qce, h, c, max_log2=16, varied=3)
    assert len(plan.sliced) >= 2
    p, amps, J = _with_mode(h, mode, lambda: run.probabilities_and_jacobian(th, xs))
    cols = [0, ne // 3, (2 * ne) // 3, ne - 1]
    a_ref, J_ref = oracle.probability_theta_gradient(_rounded(c), xs, ne, couplers=cols)
    assert oracle.fidelity(amps, a_ref) >= 1 - 1e-6
    assert np.max(np.abs(amps - a_ref)) <= 1e-5 * np.max(np.abs(a_ref))
    scale = np.max(np.abs(J_ref[:, cols]))
    assert scale > 0
    assert np.max(np.abs(J[:, cols] - J_ref[:, cols])) <= 2e-5 * scale


def test_sliced_equals_unsliced(qce, h):
    base = synth.grid_circuit(3, 4, 8, seed=6, pattern="ABCDCDAB")
    th = synth.coupler_thetas(base["n_couplers"], seed=6)
    c = synth.with_thetas(base, th)
    xs = synth.random_bitstrings(12, 3, seed=2)
    run_full, plan_full = _runner(qce, h, c, max_log2=30)
    run_sl, plan_sl = _runner(qce, h, c, max_log2=5, varied=3)
    assert len(plan_sl.sliced) >= 2 and not plan_full.sliced
    h.set_mode("fp32")
    try:
        _, a1, J1 = run_full.probabilities_and_jacobian(th, xs)
        _, a2, J2 = run_sl.probabilities_and_jacobian(th, xs)
    finally:
        h.set_mode("auto")
    assert np.max(np.abs(a1 - a2)) <= 1e-6 * np.max(np.abs(a1))
    assert np.max(np.abs(J1 - J2)) <= 2e-5 * np.max(np.abs(J1))


def test_central_finite_differences(qce, h):
    base = synth.grid_circuit(3, 4, 6, seed=8, pattern="ABCD")
    th = synth.coupler_thetas(base["n_couplers"], seed=8)
    c = synth.with_thetas(base, th)
    xs = synth.random_bitstrings(12, 2, seed=1)
    run, _ = _runner(qce, h, c)
    p, _, J = run.probabilities_and_jacobian(th, xs)
    step = 1e-3
    for e in (0, base["n_couplers"] // 2, base["n_couplers"] - 1):
        tp, tm = th.copy(), th.copy()
        tp[e] += np.float32(step)
        tm[e] -= np.float32(step)
        pp, _, _ = run.probabilities_and_jacobian(tp, xs)
        pm, _, _ = run.probabilities_and_jacobian(tm, xs)
        fd = (pp - pm) / (float(tp[e]) - float(tm[e]))
        assert np.max(np.abs(fd - J[:, e])) <= 1e-2 * np.max(np.abs(J)) + 1e-9


def test_autograd_function(qce, h):
    from paper_2303_08989_amd.grad import circuit_probabilities
    base = synth.grid_circuit(2, 3, 5, seed=2, pattern="ABCD")
    th = synth.coupler_thetas(base["n_couplers"], seed=2)
    c = synth.with_thetas(base, th)
    xs = synth.random_bitstrings(6, 4, seed=3)
    run, _ = _runner(qce, h, c)
    t = torch.tensor(th, requires_grad=True)
    p = circuit_probabilities(run, t, xs)
    w = torch.tensor([1.0, -2.0, 0.5, 3.0], dtype=p.dtype)
    (p * w).sum().backward()
    _, J_ref = oracle.probability_theta_gradient(_rounded(c), xs, base["n_couplers"])
    want = J_ref.T @ w.numpy()
    assert np.max(np.abs(t.grad.numpy() - want)) <= 2e-5 * np.max(np.abs(want))


@pytest.mark.parametrize("max_log2", [30, 9])
def test_gradient_graph_equals_eager(qce, h, max_log2):
    # the captured forward + reverse passes, replayed per bitstring, give
    # the eager runner's probabilities and Jacobian bit for bit (the same
    # kernels in the same order); max_log2 = 9 slices the network, which
    # also fixes sliced labels on some <x| leaves
    from paper_2303_08989_amd import tn
    from paper_2303_08989_amd.grad import GradientGraph
    c0 = synth.grid_circuit(3, 4, 8, seed=2, pattern="ABCDCDAB")
    th = synth.coupler_thetas(c0["n_couplers"], seed=3)
    c = synth.with_thetas(c0, th)
    run, plan = _runner(qce, h, c, max_log2=max_log2)
    if max_log2 == 9:
        from paper_2303_08989_amd.executor import CircuitPlan
        wires = [labels[0] for _, labels in tn.circuit_network(c, 0)[-c["n"]:]]
        plan = CircuitPlan(c, path=plan.path, sliced=list(plan.sliced) + wires[:1])
        from paper_2303_08989_amd.grad import GradientRunner
        run = GradientRunner(h, plan)
    xs = synth.random_bitstrings(12, 5, seed=4)
    p_e, a_e, J_e = run.probabilities_and_jacobian(th, xs)
    gg = GradientGraph(plan, th, mode="auto")
    try:
        if max_log2 == 9:
            assert any(f is not None for _, f, _ in gg.xslots)
        p_g, a_g, J_g = gg.probabilities_and_jacobian(xs)
        assert np.array_equal(a_g, a_e) and np.array_equal(J_g, J_e)
        # the same angles, again, after other replays
        _, a_g2, J_g2 = gg.probabilities_and_jacobian(xs[::-1])
        assert np.array_equal(a_g2, a_e[::-1]) and np.array_equal(J_g2, J_e[::-1])
    finally:
        gg.close()


def test_gradient_graph_emulated_modes_equals_eager(qce, h):
    # statistics and selection on every GEMM (size policy (0, 0)): the
    # captured passes run the device-side mode flag, the split and the
    # emulated GEMMs inside the graph and must still equal the eager runner
    # under the same policy, bit for bit, replay after replay
    from paper_2303_08989_amd.grad import GradientGraph
    c0 = synth.grid_circuit(3, 4, 8, seed=2, pattern="ABCDCDAB")
    th = synth.coupler_thetas(c0["n_couplers"], seed=3)
    c = synth.with_thetas(c0, th)
    run, plan = _runner(qce, h, c, max_log2=30)
    xs = synth.random_bitstrings(12, 4, seed=6)
    h.set_size_policy(0, 0)
    try:
        _, a_e, J_e = run.probabilities_and_jacobian(th, xs)
    finally:
        h.set_size_policy(*h.default_size_policy)
    gg = GradientGraph(plan, th, mode="auto", size_policy=(0, 0))
    try:
        for _ in range(2):
            _, a_g, J_g = gg.probabilities_and_jacobian(xs)
            assert np.array_equal(a_g, a_e) and np.array_equal(J_g, J_e)
    finally:
        gg.close()
    # and close to the plain-FP32 Jacobian
    _, _, J32 = _with_mode(h, "fp32", lambda: run.probabilities_and_jacobian(th, xs))
    assert np.max(np.abs(J_e - J32)) <= 1e-4 * np.max(np.abs(J32))


@pytest.mark.parametrize("max_log2", [30, 9])
def test_gradient_graph_new_angles_without_recapture(qce, h, max_log2):
    # one captured graph, angles changed by set_thetas (fSim leaves and
    # derivatives re-uploaded, sliced variants included): equal to the eager
    # runner at each angle vector, bit for bit, and back again
    from paper_2303_08989_amd.grad import GradientGraph
    c0 = synth.grid_circuit(3, 4, 8, seed=2, pattern="ABCDCDAB")
    ne = c0["n_couplers"]
    th1 = synth.coupler_thetas(ne, seed=3)
    th2 = synth.coupler_thetas(ne, seed=11)
    run, plan = _runner(qce, h, synth.with_thetas(c0, th1), max_log2=max_log2)
    xs = synth.random_bitstrings(12, 3, seed=5)
    gg = GradientGraph(plan, th1, mode="auto")
    try:
        for th in (th2, th1, th2):
            _, a_e, J_e = run.probabilities_and_jacobian(th, xs)
            _, a_g, J_g = gg.probabilities_and_jacobian(xs, thetas=th)
            assert np.array_equal(a_g, a_e) and np.array_equal(J_g, J_e)
    finally:
        gg.close()


def test_autograd_function_on_a_graph(qce, h):
    # the autograd function driven by a GradientGraph over several angle
    # updates matches the FP64 oracle gradient at each
    from paper_2303_08989_amd.grad import GradientGraph, circuit_probabilities
    from paper_2303_08989_amd.executor import CircuitPlan
    base = synth.grid_circuit(2, 3, 5, seed=2, pattern="ABCD")
    ne = base["n_couplers"]
    xs = synth.random_bitstrings(6, 4, seed=3)
    th0 = synth.coupler_thetas(ne, seed=2)
    plan = CircuitPlan(synth.with_thetas(base, th0), max_log2=30, restarts=2)
    gg = GradientGraph(plan, th0, mode="auto")
    try:
        w = torch.tensor([1.0, -2.0, 0.5, 3.0], dtype=torch.float64)
        for seed in (2, 7):
            th = synth.coupler_thetas(ne, seed=seed)
            t = torch.tensor(th, requires_grad=True)
            (circuit_probabilities(gg, t, xs) * w).sum().backward()
            _, J_ref = oracle.probability_theta_gradient(_rounded(synth.with_thetas(base, th)), xs, ne)
            want = J_ref.T @ w.numpy()
            assert np.max(np.abs(t.grad.numpy() - want)) <= 2e-5 * np.max(np.abs(want))
    finally:
        gg.close()
