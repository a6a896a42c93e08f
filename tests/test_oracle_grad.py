"""Pins of the FP64 oracle gradient of |<x|U|0>|^2 with respect to the
per-coupler fSim angles: a closed form, central finite differences of the
(separately pinned) state-vector probability, and conservation of total
probability."""
import math

import numpy as np
import pytest

import oracle
import synth


def _two_qubit(theta, phi=math.pi / 6):
    # X on qubit 1 prepares |01>, then fSim on (0, 1): <01|psi> = cos t,
    # <10|psi> = -i sin t
    g = {"name": "fsim", "qubits": [0, 1], "matrix": synth.gate_matrix("fsim", theta, phi),
         "coupler": 0, "theta": theta, "phi": phi}
    return {"n": 2, "n_couplers": 1,
            "gates": [{"name": "X", "qubits": [1], "matrix": synth.gate_matrix("X")}, g]}


@pytest.mark.parametrize("theta", [0.3, 1.1, 2.5])
def test_closed_form_two_qubits(theta):
    c = _two_qubit(theta)
    a, g = oracle.probability_theta_gradient(c, [0b10, 0b01, 0b00, 0b11])
    assert abs(a[0] - (-1j * math.sin(theta))) < 1e-15 and abs(a[1] - math.cos(theta)) < 1e-15
    assert g[0, 0] == pytest.approx(math.sin(2 * theta), abs=1e-14)
    assert g[1, 0] == pytest.approx(-math.sin(2 * theta), abs=1e-14)
    assert g[2, 0] == 0.0 and g[3, 0] == 0.0


def test_derivative_matrix_finite_difference():
    th, phi, h = 0.7, 0.4, 1e-6
    fd = (synth.gate_matrix("fsim", th + h, phi) - synth.gate_matrix("fsim", th - h, phi)) / (2 * h)
    assert np.max(np.abs(fd - oracle.fsim_theta_derivative(th, phi))) < 1e-9


@pytest.mark.parametrize("shape,depth,seed", [((2, 3), 5, 0), ((3, 3), 4, 1)])
def test_gradient_matches_central_differences(shape, depth, seed):
    base = synth.grid_circuit(*shape, depth, seed=seed, pattern="ABCD")
    ne = base["n_couplers"]
    th = synth.coupler_thetas(ne, seed=seed).astype(np.float64)
    c = synth.with_thetas(base, th)
    xs = synth.random_bitstrings(c["n"], 5, seed=seed + 7)
    _, g = oracle.probability_theta_gradient(c, xs, ne)
    h = 1e-5
    for e in range(ne):
        tp, tm = th.copy(), th.copy()
        tp[e] += h
        tm[e] -= h
        pp = np.abs(oracle.statevector_amplitudes(synth.with_thetas(base, tp), xs)) ** 2
        pm = np.abs(oracle.statevector_amplitudes(synth.with_thetas(base, tm), xs)) ** 2
        fd = (pp - pm) / (2 * h)
        assert np.max(np.abs(fd - g[:, e])) <= 1e-8 * max(1.0, np.max(np.abs(g)))


def test_total_probability_is_stationary():
    # sum_x p_x = 1 for every theta, so sum_x dp_x/dtheta_e = 0
    base = synth.grid_circuit(2, 3, 4, seed=3, pattern="ABCD")
    c = synth.with_thetas(base, synth.coupler_thetas(base["n_couplers"], seed=3))
    xs = list(range(1 << c["n"]))
    a, g = oracle.probability_theta_gradient(c, xs)
    assert abs(np.sum(np.abs(a) ** 2) - 1) < 1e-12
    assert np.max(np.abs(g.sum(axis=0))) < 1e-12
    assert np.max(np.abs(g)) > 1e-3          # not trivially zero


def test_shared_coupler_sums_occurrences():
    # two fSim gates on one coupler: the gradient is the sum of both
    # occurrences' contributions (finite difference of the shared angle)
    th = 0.9
    g1 = {"name": "fsim", "qubits": [0, 1], "matrix": synth.gate_matrix("fsim", th, 0.3),
          "coupler": 0, "theta": th, "phi": 0.3}
    h_gate = {"name": "sqrtX", "qubits": [0], "matrix": synth.gate_matrix("sqrtX")}
    c = {"n": 2, "n_couplers": 1, "gates": [h_gate, g1, dict(h_gate), dict(g1)]}
    xs = [0, 1, 2, 3]
    _, g = oracle.probability_theta_gradient(c, xs)
    h = 1e-6

    def probs(t):
        cc = dict(c)
        cc["gates"] = [dict(x, matrix=synth.gate_matrix("fsim", t, 0.3), theta=t) if x["name"] == "fsim" else x
                       for x in c["gates"]]
        return np.abs(oracle.statevector_amplitudes(cc, xs)) ** 2
    fd = (probs(th + h) - probs(th - h)) / (2 * h)
    assert np.max(np.abs(fd - g[:, 0])) < 1e-9


def test_coupler_subset_equals_full_columns():
    # restricting the product rule to some couplers gives exactly those
    # columns of the full gradient (and zeros elsewhere)
    base = synth.grid_circuit(2, 3, 5, seed=3, pattern="ABCD")
    ne = base["n_couplers"]
    c = synth.with_thetas(base, synth.coupler_thetas(ne, seed=3).astype(np.float64))
    xs = synth.random_bitstrings(c["n"], 4, seed=1)
    a_full, g_full = oracle.probability_theta_gradient(c, xs, ne)
    sub = [0, ne - 1]
    a_sub, g_sub = oracle.probability_theta_gradient(c, xs, ne, couplers=sub)
    assert np.array_equal(a_full, a_sub)
    assert np.array_equal(g_sub[:, sub], g_full[:, sub])
    rest = [e for e in range(ne) if e not in sub]
    assert not g_sub[:, rest].any()
