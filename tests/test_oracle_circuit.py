"""Pins of the circuit oracles (Sec. 2.2; Sec. 5.3, Eq. 4): closed forms
(H|0>, GHZ, identity, product states), normalisation, agreement of the two
independent routes (state vector and tensor network) and slicing
invariance."""
import json
import math
import os

import numpy as np
import pytest

import oracle
import synth

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_examples.json")))


def test_hadamard_golden():
    g = GOLD["hadamard_on_zero"]
    circ = {"n": 1, "gates": [{"name": "H", "qubits": [0], "matrix": synth.gate_matrix("H")}]}
    want = np.array(g["amplitudes_re"]) + 1j * np.array(g["amplitudes_im"])
    assert np.allclose(oracle.statevector(circ), want, atol=1e-15)
    assert np.allclose([oracle.tn_amplitude(circ, x) for x in (0, 1)], want, atol=1e-15)


def test_t_gate_golden():
    g = GOLD["t_gate"]
    T = synth.gate_matrix("T")
    assert np.allclose(np.diag(T), np.array(g["diag_re"]) + 1j * np.array(g["diag_im"]), atol=1e-15)


@pytest.mark.parametrize("n", [3, 6, 9])
def test_ghz(n):
    c = synth.ghz_circuit(n)
    psi = oracle.statevector(c)
    want = np.zeros(1 << n, dtype=np.complex128)
    want[0] = want[-1] = 1 / math.sqrt(2)
    assert np.allclose(psi, want, atol=1e-14)
    for x in (0, (1 << n) - 1, 1, 5 % (1 << n)):
        assert abs(oracle.tn_amplitude(c, x) - want[x]) < 1e-14


def test_identity_circuit():
    c = synth.identity_circuit(6, seed=2)
    psi = oracle.statevector(c)
    want = np.zeros(64, dtype=np.complex128)
    want[0] = 1
    assert np.allclose(psi, want, atol=1e-13)
    assert abs(oracle.tn_amplitude(c, 0) - 1) < 1e-13
    assert abs(oracle.tn_amplitude(c, 37)) < 1e-13


def test_product_state_closed_form():
    n = 5
    c = synth.product_circuit(n, seed=4, layers=3)
    # per-qubit single-qubit unitary, applied in order
    U = [np.eye(2, dtype=np.complex128) for _ in range(n)]
    for g in c["gates"]:
        q = g["qubits"][0]
        U[q] = g["matrix"] @ U[q]
    for x in range(1 << n):
        want = np.prod([U[q][(x >> (n - 1 - q)) & 1, 0] for q in range(n)])
        assert abs(oracle.tn_amplitude(c, x) - want) < 1e-14
        assert abs(oracle.statevector(c)[x] - want) < 1e-14


def test_norm_and_routes_agree_config1():
    # 12-qubit 3x4 grid, depth 8, ABCD layering, fSim(pi/2, pi/6)
    c = synth.grid_circuit(3, 4, 8, seed=0)
    psi = oracle.statevector(c)
    assert abs(np.sum(np.abs(psi) ** 2) - 1) < 1e-12
    xs = synth.random_bitstrings(12, 10, seed=1)
    tn = np.array([oracle.tn_amplitude(c, x) for x in xs])
    assert np.max(np.abs(tn - psi[xs])) < 1e-12


def test_slicing_invariance():
    c = synth.grid_circuit(2, 3, 4, seed=5)
    x = 0b101101
    full = oracle.tn_amplitude(c, x)
    tensors = oracle.tn_build(c, x)
    # slice three internal wire labels (edges between gates)
    labels = sorted({lab for _, ls in tensors for lab in ls})
    sliced = [labels[len(labels) // 3], labels[len(labels) // 2], labels[2 * len(labels) // 3]]
    assert abs(oracle.tn_amplitude_sliced(c, x, sliced) - full) < 1e-13


def test_fidelity():
    a = np.array([1 + 1j, 2 - 1j])
    assert oracle.fidelity(a, a) == pytest.approx(1.0)
    assert oracle.fidelity(a * np.exp(0.3j), a) == pytest.approx(1.0)
    assert oracle.fidelity(np.array([1, 0]), np.array([0, 1])) == 0.0
