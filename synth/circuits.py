"""Seeded random quantum circuits on 2-D qubit grids.

A circuit is a plain description: ``{"n": n_qubits, "gates": [...]}`` where
each gate is ``{"name": str, "qubits": [q] or [q1, q2], "matrix": ndarray}``
with a 2x2 or 4x4 complex128 unitary, applied in list order to |0...0>.  For
a two-qubit gate the basis order is |b1 b2> with b1 the bit of ``qubits[0]``
(index 2*b1 + b2).  Bitstring convention: qubit q is bit n-1-q of the
integer x, so qubit 0 is the most significant bit.

Gate set (standard definitions; the paper names the circuit family, Sec. 5.3,
but prints no matrices):

* sqrt(P) = (1+i)/2 * (I - i P) for P in {X, Y, W = (X+Y)/sqrt 2};
* fSim(theta, phi) = [[1,0,0,0],[0,cos t,-i sin t,0],[0,-i sin t,cos t,0],
  [0,0,0,exp(-i phi)]], used with theta = pi/2, phi = pi/6;
* H and T as defined in Sec. 2.2, CZ = fSim(0, pi), and CNOT for GHZ tests.

Random grid circuits: R x C grid, qubit q = r*C + c (optionally with sites
removed and the rest renumbered).  One cycle is a layer of single-qubit gates
drawn uniformly from {sqrt X, sqrt Y, sqrt W} (cycle-major, qubit-ascending
draws from ``numpy.random.default_rng(seed)``) followed by the two-qubit
layer ``pattern[c % len(pattern)]``; a final single-qubit layer closes the
circuit.  Coupler layers: A = horizontal (r,c)-(r,c+1) with c even,
B = horizontal with c odd, C = vertical (r,c)-(r+1,c) with r even,
D = vertical with r odd.  This brickwork is a synthetic stand-in for the
rectangular-lattice and Sycamore circuits of Sec. 5.3, whose instance files
are not available.
"""
import math
import numpy as np

_I2 = np.eye(2, dtype=np.complex128)
_X = np.array([[0, 1], [1, 0]], dtype=np.complex128)
_Y = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
_W = (_X + _Y) / math.sqrt(2.0)


def _sqrt_pauli(p):
    return (1 + 1j) / 2 * (_I2 - 1j * p)


def _exact_trig(angle):
    """cos and sin with exact values at multiples of pi/2 (math.cos(pi/2) is
    6e-17, not 0; the gate's entries there are exactly 0 and +-1)."""
    q = angle / (math.pi / 2)
    if abs(q - round(q)) < 1e-12:
        return {0: (1.0, 0.0), 1: (0.0, 1.0), 2: (-1.0, 0.0), 3: (0.0, -1.0)}[int(round(q)) % 4]
    return math.cos(angle), math.sin(angle)


def _exact_phase(phi):
    c, s = _exact_trig(phi)
    return complex(c, s)


def fsim(theta, phi):
    c, s = _exact_trig(theta)
    return np.array([[1, 0, 0, 0],
                     [0, c, -1j * s, 0],
                     [0, -1j * s, c, 0],
                     [0, 0, 0, _exact_phase(-phi)]], dtype=np.complex128)


def gate_matrix(name, theta=math.pi / 2, phi=math.pi / 6):
    if name == "sqrtX":
        return _sqrt_pauli(_X)
    if name == "sqrtY":
        return _sqrt_pauli(_Y)
    if name == "sqrtW":
        return _sqrt_pauli(_W)
    if name == "H":
        return np.array([[1, 1], [1, -1]], dtype=np.complex128) / math.sqrt(2.0)
    if name == "T":
        return np.array([[1, 0], [0, _exact_phase(math.pi / 4)]], dtype=np.complex128)
    if name == "X":
        return _X.copy()
    if name == "I":
        return _I2.copy()
    if name == "fsim":
        return fsim(theta, phi)
    if name == "CZ":
        return fsim(0.0, math.pi)
    if name == "CNOT":
        m = np.eye(4, dtype=np.complex128)
        m[2:, 2:] = _X
        return m
    raise ValueError(f"unknown gate {name!r}")


ONE_QUBIT_SET = ("sqrtX", "sqrtY", "sqrtW")


def _layer_pairs(rows, cols, layer, alive):
    pairs = []
    if layer in "AB":
        parity = 0 if layer == "A" else 1
        for r in range(rows):
            for c in range(parity, cols - 1, 2):
                pairs.append(((r, c), (r, c + 1)))
    elif layer in "CD":
        parity = 0 if layer == "C" else 1
        for r in range(parity, rows - 1, 2):
            for c in range(cols):
                pairs.append(((r, c), (r + 1, c)))
    else:
        raise ValueError(f"unknown coupler layer {layer!r}")
    return [(p, q) for p, q in pairs if p in alive and q in alive]


def grid_circuit(rows, cols, depth, seed, pattern="ABCD", removed=(),
                 theta=math.pi / 2, phi=math.pi / 6):
    """Random grid circuit of ``depth`` cycles (see module docstring).

    ``removed`` lists (r, c) grid sites without a qubit; remaining sites are
    numbered row-major.  Each two-qubit gate records its coupler index
    (``"coupler"``: position in the sorted list of distinct couplers) so that
    per-coupler angles can be attached to it.
    """
    rng = np.random.default_rng(seed)
    sites = [(r, c) for r in range(rows) for c in range(cols) if (r, c) not in set(removed)]
    index = {s: i for i, s in enumerate(sites)}
    alive = set(sites)
    n = len(sites)
    couplers = {}
    for layer in "ABCD":
        for p, q in _layer_pairs(rows, cols, layer, alive):
            couplers.setdefault((index[p], index[q]), None)
    coupler_ids = {cq: i for i, cq in enumerate(sorted(couplers))}
    gates = []

    def one_qubit_layer():
        draws = rng.integers(0, len(ONE_QUBIT_SET), n)
        for q in range(n):
            name = ONE_QUBIT_SET[int(draws[q])]
            gates.append({"name": name, "qubits": [q], "matrix": gate_matrix(name)})

    for cyc in range(depth):
        one_qubit_layer()
        layer = pattern[cyc % len(pattern)]
        for p, q in _layer_pairs(rows, cols, layer, alive):
            qa, qb = index[p], index[q]
            gates.append({"name": "fsim", "qubits": [qa, qb],
                          "matrix": gate_matrix("fsim", theta, phi),
                          "coupler": coupler_ids[(qa, qb)],
                          "theta": theta, "phi": phi})
    one_qubit_layer()
    return {"n": n, "gates": gates, "rows": rows, "cols": cols,
            "sites": sites, "n_couplers": len(coupler_ids)}


def with_thetas(circuit, thetas):
    """Copy of a grid circuit whose fSim gates take the angle of their
    coupler: gate on coupler e gets fSim(thetas[e], its phi)."""
    out = dict(circuit)
    gates = []
    for g in circuit["gates"]:
        if g.get("name") == "fsim" and "coupler" in g:
            th = float(thetas[g["coupler"]])
            g = dict(g, theta=th, matrix=gate_matrix("fsim", th, g["phi"]))
        gates.append(g)
    out["gates"] = gates
    return out


def coupler_thetas(n_couplers, seed, low=0.2, high=1.4):
    """Seeded per-coupler angles (radians), uniform in [low, high)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(low, high, n_couplers).astype(np.float32)


# 53-qubit stand-in: a 6 x 9 grid with one corner site removed.
GRID_53 = dict(rows=6, cols=9, removed=((5, 8),))


def ghz_circuit(n):
    """H on qubit 0, then a CNOT chain 0->1->...->n-1: (|0..0> + |1..1>)/sqrt 2."""
    gates = [{"name": "H", "qubits": [0], "matrix": gate_matrix("H")}]
    for q in range(n - 1):
        gates.append({"name": "CNOT", "qubits": [q, q + 1], "matrix": gate_matrix("CNOT")})
    return {"n": n, "gates": gates}


def identity_circuit(n, seed, layers=3):
    """Random gates each followed by its inverse: the overall unitary is I."""
    rng = np.random.default_rng(seed)
    gates = []
    for _ in range(layers):
        for q in range(n):
            name = ONE_QUBIT_SET[int(rng.integers(0, 3))]
            g = gate_matrix(name)
            gates.append({"name": name, "qubits": [q], "matrix": g})
            gates.append({"name": name + "^-1", "qubits": [q], "matrix": g.conj().T.copy()})
        for q in range(0, n - 1, 2):
            g = gate_matrix("fsim")
            gates.append({"name": "fsim", "qubits": [q, q + 1], "matrix": g})
            gates.append({"name": "fsim^-1", "qubits": [q, q + 1], "matrix": g.conj().T.copy()})
    return {"n": n, "gates": gates}


def product_circuit(n, seed, layers=2):
    """Only single-qubit gates: amplitude factorises over qubits."""
    rng = np.random.default_rng(seed)
    gates = []
    for _ in range(layers):
        for q in range(n):
            name = ONE_QUBIT_SET[int(rng.integers(0, 3))]
            gates.append({"name": name, "qubits": [q], "matrix": gate_matrix(name)})
    return {"n": n, "gates": gates}


def random_bitstrings(n, count, seed):
    """``count`` random n-bit integers (qubit q = bit n-1-q)."""
    rng = np.random.default_rng(seed)
    return [int(x) for x in rng.integers(0, 1 << n, count, dtype=np.uint64)]
