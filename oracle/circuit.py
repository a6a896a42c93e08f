"""Circuit amplitudes <x|U|0...0> in complex128 (Sec. 5.3, Eq. 4).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Two independent routes:

* ``statevector``: brute force, the 2^n state updated gate by gate
  (Sec. 1, the state-vector method); qubit q is axis q of the (2,)*n state,
  so the flat index has qubit 0 as its most significant bit.
* ``probability_theta_gradient``: d|<x|U|0>|^2 / d theta_e for per-coupler
  fSim angles, by the product rule written out (parity unpinned in the
  paper, which does not differentiate; pinned here by closed forms, finite
  differences and probability conservation in the tests).
* ``tn_amplitude``: the circuit as a tensor network (Sec. 2.2): |0> and <x|
  are rank-1 tensors, a k-qubit gate is a rank-2k tensor, every wire segment
  is a label; the network is contracted pairwise with the nested-loop
  contraction of ``core.zcontract`` in the oracle's own fixed order
  (tensors in creation order).  ``tn_amplitude_sliced`` fixes chosen labels
  to every combination of values and sums the slice results (Sec. 5.3).
"""
import itertools

import numpy as np

from .core import zcontract


def statevector(circuit):
    n = circuit["n"]
    psi = np.zeros((2,) * n, dtype=np.complex128)
    psi[(0,) * n] = 1.0
    for g in circuit["gates"]:
        qs = list(g["qubits"])
        k = len(qs)
        U = np.asarray(g["matrix"], dtype=np.complex128).reshape((2,) * (2 * k))
        # new[o..] = sum_i U[o.., i..] psi[.. i ..]
        psi = np.tensordot(U, psi, axes=(list(range(k, 2 * k)), qs))
        # tensordot puts the gate's output axes first; move them back
        psi = np.moveaxis(psi, list(range(k)), qs)
    return psi.reshape(-1)


def statevector_amplitudes(circuit, bitstrings):
    psi = statevector(circuit)
    return np.array([psi[int(x)] for x in bitstrings], dtype=np.complex128)


def tn_build(circuit, x):
    """Tensor list [(tensor, labels)] for <x|U|0>.  Labels are ints."""
    n = circuit["n"]
    tensors = []
    nxt = [0]

    def new_label():
        nxt[0] += 1
        return nxt[0] - 1

    cur = []
    for q in range(n):
        lab = new_label()
        cur.append(lab)
        tensors.append((np.array([1.0, 0.0], dtype=np.complex128), [lab]))
    for g in circuit["gates"]:
        qs = list(g["qubits"])
        k = len(qs)
        U = np.asarray(g["matrix"], dtype=np.complex128).reshape((2,) * (2 * k))
        outs = [new_label() for _ in qs]
        tensors.append((U, outs + [cur[q] for q in qs]))
        for q, o in zip(qs, outs):
            cur[q] = o
    for q in range(n):
        bit = (int(x) >> (n - 1 - q)) & 1
        v = np.zeros(2, dtype=np.complex128)
        v[bit] = 1.0
        tensors.append((v, [cur[q]]))
    return tensors


def _contract_sequential(tensors):
    T, lt = tensors[0]
    for U, lu in tensors[1:]:
        shared = [lab for lab in lt if lab in lu]
        out = [lab for lab in lt if lab not in shared] + [lab for lab in lu if lab not in shared]
        T = zcontract(T, lt, U, lu, out)
        lt = out
    assert T.size == 1
    return complex(T.reshape(-1)[0])


def tn_amplitude(circuit, x):
    return _contract_sequential(tn_build(circuit, x))


def _fix_label(T, labels, lab, value):
    if lab not in labels:
        return T, labels
    ax = labels.index(lab)
    T = np.take(T, value, axis=ax)
    return T, [l for l in labels if l != lab]


def tn_amplitude_sliced(circuit, x, sliced_labels):
    """Sum over all assignments of ``sliced_labels`` (each of extent 2) of the
    network with those labels fixed (Sec. 5.3, slicing)."""
    base = tn_build(circuit, x)
    total = 0.0 + 0.0j
    for vals in itertools.product((0, 1), repeat=len(sliced_labels)):
        ts = []
        for T, lt in base:
            for lab, v in zip(sliced_labels, vals):
                T, lt = _fix_label(T, lt, lab, v)
            ts.append((np.asarray(T, dtype=np.complex128), lt))
        # rank-0 leftovers are scalar factors
        scal = 1.0 + 0.0j
        rest = []
        for T, lt in ts:
            if len(lt) == 0:
                scal *= complex(T)
            else:
                rest.append((T, lt))
        total += scal * (_contract_sequential(rest) if rest else 1.0)
    return total


def fsim_theta_derivative(theta, phi):
    """d fSim(theta, phi) / d theta: the middle block [[cos, -i sin],
    [-i sin, cos]] differentiates to [[-sin, -i cos], [-i cos, -sin]]; the
    |00> and |11> entries do not depend on theta."""
    c, s = np.cos(theta), np.sin(theta)
    d = np.zeros((4, 4), dtype=np.complex128)
    d[1, 1] = d[2, 2] = -s
    d[1, 2] = d[2, 1] = -1j * c
    return d


def probability_theta_gradient(circuit, bitstrings, n_couplers=None, couplers=None):
    """Amplitudes a_x and the gradient of p_x = |a_x|^2 with respect to the
    per-coupler fSim angles theta_e, in complex128.

    U is the product of the circuit's gates, so by the product rule
    dU/dtheta_e is the sum, over the fSim gates g on coupler e, of U with g
    replaced by dg/dtheta; then dp/dtheta_e = 2 Re(conj(a) da/dtheta_e).
    Each replaced circuit is evaluated by the state vector.  ``couplers``
    (optional) limits the work to those couplers' columns; the other columns
    stay 0.  Returns (a of shape (X,), grad of shape (X, n_couplers))."""
    gates = circuit["gates"]
    if n_couplers is None:
        n_couplers = circuit.get("n_couplers", 1 + max(g["coupler"] for g in gates if "coupler" in g))
    wanted = None if couplers is None else set(int(e) for e in couplers)
    a = statevector_amplitudes(circuit, bitstrings)
    grad = np.zeros((len(bitstrings), n_couplers), dtype=np.float64)
    for gi, g in enumerate(gates):
        if g.get("name") != "fsim" or "coupler" not in g:
            continue
        if wanted is not None and g["coupler"] not in wanted:
            continue
        mod = dict(circuit)
        mod["gates"] = list(gates)
        mod["gates"][gi] = dict(g, matrix=fsim_theta_derivative(g["theta"], g["phi"]))
        da = statevector_amplitudes(mod, bitstrings)
        grad[:, g["coupler"]] += 2.0 * np.real(np.conj(a) * da)
    return a, grad


def fidelity(a, b):
    """Fidelity of an amplitude vector a against a reference b over the same
    bitstrings: |sum conj(b) a|^2 / (sum |a|^2 * sum |b|^2), in FP64.

    The paper plots a fidelity (Sec. 1-2) without defining it; this is the
    normalised overlap of the two amplitude vectors."""
    a = np.asarray(a, dtype=np.complex128)
    b = np.asarray(b, dtype=np.complex128)
    num = abs(np.vdot(b, a)) ** 2
    den = float(np.vdot(a, a).real * np.vdot(b, b).real)
    return float(num / den) if den > 0 else 1.0
