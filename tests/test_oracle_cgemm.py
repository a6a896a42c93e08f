"""Pins of the oracle's CGEMM and contraction to facts outside the oracle:
exact integer arithmetic, closed forms, and the reduction of a contraction to
a matrix product.  (Sec. 3, CGEMM as four real products; Sec. 2.2.)"""
import itertools

import numpy as np
import pytest

import oracle
import synth


def _py_cgemm(A, B, opA, opB, alpha, beta, C0):
    """Brute force with Python integers / complex ints (exact)."""
    def op(M, o):
        M = [[complex(int(v.real), int(v.imag)) for v in row] for row in M.tolist()]
        if o == "N":
            return M
        T = [list(r) for r in zip(*M)]
        if o == "C":
            T = [[v.conjugate() for v in r] for r in T]
        return T
    a = op(A, opA)
    b = op(B, opB)
    m, k, n = len(a), len(b), len(b[0])
    out = []
    for i in range(m):
        row = []
        for j in range(n):
            s = 0
            for l in range(k):
                # exact integer complex product
                ar, ai = int(a[i][l].real), int(a[i][l].imag)
                br, bi = int(b[l][j].real), int(b[l][j].imag)
                s += complex(ar * br - ai * bi, ar * bi + ai * br)
            v = alpha * s
            if beta != 0:
                v += beta * complex(C0[i][j])
            row.append(v)
        out.append(row)
    return np.array(out, dtype=np.complex128)


@pytest.mark.parametrize("opA,opB", list(itertools.product("NTC", "NTC")))
def test_integer_bruteforce_all_ops(opA, opB):
    rng = np.random.default_rng(hash((opA, opB)) % 1000)
    m, n, k = 5, 4, 7
    a = synth.random_matrix(*((m, k) if opA == "N" else (k, m)), "int", rng)
    b = synth.random_matrix(*((k, n) if opB == "N" else (n, k)), "int", rng)
    C0 = synth.random_matrix(m, n, "int", rng).astype(np.complex128)
    for alpha, beta in [(1, 0), (complex(2, -3), complex(-1, 2))]:
        got = oracle.cgemm(a, b, opA, opB, alpha, beta, C0)
        want = _py_cgemm(a, b, opA, opB, alpha, beta, C0)
        assert np.array_equal(got, want)


def test_imaginary_part_uses_ai_br():
    # Sec. 3 prints the imaginary part as Ar*Bi + Ar*Bi; the complex product
    # needs Ar*Bi + Ai*Br.  A = i (purely imaginary), B = 1 gives i only with
    # the Ai*Br term.
    A = np.array([[1j]], dtype=np.complex64)
    B = np.array([[1.0]], dtype=np.complex64)
    assert oracle.cgemm(A, B)[0, 0] == 1j


def test_identity_right_factor():
    rng = np.random.default_rng(3)
    a = synth.random_matrix(17, 9, "a", rng)
    eye = np.eye(9, dtype=np.complex64)
    assert np.array_equal(oracle.cgemm(a, eye), a.astype(np.complex128))


def _hadamard(n):
    H = np.array([[1.0]])
    while H.shape[0] < n:
        H = np.block([[H, H], [H, -H]])
    return H


@pytest.mark.parametrize("n", [8, 64])
def test_hadamard_closed_form(n):
    # ((1+i) H) ((1-i) H)^T = (1+i)(1-i) H H^T = 2 n I, exactly
    H = _hadamard(n)
    A = ((1 + 1j) * H).astype(np.complex64)
    B = ((1 - 1j) * H).astype(np.complex64)
    C = oracle.cgemm(A, B, "N", "T")
    assert np.array_equal(C, 2 * n * np.eye(n))
    # conjugate transpose: A A^H = |1+i|^2 H H^T = 2 n I
    C2 = oracle.cgemm(A, A, "N", "C")
    assert np.array_equal(C2, 2 * n * np.eye(n))


def test_empty_dimensions():
    A = np.zeros((3, 0), dtype=np.complex64)
    B = np.zeros((0, 4), dtype=np.complex64)
    assert np.array_equal(oracle.cgemm(A, B), np.zeros((3, 4)))


def test_rel_fro():
    C = np.array([[3 + 4j]])
    assert oracle.rel_fro(C, C) == 0.0
    assert oracle.rel_fro(2 * C, C) == pytest.approx(1.0)
    assert oracle.rel_fro(C, np.zeros_like(C)) == pytest.approx(5.0)


# --- contraction ---------------------------------------------------------

def _py_contract(A, la, B, lb, lc, ext):
    """Brute force over every label assignment (Python complex, tiny sizes)."""
    labels = sorted(set(la) | set(lb))
    out = np.zeros(tuple(ext[x] for x in lc), dtype=np.complex128)
    for vals in itertools.product(*[range(ext[x]) for x in labels]):
        v = dict(zip(labels, vals))
        out[tuple(v[x] for x in lc)] += complex(A[tuple(v[x] for x in la)]) * complex(B[tuple(v[x] for x in lb)])
    return out


@pytest.mark.parametrize("seed", range(6))
def test_contract_bruteforce(seed):
    net = synth.random_network(seed, n_contracted=1 + seed % 3, n_free_a=1 + seed % 2,
                               n_free_b=2 - seed % 2, max_extent=3, dist="int")
    got = oracle.zcontract(net["A"], net["la"], net["B"], net["lb"], net["lc"])
    want = _py_contract(net["A"], net["la"], net["B"], net["lb"], net["lc"], net["extents"])
    assert np.array_equal(got, want)


def test_contract_reduces_to_matrix_product():
    rng = np.random.default_rng(11)
    A = synth.random_matrix(6, 5, "int", rng)   # labels (i, k)
    B = synth.random_matrix(5, 7, "int", rng)   # labels (k, j)
    C = oracle.zcontract(np.ascontiguousarray(A), [0, 1], np.ascontiguousarray(B), [1, 2], [0, 2])
    want = _py_cgemm(A, B, "N", "N", 1, 0, None)
    assert np.array_equal(C, want)


def test_contract_output_permutation_is_exact():
    net = synth.random_network(5, 2, 2, 2, max_extent=3)
    C = oracle.zcontract(net["A"], net["la"], net["B"], net["lb"], net["lc"])
    perm = list(reversed(range(len(net["lc"]))))
    lc2 = [net["lc"][p] for p in perm]
    C2 = oracle.zcontract(net["A"], net["la"], net["B"], net["lb"], lc2)
    assert np.array_equal(np.transpose(C, perm), C2)


def test_contract_rejects_dangling_labels():
    A = np.ones((2, 2), dtype=np.complex64)
    with pytest.raises(ValueError):
        oracle.zcontract(A, [0, 3], A, [1, 2], [1, 2])      # label summed over one input
    with pytest.raises(ValueError):
        oracle.zcontract(A, [0, 1], A, [1, 2], [0, 2, 9])   # output label in no input


def test_zcontract_batch_labels_are_independent_contractions():
    # a label in A, B and C indexes one independent contraction per value:
    # the result equals the per-value contractions stacked along that label,
    # and the batched matrix product numpy computes
    rng = np.random.default_rng(21)
    A = (rng.standard_normal((3, 4, 5)) + 1j * rng.standard_normal((3, 4, 5))).astype(np.complex64)
    B = (rng.standard_normal((5, 3, 2)) + 1j * rng.standard_normal((5, 3, 2))).astype(np.complex64)
    # labels: batch 0 (extent 3), row 1 (4), contracted 2 (5), col 3 (2)
    C = oracle.zcontract(A, [0, 1, 2], B, [2, 0, 3], [1, 0, 3])
    for b in range(3):
        per = oracle.zcontract(A[b], [1, 2], B[:, b, :], [2, 3], [1, 3])
        assert np.array_equal(C[:, b, :], per)
    want = np.matmul(A.astype(np.complex128), np.transpose(B, (1, 0, 2)).astype(np.complex128))
    assert np.max(np.abs(np.transpose(C, (1, 0, 2)) - want)) < 1e-12


def test_zcontract_batch_only_label():
    # every label batch: an elementwise product
    a = np.array([1 + 2j, 3 - 1j], dtype=np.complex64)
    b = np.array([2 - 1j, 1j], dtype=np.complex64)
    c = oracle.zcontract(a, [7], b, [7], [7])
    assert np.array_equal(c, a.astype(np.complex128) * b.astype(np.complex128))


def test_zcontract_batch_bruteforce():
    rng = np.random.default_rng(4)
    ext = {0: 2, 1: 3, 2: 2, 3: 3, 4: 2}
    la, lb, lc = [0, 4, 1, 2], [2, 3, 0, 4], [3, 0, 1, 4]      # 0 and 4 batch, 2 summed
    A = synth.random_matrix(1, 24, "int", rng).reshape(tuple(ext[x] for x in la))
    B = synth.random_matrix(1, 24, "int", rng).reshape(tuple(ext[x] for x in lb))
    assert np.array_equal(oracle.zcontract(A, la, B, lb, lc), _py_contract(A, la, B, lb, lc, ext))
