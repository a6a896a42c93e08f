"""Host logic of the adjoint gradient (tree walk, adjoint bookkeeping,
slice handling, leaf caching): the GradientRunner driven by a plain
complex128 einsum stand-in for the library's contraction, against the FP64
oracle gradient.  No GPU."""
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

    def acc(h, src, dst):
        v = complex(src.reshape(-1)[0])
        dst[0] += v.real
        dst[1] += v.imag
    monkeypatch.setattr(qce, "accumulate_f64", acc)
    return qce


@pytest.mark.parametrize("max_log2,varied", [(30, 4), (3, 3)])
def test_adjoint_walk_matches_oracle(standin, max_log2, varied):
    from paper_2303_08989_amd.executor import CircuitPlan
    from paper_2303_08989_amd.grad import GradientRunner
    base = synth.grid_circuit(2, 3, 5, seed=11, pattern="ABCD")
    th = synth.coupler_thetas(base["n_couplers"], seed=11)
    c = synth.with_thetas(base, th)
    plan = CircuitPlan(c, max_log2=max_log2, restarts=1, varied=varied)
    if max_log2 < 30:
        assert plan.sliced
    run = GradientRunner(None, plan, device="cpu")
    xs = synth.random_bitstrings(6, 5, seed=12)
    p, amps, J = run.probabilities_and_jacobian(th, xs)
    # the oracle on the matrices the runner builds (angles rounded to FP32)
    ref_c = synth.with_thetas(base, th.astype(np.float64))
    ref_c["gates"] = [dict(g, matrix=np.asarray(g["matrix"]).astype(np.complex64).astype(np.complex128))
                      for g in ref_c["gates"]]
    a_ref, J_ref = oracle.probability_theta_gradient(ref_c, xs, base["n_couplers"])
    assert np.max(np.abs(amps - a_ref)) < 1e-6
    assert np.max(np.abs(J - J_ref)) <= 1e-5 * np.max(np.abs(J_ref))
