"""The CGEMM entry point that allocates nothing (qce_cgemm_emulated_noalloc,
fixed per-GPU scratch), through the C-ABI: its output equals
qce_cgemm_emulated's bit for bit on the same inputs, on two calls in a row
(the second smaller, so stale scratch contents from the first are present),
it runs with a handle whose own workspace is too small for the GEMM, and a
shape beyond the scratch is rejected before anything is enqueued."""
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


def dev(a):
    return torch.from_numpy(np.asfortranarray(a).ravel(order="F").copy()).to("cuda")


def host(t, rows, cols, ld):
    flat = t.cpu().numpy()
    out = np.empty((rows, cols), dtype=np.complex64, order="F")
    for j in range(cols):
        out[:, j] = flat[j * ld:j * ld + rows]
    return out


def bits(x):
    return np.ascontiguousarray(x).view(np.uint32)


@pytest.mark.parametrize("mode", ["auto", "fp32", "bf16x3"])
def test_noalloc_equals_allocating_entry(qce, mode):
    ref_h = qce.Handle(0)
    na_h = qce.Handle(0)
    tiny = torch.zeros(64, dtype=torch.complex64, device="cuda")
    try:
        na_h.set_workspace(tiny)  # 512 bytes: the allocating entry could not run here
        rng = np.random.default_rng(17)
        cases = [(1000, 900, 700, "N", "T", "a"), (300, 200, 96, "C", "N", "b"), (40, 300, 5, "N", "N", "a")]
        for m, n, k, opA, opB, dist in cases:
            sa = (m, k) if opA == "N" else (k, m)
            sb = (k, n) if opB == "N" else (n, k)
            A = synth.random_matrix(*sa, dist, rng)
            B = synth.random_matrix(*sb, dist, rng)
            C0 = synth.random_matrix(m, n, "a", rng)
            ldc = m + 3
            C0p = np.zeros((ldc, n), np.complex64)
            C0p[:m] = C0
            dA, dB = dev(A), dev(B)
            outs = []
            for h, fn in ((ref_h, qce.cgemm), (na_h, qce.cgemm_noalloc)):
                h.set_mode(mode)
                dC = dev(C0p)
                fn(h, opA, opB, m, n, k, dA, sa[0], dB, sb[0], dC, ldc, alpha=1.5 - 0.5j, beta=0.25j)
                torch.cuda.synchronize()
                outs.append((host(dC, m, n, ldc), h.last_decision()))
            assert np.array_equal(bits(outs[0][0]), bits(outs[1][0])), (m, n, k, mode)
            assert outs[0][1] == outs[1][1]
            # and the value is the product to FP32 accuracy
            exact = oracle.cgemm(A, B, opA, opB, 1.5 - 0.5j, 0.25j, C0)
            assert oracle.rel_fro(outs[1][0], exact) < 1e-5
        # the allocating entry point cannot grow the caller's tiny workspace
        with pytest.raises(qce.QceError):
            qce.cgemm(na_h, "N", "N", 512, 512, 512, torch.zeros(512 * 512, dtype=torch.complex64, device="cuda"),
                      512, torch.zeros(512 * 512, dtype=torch.complex64, device="cuda"), 512,
                      torch.zeros(512 * 512, dtype=torch.complex64, device="cuda"), 512)
    finally:
        na_h.close()
        ref_h.close()


def test_noalloc_rejects_oversize(qce):
    h = qce.Handle(0)
    try:
        m = n = k = 4096
        assert qce.cgemm_workspace_size(m, n, k) > qce.noalloc_scratch_bytes()
        A = torch.ones(m * k, dtype=torch.complex64, device="cuda")
        C = torch.full((m * n,), 7.0, dtype=torch.complex64, device="cuda")
        with pytest.raises(qce.QceError) as e:
            qce.cgemm_noalloc(h, "N", "N", m, n, k, A, m, A, k, C, m)
        assert e.value.status == 1 and "scratch" in str(e.value)
        torch.cuda.synchronize()
        assert bool((C == 7.0).all())  # nothing enqueued
    finally:
        h.close()
