"""GPU parity of the grouped CGEMM (qce_cgemm_grouped: uneven GEMMs in one
statistics, one split and one persistent GEMM launch, each entry with its
own device-side mode) and of grouped contractions (qce_contract inside a
group), through the C-ABI: integer inputs bit-exact against the FP64 oracle
in every mode, float entries bit-equal to the same GEMM run alone where the
k splits agree, per-entry decisions equal to the oracle's rule, emulated
values within the oracle's emulation bound, and graph replays equal to the
eager launch."""
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


def dev(a):
    return torch.from_numpy(np.asfortranarray(a).ravel(order="F").copy()).to("cuda")


def host(t, rows, cols, ld):
    flat = t.cpu().numpy()
    out = np.empty((rows, cols), dtype=np.complex64, order="F")
    for j in range(cols):
        out[:, j] = flat[j * ld:j * ld + rows]
    return out


def stored(m, n, k, opA, opB):
    sa = (m, k) if opA == "N" else (k, m)
    sb = (k, n) if opB == "N" else (n, k)
    return sa, sb


def op(X, o):
    return X if o == "N" else (X.T if o == "T" else X.conj().T)


class Case:
    """One GEMM of a group: stored operands, C with a padded leading dimension."""

    def __init__(self, m, n, k, dist, rng, opA="N", opB="N", alpha=1.0, beta=0.0, pad=0):
        self.m, self.n, self.k, self.opA, self.opB = m, n, k, opA, opB
        self.alpha, self.beta = alpha, beta
        sa, sb = stored(m, n, k, opA, opB)
        self.A = synth.random_matrix(sa[0], sa[1], dist, rng)
        self.B = synth.random_matrix(sb[0], sb[1], dist, rng)
        self.ldc = m + pad
        self.C0 = synth.random_matrix(m, n, "int", rng) if beta != 0 else np.zeros((m, n), np.complex64)

    def desc(self):
        sa, sb = stored(self.m, self.n, self.k, self.opA, self.opB)
        C0 = np.zeros((self.ldc, self.n), np.complex64)
        C0[:self.m] = self.C0
        self.dA, self.dB, self.dC = dev(self.A), dev(self.B), dev(C0)
        return {"opA": self.opA, "opB": self.opB, "m": self.m, "n": self.n, "k": self.k,
                "A": self.dA, "lda": max(1, sa[0]), "B": self.dB, "ldb": max(1, sb[0]),
                "C": self.dC, "ldc": self.ldc, "alpha": self.alpha, "beta": self.beta}

    def result(self):
        return host(self.dC, self.m, self.n, self.ldc)

    def exact(self):
        return oracle.cgemm(self.A, self.B, self.opA, self.opB, self.alpha, self.beta, self.C0)


def run_group(qce, h, cases, mode="auto"):
    h.set_mode(mode)
    descs = [c.desc() for c in cases]
    qce.cgemm_grouped(h, descs)
    torch.cuda.synchronize()
    decs = [h.batch_decision(i) for i in range(len(cases))]
    h.set_mode("auto")
    return [c.result() for c in cases], decs


def run_alone(qce, h, c, mode="auto"):
    h.set_mode(mode)
    d = c.desc()
    qce.cgemm(h, c.opA, c.opB, c.m, c.n, c.k, d["A"], d["lda"], d["B"], d["ldb"], d["C"], d["ldc"],
              c.alpha, c.beta)
    torch.cuda.synchronize()
    dec = h.last_decision()
    h.set_mode("auto")
    return c.result(), dec


# uneven matrix-core shapes (several tiles, ragged edges, a long-k entry that
# splits k, a short-k narrow entry), an irregular shape and k == 0
MIXED = [(200, 150, 96, "N", "N"), (130, 100, 3000, "T", "N"), (512, 64, 64, "N", "T"),
         (300, 257, 33, "C", "C"), (40, 300, 5, "N", "N"), (64, 70, 0, "N", "N"),
         (129, 33, 17, "T", "C"), (1000, 40, 520, "N", "N")]


@pytest.mark.parametrize("mode", ["auto", "fp16x2", "fp16x2_scaled", "bf16x3", "fp32"])
def test_integer_exact_every_mode(qce, h, mode):
    rng = np.random.default_rng(11)
    cases = [Case(m, n, k, "int", rng, oa, ob, alpha=(2 - 1j) if i == 1 else 1.0,
                  beta=(1 + 1j) if i in (1, 5) else 0.0, pad=i % 3)
             for i, (m, n, k, oa, ob) in enumerate(MIXED)]
    out, _ = run_group(qce, h, cases, mode)
    for i, c in enumerate(cases):
        assert np.array_equal(out[i].astype(np.complex128), c.exact()), (mode, i)


@pytest.mark.parametrize("tile", [64, 128])
def test_auto_mixed_modes_equal_alone(qce, h, tile):
    # one launch whose entries select FP16X2, FP16X2_SCALED, BF16X3 and FP32
    # on the device; every entry splits k alone as it does in the group (at
    # most 3 splits, capped by its k), so it equals the same GEMM run alone
    # bit for bit
    rng = np.random.default_rng(5 + tile)
    specs = [(300, 200, 96, "a"), (260, 130, 480, "b"), (150, 300, 200, "c"), (128, 128, 64, "u"),
             (97, 211, 45, "a")]
    cases = [Case(m, n, k, d, rng, pad=1) for m, n, k, d in specs]
    # one entry with large values: stage 1 fails on e_max > 14 -> scaled
    cases[3].A = (cases[3].A * 2.0 ** 20).astype(np.complex64)
    h.set_gemm_tile(tile)
    try:
        out, decs = run_group(qce, h, cases, "auto")
        for i, c in enumerate(cases):
            alone, dec1 = run_alone(qce, h, c, "auto")
            Aop, Bop = op(c.A, c.opA), op(c.B, c.opB)
            mode, sa, sb = oracle.select_mode(oracle.exp_stats(Aop), oracle.exp_stats(Bop))
            assert decs[i]["mode"] == mode == dec1["mode"], (i, decs[i], mode)
            assert (decs[i]["sA"], decs[i]["sB"]) == (sa, sb), i
            assert np.array_equal(out[i], alone), i
    finally:
        h.set_gemm_tile(0)
    got = sorted({d["mode"] for d in decs})
    assert got == [oracle.MODE_FP16X2, oracle.MODE_FP16X2_SCALED, oracle.MODE_BF16X3, oracle.MODE_FP32]


def test_emulation_bound_with_split_k(qce, h):
    # long k with few tiles: the group splits k; every entry stays within
    # the oracle's emulation value (4 u sqrt(k) relative) and within 2x the
    # FP32 mode's error against the exact product
    rng = np.random.default_rng(3)
    specs = [(128, 96, 4096, "a"), (64, 256, 2500, "b"), (200, 64, 3000, "u")]
    cases = [Case(m, n, k, d, rng) for m, n, k, d in specs]
    out, decs = run_group(qce, h, cases, "auto")
    out32, _ = run_group(qce, h, cases, "fp32")
    u = 2.0 ** -24
    for i, c in enumerate(cases):
        exact = c.exact()
        emu = oracle.emulated_cgemm(c.A, c.B, decs[i]["mode"], decs[i]["sA"], decs[i]["sB"])
        assert oracle.rel_fro(out[i], emu) <= 4 * u * np.sqrt(c.k), i
        assert oracle.rel_fro(out[i], exact) <= max(2 * oracle.rel_fro(out32[i], exact), 4 * u), i


def test_many_uneven_entries(qce, h):
    # 150 GEMMs of random shapes in one call (padding ids between entries,
    # both tiles' choice by the table), integer-exact
    rng = np.random.default_rng(21)
    cases = []
    for i in range(150):
        m, n = int(rng.integers(32, 260)), int(rng.integers(32, 260))
        k = int(rng.integers(16, 700))
        ops = ["N", "T", "C"]
        cases.append(Case(m, n, k, "int", rng, ops[i % 3], ops[(i // 3) % 3]))
    out, decs = run_group(qce, h, cases, "auto")
    for i, c in enumerate(cases):
        assert np.array_equal(out[i].astype(np.complex128), c.exact()), i
        assert decs[i]["mode"] == oracle.MODE_FP16X2, i


def test_single_entry_equals_alone_with_split(qce, h):
    # one entry: the group's tile and k splits are those of the GEMM alone
    rng = np.random.default_rng(8)
    c = Case(256, 192, 5000, "a", rng)
    out, dec = run_group(qce, h, [c], "auto")
    alone, dec1 = run_alone(qce, h, c, "auto")
    assert np.array_equal(out[0], alone)
    assert dec[0]["mode"] == dec1["mode"]


def test_empty_and_errors(qce, h):
    rng = np.random.default_rng(2)
    qce.cgemm_grouped(h, [])  # no-op
    good = Case(64, 64, 32, "int", rng)
    bad = Case(64, 64, 32, "int", rng)
    d0, d1 = good.desc(), bad.desc()
    d1["lda"] = 10  # < m
    before = d0["C"].clone()
    with pytest.raises(qce.QceError) as e:
        qce.cgemm_grouped(h, [d0, d1])
    assert "entry 1" in str(e.value)
    torch.cuda.synchronize()
    assert torch.equal(d0["C"], before)  # nothing enqueued
    # an entry with an empty output is skipped
    z = Case(64, 64, 32, "int", rng)
    dz = z.desc()
    dz["n"] = 0
    qce.cgemm_grouped(h, [dz, good.desc()])
    torch.cuda.synchronize()
    assert np.array_equal(good.result().astype(np.complex128), good.exact())


def test_graph_replays_equal_eager(qce, h):
    # the persistent launch clears its tile counters itself: replays of a
    # captured grouped call (on a handle of its own, as a captured pass
    # keeps its workspace and descriptors), with new inputs and eager work
    # in between, each equal the eager call on the same inputs
    rng = np.random.default_rng(9)
    cases = [Case(m, n, k, d, rng) for m, n, k, d in
             [(300, 200, 96, "a"), (130, 100, 3000, "b"), (256, 64, 64, "a")]]
    descs = [c.desc() for c in cases]
    hg = qce.Handle(0)
    try:
        qce.cgemm_grouped(hg, descs)  # eager once: workspace sized
        torch.cuda.synchronize()
        qce.group_reset(hg, 1 << 20)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            qce.cgemm_grouped(hg, descs)
        torch.cuda.synchronize()
        for rep in range(3):
            new = [Case(c.m, c.n, c.k, "a" if rep % 2 else "b", rng) for c in cases]
            for c, d in zip(new, descs):
                d["A"].copy_(dev(c.A))
                d["B"].copy_(dev(c.B))
            g.replay()
            torch.cuda.synchronize()
            got = [host(d["C"], c.m, c.n, c.ldc) for c, d in zip(cases, descs)]
            ref = [torch.zeros_like(d["C"]) for d in descs]
            qce.cgemm_grouped(h, [dict(d, C=r) for d, r in zip(descs, ref)])
            torch.cuda.synchronize()
            for i, (c, r) in enumerate(zip(cases, ref)):
                assert np.array_equal(got[i], host(r, c.m, c.n, c.ldc)), (rep, i)
        del g
    finally:
        hg.close()


def contract_cases(rng):
    """Contractions whose GEMMs take the panel path (outputs wider than 64
    or k above 128): operands already in GEMM order, an operand that needs a
    permute (extents 4, so no bit-permuted read), an output order that needs
    a permute, and batch labels (outermost, and not outermost)."""
    def tensor(shape):
        n = int(np.prod(shape))
        return synth.random_matrix(1, n, "int", rng).reshape(shape)
    out = []
    f_a, k_, f_b = list(range(0, 7)), list(range(7, 14)), list(range(14, 21))
    out.append((tensor((2,) * 14), f_a + k_, tensor((2,) * 14), k_ + f_b, f_b + f_a))
    la = [20, 30, 21, 31, 22, 32, 23]
    lb = [30, 31, 32, 40, 41, 42, 43]
    A4, B4 = tensor((4,) * 7), tensor((4,) * 7)
    out.append((A4, la, B4, lb, [40, 41, 42, 43, 20, 21, 22, 23]))
    out.append((A4, la, B4, lb, [20, 40, 21, 41, 22, 42, 23, 43]))
    bt, fa, kk, fb = [50, 51], list(range(60, 67)), list(range(70, 77)), list(range(80, 87))
    out.append((tensor((2,) * 16), bt + fa + kk, tensor((2,) * 16), bt + kk + fb, bt + fb + fa))
    out.append((tensor((2,) * 16), [fa[0]] + bt + fa[1:] + kk, tensor((2,) * 16), bt + kk + fb, bt + fb + fa))
    return out


def test_contract_group_equals_ungrouped_and_oracle(qce, h):
    rng = np.random.default_rng(4)
    cases = contract_cases(rng)
    h.set_mode("auto")
    h.set_size_policy(32, 32)  # every one of these takes statistics
    try:
        ins = [(torch.from_numpy(A.astype(np.complex64)).cuda(), la, torch.from_numpy(B.astype(np.complex64)).cuda(),
                lb, lc) for A, la, B, lb, lc in cases]
        alone = [qce.contract(h, dA, la, dB, lb, lc) for dA, la, dB, lb, lc in ins]
        torch.cuda.synchronize()
        alone = [a.cpu().numpy() for a in alone]
        with qce.group(h):
            grouped = [qce.contract(h, dA, la, dB, lb, lc) for dA, la, dB, lb, lc in ins]
        torch.cuda.synchronize()
        for i, ((A, la, B, lb, lc), g) in enumerate(zip(cases, grouped)):
            g = g.cpu().numpy()
            ref = oracle.zcontract(A.astype(np.complex64), la, B.astype(np.complex64), lb, lc)
            assert np.array_equal(g.astype(np.complex128), ref), i
            assert np.array_equal(g, alone[i]), i
    finally:
        h.set_size_policy(*h.default_size_policy)
