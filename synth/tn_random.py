"""Random tensor networks / pairwise contractions for parity tests.

``random_network(seed, ...)`` returns a single pairwise contraction problem
(A with labels la, B with labels lb, output labels lc) with random extents
and complex64 entries; the labels shared by A and B and absent from lc are
summed.  Tensors are dense row-major (C order).
"""
import numpy as np
from .gemm_inputs import _component


def random_network(seed, n_contracted=2, n_free_a=2, n_free_b=2, max_extent=4,
                   dist="a", shuffle_output=True, extents=None):
    rng = np.random.default_rng(seed)
    nl = n_contracted + n_free_a + n_free_b
    labels = [int(x) for x in rng.permutation(100)[:nl]]
    if extents is None:
        ext = {lab: int(rng.integers(1, max_extent + 1)) for lab in labels}
    else:
        ext = {lab: int(extents[i % len(extents)]) for i, lab in enumerate(labels)}
    kl = labels[:n_contracted]
    fa = labels[n_contracted:n_contracted + n_free_a]
    fb = labels[n_contracted + n_free_a:]
    la = list(kl + fa)
    lb = list(kl + fb)
    rng.shuffle(la)
    rng.shuffle(lb)
    lc = list(fa + fb)
    if shuffle_output:
        rng.shuffle(lc)

    def tensor(lbls):
        shape = tuple(ext[x] for x in lbls)
        n = int(np.prod(shape)) if shape else 1
        t = np.empty(n, dtype=np.complex64)
        t.real = _component(rng, dist, n).astype(np.float32)
        t.imag = _component(rng, dist, n).astype(np.float32)
        return t.reshape(shape)

    return {"A": tensor(la), "la": la, "B": tensor(lb), "lb": lb, "lc": lc,
            "extents": ext}
