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


def random_closed_network(seed, n_nodes=10, dmin=2, dmax=4):
    """Label sets of a connected random network without open legs: node
    degrees drawn in [dmin, dmax] (the paper's exploratory network: 10 nodes
    with 2 to 4 legs, Sec. 5.2), legs paired at random (no self-loops),
    redrawn until connected.  Returns a list of label tuples, one per node;
    label e joins exactly two nodes."""
    rng = np.random.default_rng(seed)
    while True:
        deg = rng.integers(dmin, dmax + 1, n_nodes)
        if deg.sum() % 2:
            continue
        stubs = np.repeat(np.arange(n_nodes), deg)
        rng.shuffle(stubs)
        edges = list(zip(stubs[0::2].tolist(), stubs[1::2].tolist()))
        if any(a == b for a, b in edges):
            continue
        parent = list(range(n_nodes))

        def find(i):
            while parent[i] != i:
                i = parent[i]
            return i
        for a, b in edges:
            parent[find(a)] = find(b)
        if len({find(i) for i in range(n_nodes)}) != 1:
            continue
        labels = [[] for _ in range(n_nodes)]
        for e, (a, b) in enumerate(edges):
            labels[a].append(e)
            labels[b].append(e)
        return [tuple(ls) for ls in labels]


TN_TYPES = (1, 2, 3)


def random_tn_tensor(shape, tn_type, rng):
    """Elements of the paper's random-network types (Sec. 5.2), complex64:
    type 1: each component N(0, 1e-4); type 2: type 1 scaled by 1e-6;
    type 3: type 2 with 10 to 20 randomly placed elements set to 1."""
    n = int(np.prod(shape)) if shape else 1
    t = np.empty(n, dtype=np.complex64)
    t.real = (rng.standard_normal(n) * 1e-2).astype(np.float32)
    t.imag = (rng.standard_normal(n) * 1e-2).astype(np.float32)
    if tn_type >= 2:
        t = (t.astype(np.complex128) * 1e-6).astype(np.complex64)
    if tn_type == 3:
        cnt = int(rng.integers(10, 21))
        t[rng.choice(n, size=min(cnt, n), replace=False)] = 1.0
    return t.reshape(shape)
