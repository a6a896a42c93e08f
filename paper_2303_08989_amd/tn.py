"""Host planning for circuit amplitudes: circuit -> tensor network ->
pairwise contraction path -> sliced labels (Sec. 2.2, Sec. 5.3).

Planning works on label structure only: every wire segment of the circuit is
one label of extent 2 shared by exactly two tensors.  No arithmetic of the
contraction happens here; the contractions run on the GPU (``executor``).

* ``circuit_network``: |0> vectors, gate tensors (rank 2k for a k-qubit
  gate, axes = outputs then inputs) and <x| vectors (Sec. 2.2).
* ``greedy_path``: repeatedly contract the pair of connected tensors whose
  contraction grows the network least, size(out) - size(a) - size(b), ties
  broken by smaller flop count; optional random perturbation for restarts.
  (The paper uses cotengra's hyper-optimised search, Sec. 5.1; this is the
  project's own greedy order.)
* ``subtree_reconfigure``: local re-optimisation of a path: every subtree cut
  at a frontier of up to 8 tensors is re-ordered optimally (dynamic
  programming over subsets) for its largest intermediate, then flops.
* ``choose_slices``: labels whose removal from every intermediate brings the
  largest intermediate under a bound, picked greedily by total cost
  (slicing, Sec. 5.3).
"""
import heapq
import math
import random

import numpy as np


def circuit_network(circuit, x):
    """Leaves [(array complex64, labels)] of <x|U|0...0> for an n-qubit circuit.

    Qubit q is bit n-1-q of x.  A gate's tensor has axes (outputs..., inputs...)
    taken from its 2^k x 2^k matrix in the basis |b1 ... bk> with b1 the bit of
    the first listed qubit.
    """
    n = circuit["n"]
    leaves = []
    nxt = [0]

    def fresh():
        nxt[0] += 1
        return nxt[0] - 1

    wire = [fresh() for _ in range(n)]
    for q in range(n):
        leaves.append((np.array([1, 0], dtype=np.complex64), (wire[q],)))
    for g in circuit["gates"]:
        qs = list(g["qubits"])
        k = len(qs)
        t = np.asarray(g["matrix"]).astype(np.complex64).reshape((2,) * (2 * k))
        outs = [fresh() for _ in qs]
        leaves.append((t, tuple(outs) + tuple(wire[q] for q in qs)))
        for q, o in zip(qs, outs):
            wire[q] = o
    for q in range(n):
        bit = (int(x) >> (n - 1 - q)) & 1
        v = np.zeros(2, dtype=np.complex64)
        v[bit] = 1
        leaves.append((v, (wire[q],)))
    return leaves


def fix_labels(arr, labels, values):
    """The sub-array of ``arr`` (axes named by ``labels``) with each label in
    ``values`` fixed to the index given there: a C-contiguous copy keeping the
    other axes in order (0-d when every label is fixed)."""
    idx = tuple(values[lab] if lab in values else slice(None) for lab in labels)
    sub = np.asarray(arr[idx])
    return np.ascontiguousarray(sub).reshape(sub.shape)


def _lsize(labels, sliced=frozenset()):
    return sum(1 for lab in labels if lab not in sliced)


def greedy_path(label_sets, seed=None, noise=0.0, alpha=1.0):
    """Pairwise contraction order for a network whose labels each join two
    tensors.  Returns [(i, j)] in SSA numbering (leaves 0..L-1, the result of
    step s is tensor L+s).  The cost of a candidate pair is
    size(out) - alpha * (size(a) + size(b)); with ``seed``/``noise`` it is
    perturbed by Gumbel noise for randomised restarts."""
    rng = random.Random(seed)
    tens = {i: frozenset(ls) for i, ls in enumerate(label_sets)}
    owner = {}
    for i, ls in tens.items():
        for lab in ls:
            owner.setdefault(lab, []).append(i)
    nid = len(label_sets)
    heap = []

    def cost(a, b):
        la, lb = tens[a], tens[b]
        out = la ^ lb
        c = 2.0 ** len(out) - alpha * (2.0 ** len(la) + 2.0 ** len(lb))
        fl = 2.0 ** len(la | lb)
        if noise:
            g = -math.log(-math.log(rng.random() + 1e-300) + 1e-300)
            c = c - noise * g * abs(c + 1.0)
        return (c, fl, min(a, b), max(a, b))

    def push_pairs(a):
        seen = set()
        for lab in tens[a]:
            for b in owner.get(lab, ()):
                if b != a and b in tens and b not in seen:
                    seen.add(b)
                    heapq.heappush(heap, (cost(a, b), a, b))

    for i in list(tens):
        push_pairs(i)
    path = []
    while len(tens) > 1:
        while heap:
            _, a, b = heapq.heappop(heap)
            if a in tens and b in tens:
                break
        else:
            # disconnected components: contract the two smallest (outer product)
            a, b = sorted(tens, key=lambda i: (len(tens[i]), i))[:2]
        la, lb = tens.pop(a), tens.pop(b)
        out = la ^ lb
        c = nid
        nid += 1
        tens[c] = out
        for lab in la & lb:
            owner.pop(lab, None)
        for lab in out:
            owner[lab] = [c if t in (a, b) else t for t in owner[lab]]
        path.append((a, b))
        push_pairs(c)
    return path


def subtree_reconfigure(label_sets, path, frontier=8, passes=4):
    """Locally optimal re-ordering of a contraction tree.

    For every node, largest tensor first, the subtree below it is cut at a
    frontier of up to ``frontier`` tensors (expanding the largest internal
    tensor each time) and the frontier's best contraction order is found by
    dynamic programming over its subsets, ranked by (largest intermediate,
    flops); a better order replaces the subtree.  Repeated for ``passes``
    sweeps or until nothing changes.  Structure only: every label joins two
    tensors, so the labels of a merged subset are the symmetric difference
    of its members' labels.  Returns a new SSA path with the same leaves."""
    L = len(label_sets)
    children = {L + s: (a, b) for s, (a, b) in enumerate(path)}
    labs = {i: frozenset(ls) for i, ls in enumerate(label_sets)}
    for v in sorted(children):
        a, b = children[v]
        labs[v] = labs[a] ^ labs[b]
    nid = L + len(path)

    def subtree_cost(v, stop):
        if v in stop:
            return (0, 0.0)
        a, b = children[v]
        wa, fa = subtree_cost(a, stop)
        wb, fb = subtree_cost(b, stop)
        return (max(wa, wb, len(labs[v])), fa + fb + 2.0 ** len(labs[a] | labs[b]))

    def remove(v, stop):
        if v in stop:
            return
        a, b = children.pop(v)
        remove(a, stop)
        remove(b, stop)

    for _ in range(passes):
        changed = 0
        for root in sorted(children, key=lambda v: (-len(labs[v]), v)):
            if root not in children:
                continue
            front = [root]
            while len(front) < frontier:
                inner = [v for v in front if v in children]
                if not inner:
                    break
                v = max(inner, key=lambda x: (len(labs[x]), x))
                front.remove(v)
                front.extend(children[v])
            n = len(front)
            if n < 3:
                continue
            col = {}
            for v in front:
                for lab in labs[v]:
                    col.setdefault(lab, len(col))
            bits = [sum(1 << col[lab] for lab in labs[v]) for v in front]
            lab_of = [0] * (1 << n)
            for S in range(1, 1 << n):
                low = S & -S
                lab_of[S] = lab_of[S ^ low] ^ bits[low.bit_length() - 1]
            best = [None] * (1 << n)
            for i in range(n):
                best[1 << i] = ((0, 0.0), None)
            for S in range(1, 1 << n):
                if S & (S - 1) == 0:
                    continue
                size = bin(lab_of[S]).count("1")
                pick = None
                sub = (S - 1) & S
                while sub:
                    other = S ^ sub
                    if sub < other:
                        (wa, fa), _ = best[sub]
                        (wb, fb), _ = best[other]
                        key = (max(wa, wb, size), fa + fb + 2.0 ** bin(lab_of[sub] | lab_of[other]).count("1"))
                        if pick is None or key < pick[0]:
                            pick = (key, (sub, other))
                    sub = (sub - 1) & S
                best[S] = pick
            full = (1 << n) - 1
            stop = set(front)
            if not best[full][0] < subtree_cost(root, stop):
                continue
            remove(root, stop)

            def build(S):
                nonlocal nid
                if S & (S - 1) == 0:
                    return front[S.bit_length() - 1]
                a, b = best[S][1]
                va, vb = build(a), build(b)
                if S == full:
                    v = root
                else:
                    v = nid
                    nid += 1
                children[v] = (va, vb)
                labs[v] = labs[va] ^ labs[vb]
                return v

            build(full)
            changed += 1
        if not changed:
            break
    # back to SSA numbering, children before parents
    kids = {x for ab in children.values() for x in ab}
    roots = [v for v in children if v not in kids]
    ren = {i: i for i in range(L)}
    out = []
    stack = [(r, False) for r in sorted(roots)]
    while stack:
        v, done = stack.pop()
        if v < L:
            continue
        if done:
            a, b = children[v]
            out.append((ren[a], ren[b]))
            ren[v] = L + len(out) - 1
        else:
            stack.append((v, True))
            a, b = children[v]
            stack.append((b, False))
            stack.append((a, False))
    return out


def tree_labels(label_sets, path):
    """Labels of every SSA tensor (leaves then intermediates)."""
    labs = [frozenset(ls) for ls in label_sets]
    for a, b in path:
        labs.append(labs[a] ^ labs[b])
    return labs


def path_cost(label_sets, path, sliced=frozenset()):
    """(max log2 intermediate size, total effective flops per slice, steps)
    with `sliced` labels removed everywhere."""
    labs = tree_labels(label_sets, path)
    L = len(label_sets)
    maxlog = 0
    flops = 0.0
    steps = []
    for s, (a, b) in enumerate(path):
        la, lb = labs[a] - sliced, labs[b] - sliced
        out = labs[L + s] - sliced
        maxlog = max(maxlog, len(out))
        k = len(la & lb)
        m, n = len(la - lb), len(lb - la)
        flops += 8.0 * 2.0 ** (m + n + k)
        steps.append((m, n, k))
    return maxlog, flops, steps


def _step_matrices(label_sets, path):
    """Boolean matrices (steps x labels): labels of each step's output and of
    the union of its two operands."""
    labs = tree_labels(label_sets, path)
    L = len(label_sets)
    universe = sorted(set().union(*labs[:L]))
    col = {lab: i for i, lab in enumerate(universe)}
    out = np.zeros((len(path), len(universe)), dtype=bool)
    uni = np.zeros((len(path), len(universe)), dtype=bool)
    for s, (a, b) in enumerate(path):
        for lab in labs[L + s]:
            out[s, col[lab]] = True
        for lab in labs[a] | labs[b]:
            uni[s, col[lab]] = True
    return universe, out, uni


def choose_slices(label_sets, path, max_log2, max_slices=None):
    """Greedy slicing: while the largest intermediate exceeds 2^max_log2,
    slice the label (among those of the largest intermediates) that gives the
    smallest total flops over all slices."""
    universe, out, uni = _step_matrices(label_sets, path)
    keep = np.ones(len(universe), dtype=bool)
    sliced = []
    while True:
        osz = (out & keep).sum(axis=1)
        maxlog = int(osz.max()) if len(osz) else 0
        if maxlog <= max_log2 or (max_slices is not None and len(sliced) >= max_slices):
            return sorted(universe[i] for i in sliced)
        usz = (uni & keep).sum(axis=1)
        cands = np.nonzero((out[osz == maxlog] & keep).any(axis=0))[0]
        # for each candidate: new max output size and total flops over all slices
        o_c = osz[:, None] - out[:, cands]
        u_c = usz[:, None] - uni[:, cands]
        new_max = o_c.max(axis=0)
        new_fl = np.exp2(u_c.astype(np.float64)).sum(axis=0) * 2.0 ** (len(sliced) + 1)
        order = np.lexsort((cands, new_fl, new_max))
        best = int(cands[order[0]])
        keep[best] = False
        sliced.append(best)


def slice_dependencies(label_sets, path, sliced):
    """Sliced labels each SSA tensor depends on (those of its leaves)."""
    S = set(sliced)
    deps = [frozenset(l for l in ls if l in S) for ls in label_sets]
    for a, b in path:
        deps.append(deps[a] | deps[b])
    return deps


def order_sliced(label_sets, path, sliced):
    """Sliced labels ordered so that the ones entering the tree latest come
    first (they are the ones varied fastest by a run over slice ids)."""
    deps = slice_dependencies(label_sets, path, sliced)
    L = len(label_sets)
    first = {}
    for s in range(len(path)):
        for lab in deps[L + s]:
            first.setdefault(lab, s)
    return sorted(sliced, key=lambda lab: (-first.get(lab, 0), lab))


def memoized_cost(label_sets, path, sliced, n_varied):
    """Effective flops of a run over slice ids [0, 2^n_varied) when a node is
    recomputed only when a varied sliced label it depends on changes."""
    ordered = order_sliced(label_sets, path, sliced)
    V = frozenset(ordered[:n_varied])
    S = frozenset(sliced)
    deps = slice_dependencies(label_sets, path, sliced)
    labs = tree_labels(label_sets, path)
    L = len(label_sets)
    tot = 0.0
    for s, (a, b) in enumerate(path):
        u = (labs[a] | labs[b]) - S
        tot += 2.0 ** len(deps[L + s] & V) * 8.0 * 2.0 ** len(u)
    return tot * 2.0 ** max(0, n_varied - len(sliced))


def best_greedy(label_sets, restarts=8, max_log2=None, seed=0, noises=(0.1, 0.3, 1.0), alphas=(1.0,),
                reconfigure=False):
    """Best of one deterministic greedy path and `restarts` randomised ones,
    for each size weight alpha of the greedy cost.  ``reconfigure``: True
    re-orders every candidate by ``subtree_reconfigure``, "best" only the
    chosen one (kept if it ranks better).  With a size bound, each path is
    sliced to it and ranked by the memoized cost of the whole amplitude
    (every slice); without, by (max intermediate, flops)."""
    def ranked(p):
        if max_log2 is None:
            ml, fl, _ = path_cost(label_sets, p)
            return (ml, fl), p, []
        sl = choose_slices(label_sets, p, max_log2)
        return (memoized_cost(label_sets, p, sl, len(sl)), len(sl)), p, sl

    best = None
    for r, alpha in ((r, a) for r in range(restarts + 1) for a in alphas):
        noise = 0.0 if r == 0 else noises[r % len(noises)]
        p = greedy_path(label_sets, seed=seed + r, noise=noise, alpha=alpha)
        if reconfigure is True:
            p = subtree_reconfigure(label_sets, p)
        cand = ranked(p)
        if best is None or cand[0] < best[0]:
            best = cand
    if reconfigure == "best":
        cand = ranked(subtree_reconfigure(label_sets, best[1]))
        if cand[0] < best[0]:
            best = cand
    return best[1], best[2]
