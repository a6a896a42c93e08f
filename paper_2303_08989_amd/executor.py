"""Sliced contraction of a circuit's tensor network on the GPU (Sec. 2.2,
Sec. 5.3): the slice loop with an FP64 device sum of the slice amplitudes.

Every pairwise contraction goes through the library's ``qce_contract``
(TTGT: device permutes when needed, then the emulated CGEMM under the size
policy); the per-slice scalars are added in FP64 on the device
(``qce_accumulate_f64``).  Host work here is planning and input marshalling:
the leaves (gate matrices, |0> and <x| vectors) are built on the host, and a
slice fixes chosen labels by selecting entries of the leaves that carry them
(every variant is uploaded before contraction starts).

Slices: with sliced labels s_0 .. s_{S-1}, slice id sigma assigns
s_i = (sigma >> i) & 1.  The labels varied by a run over slice ids
[0, 2^V) are s_0 .. s_{V-1}; the planner orders them so that those labels
enter the contraction tree as late as possible.  A node's result is kept
between slices while the slice labels it depends on are unchanged and its
parent will need it again (its sibling depends on a label it does not).
"""
from contextlib import nullcontext

import numpy as np

from . import tn


class CircuitPlan:
    """Planning (structure only, independent of the bitstring)."""

    def __init__(self, circuit, max_log2=28, restarts=8, seed=0, varied=6, path=None, sliced=None,
                 alphas=(1.0, 1.5), noises=(0.1, 0.3), reconfigure=True):
        self.circuit = circuit
        leaves = tn.circuit_network(circuit, 0)
        self.label_sets = [tuple(l) for _, l in leaves]
        L = len(self.label_sets)
        if path is None:
            path, sl = tn.best_greedy(self.label_sets, restarts=restarts, max_log2=max_log2, seed=seed,
                                      alphas=alphas, noises=noises, reconfigure=reconfigure)
            if sliced is None:
                sliced = sl
        self.path = list(path)
        sliced = list(sliced or [])
        labs = tn.tree_labels(self.label_sets, self.path)
        S = set(sliced)
        deps = [frozenset(l for l in self.label_sets[i] if l in S) for i in range(L)]
        for a, b in self.path:
            deps.append(deps[a] | deps[b])
        # sliced labels entering the tree latest vary fastest
        self.sliced = tn.order_sliced(self.label_sets, self.path, sliced)
        self.varied = self.sliced[:min(varied, len(self.sliced))]
        self.deps = deps
        self.labels = [tuple(x for x in self.label_sets[i] if x not in S) for i in range(L)]
        self.parent = {}
        for s, (a, b) in enumerate(self.path):
            self.parent[a] = (L + s, b)
            self.parent[b] = (L + s, a)
        ml, fl, steps = tn.path_cost(self.label_sets, self.path, frozenset(self.sliced))
        self.max_log2 = ml
        self.flops_per_slice = fl
        self.gemm_shapes = steps  # log2 (m, n, k) per step
        self.varied_cost = tn.memoized_cost(self.label_sets, self.path, self.sliced, len(self.varied))
        self.total_cost = tn.memoized_cost(self.label_sets, self.path, self.sliced, len(self.sliced))

    @property
    def n_slices(self):
        return 1 << len(self.sliced)


def batched_pass_estimate(plan, n_batch, flops_per_s=150e12, bytes_per_s=4e12, launch_s=2e-6):
    """Estimated device seconds of one ``BatchedExecutor`` pass of ``plan``
    with its first ``n_batch`` sliced labels kept as batch labels: per step
    the larger of its flop time (8 m n k per entry) and the time to read both
    operands and write the result, plus one launch.  Used to choose between
    contraction orders for the batched pass, whose intermediates carry the
    batch labels (so an order that is best per slice need not be best
    batched)."""
    batch = set(plan.sliced[:n_batch])
    outer = set(plan.sliced[n_batch:])
    labs = [frozenset(ls) - outer for ls in plan.label_sets]
    total = 0.0
    for a, b in plan.path:
        la, lb = labs[a], labs[b]
        shared = la & lb
        out = (la ^ lb) | (shared & batch)
        labs.append(out)
        m, n = 2.0 ** len(la - shared), 2.0 ** len(lb - shared)
        k, count = 2.0 ** len(shared - batch), 2.0 ** len(shared & batch)
        flops = 8.0 * m * n * k * count
        nbytes = 8.0 * (2.0 ** len(la) + 2.0 ** len(lb) + 2.0 ** len(out))
        total += max(flops / flops_per_s, nbytes / bytes_per_s) + launch_s
    return total


def plan_for_batching(circuit, max_log2, n_batch, restarts=4, seed=0):
    """The contraction order for batched passes: the plain greedy search
    and its best candidate re-ordered by subtree reconfiguration are both
    planned, and the one with the smaller ``batched_pass_estimate`` is
    returned (with its estimate in ``plan.batched_estimate``)."""
    cands = [CircuitPlan(circuit, max_log2=max_log2, restarts=restarts, seed=seed, varied=n_batch,
                         alphas=(1.0,), noises=(0.1, 0.3, 1.0), reconfigure=False),
             CircuitPlan(circuit, max_log2=max_log2, restarts=restarts, seed=seed, varied=n_batch,
                         reconfigure="best")]
    for p in cands:
        p.batched_estimate = batched_pass_estimate(p, n_batch)
    return min(cands, key=lambda p: p.batched_estimate)


def level_batches(path, n_leaves, steps):
    """The path steps `steps` (ascending) in tree levels: a step is one level
    above the highest of its operands computed among `steps` (leaves and
    nodes computed earlier count as level 0), so the steps of one level are
    independent of each other and every operand of a level is ready before
    it.  Returns the levels in order, each a list of steps in path order."""
    lev = {}
    for s in steps:
        a, b = path[s]
        lev[n_leaves + s] = 1 + max(lev.get(a, 0), lev.get(b, 0))
    levels = {}
    for s in steps:
        levels.setdefault(lev[n_leaves + s], []).append(s)
    return [levels[k] for k in sorted(levels)]


class Executor:
    """Runs a CircuitPlan on one GPU through the C-ABI.  (`device` "cpu" is
    for tests of the host logic with a stand-in contraction.)"""

    def __init__(self, handle, plan, device="cuda"):
        import torch
        self.torch = torch
        self.h = handle
        self.plan = plan
        self.device = device
        self._out_labels = {}

    def _leaf_variants(self, x):
        """Device tensors of every leaf for bitstring x, with all variants of
        leaves that carry sliced labels: {(leaf, values): tensor}.  They are
        views of one device buffer filled by a single host-to-device copy."""
        torch = self.torch
        p = self.plan
        leaves = tn.circuit_network(p.circuit, x)
        S = p.sliced
        pos = {lab: i for i, lab in enumerate(S)}
        host = []
        for i, (arr, labels) in enumerate(leaves):
            sl = [lab for lab in labels if lab in pos]
            if not sl:
                host.append(((i, ()), np.ascontiguousarray(arr)))
                continue
            for vals in np.ndindex(*(2,) * len(sl)):
                host.append(((i, tuple(vals)), tn.fix_labels(arr, labels, dict(zip(sl, vals)))))
        flat = np.concatenate([a.reshape(-1) for _, a in host]).astype(np.complex64, copy=False)
        dev = torch.from_numpy(flat).to(self.device)
        out = {}
        off = 0
        for key, a in host:
            out[key] = dev[off:off + a.size].view(a.shape)
            off += a.size
        return out

    def amplitude(self, x, slice_ids=None, acc=None, slice_out=None, grouped=True):
        """Sum over `slice_ids` (default: all) of the sliced network values,
        accumulated in FP64 on the device.  Returns the device float64[2]
        accumulator.  `slice_out` (device complex64, one entry per slice id)
        optionally receives each slice's value.  `grouped`: the recomputed
        steps of a slice run level by level (a step one level above the
        recomputed steps it consumes), each level inside one library group,
        so that its small contractions share one launch; otherwise in path
        order, one launch each."""
        import paper_2303_08989_amd as qce
        torch = self.torch
        p = self.plan
        if slice_ids is None:
            slice_ids = range(p.n_slices)
        if acc is None:
            acc = torch.zeros(2, dtype=torch.float64, device=self.device)
        leaves = self._leaf_variants(x)
        L = len(p.label_sets)
        pos = {lab: i for i, lab in enumerate(p.sliced)}
        cache = {}  # node -> (key, tensor)
        root = L + len(p.path) - 1 if p.path else None
        children = {L + s: (a, b) for s, (a, b) in enumerate(p.path)}
        varied = set(p.varied)
        n_done = 0
        for sigma in slice_ids:
            val = {lab: (sigma >> i) & 1 for lab, i in pos.items()}

            def key_of(node):
                return tuple(val[lab] for lab in sorted(p.deps[node]))

            def leaf(i):
                sl = [lab for lab in p.label_sets[i] if lab in pos]
                return leaves[(i, tuple(val[lab] for lab in sl))]

            if root is None:
                qce.accumulate_f64(self.h, leaf(0).reshape(-1)[:1], acc)
                if slice_out is not None:
                    slice_out[n_done:n_done + 1].copy_(leaf(0).reshape(-1)[:1])
                n_done += 1
                continue
            # nodes to (re)compute this slice: top-down from the root, a node
            # is needed when its parent is recomputed and it is not cached
            # with the current values of the slice labels it depends on
            need = set()
            stack = [root]
            while stack:
                node = stack.pop()
                hit = cache.get(node)
                if node != root and hit is not None and hit[0] == key_of(node):
                    continue
                need.add(node)
                for ch in children[node]:
                    if ch >= L:
                        stack.append(ch)
            vals = {}
            order = [s for s in range(len(p.path)) if L + s in need]
            batches = level_batches(p.path, L, order) if grouped else [[s] for s in order]
            for steps in batches:
                with (qce.group(self.h) if grouped and self.device != "cpu" else nullcontext()):
                    for s in steps:
                        self._step(s, leaf, vals, cache, key_of, varied)
            qce.accumulate_f64(self.h, vals[root].reshape(-1)[:1], acc)
            if slice_out is not None:
                slice_out[n_done:n_done + 1].copy_(vals[root].reshape(-1)[:1])
            n_done += 1
        return acc

    def _step(self, s, leaf, vals, cache, key_of, varied):
        """Contraction step s of the path for the current slice."""
        import paper_2303_08989_amd as qce
        p = self.plan
        L = len(p.label_sets)
        node = L + s
        a, b = p.path[s]
        ta = leaf(a) if a < L else (vals.pop(a) if a in vals else cache[a][1])
        tb = leaf(b) if b < L else (vals.pop(b) if b in vals else cache[b][1])
        la = p.labels[a] if a < L else self._out_labels[a]
        lb = p.labels[b] if b < L else self._out_labels[b]
        shared = set(la) & set(lb)
        lc = [lab for lab in lb if lab not in shared] + [lab for lab in la if lab not in shared]
        self._out_labels[node] = tuple(lc)
        out = qce.contract(self.h, ta, list(la), tb, list(lb), lc)
        vals[node] = out
        # keep when the parent will be recomputed while this node
        # stays the same (its sibling depends on a varied label it
        # does not depend on)
        par = p.parent.get(node)
        if par is not None and (p.deps[par[1]] - p.deps[node]) & varied:
            cache[node] = (key_of(node), out)
        elif node in cache:
            del cache[node]


class BatchedExecutor:
    """Runs a CircuitPlan with the first ``n_batch`` sliced labels (those
    entering the tree latest) kept as batch labels instead of fixed: one
    pass over the tree computes the 2^n_batch slices that differ only in
    those labels, every contraction being one batched GEMM over the batch
    labels both operands carry (``qce_contract`` with batch labels; a node
    that depends on no batch label is computed once, which is the
    memoization of ``Executor`` for free).  The root is the tensor of the
    pass's slice values, summed in FP64 on the device.  The remaining sliced
    labels are looped over ("outer" slices): outer value o covers slice ids
    [o * 2^n_batch, (o + 1) * 2^n_batch) of ``Executor``."""

    def __init__(self, handle, plan, n_batch, device="cuda"):
        import torch
        self.torch = torch
        self.device = device
        self.h = handle
        self.plan = plan
        self.n_batch = min(int(n_batch), len(plan.sliced))
        self.batch_labels = list(plan.sliced[:self.n_batch])
        self.outer_labels = list(plan.sliced[self.n_batch:])
        self._bpos = {lab: i for i, lab in enumerate(self.batch_labels)}

    @property
    def n_outer(self):
        return 1 << len(self.outer_labels)

    def max_intermediate(self):
        """log2 of the largest tensor of a pass (elements)."""
        p = self.plan
        L = len(p.label_sets)
        B = set(self.batch_labels)
        outer = set(self.outer_labels)
        labs = [frozenset(ls) - outer for ls in p.label_sets]
        best = max((len(x) for x in labs), default=0)
        for a, b in p.path:
            out = (labs[a] ^ labs[b]) | (labs[a] & labs[b] & B)
            labs.append(out)
            best = max(best, len(out))
        return best

    def _leaves(self, x, o, cache=None):
        """Device leaves for bitstring x with the outer labels fixed by o."""
        return self._leaves_and_xbuf(x, o, cache)[0]

    def _leaves_and_xbuf(self, x, o, cache=None):
        """``_leaves`` and the one device buffer the <x| leaves (the last n)
        are views of: they go up in one host-to-device copy."""
        torch = self.torch
        p = self.plan
        opos = {lab: i for i, lab in enumerate(self.outer_labels)}
        leaves = tn.circuit_network(p.circuit, x)
        first_x = len(leaves) - p.circuit["n"]
        out = []
        xs = []
        for i, (arr, labels) in enumerate(leaves):
            fixed = {lab: (o >> opos[lab]) & 1 for lab in labels if lab in opos}
            kept = [lab for lab in labels if lab not in opos]
            if i >= first_x:
                xs.append((tn.fix_labels(arr, labels, fixed), kept))
                continue
            key = (i, tuple(fixed[lab] for lab in labels if lab in opos))
            if cache is not None and key in cache:
                t = cache[key]
            else:
                t = torch.from_numpy(tn.fix_labels(arr, labels, fixed)).to(self.device)
                if cache is not None:
                    cache[key] = t           # gate and |0> leaves do not depend on x
            out.append((t, kept))
        flat = None
        if xs:
            flat = torch.from_numpy(np.concatenate([a.reshape(-1) for a, _ in xs])).to(self.device)
            off = 0
            for a, kept in xs:
                out.append((flat[off:off + a.size].view(a.shape), kept))
                off += a.size
        return out, flat

    def _levels(self):
        """Contraction steps grouped by tree level (a step's level is one more
        than its children's): the steps of one level are independent."""
        p = self.plan
        L = len(p.label_sets)
        lev = [0] * L
        groups = {}
        for s, (a, b) in enumerate(p.path):
            lev.append(1 + max(lev[a], lev[b]))
            groups.setdefault(lev[-1], []).append(s)
        return [groups[k] for k in sorted(groups)]

    def run_pass(self, leaves, grouped=True):
        """One pass over the tree on the given device leaves; returns the root
        tensor and its labels (a subset of the batch labels).  ``grouped``:
        the steps of each tree level run inside one library group, so their
        small contractions share one launch."""
        import paper_2303_08989_amd as qce
        p = self.plan
        L = len(p.label_sets)
        B = self._bpos
        vals = {i: leaves[i] for i in range(L)}

        def step(s):
            a, b = p.path[s]
            ta, la = vals.pop(a)
            tb, lb = vals.pop(b)
            shared = set(la) & set(lb)
            bt = sorted((lab for lab in shared if lab in B), key=lambda lab: B[lab])
            lc = bt + [lab for lab in lb if lab not in shared] + [lab for lab in la if lab not in shared]
            vals[L + s] = (qce.contract(self.h, ta, list(la), tb, list(lb), lc), lc)

        if grouped and self.device != "cpu":
            for level in self._levels():
                with qce.group(self.h):
                    for s in level:
                        step(s)
        else:
            for s in range(len(p.path)):
                step(s)
        return vals[L + len(p.path) - 1] if p.path else vals[0]

    def amplitude(self, x, outer_ids=None, acc=None, cache=None, grouped=True):
        """Sum over the outer slices ``outer_ids`` (default: all) of the
        batched passes, accumulated in FP64 on the device; returns the
        float64[2] accumulator."""
        import paper_2303_08989_amd as qce
        torch = self.torch
        if acc is None:
            acc = torch.zeros(2, dtype=torch.float64, device=self.device)
        if outer_ids is None:
            outer_ids = range(self.n_outer)
        for o in outer_ids:
            root, _ = self.run_pass(self._leaves(x, o, cache), grouped)
            qce.accumulate_n_f64(self.h, root.reshape(-1), acc)
        return acc


class GraphPass:
    """One batched pass (``BatchedExecutor``) captured once in a HIP graph
    and replayed per bitstring and outer value.  Between replays only leaf
    data changes, overwritten in place by host-to-device copies from pinned
    memory outside the graph: the <x| leaves per bitstring, and the leaves
    that carry outer labels (fixed to the outer value's bits) when the outer
    value changes (``set_outer``).

    The graph owns a handle of its own, so its workspace (whose address the
    captured kernels hold) is never reallocated by other calls; a warm-up
    pass sizes it before capture.  No memset is captured: the accumulator is
    cleared by a fill kernel inside the graph."""

    def __init__(self, plan, n_batch, outer=0, device=0, mode=None):
        import torch
        import paper_2303_08989_amd as qce
        self.torch = torch
        self.qce = qce
        self.h = qce.Handle(device)
        if mode is not None:
            self.h.set_mode(mode)        # fixed for the captured pass
        self.bx = BatchedExecutor(self.h, plan, n_batch)
        self.outer = outer
        self.n = plan.circuit["n"]
        self._opos = {lab: i for i, lab in enumerate(self.bx.outer_labels)}
        # The <x| leaves are views of one device buffer, refilled per
        # bitstring by one copy from pinned memory.  Per qubit: its offset in
        # the buffer and, if its final wire is an outer label, that label's
        # index among the outer labels (the leaf is then a scalar fixed by
        # the outer value's bit).
        self.leaves, self.xbuf = self.bx._leaves_and_xbuf(0, outer)
        net = tn.circuit_network(plan.circuit, 0)
        wires = [labels[0] for _, labels in net[-self.n:]] if self.n else []
        self.xslots = []
        off = 0
        for w in wires:
            bit = self._opos.get(w)
            self.xslots.append((off, bit))
            off += 1 if bit is not None else 2
        assert self.n == 0 or off == self.xbuf.numel()
        self.xhost = torch.zeros(max(off, 1), dtype=torch.complex64, pin_memory=True)
        self.xdone = torch.cuda.Event()
        self.xdone.record()
        # the gate leaves that carry outer labels become views of a second
        # buffer, refilled by set_outer: (leaf, offset, elements)
        first_x = len(net) - self.n
        self._gates = [(arr, labels) for arr, labels in net[:first_x]]
        self.oslots, total = [], 0
        for i, (arr, labels) in enumerate(self._gates):
            if any(lab in self._opos for lab in labels):
                t = self.leaves[i][0]
                self.oslots.append((i, total, t.numel()))
                total += t.numel()
        self.obuf = torch.zeros(max(total, 1), dtype=torch.complex64, device="cuda")
        for i, off, size in self.oslots:
            t, kept = self.leaves[i]
            view = self.obuf[off:off + size].view(t.shape)
            view.copy_(t)
            self.leaves[i] = (view, kept)
        self.ohost = torch.zeros(max(total, 1), dtype=torch.complex64, pin_memory=True)
        self.odone = torch.cuda.Event()
        self.odone.record()
        self.acc = torch.zeros(2, dtype=torch.float64, device="cuda")
        root, _ = self.bx.run_pass(self.leaves)            # warm-up: workspace, allocator
        torch.cuda.synchronize()
        qce.group_reset(self.h, 64 << 20)                   # room for the captured groups' descriptors
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self.acc.zero_()
            root, _ = self.bx.run_pass(self.leaves)
            qce.accumulate_n_f64(self.h, root.reshape(-1), self.acc)
        self.root = root

    @property
    def n_outer(self):
        return self.bx.n_outer

    def set_outer(self, outer):
        """Outer value for the following replays: the leaves that carry outer
        labels are refilled (one copy) for slice ids [outer * 2^b, (outer +
        1) * 2^b), b the number of batch labels."""
        if not 0 <= int(outer) < self.n_outer:
            raise ValueError(f"outer value {outer} outside [0, {self.n_outer})")
        outer = int(outer)
        if self.oslots:
            self.odone.synchronize()          # the previous copy has read the pinned buffer
            hv = self.ohost.numpy()
            for i, off, size in self.oslots:
                arr, labels = self._gates[i]
                fixed = {lab: (outer >> self._opos[lab]) & 1 for lab in labels if lab in self._opos}
                hv[off:off + size] = tn.fix_labels(arr, labels, fixed).reshape(-1)
            self.obuf.copy_(self.ohost[: self.obuf.numel()], non_blocking=True)
            self.odone.record()
        self.outer = outer

    def amplitude(self, x, outer=None):
        """Replay for bitstring x (and outer value ``outer``, default the
        current one); returns the device float64[2] sum of the pass's slice
        values (valid until the next replay)."""
        if outer is not None and int(outer) != self.outer:
            self.set_outer(outer)
        if self.n:
            self.xdone.synchronize()          # the previous copy has read the pinned buffer
            hv = self.xhost.numpy()
            hv[:] = 0
            for q, (off, bit) in enumerate(self.xslots):
                xb = (int(x) >> (self.n - 1 - q)) & 1
                if bit is None:
                    hv[off + xb] = 1
                elif (self.outer >> bit) & 1 == xb:
                    hv[off] = 1
            self.xbuf.copy_(self.xhost[: self.xbuf.numel()], non_blocking=True)
            self.xdone.record()
        self.graph.replay()
        return self.acc

    def close(self):
        self.graph = None
        self.h.close()
