"""Gradients of circuit probabilities with respect to fSim angles: a
hand-written adjoint through the contraction tree.

For a bitstring x the amplitude a = <x|U|0> is the value of the circuit's
tensor network (Sec. 2.2), contracted pairwise along the plan's tree, and
p = |a|^2.  Every fSim gate on coupler e carries the angle theta_e (one
trainable angle per coupler, shared by all cycles that use the coupler).

Reverse pass.  a is a holomorphic (multilinear) function of every leaf
tensor, so its adjoint E_T = da/dT (same labels as T) flows down the tree:
E_root = 1 and, for a node C = sum_K A B,

    E_A = sum_{free(B)} E_C B      (labels of A),
    E_B = sum_{free(A)} E_C A      (labels of B),

each one more pairwise contraction through ``qce_contract`` on the emulated
GEMM (the same TTGT path, statistics and mode selection as the forward
pass).  For an fSim leaf G_g, s_g = sum E_g * dG_g/dtheta (a full
contraction over its four labels) is da/dtheta from that occurrence; the
s_g of one coupler are added in FP64 on the device, as is the slice sum of
a.  Then dp/dtheta_e = 2 Re(conj(a) sum_g s_g).

Checkpointing: the forward pass of a slice keeps every intermediate of the
tree (the values the reverse pass needs as the sibling operand B or A);
each is released as soon as the reverse pass has used it, and slices are
processed one at a time, so the peak is one slice's intermediates.
Subtrees that hold no fSim leaf are not differentiated.

Host work is marshalling only: leaf tensors (gate matrices from the angles,
|0> and <x| vectors, sliced variants) are built on the host and uploaded;
the final combination 2 Re(conj(a) D_e) and J^T g in the autograd function
act on the handful of FP64 scalars the device returns.
"""
import math

import numpy as np

from . import tn


def fsim_matrix(theta, phi):
    """fSim(theta, phi) in the basis |00>, |01>, |10>, |11> (complex128)."""
    c, s = math.cos(theta), math.sin(theta)
    m = np.zeros((4, 4), dtype=np.complex128)
    m[0, 0] = 1.0
    m[1, 1] = m[2, 2] = c
    m[1, 2] = m[2, 1] = -1j * s
    m[3, 3] = complex(math.cos(phi), -math.sin(phi))
    return m


def fsim_dtheta(theta, phi):
    """d fSim(theta, phi) / d theta."""
    c, s = math.cos(theta), math.sin(theta)
    m = np.zeros((4, 4), dtype=np.complex128)
    m[1, 1] = m[2, 2] = -s
    m[1, 2] = m[2, 1] = -1j * c
    return m


def _flops(A, B, la, lb):
    """8 m n k of a pairwise contraction (each label counted once)."""
    ext = dict(zip(la, A.shape))
    ext.update(zip(lb, B.shape))
    n = 1
    for e in ext.values():
        n *= int(e)
    return 8.0 * n


class GradientRunner:
    """Probabilities and their theta-gradients for one circuit structure and
    contraction plan (``executor.CircuitPlan``), on the handle's GPU."""

    def __init__(self, handle, plan, device="cuda"):
        import torch
        self.torch = torch
        self.device = device
        self.h = handle
        self.flops = 0.0           # 8mnk of every contraction issued (forward and reverse)
        self.last_pass_calls = 0   # upper bound on the contraction calls of the last pass
        self.plan = plan
        circ = plan.circuit
        self.n = circ["n"]
        self.n_couplers = circ.get("n_couplers", 0)
        # leaf index of each gate: n |0> vectors come first
        self.fsim_leaf = {}        # leaf -> (coupler, phi)
        for gi, g in enumerate(circ["gates"]):
            if g.get("name") == "fsim" and "coupler" in g:
                self.fsim_leaf[self.n + gi] = (int(g["coupler"]), float(g["phi"]))
        L = len(plan.label_sets)
        # which nodes have an fSim leaf below them
        self.has_param = [i in self.fsim_leaf for i in range(L)]
        for a, b in plan.path:
            self.has_param.append(self.has_param[a] or self.has_param[b])

    # ---- leaves ---------------------------------------------------------
    def _circuit_at(self, thetas):
        circ = dict(self.plan.circuit)
        gates = []
        for g in circ["gates"]:
            if g.get("name") == "fsim" and "coupler" in g:
                g = dict(g, matrix=fsim_matrix(float(thetas[g["coupler"]]), float(g["phi"])))
            gates.append(g)
        circ["gates"] = gates
        return circ

    def _variants(self, arr, labels, pos):
        """{values of the sliced labels it carries: device tensor}."""
        torch = self.torch
        sl = [lab for lab in labels if lab in pos]
        if not sl:
            return {(): torch.from_numpy(np.ascontiguousarray(arr)).to(self.device)}
        out = {}
        for vals in np.ndindex(*(2,) * len(sl)):
            out[tuple(vals)] = torch.from_numpy(tn.fix_labels(arr, labels, dict(zip(sl, vals)))).to(self.device)
        return out

    def _leaves(self, thetas, x, cache):
        """Device variants of every leaf and of every fSim leaf's derivative.
        Gate leaves (and derivatives) depend only on the angles and are
        uploaded once per angle vector; the <x| vectors (the last n leaves)
        once per bitstring."""
        p = self.plan
        pos = {lab: i for i, lab in enumerate(p.sliced)}
        leaves = tn.circuit_network(self._circuit_at(thetas), x)
        nl = len(leaves)
        if "gates" not in cache:
            cache["gates"] = [self._variants(arr, labels, pos) for arr, labels in leaves[: nl - self.n]]
            dvals = {}
            for i, (cpl, phi) in self.fsim_leaf.items():
                d = fsim_dtheta(float(thetas[cpl]), phi).astype(np.complex64).reshape(2, 2, 2, 2)
                dvals[i] = self._variants(d, leaves[i][1], pos)
            cache["d"] = dvals
        vals = cache["gates"] + [self._variants(arr, labels, pos) for arr, labels in leaves[nl - self.n:]]
        return vals, cache["d"]

    # ---- one bitstring ----------------------------------------------------
    def amplitude_and_derivatives(self, thetas, x, slice_ids=None, cache=None):
        """Device float64 accumulators (a[2], D[n_couplers, 2]) with
        a = sum over slices of the amplitude and D_e = da/dtheta_e.
        ``cache`` (a dict) keeps the angle-dependent leaves between calls
        with the same angles."""
        torch = self.torch
        vals, dvals = self._leaves(thetas, x, {} if cache is None else cache)
        acc_a = torch.zeros(2, dtype=torch.float64, device=self.device)
        acc_d = torch.zeros((max(1, self.n_couplers), 2), dtype=torch.float64, device=self.device)
        self._pass(vals, dvals, slice_ids, acc_a, acc_d)
        return acc_a, acc_d

    def _levels(self):
        """Forward steps grouped by tree level (a step is one level above its
        children) and reverse steps grouped by depth below the root: the
        steps of one group are independent of each other."""
        p = self.plan
        L = len(p.label_sets)
        lev = [0] * L
        fwd = {}
        for s, (a, b) in enumerate(p.path):
            lev.append(1 + max(lev[a], lev[b]))
            fwd.setdefault(lev[-1], []).append(s)
        depth = {L + len(p.path) - 1: 0}
        rev = {}
        for s in range(len(p.path) - 1, -1, -1):
            d = depth[L + s]
            rev.setdefault(d, []).append(s)
            for ch in p.path[s]:
                depth[ch] = d + 1
        return [fwd[k] for k in sorted(fwd)], [rev[k] for k in sorted(rev)]

    def _pass(self, vals, dvals, slice_ids, acc_a, acc_d, grouped=True):
        """Every device operation of one bitstring: for each slice the
        forward pass (keeping the checkpoints) and the reverse pass, adding
        the slice's amplitude to acc_a and each fSim occurrence's
        derivative to its coupler's row of acc_d (FP64, on the device).
        The sequence of calls depends only on the plan, not on the leaf
        values, so it can be captured once and replayed.

        ``grouped``: the independent steps of each forward tree level and of
        each reverse depth run inside one library group, so their small
        contractions share one launch.  A grouped result exists only once
        its group has ended, so the derivative contraction of an fSim
        occurrence runs in the next group and its FP64 accumulation after
        that group."""
        import paper_2303_08989_amd as qce
        from contextlib import nullcontext
        torch = self.torch
        p = self.plan
        L = len(p.label_sets)
        pos = {lab: i for i, lab in enumerate(p.sliced)}
        if slice_ids is None:
            slice_ids = range(p.n_slices)
        use_groups = grouped and self.device != "cpu"
        fwd_levels, rev_levels = self._levels() if p.path else ([], [])

        def group():
            return qce.group(self.h) if use_groups else nullcontext()

        one = torch.ones((), dtype=torch.complex64, device=self.device)
        calls = 0
        for sigma in slice_ids:
            v = {lab: (sigma >> i) & 1 for lab, i in pos.items()}

            def key(i):
                return tuple(v[lab] for lab in p.label_sets[i] if lab in pos)

            def leaf(i):
                return vals[i][key(i)]

            if not p.path:
                qce.accumulate_f64(self.h, leaf(0).reshape(-1)[:1], acc_a)
                continue
            calls += 2 * len(p.path) + len(self.fsim_leaf)     # at most, per slice
            # forward, keeping every intermediate (the checkpoints)
            node_val, node_lab = {}, {i: tuple(p.labels[i]) for i in range(L)}
            for level in fwd_levels:
                with group():
                    for s in level:
                        a, b = p.path[s]
                        ta = leaf(a) if a < L else node_val[a]
                        tb = leaf(b) if b < L else node_val[b]
                        la, lb = node_lab[a], node_lab[b]
                        shared = set(la) & set(lb)
                        lc = [lab for lab in lb if lab not in shared] + [lab for lab in la if lab not in shared]
                        node_lab[L + s] = tuple(lc)
                        node_val[L + s] = qce.contract(self.h, ta, list(la), tb, list(lb), lc)
                        self.flops += _flops(ta, tb, la, lb)
            root = L + len(p.path) - 1
            qce.accumulate_f64(self.h, node_val[root].reshape(-1)[:1], acc_a)
            # reverse pass, one group per depth below the root
            # adjoints keep the contraction's own output order (no output
            # permute); adj_lab holds each adjoint's label order
            adj, adj_lab = {root: one}, {root: ()}
            pending = []          # (E of an fSim leaf, its labels, leaf) awaiting its derivative contraction
            for level in rev_levels + [[]]:
                sg = []
                with group():
                    for E_g, lab_g, g in pending:
                        dG = dvals[g][key(g)]
                        sg.append((qce.contract(self.h, E_g, list(lab_g), dG, list(node_lab[g]), []),
                                   self.fsim_leaf[g][0]))
                    pending = []
                    for s in level:
                        node = L + s
                        E = adj.pop(node, None)
                        a, b = p.path[s]
                        if E is None:
                            continue
                        E_lab = adj_lab.pop(node)
                        for ch, other in ((a, b), (b, a)):
                            if not self.has_param[ch]:
                                continue
                            t_other = leaf(other) if other < L else node_val[other]
                            lo = node_lab[other]
                            # the child's labels: the other operand's labels it
                            # shares, then the adjoint's labels the other lacks
                            lc = [lab for lab in lo if lab not in E_lab] + [lab for lab in E_lab if lab not in lo]
                            E_ch = qce.contract(self.h, E, list(E_lab), t_other, list(lo), lc)
                            self.flops += _flops(E, t_other, E_lab, lo)
                            if ch < L:
                                pending.append((E_ch, tuple(lc), ch))
                            else:
                                adj[ch] = E_ch
                                adj_lab[ch] = tuple(lc)
                for s_g, cpl in sg:
                    qce.accumulate_f64(self.h, s_g.reshape(-1)[:1], acc_d[cpl])
                # the forward values this depth consumed are no longer needed
                for s in level:
                    a, b = p.path[s]
                    node_val.pop(a, None)
                    node_val.pop(b, None)
            node_val.clear()
        self.last_pass_calls = calls

    def probabilities_and_jacobian(self, thetas, bitstrings, slice_ids=None):
        """p_x = |a_x|^2 (float64, shape (X,)), the amplitudes (complex128)
        and J[x, e] = dp_x / dtheta_e (float64, shape (X, n_couplers))."""
        thetas = np.asarray(thetas, dtype=np.float32)
        cache = {}
        accs = [self.amplitude_and_derivatives(thetas, x, slice_ids, cache) for x in bitstrings]
        if self.device != "cpu":
            self.torch.cuda.synchronize()
        return _combine(accs, self.n_couplers)


def _combine(accs, n_couplers):
    """(p, amplitudes, J) from per-bitstring device accumulators (a, D):
    p = |a|^2 and J[x, e] = 2 Re(conj(a) D_e)."""
    amps = np.empty(len(accs), dtype=np.complex128)
    J = np.zeros((len(accs), n_couplers), dtype=np.float64)
    for i, (acc_a, acc_d) in enumerate(accs):
        ar, ai = acc_a.cpu().numpy()
        d = acc_d.cpu().numpy()[:n_couplers]
        amps[i] = complex(ar, ai)
        J[i] = 2.0 * (ar * d[:, 0] + ai * d[:, 1])
    return np.abs(amps) ** 2, amps, J


class GradientGraph:
    """The forward and reverse passes of ``GradientRunner`` captured once in
    a HIP graph and replayed per bitstring and angle vector.

    The <x| leaves (the last n) depend on the bitstring and the fSim leaves
    and their derivatives on the angles: each device variant of those leaves
    is a view of one of two buffers, refilled by one copy from pinned memory
    before a replay (``_upload``) or on ``set_thetas`` (an event keeps the
    host from rewriting a pinned buffer before its previous copy has run).
    The
    graph owns its handle, so the workspace whose address the captured
    kernels hold is never reallocated; a warm-up pass sizes it before
    capture.  The accumulators are cleared by fill kernels inside the graph
    (no memset is captured)."""

    def __init__(self, plan, thetas, device=0, mode="auto", slice_ids=None, size_policy=None):
        import torch
        import paper_2303_08989_amd as qce
        self.torch = torch
        self.h = qce.Handle(device)
        self.h.set_mode(mode)            # fixed for the captured passes
        if size_policy is not None:
            self.h.set_size_policy(*size_policy)
        self.run = GradientRunner(self.h, plan)
        self.n = self.run.n
        self.n_couplers = self.run.n_couplers
        self.thetas = np.asarray(thetas, dtype=np.float32)
        vals, dvals = self.run._leaves(self.thetas, 0, {})
        # every variant of the <x| leaves becomes a view of one buffer;
        # per variant: its offset, the value of the sliced label it is fixed
        # by (it is then a scalar) or None, and its qubit
        nl = len(vals)
        layout, total = [], 0
        for q in range(self.n):
            i = nl - self.n + q
            for key, t in vals[i].items():
                layout.append((i, key, q, total, t.shape))
                total += t.numel()
        self.xbuf = torch.zeros(max(total, 1), dtype=torch.complex64, device="cuda")
        self.xslots = []
        for i, key, q, off, shape in layout:
            vals[i][key] = self.xbuf[off:off + int(np.prod(shape, dtype=np.int64))].view(shape)
            self.xslots.append((off, key[0] if key else None, q))
        self.xhost = torch.zeros(max(total, 1), dtype=torch.complex64, pin_memory=True)
        self.xdone = torch.cuda.Event()
        self.xdone.record()
        # likewise every variant of the fSim leaves and of their derivatives:
        # (leaf, 0 = gate / 1 = derivative, variant key, offset, elements)
        tlayout, ttotal = [], 0
        for i in sorted(self.run.fsim_leaf):
            for which, src in ((0, vals), (1, dvals)):
                for key, t in src[i].items():
                    tlayout.append((i, which, key, ttotal, t.shape))
                    ttotal += t.numel()
        self.tbuf = torch.zeros(max(ttotal, 1), dtype=torch.complex64, device="cuda")
        self.tslots = []
        for i, which, key, off, shape in tlayout:
            src = vals if which == 0 else dvals
            size = int(np.prod(shape, dtype=np.int64))
            view = self.tbuf[off:off + size].view(shape)
            view.copy_(src[i][key])
            src[i][key] = view
            self.tslots.append((i, which, key, off, size))
        self.thost = torch.zeros(max(ttotal, 1), dtype=torch.complex64, pin_memory=True)
        self.tdone = torch.cuda.Event()
        self.tdone.record()
        self.acc_a = torch.zeros(2, dtype=torch.float64, device="cuda")
        self.acc_d = torch.zeros((max(1, self.n_couplers), 2), dtype=torch.float64, device="cuda")
        self._upload(0)
        self.run._pass(vals, dvals, slice_ids, self.acc_a, self.acc_d)   # warm-up: workspace, allocator
        torch.cuda.synchronize()
        # descriptor room for every group of one captured pass (a recorded
        # contraction takes under 1 KB of descriptors)
        qce.group_reset(self.h, (self.run.last_pass_calls << 10) + (1 << 20))
        self.run.flops = 0.0
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self.acc_a.zero_()
            self.acc_d.zero_()
            self.run._pass(vals, dvals, slice_ids, self.acc_a, self.acc_d)
        self.flops_per_pass = self.run.flops   # 8mnk of every contraction of one replay
        self._keep = (vals, dvals)

    def _upload(self, x):
        """Write the <x| leaves of bitstring x into the device buffer."""
        self.xdone.synchronize()          # the previous copy has read the pinned buffer
        hv = self.xhost.numpy()
        hv[:] = 0
        for off, fixed, q in self.xslots:
            bit = (int(x) >> (self.n - 1 - q)) & 1
            if fixed is None:
                hv[off + bit] = 1
            elif fixed == bit:
                hv[off] = 1
        self.xbuf.copy_(self.xhost[: self.xbuf.numel()], non_blocking=True)
        self.xdone.record()

    def set_thetas(self, thetas):
        """Angles for the following replays: the fSim leaves and their
        derivatives are rebuilt on the host and uploaded in one copy (no
        recapture)."""
        from . import tn
        th = np.asarray(thetas, dtype=np.float32)
        p = self.run.plan
        pos = {lab: i for i, lab in enumerate(p.sliced)}
        leaves = tn.circuit_network(self.run._circuit_at(th), 0)
        self.tdone.synchronize()          # the previous copy has read the pinned buffer
        hv = self.thost.numpy()
        for i, which, key, off, size in self.tslots:
            labels = leaves[i][1]
            if which == 0:
                arr = leaves[i][0]
            else:
                cpl, phi = self.run.fsim_leaf[i]
                arr = fsim_dtheta(float(th[cpl]), phi).astype(np.complex64).reshape(2, 2, 2, 2)
            sl = [lab for lab in labels if lab in pos]
            hv[off:off + size] = tn.fix_labels(arr, labels, dict(zip(sl, key))).reshape(-1)
        self.tbuf.copy_(self.thost[: self.tbuf.numel()], non_blocking=True)
        self.tdone.record()
        self.thetas = th

    def amplitude_and_derivatives(self, x):
        """Replay for bitstring x: the device accumulators (a[2], D[E, 2]),
        valid until the next replay."""
        self._upload(x)
        self.graph.replay()
        return self.acc_a, self.acc_d

    def probabilities_and_jacobian(self, bitstrings, thetas=None):
        """As ``GradientRunner.probabilities_and_jacobian``, at ``thetas``
        (uploaded first) or at the angles set last."""
        if thetas is not None and not np.array_equal(np.asarray(thetas, dtype=np.float32), self.thetas):
            self.set_thetas(thetas)
        accs = []
        for x in bitstrings:
            a, d = self.amplitude_and_derivatives(x)
            accs.append((a.clone(), d.clone()))
        self.torch.cuda.synchronize()
        return _combine(accs, self.n_couplers)

    def close(self):
        self.graph = None
        self._keep = None
        self.h.close()


def circuit_probabilities(runner, thetas, bitstrings, slice_ids=None):
    """p_x(theta) for the bitstrings as a differentiable torch function of
    the FP32 angle tensor ``thetas`` (one per coupler).  ``runner`` is a
    ``GradientRunner`` (eager passes) or a ``GradientGraph`` (captured
    passes; ``slice_ids`` are then the ones it was captured with)."""
    import torch

    class _Probabilities(torch.autograd.Function):
        @staticmethod
        def forward(ctx, th):
            if isinstance(runner, GradientGraph):
                p, _, J = runner.probabilities_and_jacobian(bitstrings, thetas=th.detach().cpu().numpy())
            else:
                p, _, J = runner.probabilities_and_jacobian(th.detach().cpu().numpy(), bitstrings, slice_ids)
            ctx.save_for_backward(torch.from_numpy(J))
            return torch.from_numpy(p).to(th.device)

        @staticmethod
        def backward(ctx, grad_p):
            (J,) = ctx.saved_tensors
            g = J.numpy().T @ grad_p.detach().cpu().numpy().astype(np.float64)
            return torch.from_numpy(g.astype(np.float32)).to(grad_p.device)

    return _Probabilities.apply(thetas)
