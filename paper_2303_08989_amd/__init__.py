"""MI355X (gfx950) emulated-FP32 complex GEMM and tensor contraction for
quantum-circuit tensor networks (arXiv 2303.08989).

The functions here only marshal arguments to the C-ABI of libqcemu.so
(``include/qcemu.h``): torch tensors provide device memory and the current
stream, every computation runs in the library's HIP kernels.  Importing the
package does not touch the GPU; the first call loads the library and fails
loudly if it is not built.

Tensors are dense row-major torch tensors (complex64 on the GPU).  The BLAS
entry point ``cgemm`` takes column-major conventions exactly as the C-ABI;
``matmul`` is the row-major convenience form.
"""
import ctypes

from . import _lib
from ._lib import (  # noqa: F401
    MODE_AUTO, MODE_BF16X3, MODE_FP16X2, MODE_FP16X2_SCALED, MODE_FP32, MODE_NAMES,
    MODE_BY_NAME, QceError,
)


def _torch():
    import torch
    return torch


def _check(h, status):
    if status != 0:
        msg = ""
        if h is not None:
            msg = _lib.load().qce_last_error(h).decode(errors="replace")
        raise QceError(status, msg)


def _mode_value(mode):
    if isinstance(mode, str):
        return _lib.MODE_BY_NAME[mode]
    return int(mode)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _c32(z):
    z = complex(z)
    return _lib.QceC32(z.real, z.imag)


class Handle:
    """A library handle on one GPU; work goes to torch's current stream."""

    def __init__(self, device=None):
        torch = _torch()
        self.lib = _lib.load()
        self.device = torch.cuda.current_device() if device is None else int(device)
        self._h = ctypes.c_void_p()
        _check(None, self.lib.qce_create(ctypes.byref(self._h), self.device))
        self._stream = None
        # the policy the handle was created with (library default or the
        # QCE_AUTO_MIN_DIM / QCE_EMUL_MIN_DIM environment), to restore it
        self.default_size_policy = self.size_policy()

    def _bind_stream(self):
        torch = _torch()
        s = torch.cuda.current_stream(self.device).cuda_stream
        if s != self._stream:
            _check(self._h, self.lib.qce_set_stream(self._h, ctypes.c_void_p(s)))
            self._stream = s
        return self._h

    def close(self):
        if self._h:
            self.lib.qce_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_mode(self, mode):
        _check(self._h, self.lib.qce_set_mode(self._h, _mode_value(mode)))

    def get_mode(self):
        m = ctypes.c_int()
        _check(self._h, self.lib.qce_get_mode(self._h, ctypes.byref(m)))
        return m.value

    def set_tolerance(self, t, t3=0.0):
        _check(self._h, self.lib.qce_set_underflow_tolerance(self._h, float(t), float(t3)))

    def set_size_policy(self, auto_min, emul_min):
        _check(self._h, self.lib.qce_set_size_policy(self._h, int(auto_min), int(emul_min)))

    def set_gemm_size_policy(self, enable=True):
        """Apply the size policy to the CGEMM entry points in AUTO mode too (Sec. 4.3)."""
        _check(self._h, self.lib.qce_set_gemm_size_policy(self._h, 1 if enable else 0))

    def size_policy(self):
        """(auto_min, emul_min) of the size policy (Sec. 4.3)."""
        a, e = ctypes.c_int64(), ctypes.c_int64()
        _check(self._h, self.lib.qce_get_size_policy(self._h, ctypes.byref(a), ctypes.byref(e)))
        return a.value, e.value

    def set_gemm_tile(self, tile):
        """Panel GEMM tile: 64, 128, or 0 for the library's tuned table."""
        _check(self._h, self.lib.qce_set_gemm_tile(self._h, int(tile)))

    def set_workspace(self, tensor):
        if tensor is None:
            _check(self._h, self.lib.qce_set_workspace(self._h, None, 0))
        else:
            nbytes = tensor.numel() * tensor.element_size()
            _check(self._h, self.lib.qce_set_workspace(self._h, _ptr(tensor), nbytes))

    def set_timing(self, enable=True):
        """Record hipEvent timings of every phase (no synchronisation)."""
        _check(self._h, self.lib.qce_set_timing(self._h, 1 if enable else 0))

    def set_timing_tag(self, tag):
        _check(self._h, self.lib.qce_set_timing_tag(self._h, int(tag)))

    def reset_timing(self):
        _check(self._h, self.lib.qce_reset_timing(self._bind_stream()))

    def timing(self, tag=-1):
        """Synchronising summary of the timing records with this tag (-1: all):
        {phase: (ms, count)} plus 'gemms_by_mode'."""
        t = _lib.QceTiming()
        _check(self._h, self.lib.qce_get_timing(self._bind_stream(), int(tag), ctypes.byref(t)))
        out = {name: (t.ms[i], t.count[i]) for i, name in enumerate(_lib.PHASES)}
        out["gemms_by_mode"] = {MODE_NAMES[i]: t.gemms_by_mode[i] for i in range(4)}
        return out

    def last_decision(self):
        """Synchronising read of the last GEMM decision record."""
        d = _lib.QceDecision()
        _check(self._h, self.lib.qce_get_last_decision(self._bind_stream(), ctypes.byref(d)))
        return _decision_dict(d)

    def batch_decision(self, index):
        """Synchronising read of entry ``index`` of the last (batched) GEMM."""
        d = _lib.QceDecision()
        _check(self._h, self.lib.qce_get_batch_decision(self._bind_stream(), int(index), ctypes.byref(d)))
        return _decision_dict(d)


def _decision_dict(d):
    return {"mode": d.mode, "mode_name": MODE_NAMES.get(d.mode, str(d.mode)),
            "sA": d.sA, "sB": d.sB, "stats_taken": d.stats_taken,
            "nnz": list(d.nnz), "n1": list(d.n1), "n2": list(d.n2), "n3": list(d.n3),
            "nonfinite": list(d.nonfinite), "emax": list(d.emax)}


def cgemm_workspace_size(m, n, k):
    return int(_lib.load().qce_cgemm_workspace_size(int(m), int(n), int(k)))


def cgemm(h, opA, opB, m, n, k, A, lda, B, ldb, C, ldc, alpha=1.0, beta=0.0):
    """BLAS CGEMM, column-major: C <- alpha op(A) op(B) + beta C (C-ABI
    ``qce_cgemm_emulated``).  A, B, C are complex64 device tensors used only
    for their data pointers."""
    hh = h._bind_stream()
    a, b = _c32(alpha), _c32(beta)
    _check(hh, h.lib.qce_cgemm_emulated(hh, _lib.OPS[opA], _lib.OPS[opB], int(m), int(n), int(k),
                                        ctypes.byref(a), _ptr(A), int(lda), _ptr(B), int(ldb),
                                        ctypes.byref(b), _ptr(C), int(ldc)))
    return C


def cgemm_noalloc(h, opA, opB, m, n, k, A, lda, B, ldb, C, ldc, alpha=1.0, beta=0.0):
    """``cgemm`` through ``qce_cgemm_emulated_noalloc``: no device memory is
    allocated; the library's fixed per-GPU scratch holds the intermediates
    (see ``noalloc_scratch_bytes``)."""
    hh = h._bind_stream()
    a, b = _c32(alpha), _c32(beta)
    _check(hh, h.lib.qce_cgemm_emulated_noalloc(hh, _lib.OPS[opA], _lib.OPS[opB], int(m), int(n), int(k),
                                                ctypes.byref(a), _ptr(A), int(lda), _ptr(B), int(ldb),
                                                ctypes.byref(b), _ptr(C), int(ldc)))
    return C


def noalloc_scratch_bytes():
    return int(_lib.load().qce_noalloc_scratch_bytes())


def cgemm_batched_workspace_size(m, n, k, batch):
    return int(_lib.load().qce_cgemm_batched_workspace_size(int(m), int(n), int(k), int(batch)))


def cgemm_strided_batched(h, opA, opB, m, n, k, A, lda, strideA, B, ldb, strideB, C, ldc, strideC,
                          batch, alpha=1.0, beta=0.0):
    """``batch`` column-major CGEMMs of one shape, entry z at A + z*strideA,
    B + z*strideB, C + z*strideC (C-ABI ``qce_cgemm_strided_batched``)."""
    hh = h._bind_stream()
    a, b = _c32(alpha), _c32(beta)
    _check(hh, h.lib.qce_cgemm_strided_batched(hh, _lib.OPS[opA], _lib.OPS[opB], int(m), int(n), int(k),
                                               ctypes.byref(a), _ptr(A), int(lda), int(strideA),
                                               _ptr(B), int(ldb), int(strideB), ctypes.byref(b),
                                               _ptr(C), int(ldc), int(strideC), int(batch)))
    return C


def cgemm_grouped(h, gemms):
    """Independent column-major CGEMMs of any shapes in one grouped call
    (C-ABI ``qce_cgemm_grouped``).  ``gemms``: sequence of dicts with keys
    opA, opB, m, n, k, A, lda, B, ldb, C, ldc and optional alpha, beta
    (A, B, C complex64 device tensors used for their data pointers)."""
    hh = h._bind_stream()
    arr = (_lib.QceGemmDesc * max(1, len(gemms)))()
    for i, g in enumerate(gemms):
        d = arr[i]
        d.opA, d.opB = _lib.OPS[g.get("opA", "N")], _lib.OPS[g.get("opB", "N")]
        d.m, d.n, d.k = int(g["m"]), int(g["n"]), int(g["k"])
        d.alpha, d.beta = _c32(g.get("alpha", 1.0)), _c32(g.get("beta", 0.0))
        d.A, d.lda = _ptr(g["A"]).value, int(g["lda"])
        d.B, d.ldb = _ptr(g["B"]).value, int(g["ldb"])
        d.C, d.ldc = _ptr(g["C"]).value, int(g["ldc"])
    _check(hh, h.lib.qce_cgemm_grouped(hh, len(gemms), arr))
    return [g["C"] for g in gemms]


def matmul(h, A, B, out=None):
    """Row-major C = A @ B for 2-D complex64 device tensors.  A row-major
    (M, K) tensor is the column-major K x M matrix A^T, so C^T = B^T A^T is
    one column-major GEMM with the operands swapped."""
    torch = _torch()
    A = A.contiguous()
    B = B.contiguous()
    M, K = A.shape
    K2, N = B.shape
    if K != K2:
        raise ValueError("inner dimensions differ")
    if out is None:
        out = torch.empty((M, N), dtype=torch.complex64, device=A.device)
    cgemm(h, "N", "N", N, M, K, B, max(1, N), A, max(1, K), out, max(1, N))
    return out


def _tensor_desc(shape):
    ext = (ctypes.c_int64 * max(1, len(shape)))(*[int(s) for s in shape])
    return _lib.QceTensor(len(shape), ext), ext


def _labels(ls):
    return (ctypes.c_int32 * max(1, len(ls)))(*[int(x) for x in ls])


def contract(h, A, la, B, lb, lc, out=None):
    """C[lc] = sum A[la] B[lb] over the labels shared by A and B (C-ABI
    ``qce_contract``).  Row-major complex64 device tensors."""
    torch = _torch()
    A = A.contiguous()
    B = B.contiguous()
    ext = {}
    for t, ls in ((A, la), (B, lb)):
        for d, lab in enumerate(ls):
            ext[lab] = t.shape[d]
    cshape = tuple(ext[x] for x in lc)
    if out is None:
        out = torch.empty(cshape, dtype=torch.complex64, device=A.device)
    ta, ka = _tensor_desc(A.shape)
    tb, kb = _tensor_desc(B.shape)
    tc, kc = _tensor_desc(cshape)
    hh = h._bind_stream()
    _check(hh, h.lib.qce_contract(hh, ctypes.byref(ta), _ptr(A), _labels(la),
                                  ctypes.byref(tb), _ptr(B), _labels(lb),
                                  ctypes.byref(tc), _ptr(out), _labels(lc)))
    if getattr(h, "_group_refs", None) is not None:
        h._group_refs.append((A, B))
    return out


class group:
    """``with group(h): ...`` records the small contractions of the block and
    runs them in one launch at its end (C-ABI ``qce_group_begin`` /
    ``qce_group_end``).  The block's contractions must be independent."""

    def __init__(self, h):
        self.h = h

    def __enter__(self):
        hh = self.h._bind_stream()
        _check(hh, self.h.lib.qce_group_begin(hh))
        self.h._group_refs = []      # operands a recorded contraction reads at the group's end
        return self

    def __exit__(self, *exc):
        hh = self.h._bind_stream()
        try:
            _check(hh, self.h.lib.qce_group_end(hh))
        finally:
            # the group's launch is enqueued: later work on the stream runs
            # after it, so the operands' memory may be reused from here on
            self.h._group_refs = None
        return False


def group_reset(h, reserve_bytes=0):
    """Drain the stream and reuse the group descriptor area from its start,
    at least ``reserve_bytes`` large (C-ABI ``qce_group_reset``)."""
    hh = h._bind_stream()
    _check(hh, h.lib.qce_group_reset(hh, int(reserve_bytes)))


def permute(h, X, perm, out=None):
    """Y = X.permute(perm) materialised by the library (C-ABI ``qce_permute``)."""
    torch = _torch()
    X = X.contiguous()
    shape = tuple(X.shape[p] for p in perm)
    if out is None:
        out = torch.empty(shape, dtype=torch.complex64, device=X.device)
    tx, kx = _tensor_desc(X.shape)
    hh = h._bind_stream()
    _check(hh, h.lib.qce_permute(hh, ctypes.byref(tx), _ptr(X), _labels(perm), _ptr(out)))
    return out


def accumulate_f64(h, src, acc):
    """acc (float64[2], device) += src (complex64 scalar, device), in FP64."""
    hh = h._bind_stream()
    _check(hh, h.lib.qce_accumulate_f64(hh, _ptr(src), _ptr(acc)))
    return acc


def accumulate_n_f64(h, src, acc):
    """acc (float64[2], device) += sum of the complex64 device tensor src, in FP64."""
    hh = h._bind_stream()
    _check(hh, h.lib.qce_accumulate_n_f64(hh, _ptr(src), int(src.numel()), _ptr(acc)))
    return acc


def fidelity_terms(h, a, b, out=None):
    """out (float64[4], device) = [re <b|a>, im <b|a>, <a|a>, <b|b>] in FP64."""
    torch = _torch()
    if out is None:
        out = torch.empty(4, dtype=torch.float64, device=a.device)
    hh = h._bind_stream()
    _check(hh, h.lib.qce_fidelity_f64(hh, _ptr(a), _ptr(b), int(a.numel()), _ptr(out)))
    return out


def expstats(h, X, rows, cols, ld):
    """Synchronising exponent statistics of a column-major matrix."""
    d = _lib.QceDecision()
    hh = h._bind_stream()
    _check(hh, h.lib.qce_expstats(hh, _ptr(X), int(rows), int(cols), int(ld), ctypes.byref(d)))
    r = _decision_dict(d)
    return {"level": r["mode"], "nnz": r["nnz"][0], "n1": r["n1"][0], "n2": r["n2"][0],
            "n3": r["n3"][0], "nonfinite": r["nonfinite"][0], "emax": r["emax"][0]}


def split(h, mode, shift, x):
    """Planar split of n complex64 values: int16 device tensor (planes, n)."""
    torch = _torch()
    mode = _mode_value(mode)
    planes = 6 if mode == MODE_BF16X3 else 4
    out = torch.empty((planes, x.numel()), dtype=torch.int16, device=x.device)
    hh = h._bind_stream()
    _check(hh, h.lib.qce_split(hh, mode, int(shift), _ptr(x), int(x.numel()), _ptr(out)))
    return out


def split_panels(h, mode, shift, X, rows, k, ld, layout=0, conj=False):
    """The GEMM path's panel writer on one operand (C-ABI
    ``qce_split_panels``): uint8 device tensor in the panel format."""
    torch = _torch()
    mode = _mode_value(mode)
    nbytes = int(h.lib.qce_panel_bytes(mode, int(rows), int(k)))
    out = torch.empty(max(nbytes, 16), dtype=torch.uint8, device=X.device)
    hh = h._bind_stream()
    _check(hh, h.lib.qce_split_panels(hh, mode, int(shift), int(layout), 1 if conj else 0, _ptr(X),
                                      int(rows), int(k), int(ld), _ptr(out)))
    return out[:nbytes]


def split_panels_bitmap(h, mode, shift, X, rsh, ksh):
    """The transpose-fused panel writer (C-ABI ``qce_split_panels_bitmap``):
    P[r][l] = X[sum bit_t(r) 2^rsh[t] + sum bit_t(l) 2^ksh[t]]."""
    torch = _torch()
    mode = _mode_value(mode)
    nr, nk = len(rsh), len(ksh)
    nbytes = int(h.lib.qce_panel_bytes(mode, 1 << nr, 1 << nk))
    out = torch.empty(max(nbytes, 16), dtype=torch.uint8, device=X.device)
    hh = h._bind_stream()
    _check(hh, h.lib.qce_split_panels_bitmap(hh, mode, int(shift), _ptr(X), nr, nk, _labels(rsh),
                                             _labels(ksh), _ptr(out)))
    return out[:nbytes]
