"""Oracle arithmetic: exact CGEMM, splits, exponent statistics, mode rule.

TEST INFRASTRUCTURE ONLY (see the package docstring).
"""
import ctypes
import os

import numpy as np

from . import build as _build

MODE_FP16X2, MODE_FP16X2_SCALED, MODE_BF16X3, MODE_FP32 = 0, 1, 2, 3
MODE_NAMES = {MODE_FP16X2: "fp16x2", MODE_FP16X2_SCALED: "fp16x2_scaled",
              MODE_BF16X3: "bf16x3", MODE_FP32: "fp32"}

_lib = None


def _clib():
    global _lib
    if _lib is None:
        # QCE_ORACLE_LIB: another build of oracle.c (the sanitizer test's)
        path = os.environ.get("QCE_ORACLE_LIB") or _build.build()
        lib = ctypes.CDLL(path)
        f64p = ctypes.POINTER(ctypes.c_double)
        f32p = ctypes.POINTER(ctypes.c_float)
        i64 = ctypes.c_int64
        lib.oracle_cgemm.restype = None
        lib.oracle_cgemm.argtypes = [i64, i64, i64, ctypes.c_int, ctypes.c_int,
                                     ctypes.c_double, ctypes.c_double, f32p, i64, f32p, i64,
                                     ctypes.c_double, ctypes.c_double, f64p, i64, f64p, i64]
        i32p = ctypes.POINTER(ctypes.c_int32)
        i64p = ctypes.POINTER(ctypes.c_int64)
        lib.oracle_zcontract.restype = ctypes.c_int
        lib.oracle_zcontract.argtypes = [ctypes.c_int, i64p, ctypes.c_int, i32p, f64p,
                                         ctypes.c_int, i32p, f64p, ctypes.c_int, i32p, f64p,
                                         ctypes.c_int, i32p]
        lib.oracle_threads.restype = ctypes.c_int
        lib.oracle_threads.argtypes = []
        _lib = lib
    return _lib


def threads():
    """OpenMP threads the C loops use."""
    return int(_clib().oracle_threads())


_OPS = {"N": 0, "T": 1, "C": 2}


def _op_shape(shape, op):
    return shape if op == "N" else (shape[1], shape[0])


def cgemm(A, B, opA="N", opB="N", alpha=1.0, beta=0.0, C0=None):
    """Exact ``alpha * op(A) @ op(B) + beta * C0`` in complex128 (nested loops).

    A and B are complex64 2-D arrays (any memory order; they are passed to the
    C loops column-major).  Returns a complex128 (m, n) array.  The complex
    product follows Sec. 3 with the imaginary part read as Ar*Bi + Ai*Br.
    """
    A = np.asfortranarray(A, dtype=np.complex64)
    B = np.asfortranarray(B, dtype=np.complex64)
    m, ka = _op_shape(A.shape, opA)
    kb, n = _op_shape(B.shape, opB)
    if ka != kb:
        raise ValueError("inner dimensions differ")
    C = np.zeros((m, n), dtype=np.complex128, order="F")
    alpha = complex(alpha)
    beta = complex(beta)
    c0p = None
    ldc0 = max(1, m)
    if C0 is not None and beta != 0:
        C0 = np.asfortranarray(C0, dtype=np.complex128)
        c0p = C0.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    lib = _clib()
    f32p = ctypes.POINTER(ctypes.c_float)
    lib.oracle_cgemm(m, n, ka, _OPS[opA], _OPS[opB], alpha.real, alpha.imag,
                     A.ctypes.data_as(f32p), max(1, A.shape[0]),
                     B.ctypes.data_as(f32p), max(1, B.shape[0]),
                     beta.real, beta.imag, c0p, ldc0,
                     C.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), max(1, m))
    return C


def rel_fro(C, Cref):
    """Relative Frobenius error ||C - Cref||_F / ||Cref||_F in FP64 (Eq. 3).

    When ||Cref||_F is zero the absolute error is returned.
    """
    C = np.asarray(C).astype(np.complex128)
    Cref = np.asarray(Cref).astype(np.complex128)
    num = np.sqrt(np.sum(np.abs(C - Cref) ** 2))
    den = np.sqrt(np.sum(np.abs(Cref) ** 2))
    return float(num / den) if den > 0 else float(num)


# ---------------------------------------------------------------------------
# Splits (Sec. 2.1, Eq. 2)
# ---------------------------------------------------------------------------

def fp16_rne(x32):
    """FP32 -> FP16, round to nearest even (numpy's conversion)."""
    return np.asarray(x32, dtype=np.float32).astype(np.float16)


def bf16_rne(x32):
    """FP32 -> bfloat16 bit patterns (uint16), round to nearest even.

    bfloat16 is the upper half of an FP32 word; rounding adds half an ulp of
    the kept part, minus one when the kept part is even, so that exact ties
    round to the even neighbour.  Finite inputs only (non-finite values are
    routed to the FP32 mode before any split).
    """
    u = np.asarray(x32, dtype=np.float32).view(np.uint32).astype(np.uint64)
    keep_lsb = (u >> np.uint64(16)) & np.uint64(1)
    u = u + np.uint64(0x7FFF) + keep_lsb
    return (u >> np.uint64(16)).astype(np.uint16)


def bf16_to_f32(b16):
    """bfloat16 bit patterns -> FP32 values (exact)."""
    return (np.asarray(b16, dtype=np.uint16).astype(np.uint32) << np.uint32(16)).view(np.float32)


def _ldexp32(x32, s):
    """x * 2^s in FP32 (exact unless the result leaves the FP32 range)."""
    return np.ldexp(np.asarray(x32, dtype=np.float32).astype(np.float64), int(s)).astype(np.float32)


def split_fp16x2(x32, s=0):
    """Two-term FP16 split of Eq. 2 applied to x * 2^s.

    hi = toLow(x'), lo = toLow((x' - toF32(hi)) * 2^11) with x' = x * 2^s.
    ``toLow`` rounds to nearest even (the paper does not state the rounding;
    round-to-nearest-even is the conversion both numpy and the GPU use).
    x' - toF32(hi) is exact in FP32.  Returns (hi, lo) as float16 arrays.
    """
    xs = _ldexp32(x32, s)
    hi = fp16_rne(xs)
    r = xs - hi.astype(np.float32)
    lo = fp16_rne(r * np.float32(2048.0))
    return hi, lo


def split_bf16x3(x32):
    """Three-term bfloat16 split: b0 = bf16(x), b1 = bf16(x - b0),
    b2 = bf16(x - b0 - b1), every subtraction exact in FP32.

    Not in the paper: CDNA4 has no TF32 matrix instruction, so this split
    takes the role of TF32TCEC (FP32 exponent range, Table 1).  Returns three
    uint16 arrays of bfloat16 bit patterns.
    """
    x = np.asarray(x32, dtype=np.float32)
    b0 = bf16_rne(x)
    r1 = x - bf16_to_f32(b0)
    b1 = bf16_rne(r1)
    r2 = r1 - bf16_to_f32(b1)
    b2 = bf16_rne(r2)
    return b0, b1, b2


def _split_complex_fp16x2(M, s):
    hr, lr = split_fp16x2(M.real.astype(np.float32), s)
    hi_, li = split_fp16x2(M.imag.astype(np.float32), s)
    hi = hr.astype(np.float64) + 1j * hi_.astype(np.float64)
    lo = lr.astype(np.float64) + 1j * li.astype(np.float64)
    return hi, lo


def _split_complex_bf16x3(M):
    parts_r = split_bf16x3(M.real.astype(np.float32))
    parts_i = split_bf16x3(M.imag.astype(np.float32))
    return [bf16_to_f32(pr).astype(np.float64) + 1j * bf16_to_f32(pi).astype(np.float64)
            for pr, pi in zip(parts_r, parts_i)]


def emulated_cgemm(A, B, mode, sA=0, sB=0):
    """FP64 value of the emulated product op(A) @ op(B) for one mode.

    * FP16X2 / FP16X2_SCALED: Eq. 2 on each of the four real products of
      Sec. 3, with A scaled by 2^sA and B by 2^sB before the split and the
      result scaled back by 2^-(sA+sB) (Sec. 4.2):
      2^-(sA+sB) * (Ahi Bhi + (Alo Bhi + Ahi Blo) / 2^11).  The product of
      the two residual parts is dropped, as in Eq. 2.
    * BF16X3: sum of the six products b_i c_j with i + j <= 2.
    * FP32: the exact product (the FP32 mode has no split).

    A, B are complex64 (m, k) and (k, n) arrays; products of the low-precision
    parts are exact in FP64 and the sums carry FP64 rounding only, so this is
    the emulation's value up to ~1e-16 relative.
    """
    A = np.asarray(A, dtype=np.complex64)
    B = np.asarray(B, dtype=np.complex64)
    if mode in (MODE_FP16X2, MODE_FP16X2_SCALED):
        if mode == MODE_FP16X2:
            sA = sB = 0
        ah, al = _split_complex_fp16x2(A, sA)
        bh, bl = _split_complex_fp16x2(B, sB)
        main = ah @ bh
        corr = al @ bh + ah @ bl
        return np.ldexp(1.0, -(sA + sB)) * (main + corr / 2048.0)
    if mode == MODE_BF16X3:
        a = _split_complex_bf16x3(A)
        b = _split_complex_bf16x3(B)
        out = np.zeros((A.shape[0], B.shape[1]), dtype=np.complex128)
        for i in range(3):
            for j in range(3 - i):
                out += a[i] @ b[j]
        return out
    if mode == MODE_FP32:
        return A.astype(np.complex128) @ B.astype(np.complex128)
    raise ValueError(mode)


# ---------------------------------------------------------------------------
# Exponent statistics and the selection rule (Sec. 4.1)
# ---------------------------------------------------------------------------

FP16_EMIN = -14   # smallest normal FP16 exponent
FP16_EMAX = 14    # the maximum exponent the paper scales to (Sec. 4.1)
BF16X3_EMIN = -110  # floor for the BF16 three-term split (third term normal)
BF16X3_EMAX = 126   # b0 = bf16(x) must not round to infinity


def exp_stats(M):
    """Exponent statistics of one operand (Sec. 4.1).

    Every real and imaginary FP32 component is one element.  Zeros are
    neutral (counted nowhere); Inf/NaN are counted in ``nonfinite``; for the
    others e = floor(log2|v|) (exact, FP32 subnormals included).
    Returns a dict with nnz, nonfinite, emax (None if nnz == 0),
    n1 = #{e >= -14} (stage 1: above the FP16 minimum normal),
    n2 = #{e >= emax - 28} (stage 2: inside the FP16 window [-14, 14] once
    shifted so that emax maps to 14), n3 = #{e >= -110} (BF16X3 floor).
    """
    M = np.asarray(M)
    if np.iscomplexobj(M):
        comps = np.concatenate([M.real.ravel(), M.imag.ravel()]).astype(np.float32)
    else:
        comps = M.ravel().astype(np.float32)
    finite = np.isfinite(comps)
    nonfinite = int((~finite).sum())
    v = np.abs(comps[finite].astype(np.float64))
    v = v[v != 0]
    nnz = int(v.size)
    if nnz == 0:
        return {"nnz": 0, "nonfinite": nonfinite, "emax": None, "n1": 0, "n2": 0, "n3": 0}
    _, ex = np.frexp(v)          # v = f * 2^ex, f in [0.5, 1)
    e = ex.astype(np.int64) - 1  # floor(log2 v)
    emax = int(e.max())
    return {"nnz": nnz, "nonfinite": nonfinite, "emax": emax,
            "n1": int((e >= FP16_EMIN).sum()),
            "n2": int((e >= emax - 28).sum()),
            "n3": int((e >= BF16X3_EMIN).sum())}


def select_level(st, t=0.1, t3=0.0):
    """Per-operand tolerance level from its statistics (Sec. 4.1).

    Readings: the underflow threshold is a fraction t of the nonzero elements
    (AUTO-t, Sec. 5.2; t = 0 admits no underflow); the FP16 minimum is the
    smallest normal number, 2^-14; an overflow guard e_max <= 14 is added to
    stage 1 (the paper checks underflow only because circuit values are at
    most 1); BF16X3 and FP32 are levels below TF32TCEC's role with their own
    tolerance t3.
    """
    if st["nonfinite"] > 0:
        return MODE_FP32
    nnz = st["nnz"]
    if nnz == 0:
        return MODE_FP16X2
    emax = st["emax"]
    if emax <= FP16_EMAX and (nnz - st["n1"]) <= t * nnz:
        return MODE_FP16X2
    if (nnz - st["n2"]) <= t * nnz:
        return MODE_FP16X2_SCALED
    if emax <= BF16X3_EMAX and (nnz - st["n3"]) <= t3 * nnz:
        return MODE_BF16X3
    return MODE_FP32


def select_mode(stA, stB, t=0.1, t3=0.0):
    """GEMM mode for a pair of operands: the most conservative of the two
    levels (Sec. 4.1: either operand failing a stage moves the GEMM down).
    In the scaled mode each operand is shifted by s = 14 - e_max (0 for an
    all-zero operand) and the result by 2^-(sA+sB) (Sec. 4.2).
    Returns (mode, sA, sB)."""
    mode = max(select_level(stA, t, t3), select_level(stB, t, t3))
    sA = sB = 0
    if mode == MODE_FP16X2_SCALED:
        sA = 0 if stA["nnz"] == 0 else FP16_EMAX - stA["emax"]
        sB = 0 if stB["nnz"] == 0 else FP16_EMAX - stB["emax"]
    return mode, sA, sB


# ---------------------------------------------------------------------------
# Pairwise contraction (Sec. 2.2)
# ---------------------------------------------------------------------------

def zcontract(A, la, B, lb, lc):
    """C[lc] = sum A[la] B[lb] in complex128 by nested loops (C odometer).

    Labels shared by A and B and absent from lc are summed; a label shared by
    A and B and present in lc is a batch label (it indexes A, B and C alike:
    one independent contraction per value, as when the sliced labels of a
    network are kept as an index instead of fixed, Sec. 5.3).  Every label of
    lc appears in at least one input.  A and B may be complex64 or complex128
    (widened exactly).  Returns a complex128 array with axes ordered as lc.
    """
    A = np.ascontiguousarray(A, dtype=np.complex128)
    B = np.ascontiguousarray(B, dtype=np.complex128)
    la, lb, lc = list(la), list(lb), list(lc)
    if A.ndim != len(la) or B.ndim != len(lb):
        raise ValueError("rank/label mismatch")
    union = []
    ext = {}
    for lbls, T in ((la, A), (lb, B)):
        for d, lab in enumerate(lbls):
            if lab in ext and ext[lab] != T.shape[d]:
                raise ValueError("extent mismatch")
            if lab not in ext:
                union.append(lab)
            ext[lab] = T.shape[d]
    summed = [lab for lab in union if lab in la and lab in lb and lab not in lc]
    for lab in lc:
        if lab not in la and lab not in lb:
            raise ValueError("output label must appear in an input")
    for lab in union:
        if lab not in lc and lab not in summed:
            raise ValueError("label summed over a single input is not supported")
    uidx = {lab: i for i, lab in enumerate(union)}
    lab_ext = np.array([ext[lab] for lab in union], dtype=np.int64)
    i32 = lambda xs: np.array([uidx[x] for x in xs], dtype=np.int32)  # noqa: E731
    a_idx, b_idx, c_idx, s_idx = i32(la), i32(lb), i32(lc), i32(summed)
    C = np.zeros(tuple(ext[lab] for lab in lc), dtype=np.complex128)
    lib = _clib()
    f64p = ctypes.POINTER(ctypes.c_double)
    i32p = ctypes.POINTER(ctypes.c_int32)
    i64p = ctypes.POINTER(ctypes.c_int64)
    lib.oracle_zcontract(len(union), lab_ext.ctypes.data_as(i64p),
                         len(la), a_idx.ctypes.data_as(i32p), A.ctypes.data_as(f64p),
                         len(lb), b_idx.ctypes.data_as(i32p), B.ctypes.data_as(f64p),
                         len(lc), c_idx.ctypes.data_as(i32p), C.ctypes.data_as(f64p),
                         len(summed), s_idx.ctypes.data_as(i32p))
    return C
