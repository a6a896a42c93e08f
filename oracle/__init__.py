"""FP64 CPU oracle for the emulated-CGEMM tensor-network hot path.

TEST INFRASTRUCTURE ONLY: this package is imported by ``tests/``, by the
entry point's smoke check and by the benchmark's CPU-baseline leg, and by
nothing else.  The product library (``paper_2303_08989_amd``) never imports,
links or runs it, and it imports nothing from the product.  Its only shared
dependency is ``synth`` (seeded input generation, no arithmetic of the
method).

What it computes, each following the paper (arXiv 2303.08989):

* ``cgemm``           exact complex GEMM in complex128 (Sec. 3, CGEMM as four
                      real products; relative error of Eq. 3);
* ``split_fp16x2``    the two-term FP16 split with the residual scaled by
                      2^11 (Sec. 2.1, Eq. 2), on a power-of-two pre-scaled
                      input (Sec. 4.2, FP16TCEC with scaling);
* ``split_bf16x3``    a three-term bfloat16 split taking the wide-exponent
                      role of the paper's TF32 split (Sec. 2.1, Table 1);
* ``emulated_cgemm``  the value the emulated CGEMM approximates: the sum of
                      split-part products kept by Eq. 2 (or the six BF16
                      products), evaluated in FP64;
* ``exp_stats`` / ``select_mode``  the exponent statistics and the
                      two-stage selection rule of Sec. 4.1;
* ``statevector_amplitudes`` / ``tn_amplitude``  amplitudes <x|U|0> of a
                      circuit (Sec. 5.3, Eq. 4) by brute-force state vector
                      and by tensor-network contraction (Sec. 2.2), the latter
                      optionally sliced (Sec. 5.3);
* ``probability_theta_gradient``  gradients of |<x|U|0>|^2 with respect to
                      per-coupler fSim angles by the product rule (not in the
                      paper; pinned by closed forms and finite differences).

Readings of the paper taken where it is silent or garbled are listed in the
docstrings of the functions that depend on them.
"""
from .core import (  # noqa: F401
    MODE_FP16X2, MODE_FP16X2_SCALED, MODE_BF16X3, MODE_FP32, MODE_NAMES,
    cgemm, rel_fro, fp16_rne, bf16_rne, bf16_to_f32, split_fp16x2, split_bf16x3,
    emulated_cgemm, exp_stats, select_level, select_mode, zcontract, threads,
)
from .circuit import (  # noqa: F401
    statevector, statevector_amplitudes, tn_build, tn_amplitude, tn_amplitude_sliced,
    fidelity, fsim_theta_derivative, probability_theta_gradient,
)
