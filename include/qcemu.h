/*
 * qcemu: FP32-accurate complex GEMM by emulation on gfx950 matrix cores, with
 * per-GEMM automatic split-format selection from exponent statistics, and
 * tensor contraction on top of it.
 *
 * Method: Ootomo, Manabe, Harada, Yokota, "Quantum Circuit Simulation by SGEMM
 * Emulation on Tensor Cores and Automatic Precision Selection" (arXiv
 * 2303.08989).  Section numbers below refer to that paper.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Complex numbers are complex64: two interleaved FP32 values (re, im),
 *   8-byte aligned (qce_c32).
 * - Matrices follow the BLAS convention: column-major, element (i, j) of a
 *   matrix with leading dimension ld sits at index i + j * ld.
 * - Tensors are dense row-major (last axis fastest), described by
 *   qce_tensor; every extent is >= 1 and the product of extents fits int64.
 * - Pointers named "device" point to memory on the handle's GPU; pointers
 *   named "host" point to CPU memory.  The caller owns every buffer it passes
 *   in; the library never frees caller memory.
 * - All device work is enqueued on the handle's stream and the call returns
 *   after enqueueing (stream-ordered, like BLAS).  Only the calls documented as
 *   "synchronises" wait for the device.
 * - Errors are reported by return value; no exception crosses this interface.
 *   On an argument error nothing is enqueued and no output is touched.
 *   NaN/Inf in the data are not errors: they force the FP32 mode and
 *   propagate per IEEE.
 * - A handle is not thread-safe: calls on one handle must come from one host
 *   thread at a time.  Calls on one handle share its statistics and workspace
 *   buffers, so they are ordered on the handle's stream.
 */
#ifndef QCEMU_H
#define QCEMU_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct qce_handle qce_handle; /* opaque */

typedef struct {
    float re, im;
} qce_c32;

typedef enum {
    QCE_SUCCESS = 0,
    QCE_ERR_INVALID_VALUE = 1, /* bad argument: sizes, strides, null pointers, labels */
    QCE_ERR_NOT_SUPPORTED = 2, /* well-formed request outside what is implemented */
    QCE_ERR_ALLOC = 3,         /* device memory allocation failed */
    QCE_ERR_HIP = 4,           /* a HIP runtime call or kernel launch failed */
    QCE_ERR_INTERNAL = 5
} qce_status;

/*
 * GEMM computing modes.
 * FP16X2         two-term FP16 split with the residual scaled by 2^11 and
 *                three products per real GEMM (Sec. 2.1, Eq. 2: FP16TCEC).
 * FP16X2_SCALED  the same after shifting each operand by a power of two so
 *                that its largest exponent becomes 14, result shifted back
 *                (Sec. 4, "FP16TCEC w/ scaling").
 * BF16X3         three-term bfloat16 split, six products; takes the role of
 *                TF32TCEC (FP32 exponent range; Sec. 2.1, Table 1), since
 *                gfx950 has no TF32 matrix instruction.
 * FP32           plain FP32 products with FP32 accumulation (the baseline
 *                role of Sec. 5; also the fallback for non-finite data).
 * AUTO           exponent statistics of both operands select one of the
 *                above on the device, with no device-to-host transfer
 *                (Sec. 4.1 and 4.2).
 */
typedef enum {
    QCE_MODE_FP16X2 = 0,
    QCE_MODE_FP16X2_SCALED = 1,
    QCE_MODE_BF16X3 = 2,
    QCE_MODE_FP32 = 3,
    QCE_MODE_AUTO = 4
} qce_mode;

typedef enum { QCE_OP_N = 0, QCE_OP_T = 1, QCE_OP_C = 2 } qce_op;

/* Row-major dense tensor shape: rank >= 0 axes with extents[0..rank-1]. */
typedef struct {
    int32_t rank;
    const int64_t *extents; /* host pointer, rank entries (may be NULL if rank == 0) */
} qce_tensor;

/*
 * Record of the most recent GEMM decision on a handle (Sec. 4.1 statistics
 * and the selected mode).  Index 0 is operand A, index 1 is operand B.
 *   nnz        nonzero finite FP32 components (real and imaginary parts are
 *              separate elements)
 *   n1         components with floor(log2|v|) >= -14 (stage 1: above the
 *              smallest normal FP16)
 *   n2         components with floor(log2|v|) >= emax - 28 (stage 2: inside
 *              the FP16 exponent window once emax is shifted to 14; taken in
 *              the same pass as the other counts); -1 when no statistics ran
 *   n3         components with floor(log2|v|) >= -110 (BF16X3 floor)
 *   nonfinite  Inf/NaN components
 *   emax       largest floor(log2|v|) (INT32_MIN when nnz == 0)
 *   sA, sB     power-of-two shifts applied in FP16X2_SCALED (else 0)
 *   stats_taken 1 if exponent statistics ran, 0 for a forced mode
 */
typedef struct {
    int32_t mode;
    int32_t sA, sB;
    int32_t stats_taken;
    int64_t nnz[2], n1[2], n2[2], n3[2], nonfinite[2];
    int32_t emax[2];
} qce_decision;

/* ---------------------------------------------------------------------- */
/* Handle                                                                 */
/* ---------------------------------------------------------------------- */

/*
 * Create a handle bound to HIP device `device`.  The handle owns its
 * statistics/decision buffers and a workspace that grows on demand.  Reads
 * the environment once (the paper selects implementations by environment
 * variable, Sec. 3):
 *   QCE_MODE           auto | fp16x2 | fp16x2s | bf16x3 | fp32
 *   QCE_UNDERFLOW_TOL  t  in [0, 1], default 0.1 (AUTO-0.1, Sec. 5.2)
 *   QCE_BF16X3_TOL     t3 in [0, 1], default 0
 *   QCE_AUTO_MIN_DIM   size policy threshold for statistics, default 512
 *   QCE_EMUL_MIN_DIM   size policy threshold for emulation, default 512
 *   QCE_FUSED_GATHER   1 (default) or 0: permute fused into the split in
 *                      qce_contract
 *   QCE_SMALLK         1 (default) or 0: GEMMs with k <= 128 and n <= 64
 *                      split their operands as they load them (no panel
 *                      pass); 0 sends them through the panel path
 *   QCE_GROUPED_GEMM   1 (default) or 0: inside a qce_contract group, the
 *                      panel-path GEMMs are recorded and run as one
 *                      grouped launch (0: they run at once, one by one)
 *   QCE_GEMM_SIZE_POLICY 0 (default) or 1: the size policy applies to the
 *                      CGEMM entry points in AUTO mode too
 *                      (qce_set_gemm_size_policy)
 * The stream is the device's null stream until qce_set_stream.
 * Errors: INVALID_VALUE (h NULL, bad device or bad environment value),
 * ALLOC, HIP.
 */
qce_status qce_create(qce_handle **h, int device);

/* Waits for the handle's stream, frees what the handle owns. NULL is a no-op. */
qce_status qce_destroy(qce_handle *h);

/*
 * Use `stream` (a hipStream_t, passed as void*) for all later work.  The
 * previous stream is synchronised first so that work on the two streams
 * cannot overlap on the handle's shared buffers.
 */
qce_status qce_set_stream(qce_handle *h, void *stream);

/* Mode for later calls (overrides QCE_MODE). INVALID_VALUE for unknown m. */
qce_status qce_set_mode(qce_handle *h, qce_mode m);
qce_status qce_get_mode(const qce_handle *h, qce_mode *m);

/*
 * Underflow tolerances of the selection rule (Sec. 4.1; AUTO-t of Sec. 5.2):
 * an operand may use an FP16 mode when at most t * nnz of its nonzero
 * components fall outside the FP16 window, and BF16X3 when at most t3 * nnz
 * fall below 2^-110.  Both in [0, 1], else INVALID_VALUE.
 */
qce_status qce_set_underflow_tolerance(qce_handle *h, double t, double t3);

/*
 * Size policy used by qce_contract when the handle mode is AUTO (Sec. 4.3):
 * min(m, n, k) >= auto_min -> AUTO (statistics + selection); so are
 * output-dominated GEMMs with k >= 64, min(m, n) >= auto_min and
 * m n k >= 8 auto_min^3 (their FP32 products outlast the write of C, and the
 * statistics read only the small operands); otherwise min(m, n, k) >=
 * emul_min -> BF16X3 (the wide-exponent emulation, as the paper uses
 * TF32TCEC there); otherwise FP32.
 * Requires 0 <= emul_min <= auto_min, else INVALID_VALUE.
 * Default auto_min = emul_min = 512: the thresholds are a calibration of
 * statistics cost against GEMM time; the paper's (2048, 512) are its A100
 * values.  The defaults suit qce_contract's grouped circuit contractions,
 * where one statistics launch serves many GEMMs; a lone 512^3 CGEMM call
 * does better with the paper's tiers (BF16X3 without statistics), see
 * qce_set_gemm_size_policy.
 */
qce_status qce_set_size_policy(qce_handle *h, int64_t auto_min, int64_t emul_min);
qce_status qce_get_size_policy(const qce_handle *h, int64_t *auto_min, int64_t *emul_min);

/*
 * Size policy for the CGEMM entry points too (Sec. 4.3, where the library
 * takes statistics only above a size and runs the smaller GEMMs on the wide
 * emulation or plain FP32): enable = 1 makes qce_cgemm_emulated,
 * qce_cgemm_emulated_noalloc, qce_cgemm_strided_batched and
 * qce_cgemm_grouped in AUTO mode run each GEMM in the mode the size policy
 * above gives its (m, n, k) -- AUTO with statistics, BF16X3 or FP32 without
 * statistics; 0 (the default) keeps AUTO = statistics on every GEMM.  The
 * environment variable QCE_GEMM_SIZE_POLICY (0 or 1) sets it at
 * qce_create.  INVALID_VALUE for other values.
 */
qce_status qce_set_gemm_size_policy(qce_handle *h, int32_t enable);

/*
 * Tile of the panel GEMM kernel for later calls: 128 (128 x 128 outputs per
 * workgroup), 64 (64 x 64, for outputs too small to occupy the device), or
 * 0 (default): the choice of the library's tile table, written by its
 * autotuner from timings of both tiles (the batched GEMM variants of Sec. 3
 * and the many small GEMMs of sliced networks, Sec. 5.3).  Results do not
 * depend on the tile, except through the number of k splits (split-k
 * shapes: few output tiles, long k), which follows the tile.
 * INVALID_VALUE for any other value.
 */
qce_status qce_set_gemm_tile(qce_handle *h, int32_t tile);

/*
 * Hand the library a caller-owned device workspace of `bytes` bytes (NULL,0
 * returns to library-owned workspace).  If a call needs more than `bytes`,
 * it fails with ALLOC and enqueues nothing.  The library never frees it.
 */
qce_status qce_set_workspace(qce_handle *h, void *device_ptr, size_t bytes);

/* Workspace bytes one qce_cgemm_emulated call of this shape needs. */
size_t qce_cgemm_workspace_size(int64_t m, int64_t n, int64_t k);

/* Workspace bytes one qce_cgemm_strided_batched call needs (0 if batch <= 0). */
size_t qce_cgemm_batched_workspace_size(int64_t m, int64_t n, int64_t k, int64_t batch);

/* ---------------------------------------------------------------------- */
/* GEMM                                                                   */
/* ---------------------------------------------------------------------- */

/*
 * C <- alpha * op(A) * op(B) + beta * C, complex64, BLAS CGEMM semantics
 * (the paper's library replaces cuBLAS CGEMM, Sec. 3), computed in the
 * handle's mode:
 *   - AUTO: exponent statistics of A and B (every element, Sec. 4 first
 *     strategy), the two-stage rule of Sec. 4.1 extended by BF16X3 and FP32
 *     levels, and device-side dispatch (Sec. 4.2): the split launch and the
 *     GEMM launch each read the device mode flag and run the selected mode,
 *     with no device-to-host transfer.  No size policy applies here.
 *   - a forced mode runs that mode without statistics (FP16X2_SCALED still
 *     takes statistics to find its shifts).
 * op(X) = X (QCE_OP_N), X^T (QCE_OP_T) or X^H (QCE_OP_C).
 * A: device, op(A) is m x k; stored as m x k (N) or k x m (T, C) with
 *    leading dimension lda >= max(1, rows stored).  B likewise, k x n, ldb.
 * C: device, m x n, ldc >= max(1, m); must not overlap A or B.
 * alpha, beta: host pointers to complex64 scalars (NULL means 1 and 0).
 *    beta == 0 means C is not read (NaN in C does not propagate).
 * A and B are read-only (the paper scales inputs in place, Sec. 4.2 note;
 * here shifted copies live in the workspace).
 * Irregular shapes -- min(m, n) < 32 or k < 16 -- run a bandwidth-bound
 * FP32 kernel in every mode, as the paper does for its irregular-shape GEMMs
 * (Sec. 5.1.2); the decision record then reports FP32 without statistics.
 * m == 0 or n == 0: success, nothing enqueued.  k == 0: C <- beta * C.
 * Errors: INVALID_VALUE for h NULL, negative sizes, bad op, ld too small,
 *   NULL A/B/C with nonzero sizes, or pointers not 8-byte aligned;
 *   ALLOC / HIP.
 */
qce_status qce_cgemm_emulated(qce_handle *h, qce_op opA, qce_op opB, int64_t m, int64_t n,
                              int64_t k, const qce_c32 *alpha, const qce_c32 *A, int64_t lda,
                              const qce_c32 *B, int64_t ldb, const qce_c32 *beta, qce_c32 *C,
                              int64_t ldc);

/*
 * qce_cgemm_emulated for callers that cannot allocate device memory: code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation.  Same arguments, semantics, errors and results (the same
 * kernels), but the call allocates nothing: the panels, k-split partial
 * tiles and statistics records live in a fixed scratch array that the
 * library holds on every GPU it runs on until the process ends
 * (qce_noalloc_scratch_bytes() bytes: 64 MiB, enough for example for
 * m = n = k = 1024), and no timing record is made.  The handle's workspace
 * is not used.
 * Every call on one GPU shares that GPU's scratch, whatever the handle: calls
 * that may overlap in time on one GPU (different streams, handles or host
 * threads) race and give wrong results; calls ordered on one stream are
 * safe.  Nothing in the scratch has to start at zero.
 * Errors: those of qce_cgemm_emulated, plus INVALID_VALUE when the shape
 * needs more scratch than the fixed size (qce_cgemm_workspace_size(m, n, k)
 * > qce_noalloc_scratch_bytes()); nothing is enqueued then.
 */
qce_status qce_cgemm_emulated_noalloc(qce_handle *h, qce_op opA, qce_op opB, int64_t m, int64_t n,
                                      int64_t k, const qce_c32 *alpha, const qce_c32 *A, int64_t lda,
                                      const qce_c32 *B, int64_t ldb, const qce_c32 *beta, qce_c32 *C,
                                      int64_t ldc);

/* Bytes of the fixed scratch of qce_cgemm_emulated_noalloc. */
size_t qce_noalloc_scratch_bytes(void);

/*
 * Synchronises the handle's stream, then copies the decision record of the
 * most recent qce_cgemm_emulated (or the last GEMM inside qce_contract) to
 * *out (host).  For tests and logging only.  INVALID_VALUE if no GEMM ran.
 */
qce_status qce_get_last_decision(qce_handle *h, qce_decision *out);

/*
 * Batched CGEMM: `batch` independent GEMMs of one shape, entry z being
 *   C_z <- alpha op(A_z) op(B_z) + beta C_z,
 *   A_z = A + z*strideA, B_z = B + z*strideB, C_z = C + z*strideC
 * (strides in complex elements; strideA / strideB may be 0 to share an
 * operand).  The batched variant of the cuBLAS-style CGEMM the paper's
 * library intercepts (Sec. 3), and the grouped launch that runs the same
 * contraction step of many slices at once (Sec. 5.3 slices).
 *
 * One launch per phase for the whole batch (statistics, selection, split,
 * GEMM: the entry is blockIdx.z), and in AUTO mode every entry takes its own
 * decision on the device (Sec. 4.1 rule per GEMM; its own shifts in
 * FP16X2_SCALED).  Irregular shapes run the bandwidth-bound kernel for every
 * entry, as qce_cgemm_emulated does.
 *
 * Errors: as qce_cgemm_emulated, plus INVALID_VALUE for batch < 0 or
 * > 65535, negative strides, or strideC < ldc*(n-1)+m with batch > 1
 * (overlapping outputs).  batch == 0 is a no-op success.
 */
qce_status qce_cgemm_strided_batched(qce_handle *h, qce_op opA, qce_op opB, int64_t m, int64_t n,
                                     int64_t k, const qce_c32 *alpha, const qce_c32 *A, int64_t lda,
                                     int64_t strideA, const qce_c32 *B, int64_t ldb, int64_t strideB,
                                     const qce_c32 *beta, qce_c32 *C, int64_t ldc, int64_t strideC,
                                     int64_t batch);

/*
 * One GEMM of a grouped call: C <- alpha op(A) op(B) + beta C with the
 * arguments of qce_cgemm_emulated (A, B, C device pointers; alpha and beta
 * by value).
 */
typedef struct {
    qce_op opA, opB;
    int64_t m, n, k;
    qce_c32 alpha, beta;
    const qce_c32 *A;
    int64_t lda;
    const qce_c32 *B;
    int64_t ldb;
    qce_c32 *C;
    int64_t ldc;
} qce_gemm_desc;

/*
 * Grouped CGEMM: `count` independent GEMMs of any shapes (descs: host array
 * of count descriptors), computed in the handle's mode -- the batched
 * variants of the cuBLAS-style CGEMM the paper's library replaces (Sec. 3),
 * for the many uneven GEMMs of one step of a sliced network (Sec. 5.3).
 *
 * All entries of matrix-core shape run together, one launch per phase: one
 * statistics launch (AUTO: every entry takes its own decision on the
 * device, Sec. 4.1 / 4.2), one split launch for both operands of every
 * entry, and one persistent GEMM launch whose workgroups take output tiles
 * of all entries from a device work list (heaviest tiles first, spread over
 * the XCDs), each tile running its own entry's mode, plus one launch adding
 * the k-split partial tiles where an entry's k is split.  The tile shape
 * (64 x 64 or 128 x 128) comes from the tuned table applied to the whole
 * group's output (or qce_set_gemm_tile).  Irregular shapes (min(m, n) < 32
 * or k < 16) and k == 0 run their own kernels as in qce_cgemm_emulated.
 * Each entry's result equals that of qce_cgemm_emulated on the same
 * arguments whenever both use the same tile and k splits (always when one
 * entry fills the device or none splits k); otherwise only the order of
 * its FP32 partial sums over k differs.
 *
 * Outputs must not overlap each other or any input.  The descriptors are
 * read before the call returns.  qce_get_batch_decision(h, i) reports entry
 * i (caller order; irregular shapes, k == 0 and empty outputs report FP32
 * without statistics).
 * Errors: INVALID_VALUE for count < 0 or > 65536, NULL descs with
 * count > 0, or any entry failing qce_cgemm_emulated's checks (the message
 * names it; nothing is enqueued); ALLOC / HIP.  count == 0: no-op success.
 */
qce_status qce_cgemm_grouped(qce_handle *h, int64_t count, const qce_gemm_desc *descs);

/*
 * Synchronises, then copies the decision record of entry `index` of the
 * most recent GEMM call (index 0 for an unbatched call).  Valid until the
 * next call on the handle.  INVALID_VALUE for an index outside the batch.
 */
qce_status qce_get_batch_decision(qce_handle *h, int64_t index, qce_decision *out);

/* ---------------------------------------------------------------------- */
/* Tensor contraction                                                     */
/* ---------------------------------------------------------------------- */

/*
 * C[lc] = sum over the labels shared by A and B of A[la] * B[lb]: one
 * pairwise contraction of a tensor network (Sec. 2.2), computed by
 * transpose-transpose-GEMM-transpose (Sec. 1): operands are permuted on the
 * device only when their labels are not already grouped as the GEMM needs,
 * the GEMM runs through the emulated CGEMM under the size policy (Sec. 4.3),
 * and the result is permuted only if lc's order requires it.  When every
 * extent is 2 (circuit tensors), there are no batch labels and the GEMM is
 * not of irregular shape, an operand that needs a transpose is not copied:
 * the split reads it through its index-bit permutation (the permute and the
 * split are one pass; the K order is then chosen for contiguous reads of
 * both operands, so the summation order over K may differ from that of the
 * copied path).  Likewise a contraction over every label of two such
 * tensors in different orders reads one through its permutation and sums
 * the products in one pass (FP32, a fixed summation order).  Both are
 * disabled by QCE_FUSED_GATHER=0 at qce_create.
 * a, b, c: host shape descriptors; A, B: device complex64 inputs; C: device
 * complex64 output of the shape c describes (must not overlap A or B).
 * la, lb, lc: host int32 label arrays of lengths a->rank, b->rank, c->rank.
 * A label in A, B and C is a batch label: one independent contraction per
 * value (the sliced labels of a network kept as an index instead of fixed,
 * Sec. 5.3); the batch runs as a strided batched GEMM
 * (qce_cgemm_strided_batched semantics, per-entry modes in AUTO), in
 * launches of at most 65535 entries, with the batch labels made outermost.
 * Requirements (else INVALID_VALUE): labels unique within each tensor; a
 * label in both A and B has equal extents there; every label of lc appears
 * in la or lb with the same extent; c's extents match.
 * NOT_SUPPORTED: a label in only one input and not in C (a trace).
 */
qce_status qce_contract(qce_handle *h, const qce_tensor *a, const void *A, const int32_t *la,
                        const qce_tensor *b, const void *B, const int32_t *lb,
                        const qce_tensor *c, void *C, const int32_t *lc);

/*
 * Grouped contractions.  Between qce_group_begin and qce_group_end,
 * every qce_contract call whose GEMM the library would run with the
 * irregular-shape kernel (min(m, n) < 32 or k < 16 per batch entry) and that
 * is small (k <= 1024, at most 2^22 output elements, at most 2^24 products)
 * is recorded instead of launched; qce_group_end runs all recorded ones in
 * one launch (one thread per output element reading the operands through
 * their strides: no transposes; FP32 fused multiply-add, k in a fixed
 * order).  Contractions whose GEMM takes the panel path (matrix-core
 * shapes other than the short-k kernel's, operands not read through a bit
 * permutation, at most 65535 batch entries) are recorded too: qce_group_end
 * runs their operand permutes, then all of them as one grouped GEMM
 * (qce_cgemm_grouped's launches: one statistics, one split, one persistent
 * GEMM launch; each entry in the mode the size policy gives it, AUTO
 * entries selecting their own), then their output permutes.  Results equal
 * those of the same contractions outside a group up to the order of FP32
 * partial sums over k where the group splits k differently.  No decision
 * record is kept for a group's GEMMs.  Other contractions in the group run
 * at once as usual.  The
 * contractions of one group must be independent (none reads another's
 * output), the operands of a recorded contraction must stay allocated and
 * unchanged until qce_group_end has been enqueued (it reads them then), and
 * a recorded output holds its value only after that launch.  This is the
 * grouped launch for launch-bound streams of tiny contractions that a
 * sliced network produces (Sec. 5.3 slices, irregular shapes of
 * Sec. 5.1.2).
 *
 * Descriptors go to a device area owned by the handle through a pinned
 * host mirror; both are reused only after the stream has drained them.
 * Under stream capture the area must already be large enough (run the work
 * once, then qce_group_reset, then capture): otherwise ALLOC.
 * INVALID_VALUE: begin with a group open, end or reset without / with one.
 */
qce_status qce_group_begin(qce_handle *h);
qce_status qce_group_end(qce_handle *h);

/*
 * Synchronises the stream, makes the descriptor area at least reserve_bytes
 * large, and reuses it from its start (before a stream capture: capture the
 * groups into a fresh area).  ALLOC if the area cannot be allocated.
 */
qce_status qce_group_reset(qce_handle *h, size_t reserve_bytes);

/*
 * Axis permutation of a dense row-major complex64 tensor (the "T" of TTGT,
 * Sec. 1): Y has axes (perm[0], ..., perm[rank-1]) of X, i.e. output axis d
 * is input axis perm[d].  X, Y: device, not overlapping.  x: host shape of X.
 * perm: host, a permutation of 0..rank-1, else INVALID_VALUE.
 */
qce_status qce_permute(qce_handle *h, const qce_tensor *x, const void *X, const int32_t *perm,
                       void *Y);

/* ---------------------------------------------------------------------- */
/* FP64 reductions (slice sum and fidelity)                               */
/* ---------------------------------------------------------------------- */

/*
 * acc2[0] += re(*src), acc2[1] += im(*src) in FP64 on the device: the sum of
 * the amplitudes of independent slices of one network (Sec. 5.3).  src and
 * acc2 are device pointers (one complex64 value, two doubles).
 */
qce_status qce_accumulate_f64(qce_handle *h, const qce_c32 *src, double *acc2);

/*
 * acc2[0..1] += (sum re, sum im) of n complex64 values src[0..n) (device),
 * in FP64: the sum of the slice amplitudes that a batched pass over sliced
 * labels returns as one tensor (Sec. 5.3).  Deterministic: fixed-order
 * per-block partial sums, then one block adds them in block order.  Uses the
 * handle's reduction scratch, so calls are stream-ordered per handle.
 * INVALID_VALUE for NULL acc2, n < 0, or NULL src with n > 0.
 */
qce_status qce_accumulate_n_f64(qce_handle *h, const qce_c32 *src, int64_t n, double *acc2);

/*
 * out4 (device, 4 doubles) <- { re(sum conj(b) a), im(sum conj(b) a),
 * sum |a|^2, sum |b|^2 } over n complex64 values of a and b (device), in
 * FP64: the terms of the fidelity |<b|a>|^2 / (<a|a><b|b>) between two
 * amplitude vectors.  n == 0 writes zeros.
 */
qce_status qce_fidelity_f64(qce_handle *h, const qce_c32 *a, const qce_c32 *b, int64_t n,
                            double *out4);

/* ---------------------------------------------------------------------- */
/* Steps of the GEMM path on their own (for tests)                         */
/* ---------------------------------------------------------------------- */

/*
 * Exponent statistics of one rows x cols complex64 matrix X (device,
 * column-major, leading dimension ld >= rows) as defined for qce_decision,
 * with stage 2 always evaluated; t selects nothing here.  Synchronises;
 * writes *out (host): nnz, n1, n2, n3, nonfinite, emax into index 0 of the
 * arrays and the operand's own tolerance level (as a qce_mode value, under
 * the handle's t, t3) into out->mode.
 */
qce_status qce_expstats(qce_handle *h, const qce_c32 *X, int64_t rows, int64_t cols, int64_t ld,
                        qce_decision *out);

/*
 * The split of Sec. 2.1 (Eq. 2) on n complex64 values x (device), written as
 * planes (device, uint16 bit patterns): mode FP16X2 writes 4 planes of n
 * values: hi(re), lo(re), hi(im), lo(im) of x * 2^shift (lo scaled by 2^11);
 * mode BF16X3 writes 6 planes: b0(re), b1(re), b2(re), b0(im), b1(im),
 * b2(im).  Plane p starts at planes + p * n.  Other modes: NOT_SUPPORTED.
 */
qce_status qce_split(qce_handle *h, qce_mode mode, int32_t shift, const qce_c32 *x, int64_t n,
                     uint16_t *planes);

/*
 * The panel writer every GEMM of the library runs (the split of Sec. 2.1,
 * Eq. 2, with the shift of Sec. 4.2), on its own for tests.  It writes the
 * operand P (rows x k) in the library's internal panel format:
 *   chunk (b, c) holds rows 128b..128b+127 and k-values 16c..16c+15 and
 *   starts at byte (b * ceil(k/16) + c) * chunk_bytes;
 *   inside a chunk, plane p, row r (0..127) and 16-byte granule g (k-values
 *   g*E..g*E+E-1, E = 8 two-byte or 4 four-byte values) sit at byte
 *   p * 128 * R + r * R + 16 * (g XOR swz(r)), R = 32 (two-byte planes) or
 *   64 (FP32 planes); swz(r) = ((r >> 2) ^ (r >> 3)) & 1 for two granules
 *   per row, and ((r >> 2) & 1) | ((((r >> 1) ^ (r >> 3)) & 1) << 1) for
 *   four;
 *   planes: FP16X2 / FP16X2_SCALED: hi(re), lo(re), hi(im), lo(im) (FP16
 *   bits of x' = x * 2^shift and of (x' - hi) * 2^11); BF16X3: b0, b1, b2 of
 *   re, then of im (bfloat16 bits); FP32: re, im (FP32 bits);
 *   rows >= rows and k-values >= k are zero.
 * qce_split_panels: layout 0 reads P[r][l] = X[r + l*ld] (ld >= rows),
 *   layout 1 reads P[r][l] = X[l + r*ld] (ld >= k); conj != 0 negates the
 *   imaginary part.  X: device complex64, 8-byte aligned.
 * qce_split_panels_bitmap: the transpose-fused layout of qce_contract:
 *   P[r][l] = X[sum_t bit_t(r) 2^rsh[t] + sum_t bit_t(l) 2^ksh[t]] for a
 *   dense tensor X of 2^(nr+nk) elements (rows = 2^nr, k = 2^nk); rsh (nr
 *   entries) and ksh (nk entries), host arrays, together a permutation of
 *   0..nr+nk-1; 5 <= nr <= 31, 4 <= nk <= 31, nr + nk <= 40.
 * mode: FP16X2 (shift 0), FP16X2_SCALED (any shift in [-150, 150]), BF16X3
 * or FP32 (shift 0), else INVALID_VALUE.  panels: device, 16-byte aligned,
 * qce_panel_bytes(mode, rows, k) bytes, written completely (padding
 * included).  Enqueued on the handle's stream.
 */
size_t qce_panel_bytes(qce_mode mode, int64_t rows, int64_t k);
qce_status qce_split_panels(qce_handle *h, qce_mode mode, int32_t shift, int32_t layout, int32_t conj,
                            const qce_c32 *X, int64_t rows, int64_t k, int64_t ld, void *panels);
qce_status qce_split_panels_bitmap(qce_handle *h, qce_mode mode, int32_t shift, const qce_c32 *X, int32_t nr,
                                   int32_t nk, const int32_t *rsh, const int32_t *ksh, void *panels);

/* ---------------------------------------------------------------------- */
/* Timing and decision log (opt-in tracing)                               */
/* ---------------------------------------------------------------------- */

/*
 * Phases a call is broken into.  An AUTO GEMM launch is credited to the
 * mode it read from the device flag.  GEMM_SKIPPED stays in the enumeration
 * (and in qce_timing) but is never recorded: no launch returns unused.
 */
typedef enum {
    QCE_PHASE_STATS = 0,   /* exponent statistics and mode selection */
    QCE_PHASE_SPLIT = 1,   /* split / scale of both operands */
    QCE_PHASE_GEMM_FP16X2 = 2,
    QCE_PHASE_GEMM_BF16X3 = 3,
    QCE_PHASE_GEMM_FP32 = 4,
    QCE_PHASE_GEMM_SKIPPED = 5,
    QCE_PHASE_PERMUTE = 6,
    QCE_PHASE_OTHER = 7,   /* scaling of C for k == 0, reductions */
    QCE_PHASE_GEMM_IRREGULAR = 8, /* bandwidth-bound FP32 kernel for irregular shapes */
    QCE_PHASE_GEMM_BATCHED = 9,   /* one launch of a batch whose entries chose their modes */
    QCE_NUM_PHASES = 10
} qce_phase;

typedef struct {
    double ms[QCE_NUM_PHASES];     /* summed device time (hipEvent intervals) */
    int64_t count[QCE_NUM_PHASES]; /* intervals summed */
    int64_t gemms_by_mode[4];      /* GEMMs per selected qce_mode (FP16X2..FP32) */
} qce_timing;

/*
 * enable != 0: from now on every phase of every call is bracketed by hipEvents
 * on the handle's stream and the selected mode of every GEMM is logged on the
 * device (no synchronisation while recording).  enable == 0 stops recording;
 * records are kept until qce_reset_timing.
 */
qce_status qce_set_timing(qce_handle *h, int enable);

/* Tag attached to the records of later calls (default 0). */
qce_status qce_set_timing_tag(qce_handle *h, int32_t tag);

/* Drop all records. */
qce_status qce_reset_timing(qce_handle *h);

/*
 * Synchronises the handle's stream and sums the records whose tag equals
 * `tag` (every record if tag < 0) into *out (host).
 */
qce_status qce_get_timing(qce_handle *h, int32_t tag, qce_timing *out);

/* Human-readable name of a status code (static string). */
const char *qce_status_string(qce_status s);

/* Last error message recorded on the handle (static storage per handle). */
const char *qce_last_error(const qce_handle *h);

#ifdef __cplusplus
}
#endif

#endif /* QCEMU_H */
