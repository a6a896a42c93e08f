/*
 * FP64 CPU oracle: complex matrix product and pairwise tensor contraction by
 * plain nested loops.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the reference the HIP path is
 * checked against; nothing in the product library links, includes or calls
 * it.  It shares no code, header or table with the GPU path.
 *
 * oracle_cgemm   C = alpha * op(A) * op(B) + beta * C0, column-major (BLAS
 *                convention), complex64 inputs widened exactly to complex128,
 *                all arithmetic in complex128.  The complex product is written
 *                out from its definition, (ar*br - ai*bi) + i(ar*bi + ai*br):
 *                the paper's CGEMM-as-four-real-products decomposition (Sec. 3;
 *                its printed imaginary part repeats the term Ar*Bi, the
 *                second term must be Ai*Br).  For every output element the
 *                sum runs over k in ascending order.
 * oracle_zcontract  C[lc] = sum over (la u lb) \ lc of A[la] * B[lb] for
 *                dense row-major complex128 tensors: Einstein summation over
 *                the shared edges of a tensor network (Sec. 2.2), by an
 *                odometer over every label.
 */
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* threads the OpenMP loops below use */
int oracle_threads(void) { return omp_get_max_threads(); }

/* op codes: 0 = N, 1 = T, 2 = C (conjugate transpose) */
static inline void load_op(const float *M, int64_t ld, int op, int64_t row, int64_t col,
                           double *re, double *im) {
    /* element (row, col) of op(M), M column-major with leading dimension ld */
    int64_t r = row, c = col;
    if (op != 0) { r = col; c = row; }
    const float *p = M + 2 * (r + c * ld);
    *re = (double)p[0];
    *im = (op == 2) ? -(double)p[1] : (double)p[1];
}

void oracle_cgemm(int64_t m, int64_t n, int64_t k, int opA, int opB,
                  double alpha_re, double alpha_im,
                  const float *A, int64_t lda, const float *B, int64_t ldb,
                  double beta_re, double beta_im, const double *C0, int64_t ldc0,
                  double *C, int64_t ldc) {
    #pragma omp parallel for schedule(dynamic, 1)
    for (int64_t j = 0; j < n; ++j) {
        double *acc = (double *)calloc((size_t)(2 * (m > 0 ? m : 1)), sizeof(double));
        for (int64_t l = 0; l < k; ++l) {
            double br, bi;
            load_op(B, ldb, opB, l, j, &br, &bi);
            for (int64_t i = 0; i < m; ++i) {
                double ar, ai;
                load_op(A, lda, opA, i, l, &ar, &ai);
                acc[2 * i] += ar * br - ai * bi;
                acc[2 * i + 1] += ar * bi + ai * br;
            }
        }
        for (int64_t i = 0; i < m; ++i) {
            double pr = acc[2 * i], pi = acc[2 * i + 1];
            double outr = alpha_re * pr - alpha_im * pi;
            double outi = alpha_re * pi + alpha_im * pr;
            if (C0 && (beta_re != 0.0 || beta_im != 0.0)) {
                double cr = C0[2 * (i + j * ldc0)], ci = C0[2 * (i + j * ldc0) + 1];
                outr += beta_re * cr - beta_im * ci;
                outi += beta_re * ci + beta_im * cr;
            }
            C[2 * (i + j * ldc)] = outr;
            C[2 * (i + j * ldc) + 1] = outi;
        }
        free(acc);
    }
}

/* Row-major strides of a tensor with the given extents. */
static void row_major_strides(int rank, const int64_t *ext, int64_t *stride) {
    int64_t s = 1;
    for (int d = rank - 1; d >= 0; --d) { stride[d] = s; s *= ext[d]; }
}

/*
 * Labels are arbitrary int32 values.  nlab / lab_ext describe the union of
 * labels (lab_ext[u] = extent of label u); la_idx[d] is the union index of
 * A's d-th label, likewise lb_idx and lc_idx.  sum_idx lists the union
 * indices that are summed.  Returns 0.
 */
int oracle_zcontract(int nlab, const int64_t *lab_ext,
                     int ra, const int32_t *la_idx, const double *A,
                     int rb, const int32_t *lb_idx, const double *B,
                     int rc, const int32_t *lc_idx, double *C,
                     int nsum, const int32_t *sum_idx) {
    int64_t *ext_a = (int64_t *)malloc(sizeof(int64_t) * (ra + 1));
    int64_t *ext_b = (int64_t *)malloc(sizeof(int64_t) * (rb + 1));
    int64_t *ext_c = (int64_t *)malloc(sizeof(int64_t) * (rc + 1));
    int64_t *str_a = (int64_t *)malloc(sizeof(int64_t) * (ra + 1));
    int64_t *str_b = (int64_t *)malloc(sizeof(int64_t) * (rb + 1));
    int64_t *str_c = (int64_t *)malloc(sizeof(int64_t) * (rc + 1));
    for (int d = 0; d < ra; ++d) ext_a[d] = lab_ext[la_idx[d]];
    for (int d = 0; d < rb; ++d) ext_b[d] = lab_ext[lb_idx[d]];
    for (int d = 0; d < rc; ++d) ext_c[d] = lab_ext[lc_idx[d]];
    row_major_strides(ra, ext_a, str_a);
    row_major_strides(rb, ext_b, str_b);
    row_major_strides(rc, ext_c, str_c);
    /* per-label stride contribution into A and B */
    int64_t *sa = (int64_t *)calloc((size_t)nlab + 1, sizeof(int64_t));
    int64_t *sb = (int64_t *)calloc((size_t)nlab + 1, sizeof(int64_t));
    for (int d = 0; d < ra; ++d) sa[la_idx[d]] += str_a[d];
    for (int d = 0; d < rb; ++d) sb[lb_idx[d]] += str_b[d];
    int64_t csize = 1, ssize = 1;
    for (int d = 0; d < rc; ++d) csize *= ext_c[d];
    for (int d = 0; d < nsum; ++d) ssize *= lab_ext[sum_idx[d]];

    #pragma omp parallel for schedule(static)
    for (int64_t oc = 0; oc < csize; ++oc) {
        /* decode the output multi-index */
        int64_t base_a = 0, base_b = 0, rem = oc;
        for (int d = 0; d < rc; ++d) {
            int64_t v = rem / str_c[d];
            rem -= v * str_c[d];
            base_a += v * sa[lc_idx[d]];
            base_b += v * sb[lc_idx[d]];
        }
        double accr = 0.0, acci = 0.0;
        for (int64_t os = 0; os < ssize; ++os) {
            /* decode the summed multi-index (last summed label fastest) */
            int64_t off_a = base_a, off_b = base_b, r2 = os;
            for (int d = nsum - 1; d >= 0; --d) {
                int64_t e = lab_ext[sum_idx[d]];
                int64_t v = r2 % e;
                r2 /= e;
                off_a += v * sa[sum_idx[d]];
                off_b += v * sb[sum_idx[d]];
            }
            double ar = A[2 * off_a], ai = A[2 * off_a + 1];
            double br = B[2 * off_b], bi = B[2 * off_b + 1];
            accr += ar * br - ai * bi;
            acci += ar * bi + ai * br;
        }
        C[2 * oc] = accr;
        C[2 * oc + 1] = acci;
    }
    free(ext_a); free(ext_b); free(ext_c);
    free(str_a); free(str_b); free(str_c);
    free(sa); free(sb);
    return 0;
}
