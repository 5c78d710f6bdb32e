/*
 * Oracle: the naive method (Section 2.1, the formula for c_ij and Algorithm 1)
 * in IEEE double precision on the host CPU.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the library links, loads or calls this
 * file; only the test suite, the smoke check and the benchmark's CPU-baseline
 * leg do.  It shares no code, header or constant with the GPU path.
 *
 * Reading of the paper (dimension names): the section on the naive method
 * writes A (m x n) times B (n x k) and reuses the letter k as the loop index;
 * the cutoff section writes A (m x k) times B (k x n).  This file uses the
 * latter: A is m x k, B is k x n, C is m x n, all row-major with leading
 * dimensions lda, ldb, ldc (in elements).  The inner index is p.
 *
 *     c_ij = sum_{p=0}^{k-1} a_ip * b_pj        (summed in the order p = 0, 1, ...)
 *
 * Loop order i-p-j: each c_ij still receives its k terms in increasing p with
 * one rounding per addition, exactly as the running sum of Algorithm 1 does;
 * only the traversal of j is hoisted inside so the compiler can vectorise it.
 * The file is compiled with -ffp-contract=off, so a*b+c is never fused and
 * every product and every sum is rounded once, in the order written.
 * OpenMP splits the rows i among threads; each c_ij is owned by one thread, so
 * the result does not depend on the thread count.
 */
#include <stdint.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Returns 0 on success, -1 on a negative size or a leading dimension shorter
 * than its row. */
int oracle_gemm_f64(int64_t m, int64_t n, int64_t k,
                    const double *A, int64_t lda,
                    const double *B, int64_t ldb,
                    double *C, int64_t ldc, int nthreads)
{
    if (m < 0 || n < 0 || k < 0) return -1;
    if ((m > 0 && lda < k) || (k > 0 && ldb < n) || (m > 0 && ldc < n)) return -1;
#ifdef _OPENMP
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(static) num_threads(nthreads)
#endif
    for (int64_t i = 0; i < m; ++i) {
        double *c = C + i * ldc;
        for (int64_t j = 0; j < n; ++j) c[j] = 0.0;
        for (int64_t p = 0; p < k; ++p) {
            const double a = A[i * lda + p];
            const double *b = B + p * ldb;
            for (int64_t j = 0; j < n; ++j) c[j] = c[j] + a * b[j];
        }
    }
    (void)nthreads;
    return 0;
}

/* Number of threads OpenMP would use by default (1 without OpenMP). */
int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
