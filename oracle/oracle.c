/*
 * Plain FP64 CPU oracle for sparse x dense products.  TEST INFRASTRUCTURE
 * ONLY: the tests, the smoke check and the CPU-baseline leg of the benchmark
 * may call it; the product path never does.  It shares no code with the HIP
 * library.
 *
 * Every function is the textbook definition written out, with no blocking,
 * fusion or reordering:
 *
 *  - oracle_spmm_f64   inner-product SpMM (Sec. 2.1): for every stored entry
 *                      e of row i, C[i,:] += vals[e] * B[col[e],:], entries in
 *                      stored order, each C row starting from 0.0.  Every
 *                      split of the hybrid format reduces to this sum
 *                      (Alg. 1 only moves entries; Alg. 2/3 add zero padding).
 *  - oracle_spmm_t_f64 dB = A^T * G computed by scattering rows of G
 *                      (no transposed matrix is ever built).
 *  - oracle_sddmm_f64  dA[e] = sum_n G[row(e),n] * B[col(e),n] for every
 *                      stored entry e (explicit zeros and duplicates too).
 *
 * Threads only split independent outputs (rows of C, column slices of dB,
 * entries of dA); every output is summed sequentially in one fixed order,
 * so results are bitwise independent of the thread count.
 */
#include <stdint.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_OK 0
#define ORACLE_EARG -1

static int check_common(int64_t m, int64_t k, int64_t n, const int64_t* row_ptr,
                        const int32_t* col, int64_t ld_in, int64_t ld_out) {
    if (m < 0 || k < 0 || n < 0 || !row_ptr) return ORACLE_EARG;
    if (ld_in < n || ld_out < n) return ORACLE_EARG;
    if (row_ptr[0] != 0) return ORACLE_EARG;
    for (int64_t i = 0; i < m; ++i)
        if (row_ptr[i + 1] < row_ptr[i]) return ORACLE_EARG;
    int64_t nnz = row_ptr[m];
    if (nnz > 0 && !col) return ORACLE_EARG;
    for (int64_t e = 0; e < nnz; ++e)
        if (col[e] < 0 || col[e] >= k) return ORACLE_EARG;
    return ORACLE_OK;
}

static int pick_threads(int nthreads) {
#ifdef _OPENMP
    return nthreads > 0 ? nthreads : omp_get_max_threads();
#else
    (void)nthreads;
    return 1;
#endif
}

/* C (m x n, row-major, ldc) = A (m x k, CSR) * B (k x n, row-major, ldb). */
int oracle_spmm_f64(int64_t m, int64_t k, const int64_t* row_ptr, const int32_t* col,
                    const double* vals, int64_t n, const double* B, int64_t ldb,
                    double* C, int64_t ldc, int nthreads) {
    int rc = check_common(m, k, n, row_ptr, col, ldb, ldc);
    if (rc) return rc;
    int nt = pick_threads(nthreads);
    (void)nt;
#pragma omp parallel for schedule(static) num_threads(nt)
    for (int64_t i = 0; i < m; ++i) {
        double* c = C + i * ldc;
        for (int64_t j = 0; j < n; ++j) c[j] = 0.0;
        for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
            const double a = vals[e];
            const double* b = B + (int64_t)col[e] * ldb;
            for (int64_t j = 0; j < n; ++j) c[j] += a * b[j];
        }
    }
    return ORACLE_OK;
}

/* dB (k x n, ld lddb) = A^T * G, G is m x n (ld ldg).  Row scatter: walk the
 * rows of A in order and add vals[e] * G[i,:] into dB[col[e],:]; each thread
 * owns a slice of the n columns, so no two threads write the same element. */
int oracle_spmm_t_f64(int64_t m, int64_t k, const int64_t* row_ptr, const int32_t* col,
                      const double* vals, int64_t n, const double* G, int64_t ldg,
                      double* dB, int64_t lddb, int nthreads) {
    int rc = check_common(m, k, n, row_ptr, col, ldg, lddb);
    if (rc) return rc;
    int nt = pick_threads(nthreads);
    if (nt > n && n > 0) nt = (int)n;
    if (nt < 1) nt = 1;
#pragma omp parallel num_threads(nt)
    {
        int t = 0, T = 1;
#ifdef _OPENMP
        t = omp_get_thread_num();
        T = omp_get_num_threads();
#endif
        int64_t j0 = n * t / T, j1 = n * (t + 1) / T;
        for (int64_t r = 0; r < k; ++r)
            for (int64_t j = j0; j < j1; ++j) dB[r * lddb + j] = 0.0;
        for (int64_t i = 0; i < m; ++i) {
            const double* g = G + i * ldg;
            for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
                const double a = vals[e];
                double* d = dB + (int64_t)col[e] * lddb;
                for (int64_t j = j0; j < j1; ++j) d[j] += a * g[j];
            }
        }
    }
    return ORACLE_OK;
}

/* dA[e] = <G[row(e),:], B[col(e),:]>, summed over n in ascending order. */
int oracle_sddmm_f64(int64_t m, int64_t k, const int64_t* row_ptr, const int32_t* col,
                     int64_t n, const double* G, int64_t ldg, const double* B,
                     int64_t ldb, double* dA, int nthreads) {
    int rc = check_common(m, k, n, row_ptr, col, ldg, ldb);
    if (rc) return rc;
    int nt = pick_threads(nthreads);
    (void)nt;
#pragma omp parallel for schedule(static) num_threads(nt)
    for (int64_t i = 0; i < m; ++i) {
        const double* g = G + i * ldg;
        for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
            const double* b = B + (int64_t)col[e] * ldb;
            double s = 0.0;
            for (int64_t j = 0; j < n; ++j) s += g[j] * b[j];
            dA[e] = s;
        }
    }
    return ORACLE_OK;
}

int oracle_max_threads(void) { return pick_threads(0); }
