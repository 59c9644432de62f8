/*
 * Plain FP64 Bellman products for the CPU oracle (test infrastructure only).
 *
 * Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg may
 * load this library.  It shares no code, header or table with the GPU
 * library; it receives the same input arrays.
 *
 * Sec. II of the paper: Q(s, a) = g(s, a) + gamma * sum_{s'} P(s, s', a) V(s'),
 * with P row-stacked (flattened-tensor equation, Sec. III-B.2): row r = s*A + a
 * of the CSR (row_ptr, col, val).  Each row is summed one entry after the
 * other in column order, each product rounded before it is added, exactly as
 * the numpy definition in ipi_oracle.q_values does (np.bincount adds its
 * weights in element order); the build uses -ffp-contract=off so that no
 * multiply-add is fused, and the two agree bit for bit.  Rows are shared out
 * over OpenMP threads; the thread count does not change any result.
 */
#include <stdint.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* Q[r] for every row r < R.  nthreads <= 0: OpenMP's default. */
void orc_q_values(int64_t R, const int64_t* row_ptr, const int32_t* col, const double* val,
                  const double* g, double gamma, const double* V, double* Q, int nthreads) {
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
#pragma omp parallel for schedule(static, 4096)
    for (int64_t r = 0; r < R; ++r) {
        double acc = 0.0;
        for (int64_t j = row_ptr[r]; j < row_ptr[r + 1]; ++j) {
            const double p = val[j] * V[col[j]];
            acc += p;
        }
        const double t = gamma * acc;
        Q[r] = g[r] + t;
    }
}

/* Threads an OpenMP parallel region of this library runs on. */
int orc_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
