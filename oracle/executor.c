/* Parallel CPU executor of a BSP schedule: the kind of executor the paper
 * times on its host (Sec. 6.1), kept with the oracle as the second CPU
 * baseline.  TEST AND BASELINE INFRASTRUCTURE ONLY: called by the tests and
 * by the CPU-baseline leg of the benchmark, never by the product library.
 *
 * The rows are processed superstep by superstep (Definition 2.1): in
 * superstep s every task (the rows of one core in s, in the order of Sec. 5)
 * runs on one thread as plain forward substitution (Eq. (2.1): acc = b_i,
 * acc = acc - A_ij x_j over the stored off-diagonals in order, x_i = acc /
 * A_ii, compiled without contraction), and all threads meet at a barrier
 * before superstep s + 1.  The barrier also makes the superstep's results
 * visible.  Each row's arithmetic is the oracle's, so x is bit for bit the
 * serial result for any valid schedule.
 *
 * Inputs: a lower-triangular CSR (the caller has checked it; this file only
 * executes), order[n] = the rows in the order of Sec. 5, task_beg[ntasks + 1]
 * = the first position of each task in `order`, super_task[S + 1] = the first
 * task of each superstep.  Tasks of a superstep go to the threads in static
 * round-robin order (task t of the superstep on thread t mod T), as the
 * cores of the paper's executor are pinned to threads. */
#include <stdint.h>
#include <omp.h>

static void run_task(const int64_t *row_ptr, const int32_t *col, const double *val, const int32_t *order,
                     int64_t beg, int64_t end, const double *b, double *x)
{
    for (int64_t t = beg; t < end; t++) {
        const int32_t i = order[t];
        const int64_t a = row_ptr[i], d = row_ptr[i + 1] - 1;   /* the diagonal is stored last */
        double acc = b[i];
        for (int64_t p = a; p < d; p++) {
            const double prod = val[p] * x[col[p]];
            acc = acc - prod;
        }
        x[i] = acc / val[d];
    }
}

/* Returns the number of threads used. */
int executor_bsp_omp(int64_t n, const int64_t *row_ptr, const int32_t *col, const double *val,
                     const int32_t *order, const int64_t *task_beg, const int32_t *super_task, int32_t S,
                     const double *b, double *x, int32_t threads)
{
    int used = 1;
    (void)n;
    if (threads < 1) threads = omp_get_max_threads();
#pragma omp parallel num_threads(threads)
    {
#pragma omp single
        used = omp_get_num_threads();
        for (int32_t s = 0; s < S; s++) {
#pragma omp for schedule(static, 1)
            for (int32_t t = super_task[s]; t < super_task[s + 1]; t++)
                run_task(row_ptr, col, val, order, task_beg[t], task_beg[t + 1], b, x);
            /* the implied barrier of the loop ends the superstep */
        }
    }
    return used;
}
