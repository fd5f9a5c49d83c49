/*
 * CPU oracle for the GrowLocal-scheduled sparse lower-triangular solve.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file: only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark use it.  It shares no code, header or table with the HIP
 * library.
 *
 * Contents, each written from the paper (arxiv 2503.05408):
 *   oracle_solve        forward substitution, Eq. (2.1), Sec. 2.2
 *   oracle_solve_upper  backward substitution, its mirror (Sec. 2.2)
 *   oracle_levels       wavefronts (level sets) of the DAG, Sec. 1 / Sec. 6.2
 *   oracle_validate     validity of a BSP schedule, Definition 2.1
 *   oracle_growlocal    the GrowLocal scheduler, Algorithm 3.1 and Sec. 3
 *   oracle_growlocal_weighted  the same with given vertex weights (used by
 *                       the block-parallel scheduling of Sec. 3.1)
 *   oracle_reorder      schedule-based symmetric permutation, Sec. 5
 *   oracle_bsp_solve    executes a schedule superstep by superstep with strict
 *                       visibility (a value computed on another core is
 *                       readable only after the barrier), Sec. 2.3
 *
 * Matrix convention: square CSR, int64 row pointers, int32 columns, binary64
 * values.  In every row the stored off-diagonal columns ascend and the
 * diagonal is the last stored entry.  The DAG has an edge (j, i) for every
 * stored off-diagonal A[i][j] (structural zeros included), and the weight of
 * vertex i is the number of stored entries in row i, diagonal included
 * (Sec. 2.2).
 *
 * Readings where the paper leaves a choice open (listed with their reasons in
 * the design notes):
 *   - Eq. (2.1) is evaluated as a running subtraction in stored column order,
 *     acc <- b_i; acc <- acc - (A_ij * x_j) for each stored j; x_i <- acc / A_ii,
 *     every operation rounded separately (no fused multiply-add, compile with
 *     -ffp-contract=off), and one correctly rounded division by the diagonal.
 *   - GrowLocal: alpha is a real number starting at alpha0 and multiplied by
 *     the growth factor; core 1 takes vertices while its count is below
 *     floor(alpha); every later core takes vertices while its weight is below
 *     Omega_1; Rule I picks the smallest ID among the vertices exclusive to the
 *     core, else the smallest ID among the vertices free at the barrier; cores
 *     are filled once each, in order; beta = sum / (max + L) in binary64; the
 *     first iteration is worthy, a later one iff beta >= theta * best (best =
 *     the largest beta of the earlier iterations of this superstep); a worthy
 *     iteration in which core 1 received fewer than floor(alpha) vertices is
 *     saturated and becomes the superstep; on the first unworthy iteration the
 *     last worthy one becomes the superstep.
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -fPIC -shared oracle.c
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_EBADCSR -1
#define OR_ENOMEM -2
#define OR_EARG -3

/* ------------------------------------------------------------------------ */
/* matrix checks                                                            */
/* ------------------------------------------------------------------------ */

/* Every row: off-diagonal columns below the row (strictly ascending when
 * `sorted` is set), then the diagonal as the last entry, with a non-zero
 * value (the matrix is non-singular, Sec. 2.2).  A symmetrically permuted
 * matrix keeps each row's entry order, so its columns need not ascend. */
static int check_rows(int64_t n, const int64_t *row_ptr, const int32_t *col, const double *val, int sorted)
{
    if (n < 0 || (n > 0 && (!row_ptr || !col))) return OR_EARG;
    if (n == 0) return OR_OK;
    if (row_ptr[0] != 0) return OR_EBADCSR;
    for (int64_t i = 0; i < n; i++) {
        int64_t a = row_ptr[i], e = row_ptr[i + 1];
        if (e <= a) return OR_EBADCSR;                 /* no diagonal */
        if (col[e - 1] != i) return OR_EBADCSR;         /* diagonal last */
        if (val && val[e - 1] == 0.0) return OR_EBADCSR;
        for (int64_t p = a; p < e - 1; p++) {
            if (col[p] < 0 || col[p] >= i) return OR_EBADCSR;
            if (sorted && p > a && col[p] <= col[p - 1]) return OR_EBADCSR;
        }
    }
    return OR_OK;
}

int oracle_check_csr(int64_t n, const int64_t *row_ptr, const int32_t *col, const double *val)
{
    return check_rows(n, row_ptr, col, val, 1);
}

/* ------------------------------------------------------------------------ */
/* forward substitution, Eq. (2.1)                                          */
/* ------------------------------------------------------------------------ */

/* x_i = (b_i - sum_{j<i} A_ij x_j) / A_ii for i = 0..n-1, rows in order.
 * b and x may be the same array (in-place solve). */
int oracle_solve(int64_t n, const int64_t *row_ptr, const int32_t *col, const double *val,
                 const double *b, double *x)
{
    int rc = check_rows(n, row_ptr, col, val, 0);
    if (rc) return rc;
    for (int64_t i = 0; i < n; i++) {
        int64_t a = row_ptr[i], e = row_ptr[i + 1] - 1;   /* e = diagonal position */
        double acc = b[i];
        for (int64_t p = a; p < e; p++) {
            double prod = val[p] * x[col[p]];
            acc = acc - prod;
        }
        x[i] = acc / val[e];
    }
    return OR_OK;
}

/* Upper-triangular CSR: in every row the diagonal is the first stored entry
 * and the off-diagonal columns ascend above it. */
static int check_rows_upper(int64_t n, const int64_t *row_ptr, const int32_t *col, const double *val)
{
    if (n < 0 || (n > 0 && (!row_ptr || !col))) return OR_EARG;
    if (n == 0) return OR_OK;
    if (row_ptr[0] != 0) return OR_EBADCSR;
    for (int64_t i = 0; i < n; i++) {
        int64_t a = row_ptr[i], e = row_ptr[i + 1];
        if (e <= a) return OR_EBADCSR;                 /* no diagonal */
        if (col[a] != i) return OR_EBADCSR;             /* diagonal first */
        if (val && val[a] == 0.0) return OR_EBADCSR;
        for (int64_t p = a + 1; p < e; p++)
            if (col[p] <= col[p - 1] || col[p] >= n) return OR_EBADCSR;
    }
    return OR_OK;
}

/* Backward substitution, the mirror of Eq. (2.1) (Sec. 2.2: an upper
 * triangular system is solved the same way in the reverse direction):
 * x_i = (b_i - sum_{j>i} A_ij x_j) / A_ii for i = n-1 down to 0, the sum as a
 * running subtraction in stored (rising column) order, one division.  b and
 * x may be the same array. */
int oracle_solve_upper(int64_t n, const int64_t *row_ptr, const int32_t *col, const double *val,
                       const double *b, double *x)
{
    int rc = check_rows_upper(n, row_ptr, col, val);
    if (rc) return rc;
    for (int64_t i = n - 1; i >= 0; i--) {
        int64_t d = row_ptr[i], e = row_ptr[i + 1];   /* d = diagonal position */
        double acc = b[i];
        for (int64_t p = d + 1; p < e; p++) {
            double prod = val[p] * x[col[p]];
            acc = acc - prod;
        }
        x[i] = acc / val[d];
    }
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* wavefronts                                                               */
/* ------------------------------------------------------------------------ */

/* level[i] = 1 for a source, else 1 + max level of its parents.  Returns the
 * number of wavefronts (= vertices on a longest path), or a negative error. */
int64_t oracle_levels(int64_t n, const int64_t *row_ptr, const int32_t *col, int32_t *level)
{
    int rc = oracle_check_csr(n, row_ptr, col, NULL);
    if (rc) return rc;
    int64_t nl = 0;
    for (int64_t i = 0; i < n; i++) {
        int32_t lv = 0;
        for (int64_t p = row_ptr[i]; p < row_ptr[i + 1] - 1; p++)
            if (level[col[p]] > lv) lv = level[col[p]];
        level[i] = lv + 1;
        if (level[i] > nl) nl = level[i];
    }
    return nl;
}

/* ------------------------------------------------------------------------ */
/* Definition 2.1                                                           */
/* ------------------------------------------------------------------------ */

#define OR_VAL_RANGE 1        /* core or superstep out of range            */
#define OR_VAL_ORDER 2        /* sigma(u) > sigma(v) for an edge (u, v)    */
#define OR_VAL_CROSS 3        /* different cores in the same superstep     */
#define OR_VAL_EMPTY 4        /* a superstep number in 0..S-1 is unused    */

/* Checks Def. 2.1 on every edge, cores in [0, k), supersteps in [0, S) with
 * every superstep non-empty.  Supersteps and cores are 0-based here. */
int oracle_validate(int64_t n, const int64_t *row_ptr, const int32_t *col, int32_t k,
                    const int32_t *pi, const int32_t *sigma, int32_t S)
{
    int rc = oracle_check_csr(n, row_ptr, col, NULL);
    if (rc) return rc;
    char *used = calloc((size_t)(S > 0 ? S : 1), 1);
    if (!used) return OR_ENOMEM;
    int res = OR_OK;
    for (int64_t v = 0; v < n && !res; v++) {
        if (pi[v] < 0 || pi[v] >= k || sigma[v] < 0 || sigma[v] >= S) { res = OR_VAL_RANGE; break; }
        used[sigma[v]] = 1;
        for (int64_t p = row_ptr[v]; p < row_ptr[v + 1] - 1; p++) {
            int32_t u = col[p];
            if (sigma[u] > sigma[v]) { res = OR_VAL_ORDER; break; }
            if (pi[u] != pi[v] && !(sigma[u] < sigma[v])) { res = OR_VAL_CROSS; break; }
        }
    }
    for (int32_t s = 0; s < S && !res; s++)
        if (!used[s]) res = OR_VAL_EMPTY;
    free(used);
    return res;
}

/* ------------------------------------------------------------------------ */
/* GrowLocal, Algorithm 3.1                                                 */
/* ------------------------------------------------------------------------ */

/* binary min-heap of vertex IDs */
typedef struct { int32_t *a; int64_t n; } heap_t;

static void heap_push(heap_t *h, int32_t v)
{
    int64_t i = h->n++;
    h->a[i] = v;
    while (i > 0) {
        int64_t par = (i - 1) / 2;
        if (h->a[par] <= h->a[i]) break;
        int32_t t = h->a[par]; h->a[par] = h->a[i]; h->a[i] = t;
        i = par;
    }
}

static int32_t heap_pop(heap_t *h)
{
    int32_t top = h->a[0];
    h->a[0] = h->a[--h->n];
    int64_t i = 0;
    for (;;) {
        int64_t l = 2 * i + 1, r = l + 1, m = i;
        if (l < h->n && h->a[l] < h->a[m]) m = l;
        if (r < h->n && h->a[r] < h->a[m]) m = r;
        if (m == i) break;
        int32_t t = h->a[m]; h->a[m] = h->a[i]; h->a[i] = t;
        i = m;
    }
    return top;
}

static int cmp_i32(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

typedef struct {
    int64_t n;
    int32_t k;
    const int64_t *w;        /* vertex weights                               */
    const int64_t *cptr;     /* children lists (transpose of the parents)    */
    const int32_t *child;
    const int32_t *rem;      /* unassigned parents at the barrier            */
    const int32_t *F;        /* free vertices at the barrier, ascending IDs  */
    int64_t nF;
    /* scratch, valid for a vertex only when stamp[v] == cur_stamp */
    int64_t *stamp;
    int64_t cur_stamp;
    int32_t *rem_it;
    int32_t *core_it;        /* -1: no parent in this superstep yet; q >= 0:
                                all such parents on core q; -2: on several   */
    heap_t X;                /* vertices exclusive to the core being filled  */
} gl_state;

/* One iteration of the inner loop of Algorithm 3.1 with parameter alpha,
 * started from the barrier state.  Writes the assignment in pick order to
 * (av, ap) and returns its length; reports beta and the count of core 1. */
static int64_t gl_iteration(gl_state *st, double alpha, double L, int32_t *av, int32_t *ap,
                            double *beta_out, int64_t *count1_out)
{
    st->cur_stamp++;
    const int64_t cap = (int64_t)floor(alpha);
    int64_t ptr = 0, na = 0;
    int64_t omega1 = 0, sum = 0, mx = 0, count1 = 0;
    for (int32_t p = 0; p < st->k; p++) {
        st->X.n = 0;
        int64_t cnt = 0, om = 0;
        for (;;) {
            if (p == 0) { if (cnt >= cap) break; }
            else        { if (om >= omega1) break; }
            int32_t v;
            if (st->X.n > 0) v = heap_pop(&st->X);          /* Rule I (i): exclusive   */
            else if (ptr < st->nF) v = st->F[ptr++];         /* Rule I (ii): smallest ID */
            else break;                                      /* nothing assignable      */
            av[na] = v; ap[na] = p; na++;
            cnt++;
            om += st->w[v];
            for (int64_t c = st->cptr[v]; c < st->cptr[v + 1]; c++) {
                int32_t u = st->child[c];
                if (st->stamp[u] != st->cur_stamp) {
                    st->stamp[u] = st->cur_stamp;
                    st->rem_it[u] = st->rem[u];
                    st->core_it[u] = -1;
                }
                st->rem_it[u]--;
                if (st->core_it[u] == -1) st->core_it[u] = p;
                else if (st->core_it[u] != p) st->core_it[u] = -2;
                /* u is ready; executable only on p if all its parents from this
                 * superstep are on p, otherwise on no core before the barrier */
                if (st->rem_it[u] == 0 && st->core_it[u] == p) heap_push(&st->X, u);
            }
        }
        if (p == 0) { omega1 = om; count1 = cnt; }
        sum += om;
        if (om > mx) mx = om;
        /* later cores can only start from a free vertex */
        if (ptr >= st->nF) break;
    }
    *beta_out = (double)sum / ((double)mx + L);      /* Eq. (3.1) */
    *count1_out = count1;
    return na;
}

/* GrowLocal.  Outputs pi (core, 0..k-1) and sigma (superstep, 0..S-1).
 * Optional trace of every iteration: superstep, alpha, beta, worthy flag,
 * up to max_trace entries; *ntrace receives the total count.
 * weight: vertex weights, or NULL for the stored entries of each row.  The
 * block-parallel form of Sec. 3.1 schedules a diagonal block as its own DAG
 * but keeps the weights of the full matrix's rows. */
int oracle_growlocal_weighted(int64_t n, const int64_t *row_ptr, const int32_t *col, const int64_t *weight,
                              int32_t k, double L, double alpha0, double growth, double theta,
                              int32_t *pi, int32_t *sigma, int32_t *S_out,
                              int64_t max_trace, int32_t *tr_s, double *tr_alpha, double *tr_beta,
                              int8_t *tr_worthy, int64_t *ntrace)
{
    int rc = oracle_check_csr(n, row_ptr, col, NULL);
    if (rc) return rc;
    if (k < 1 || !(alpha0 >= 1.0) || !(growth > 1.0) || !(L >= 0.0)) return OR_EARG;
    int64_t nt = 0;
    if (n == 0) { *S_out = 0; if (ntrace) *ntrace = 0; return OR_OK; }

    int64_t *w = malloc(sizeof(int64_t) * n);
    int64_t *cptr = calloc((size_t)n + 1, sizeof(int64_t));
    int32_t *rem = malloc(sizeof(int32_t) * n);
    int64_t m = row_ptr[n] - n;
    int32_t *child = malloc(sizeof(int32_t) * (m > 0 ? m : 1));
    int64_t *fill = malloc(sizeof(int64_t) * n);
    int32_t *F = malloc(sizeof(int32_t) * n);
    int32_t *F2 = malloc(sizeof(int32_t) * n);
    int8_t *assigned = calloc((size_t)n, 1);
    int64_t *stamp = calloc((size_t)n, sizeof(int64_t));
    int32_t *rem_it = malloc(sizeof(int32_t) * n);
    int32_t *core_it = malloc(sizeof(int32_t) * n);
    int32_t *heap = malloc(sizeof(int32_t) * n);
    int32_t *av = malloc(sizeof(int32_t) * n), *ap = malloc(sizeof(int32_t) * n);
    int32_t *bv = malloc(sizeof(int32_t) * n), *bp = malloc(sizeof(int32_t) * n);
    if (!w || !cptr || !rem || !child || !fill || !F || !F2 || !assigned || !stamp || !rem_it ||
        !core_it || !heap || !av || !ap || !bv || !bp) { rc = OR_ENOMEM; goto done; }

    for (int64_t v = 0; v < n; v++) {
        w[v] = weight ? weight[v] : row_ptr[v + 1] - row_ptr[v];
        rem[v] = (int32_t)(row_ptr[v + 1] - row_ptr[v] - 1);
        for (int64_t p = row_ptr[v]; p < row_ptr[v + 1] - 1; p++) cptr[col[p] + 1]++;
    }
    for (int64_t v = 0; v < n; v++) cptr[v + 1] += cptr[v];
    for (int64_t v = 0; v < n; v++) fill[v] = cptr[v];
    for (int64_t v = 0; v < n; v++)
        for (int64_t p = row_ptr[v]; p < row_ptr[v + 1] - 1; p++) child[fill[col[p]]++] = (int32_t)v;

    int64_t nF = 0;
    for (int64_t v = 0; v < n; v++) if (rem[v] == 0) F[nF++] = (int32_t)v;

    gl_state st = { n, k, w, cptr, child, rem, F, nF, stamp, 0, rem_it, core_it, { heap, 0 } };
    int64_t nassigned = 0;
    int32_t s = 0;
    while (nassigned < n) {
        st.F = F; st.nF = nF;
        double alpha = alpha0, best = 0.0, beta = 0.0;
        int64_t count1 = 0, nbest = 0;
        int iter = 0;
        for (;;) {
            int64_t na = gl_iteration(&st, alpha, L, av, ap, &beta, &count1);
            int worthy = (iter == 0) || (beta >= theta * best);
            if (tr_s && nt < max_trace) {
                tr_s[nt] = s; tr_alpha[nt] = alpha; tr_beta[nt] = beta; tr_worthy[nt] = (int8_t)worthy;
            }
            nt++;
            if (!worthy) break;                      /* keep the last worthy one */
            /* this iteration is now the last worthy one */
            int32_t *t;
            t = bv; bv = av; av = t;
            t = bp; bp = ap; ap = t;
            nbest = na;
            if (iter == 0 || beta > best) best = beta;
            if (count1 < (int64_t)floor(alpha)) break; /* saturated */
            alpha = growth * alpha;
            iter++;
        }
        /* commit the chosen iteration as superstep s */
        int64_t nnew = 0;
        for (int64_t i = 0; i < nbest; i++) {
            int32_t v = bv[i];
            assigned[v] = 1; pi[v] = bp[i]; sigma[v] = s;
        }
        nassigned += nbest;
        for (int64_t i = 0; i < nbest; i++) {
            int32_t v = bv[i];
            for (int64_t c = cptr[v]; c < cptr[v + 1]; c++) {
                int32_t u = child[c];
                if (--rem[u] == 0 && !assigned[u]) F2[nnew++] = u;
            }
        }
        /* free set of the next barrier: the old free vertices not taken plus
         * the vertices whose last parents were assigned in superstep s */
        int64_t nf2 = nnew;
        for (int64_t i = 0; i < nF; i++) if (!assigned[F[i]]) F2[nf2++] = F[i];
        qsort(F2, (size_t)nf2, sizeof(int32_t), cmp_i32);
        int32_t *t = F; F = F2; F2 = t;
        nF = nf2;
        s++;
    }
    *S_out = s;
    rc = OR_OK;
done:
    if (ntrace) *ntrace = nt;
    free(w); free(cptr); free(rem); free(child); free(fill); free(F); free(F2); free(assigned);
    free(stamp); free(rem_it); free(core_it); free(heap); free(av); free(ap); free(bv); free(bp);
    return rc;
}

int oracle_growlocal(int64_t n, const int64_t *row_ptr, const int32_t *col,
                     int32_t k, double L, double alpha0, double growth, double theta,
                     int32_t *pi, int32_t *sigma, int32_t *S_out,
                     int64_t max_trace, int32_t *tr_s, double *tr_alpha, double *tr_beta,
                     int8_t *tr_worthy, int64_t *ntrace)
{
    return oracle_growlocal_weighted(n, row_ptr, col, NULL, k, L, alpha0, growth, theta, pi, sigma, S_out,
                                     max_trace, tr_s, tr_alpha, tr_beta, tr_worthy, ntrace);
}

/* ------------------------------------------------------------------------ */
/* reordering, Sec. 5                                                       */
/* ------------------------------------------------------------------------ */

typedef struct { int32_t s, p, v; } or_key;

static int or_key_cmp(const void *a, const void *b)
{
    const or_key *x = a, *y = b;
    if (x->s != y->s) return x->s < y->s ? -1 : 1;
    if (x->p != y->p) return x->p < y->p ? -1 : 1;
    return (x->v > y->v) - (x->v < y->v);
}

/* perm[t] = the vertex at position t when vertices are listed by superstep,
 * then core, then original ID.  The permuted matrix row t is row perm[t] of A
 * with every column j renamed to inv[j]; the entries keep their stored order.
 * row_ptr2 has n+1 entries; col2/val2 have nnz entries.  Any output pointer
 * may be NULL to skip it. */
int oracle_reorder(int64_t n, const int64_t *row_ptr, const int32_t *col, const double *val,
                   const int32_t *pi, const int32_t *sigma, int32_t *perm,
                   int64_t *row_ptr2, int32_t *col2, double *val2)
{
    if (n == 0) { if (row_ptr2) row_ptr2[0] = 0; return OR_OK; }
    /* order = comparison sort of the (sigma, pi, id) triples */
    or_key *keys = malloc(sizeof(or_key) * n);
    int32_t *inv = malloc(sizeof(int32_t) * n);
    if (!keys || !inv) { free(keys); free(inv); return OR_ENOMEM; }
    for (int64_t v = 0; v < n; v++) { keys[v].s = sigma[v]; keys[v].p = pi[v]; keys[v].v = (int32_t)v; }
    qsort(keys, (size_t)n, sizeof(or_key), or_key_cmp);
    for (int64_t t = 0; t < n; t++) { perm[t] = keys[t].v; inv[keys[t].v] = (int32_t)t; }
    if (row_ptr2) {
        row_ptr2[0] = 0;
        for (int64_t t = 0; t < n; t++) {
            int32_t v = perm[t];
            int64_t len = row_ptr[v + 1] - row_ptr[v];
            row_ptr2[t + 1] = row_ptr2[t] + len;
            for (int64_t q = 0; q < len; q++) {
                if (col2) col2[row_ptr2[t] + q] = inv[col[row_ptr[v] + q]];
                if (val2) val2[row_ptr2[t] + q] = val[row_ptr[v] + q];
            }
        }
    }
    free(keys); free(inv);
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* BSP execution with strict visibility                                     */
/* ------------------------------------------------------------------------ */

/* Runs the rows superstep by superstep, core by core, each core's rows in ID
 * order.  Reading x_j is allowed only if j was computed in an earlier
 * superstep, or earlier on the same core in the same superstep; any other read
 * makes the call return 100 and report the reading row in *bad_row.
 * On success x equals the serial forward substitution bit for bit. */
int oracle_bsp_solve(int64_t n, const int64_t *row_ptr, const int32_t *col, const double *val,
                     const double *b, const int32_t *pi, const int32_t *sigma,
                     double *x, int64_t *bad_row)
{
    int rc = oracle_check_csr(n, row_ptr, col, val);
    if (rc) return rc;
    int32_t *perm = malloc(sizeof(int32_t) * (n > 0 ? n : 1));
    int8_t *done = calloc((size_t)(n > 0 ? n : 1), 1);
    if (!perm || !done) { free(perm); free(done); return OR_ENOMEM; }
    rc = oracle_reorder(n, row_ptr, col, val, pi, sigma, perm, NULL, NULL, NULL);
    for (int64_t t = 0; t < n && !rc; t++) {
        int32_t v = perm[t];
        int64_t a = row_ptr[v], e = row_ptr[v + 1] - 1;
        double acc = b[v];
        for (int64_t p = a; p < e; p++) {
            int32_t j = col[p];
            int visible = (sigma[j] < sigma[v]) ||
                          (sigma[j] == sigma[v] && pi[j] == pi[v] && done[j]);
            if (!visible) { rc = 100; if (bad_row) *bad_row = v; break; }
            double prod = val[p] * x[j];
            acc = acc - prod;
        }
        if (rc) break;
        x[v] = acc / val[e];
        done[v] = 1;
    }
    free(perm); free(done);
    return rc;
}
