/*
 * Plain FP64 CPU oracle for Cleora propagation (Rychalska et al., "Cleora:
 * A Simple, Strong and Scalable Graph Embedding Scheme", arXiv 2102.02302).
 *
 * TEST INFRASTRUCTURE.  Only the tests, the smoke check and the CPU-baseline
 * leg of the benchmark may load this code.  It shares nothing with the GPU
 * library: no headers, no helpers, no tables.  It is written to be checked
 * by eye against the paper, not to be fast: one row loop (OpenMP), FP64
 * throughout, columns of a row summed in ascending order.
 *
 * What it computes (Section 3.2 and Algorithm 1 of the paper):
 *   A[a][b]  = e_ab, the number of edges a->b or the sum of their weights;
 *              an undirected edge {a,b} counts for both a->b and b->a, a loop
 *              {a,a} counts once (Section 3.2; both directions are stored,
 *              Section 4.5).
 *   M[a][b]  = e_ab / deg(a), with deg(a) = sum_b e_ab (row-stochastic).
 *   T_0      ~ U(-1,1), N x d, drawn from a counter-based generator.
 *   T_i      = row-L2-normalise(M . T_{i-1}), i = 1..I; output T_I.
 * Readings where the paper is silent (empty rows, exact zero norms, the
 * generator, self-loops) are listed in the repository's design notes; the
 * flags below select them.
 *
 * Parity status: every function here is pinned by CPU tests against
 * independent definitions (dense recurrences, closed forms, invariants,
 * brute force); none is "parity unpinned".
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_EMPTY_KEEP 1u /* an empty row keeps its previous row (normalised) */
#define ORACLE_NO_NORM 2u    /* skip the row normalisation (plain M^k . T_0) */

/* ------------------------------------------------------------------ init */

/* SplitMix64 output function (Steele, Lea and Flood, "Fast Splittable
 * Pseudorandom Number Generators", OOPSLA 2014): the value the generator
 * returns when its state is x before the golden-gamma increment. */
uint64_t oracle_splitmix64(uint64_t x)
{
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* Entry (i, j) of T_0 (Section 3.2: T_0 ~ U(-1,1)).  Counter = i*d + j with
 * i the node's own (graph-local) index; the top 24 bits of the hash give
 * k in [0, 2^24) and u = k / 2^23 - 1, a value in [-1, 1) that float32
 * represents exactly. */
double oracle_uniform(uint64_t seed, int64_t i, int32_t d, int32_t j)
{
    uint64_t counter = (uint64_t)i * (uint64_t)d + (uint64_t)j;
    uint64_t x = oracle_splitmix64(seed ^ oracle_splitmix64(counter));
    double k = (double)(x >> 40);
    return k / 8388608.0 - 1.0;
}

/* T_0 for rows row0 .. row0+n-1 of a graph, written row-major into T. */
void oracle_init(uint64_t seed, int64_t row0, int64_t n, int32_t d, double *T)
{
    int64_t i;
#pragma omp parallel for schedule(static)
    for (i = 0; i < n; i++)
        for (int32_t j = 0; j < d; j++)
            T[i * d + j] = oracle_uniform(seed, row0 + i, d, j);
}

/* T_0 rows for arbitrary global ids: row i of T is T_0 row ids[i]. */
void oracle_init_ids(uint64_t seed, const int32_t *ids, int64_t n, int32_t d, double *T)
{
    int64_t i;
#pragma omp parallel for schedule(static)
    for (i = 0; i < n; i++)
        for (int32_t j = 0; j < d; j++)
            T[i * d + j] = oracle_uniform(seed, ids[i], d, j);
}

/* ------------------------------------------------------ adjacency build */

typedef struct {
    int32_t col;
    double w;
} entry_t;

static int entry_cmp(const void *pa, const void *pb)
{
    const entry_t *a = (const entry_t *)pa, *b = (const entry_t *)pb;
    if (a->col != b->col) return a->col < b->col ? -1 : 1;
    if (a->w != b->w) return a->w < b->w ? -1 : 1;
    return 0;
}

/* Upper bound on stored entries before merging repeated pairs. */
int64_t oracle_entry_bound(int64_t m, int directed)
{
    return directed ? m : 2 * m;
}

/* Build A (Section 3.2) as CSR: rows ascending, columns ascending within a
 * row, repeated (a,b) pairs merged by summing their counts or weights.
 * Inputs: n nodes, m edges (src[e], dst[e]), optional float32 weights w
 * (NULL: each edge counts 1).  Outputs (caller-allocated): row_ptr[n+1],
 * col[cap], aval[cap] with cap >= oracle_entry_bound(m, directed); *nnz gets
 * the number of merged entries.
 * Returns 0, or -1 if an id is outside [0, n) or a weight is not finite and
 * positive, or -2 if memory runs out. */
int oracle_build_adjacency(int64_t n, int64_t m, const int32_t *src, const int32_t *dst,
                           const float *w, int directed, int64_t *row_ptr, int32_t *col,
                           double *aval, int64_t *nnz)
{
    for (int64_t e = 0; e < m; e++) {
        if (src[e] < 0 || src[e] >= n || dst[e] < 0 || dst[e] >= n) return -1;
        if (w && !(isfinite(w[e]) && w[e] > 0.0f)) return -1;
    }
    int64_t *count = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    if (!count) return -2;
    for (int64_t e = 0; e < m; e++) {
        count[src[e]]++;
        if (!directed && src[e] != dst[e]) count[dst[e]]++;
    }
    int64_t *start = (int64_t *)malloc(((size_t)n + 1) * sizeof(int64_t));
    int64_t total = oracle_entry_bound(m, directed);
    entry_t *ent = (entry_t *)malloc((size_t)(total > 0 ? total : 1) * sizeof(entry_t));
    if (!start || !ent) {
        free(count); free(start); free(ent);
        return -2;
    }
    start[0] = 0;
    for (int64_t a = 0; a < n; a++) start[a + 1] = start[a] + count[a];
    memset(count, 0, ((size_t)n + 1) * sizeof(int64_t));
    for (int64_t e = 0; e < m; e++) {
        double we = w ? (double)w[e] : 1.0;
        int32_t a = src[e], b = dst[e];
        ent[start[a] + count[a]].col = b;
        ent[start[a] + count[a]].w = we;
        count[a]++;
        if (!directed && a != b) {
            ent[start[b] + count[b]].col = a;
            ent[start[b] + count[b]].w = we;
            count[b]++;
        }
    }
    int64_t out = 0;
    row_ptr[0] = 0;
    for (int64_t a = 0; a < n; a++) {
        int64_t lo = start[a], hi = start[a + 1];
        qsort(ent + lo, (size_t)(hi - lo), sizeof(entry_t), entry_cmp);
        for (int64_t p = lo; p < hi; p++) {
            if (p > lo && ent[p].col == ent[p - 1].col) {
                aval[out - 1] += ent[p].w;
            } else {
                col[out] = ent[p].col;
                aval[out] = ent[p].w;
                out++;
            }
        }
        row_ptr[a + 1] = out;
    }
    *nnz = out;
    free(count); free(start); free(ent);
    return 0;
}

/* M = D^-1 A (Section 3.2): deg[a] = sum_b A[a][b]; mval[p] = aval[p] / deg[a].
 * Rows without entries get deg 0 and no values. */
void oracle_transition(int64_t n, const int64_t *row_ptr, const double *aval, double *mval,
                       double *deg)
{
    int64_t a;
#pragma omp parallel for schedule(dynamic, 1024)
    for (a = 0; a < n; a++) {
        double s = 0.0;
        for (int64_t p = row_ptr[a]; p < row_ptr[a + 1]; p++) s += aval[p];
        deg[a] = s;
        for (int64_t p = row_ptr[a]; p < row_ptr[a + 1]; p++) mval[p] = aval[p] / s;
    }
}

/* --------------------------------------------------------- propagation */

/* One iteration of Algorithm 1's inner loop for rows [r0, r1):
 *   U_a = sum_b M[a][b] T_in[b]   (columns b ascending)
 *   T_out[a] = U_a / ||U_a||_2, or the zero row when ||U_a|| = 0.
 * With ORACLE_EMPTY_KEEP an empty row a uses U_a = T_in[a];
 * with ORACLE_NO_NORM the division is skipped. */
void oracle_step_rows(int64_t r0, int64_t r1, int32_t d, const int64_t *row_ptr,
                      const int32_t *col, const double *mval, const double *T_in,
                      double *T_out, unsigned flags)
{
    int64_t a;
#pragma omp parallel for schedule(dynamic, 256)
    for (a = r0; a < r1; a++) {
        double *u = T_out + a * d;
        for (int32_t j = 0; j < d; j++) u[j] = 0.0;
        if (row_ptr[a] == row_ptr[a + 1] && (flags & ORACLE_EMPTY_KEEP)) {
            for (int32_t j = 0; j < d; j++) u[j] = T_in[a * d + j];
        }
        for (int64_t p = row_ptr[a]; p < row_ptr[a + 1]; p++) {
            const double *t = T_in + (int64_t)col[p] * d;
            for (int32_t j = 0; j < d; j++) u[j] += mval[p] * t[j];
        }
        if (flags & ORACLE_NO_NORM) continue;
        double ss = 0.0;
        for (int32_t j = 0; j < d; j++) ss += u[j] * u[j];
        double norm = sqrt(ss);
        for (int32_t j = 0; j < d; j++) u[j] = norm > 0.0 ? u[j] / norm : 0.0;
    }
}

/* I iterations (Algorithm 1): T holds T_0 on entry and T_I on return;
 * tmp is an n x d scratch buffer.  k = 0 leaves T_0 untouched. */
void oracle_propagate(int64_t n, int32_t d, const int64_t *row_ptr, const int32_t *col,
                      const double *mval, double *T, double *tmp, int k, unsigned flags)
{
    for (int t = 0; t < k; t++) {
        oracle_step_rows(0, n, d, row_ptr, col, mval, T, tmp, flags);
        memcpy(T, tmp, (size_t)n * (size_t)d * sizeof(double));
    }
}

/* ------------------------------------------------ sampled rows, k = 1 */

/* Rows `rows[0..r)` of A only (Section 3.2 definition applied to a subset
 * of rows): entries of every edge whose source (or, undirected, either end)
 * is a listed row, merged as in oracle_build_adjacency.  in_sample[a] is
 * the position of row a in `rows` plus one, 0 if a is not listed (caller
 * provides it, size n).  Outputs: sub_ptr[r+1], col[cap], aval[cap];
 * *nnz gets the total.  Returns 0, -1 on invalid input, -2 on no memory,
 * -3 if cap is too small. */
int oracle_adjacency_rows(int64_t n, int64_t m, const int32_t *src, const int32_t *dst,
                          const float *w, int directed, const int64_t *in_sample, int64_t r,
                          int64_t *sub_ptr, int32_t *col, double *aval, int64_t cap,
                          int64_t *nnz)
{
    int64_t *count = (int64_t *)calloc((size_t)r + 1, sizeof(int64_t));
    if (!count) return -2;
    for (int64_t e = 0; e < m; e++) {
        if (src[e] < 0 || src[e] >= n || dst[e] < 0 || dst[e] >= n) {
            free(count);
            return -1;
        }
        if (w && !(isfinite(w[e]) && w[e] > 0.0f)) {
            free(count);
            return -1;
        }
        if (in_sample[src[e]]) count[in_sample[src[e]] - 1]++;
        if (!directed && src[e] != dst[e] && in_sample[dst[e]]) count[in_sample[dst[e]] - 1]++;
    }
    int64_t *start = (int64_t *)malloc(((size_t)r + 1) * sizeof(int64_t));
    if (!start) {
        free(count);
        return -2;
    }
    start[0] = 0;
    for (int64_t i = 0; i < r; i++) start[i + 1] = start[i] + count[i];
    int64_t total = start[r];
    entry_t *ent = (entry_t *)malloc((size_t)(total > 0 ? total : 1) * sizeof(entry_t));
    if (!ent) {
        free(count); free(start);
        return -2;
    }
    memset(count, 0, ((size_t)r + 1) * sizeof(int64_t));
    for (int64_t e = 0; e < m; e++) {
        double we = w ? (double)w[e] : 1.0;
        int64_t ia = in_sample[src[e]], ib = in_sample[dst[e]];
        if (ia) {
            ent[start[ia - 1] + count[ia - 1]].col = dst[e];
            ent[start[ia - 1] + count[ia - 1]].w = we;
            count[ia - 1]++;
        }
        if (!directed && src[e] != dst[e] && ib) {
            ent[start[ib - 1] + count[ib - 1]].col = src[e];
            ent[start[ib - 1] + count[ib - 1]].w = we;
            count[ib - 1]++;
        }
    }
    int64_t out = 0;
    sub_ptr[0] = 0;
    for (int64_t i = 0; i < r; i++) {
        int64_t lo = start[i], hi = start[i + 1];
        qsort(ent + lo, (size_t)(hi - lo), sizeof(entry_t), entry_cmp);
        for (int64_t p = lo; p < hi; p++) {
            if (p > lo && ent[p].col == ent[p - 1].col) {
                aval[out - 1] += ent[p].w;
            } else {
                if (out >= cap) {
                    free(count); free(start); free(ent);
                    return -3;
                }
                col[out] = ent[p].col;
                aval[out] = ent[p].w;
                out++;
            }
        }
        sub_ptr[i + 1] = out;
    }
    *nnz = out;
    free(count); free(start); free(ent);
    return 0;
}

/* T_1 for r sampled rows straight from the seed: with M_ab = e_ab/deg(a)
 * for the listed rows (sub-CSR from oracle_adjacency_rows),
 *   T_1[a] = normalise( sum_b M_ab T_0[b] ),  T_0[b][j] = oracle_uniform(seed, b, d, j)
 * (Algorithm 1, first iteration).  Empty rows give zero rows, or T_0[a]
 * normalised with ORACLE_EMPTY_KEEP.  out is r x d. */
void oracle_t1_rows(int64_t r, const int32_t *rows, int32_t d, uint64_t seed,
                    const int64_t *sub_ptr, const int32_t *col, const double *aval, double *out,
                    unsigned flags)
{
    int64_t i;
#pragma omp parallel for schedule(dynamic, 4)
    for (i = 0; i < r; i++) {
        double *u = out + i * d;
        double deg = 0.0;
        for (int64_t p = sub_ptr[i]; p < sub_ptr[i + 1]; p++) deg += aval[p];
        for (int32_t j = 0; j < d; j++) u[j] = 0.0;
        if (sub_ptr[i] == sub_ptr[i + 1] && (flags & ORACLE_EMPTY_KEEP))
            for (int32_t j = 0; j < d; j++) u[j] = oracle_uniform(seed, rows[i], d, j);
        for (int64_t p = sub_ptr[i]; p < sub_ptr[i + 1]; p++) {
            double mab = aval[p] / deg;
            for (int32_t j = 0; j < d; j++) u[j] += mab * oracle_uniform(seed, col[p], d, j);
        }
        double ss = 0.0;
        for (int32_t j = 0; j < d; j++) ss += u[j] * u[j];
        double norm = sqrt(ss);
        for (int32_t j = 0; j < d; j++) u[j] = norm > 0.0 ? u[j] / norm : 0.0;
    }
}

/* ------------------------------------------------------------- threads */

void oracle_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int oracle_get_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
