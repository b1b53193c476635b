/*
 * Floyd–Warshall ORACLE — test infrastructure only.
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may load or call this file's library.  It shares no code, header, table or
 * helper with the GPU library; it is deliberately plain and slow.
 *
 * What it computes (the paper, Section "Floyd-Warshall Algorithm"): the
 * input is an N x N matrix D whose entry (i,j) is the direct distance from
 * node i to node j; after N iterations, iteration k having tried every pair
 * (i,j) through the intermediate node k, D(i,j) is the shortest distance from
 * i to j.  A second N x N matrix P is produced when paths must be rebuilt.
 *
 * Written out here as the textbook recurrence over the matrices D^(k):
 *
 *     D^(k)(i,j) = min( D^(k-1)(i,j),  D^(k-1)(i,k) (+) D^(k-1)(k,j) )
 *
 * for k = 0..N-1 in order, all (i,j) of step k reading step k-1's values.
 *
 * Readings of points the paper leaves open (each one is also listed in the
 * design notes of the repository):
 *   - "No edge" is INF = 1073741823 for int32 weights and +inf for floating
 *     point.  (+) saturates at INF: a sum with an INF operand is INF.
 *   - Integer sums are formed in int64; floating-point weights are widened to
 *     double and summed in double (exact for integer-valued float32 inputs).
 *   - The comparison is strict: a candidate replaces D(i,j) only if smaller.
 *   - P is the canonical predecessor matrix: P(i,j) is the vertex just before
 *     j on a shortest i->j path, the smallest such vertex when several
 *     shortest paths end differently.  It is carried through the same
 *     recurrence by comparing (distance, candidate predecessor) pairs
 *     lexicographically, the candidate through k being P^(k-1)(k,j).
 *     Before iteration 0, P(i,j) = i for every edge i != j and NONE
 *     (= INT32_MAX, worse than any vertex) otherwise; afterwards NONE, the
 *     diagonal and unreachable pairs read -1.
 *   - A negative diagonal entry after the last iteration means a negative
 *     cycle; the status is then ORC_NEGATIVE_CYCLE and D is unspecified.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_INF   1073741823LL
#define ORC_NONE  INT32_MAX

enum { ORC_OK = 0, ORC_INVALID_VALUE = 2, ORC_NEGATIVE_CYCLE = 3, ORC_NOMEM = 4 };

/* ------------------------------------------------------------ preconditions */

/* Largest |w| allowed for int32 weights at size n: (n-1)|w| < 2^28 keeps
 * every path length and every intermediate sum far from the INF sentinel. */
int64_t oracle_weight_bound(int64_t n)
{
    return n <= 1 ? (1LL << 28) - 1 : ((1LL << 28) - 1) / (n - 1);
}

int oracle_check_i32(const int32_t *W, int64_t n)
{
    const int64_t bound = oracle_weight_bound(n);
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < n; ++j) {
            const int64_t w = W[i * n + j];
            if (i == j) {
                if (w != 0) return ORC_INVALID_VALUE;
            } else if (w != ORC_INF && (w > bound || w < -bound)) {
                return ORC_INVALID_VALUE;
            }
        }
    return ORC_OK;
}

int oracle_check_f32(const float *W, int64_t n)
{
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < n; ++j) {
            const float w = W[i * n + j];
            if (isnan(w) || w == -INFINITY) return ORC_INVALID_VALUE;
            if (i == j && w != 0.0f) return ORC_INVALID_VALUE;
        }
    return ORC_OK;
}

/* ------------------------------------------------------------ predecessors */

void oracle_pred_init_i32(const int32_t *W, int32_t *P, int64_t n)
{
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < n; ++j)
            P[i * n + j] = (i != j && W[i * n + j] != ORC_INF) ? (int32_t)i : ORC_NONE;
}

void oracle_pred_init_f64(const double *W, int32_t *P, int64_t n)
{
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < n; ++j)
            P[i * n + j] = (i != j && W[i * n + j] != INFINITY) ? (int32_t)i : ORC_NONE;
}

/* --------------------------------------------------------- the recurrence */

static inline int64_t sat_add(int64_t a, int64_t b)
{
    if (a == ORC_INF || b == ORC_INF) return ORC_INF;
    int64_t s = a + b;
    if (s > ORC_INF) s = ORC_INF;           /* saturate at the sentinel */
    if (s < -(int64_t)INT32_MAX) s = -(int64_t)INT32_MAX;  /* only with negative cycles */
    return s;
}

/* Iterations k0 <= k < k1 of the recurrence on int32 distances, in place.
 * P may be NULL (distances only). */
int oracle_fw_i32_steps(int32_t *D, int32_t *P, int64_t n, int64_t k0, int64_t k1, int threads)
{
    int32_t *drow = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    int32_t *prow = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    if (!drow || !prow) { free(drow); free(prow); return ORC_NOMEM; }
    if (threads < 1) threads = 1;
    for (int64_t k = k0; k < k1; ++k) {
        /* step k reads row k and column k of D^(k-1) */
        memcpy(drow, D + k * n, (size_t)n * sizeof(int32_t));
        if (P) memcpy(prow, P + k * n, (size_t)n * sizeof(int32_t));
#pragma omp parallel for num_threads(threads) schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            const int64_t a = D[i * n + k];
            int32_t *di = D + i * n;
            int32_t *pi = P ? P + i * n : NULL;
            for (int64_t j = 0; j < n; ++j) {
                const int64_t s = sat_add(a, drow[j]);
                const int64_t d = di[j];
                if (s < d) {
                    di[j] = (int32_t)s;
                    if (pi) pi[j] = prow[j];
                } else if (pi && s == d && s != ORC_INF && prow[j] < pi[j]) {
                    pi[j] = prow[j];
                }
            }
        }
    }
    free(drow);
    free(prow);
    return ORC_OK;
}

/* Same recurrence in double precision; INF is +inf. */
int oracle_fw_f64_steps(double *D, int32_t *P, int64_t n, int64_t k0, int64_t k1, int threads)
{
    double *drow = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    int32_t *prow = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    if (!drow || !prow) { free(drow); free(prow); return ORC_NOMEM; }
    if (threads < 1) threads = 1;
    for (int64_t k = k0; k < k1; ++k) {
        memcpy(drow, D + k * n, (size_t)n * sizeof(double));
        if (P) memcpy(prow, P + k * n, (size_t)n * sizeof(int32_t));
#pragma omp parallel for num_threads(threads) schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            const double a = D[i * n + k];
            double *di = D + i * n;
            int32_t *pi = P ? P + i * n : NULL;
            for (int64_t j = 0; j < n; ++j) {
                const double s = a + drow[j];
                const double d = di[j];
                if (s < d) {
                    di[j] = s;
                    if (pi) pi[j] = prow[j];
                } else if (pi && s == d && s != INFINITY && prow[j] < pi[j]) {
                    pi[j] = prow[j];
                }
            }
        }
    }
    free(drow);
    free(prow);
    return ORC_OK;
}

/* After the last iteration: detect negative cycles, give P its output form. */
int oracle_finalize_i32(const int32_t *D, int32_t *P, int64_t n)
{
    int status = ORC_OK;
    for (int64_t i = 0; i < n; ++i)
        if (D[i * n + i] < 0) status = ORC_NEGATIVE_CYCLE;
    if (P)
        for (int64_t i = 0; i < n; ++i)
            for (int64_t j = 0; j < n; ++j)
                if (i == j || D[i * n + j] == ORC_INF || P[i * n + j] == ORC_NONE)
                    P[i * n + j] = -1;
    return status;
}

int oracle_finalize_f64(const double *D, int32_t *P, int64_t n)
{
    int status = ORC_OK;
    for (int64_t i = 0; i < n; ++i)
        if (D[i * n + i] < 0) status = ORC_NEGATIVE_CYCLE;
    if (P)
        for (int64_t i = 0; i < n; ++i)
            for (int64_t j = 0; j < n; ++j)
                if (i == j || D[i * n + j] == INFINITY || P[i * n + j] == ORC_NONE)
                    P[i * n + j] = -1;
    return status;
}

/* Whole solve: initialise P (if wanted), run all N iterations, finalise. */
int oracle_fw_i32(int32_t *D, int32_t *P, int64_t n, int threads)
{
    if (P) oracle_pred_init_i32(D, P, n);
    int st = oracle_fw_i32_steps(D, P, n, 0, n, threads);
    if (st != ORC_OK) return st;
    return oracle_finalize_i32(D, P, n);
}

int oracle_fw_f64(double *D, int32_t *P, int64_t n, int threads)
{
    if (P) oracle_pred_init_f64(D, P, n);
    int st = oracle_fw_f64_steps(D, P, n, 0, n, threads);
    if (st != ORC_OK) return st;
    return oracle_finalize_f64(D, P, n);
}

/* ---------------------------------------------------------- one row alone
 *
 * Row src of the result, for sizes where the full N^3 recurrence is too
 * slow: the same quantity by its definition, the least total weight over
 * all src->j paths, found by label correcting (a vertex is re-scanned
 * whenever its distance drops, which stays exact with negative edge weights
 * as long as no negative cycle is reachable; Bellman-Ford's bound of N-1
 * improvements per vertex detects one).  The predecessor is then the
 * closed form of the canonical rule:
 *     P(src,j) = min { v != j : W(v,j) finite, D(src,v) (+) W(v,j) = D(src,j) }.
 */
int oracle_row_i32(const int32_t *W, int64_t n, int64_t src, int32_t *drow, int32_t *prow)
{
    int64_t *dist = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    int64_t *queue = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    char *inq = (char *)calloc((size_t)n, 1);
    int64_t *count = (int64_t *)calloc((size_t)n, sizeof(int64_t));
    if (!dist || !queue || !inq || !count) {
        free(dist); free(queue); free(inq); free(count);
        return ORC_NOMEM;
    }
    for (int64_t v = 0; v < n; ++v) dist[v] = ORC_INF;
    dist[src] = 0;
    int64_t head = 0, size = 0;
    queue[0] = src; inq[src] = 1; size = 1;
    int status = ORC_OK;
    while (size > 0 && status == ORC_OK) {
        const int64_t u = queue[head];
        head = (head + 1) % n; --size; inq[u] = 0;
        const int32_t *wu = W + u * n;
        for (int64_t v = 0; v < n; ++v) {
            if (v == u || wu[v] == ORC_INF) continue;
            const int64_t s = sat_add(dist[u], wu[v]);
            if (s < dist[v]) {
                dist[v] = s;
                if (++count[v] >= n) { status = ORC_NEGATIVE_CYCLE; break; }
                if (!inq[v]) { queue[(head + size) % n] = v; ++size; inq[v] = 1; }
            }
        }
    }
    if (dist[src] < 0) status = ORC_NEGATIVE_CYCLE;
    for (int64_t j = 0; j < n; ++j) drow[j] = (int32_t)dist[j];
    if (prow) {
        for (int64_t j = 0; j < n; ++j) prow[j] = ORC_NONE;
        for (int64_t v = 0; v < n; ++v) {          /* ascending v: first match is the minimum */
            if (dist[v] == ORC_INF) continue;
            const int32_t *wv = W + v * n;
            for (int64_t j = 0; j < n; ++j) {
                if (j == v || prow[j] != ORC_NONE || wv[j] == ORC_INF || dist[j] == ORC_INF)
                    continue;
                if (sat_add(dist[v], wv[j]) == dist[j]) prow[j] = (int32_t)v;
            }
        }
        for (int64_t j = 0; j < n; ++j)
            if (j == src || dist[j] == ORC_INF || prow[j] == ORC_NONE) prow[j] = -1;
    }
    free(dist); free(queue); free(inq); free(count);
    return status;
}

/* Float weights (read as float32, summed in double). */
int oracle_row_f64(const float *W, int64_t n, int64_t src, double *drow, int32_t *prow)
{
    int64_t *queue = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    char *inq = (char *)calloc((size_t)n, 1);
    int64_t *count = (int64_t *)calloc((size_t)n, sizeof(int64_t));
    if (!queue || !inq || !count) { free(queue); free(inq); free(count); return ORC_NOMEM; }
    double *dist = drow;
    for (int64_t v = 0; v < n; ++v) dist[v] = INFINITY;
    dist[src] = 0.0;
    int64_t head = 0, size = 1;
    queue[0] = src; inq[src] = 1;
    int status = ORC_OK;
    while (size > 0 && status == ORC_OK) {
        const int64_t u = queue[head];
        head = (head + 1) % n; --size; inq[u] = 0;
        const float *wu = W + u * n;
        for (int64_t v = 0; v < n; ++v) {
            if (v == u || wu[v] == INFINITY) continue;
            const double s = dist[u] + (double)wu[v];
            if (s < dist[v]) {
                dist[v] = s;
                if (++count[v] >= n) { status = ORC_NEGATIVE_CYCLE; break; }
                if (!inq[v]) { queue[(head + size) % n] = v; ++size; inq[v] = 1; }
            }
        }
    }
    if (dist[src] < 0) status = ORC_NEGATIVE_CYCLE;
    if (prow) {
        for (int64_t j = 0; j < n; ++j) prow[j] = ORC_NONE;
        for (int64_t v = 0; v < n; ++v) {
            if (dist[v] == INFINITY) continue;
            const float *wv = W + v * n;
            for (int64_t j = 0; j < n; ++j) {
                if (j == v || prow[j] != ORC_NONE || wv[j] == INFINITY || dist[j] == INFINITY)
                    continue;
                if (dist[v] + (double)wv[j] == dist[j]) prow[j] = (int32_t)v;
            }
        }
        for (int64_t j = 0; j < n; ++j)
            if (j == src || dist[j] == INFINITY || prow[j] == ORC_NONE) prow[j] = -1;
    }
    free(queue); free(inq); free(count);
    return status;
}
