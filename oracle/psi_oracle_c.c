/*
 * psi_oracle_c.c — plain FP64 CPU oracle of Power-ψ in C with OpenMP.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the package's smoke check
 * and the benchmark's CPU-baseline leg load this library.  It shares no code,
 * header or table with the HIP library; its input is the raw edge list and the
 * activity vectors as the seeded generators write them.
 *
 * What it computes (Arhachoui, Bautista, Danisch, Giovanidis, ASONAM 2022):
 *   - po_build: the graph is unweighted with no self-loops (Sec. II), so
 *     self-loops and repeated edges are dropped and counted; then the matrix
 *     A of Sec. II, stored by leader i (its column): for every follower j of
 *     i, a_ji = μ_i / den_j with den_j = Σ_{ℓ∈L(j)} (λ_ℓ + μ_ℓ) summed over
 *     the leaders of j in ascending id order; c_i = μ_i/(λ_i+μ_i) and
 *     d_i = λ_i/(λ_i+μ_i) (the diagonals of C and D, Sec. III-A).  A user
 *     with no leaders has den = 0 and a zero row of A and B.
 *   - po_power_psi: Algorithm 2 — the recursion s_t = Aᵀ s_{t−1} + c of
 *     eq. (power_psi) from s_0 = c (or a given start), ended by the test of
 *     eq. (condition) on ε_t = ‖s_t − s_{t−1}‖₁ (times ‖B‖ in mode 1, divided
 *     by ‖s_t‖₁ in mode 2), starting from a gap of 1; then
 *     ψ = (Bᵀ s + d)/N from the final s, with b_ji = λ_i/den_j.
 *   - po_residual: r = Aᵀ s + c − s, the fixed-point residual of
 *     eq. (power_psi), for any given s;  po_final: ψ = (Bᵀ s + d)/N.
 *
 * Sums: (Aᵀ s)_i adds a_ji s_j over the followers j of i in ascending id
 * order, starting from 0, and c_i is added afterwards; every L1 norm adds
 * blocks of 4096 users in order, each block in order, so every result is the
 * same for any number of threads.  No reordering, fusion or blocking of the
 * arithmetic beyond that.  The build sorts with OpenMP counting sorts whose
 * rows are then sorted by id, so its output does not depend on thread order.
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -shared -fPIC.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>

enum { PO_OK = 0, PO_EINVAL = 1, PO_ENOTCONV = 2, PO_ENUMERIC = 4, PO_ENOMEM = 7 };

typedef struct po_graph {
    int64_t n;
    int64_t m;              /* edges kept                               */
    int64_t m_in;           /* edges given                              */
    int64_t n_self_loops;
    int64_t n_duplicates;
    int64_t n_no_leaders;
    int64_t max_followers;
    int64_t* row;           /* [n+1]: followers of leader i             */
    int32_t* fol;           /* [m]:   follower ids, ascending per row   */
    double* a;              /* [m]:   a_ji = μ_i / den_j                 */
    double* den;            /* [n]                                       */
    double* lam;            /* [n]                                       */
    double* mu;             /* [n]                                       */
    double* c;              /* [n]                                       */
    double* d;              /* [n]                                       */
} po_graph;

static char g_err[256];
const char* po_last_error(void) { return g_err; }

static void set_err(const char* s) {
    strncpy(g_err, s, sizeof g_err - 1);
    g_err[sizeof g_err - 1] = 0;
}

void po_set_threads(int k) {
    if (k > 0) omp_set_num_threads(k);
}

int po_max_threads(void) { return omp_get_max_threads(); }

static int cmp_i32(const void* x, const void* y) {
    int32_t a = *(const int32_t*)x, b = *(const int32_t*)y;
    return (a > b) - (a < b);
}

void po_free(po_graph* g) {
    if (!g) return;
    free(g->row); free(g->fol); free(g->a); free(g->den);
    free(g->lam); free(g->mu); free(g->c); free(g->d);
    free(g);
}

/* Rows of `key` with the values `val` (edges with skip[k] set are left out):
 * counting sort (scatter order depends on threads), then every row sorted by
 * value, so the result does not.  ptr: [n+1], out: [number kept]. */
static void rows_by_key(int64_t n, int64_t m, const int32_t* key, const int32_t* val,
                        const uint8_t* skip, int64_t* ptr, int32_t* out) {
    int64_t* cur = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < m; ++k) {
        if (skip && skip[k]) continue;
#pragma omp atomic
        cur[key[k] + 1]++;
    }
    ptr[0] = 0;
    for (int64_t i = 0; i < n; ++i) ptr[i + 1] = ptr[i] + cur[i + 1];
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) cur[i] = ptr[i];
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < m; ++k) {
        if (skip && skip[k]) continue;
        int64_t at;
#pragma omp atomic capture
        at = cur[key[k]]++;
        out[at] = val[k];
    }
    free(cur);
#pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t i = 0; i < n; ++i)
        qsort(out + ptr[i], (size_t)(ptr[i + 1] - ptr[i]), sizeof(int32_t), cmp_i32);
}

/* Build the operator from the raw edge list: edge k means follower[k]
 * follows leader[k].  Returns PO_OK and *out, or an error (po_last_error). */
int po_build(int64_t n, int64_t m, const int32_t* follower, const int32_t* leader,
             const double* lam, const double* mu, po_graph** out) {
    *out = NULL;
    if (n <= 0 || m < 0) { set_err("n must be > 0 and m >= 0"); return PO_EINVAL; }
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (int64_t k = 0; k < m; ++k)
        if (follower[k] < 0 || follower[k] >= n || leader[k] < 0 || leader[k] >= n) bad |= 1;
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (int64_t i = 0; i < n; ++i)
        if (!(isfinite(lam[i]) && lam[i] > 0 && isfinite(mu[i]) && mu[i] >= 0)) bad |= 2;
    if (bad & 1) { set_err("edge endpoint out of range"); return PO_EINVAL; }
    if (bad & 2) { set_err("need finite lambda > 0 and mu >= 0"); return PO_EINVAL; }

    po_graph* g = (po_graph*)calloc(1, sizeof(po_graph));
    g->n = n;
    g->m_in = m;
    uint8_t* loop = (uint8_t*)malloc((size_t)(m > 0 ? m : 1));
    int64_t loops = 0;
#pragma omp parallel for schedule(static) reduction(+ : loops)
    for (int64_t k = 0; k < m; ++k) {
        loop[k] = follower[k] == leader[k];
        loops += loop[k];
    }
    g->n_self_loops = loops;

    /* followers of each leader, ascending, repeats removed */
    int64_t* ptr = (int64_t*)malloc(((size_t)n + 1) * sizeof(int64_t));
    int32_t* fol = (int32_t*)malloc((size_t)(m - loops > 0 ? m - loops : 1) * sizeof(int32_t));
    if (!loop || !ptr || !fol) { set_err("out of host memory"); free(loop); free(ptr); free(fol); po_free(g); return PO_ENOMEM; }
    rows_by_key(n, m, leader, follower, loop, ptr, fol);
    free(loop);
    int64_t* kept = (int64_t*)malloc(((size_t)n + 1) * sizeof(int64_t));
    kept[0] = 0;
#pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t i = 0; i < n; ++i) {
        int64_t w = ptr[i];
        for (int64_t e = ptr[i]; e < ptr[i + 1]; ++e)
            if (e == ptr[i] || fol[e] != fol[e - 1]) fol[w++] = fol[e];
        kept[i + 1] = w - ptr[i];
    }
    g->row = (int64_t*)malloc(((size_t)n + 1) * sizeof(int64_t));
    g->row[0] = 0;
    for (int64_t i = 0; i < n; ++i) g->row[i + 1] = g->row[i] + kept[i + 1];
    free(kept);
    g->m = g->row[n];
    g->n_duplicates = (m - loops) - g->m;
    g->fol = (int32_t*)malloc((size_t)(g->m > 0 ? g->m : 1) * sizeof(int32_t));
    int64_t maxf = 0;
#pragma omp parallel for schedule(dynamic, 1024) reduction(max : maxf)
    for (int64_t i = 0; i < n; ++i) {
        int64_t len = g->row[i + 1] - g->row[i];
        memcpy(g->fol + g->row[i], fol + ptr[i], (size_t)len * sizeof(int32_t));
        if (len > maxf) maxf = len;
    }
    g->max_followers = maxf;
    free(fol);

    /* leaders of each follower, ascending: den_j in that order */
    int32_t* lead_of = (int32_t*)malloc((size_t)(g->m > 0 ? g->m : 1) * sizeof(int32_t));
    int32_t* fol_key = (int32_t*)malloc((size_t)(g->m > 0 ? g->m : 1) * sizeof(int32_t));
    int32_t* lead_val = (int32_t*)malloc((size_t)(g->m > 0 ? g->m : 1) * sizeof(int32_t));
    if (!lead_of || !fol_key || !lead_val) { set_err("out of host memory"); free(lead_of); free(fol_key); free(lead_val); free(ptr); po_free(g); return PO_ENOMEM; }
#pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t i = 0; i < n; ++i)
        for (int64_t e = g->row[i]; e < g->row[i + 1]; ++e) {
            fol_key[e] = g->fol[e];
            lead_val[e] = (int32_t)i;
        }
    rows_by_key(n, g->m, fol_key, lead_val, NULL, ptr, lead_of);
    free(fol_key);
    free(lead_val);

    g->lam = (double*)malloc((size_t)n * sizeof(double));
    g->mu = (double*)malloc((size_t)n * sizeof(double));
    g->den = (double*)malloc((size_t)n * sizeof(double));
    g->c = (double*)malloc((size_t)n * sizeof(double));
    g->d = (double*)malloc((size_t)n * sizeof(double));
    int64_t empty = 0;
#pragma omp parallel for schedule(static) reduction(+ : empty)
    for (int64_t j = 0; j < n; ++j) {
        double s = 0.0;
        for (int64_t e = ptr[j]; e < ptr[j + 1]; ++e) s += lam[lead_of[e]] + mu[lead_of[e]];
        g->den[j] = s;
        empty += ptr[j + 1] == ptr[j];
        g->lam[j] = lam[j];
        g->mu[j] = mu[j];
        g->c[j] = mu[j] / (lam[j] + mu[j]);
        g->d[j] = lam[j] / (lam[j] + mu[j]);
    }
    g->n_no_leaders = empty;
    free(lead_of);
    free(ptr);

    g->a = (double*)malloc((size_t)(g->m > 0 ? g->m : 1) * sizeof(double));
    if (!g->a) { set_err("out of host memory"); po_free(g); return PO_ENOMEM; }
#pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t i = 0; i < n; ++i)
        for (int64_t e = g->row[i]; e < g->row[i + 1]; ++e) g->a[e] = g->mu[i] / g->den[g->fol[e]];
    *out = g;
    return PO_OK;
}

/* stats: n, m, m_in, self-loops, duplicates, users with no leaders, longest row */
void po_stats(const po_graph* g, int64_t* out7) {
    out7[0] = g->n; out7[1] = g->m; out7[2] = g->m_in; out7[3] = g->n_self_loops;
    out7[4] = g->n_duplicates; out7[5] = g->n_no_leaders; out7[6] = g->max_followers;
}

/* c, d, den (any may be NULL) copied out */
void po_vectors(const po_graph* g, double* c, double* d, double* den) {
    if (c) memcpy(c, g->c, (size_t)g->n * sizeof(double));
    if (d) memcpy(d, g->d, (size_t)g->n * sizeof(double));
    if (den) memcpy(den, g->den, (size_t)g->n * sizeof(double));
}

/* CSR of the leader-major rows: row [n+1] (int64) and fol [m] (int32) */
void po_rows(const po_graph* g, int64_t* row, int32_t* fol) {
    if (row) memcpy(row, g->row, ((size_t)g->n + 1) * sizeof(int64_t));
    if (fol) memcpy(fol, g->fol, (size_t)g->m * sizeof(int32_t));
}

/* L1 sum in blocks of 4096 in order (same for any thread count) */
static double l1_fixed(int64_t n, const double* x, const double* y) {
    int64_t nb = (n + 4095) / 4096;
    double* part = (double*)malloc((size_t)(nb > 0 ? nb : 1) * sizeof(double));
#pragma omp parallel for schedule(static)
    for (int64_t b = 0; b < nb; ++b) {
        int64_t e = (b + 1) * 4096 < n ? (b + 1) * 4096 : n;
        double s = 0.0;
        for (int64_t i = b * 4096; i < e; ++i) s += fabs(y ? x[i] - y[i] : x[i]);
        part[b] = s;
    }
    double s = 0.0;
    for (int64_t b = 0; b < nb; ++b) s += part[b];
    free(part);
    return s;
}

/* out_i = (Aᵀ s)_i + c_i */
static void step(const po_graph* g, const double* s, double* out) {
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < g->n; ++i) {
        double y = 0.0;
        for (int64_t e = g->row[i]; e < g->row[i + 1]; ++e) y += g->a[e] * s[g->fol[e]];
        out[i] = y + g->c[i];
    }
}

/* ψ = (Bᵀ s + d)/N, b_ji = λ_i / den_j */
void po_final(const po_graph* g, const double* s, double* psi) {
    const double n = (double)g->n;
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < g->n; ++i) {
        double y = 0.0;
        for (int64_t e = g->row[i]; e < g->row[i + 1]; ++e) {
            int32_t j = g->fol[e];
            y += (g->lam[i] / g->den[j]) * s[j];
        }
        psi[i] = (y + g->d[i]) / n;
    }
}

/* r = Aᵀ s + c − s (per user); returns ‖r‖₁ */
double po_residual(const po_graph* g, const double* s, double* r) {
    double* y = r ? r : (double*)malloc((size_t)g->n * sizeof(double));
    step(g, s, y);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < g->n; ++i) y[i] -= s[i];
    double l1 = l1_fixed(g->n, y, NULL);
    if (!r) free(y);
    return l1;
}

/* ‖B‖ (mode 0) or κ (mode 1): the largest row sum of B or A, row j = follower */
double po_row_sum_max(const po_graph* g, int mode) {
    double* rs = (double*)calloc((size_t)g->n, sizeof(double));
    /* row j of A / B collects μ_i/den_j (λ_i/den_j) over its leaders i; rows
     * are visited by leader here, so the sums go through one thread */
    for (int64_t i = 0; i < g->n; ++i)
        for (int64_t e = g->row[i]; e < g->row[i + 1]; ++e) {
            int32_t j = g->fol[e];
            rs[j] += (mode ? g->mu[i] : g->lam[i]) / g->den[j];
        }
    double mx = 0.0;
    for (int64_t j = 0; j < g->n; ++j) mx = rs[j] > mx ? rs[j] : mx;
    free(rs);
    return mx;
}

typedef void (*po_progress_fn)(int64_t t, double gap);

/* Algorithm 2.  steps >= 0 runs exactly that many steps whatever the gap.
 * s0 (may be NULL = c); s_out, psi_out: [n] (either may be NULL).
 * info[0] = iterations, info[1] = final gap (tol_mode units), info[2] = last
 * ‖s_t − s_{t−1}‖₁, info[3] = wall seconds of the iteration, info[4] = wall
 * seconds of the final ψ pass.  progress (may be NULL) is called after every
 * step with t and the gap, outside any parallel region. */
int po_power_psi(const po_graph* g, double tol, int tol_mode, int64_t max_iter, int64_t steps,
                 const double* s0, double* s_out, double* psi_out, double* info,
                 po_progress_fn progress) {
    if (!(tol > 0)) { set_err("tolerance must be positive"); return PO_EINVAL; }
    if (tol_mode < 0 || tol_mode > 2) { set_err("unknown tol_mode"); return PO_EINVAL; }
    const int64_t n = g->n;
    double* s = (double*)malloc((size_t)n * sizeof(double));
    double* nx = (double*)malloc((size_t)n * sizeof(double));
    if (!s || !nx) { free(s); free(nx); set_err("out of host memory"); return PO_ENOMEM; }
    memcpy(s, s0 ? s0 : g->c, (size_t)n * sizeof(double));
    double bnorm = tol_mode == 1 ? po_row_sum_max(g, 0) : 0.0;
    double gap = 1.0, l1 = 0.0;
    int64_t t = 0;
    int rc = PO_OK;
    double t0 = omp_get_wtime();
    while (steps >= 0 ? t < steps : gap > tol) {
        if (t >= max_iter) { rc = PO_ENOTCONV; set_err("Power-psi did not converge"); break; }
        step(g, s, nx);
        l1 = l1_fixed(n, nx, s);
        gap = l1;
        if (tol_mode == 1) gap *= bnorm;
        if (tol_mode == 2) gap /= l1_fixed(n, nx, NULL);
        double* tmp = s; s = nx; nx = tmp;
        ++t;
        if (progress) progress(t, gap);
        if (!isfinite(gap)) { rc = PO_ENUMERIC; set_err("the step size is not finite"); break; }
    }
    double t1 = omp_get_wtime();
    if (psi_out) po_final(g, s, psi_out);
    double t2 = omp_get_wtime();
    if (s_out) memcpy(s_out, s, (size_t)n * sizeof(double));
    if (info) { info[0] = (double)t; info[1] = gap; info[2] = l1; info[3] = t1 - t0; info[4] = t2 - t1; }
    free(s);
    free(nx);
    return rc;
}
