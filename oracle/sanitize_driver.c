/*
 * sanitize_driver.c -- TEST INFRASTRUCTURE ONLY: runs every step of the CPU oracle once on small
 * graphs so that a build with AddressSanitizer and UndefinedBehaviorSanitizer (gcc, host code)
 * can check it for out-of-bounds accesses, leaks and undefined behaviour.  Exit status 0 when
 * every call returned its success code.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int ustd_oracle_validate(int64_t n, const int64_t *rp, const int32_t *col);
int32_t ustd_oracle_bfs(int64_t n, const int64_t *rp, const int32_t *col, int32_t u, int32_t *dist, int32_t *parB);
int32_t ustd_oracle_max_degree_pivot(int64_t n, const int64_t *rp);
int64_t ustd_oracle_trees(int64_t n, const int64_t *rp, const int32_t *col, int32_t u, const int32_t *parB,
                          uint64_t seed, int64_t tree_begin, int64_t tree_count, int32_t *parents, int64_t *steps,
                          int64_t *counts);
int ustd_oracle_diag_lpinv(int64_t n, const int64_t *rp, const int32_t *col, int32_t u, double eps, double delta,
                           double kappa, uint64_t seed, int64_t tau_override, double solve_tol, int64_t solve_maxit,
                           double *diag, int64_t *counts_out, int64_t *tau_out, int32_t *ecc_out, int64_t *steps_out,
                           double *relres_out);
int ustd_oracle_diag_lpinv_weighted(int64_t n, const int64_t *rp, const int32_t *col, const double *w, int32_t u,
                                    double eps, double delta, double kappa, uint64_t seed, int64_t tau_override,
                                    double solve_tol, int64_t solve_maxit, double *diag, int64_t *acc_out,
                                    int64_t *tau_out, int32_t *shift_out, double *rho_out, int64_t *steps_out,
                                    double *relres_out);

/* side x side grid with one pendant path of `tail` vertices at the last corner (a cut vertex) */
static void build(int side, int tail, int64_t **rp_out, int32_t **col_out, int64_t *n_out) {
    const int64_t n = (int64_t)side * side + tail;
    int64_t *deg = calloc((size_t)n, sizeof(int64_t));
    int32_t (*e)[2] = malloc(sizeof(int32_t[2]) * (size_t)(4 * n));
    int64_t m = 0;
    for (int i = 0; i < side; ++i)
        for (int j = 0; j < side; ++j) {
            const int v = i * side + j;
            if (j + 1 < side) { e[m][0] = v; e[m][1] = v + 1; ++m; }
            if (i + 1 < side) { e[m][0] = v; e[m][1] = v + side; ++m; }
        }
    for (int k = 0; k < tail; ++k) {
        e[m][0] = (k == 0) ? side * side - 1 : side * side + k - 1;
        e[m][1] = side * side + k;
        ++m;
    }
    for (int64_t k = 0; k < m; ++k) { deg[e[k][0]]++; deg[e[k][1]]++; }
    int64_t *rp = malloc(sizeof(int64_t) * (size_t)(n + 1));
    rp[0] = 0;
    for (int64_t v = 0; v < n; ++v) rp[v + 1] = rp[v] + deg[v];
    int32_t *col = malloc(sizeof(int32_t) * (size_t)rp[n]);
    int64_t *fill = calloc((size_t)n, sizeof(int64_t));
    for (int64_t k = 0; k < m; ++k) {
        const int a = e[k][0], b = e[k][1];
        col[rp[a] + fill[a]++] = b;
        col[rp[b] + fill[b]++] = a;
    }
    for (int64_t v = 0; v < n; ++v)  /* ascending rows (insertion sort; rows are short) */
        for (int64_t x = rp[v] + 1; x < rp[v + 1]; ++x)
            for (int64_t y = x; y > rp[v] && col[y - 1] > col[y]; --y) {
                const int32_t t = col[y]; col[y] = col[y - 1]; col[y - 1] = t;
            }
    free(deg); free(e); free(fill);
    *rp_out = rp; *col_out = col; *n_out = n;
}

int main(void) {
    int bad = 0;
    for (int s = 2; s <= 9; s += 7) {
        int64_t *rp, n;
        int32_t *col;
        build(s, 3, &rp, &col, &n);
        bad |= ustd_oracle_validate(n, rp, col) != 0;
        const int32_t u = ustd_oracle_max_degree_pivot(n, rp);
        int32_t *dist = malloc(sizeof(int32_t) * (size_t)n), *parB = malloc(sizeof(int32_t) * (size_t)n);
        ustd_oracle_bfs(n, rp, col, u, dist, parB);
        int32_t *par = malloc(sizeof(int32_t) * (size_t)(3 * n));
        int64_t steps[3], *cnt = calloc((size_t)n, sizeof(int64_t));
        bad |= ustd_oracle_trees(n, rp, col, u, parB, 7, 5, 3, par, steps, cnt) != 0;
        double *diag = malloc(sizeof(double) * (size_t)n), rr = 0.0, rho = 0.0;
        int64_t tau = 0, st = 0;
        int32_t ecc = 0, k = 0;
        bad |= ustd_oracle_diag_lpinv(n, rp, col, u, 0.3, 0.0, 0.0, 1, 40, 1e-12, 0, diag, cnt, &tau, &ecc, &st, &rr) != 0;
        double *w = malloc(sizeof(double) * (size_t)rp[n]);
        for (int64_t v = 0; v < n; ++v)  /* symmetric conductances: 1 + (min + max) mod 3 */
            for (int64_t x = rp[v]; x < rp[v + 1]; ++x) w[x] = 1.0 + (double)((v + col[x]) % 3);
        bad |= ustd_oracle_diag_lpinv_weighted(n, rp, col, w, u, 0.3, 0.0, 0.0, 2, 30, 1e-12, 0, diag, cnt, &tau, &k,
                                                &rho, &st, &rr) != 0;
        free(dist); free(parB); free(par); free(cnt); free(diag); free(w); free(rp); free(col);
    }
    printf(bad ? "oracle calls failed\n" : "ok\n");
    return bad;
}
