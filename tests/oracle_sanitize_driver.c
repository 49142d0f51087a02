/* Drives every entry point of the CPU oracle (oracle/mmgap_oracle.c) on small
 * deterministic inputs, for a build under the address and undefined-behaviour
 * sanitizers (tests/test_sanitizers_cpu.py).  Prints one checksum line. */
#include "../oracle/mmgap_oracle.c"

#include <stdio.h>

static uint32_t lcg_state = 12345u;
static float urand(void)
{
    lcg_state = lcg_state * 1664525u + 1013904223u;
    return (float)(lcg_state >> 8) / 16777216.0f - 0.5f;
}

int main(void)
{
    double sum = 0.0;
    const int shapes[3][2] = {{8, 1}, {16, 2}, {32, 3}};
    for (int sidx = 0; sidx < 3; ++sidx) {
        const int K = shapes[sidx][0], q = shapes[sidx][1], N = K * q;
        const int n = 7, ipg = 3, n_g = (n + ipg - 1) / ipg, chains = 5, sweeps = 4;
        signed char w[4] = {1, 1, 1, 1};
        for (int b = 0; b < q; ++b) w[b] = (signed char)(1 << (q - 1 - b));
        float *A = malloc(sizeof(float) * (size_t)K * K);
        float *G = malloc(sizeof(float) * (size_t)n_g * K * K);
        float *f = malloc(sizeof(float) * (size_t)n * K);
        signed char *xfb = malloc((size_t)n * K);
        for (int g = 0; g < n_g; ++g) {
            for (int e = 0; e < K * K; ++e) A[e] = urand();
            for (int i = 0; i < K; ++i)
                for (int j = 0; j < K; ++j) {
                    float acc = 0.0f;
                    for (int l = 0; l < K; ++l) acc += A[l * K + i] * A[l * K + j];
                    G[(size_t)g * K * K + i * K + j] = acc;
                }
        }
        for (int e = 0; e < n * K; ++e) {
            f[e] = urand();
            xfb[e] = (signed char)(2 * (int)(4.0f * (urand() + 0.5f)) - 3);
            if (q == 1) xfb[e] = xfb[e] > 0 ? 1 : -1;
        }
        float beta2[4] = {0.1f, 0.5f, 1.0f, 2.0f};
        uint32_t ids[7] = {3, 4, 5, 6, 7, 8, 9};      /* G indices 1..3 with g_base 1 */
        signed char *sp = malloc((size_t)n * N);
        float *e = malloc(sizeof(float) * n), *ce = malloc(sizeof(float) * n * chains);
        double *e64 = malloc(sizeof(double) * n);
        int *win = malloc(sizeof(int) * n);
        if (oracle_solve(n, K, q, w, G, ipg, 1, f, xfb, ids, chains, sweeps, beta2, 99, 1, sp, e,
                         win, ce, 1) != 0) return 2;
        for (int i = 0; i < n; ++i) sum += e[i] + win[i];
        if (oracle_solve(n, K, q, w, G, ipg, 0, f, NULL, NULL, chains, sweeps, beta2, 98, 0, sp, e,
                         win, NULL, 1) != 0) return 3;
        for (int i = 0; i < n; ++i) sum += e[i];
        if (oracle_solve_exact(n, K, q, w, G, ipg, 1, f, xfb, ids, chains, sweeps, beta2, 97, 1,
                               sp, e64, win, 1) != 0) return 4;
        for (int i = 0; i < n; ++i) sum += e64[i];
        if (N <= 32) {
            const float params[7] = {0.02f, 2.0f, 0.9f, 1.0f, 1.0f, 1.0f, 0.1f};
            if (oracle_cim_solve(n, K, q, w, G, ipg, 0, f, xfb, NULL, chains, 8, params, 96, 0, sp,
                                 e, win, ce, 1) != 0) return 5;
            for (int i = 0; i < n; ++i) sum += e[i];
        }
        float *fo = malloc(sizeof(float) * n * K);
        if (oracle_delta_fields(n, K, G, ipg, 0, f, xfb, NULL, fo) != 0) return 6;
        for (int i = 0; i < n * K; ++i) sum += fo[i];
        sum += oracle_level_energy(K, G, f, xfb);
        free(fo); free(A); free(G); free(f); free(xfb); free(sp); free(e); free(ce); free(e64);
        free(win);
    }
    {
        const int n_sc = 3, n_sym = 2, n_u = 4, n_t = 6, K = 2 * n_u;
        float *H = malloc(sizeof(float) * 2 * n_sc * n_u * n_t);
        float *u = malloc(sizeof(float) * 2 * n_sc * n_sym * n_u);
        for (int i = 0; i < 2 * n_sc * n_u * n_t; ++i) H[i] = urand();
        for (int i = 0; i < 2 * n_sc * n_sym * n_u; ++i) u[i] = urand();
        float *Gv = malloc(sizeof(float) * n_sc * K * K), *fv = malloc(sizeof(float) * n_sc * n_sym * K);
        double *Ai = malloc(sizeof(double) * 2 * n_sc * n_u * n_u);
        if (oracle_vpp_build(n_sc, n_sym, n_u, n_t, H, u, 2.5, Gv, fv, Ai, 1) != 0) return 7;
        for (int i = 0; i < n_sc * K * K; ++i) sum += Gv[i];
        free(H); free(u); free(Gv); free(fv); free(Ai);
    }
    uint32_t table[1025];
    oracle_accept_table(table);
    sum += table[100] + oracle_draw16(5, 6, 7, 8, 9) + oracle_accept(1.5f, 1000u);
    printf("checksum %.6e\n", sum);
    return 0;
}
