/* Test infrastructure: exercises the CPU oracle (oracle/oracle.c) on small
 * inputs, edge cases included, so that it can be built and run under the host
 * address and undefined-behaviour sanitizers (tests/test_oracle_sanitizers.py).
 * Exit status 0 when every call returns; the sanitizers abort otherwise. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int oracle_correlate(const double *R, int N, int T, long ld, double *C, int32_t *status);
void oracle_fitness(const double *C, int N, const int32_t *pop, int P, double *fit, int32_t *n_s, double *c_s,
                    double *mag, int32_t *status);
void oracle_split_bf16(const double *C, long count, uint16_t *hi, uint16_t *lo);
void oracle_ewma(const double *R, int N, int T, long ld, double lambda, int reset, int market, double *S, double *C,
                 int32_t *status);
int oracle_evolve_term(const double *C, int N, int P, int E, int selection, uint32_t p_cross_thr, uint32_t p_mut_thr,
                       uint64_t seed, uint32_t inst, uint32_t gen0, int G, int init, int stall_gens, double tol,
                       int32_t *pop, double *fit, double *stats, int32_t *status, double state[4]);
void oracle_best(const double *f, const int32_t *pop, int P, int N, int32_t *out_labels, double *out_f,
                 int32_t *out_idx);
long oracle_brute_force(const double *C, int N, double tie_tol, double *best_f, int32_t *best_lab, long *n_best);

static uint64_t lcg = 0x9E3779B97F4A7C15ull;
static double urand(void) {
    lcg = lcg * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(lcg >> 11) * (1.0 / 9007199254740992.0);
}

int main(void) {
    enum { N = 12, T = 40, P = 16, G = 4, E = 2 };
    static double R[N * T], C[N * N], S[N * N], Ce[N * N], fit[P], cs[P * N], mag[P], stats[(G + 1) * 4];
    static int32_t pop[P * N], ns[P * N], st[8], lab[N], idx;
    static uint16_t hi[N * N], lo[N * N];
    for (int i = 0; i < N * T; ++i) R[i] = urand() - 0.5;
    for (int t = 0; t < T; ++t) R[3 * T + t] = 1.0;            /* a zero-variance stock */
    memset(st, 0, sizeof st);
    if (oracle_correlate(R, N, T, T, C, st) != 0) return 1;
    oracle_split_bf16(C, (long)N * N, hi, lo);
    for (int p = 0; p < P; ++p)
        for (int j = 0; j < N; ++j) pop[p * N + j] = (int32_t)((p * 7 + j * 3) % (p % 4 + 1));
    pop[5 * N + 2] = N;                                        /* a label out of range */
    pop[6 * N + 0] = -1;
    for (int j = 0; j < N; ++j) pop[7 * N + j] = j;            /* all singletons */
    oracle_fitness(C, N, pop, P, fit, ns, cs, mag, st);
    oracle_fitness(C, 1, pop, 1, fit, ns, cs, mag, st);        /* N = 1 */
    double state[4] = {-INFINITY, 0.0, 0.0, 0.0};
    for (int sel = 0; sel < 2; ++sel) {
        state[0] = -INFINITY; state[1] = state[2] = state[3] = 0.0;
        oracle_evolve_term(C, N, P, E, sel, 0xE6666666u, 0x15555555u, 7, 3, 0, G, 1, 2, 1e-5, pop, fit, stats, st,
                           state);
    }
    oracle_best(fit, pop, P, N, lab, &fit[0], &idx);
    oracle_ewma(R, N, T, T, 0.98, 1, 1, S, Ce, st);
    oracle_ewma(R, N, T / 2, T, 0.98, 0, 0, S, Ce, st);
    double bf;
    long nb;
    int32_t bl[6];
    if (oracle_brute_force(C, 6, 1e-12, &bf, bl, &nb) != 203) return 2;   /* Bell(6) */
    printf("ok %d\n", idx);
    return 0;
}
