/*
 * oracle.c -- plain, slow, FP64 CPU oracle for the Giada-Marsili cluster
 * likelihood and the master-slave genetic algorithm built on it.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product path may include, link,
 * load or call this file. Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg use it. It shares no code, header, table or
 * helper with the HIP library.
 *
 * Paper: Hendricks, Gebbie & Wilcox, "High-speed detection of emergent market
 * clustering via an unsupervised parallel genetic algorithm" (arXiv 1403.4099).
 *
 * Every function is the plain definition written out (correlation, n_s, c_s,
 * L_c, brute force) or the GA's steps in the paper's order (Algorithm 1),
 * with the operator choices fixed here (tournament of two, uniform
 * crossover, per-gene random-replacement mutation, elitism), driven by the
 * Philox4x32-10 counter-based generator written from its published
 * definition (Salmon, Moraes, Dror & Shaw, "Parallel random numbers: as easy
 * as 1, 2, 3", SC'11).
 *
 * Conventions (the paper is silent on them; each reading is listed in the
 * design notes):
 *   - labels are 0-based int32 in [0, N) (the paper's Eq. 9 uses 1..K, K = N);
 *   - natural log; literal Eq. 8 also for c_s < n_s;
 *   - an individual with a label outside [0, N), or with a cluster n_s > 1
 *     whose c_s is not inside (0, n_s^2), has fitness -inf;
 *   - status[0] counts individuals with an out-of-range label, status[1] the
 *     clusters outside the domain, status[2] zero-variance stocks,
 *     status[3] individuals whose fitness is -inf.
 *
 * Parity pins (each checked by the CPU test-suite, none by re-typing the
 * formula): closed form -1/2 log det C on exact block matrices (numpy
 * slogdet), N = 2 closed form, L_c = 0 at C = I, invariances, numpy
 * corrcoef for the correlation, published Philox known-answer vectors,
 * brute force over all set partitions, GA statistics and recovery of
 * planted clusters.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ST_LABEL 0
#define ST_DOMAIN 1
#define ST_ZEROVAR 2
#define ST_NONFINITE 3

/* ------------------------------------------------------------------ */
/* Pearson correlation, Eq. 7 (Section 2.2.3), on rows demeaned first  */
/* (the paper normalises the data to zero mean, Eq. 2).                 */
/* ------------------------------------------------------------------ */
/* R is N x T row-major (row stride ld). C is N x N row-major.
 * For each stock i: mu_i = sum_t R_it / T, x_it = R_it - mu_i,
 * s_i = sum_t x_it^2 (t ascending). C_ij = (sum_t x_it x_jt) / sqrt(s_i s_j)
 * for i < j, mirrored; C_ii = 1; clamped to [-1, 1]. A stock with s_i = 0 has
 * its off-diagonal row and column set to 0 and is counted in status[2]. */
int oracle_correlate(const double *R, int N, int T, long ld, double *C, int32_t *status)
{
    if (N < 1 || T < 2) return -1;
    double *X = (double *)malloc((size_t)N * T * sizeof(double));
    double *s = (double *)malloc((size_t)N * sizeof(double));
    if (!X || !s) { free(X); free(s); return -2; }
    for (int i = 0; i < N; ++i) {
        double mu = 0.0;
        for (int t = 0; t < T; ++t) mu += R[(size_t)i * ld + t];
        mu /= (double)T;
        double ss = 0.0;
        for (int t = 0; t < T; ++t) {
            double x = R[(size_t)i * ld + t] - mu;
            X[(size_t)i * T + t] = x;
            ss += x * x;
        }
        s[i] = ss;
        if (ss == 0.0 && status) status[ST_ZEROVAR] += 1;
    }
    for (int i = 0; i < N; ++i) {
        C[(size_t)i * N + i] = 1.0;
        for (int j = i + 1; j < N; ++j) {
            double v;
            if (s[i] == 0.0 || s[j] == 0.0) {
                v = 0.0;
            } else {
                double dot = 0.0;
                for (int t = 0; t < T; ++t) dot += X[(size_t)i * T + t] * X[(size_t)j * T + t];
                v = dot / sqrt(s[i] * s[j]);
                if (v > 1.0) v = 1.0;
                if (v < -1.0) v = -1.0;
            }
            C[(size_t)i * N + j] = v;
            C[(size_t)j * N + i] = v;
        }
    }
    free(X);
    free(s);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Fitness of one labeling: Eqs. 5, 6 and 8 (Section 2.2.3).           */
/* ------------------------------------------------------------------ */
/* n_s = #{i : s_i = s}                                   (Eq. 5)
 * c_s = sum_i sum_j C_ij [s_i = s][s_j = s]              (Eq. 6), pairs in row-major order
 * L_c = 1/2 sum_{s: n_s > 1} [ log(n_s / c_s)
 *                              + (n_s - 1) log((n_s^2 - n_s) / (n_s^2 - c_s)) ]   (Eq. 8)
 * Optional outputs (nullable): n_s[N], c_s[N] per label value, and mag, the
 * sum of the absolute values of the two log terms (times 1/2), used as the
 * scale of the comparison tolerance when L_c is a difference of large terms. */
double oracle_fitness_one(const double *C, int N, const int32_t *lab,
                          int32_t *n_out, double *c_out, double *mag_out, int32_t *status)
{
    int32_t *n = (int32_t *)calloc((size_t)(N > 0 ? N : 1), sizeof(int32_t));
    double *c = (double *)calloc((size_t)(N > 0 ? N : 1), sizeof(double));
    double L = 0.0, mag = 0.0;
    int bad_label = 0, bad_domain = 0;

    for (int i = 0; i < N; ++i)
        if (lab[i] < 0 || lab[i] >= N) bad_label = 1;

    if (bad_label) {
        if (status) { status[ST_LABEL] += 1; status[ST_NONFINITE] += 1; }
        if (n_out) memset(n_out, 0, sizeof(int32_t) * (size_t)N);
        if (c_out) memset(c_out, 0, sizeof(double) * (size_t)N);
        if (mag_out) *mag_out = 0.0;
        free(n); free(c);
        return -INFINITY;
    }
    for (int i = 0; i < N; ++i) n[lab[i]] += 1;
    for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j)
            if (lab[i] == lab[j]) c[lab[i]] += C[(size_t)i * N + j];

    for (int s = 0; s < N; ++s) {
        if (n[s] <= 1) continue;
        double ns = (double)n[s];
        double cs = c[s];
        double n2 = ns * ns;
        if (!(cs > 0.0 && cs < n2)) { bad_domain += 1; continue; }
        double t1 = log(ns / cs);
        double t2 = (ns - 1.0) * log((n2 - ns) / (n2 - cs));
        L += t1 + t2;
        mag += fabs(t1) + fabs(t2);
    }
    if (n_out) memcpy(n_out, n, sizeof(int32_t) * (size_t)N);
    if (c_out) memcpy(c_out, c, sizeof(double) * (size_t)N);
    free(n); free(c);
    if (bad_domain) {
        if (status) { status[ST_DOMAIN] += bad_domain; status[ST_NONFINITE] += 1; }
        if (mag_out) *mag_out = 0.0;
        return -INFINITY;
    }
    if (mag_out) *mag_out = 0.5 * mag;
    return 0.5 * L;
}

/* Fitness of a population pop (P x N row-major). Outputs per individual;
 * n_s and c_s (nullable) are P x N, mag (nullable) is P. */
void oracle_fitness(const double *C, int N, const int32_t *pop, int P, double *fit,
                    int32_t *n_s, double *c_s, double *mag, int32_t *status)
{
    for (int p = 0; p < P; ++p)
        fit[p] = oracle_fitness_one(C, N, pop + (size_t)p * N,
                                    n_s ? n_s + (size_t)p * N : NULL,
                                    c_s ? c_s + (size_t)p * N : NULL,
                                    mag ? mag + p : NULL, status);
}

/* ------------------------------------------------------------------ */
/* Online EWMA correlation (Section 4.2.5, data pre-processing): market */
/* mode removed, then an exponentially weighted covariance with         */
/* forgetting factor lambda, then the correlation of that covariance.   */
/* ------------------------------------------------------------------ */
/* R is N x T (row stride ld), the T newest returns in time order. S (N x N)
 * is the covariance state: when reset != 0 it starts at 0, otherwise the
 * call continues from it. For each t in order: m_t = (1/N) sum_i R_it when
 * market != 0 (the equal-weight market return, removed from every stock),
 * else 0; x_i = R_it - m_t; S_ij <- lambda S_ij + (1 - lambda) x_i x_j.
 * Then C_ij = S_ij / sqrt(S_ii S_jj) clamped to [-1, 1], C_ii = 1, and a
 * stock with S_ii = 0 gets 0 off the diagonal (counted in status[2]). The
 * paper does not give its market-mode estimator or the EWMA's exact form;
 * these are the readings taken here. */
void oracle_ewma(const double *R, int N, int T, long ld, double lambda, int reset, int market,
                 double *S, double *C, int32_t *status)
{
    if (reset)
        for (long e = 0; e < (long)N * N; ++e) S[e] = 0.0;
    double *x = (double *)malloc(sizeof(double) * (size_t)(N > 0 ? N : 1));
    for (int t = 0; t < T; ++t) {
        double m = 0.0;
        if (market) {
            for (int i = 0; i < N; ++i) m += R[(size_t)i * ld + t];
            m /= (double)N;
        }
        for (int i = 0; i < N; ++i) x[i] = R[(size_t)i * ld + t] - m;
        for (int i = 0; i < N; ++i)
            for (int j = 0; j < N; ++j)
                S[(size_t)i * N + j] = lambda * S[(size_t)i * N + j] + (1.0 - lambda) * x[i] * x[j];
    }
    free(x);
    for (int i = 0; i < N; ++i)
        if (S[(size_t)i * N + i] == 0.0 && status) status[ST_ZEROVAR] += 1;
    for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j) {
            double v;
            const double a = S[(size_t)i * N + i], b = S[(size_t)j * N + j];
            if (i == j) v = 1.0;
            else if (a == 0.0 || b == 0.0) v = 0.0;
            else {
                v = S[(size_t)i * N + j] / sqrt(a * b);
                if (v > 1.0) v = 1.0;
                if (v < -1.0) v = -1.0;
            }
            C[(size_t)i * N + j] = v;
        }
}

/* ------------------------------------------------------------------ */
/* BF16 hi + lo split of C (mixed-precision form).                      */
/* ------------------------------------------------------------------ */
/* Round x to the nearest bfloat16 value, ties to even, in one rounding from
 * the FP64 value. bfloat16 keeps 8 significant bits and the float32
 * exponent range; below 2^-126 the spacing is fixed at 2^-133. */
static double round_bf16(double x)
{
    if (x == 0.0 || !isfinite(x)) return x;
    int e;
    (void)frexp(x, &e);              /* x = m 2^e, 0.5 <= |m| < 1 */
    int q = e - 8;                   /* spacing of 8 significant bits */
    if (q < -133) q = -133;
    return ldexp(nearbyint(ldexp(x, -q)), q);   /* nearbyint rounds half to even */
}

static uint16_t bf16_bits(double r)
{
    float f = (float)r;              /* exact: r is a bfloat16 value */
    uint32_t u;
    memcpy(&u, &f, sizeof u);
    return (uint16_t)(u >> 16);
}

/* hi = bf16(C), lo = bf16(C - hi); C - hi is exact in FP64. */
void oracle_split_bf16(const double *C, long count, uint16_t *hi, uint16_t *lo)
{
    for (long k = 0; k < count; ++k) {
        double h = round_bf16(C[k]);
        double l = round_bf16(C[k] - h);
        hi[k] = bf16_bits(h);
        lo[k] = bf16_bits(l);
    }
}

/* ------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon et al., SC'11).                                */
/* ------------------------------------------------------------------ */
/* Each of the 10 rounds multiplies counter words 0 and 2 by the two round
 * multipliers, keeps high and low product halves, xors the high halves with
 * the other two counter words and the round key, and permutes. The key is
 * advanced by the two Weyl constants between rounds. */
void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) { k0 += W0; k1 += W1; }
        uint64_t a = (uint64_t)M0 * (uint64_t)x0;
        uint64_t b = (uint64_t)M1 * (uint64_t)x2;
        uint32_t y0 = (uint32_t)(b >> 32) ^ x1 ^ k0;
        uint32_t y1 = (uint32_t)b;
        uint32_t y2 = (uint32_t)(a >> 32) ^ x3 ^ k1;
        uint32_t y3 = (uint32_t)a;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Counter layout for the GA's random draws. Word 3 carries the draw's purpose
 * (tag, 4 bits) and the GA instance id; word 2 the generation; word 1 the
 * individual (or child slot); word 0 a block index within the individual. */
#define TAG_INIT 0u
#define TAG_SEL 1u
#define TAG_XOV 2u
#define TAG_MUT 3u
#define TAG_SUS 4u
#define TAG_SHUF 5u

static void draw(uint32_t w0, uint32_t w1, uint32_t gen, uint32_t tag, uint32_t inst,
                 uint64_t seed, uint32_t out[4])
{
    uint32_t ctr[4] = { w0, w1, gen, tag | (inst << 4) };
    uint32_t key[2] = { (uint32_t)(seed & 0xFFFFFFFFu), (uint32_t)(seed >> 32) };
    oracle_philox4x32_10(ctr, key, out);
}

/* Map a uniform 32-bit word to [0, m): floor(w m / 2^32). */
static uint32_t scale_u32(uint32_t w, uint32_t m)
{
    return (uint32_t)(((uint64_t)w * (uint64_t)m) >> 32);
}

/* ------------------------------------------------------------------ */
/* GA steps (Section 3.1 operators; Algorithm 1 of Section 4.2.3).      */
/* ------------------------------------------------------------------ */
/* Initial population (Algorithm 1, "create initial population"): gene i of
 * individual p is uniform in [0, N), from word i%4 of draw (i/4, p). */
void oracle_init_pop(int N, int P, uint64_t seed, uint32_t inst, uint32_t gen0, int32_t *pop)
{
    for (int p = 0; p < P; ++p)
        for (int i = 0; i < N; ++i) {
            uint32_t w[4];
            draw((uint32_t)(i / 4), (uint32_t)p, gen0, TAG_INIT, inst, seed, w);
            pop[(size_t)p * N + i] = (int32_t)scale_u32(w[i % 4], (uint32_t)N);
        }
}

/* a ranks before b: higher fitness first, then lower index. -inf is lowest. */
static int ranks_before(const double *f, int a, int b)
{
    if (f[a] > f[b]) return 1;
    if (f[a] < f[b]) return 0;
    return a < b;
}

/* Full ranking (selection sort by the order above; slow and plain). */
void oracle_rank(const double *f, int P, int32_t *order)
{
    char *used = (char *)calloc((size_t)P, 1);
    for (int r = 0; r < P; ++r) {
        int best = -1;
        for (int p = 0; p < P; ++p) {
            if (used[p]) continue;
            if (best < 0 || ranks_before(f, p, best)) best = p;
        }
        used[best] = 1;
        order[r] = best;
    }
    free(used);
}

/* Tournament of two: the better of candidates a and b; a tie goes to the
 * lower index. */
static int tournament2(const double *f, int a, int b)
{
    if (f[a] > f[b]) return a;
    if (f[b] > f[a]) return b;
    return a < b ? a : b;
}

/* ---- Stochastic universal sampling after rank scaling --------------- */
/* Algorithm 1 scales the fitness and then selects; Section 3.1 names the
 * selection: stochastic universal sampling (Baker, 1987), where individuals
 * occupy consecutive segments of a line in proportion to their (scaled)
 * fitness and the line is read at equally spaced points from one random
 * offset. The paper does not say which scaling; the reading here ranks
 * (fitness desc, index asc) and gives rank r (1 = best) the weight
 * floor(2^24 / sqrt(r)) = floor(sqrt(floor(2^48 / r))), computed in exact
 * integer arithmetic, and an individual with fitness -inf weight 0 (if every
 * individual has -inf, all weights are 1). Integer weights keep the segment
 * boundaries exact. */
static uint64_t isqrt_u64(uint64_t x)
{
    /* largest y with y * y <= x, one bit at a time from the top */
    uint64_t y = 0;
    for (int b = 31; b >= 0; --b) {
        uint64_t t = y | ((uint64_t)1 << b);
        if (t * t <= x) y = t;
    }
    return y;
}

static uint64_t sus_weight(int r)
{
    return isqrt_u64(((uint64_t)1 << 48) / (uint64_t)r);
}

/* Pseudo-random permutation of [0, n) (a four-round Feistel network on
 * 2h-bit words, 4^h >= n, with round function word 0 of Philox draw
 * (right half, round) [SHUF], applied again while the value is >= n). */
uint32_t oracle_shuffle_index(uint32_t x, uint32_t n, uint64_t seed, uint32_t inst, uint32_t gen)
{
    int h = 1;
    while (((uint64_t)1 << (2 * h)) < (uint64_t)n) ++h;
    const uint32_t mask = (1u << h) - 1u;
    do {
        uint32_t L = x >> h, R = x & mask;
        for (uint32_t round = 0; round < 4; ++round) {
            uint32_t w[4];
            draw(R, round, gen, TAG_SHUF, inst, seed, w);
            uint32_t t = R;
            R = L ^ (w[0] & mask);
            L = t;
        }
        x = (L << h) | R;
    } while (x >= n);
    return x;
}

/* Parents of the P - E children: parents[2j], parents[2j+1] for child E + j.
 * n = 2(P - E) pointers; with W = total weight and u = floor(w0 W / 2^32)
 * (w0: word 0 of draw (0, 0xFFFFFFFF) [SUS]), pointer k sits at
 * floor((u + k W) / n) and selects the individual whose segment [cum_{p-1},
 * cum_p) holds it (cum: inclusive prefix sums of the weights in index
 * order). The selected list is then shuffled: parents[k] = sel[pi(k)]. */
void oracle_sus_parents(const double *f, int P, int E, uint64_t seed, uint32_t inst, uint32_t gen,
                        int32_t *parents)
{
    const int n = 2 * (P - E);
    if (n <= 0) return;
    int32_t *order = (int32_t *)malloc(sizeof(int32_t) * (size_t)P);
    uint64_t *w = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)P);
    uint64_t *cum = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)P);
    int32_t *sel = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    oracle_rank(f, P, order);
    int any = 0;
    for (int r = 0; r < P; ++r) {
        int p = order[r];
        w[p] = isfinite(f[p]) ? sus_weight(r + 1) : 0;
        any |= w[p] != 0;
    }
    if (!any)
        for (int p = 0; p < P; ++p) w[p] = 1;
    uint64_t acc = 0;
    for (int p = 0; p < P; ++p) { acc += w[p]; cum[p] = acc; }
    const uint64_t W = acc;
    uint32_t wd[4];
    draw(0u, 0xFFFFFFFFu, gen, TAG_SUS, inst, seed, wd);
    const uint64_t u = (uint64_t)(((unsigned __int128)wd[0] * W) >> 32);
    int p = 0;
    for (int k = 0; k < n; ++k) {
        const uint64_t pos = (u + (uint64_t)k * W) / (uint64_t)n;
        while (cum[p] <= pos) ++p;
        sel[k] = p;
    }
    for (int k = 0; k < n; ++k)
        parents[k] = sel[oracle_shuffle_index((uint32_t)k, (uint32_t)n, seed, inst, gen)];
    free(order); free(w); free(cum); free(sel);
}

/* One replacement step from population pop with fitness f (generation gen)
 * into out (Algorithm 1: elitism, selection, crossover, mutation,
 * replacement; Section 3.1).
 *   - out[0..E) are the E fittest individuals, copied unchanged;
 *   - each child c in [E, P), selection 0: parent A is the winner of a
 *     tournament between draws w0, w1 of (0, c) [SEL]; parent B between w2,
 *     w3; indices are scale_u32(w, P). Selection 1: parents 2(c - E) and
 *     2(c - E) + 1 of oracle_sus_parents;
 *   - crossover happens when word 0 of draw (0, c) [XOV] is below
 *     p_cross_thr; then gene j comes from B when bit j%32 of word (j%128)/32
 *     of draw (1 + j/128, c) [XOV] is set, otherwise from A;
 *   - mutation: draw (j/2, c) [MUT] gives words (2(j%2), 2(j%2)+1) = (d, v);
 *     when d < p_mut_thr gene j becomes scale_u32(v, N). */
void oracle_breed_sel(const int32_t *pop, const double *f, int N, int P, int E, int selection,
                      uint32_t p_cross_thr, uint32_t p_mut_thr, uint64_t seed, uint32_t inst,
                      uint32_t gen, int32_t *out)
{
    int32_t *order = (int32_t *)malloc(sizeof(int32_t) * (size_t)P);
    oracle_rank(f, P, order);
    for (int e = 0; e < E; ++e)
        memcpy(out + (size_t)e * N, pop + (size_t)order[e] * N, sizeof(int32_t) * (size_t)N);
    free(order);
    int32_t *par = NULL;
    if (selection == 1) {
        par = (int32_t *)malloc(sizeof(int32_t) * (size_t)(2 * (P - E) + 1));
        oracle_sus_parents(f, P, E, seed, inst, gen, par);
    }

    for (int c = E; c < P; ++c) {
        uint32_t ws[4], wx[4];
        int A, B;
        if (selection == 1) {
            A = par[2 * (c - E)];
            B = par[2 * (c - E) + 1];
        } else {
            draw(0u, (uint32_t)c, gen, TAG_SEL, inst, seed, ws);
            A = tournament2(f, (int)scale_u32(ws[0], (uint32_t)P), (int)scale_u32(ws[1], (uint32_t)P));
            B = tournament2(f, (int)scale_u32(ws[2], (uint32_t)P), (int)scale_u32(ws[3], (uint32_t)P));
        }
        draw(0u, (uint32_t)c, gen, TAG_XOV, inst, seed, wx);
        int cross = wx[0] < p_cross_thr;
        for (int j = 0; j < N; ++j) {
            int32_t gene = pop[(size_t)A * N + j];
            if (cross) {
                uint32_t wb[4];
                draw(1u + (uint32_t)(j / 128), (uint32_t)c, gen, TAG_XOV, inst, seed, wb);
                int r = j % 128;
                if ((wb[r / 32] >> (r % 32)) & 1u) gene = pop[(size_t)B * N + j];
            }
            uint32_t wm[4];
            draw((uint32_t)(j / 2), (uint32_t)c, gen, TAG_MUT, inst, seed, wm);
            uint32_t d = wm[2 * (j % 2)], v = wm[2 * (j % 2) + 1];
            if (d < p_mut_thr) gene = (int32_t)scale_u32(v, (uint32_t)N);
            out[(size_t)c * N + j] = gene;
        }
    }
    free(par);
}

void oracle_breed(const int32_t *pop, const double *f, int N, int P, int E,
                  uint32_t p_cross_thr, uint32_t p_mut_thr, uint64_t seed, uint32_t inst,
                  uint32_t gen, int32_t *out)
{
    oracle_breed_sel(pop, f, N, P, E, 0, p_cross_thr, p_mut_thr, seed, inst, gen, out);
}

/* Per-generation statistics (Algorithm 1, "evaluate state and statistics"):
 * best fitness, mean of the finite fitnesses (-inf when there are none),
 * number of -inf individuals, index of the best (lowest index among ties). */
void oracle_stats(const double *f, int P, double out[4])
{
    int arg = 0;
    double sum = 0.0;
    int nfin = 0, ninv = 0;
    for (int p = 0; p < P; ++p) {
        if (ranks_before(f, p, arg)) arg = p;
        if (isfinite(f[p])) { sum += f[p]; nfin += 1; } else ninv += 1;
    }
    out[0] = P > 0 ? f[arg] : -INFINITY;
    out[1] = nfin > 0 ? sum / (double)nfin : -INFINITY;
    out[2] = (double)ninv;
    out[3] = (double)arg;
}

/* Termination test (Algorithm 1, "determine if termination criteria are
 * met"; Table 3 gives an error tolerance and a number of stall generations).
 * state = {ref, stall, stopped, gens}. The best fitness b of the generation
 * just evaluated improves on the reference ref when ref is not finite and b
 * is, or when b > ref + tol * max(1, |ref|); an improvement sets ref = b and
 * stall = 0, anything else adds one stall generation. With stall_gens > 0 the
 * run stops once stall reaches stall_gens. */
static void term_update(double state[4], double b, int stall_gens, double tol)
{
    double ref = state[0];
    int improved = isfinite(ref) ? (b > ref + tol * fmax(1.0, fabs(ref))) : isfinite(b);
    if (improved) {
        state[0] = b;
        state[1] = 0.0;
    } else {
        state[1] += 1.0;
    }
    if (stall_gens > 0 && state[1] >= (double)stall_gens) state[2] = 1.0;
}

/* The termination test alone, for lockstep checks: one evaluated generation
 * with best fitness b applied to state = {ref, stall, stopped, gens}. */
void oracle_term_test(double state[4], double b, int stall_gens, double tol)
{
    term_update(state, b, stall_gens, tol);
}

/* Up to G generations of Algorithm 1 from generation gen0, then a final
 * fitness. If init != 0 the population is first filled by oracle_init_pop at
 * gen0 and state is reset to {-inf, 0, 0, 0}. Each generation: evaluate,
 * record statistics row g, apply the termination test, and, unless the run
 * has stopped, breed generation g + 1 (state[3] counts the generations bred).
 * Algorithm 1 tests each generation once: a call that continues a state that
 * has already tested a generation (ref finite or stall > 0) starts from the
 * population the previous call tested last, so its first evaluation records
 * statistics but does not enter the test again; splitting a run into several
 * calls therefore gives the same run as one call.
 * A stopped run keeps its last population: nothing further is evaluated,
 * recorded or bred, in this call or a later one with the same state. pop
 * (P x N) is updated in place; fit (P) holds the fitness of the final
 * population; stats (nullable) receives up to G + 1 rows of oracle_stats,
 * rows after a stop are left untouched. stall_gens = 0 disables the test.
 * selection: 0 tournaments of two, 1 stochastic universal sampling. */
int oracle_evolve_term(const double *C, int N, int P, int E, int selection, uint32_t p_cross_thr,
                       uint32_t p_mut_thr, uint64_t seed, uint32_t inst, uint32_t gen0, int G, int init,
                       int stall_gens, double tol, int32_t *pop, double *fit, double *stats,
                       int32_t *status, double state[4])
{
    if (N < 1 || P < 1 || E < 0 || E >= P || G < 0 || stall_gens < 0) return -1;
    if (selection != 0 && selection != 1) return -1;
    int32_t *next = (int32_t *)malloc(sizeof(int32_t) * (size_t)P * (size_t)N);
    if (!next) return -2;
    if (init) {
        oracle_init_pop(N, P, seed, inst, gen0, pop);
        state[0] = -INFINITY;
        state[1] = state[2] = state[3] = 0.0;
    }
    if (state[2] != 0.0) {
        /* already stopped: fit is the fitness of the kept population */
        oracle_fitness(C, N, pop, P, fit, NULL, NULL, NULL, NULL);
        free(next);
        return 0;
    }
    const int tested = isfinite(state[0]) || state[1] != 0.0;
    double row[4];
    for (int g = 0; g <= G; ++g) {
        oracle_fitness(C, N, pop, P, fit, NULL, NULL, NULL, status);
        oracle_stats(fit, P, row);
        if (stats) memcpy(stats + 4 * (size_t)g, row, sizeof(row));
        if (g > 0 || !tested) term_update(state, row[0], stall_gens, tol);
        if (g == G || state[2] != 0.0) break;
        oracle_breed_sel(pop, fit, N, P, E, selection, p_cross_thr, p_mut_thr, seed, inst,
                         gen0 + (uint32_t)g, next);
        memcpy(pop, next, sizeof(int32_t) * (size_t)P * (size_t)N);
        state[3] += 1.0;
    }
    free(next);
    return 0;
}

/* G generations of Algorithm 1 with no termination test, then a final
 * fitness: G + 1 statistics rows. */
int oracle_evolve(const double *C, int N, int P, int E, uint32_t p_cross_thr, uint32_t p_mut_thr,
                  uint64_t seed, uint32_t inst, uint32_t gen0, int G, int init,
                  int32_t *pop, double *fit, double *stats, int32_t *status)
{
    double state[4] = {-INFINITY, 0.0, 0.0, 0.0};
    return oracle_evolve_term(C, N, P, E, 0, p_cross_thr, p_mut_thr, seed, inst, gen0, G, init, 0, 0.0,
                              pop, fit, stats, status, state);
}

/* ------------------------------------------------------------------ */
/* Result reporting (Algorithm 1, "report on results").                 */
/* ------------------------------------------------------------------ */
/* Relabel in first-occurrence order: the first stock's cluster becomes 0,
 * the next new cluster 1, and so on (a restricted-growth string). Labels
 * outside [0, N) are copied unchanged. */
void oracle_canonical(const int32_t *lab, int N, int32_t *out)
{
    int32_t *map = (int32_t *)malloc(sizeof(int32_t) * (size_t)(N > 0 ? N : 1));
    for (int s = 0; s < N; ++s) map[s] = -1;
    int next = 0;
    for (int i = 0; i < N; ++i) {
        int32_t l = lab[i];
        if (l < 0 || l >= N) { out[i] = l; continue; }
        if (map[l] < 0) map[l] = next++;
        out[i] = map[l];
    }
    free(map);
}

/* Fittest individual (lowest index among ties) in canonical form. */
void oracle_best(const double *f, const int32_t *pop, int P, int N,
                 int32_t *out_labels, double *out_f, int32_t *out_idx)
{
    int arg = 0;
    for (int p = 1; p < P; ++p)
        if (ranks_before(f, p, arg)) arg = p;
    oracle_canonical(pop + (size_t)arg * N, N, out_labels);
    *out_f = f[arg];
    *out_idx = arg;
}

/* ------------------------------------------------------------------ */
/* Brute force over every set partition of N stocks (small N only).     */
/* ------------------------------------------------------------------ */
/* Enumerates restricted-growth strings a (a_0 = 0, a_i <= 1 + max a_<i),
 * one per set partition, evaluates Eq. 8 on each, and returns the number of
 * partitions visited. best_f receives the maximum, best_lab the first
 * maximiser in enumeration order, n_best how many partitions are within
 * tie_tol of the maximum. */
long oracle_brute_force(const double *C, int N, double tie_tol, double *best_f, int32_t *best_lab,
                        long *n_best)
{
    if (N < 1 || N > 14) return -1;
    int32_t a[16], mx[16];
    long count = 0, nb = 0;
    double bf = -INFINITY;
    for (int i = 0; i < N; ++i) { a[i] = 0; mx[i] = 0; }
    for (;;) {
        double L = oracle_fitness_one(C, N, a, NULL, NULL, NULL, NULL);
        count += 1;
        if (L > bf + tie_tol) {
            bf = L; nb = 1;
            memcpy(best_lab, a, sizeof(int32_t) * (size_t)N);
        } else if (fabs(L - bf) <= tie_tol) {
            nb += 1;
        }
        /* next restricted-growth string: increment the last position that can grow */
        int i = N - 1;
        while (i > 0 && a[i] == mx[i - 1] + 1) --i;
        if (i == 0) break;
        a[i] += 1;
        mx[i] = a[i] > mx[i - 1] ? a[i] : mx[i - 1];
        for (int k = i + 1; k < N; ++k) { a[k] = 0; mx[k] = mx[i]; }
    }
    *best_f = bf;
    *n_best = nb;
    return count;
}
