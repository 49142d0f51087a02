/*
 * mmgap_oracle.c -- plain, slow CPU oracle for the Ising hot path of the
 * MIMO detector / vector-perturbation precoder of "MMGaP: Multi-User MIMO
 * Detection and Precoding using GPU-assisted Physics-inspired Computation".
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header or constant table with the GPU library; both follow the same written
 * arithmetic contract so that their chains can be compared spin for spin.
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -fno-fast-math -fopenmp -shared -fPIC
 * (no fused multiply-add except the explicit fmaf() calls below; float
 * arithmetic in float, RNE).
 *
 * What is computed (paper §3.2 "Processing Flow" and §2.3):
 *   * every MIMO problem becomes an Ising problem; N independent anneals are
 *     run on it from random initial states, each anneal's *final* state is a
 *     candidate, candidates are ranked by the ML objective (Eq. ml), and the
 *     MMSE solution replaces a candidate whose energy is larger;
 *   * the anneal here is a single-spin-flip Metropolis chain on the structured
 *     (level-domain) Ising form E(x) = x^T G x - 2 f^T x with
 *     x_k = sum_b w_b s_{k,b}, s in {-1,+1}.
 *
 * The chain arithmetic, in the order the oracle performs it (float32, RNE;
 * "fma" is a single-rounding fused multiply-add, fmaf):
 *   field of k    g_k = fma(G_k,K-1, x_K-1, ... fma(G_k0, x_0, -f_k))   (l ascending),
 *                 recomputed from the current levels at every visit of k
 *   flip of s_i   i = k*q + b, d = -2 w_b s_i                     (a power of two)
 *                 dE = d * ((g_k + g_k) + d * G_kk);  z = beta2_t * dE
 *                 j = floor(64 z) clamped to [0, 1024] (z <= 0 or NaN -> 0)
 *                 accept iff m < T[j], m the 16-bit Philox draw,
 *                 T[j] = round(2^16 * 2^(-j/64)) for j < 1024, T[1024] = 0
 *   on accept     s_i = -s_i;  x_k = x_k + d;  g_k = fma(G_kk, d, g_k)
 *   energy        E = fma(x_K-1, g_K-1 - f_K-1, ... fma(x_0, g_0 - f_0, 0))
 *                 with fresh fields g;  E = x^T G x - 2 f^T x
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Philox4x32-10: J. K. Salmon, M. A. Moraes, R. O. Dror, D. E. Shaw,
 * "Parallel random numbers: as easy as 1, 2, 3", SC'11.  Each round takes the
 * 32x32->64-bit products of the two multipliers with counter words 0 and 2,
 * and forms the new counter (hi1^c1^k0, lo1, hi0^c3^k1, lo0); the key is
 * advanced by the two Weyl constants between rounds.                        */
static const uint32_t PHILOX_MUL_A = 0xD2511F53u;
static const uint32_t PHILOX_MUL_B = 0xCD9E8D57u;
static const uint32_t PHILOX_WEYL_A = 0x9E3779B9u;
static const uint32_t PHILOX_WEYL_B = 0xBB67AE85u;

void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += PHILOX_WEYL_A;
            k1 += PHILOX_WEYL_B;
        }
        uint64_t pa = (uint64_t)PHILOX_MUL_A * (uint64_t)c0;
        uint64_t pb = (uint64_t)PHILOX_MUL_B * (uint64_t)c2;
        uint32_t n0 = (uint32_t)(pb >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)pb;
        uint32_t n2 = (uint32_t)(pa >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)pa;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* The 16-bit draw used for spin i at sweep t of chain ch of instance inst:
 * counter (i/8, t, ch, inst), key (seed_lo, seed_hi); word (i%8)/2, low half
 * for even i, high half for odd i.  Initial spins use t = 0xFFFFFFFF.       */
static uint32_t draw16(uint32_t i, uint32_t t, uint32_t ch, uint32_t inst, const uint32_t key[2])
{
    uint32_t ctr[4] = {i / 8u, t, ch, inst};
    uint32_t out[4];
    oracle_philox4x32_10(ctr, key, out);
    uint32_t word = out[(i % 8u) / 2u];
    return (i % 2u == 0u) ? (word & 0xFFFFu) : (word >> 16);
}

uint32_t oracle_draw16(uint32_t i, uint32_t t, uint32_t ch, uint32_t inst, uint64_t seed)
{
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    return draw16(i, t, ch, inst, key);
}

/* ------------------------------------------------------------------------ */
/* Metropolis acceptance with a 16-bit uniform: the move is accepted with
 * probability 2^-z, z = beta * dE * log2(e) (beta2 = beta log2 e).  z is
 * quantised down to a multiple of 1/64 and the threshold is tabulated:
 * T[j] = round(2^16 * 2^(-j/64)) (no entry lies within 1e-3 of a rounding tie,
 * so any double-precision exp2 gives the same integers); T[1024] = 0 rejects
 * every move with z >= 16.  Accept iff m < T[j]: probability T[j] / 2^16.    */
#define ACCEPT_STEPS 1024
static uint32_t accept_table[ACCEPT_STEPS + 1];
static int accept_ready = 0;

static void accept_init(void)
{
    if (accept_ready) return;
    for (int j = 0; j < ACCEPT_STEPS; ++j)
        accept_table[j] = (uint32_t)llround(65536.0 * exp2(-(double)j / 64.0));
    accept_table[ACCEPT_STEPS] = 0u;
    accept_ready = 1;
}

static uint32_t accept_index(float z)
{
    const float zs = z * 64.0f;                 /* exact */
    if (!(zs > 0.0f)) return 0u;                /* downhill, flat or NaN */
    if (zs >= (float)ACCEPT_STEPS) return ACCEPT_STEPS;
    return (uint32_t)zs;                        /* floor of a positive value */
}

static int metropolis_accept(float z, uint32_t m)
{
    return m < accept_table[accept_index(z)];
}

int oracle_accept(float z, uint32_t m)
{
    accept_init();
    return metropolis_accept(z, m);
}

void oracle_accept_table(uint32_t *out)
{
    accept_init();
    for (int j = 0; j <= ACCEPT_STEPS; ++j) out[j] = accept_table[j];
}

/* ------------------------------------------------------------------------ */
/* Level-domain helpers.                                                     */

/* local field of dimension k: g_k = (G x)_k - f_k as a chain of fused
 * multiply-adds over l ascending, starting from -f_k                      */
static float field_row(int K, const float *G, const float *f, const float *x, int k)
{
    float acc = -f[k];
    for (int l = 0; l < K; ++l) acc = fmaf(G[k * K + l], x[l], acc);
    return acc;
}

/* E = x^T G x - 2 f^T x written as sum_k x_k (g_k - f_k) with g = G x - f,
 * accumulated by fused multiply-adds over k ascending                     */
static float level_energy(int K, const float *G, const float *f, const float *x)
{
    float acc = 0.0f;
    for (int k = 0; k < K; ++k) {
        const float diff = field_row(K, G, f, x, k) - f[k];
        acc = fmaf(x[k], diff, acc);
    }
    return acc;
}

static void levels_from_spins(int K, int q, const signed char *w, const signed char *s, float *x)
{
    for (int k = 0; k < K; ++k) {
        int lv = 0;
        for (int b = 0; b < q; ++b) lv += (int)w[b] * (int)s[k * q + b];
        x[k] = (float)lv;
    }
}

/* Spins representing level lv: MSB first, s_b = +1 if the remainder is
 * positive, else -1.  Exact for binary weights and for unit weights.       */
static void spins_from_level(int q, const signed char *w, int lv, signed char *s)
{
    int rem = lv;
    for (int b = 0; b < q; ++b) {
        s[b] = (rem > 0) ? 1 : -1;
        rem -= (int)w[b] * (int)s[b];
    }
}

/* Total order on candidate energies: numeric, all NaNs after everything.  */
static int energy_less(float a, float b)
{
    int an = isnan(a), bn = isnan(b);
    if (an) return 0;
    if (bn) return 1;
    return a < b;
}

/* One anneal: returns the final energy, writes the final spins (N = K*q).
 * Sweeps visit the dimensions k = 0..K-1 in order and, within k, its spins
 * b = 0..q-1 (spin index i = k q + b, most significant weight first).     */
static float run_chain(int K, int q, const signed char *w, const float *G, const float *f,
                       const signed char *xfb, int sweeps, const float *beta2,
                       const uint32_t key[2], uint32_t inst, uint32_t ch, int init_mode,
                       signed char *s, float *x)
{
    const int N = K * q;
    if (init_mode == 1 && xfb != NULL) {
        for (int k = 0; k < K; ++k) spins_from_level(q, w, (int)xfb[k], s + k * q);
    } else {
        for (int i = 0; i < N; ++i) {
            uint32_t d = draw16((uint32_t)i, 0xFFFFFFFFu, ch, inst, key);
            s[i] = (d & 0x8000u) ? -1 : 1;
        }
    }
    levels_from_spins(K, q, w, s, x);

    for (int t = 0; t < sweeps; ++t) {
        const float b2 = beta2[t];
        for (int k = 0; k < K; ++k) {
            const float gkk = G[k * K + k];
            float g = field_row(K, G, f, x, k);
            for (int b = 0; b < q; ++b) {
                const int i = k * q + b;
                const float delta = (float)(-2 * (int)w[b] * (int)s[i]);
                const float twice = g + g;
                const float curv = delta * gkk;
                const float inner = twice + curv;
                const float dE = delta * inner;
                const float z = b2 * dE;
                const uint32_t m = draw16((uint32_t)i, (uint32_t)t, ch, inst, key);
                if (metropolis_accept(z, m)) {
                    s[i] = (signed char)(-s[i]);
                    x[k] = x[k] + delta;
                    g = fmaf(gkk, delta, g);
                }
            }
        }
    }
    levels_from_spins(K, q, w, s, x);
    return level_energy(K, G, f, x);
}

/*
 * oracle_solve: best-of-C annealed candidates per instance, with fallback.
 *   G            [n_G][K][K] float, symmetric; instance n uses G[inst_of(n)/inst_per_G]
 *   f            [n][K] float
 *   x_fb         [n][K] int8 levels or NULL (no fallback)
 *   inst_ids     [n] uint32 Philox instance index of each instance, or NULL (0..n-1).
 *                G is indexed by inst_ids[n] / inst_per_G minus g_base.
 *   beta2        [sweeps] float
 *   spins_out    [n][K*q] int8 (+1/-1); e_out [n]; win_out [n] (chain index, C = fallback)
 *   chain_e_out  [n][C] float or NULL (energy of every chain's final state)
 */
int oracle_solve(int n, int K, int q, const signed char *w, const float *G, int inst_per_G,
                 long g_base, const float *f, const signed char *x_fb, const uint32_t *inst_ids,
                 int chains, int sweeps, const float *beta2, uint64_t seed, int init_mode,
                 signed char *spins_out, float *e_out, int *win_out, float *chain_e_out,
                 int nthreads)
{
    if (n < 0 || K <= 0 || q <= 0 || chains <= 0 || sweeps < 0 || inst_per_G <= 0) return -1;
    accept_init();
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    const int N = K * q;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    int bad = 0;
#pragma omp parallel
    {
        signed char *s = (signed char *)malloc((size_t)N);
        signed char *sbest = (signed char *)malloc((size_t)N);
        float *x = (float *)malloc(sizeof(float) * (size_t)K);
        if (!s || !sbest || !x) {
#pragma omp atomic write
            bad = 1;
        } else {
#pragma omp for schedule(dynamic, 4)
            for (int idx = 0; idx < n; ++idx) {
                const uint32_t inst = inst_ids ? inst_ids[idx] : (uint32_t)idx;
                const long gi = (long)(inst / (uint32_t)inst_per_G) - g_base;
                const float *Gi = G + (size_t)gi * (size_t)K * (size_t)K;
                const float *fi = f + (size_t)idx * (size_t)K;
                const signed char *xi = x_fb ? x_fb + (size_t)idx * (size_t)K : NULL;
                float ebest = 0.0f;
                int win = -1;
                for (int ch = 0; ch < chains; ++ch) {
                    float e = run_chain(K, q, w, Gi, fi, xi, sweeps, beta2, key, inst,
                                        (uint32_t)ch, init_mode, s, x);
                    if (chain_e_out) chain_e_out[(size_t)idx * (size_t)chains + (size_t)ch] = e;
                    if (win < 0 || energy_less(e, ebest)) {
                        ebest = e;
                        win = ch;
                        memcpy(sbest, s, (size_t)N);
                    }
                }
                if (xi) {
                    for (int k = 0; k < K; ++k) x[k] = (float)xi[k];
                    float efb = level_energy(K, Gi, fi, x);
                    if (energy_less(efb, ebest)) {
                        ebest = efb;
                        win = chains;
                        for (int k = 0; k < K; ++k) spins_from_level(q, w, (int)xi[k], sbest + k * q);
                    }
                }
                memcpy(spins_out + (size_t)idx * (size_t)N, sbest, (size_t)N);
                e_out[idx] = ebest;
                if (win_out) win_out[idx] = win;
            }
        }
        free(s); free(sbest); free(x);
    }
    return bad ? -2 : 0;
}

/* ------------------------------------------------------------------------ */
/* Plain Metropolis reference (a quality reference, NOT a parity target).
 *
 * The same anneal as run_chain -- same sweep order, same initial spins, the
 * same 16-bit draw m for every attempt -- but taken from the definitions, in
 * float64, with none of the choices the chain contract above makes for speed:
 *   g_k  = sum_l G_kl x_l - f_k, summed afresh at every attempt
 *   dE   = E(x with s_i flipped) - E(x) = d (2 g_k + d G_kk),  d = -2 w_b s_i
 *   accept iff dE <= 0 or u < 2^(-beta2_t dE) = exp(-beta_t dE),
 *        u = (m + 1/2) / 2^16 (the draw's uniform, no table, z not quantised)
 * and the candidates ranked by the float64 energy x^T G x - 2 f^T x (lowest
 * chain index on ties; the fallback only if strictly lower).  Comparing its
 * results with oracle_solve's over many instances measures what the tabulated
 * acceptance (z floored to 1/64, probability up to 1.1% above 2^-z) and the
 * float32 chain arithmetic change in the solution quality.                  */
static double field_exact(int K, const float *G, const float *f, const double *x, int k)
{
    double acc = 0.0;
    for (int l = 0; l < K; ++l) acc += (double)G[k * K + l] * x[l];
    return acc - (double)f[k];
}

static double energy_exact(int K, const float *G, const float *f, const double *x)
{
    double e = 0.0;
    for (int k = 0; k < K; ++k) {
        double gx = 0.0;
        for (int l = 0; l < K; ++l) gx += (double)G[k * K + l] * x[l];
        e += x[k] * gx - 2.0 * (double)f[k] * x[k];
    }
    return e;
}

static double run_chain_exact(int K, int q, const signed char *w, const float *G, const float *f,
                              const signed char *xfb, int sweeps, const float *beta2,
                              const uint32_t key[2], uint32_t inst, uint32_t ch, int init_mode,
                              signed char *s, double *x)
{
    const int N = K * q;
    if (init_mode == 1 && xfb != NULL) {
        for (int k = 0; k < K; ++k) spins_from_level(q, w, (int)xfb[k], s + k * q);
    } else {
        for (int i = 0; i < N; ++i) {
            uint32_t d = draw16((uint32_t)i, 0xFFFFFFFFu, ch, inst, key);
            s[i] = (d & 0x8000u) ? -1 : 1;
        }
    }
    for (int k = 0; k < K; ++k) {
        int lv = 0;
        for (int b = 0; b < q; ++b) lv += (int)w[b] * (int)s[k * q + b];
        x[k] = (double)lv;
    }
    for (int t = 0; t < sweeps; ++t) {
        const double b2 = (double)beta2[t];
        for (int k = 0; k < K; ++k) {
            const double gkk = (double)G[k * K + k];
            for (int b = 0; b < q; ++b) {
                const int i = k * q + b;
                const double d = (double)(-2 * (int)w[b] * (int)s[i]);
                const double g = field_exact(K, G, f, x, k);
                const double dE = d * (2.0 * g + d * gkk);
                const uint32_t m = draw16((uint32_t)i, (uint32_t)t, ch, inst, key);
                const double u = ((double)m + 0.5) / 65536.0;
                if (dE <= 0.0 || u < exp2(-b2 * dE)) {
                    s[i] = (signed char)(-s[i]);
                    x[k] += d;
                }
            }
        }
    }
    return energy_exact(K, G, f, x);
}

/* oracle_solve_exact: as oracle_solve (same arguments and layouts) with the
 * plain reference chain above; e_out holds float64 energies.               */
int oracle_solve_exact(int n, int K, int q, const signed char *w, const float *G, int inst_per_G,
                       long g_base, const float *f, const signed char *x_fb,
                       const uint32_t *inst_ids, int chains, int sweeps, const float *beta2,
                       uint64_t seed, int init_mode, signed char *spins_out, double *e_out,
                       int *win_out, int nthreads)
{
    if (n < 0 || K <= 0 || q <= 0 || chains <= 0 || sweeps < 0 || inst_per_G <= 0) return -1;
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    const int N = K * q;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    int bad = 0;
#pragma omp parallel
    {
        signed char *s = (signed char *)malloc((size_t)N);
        signed char *sbest = (signed char *)malloc((size_t)N);
        double *x = (double *)malloc(sizeof(double) * (size_t)K);
        if (!s || !sbest || !x) {
#pragma omp atomic write
            bad = 1;
        } else {
#pragma omp for schedule(dynamic, 4)
            for (int idx = 0; idx < n; ++idx) {
                const uint32_t inst = inst_ids ? inst_ids[idx] : (uint32_t)idx;
                const long gi = (long)(inst / (uint32_t)inst_per_G) - g_base;
                const float *Gi = G + (size_t)gi * (size_t)K * (size_t)K;
                const float *fi = f + (size_t)idx * (size_t)K;
                const signed char *xi = x_fb ? x_fb + (size_t)idx * (size_t)K : NULL;
                double ebest = 0.0;
                int win = -1;
                for (int ch = 0; ch < chains; ++ch) {
                    const double e = run_chain_exact(K, q, w, Gi, fi, xi, sweeps, beta2, key,
                                                     inst, (uint32_t)ch, init_mode, s, x);
                    if (win < 0 || e < ebest) {
                        ebest = e;
                        win = ch;
                        memcpy(sbest, s, (size_t)N);
                    }
                }
                if (xi) {
                    for (int k = 0; k < K; ++k) x[k] = (double)xi[k];
                    const double efb = energy_exact(K, Gi, fi, x);
                    if (efb < ebest) {
                        ebest = efb;
                        win = chains;
                        for (int k = 0; k < K; ++k) spins_from_level(q, w, (int)xi[k], sbest + k * q);
                    }
                }
                memcpy(spins_out + (size_t)idx * (size_t)N, sbest, (size_t)N);
                e_out[idx] = ebest;
                if (win_out) win_out[idx] = win;
            }
        }
        free(s); free(sbest); free(x);
    }
    return bad ? -2 : 0;
}

/* ------------------------------------------------------------------------ */
/* CIM-CAC anneals (paper §2.3, Eqs. cim1 and cim2; §3.2 "Matrix-Vector
 * Multiplication Optimization" and Appendix A for the integration).
 *
 * Each spin i = k q + b of the structured problem, and one auxiliary spin a
 * that carries the field, gets a real amplitude x_i and an error variable
 * e_i > 0.  With the spin couplings J_ij = -2 w_i w_j G_{k(i)k(j)} (i != j) and
 * fields h_i = 2 w_i f_{k(i)} of the level-domain energy, the model is
 *   dx_i/dt = (p - 1) x_i - x_i^3 + eps e_i c_i,
 *   de_i/dt = -zeta (x_i^2 - a) e_i,
 *   c_i = sum_{j != i} J_ij x_j + h_i x_a,   c_a = sum_i h_i x_i,
 * integrated by explicit Euler steps of length dt; the coupling terms c are
 * recomputed every f_mvm steps and held in between.  Through the structure,
 * the coupling of spin i = (k, b) is
 *   c_i = (-2 w_b) (g_k - G_kk (w_b x_i)) + (2 w_b f_k) x_a,
 *   g_k = sum_l G_kl X_l,   X_l = sum_b w_b x_{l,b},
 *   c_a = sum_k (2 f_k) X_k,
 * one K x K product instead of an N x N one.  The final spins are
 * s_i = sign(x_i) sign(x_a) (the auxiliary spin fixes the global sign).
 *
 * Arithmetic (float32, RNE, fmaf = one rounding):
 *   X_l  = fma(w_{q-1}, x_{l,q-1}, ... fma(w_0, x_{l,0}, 0))        b ascending
 *   g_k  = fma(G_k,K-1, X_K-1, ... fma(G_k0, X_0, 0))                l ascending
 *   c_i  = ((-2 w_b) * (g_k - G_kk * (w_b * x_i))) + ((2 w_b f_k) * x_a)
 *   c_a  = fma(2 f_K-1, X_K-1, ... fma(2 f_0, X_0, 0))               k ascending
 *   step, for every amplitude from the values before the step:
 *     s2 = x * x;  dx = ((p - 1) * x - s2 * x) + (eps * e) * c;  x' = x + dt * dx
 *     de = (-zeta) * ((s2 - a) * e);  e' = max(e + dt * de, 2^-20)
 *   init: e = 1; random start: x_i = amp0 * ((d_i - 32768) / 32768) with d_i
 *     the 16-bit Philox draw (i, 0xFFFFFFFF, chain, instance) of spin i and
 *     d_a the draw (0xFFFFFFF8, 0xFFFFFFFF, chain, instance); fallback start:
 *     x_i = amp0 s_i of the fallback levels' spins, x_a = amp0.
 * The coupling terms are taken at steps t = 0, f_mvm, 2 f_mvm, ...       */
typedef struct {
    float dt;
    int f_mvm;
    float p, a, zeta, eps, amp0;
} cim_params;

static float cim_chain(int K, int q, const signed char *w, const float *G, const float *f,
                       const signed char *xfb, int steps, const cim_params *P,
                       const uint32_t key[2], uint32_t inst, uint32_t ch, int init_mode,
                       signed char *s, float *xl, float *amp, float *err, float *cpl)
{
    const int N = K * q;
    const float inv = 1.0f / 32768.0f;           /* exact */
    if (init_mode == 1 && xfb != NULL) {
        for (int k = 0; k < K; ++k) spins_from_level(q, w, (int)xfb[k], s + k * q);
        for (int i = 0; i < N; ++i) amp[i] = P->amp0 * (float)s[i];
        amp[N] = P->amp0;
    } else {
        for (int i = 0; i < N; ++i) {
            const uint32_t d = draw16((uint32_t)i, 0xFFFFFFFFu, ch, inst, key);
            amp[i] = P->amp0 * ((float)((int)d - 32768) * inv);
        }
        const uint32_t d = draw16(0xFFFFFFF8u, 0xFFFFFFFFu, ch, inst, key);
        amp[N] = P->amp0 * ((float)((int)d - 32768) * inv);
    }
    for (int i = 0; i <= N; ++i) err[i] = 1.0f;
    const float pm1 = P->p - 1.0f;
    const float nzeta = -P->zeta;
    const float efloor = 1.0f / 1048576.0f;      /* 2^-20 */
    for (int t = 0; t < steps; ++t) {
        if (t % P->f_mvm == 0) {
            for (int l = 0; l < K; ++l) {
                float X = 0.0f;
                for (int b = 0; b < q; ++b) X = fmaf((float)w[b], amp[l * q + b], X);
                xl[l] = X;
            }
            const float xa = amp[N];
            float ca = 0.0f;
            for (int k = 0; k < K; ++k) {
                float g = 0.0f;
                for (int l = 0; l < K; ++l) g = fmaf(G[k * K + l], xl[l], g);
                const float gkk = G[k * K + k];
                for (int b = 0; b < q; ++b) {
                    const int i = k * q + b;
                    const float wb = (float)w[b];
                    const float self = gkk * (wb * amp[i]);
                    const float inner = g - self;
                    const float t1 = (-2.0f * wb) * inner;
                    const float t2 = ((2.0f * wb) * f[k]) * xa;
                    cpl[i] = t1 + t2;
                }
                ca = fmaf(2.0f * f[k], xl[k], ca);
            }
            cpl[N] = ca;
        }
        for (int i = 0; i <= N; ++i) {
            const float x = amp[i], e = err[i];
            const float s2 = x * x;
            const float lin = pm1 * x;
            const float cub = s2 * x;
            const float drift = lin - cub;
            const float gain = P->eps * e;
            const float push = gain * cpl[i];
            const float dx = drift + push;
            const float step = P->dt * dx;
            const float t1 = s2 - P->a;
            const float t2 = t1 * e;
            const float de = nzeta * t2;
            const float estep = P->dt * de;
            const float en = e + estep;
            amp[i] = x + step;
            err[i] = en > efloor ? en : efloor;
        }
    }
    const int sa_neg = amp[N] < 0.0f;
    for (int i = 0; i < N; ++i) {
        const int neg = amp[i] < 0.0f;
        s[i] = (signed char)((neg != sa_neg) ? -1 : 1);
    }
    levels_from_spins(K, q, w, s, xl);
    return level_energy(K, G, f, xl);
}

/*
 * oracle_cim_solve: as oracle_solve, with CIM-CAC anneals of `steps` Euler
 * steps in place of the Metropolis chains (same selection and fallback).
 *   params [7] float: dt, f_mvm (integral, >= 1), p, a, zeta, eps, amp0
 */
int oracle_cim_solve(int n, int K, int q, const signed char *w, const float *G, int inst_per_G,
                     long g_base, const float *f, const signed char *x_fb,
                     const uint32_t *inst_ids, int chains, int steps, const float *params,
                     uint64_t seed, int init_mode, signed char *spins_out, float *e_out,
                     int *win_out, float *chain_e_out, int nthreads)
{
    if (n < 0 || K <= 0 || q <= 0 || chains <= 0 || steps < 0 || inst_per_G <= 0 || !params)
        return -1;
    cim_params P;
    P.dt = params[0];
    P.f_mvm = (int)params[1];
    P.p = params[2];
    P.a = params[3];
    P.zeta = params[4];
    P.eps = params[5];
    P.amp0 = params[6];
    if (P.f_mvm < 1) return -1;
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    const int N = K * q;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    int bad = 0;
#pragma omp parallel
    {
        signed char *s = (signed char *)malloc((size_t)N);
        signed char *sbest = (signed char *)malloc((size_t)N);
        float *xl = (float *)malloc(sizeof(float) * (size_t)K);
        float *amp = (float *)malloc(sizeof(float) * (size_t)(N + 1));
        float *err = (float *)malloc(sizeof(float) * (size_t)(N + 1));
        float *cpl = (float *)malloc(sizeof(float) * (size_t)(N + 1));
        if (!s || !sbest || !xl || !amp || !err || !cpl) {
#pragma omp atomic write
            bad = 1;
        } else {
#pragma omp for schedule(dynamic, 4)
            for (int idx = 0; idx < n; ++idx) {
                const uint32_t inst = inst_ids ? inst_ids[idx] : (uint32_t)idx;
                const long gi = (long)(inst / (uint32_t)inst_per_G) - g_base;
                const float *Gi = G + (size_t)gi * (size_t)K * (size_t)K;
                const float *fi = f + (size_t)idx * (size_t)K;
                const signed char *xi = x_fb ? x_fb + (size_t)idx * (size_t)K : NULL;
                float ebest = 0.0f;
                int win = -1;
                for (int ch = 0; ch < chains; ++ch) {
                    float e = cim_chain(K, q, w, Gi, fi, xi, steps, &P, key, inst, (uint32_t)ch,
                                        init_mode, s, xl, amp, err, cpl);
                    if (chain_e_out) chain_e_out[(size_t)idx * (size_t)chains + (size_t)ch] = e;
                    if (win < 0 || energy_less(e, ebest)) {
                        ebest = e;
                        win = ch;
                        memcpy(sbest, s, (size_t)N);
                    }
                }
                if (xi) {
                    for (int k = 0; k < K; ++k) xl[k] = (float)xi[k];
                    float efb = level_energy(K, Gi, fi, xl);
                    if (energy_less(efb, ebest)) {
                        ebest = efb;
                        win = chains;
                        for (int k = 0; k < K; ++k) spins_from_level(q, w, (int)xi[k], sbest + k * q);
                    }
                }
                memcpy(spins_out + (size_t)idx * (size_t)N, sbest, (size_t)N);
                e_out[idx] = ebest;
                if (win_out) win_out[idx] = win;
            }
        }
        free(s); free(sbest); free(xl); free(amp); free(err); free(cpl);
    }
    return bad ? -2 : 0;
}

/*
 * oracle_delta_fields: fields of the Ising problem around a guess (paper §2.3,
 * the Delta-Ising form the paper builds around its MMSE / MMSE-SIC guess; Fig. 5
 * and §3.2 "MMGaP-E").  With levels x = x_g + z the energy
 * x^T G x - 2 f^T x equals z^T G z - 2 (f - G x_g)^T z plus a constant, so the
 * search over the moves z uses the couplings G unchanged and the fields
 *   f'_k = f_k - fma(G_k,K-1, xg_K-1, ... fma(G_k0, xg_0, 0))        (l ascending).
 *   G [n_G][K][K]; f, xg, f_out [n][K]; instance idx uses G[inst / inst_per_G - g_base]
 *   with inst = inst_ids[idx] (or idx).
 */
int oracle_delta_fields(int n, int K, const float *G, int inst_per_G, long g_base, const float *f,
                        const signed char *xg, const uint32_t *inst_ids, float *f_out)
{
    if (n < 0 || K <= 0 || inst_per_G <= 0) return -1;
    for (int idx = 0; idx < n; ++idx) {
        const uint32_t inst = inst_ids ? inst_ids[idx] : (uint32_t)idx;
        const long gi = (long)(inst / (uint32_t)inst_per_G) - g_base;
        const float *Gi = G + (size_t)gi * (size_t)K * (size_t)K;
        for (int k = 0; k < K; ++k) {
            float g = 0.0f;
            for (int l = 0; l < K; ++l) g = fmaf(Gi[k * K + l], (float)xg[(size_t)idx * K + l], g);
            f_out[(size_t)idx * K + k] = f[(size_t)idx * K + k] - g;
        }
    }
    return 0;
}

/* One CIM-CAC anneal's amplitudes and error variables after `steps` steps
 * (the N spins, then the auxiliary one), for the invariant tests.          */
int oracle_cim_trajectory(int K, int q, const signed char *w, const float *G, const float *f,
                          const signed char *xfb, int steps, const float *params, uint64_t seed,
                          uint32_t inst, uint32_t ch, int init_mode, float *amp_out, float *err_out,
                          signed char *spins_out, float *e_out)
{
    if (K <= 0 || q <= 0 || steps < 0 || !params || (int)params[1] < 1) return -1;
    cim_params P = {params[0], (int)params[1], params[2], params[3], params[4], params[5],
                    params[6]};
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    const int N = K * q;
    signed char *s = (signed char *)malloc((size_t)N);
    float *xl = (float *)malloc(sizeof(float) * (size_t)K);
    float *cpl = (float *)malloc(sizeof(float) * (size_t)(N + 1));
    if (!s || !xl || !cpl) { free(s); free(xl); free(cpl); return -2; }
    const float e = cim_chain(K, q, w, G, f, xfb, steps, &P, key, inst, ch, init_mode, s, xl,
                              amp_out, err_out, cpl);
    if (spins_out) memcpy(spins_out, s, (size_t)N);
    if (e_out) *e_out = e;
    free(s); free(xl); free(cpl);
    return 0;
}

/* Energy of given levels with the chains' float32 arithmetic.             */
float oracle_level_energy(int K, const float *G, const float *f, const signed char *lv)
{
    float x[256];
    if (K <= 0 || K > 256) return NAN;
    for (int k = 0; k < K; ++k) x[k] = (float)lv[k];
    return level_energy(K, G, f, x);
}

/* ------------------------------------------------------------------------ */
/* Vector-perturbation couplings (paper §3.3, Eqs. VPP and its rewriting with
 * y~ = W u, H_p = -tau W / 2).  With W = H^H (H H^H)^-1 the Gram of H_p is
 * (tau/2)^2 (H H^H)^-1 and its matched filter is -(tau/2) (H H^H)^-1 u, so
 * the couplings need A^-1 for A = H H^H only.  A^-1 is formed in double by a
 * fixed sequence of IEEE operations (so that two implementations following
 * the same sequence agree bit for bit):
 *   A_il  = sum_j H_ij conj(H_lj)              j ascending, i >= l, mirrored
 *   LDL^H d_j = Re A_jj - sum_{k<j} ((Re L_jk)^2 + (Im L_jk)^2) d_k
 *         L_ij = (A_ij - sum_{k<j} (L_ik conj(L_jk)) d_k) / d_j
 *   M = L^-1   M_im = -sum_{k=m}^{i-1} L_ik M_km  (M_mm = 1)
 *   A^-1_il = sum_{k=i}^{n-1} (conj(M_ki) M_kl) / d_k   i >= l, mirrored (conj)
 *   z = A^-1 u  z_i = sum_l A^-1_il u_l         l ascending
 * Complex products: (a+bi)(c+di) = (ac - bd) + (ad + bc)i and
 * conj(a+bi)(c+di) = (ac + bd) + (ad - bc)i, each product and sum rounded.  */
typedef struct { double re, im; } cplx;

static cplx cmul(cplx a, cplx b) { cplx r; r.re = a.re * b.re - a.im * b.im; r.im = a.re * b.im + a.im * b.re; return r; }
static cplx cmulc(cplx a, cplx b) { cplx r; r.re = a.re * b.re + a.im * b.im; r.im = a.re * b.im - a.im * b.re; return r; }

/* A^-1 of A = H H^H for one subcarrier.  H: [n_u][n_t] complex64 interleaved;
 * out: [n_u][n_u] complex double interleaved.  n_u <= 32.                  */
static void vpp_gram_inverse(int n_u, int n_t, const float *H, cplx *Ainv)
{
    cplx A[32 * 32], L[32 * 32], M[32 * 32];
    double d[32];
    const int n = n_u;
    for (int i = 0; i < n; ++i) {
        for (int l = 0; l <= i; ++l) {
            double re = 0.0, im = 0.0;
            for (int j = 0; j < n_t; ++j) {
                double a = H[2 * (i * n_t + j)], b = H[2 * (i * n_t + j) + 1];
                double c = H[2 * (l * n_t + j)], e = H[2 * (l * n_t + j) + 1];
                double pre = a * c + b * e;   /* H_ij conj(H_lj) */
                double pim = b * c - a * e;
                re = re + pre;
                im = im + pim;
            }
            A[i * n + l].re = re; A[i * n + l].im = im;
            A[l * n + i].re = re; A[l * n + i].im = -im;
        }
    }
    for (int j = 0; j < n; ++j) {
        double dj = A[j * n + j].re;
        for (int k = 0; k < j; ++k) {
            cplx v = L[j * n + k];
            double t = v.re * v.re + v.im * v.im;
            t = t * d[k];
            dj = dj - t;
        }
        d[j] = dj;
        for (int i = j + 1; i < n; ++i) {
            cplx s = A[i * n + j];
            for (int k = 0; k < j; ++k) {
                cplx v = cmulc(L[j * n + k], L[i * n + k]);   /* L_ik conj(L_jk) */
                v.re = v.re * d[k];
                v.im = v.im * d[k];
                s.re = s.re - v.re;
                s.im = s.im - v.im;
            }
            L[i * n + j].re = s.re / d[j];
            L[i * n + j].im = s.im / d[j];
        }
    }
    for (int m = 0; m < n; ++m) {
        M[m * n + m].re = 1.0; M[m * n + m].im = 0.0;
        for (int i = m + 1; i < n; ++i) {
            cplx s = {0.0, 0.0};
            for (int k = m; k < i; ++k) {
                cplx v = cmul(L[i * n + k], M[k * n + m]);
                s.re = s.re + v.re;
                s.im = s.im + v.im;
            }
            M[i * n + m].re = -s.re; M[i * n + m].im = -s.im;
        }
    }
    for (int i = 0; i < n; ++i) {
        for (int l = 0; l <= i; ++l) {
            cplx acc = {0.0, 0.0};
            for (int k = i; k < n; ++k) {
                cplx v = cmulc(M[k * n + i], M[k * n + l]);   /* conj(M_ki) M_kl */
                v.re = v.re / d[k];
                v.im = v.im / d[k];
                acc.re = acc.re + v.re;
                acc.im = acc.im + v.im;
            }
            Ainv[i * n + l] = acc;
            Ainv[l * n + i].re = acc.re; Ainv[l * n + i].im = -acc.im;
        }
    }
}

/*
 * oracle_vpp_build: VPP Ising couplings for a slot.
 *   H [n_sc][n_u][n_t] complex64; u [n_sc][n_sym][n_u] complex64; tau > 0.
 *   G_out [n_sc][2n_u][2n_u] float = (tau/2)^2 * real form of A^-1
 *   f_out [n_sc*n_sym][2n_u] float = -(tau/2) * [Re z; Im z],  z = A^-1 u
 *   Ainv_out [n_sc][n_u][n_u] complex double (may be NULL)
 * Real form of X + iY: [[X, -Y], [Y, X]].
 */
int oracle_vpp_build(int n_sc, int n_sym, int n_u, int n_t, const float *H, const float *u,
                     double tau, float *G_out, float *f_out, double *Ainv_out, int nthreads)
{
    if (n_u <= 0 || n_u > 32 || n_t <= 0 || n_sc < 0 || n_sym <= 0 || !(tau > 0.0)) return -1;
    const double ht = 0.5 * tau;
    const double sg = ht * ht;
    const double sf = -ht;
    const int K = 2 * n_u;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
#pragma omp parallel for schedule(dynamic, 8)
    for (int sc = 0; sc < n_sc; ++sc) {
        cplx Ainv[32 * 32];
        vpp_gram_inverse(n_u, n_t, H + (size_t)sc * (size_t)n_u * (size_t)n_t * 2u, Ainv);
        if (Ainv_out) {
            for (int e = 0; e < n_u * n_u; ++e) {
                Ainv_out[((size_t)sc * n_u * n_u + e) * 2] = Ainv[e].re;
                Ainv_out[((size_t)sc * n_u * n_u + e) * 2 + 1] = Ainv[e].im;
            }
        }
        float *Gs = G_out + (size_t)sc * (size_t)K * (size_t)K;
        for (int i = 0; i < n_u; ++i) {
            for (int l = 0; l < n_u; ++l) {
                cplx a = Ainv[i * n_u + l];
                Gs[i * K + l] = (float)(sg * a.re);
                Gs[(i + n_u) * K + (l + n_u)] = (float)(sg * a.re);
                Gs[i * K + (l + n_u)] = (float)(sg * (-a.im));
                Gs[(i + n_u) * K + l] = (float)(sg * a.im);
            }
        }
        for (int sym = 0; sym < n_sym; ++sym) {
            const float *us = u + ((size_t)sc * n_sym + sym) * (size_t)n_u * 2u;
            float *fs = f_out + ((size_t)sc * n_sym + sym) * (size_t)K;
            for (int i = 0; i < n_u; ++i) {
                cplx z = {0.0, 0.0};
                for (int l = 0; l < n_u; ++l) {
                    cplx ul = {(double)us[2 * l], (double)us[2 * l + 1]};
                    cplx v = cmul(Ainv[i * n_u + l], ul);
                    z.re = z.re + v.re;
                    z.im = z.im + v.im;
                }
                fs[i] = (float)(sf * z.re);
                fs[i + n_u] = (float)(sf * z.im);
            }
        }
    }
    return 0;
}

int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
