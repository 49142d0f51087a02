/*
 * mmgap.h -- C ABI of the MI355X (gfx950) Ising hot path for uplink ML-MIMO
 * detection and downlink vector-perturbation precoding, after "MMGaP:
 * Multi-User MIMO Detection and Precoding using GPU-assisted Physics-inspired
 * Computation" (arXiv 2510.01579).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  * Buffers are DEVICE pointers owned by the caller unless marked (host).
 *    The library keeps no caller pointer after a call returns.
 *  * Complex data are interleaved complex64 (re, im float32 pairs), row-major.
 *  * Every compute call is asynchronous on `stream` (a hipStream_t; NULL means
 *    the legacy default stream).  Results are valid once the stream reaches
 *    the point where the call was enqueued.
 *  * Return value: MMGAP_OK (0) or a negative mmgap_status.  A message for the
 *    last failure of a context is returned by mmgap_last_error(ctx).  Nothing
 *    throws across this boundary.  Host-side checks (shapes, NULL pointers,
 *    unsupported sizes) fail before anything is enqueued; a device fault or a
 *    failed launch is reported as MMGAP_EDEVICE.
 *  * Instance numbering: problem instance n = sc * n_sym + sym of a call.  The
 *    Philox stream of every chain is keyed by (schedule.seed, schedule.inst_base
 *    + n, chain, sweep, spin), so results do not depend on how instances are
 *    grouped into launches, and a call on subcarriers [a, b) of a slot with
 *    inst_base = a * n_sym draws exactly the random numbers that a call on the
 *    whole slot draws for them (paper §5.3: the subcarriers of a slot are split
 *    over GPUs with no exchange between them).
 *  * Sizes (MMGAP_EUNSUPPORTED outside them): DET n_tx <= 32 users, more than
 *    16 users only with QPSK or 16-QAM, n_rx <= 64; VPP n_rx <= 16 users,
 *    n_tx <= 64 antennas; n_sym <= 64; chains 1..1024; sweeps 1..8192.  The
 *    entry points around MMSE-SIC need n_tx <= 16, CIM-CAC dynamics K <= 32
 *    and K q <= 64 spins (K padded to 8, 16 or 32).  Batches and the server:
 *    jobs with stages K <= 32; jobs of the persistent kernels chains <= 256;
 *    detection with more than 16 users (binary encoding) runs the plain
 *    path's launches inside the batch.
 *  * A context must not be used by two host threads at once.
 *
 * Problem statement (paper §2.1 Eq. 1 and Eq. ml; §2.2; §3.3):
 *   DET  y = H x + noise, H is n_rx x n_tx per subcarrier, x in Omega^n_tx
 *        (square M-QAM, unit average energy); find argmin ||y - H x||^2.
 *   VPP  H is n_rx (users) x n_tx (antennas); W = H^H (H H^H)^-1 (zero forcing);
 *        find v in {-1,0,1}^(2 n_rx) (real and imaginary part of a Gaussian
 *        integer per user) minimising ||W (u + tau v)||^2.
 * Ising reduction (paper §2.3, §3.2; level-domain form of this library):
 *   E(x) = x^T G x - 2 f^T x,  x_k = sum_b w_b s_{k,b},  s in {-1,+1},
 *   K real dimensions, q spins per dimension, spin index i = k q + b.
 *   DET: K = 2 n_tx, q = log2(M)/2, w_b = 2^(q-1-b), G = c^2 H_r^T H_r,
 *        f = c H_r^T y_r (H_r, y_r: real decomposition), so that
 *        E(x) = ||y - c H_r x||^2 - ||y||^2.
 *   VPP: K = 2 n_rx, q = 2, w = (1, 1), levels {-2, 0, 2} = 2 v,
 *        G = (tau/2)^2 Re-form((H H^H)^-1), f = -(tau/2) Re-form((H H^H)^-1 u),
 *        so that E(x) = ||W (u + tau v)||^2 - ||W u||^2.
 */
#ifndef MMGAP_H
#define MMGAP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MMGAP_OK = 0,
    MMGAP_EINVAL = -1,        /* bad argument: NULL pointer, negative size, bad enum */
    MMGAP_ENOMEM = -2,        /* scratch would exceed the context's HBM budget */
    MMGAP_EDEVICE = -3,       /* HIP runtime or launch failure */
    MMGAP_EUNSUPPORTED = -4,  /* valid but outside the supported sizes */
    MMGAP_EBUSY = -5          /* serving queue full or budget exhausted (server only) */
} mmgap_status;

enum { MMGAP_KIND_DET = 0, MMGAP_KIND_VPP = 1 };

typedef struct mmgap_ctx mmgap_ctx;

/* Create a context on HIP device `device`.  hbm_budget_bytes caps the scratch
 * the context may hold (0 = 16 GiB).  *out receives the context. */
int mmgap_create(mmgap_ctx **out, int device, size_t hbm_budget_bytes);
/* Synchronise the context's device, free its scratch, destroy it. */
int mmgap_destroy(mmgap_ctx *ctx);
/* Message of the last failure of `ctx` (or of mmgap_create when ctx is NULL).
 * The string stays valid until the next call on the same context. */
const char *mmgap_last_error(const mmgap_ctx *ctx);

typedef struct {
    int kind;          /* MMGAP_KIND_DET or MMGAP_KIND_VPP */
    int n_rx, n_tx;    /* H is n_rx x n_tx; DET: n_tx <= 32 (more than 16 only with qam 4
                          or 16), n_rx <= 64; VPP: n_rx <= 16, n_tx <= 64 */
    int qam;           /* 4, 16 or 64 */
    int n_sc, n_sym;   /* H is held per subcarrier for n_sym symbols; n_sym <= 64 */
    float noise_var;   /* DET: sigma^2 per complex receive sample (MMSE regulariser) */
    float tau;         /* VPP: perturbation spacing; <= 0 selects 2 sqrt(M) c = 2 (c_max + d/2) */
} mmgap_problem;

/* Anneal dynamics of a schedule. */
enum { MMGAP_DYN_METROPOLIS = 0, MMGAP_DYN_CIM = 1 };

/*
 * Constants of the CIM-CAC model (paper §2.3 Eqs. cim1/cim2; §3.2 and Appendix
 * A for the integration): amplitudes x_i and error variables e_i of every spin
 * and of one auxiliary spin that carries the field,
 *   dx_i/dt = (p - 1) x_i - x_i^3 + eps e_i c_i,  de_i/dt = -zeta (x_i^2 - a) e_i,
 * c_i the coupling term (sum_{j != i} J_ij x_j + h_i x_a, and sum_i h_i x_i for
 * the auxiliary spin), integrated by explicit Euler steps of length dt with the
 * coupling term recomputed every f_mvm steps; e_i starts at 1 and is kept
 * >= 2^-20; initial amplitudes amp0 * u, u uniform in [-1, 1) from Philox
 * (random start) or amp0 times the fallback's spins (fallback start).  The
 * final spins are sign(x_i) sign(x_a).
 */
typedef struct {
    float dt;              /* Euler step, finite and > 0 */
    int f_mvm;             /* steps between recomputations of the coupling term, >= 1 */
    float p, a, zeta, eps; /* model constants, finite */
    float amp0;            /* initial amplitude scale, finite */
} mmgap_cim_params;

typedef struct {
    int chains;            /* independent anneals per instance, 1..1024 */
    int sweeps;            /* Metropolis: full sweeps over all spins per anneal; CIM: Euler
                              steps per anneal; 1..8192 */
    const float *beta2;    /* (host) Metropolis: [sweeps] inverse temperature times log2(e)
                              per sweep, >= 0, finite; CIM: unused (may be NULL) */
    uint64_t seed;         /* Philox4x32-10 key: (seed & 0xffffffff, seed >> 32) */
    int init;              /* 0: random initial spins from Philox; 1: start from the fallback levels */
    int dynamics;          /* MMGAP_DYN_METROPOLIS (0, also for zero-initialised schedules) or
                              MMGAP_DYN_CIM (plain entry points only; K <= 32, K q <= 64) */
    const mmgap_cim_params *cim;  /* (host) constants of MMGAP_DYN_CIM, else unused */
    uint32_t inst_base;    /* Philox instance index of the call's instance 0 (0 for a whole
                              slot; a * n_sym for a call on subcarriers [a, b) of it) */
} mmgap_schedule;

/*
 * mmgap_build_ising -- pre-processing (paper §3.2 "pre-processing kernel": the
 * Ising coefficients of every problem instance; §3.3 for VPP) plus the linear
 * fallback (§2.1 MMSE for DET; the all-zeros perturbation for VPP, §3.3).
 *   H        [n_sc][n_rx][n_tx] complex64
 *   y_or_u   DET: y [n_sc][n_sym][n_rx] complex64; VPP: u [n_sc][n_sym][n_rx] complex64
 *   G        [n_sc][K][K] float32, symmetric (out)
 *   f        [n_sc*n_sym][K] float32 (out)
 *   x_fallback [n_sc*n_sym][K] int8 levels (out, nullable): DET = MMSE estimate
 *            sliced to the nearest PAM level; VPP = 0
 *   J_dense  [n_sc][N][N] float32 (out, nullable), N = K q: spin couplings,
 *            J_ij = -2 w_i w_j G_{k(i)k(j)}, zero diagonal
 *   h_dense  [n_sc*n_sym][N] float32 (out, nullable): h_i = 2 w_i f_{k(i)}
 *   e_const  [n_sc*n_sym] float32 (out, nullable): sum_i w_i^2 G_{k(i)k(i)} plus
 *            ||y||^2 (DET) or ||W u||^2 (VPP), so that
 *            -sum_{i<j} J_ij s_i s_j - sum_i h_i s_i + e_const is the residual
 *            ||y - H x||^2 (DET) or the transmit energy ||W (u + tau v)||^2 (VPP).
 * Couplings and fields are accumulated in float64 and rounded once to float32.
 */
int mmgap_build_ising(mmgap_ctx *ctx, const mmgap_problem *prob, const void *H,
                      const void *y_or_u, float *G, float *f, signed char *x_fallback,
                      float *J_dense, float *h_dense, float *e_const, void *stream);

/*
 * mmgap_solve -- solver + post-processing (paper §3.2 "solver kernel" and
 * "post-processing kernel"): `chains` independent single-spin-flip Metropolis
 * anneals per instance from random initial states, each anneal's final state a
 * candidate ranked by its energy, the best candidate kept; a fallback
 * replaces it only when its energy is strictly lower.
 *   n_inst       number of instances (>= 0)
 *   K, q, w      structure: K <= 64 real dimensions with q <= 4 spins each for
 *                K <= 32 and q <= 2 for K > 32, w (host) [q] int8 weights, each a
 *                power of two in 1..64
 *   G            [n_inst/inst_per_G rounded up][K][K] float32, symmetric; instance n uses
 *                G[n / inst_per_G]
 *   f            [n_inst][K] float32
 *   x_fallback   [n_inst][K] int8 levels (nullable: no fallback)
 *   spins_out    [n_inst][K*q] int8, +1/-1 (out)
 *   e_out        [n_inst] float32 energy x^T G x - 2 f^T x of the result (out)
 *   win_out      [n_inst] int32 winning chain index, `chains` = fallback (out, nullable)
 * Chain arithmetic (float32, round-to-nearest, fma = single-rounding fused
 * multiply-add).  Sweeps visit the dimensions k = 0..K-1 and, within k, the
 * spins b = 0..q-1 (i = k q + b).  At each visit of k the field
 * g_k = (G x)_k - f_k is recomputed as fma(G_k,K-1, x_K-1, ... fma(G_k0, x_0, -f_k));
 * a flip of spin i changes x_k by d = -2 w_b s_i with dE = d ((g_k + g_k) + d G_kk),
 * z = beta2_t dE, and is accepted iff m < T[j], where m is the 16-bit Philox
 * draw of (spin i, sweep t, chain, instance n) -- Philox4x32-10 with counter
 * (i/8, t, chain, inst_base + n) and key (seed_lo, seed_hi), low half of word (i%8)/2 for
 * even i, high half for odd i --, j = floor(64 z) clamped to
 * [0, 1024] (z <= 0 or NaN gives 0) and T[j] = round(2^16 2^(-j/64)),
 * T[1024] = 0; on acceptance x_k += d and g_k = fma(G_kk, d, g_k).  Initial
 * spins: s_i = -1 iff bit 15 of the draw of (i, 0xffffffff, chain, inst_base + n) is set.
 * Energies E = fma(x_K-1, g_K-1 - f_K-1, ... fma(x_0, g_0 - f_0, 0)) with
 * fresh fields.  Ties in energy keep the lowest chain index.
 * With sched->dynamics = MMGAP_DYN_CIM each anneal is instead `sweeps` Euler
 * steps of the CIM-CAC model (mmgap_cim_params), N = K q <= 64 (K <= 32), with the
 * float32 arithmetic (every operation rounded once, fma as above)
 *   X_l = fma(w_q-1, x_(l,q-1), ... fma(w_0, x_(l,0), 0)),
 *   g_k = fma(G_k,K-1, X_K-1, ... fma(G_k0, X_0, 0)),
 *   c_i = ((-2 w_b) (g_k - G_kk (w_b x_i))) + ((2 w_b f_k) x_a)  for i = k q + b,
 *   c_a = fma(2 f_K-1, X_K-1, ... fma(2 f_0, X_0, 0)),
 * recomputed at steps t = 0, f_mvm, 2 f_mvm, ..., and per step, for every
 * amplitude from the values before the step,
 *   s2 = x x,  dx = ((p - 1) x - s2 x) + (eps e) c,  x' = x + dt dx,
 *   e' = e + dt ((-zeta) ((s2 - a) e)), replaced by 2^-20 unless greater,
 * with p - 1 and -zeta rounded once in float32.  Random start: x_i = amp0 (u / 32768)
 * for the signed 16-bit value u = d - 32768 of the draw d of (i, 0xffffffff,
 * chain, inst_base + n), x_a likewise from the draw of (0xfffffff8, 0xffffffff,
 * chain, inst_base + n);
 * fallback start: x_i = amp0 s_i of the fallback's spins, x_a = amp0.  Final
 * spin i is -1 iff (x_i < 0) differs from (x_a < 0); energies and selection as
 * above.
 */
int mmgap_solve(mmgap_ctx *ctx, int n_inst, int K, int q, const signed char *w,
                const float *G, int inst_per_G, const float *f, const signed char *x_fallback,
                const mmgap_schedule *sched, signed char *spins_out, float *e_out,
                int *win_out, void *stream);

/*
 * mmgap_detect -- uplink ML-MIMO detection (paper §3.2; Eq. ml): build,
 * anneal, select, decode.  H [n_sc][n_rx][n_tx], y [n_sc][n_sym][n_rx]
 * complex64; prob->kind must be MMGAP_KIND_DET.
 *   sym_out     [n_sc*n_sym][n_tx] uint8 Gray-labelled symbol indices (out): for
 *               PAM levels (lI, lQ), p = (l + 2^q - 1)/2, g = p ^ (p >> 1),
 *               index = (gI << q) | gQ; the point is c (lI + j lQ)
 *   metric_out  [n_sc*n_sym] float32 ||y - H x||^2 of the result, evaluated in
 *               float64 (out, nullable)
 */
int mmgap_detect(mmgap_ctx *ctx, const mmgap_problem *prob, const void *H, const void *y,
                 const mmgap_schedule *sched, unsigned char *sym_out, float *metric_out,
                 void *stream);

/*
 * mmgap_detect_noalloc -- mmgap_detect for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): the same arguments, launches and results, bit for bit,
 * but its scratch (couplings, fields, fallback levels, every chain's energy
 * and spins) lives in a fixed array of 128 MiB per device that the library
 * holds until the process ends; the call allocates nothing, neither device
 * nor host memory.  The scratch it needs is
 *   4 n_sc KT^2 + 5 I KT + 4 I C (1 + ceil(KT q / 32)) bytes (each term
 *   rounded up to 256), I = n_sc n_sym, KT = 2 n_tx rounded up to 8, 16, 32 or 64,
 * e.g. 27 MB for a 3276 x 12 8x8 16-QAM slot at 64 chains; a call above 128 MiB
 * returns MMGAP_EUNSUPPORTED with nothing launched (split it by subcarriers,
 * with schedule.inst_base = first subcarrier x n_sym to keep the random
 * streams of the whole call).  Every call on one device shares that device's
 * array: calls on one context are ordered like the context's other calls, but
 * calls that overlap on one device through different contexts or threads race
 * and give undefined results.  Nothing in the array needs clearing: each call
 * writes every value it reads.
 */
int mmgap_detect_noalloc(mmgap_ctx *ctx, const mmgap_problem *prob, const void *H,
                         const void *y, const mmgap_schedule *sched, unsigned char *sym_out,
                         float *metric_out, void *stream);

/*
 * mmgap_cim_chains -- every CIM-CAC anneal's own final state, for studies of
 * the integration (paper Appendix A: the sign of the final amplitudes and
 * whether the integration diverged, against a fine-step reference with the
 * same initial values).  Arguments as mmgap_solve; sched must select
 * MMGAP_DYN_CIM (else MMGAP_EINVAL), K (padded) <= 32 and K q (padded) <= 64.
 * No selection.
 *   spins_out     [n_inst][chains][K q] int8 +-1, sign(x_i) sign(x_a) (out)
 *   e_out         [n_inst][chains] float32 energies of those spins (out, nullable)
 *   diverged_out  [n_inst][chains] uint8 (out, nullable): 1 where an amplitude of a
 *                 real spin or of the auxiliary one ended beyond 1000 in magnitude or
 *                 not finite, or such an error variable ended not finite
 */
int mmgap_cim_chains(mmgap_ctx *ctx, int n_inst, int K, int q, const signed char *w,
                     const float *G, int inst_per_G, const float *f,
                     const signed char *x_fallback, const mmgap_schedule *sched,
                     signed char *spins_out, float *e_out, unsigned char *diverged_out,
                     void *stream);

/*
 * mmgap_detect_delta -- uplink detection by moves around a guess (paper §2.3,
 * the Delta-Ising form built around an initial guess, Fig. 5; §3.2 MMGaP-E,
 * several stages each starting from the previous stage's solution).  Every
 * real dimension may move by z in {-2, 0, 2} levels (the neighbouring
 * constellation point either way), two unit-weight spins each; with levels
 * x = x_g + z the problem keeps the couplings G and takes the fields
 * f' = f - G x_g, f'_k = f_k - fma(G_k,K-1, xg_K-1, ... fma(G_k0, xg_0, 0)).
 * Each of `stages` (1..64) stages anneals it with sched (Metropolis or CIM-CAC,
 * as mmgap_solve with q = 2, w = {1, 1}; Philox key = sched->seed + stage), the
 * zero move as the fallback; the winning move is applied, clamped to
 * +-(sqrt(M) - 1), and kept iff the float32 energy x^T G x - 2 f^T x (the
 * arithmetic of mmgap_solve) is strictly lower than the guess's.  The final
 * guess is decoded as in mmgap_detect.
 *   guess   [n_sc*n_sym][2 n_tx] int8 odd levels (nullable: the sliced MMSE
 *           estimate of mmgap_build_ising)
 *   sym_out, metric_out   as in mmgap_detect
 */
int mmgap_detect_delta(mmgap_ctx *ctx, const mmgap_problem *prob, const void *H, const void *y,
                       const mmgap_schedule *sched, int stages, const signed char *guess,
                       unsigned char *sym_out, float *metric_out, void *stream);

/*
 * mmgap_detect_sic -- ordered MMSE successive interference cancellation, the
 * MMSE-SIC baseline of the paper's evaluation (§1, §4) and the second initial
 * guess of MMGaP-E (§3.2).  The paper does not state the ordering rule; here,
 * with P = (H_R^H H_R + sigma^2 I)^-1 over the users R not yet detected, each
 * step detects the user i of R with the smallest Re P_ii (the smallest MMSE
 * error variance; the lowest index among equals), estimates it by the row
 * P_i,R H_R^H applied to the residual, slices the estimate per real dimension
 * to the nearest odd PAM level (clamped), and subtracts h_i c (lI + j lQ)
 * from the residual.  The ordering depends on H and sigma^2 only.  float64
 * throughout; n_tx <= 16, n_rx <= 64 (else MMGAP_EUNSUPPORTED).
 * H [n_sc][n_rx][n_tx], y [n_sc][n_sym][n_rx] complex64 (device).
 *   sym_out     as in mmgap_detect (nullable)
 *   metric_out  as in mmgap_detect (nullable; needs sym_out)
 *   levels_out  [n_sc*n_sym][2 n_tx] int8 odd levels, real parts then
 *               imaginary (out, nullable)
 *   order_out   [n_sc][n_tx] int32: the user detected at each step (out, nullable)
 */
int mmgap_detect_sic(mmgap_ctx *ctx, const mmgap_problem *prob, const void *H, const void *y,
                     unsigned char *sym_out, float *metric_out, signed char *levels_out,
                     int *order_out, void *stream);

/*
 * mmgap_detect_e -- MMGaP-E (paper §3.2, Fig. 6): per problem two chains of
 * `stages` stages of moves around a guess as in mmgap_detect_delta, one from
 * the sliced MMSE estimate (Philox keys sched->seed + s) and one from the
 * MMSE-SIC estimate of mmgap_detect_sic (keys sched->seed + 64 + s); the
 * output is the better final answer by the float32 energy x^T G x - 2 f^T x,
 * the MMSE-SIC chain's only if strictly lower.  Same limits as both.  Where
 * the one-launch search runs (mmgap_set_option) the MMSE-SIC estimate, the
 * build and the search follow one another on `stream`; through the stage
 * launches, with both chains, the MMSE-SIC estimate and its chain run on a
 * second stream of the context, forked from and joined back into `stream`
 * (the call stays ordered on `stream` like every other call).
 *   guesses       MMGAP_GUESS_MMSE | MMGAP_GUESS_SIC runs both chains (the
 *                 paper's MMGaP-E); one of them runs that chain alone, whose
 *                 answer is then the output (else MMGAP_EINVAL)
 *   sym_out, metric_out   as in mmgap_detect
 *   from_sic_out  [n_sc*n_sym] uint8, 1 where the MMSE-SIC chain's answer was
 *                 taken (out, nullable)
 */
#define MMGAP_GUESS_MMSE 1
#define MMGAP_GUESS_SIC 2
int mmgap_detect_e(mmgap_ctx *ctx, const mmgap_problem *prob, const void *H, const void *y,
                   const mmgap_schedule *sched, int stages, int guesses, unsigned char *sym_out,
                   float *metric_out, unsigned char *from_sic_out, void *stream);

/*
 * mmgap_vpp_precode -- downlink vector-perturbation precoding (paper §2.2 Eq.
 * VPP, §3.3): the same solver on (H_p = -tau W/2, y~ = W u) with the all-zeros
 * fallback.  H [n_sc][n_rx][n_tx], u [n_sc][n_sym][n_rx] complex64;
 * prob->kind must be MMGAP_KIND_VPP.
 *   v_out      [n_sc*n_sym][2 n_rx] int8 in {-1,0,1}: real parts then imaginary (out)
 *   x_out      [n_sc*n_sym][n_tx] complex64 W (u + tau v), float64 internally (out, nullable)
 *   gamma_out  [n_sc*n_sym] float32 ||W (u + tau v)||^2 (out, nullable)
 */
int mmgap_vpp_precode(mmgap_ctx *ctx, const mmgap_problem *prob, const void *H, const void *u,
                      const mmgap_schedule *sched, signed char *v_out, void *x_out,
                      float *gamma_out, void *stream);

/*
 * Batches: many jobs of mixed kinds and sizes in ONE persistent launch (paper
 * §3.2 executes each stage as its own kernel over all instances; here the three
 * stages of every instance run back to back inside one kernel that takes work
 * items from a device queue, so that one launch serves a mixed workload).
 *
 * A job is one call's worth of work: a problem, its schedule, its inputs and
 * its outputs, exactly as for mmgap_detect / mmgap_vpp_precode:
 *   DET  y_or_u = y; out0 = sym_out [n_sc*n_sym][n_tx] uint8 (required),
 *        out1 = metric_out [n_sc*n_sym] float32 (nullable), out2 unused.
 *   VPP  y_or_u = u; out0 = v_out [n_sc*n_sym][2 n_rx] int8 (required),
 *        out1 = x_out [n_sc*n_sym][n_tx] complex64 (nullable),
 *        out2 = gamma_out [n_sc*n_sym] float32 (nullable).
 * stages = 0: the problem as mmgap_detect / mmgap_vpp_precode solve it; DET
 * with stages >= 1: detection by moves around the sliced MMSE estimate as
 * mmgap_detect_delta with that many stages (the stages of a work item run
 * inside the item's workgroup), or, with guesses != 0, as mmgap_detect_e with
 * those guesses (paper §3.2 Fig. 6, MMGaP-E; the MMSE-SIC guess of a work
 * item is computed in its workgroup after the build); out2 then takes
 * from_sic_out [n_sc*n_sym] uint8 (nullable).
 * Every output of a job is bit-identical to that of the single-job entry point
 * on the same arguments, whatever else is in the batch: a chain's random stream
 * depends only on the job's seed and its instance and chain index.
 * Limits: those of the single-job calls, K <= 32 real dimensions (DET n_tx <=
 * 16, VPP n_rx <= 16) and chains <= 256.
 */
typedef struct {
    mmgap_problem prob;
    mmgap_schedule sched;     /* beta2 is copied at plan creation */
    const void *H;            /* device, [n_sc][n_rx][n_tx] complex64 */
    const void *y_or_u;       /* device, [n_sc][n_sym][n_rx] complex64 */
    void *out0, *out1, *out2; /* device, see above */
    int stages;               /* 0, or DET: stages of moves around a guess (1..64) */
    int guesses;              /* DET with stages >= 1: 0 (= MMGAP_GUESS_MMSE) or a set of
                                 MMGAP_GUESS_* as for mmgap_detect_e; MMGAP_GUESS_SIC needs
                                 the MMSE-SIC factors to fit a work item's LDS (16 x 16 up to
                                 34 receive antennas; 8 users up to 27); out2 = from_sic_out */
} mmgap_job;

typedef struct mmgap_plan mmgap_plan;

enum {
    MMGAP_PLAN_GRAPH = 1,        /* record the launch as a HIP graph, replayed by each launch */
    MMGAP_PLAN_PERSISTENT = 2    /* every Metropolis job through the persistent kernels */
};

/*
 * mmgap_plan_create -- validate `n_jobs` jobs (host array), copy their
 * descriptors and schedules to the device, cut them into work items (one
 * subcarrier and up to 4, 2 or 1 symbols for <= 64, <= 128, <= 256 chains)
 * grouped by register class of the problem size (K <= 8 or K <= 16 with QPSK;
 * K <= 16 with 16-QAM; larger) and ordered by decreasing cost within a class,
 * and allocate the plan's own device scratch (fields and fallbacks; the
 * couplings, H and the VPP inverse of a work item stay in LDS), counted against
 * the context's HBM budget.  Three kinds of jobs run with launches of their
 * own inside the batch instead of work items: CIM-CAC jobs (binary encoding,
 * stages = 0; the build, anneal and selection launches of mmgap_detect /
 * mmgap_vpp_precode; CIM-CAC with stages is refused with MMGAP_EUNSUPPORTED);
 * Metropolis jobs wider than the persistent kernels' 32 padded dimensions
 * (detection with 17 to 32 users, binary encoding: the build, anneal and
 * selection launches of mmgap_detect; with stages they are refused with
 * MMGAP_EUNSUPPORTED); and, unless flags has MMGAP_PLAN_PERSISTENT, jobs with
 * stages that the one-launch search of mmgap_detect_e can run (the build, the
 * MMSE-SIC guess where asked, the search).  The outputs are the same either
 * way.  A launch
 * is: the MMSE-SIC launches, the own-launch jobs in order, then one
 * persistent kernel per class present, largest class first.  `blocks` =
 * workgroups of each persistent kernel, 0 = as many as the device holds at
 * once.  flags: MMGAP_PLAN_GRAPH and/or MMGAP_PLAN_PERSISTENT, or 0.
 * The plan stores the jobs' device pointers, not their contents: inputs may be
 * rewritten between launches; they must stay allocated until the plan is
 * destroyed.  Plans are independent of the context's other calls and must be
 * destroyed before their context.  On failure *out is NULL and nothing is held.
 */
int mmgap_plan_create(mmgap_ctx *ctx, int n_jobs, const mmgap_job *jobs, int flags, int blocks,
                      mmgap_plan **out);
/* Enqueue one execution of every job of the plan on `stream`.  Launches of the
 * same plan run one after another, also when issued on different streams. */
int mmgap_plan_launch(mmgap_plan *plan, void *stream);
/* (host) Work items of the plan and the largest workgroup count of its kernels. */
int mmgap_plan_info(const mmgap_plan *plan, int *n_items, int *blocks);
/* Wait for the plan's launches and free it (NULL is a no-op). */
int mmgap_plan_destroy(mmgap_plan *plan);

/*
 * Serving (continuous batching).  A context may run one server: a native
 * thread that admits submitted jobs (mmgap_job, as for plans) in arrival
 * order while room in its HBM arena and a free in-flight slot allow, launches
 * each admitted group of jobs as one batch of the persistent fused kernels on
 * its own stream, so that batches overlap on the device, and observes their
 * completion.  A batch's launches are recorded as a HIP graph and replayed;
 * each in-flight slot keeps its executable graph and updates it in place while
 * batches launch the same kernel classes.  Jobs submitted while others run are admitted as soon as slots
 * and memory free up.  Every job's outputs equal those of the single-job entry
 * points (the Philox streams do not depend on batching).  Inputs and outputs
 * stay on the device; the server keeps the job's pointers until the job is
 * reported done, and copies its schedule.
 *
 * mmgap_server_start -- start the server: max_inflight concurrent batches
 *   (1..8; each has its own stream), arena_bytes of HBM for the jobs' scratch
 *   (0 = 1 GiB), taken from the context's budget (MMGAP_ENOMEM if it does not
 *   fit), max_batch_jobs jobs per batch at most (0 = 64).  MMGAP_EBUSY if a
 *   server is running.
 * mmgap_server_submit -- queue one job; *job_id receives its id (> 0).  Work
 *   already enqueued on `stream` (e.g. the copies that produced H and y) is
 *   waited for before the job starts.  MMGAP_ENOMEM if the job could never fit
 *   the arena, MMGAP_EBUSY if 4096 jobs are waiting, and the argument errors
 *   of mmgap_plan_create.
 * mmgap_server_poll -- *done = 1 once the job's outputs are complete, with
 *   *latency_us (nullable) = microseconds from its submission to the moment
 *   the server saw it complete; a job reported done is forgotten (a later poll
 *   of its id is MMGAP_EINVAL).  Returns the job's status (MMGAP_EDEVICE if its
 *   batch failed).
 * mmgap_server_stats -- latency accounting of the jobs completed since the
 *   server started (or since the last call with reset != 0): how many, how
 *   many took longer than deadline_us (submission to observed completion, as
 *   mmgap_server_poll reports it), the nearest-rank 50th and 99th percentiles
 *   and the maximum, in microseconds (all 0 when none completed).  reset != 0
 *   starts a new accounting period after reading.  MMGAP_EINVAL without a
 *   server, with out NULL or a negative deadline.
 * mmgap_server_drain -- wait until every submitted job is complete.
 * mmgap_server_stop -- drain, stop the thread, free the arena and streams
 *   (also done by mmgap_destroy).
 * Like every call on a context, submit/poll/drain/stop must not be made from
 * two host threads at once; the server's own thread uses none of the
 * context's other state.
 */
int mmgap_server_start(mmgap_ctx *ctx, int max_inflight, size_t arena_bytes, int max_batch_jobs);
int mmgap_server_submit(mmgap_ctx *ctx, const mmgap_job *job, void *stream,
                        unsigned long long *job_id);
int mmgap_server_poll(mmgap_ctx *ctx, unsigned long long job_id, int *done, double *latency_us);
typedef struct {
    unsigned long long completed;   /* jobs completed in the period */
    unsigned long long missed;      /* of those, latency > deadline_us */
    double p50_us, p99_us, max_us;
} mmgap_server_stats_t;
int mmgap_server_stats(mmgap_ctx *ctx, double deadline_us, int reset, mmgap_server_stats_t *out);
int mmgap_server_drain(mmgap_ctx *ctx);
int mmgap_server_stop(mmgap_ctx *ctx);

/*
 * Tracing.  mmgap_set_profiling(ctx, 1) (re)starts recording: every later
 * compute call records HIP events on its stream around its stages, keeping the
 * last 256 calls.  mmgap_last_profile waits for those events and writes, oldest
 * call first, three host floats per call -- elapsed milliseconds of the build
 * (0 for mmgap_solve), the anneal kernel and the select/decode kernel -- for
 * at most capacity/3 of the most recent calls.  Returns the number of floats
 * written, or a negative mmgap_status (MMGAP_EINVAL if profiling is off or no
 * call was recorded).  Recording adds no synchronisation to the calls.
 */
int mmgap_set_profiling(mmgap_ctx *ctx, int enable);
int mmgap_last_profile(mmgap_ctx *ctx, float *ms, int capacity);

/*
 * Options of a context (results never depend on them).
 * MMGAP_OPT_STAGE_LAUNCHES -- value 1: mmgap_detect_delta and mmgap_detect_e
 *   run each stage as separate launches (move fields, anneal, selection) and
 *   choose between the two guesses in a launch of its own.  Value 0 (the
 *   default): with Metropolis anneals, KT <= 32, chains <= 64 and n_rx at
 *   most twice the lanes an instance takes (4 to 64: the power of two at
 *   least the chain count, and larger when fewer instances than 64 / lanes
 *   divide n_sym) every stage, both chains, the choice and the decode run in
 *   one launch after the build (paper §3.2: one pass of the hot path per
 *   stage, without the round trips through device memory).  The outputs are
 *   identical; the option is there for measurement and tests.
 * Returns MMGAP_OK, or MMGAP_EINVAL for an unknown option or value.
 */
enum { MMGAP_OPT_STAGE_LAUNCHES = 1 };
int mmgap_set_option(mmgap_ctx *ctx, int option, int value);

#ifdef __cplusplus
}
#endif

#endif /* MMGAP_H */
