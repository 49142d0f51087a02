// Internal interface between the C ABI (capi.hip) and the device code
// (kernels.hip).  Not installed; the public interface is include/mmgap.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mmgap {

// Supported structure of the anneal kernels: K padded up to KT in {8,16,32},
// q in 1..4 spins per real dimension.
constexpr int kMaxK = 64;
constexpr int kMaxQ = 4;
constexpr int kMaxChains = 1024;
constexpr int kMaxSweeps = 8192;
constexpr int kMaxStages = 64;     // stages of detection around a guess
// Metropolis threshold table: T[j] = round(2^16 2^(-j/64)), j < 1024; T[1024] = 0
constexpr int kAcceptTable = 1025;

inline int padded_k(int K) { return K <= 8 ? 8 : (K <= 16 ? 16 : (K <= 32 ? 32 : 64)); }
inline int spin_words(int KT, int q) { return (KT * q + 31) / 32; }

struct DetBuildArgs {
    const float2 *H;        // [n_sc][n_r][n_t]
    const float2 *y;        // [n_sc][n_sym][n_r]
    int n_sc, n_r, n_t, n_sym;
    int ld;                 // leading dimension of G / f / x_fb outputs (>= 2 n_t)
    int qtop;               // 2^q - 1, the largest PAM level
    double c, c2;           // constellation scale and its square
    double noise_var;
    float *G;               // [n_sc][ld][ld]
    float *f;               // [n_sc*n_sym][ld]
    signed char *x_fb;      // [n_sc*n_sym][ld] or null
    double *ynorm;          // [n_sc*n_sym] ||y||^2 or null
};

struct VppBuildArgs {
    const float2 *H;        // [n_sc][n_u][n_t]
    const float2 *u;        // [n_sc][n_sym][n_u]
    int n_sc, n_u, n_t, n_sym;
    int ld;
    double tau;
    float *G;               // [n_sc][ld][ld]
    float *f;               // [n_sc*n_sym][ld]
    signed char *x_fb;      // [n_sc*n_sym][ld] zeros, or null
    double2 *Ainv;          // [n_sc][n_u][n_u] or null
    double *unorm;          // [n_sc*n_sym] u^H A^-1 u or null
};

// CIM-CAC model constants as the kernels use them: p - 1 and -zeta rounded
// once in float32 on the host.
struct CimParams {
    float dt, pm1, a, nzeta, eps, amp0;
    int f_mvm;
};

struct AnnealArgs {
    const float *G;         // [n_G][KT][KT]
    int inst_per_G;
    const float *f;         // [n_inst][KT]
    const signed char *x_fb;// [n_inst][KT] (init from fallback) or null
    const float *beta2;     // [sweeps] device
    const uint32_t *accept_table;  // [kAcceptSteps + 1] device
    int sweeps, chains, n_inst;
    int w[kMaxQ];           // spin weights (powers of two)
    uint32_t key0, key1;
    uint32_t inst_base;     // Philox instance index of instance 0 of the launch
    int init_mode;
    int glanes;             // 0: one instance per wavefront (or several wavefronts per
                            // instance); else lanes per instance, a power of two in
                            // [chains, 32]: 64/glanes instances per wavefront share a G
                            // (64/glanes must divide inst_per_G)
    float *chain_E;         // [n_inst][chains]
    uint32_t *chain_S;      // [n_inst][chains][NW]
    CimParams cim;          // launch_cim only (sweeps = Euler steps, beta2 unused)
    unsigned char *chain_div;   // launch_cim: [n_inst][chains] divergence flags, or null
    int n_real;             // launch_cim: spins K q without the padding (divergence check)
};

// Largest final amplitude magnitude of a CIM-CAC run that is not counted as
// diverged (the fixed points of the amplitudes are O(1)).
constexpr float kCimDivergeBound = 1000.0f;

// Spin words [n][NW] (bit set = -1) -> int8 spins [n][N].
hipError_t launch_chain_spins(const uint32_t *S, int NW, int N, size_t n, signed char *out,
                              hipStream_t s);

enum SelectMode { kSelectSolve = 0, kSelectDet = 1, kSelectVpp = 2, kSelectDelta = 3 };

struct SelectArgs {
    int mode;
    int n_inst, K, KT, q, chains;
    int w[kMaxQ];
    const float *G;         // [n_G][KT][KT]
    int inst_per_G;
    const float *f;         // [n_inst][KT]
    const signed char *x_fb;// [n_inst][KT] or null
    const float *chain_E;
    const uint32_t *chain_S;
    // solve outputs
    signed char *spins_out; // [n_inst][K*q]
    float *e_out;           // [n_inst]
    int *win_out;           // [n_inst] or null
    // detection decode
    const float2 *H;        // DET [n_sc][n_r][n_t]; VPP [n_sc][n_u][n_tx]
    const float2 *y;        // DET y [n_sc][n_sym][n_r]; VPP u [n_sc][n_sym][n_u]
    int n_rows, n_cols, n_sym;
    double c;
    unsigned char *sym_out; // [n_inst][n_t]
    float *metric_out;      // [n_inst] or null
    // VPP decode
    const double2 *Ainv;    // [n_sc][n_u][n_u]
    double tau;
    signed char *v_out;     // [n_inst][2 n_u]
    float2 *x_out;          // [n_inst][n_tx] or null
    float *gamma_out;       // [n_inst] or null
    // detection around a guess (kSelectDelta): the winning move z (levels in
    // {-2, 0, 2}) is applied to guess, clamped to +-qtop, and kept when the
    // float32 energy with the full fields drops; decode != 0 then decodes the
    // guess as kSelectDet does
    signed char *guess;     // [n_inst][KT] in/out
    const float *f_full;    // [n_inst][KT]
    int qtop, decode, dq;   // dq: bits per real dimension of the constellation (decode)
};

// Fields of the move problem around a guess: f' = f - G x_g per instance.
struct DeltaPrepArgs {
    const float *G;         // [n_G][KT][KT]
    int inst_per_G;
    const float *f;         // [n_inst][KT]
    const signed char *guess;   // [n_inst][KT]
    float *f_out;           // [n_inst][KT]
    int n_inst, KT;
};

// Ordered MMSE-SIC detection (one wavefront per subcarrier).
struct SicArgs {
    const float2 *H;        // [n_sc][n_r][n_t]
    const float2 *y;        // [n_sc][n_sym][n_r]
    int n_sc, n_r, n_t, n_sym;
    int q;                  // bits per real dimension
    double c;               // constellation scale
    double noise_var;
    signed char *levels;    // [n_sc*n_sym][ldl] or null; zero beyond 2 n_t
    int ldl;
    unsigned char *sym_out; // [n_sc*n_sym][n_t] or null
    float *metric_out;      // [n_sc*n_sym] or null (needs sym_out)
    int *order_out;         // [n_sc][n_t] or null
};

// The better of two level vectors per instance by float32 energy, then decode.
struct PickArgs {
    const float *G;         // [n_G][KT][KT]
    int inst_per_G;
    const float *f;         // [n_inst][KT] fields of the detection problem
    const signed char *xa;  // [n_inst][KT] first candidate
    const signed char *xb;  // [n_inst][KT] second candidate (wins only if strictly lower)
    int n_inst, K, KT, q;
    const float2 *H;
    const float2 *y;
    int n_rows, n_cols, n_sym;
    double c;
    unsigned char *sym_out; // [n_inst][n_t]
    float *metric_out;      // [n_inst] or null
    unsigned char *from_b;  // [n_inst] or null: 1 where the second candidate won
};

// Detection by moves around one or two guesses in one launch (the stages,
// selections, choice and decode of DeltaPrepArgs + AnnealArgs + SelectArgs
// (kSelectDelta) + PickArgs, with identical results).  Metropolis anneals,
// two unit-weight spins per real dimension.
struct SearchArgs {
    const float *G;         // [n_G][KT][KT] detection couplings (exactly symmetric)
    int inst_per_G;         // instances per G (n_sym)
    const float *f;         // [n_inst][KT] fields of the detection problem
    const signed char *guess_a; // [n_inst][KT] guess of the chain with keys seed + s, or null
    const signed char *guess_b; // [n_inst][KT] guess of the chain with keys
                                // seed + kMaxStages + s, or null (B wins only if strictly lower)
    const float *beta2;     // [sweeps] device
    const uint32_t *accept_table;
    int n_inst, K, sweeps, chains, stages, init_mode;
    int glanes;             // lanes per instance: a power of two in [max(chains, 4), 64];
                            // 64 / glanes must divide inst_per_G
    uint32_t key0, key1, inst_base;
    int dq;                 // bits per real dimension (clamp to +-(2^dq - 1), decode)
    const float2 *H;        // [n_sc][n_rows][n_cols]
    const float2 *y;        // [n_sc][n_sym][n_rows]; n_rows <= 2 glanes
    int n_rows, n_cols, n_sym;
    double c;
    unsigned char *sym_out; // [n_inst][n_cols]
    float *metric_out;      // [n_inst] or null
    unsigned char *from_b;  // [n_inst] or null: 1 where the answer is chain B's
};

struct ExpandArgs {
    const float *G;         // [n_sc][K][K] (unpadded)
    const float *f;         // [n_inst][K]
    const double *norm;     // [n_inst] ||y||^2 or u^H A^-1 u
    int n_sc, n_sym, K, q;
    int w[kMaxQ];
    float *J;               // [n_sc][N][N] or null
    float *h;               // [n_inst][N] or null
    float *e_const;         // [n_inst] or null
};

// One job of the fused persistent kernel (device copy, read wave-uniformly).
struct FusedJob {
    int kind;               // 0 detection, 1 VPP
    int variant;            // anneal variant: fused_variant(KT, Q)
    int KT, Q, K;
    int n_rows, n_cols;     // H is n_rows x n_cols (DET: n_r x n_t; VPP: n_u x n_tx)
    int n_sym, n_sc;
    int chains, sweeps, init, wpi;
    int stages;             // 0, or detection by moves around the MMSE guess: stages
    int dq;                 // bits per real dimension of the constellation (decode, clamp)
    int glanes;             // 0, or lanes per instance (power of two in [max(chains, 4), 32])
                            // with 64/glanes instances of the item per wavefront
    int ldf;                // row stride of f in floats: a multiple of 32 (128 bytes), >= KT
    int w[kMaxQ];
    uint32_t key0, key1;
    uint32_t inst_base;     // Philox instance index of the job's instance 0
    double c, c2, noise_var, tau;
    const float2 *H;
    const float2 *y;        // y (DET) or u (VPP)
    const float *beta2;     // [sweeps] device
    float *f;               // [n_sc*n_sym][ldf] scratch
    float *fp;              // [n_sc*n_sym][ldf] scratch: move fields f - G x_g (stages > 0)
    signed char *x_fb;      // [n_sc*n_sym][KT] scratch
    int guesses;            // stages > 0: chains from 1 the MMSE guess, 2 the MMSE-SIC
                            // guess, 3 both (MMGaP-E: the better answer)
    signed char *x_sic;     // [n_sc*n_sym][KT] scratch: the MMSE-SIC chain's guess, written
                            // by the batch's MMSE-SIC launch before the persistent kernels
    void *out0, *out1, *out2;   // DET: sym, metric, from-SIC flags; VPP: v, x, gamma
};
// A work item: symbols sym0..sym0+ns-1 of subcarrier sc of job `job`.
struct FusedItem {
    int job, sc, sym0, ns;
};

// Anneal variant of (KT, q) in the fused path (0..8), -1 if there is none;
// the register class (0..2) of a variant, -1 if invalid.  One persistent
// kernel per class, each with its own work counter.
constexpr int kFusedClasses = 3;
int fused_variant(int KT, int q);
int fused_kernel_class(int variant);
// Zero the kFusedClasses work counters (a kernel, so that it can be recorded
// in a graph).
hipError_t launch_fused_reset(unsigned int *counters, hipStream_t s);
// The persistent kernel of class `cls` over `n_items` items of that class.
hipError_t launch_fused(int cls, const FusedJob *jobs, const FusedItem *items, int n_items,
                        unsigned int *counter, const uint32_t *accept_table, int blocks,
                        hipStream_t s);
hipError_t fused_blocks_per_cu(int cls, int *blocks);

hipError_t launch_det_build(const DetBuildArgs &a, hipStream_t s);
hipError_t launch_vpp_build(const VppBuildArgs &a, hipStream_t s);
hipError_t launch_anneal(int KT, int q, const AnnealArgs &a, hipStream_t s);
// CIM-CAC anneals (same outputs as launch_anneal); KT q <= 32 one lane per
// anneal, (KT, q) in {(16, 3), (16, 4), (32, 2)} two lanes per anneal.
hipError_t launch_cim(int KT, int q, const AnnealArgs &a, hipStream_t s);
hipError_t launch_select(const SelectArgs &a, hipStream_t s);
hipError_t launch_delta_prep(const DeltaPrepArgs &a, hipStream_t s);
hipError_t launch_sic(const SicArgs &a, hipStream_t s);
hipError_t launch_pick(const PickArgs &a, hipStream_t s);
// KT in {8, 16, 32}: the padded dimension count of the detection problem.
hipError_t launch_search(int KT, const SearchArgs &a, hipStream_t s);
hipError_t launch_expand(const ExpandArgs &a, hipStream_t s);
// copy [n][K][K] -> [n][KT][KT] (and [m][K] -> [m][KT]) with zero padding
hipError_t launch_pad_matrix(const float *src, float *dst, int n, int K, int KT, hipStream_t s);
hipError_t launch_pad_rows_f32(const float *src, float *dst, int m, int K, int KT, hipStream_t s);
hipError_t launch_fill_u8(void *dst, unsigned char v, size_t n, hipStream_t s);
hipError_t launch_pad_rows_i8(const signed char *src, signed char *dst, int m, int K, int KT,
                              hipStream_t s);

}  // namespace mmgap
