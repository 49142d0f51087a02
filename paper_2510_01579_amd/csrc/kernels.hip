// Device code of the Ising hot path (gfx950 / CDNA4, wave64).
//
// Shared device functions (used by both launch paths, so that both compute
// the same values):
//  * build_det_sc / build_vpp_sc -- pre-processing of one subcarrier: the Ising
//    couplings G and fields f (paper §3.2 pre-processing kernel; §3.3 for the
//    vector-perturbation rewriting) and the linear fallback (§2.1 MMSE).
//  * anneal_lane<KT,Q> -- one single-spin-flip Metropolis anneal per lane
//    (paper §3.2: one anneal per thread, no synchronisation between anneals).
//  * fallback_energy, winning_levels, decode_det / decode_vpp -- post-processing:
//    best anneal, fallback rule, decode and float64 metrics (§3.2).
// Plain path: k_det_build / k_vpp_build -> k_anneal -> k_select, one launch per
// stage and problem size.  Fused path: k_fused, one persistent launch over a
// device work queue of (job, subcarrier, symbols) items of mixed sizes.
//
// Floating point: float32 chain state with round-to-nearest and no implicit
// contraction (this file is compiled with -ffp-contract=off and the pragma
// below).  Fused multiply-adds appear only where written as fmaf(); each one
// is either part of the arithmetic contract (field rows, energies) or has an
// exact product, so that it equals the separately rounded form.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cfloat>

#include "kernels.h"

#pragma clang fp contract(off)

namespace mmgap {
namespace {

constexpr int kBlock = 256;
constexpr int kWavesPerBlock = kBlock / 64;
constexpr int kAcceptSteps = 1024;

// ---------------------------------------------------------------------------
// Philox4x32-10 counter-based generator (Salmon, Moraes, Dror, Shaw, SC'11,
// "Parallel random numbers: as easy as 1, 2, 3").  Ten rounds of two 32x32
// multiplications with word swapping and a Weyl-sequence key schedule.
__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t pa = (uint64_t)0xD2511F53u * c[0];
        const uint64_t pb = (uint64_t)0xCD9E8D57u * c[2];
        // three-input XOR in one instruction (truth table 0x96: odd parity)
        const uint32_t n0 = __builtin_amdgcn_bitop3_b32((uint32_t)(pb >> 32), c[1], k0, 0x96);
        const uint32_t n2 = __builtin_amdgcn_bitop3_b32((uint32_t)(pa >> 32), c[3], k1, 0x96);
        c[1] = (uint32_t)pb;
        c[3] = (uint32_t)pa;
        c[0] = n0;
        c[2] = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

// ---------------------------------------------------------------------------
// Complex double helpers with a fixed operation order.
struct cd {
    double re, im;
};
__device__ __forceinline__ cd cmul(cd a, cd b)
{
    cd r;
    r.re = a.re * b.re - a.im * b.im;
    r.im = a.re * b.im + a.im * b.re;
    return r;
}
// conj(a) * b
__device__ __forceinline__ cd cmulc(cd a, cd b)
{
    cd r;
    r.re = a.re * b.re + a.im * b.im;
    r.im = a.re * b.im - a.im * b.re;
    return r;
}
__device__ __forceinline__ cd ld2(const double2 &v) { return cd{v.x, v.y}; }
__device__ __forceinline__ double2 st2(cd v) { return make_double2(v.re, v.im); }

// upper-triangle pair p (row-major, i <= j) of an n x n matrix
__device__ __forceinline__ void upper_pair(int p, int n, int &i, int &j)
{
    int row = 0, rem = p;
    while (rem >= n - row) {
        rem -= n - row;
        ++row;
    }
    i = row;
    j = row + rem;
}

// Hides a pointer's value from the optimiser so that loads through it are
// issued where written instead of being hoisted out of the sweep loop into
// registers.  The result lives in the constant
// address space, so wave-uniform loads through it use the scalar cache.  The
// pointer must be wave-uniform and known to the compiler as such.
typedef const float __attribute__((address_space(4))) cfloat;
__device__ __forceinline__ cfloat *opaque(const float *p)
{
    uint64_t v = (uint64_t)p;
    asm volatile("; row %0" : "+s"(v));
    return (cfloat *)v;
}
// Same for a wave-uniform 32-bit value (keeps the Philox round keys from
// being precomputed for all rounds and held in registers across the loop).
__device__ __forceinline__ uint32_t opaque_u32(uint32_t v)
{
    asm volatile("; key %0" : "+s"(v));
    return v;
}

// The workgroup index in an order where consecutive indices run on one XCD:
// the dispatcher deals workgroups p = 0, 1, 2, ... to the 8 XCDs in turn (p mod
// 8), so XCD x receives ceil or floor of n / 8 of them; they take consecutive
// logical indices, and workgroups that share data (one subcarrier's couplings)
// meet in one XCD's L2.  A bijection of [0, n).
constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_block(int p, int n)
{
    const int q = n / kXcds, r = n % kXcds;
    const int x = p % kXcds, i = p / kXcds;
    return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + i;
}

// Orders LDS writes of some lanes before LDS reads of other lanes of the same
// wavefront.
__device__ __forceinline__ void wave_sync_lds()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ---------------------------------------------------------------------------
// Detection build of one subcarrier (all threads of the block, a multiple of
// 64 of them):
//   Cg = H^H H (float64 matrix cores, upper triangle mirrored) -> G (real form, x c^2)
//   F  = H^H y per symbol (float64 matrix cores)               -> f (real form, x c)
//   MMSE (Cg + sigma^2 I)^-1 F by a Gauss-Jordan inverse, sliced to the nearest PAM level.
// Writes G (ld x ld, zero padded) to Gout and, for symbols sym0..sym0+ns-1,
// the field rows to fout, the fallback levels to xout (if non-null) and ||y||^2
// to ynorm (if non-null).  nt <= NT, nr <= NR <= 64, ns <= NS.
typedef double mfma_v4d __attribute__((ext_vector_type(4)));

// A complex float32 value in LDS scratch (a plain pair, so that the scratch
// structs stay trivial types).
struct cf32 {
    float x, y;
};
__device__ __forceinline__ cf32 to_cf32(float2 v) { return cf32{v.x, v.y}; }

// NR: the most receive antennas the scratch holds (H of the subcarrier).
template <int NT, int NS, int NR = 64>
struct DetSharedT {
    cf32 Hs[NR * NT];
    double2 Cg[NT * NT];
    double2 Fs[NS * (NT + 1)];   // rows padded to NT + 1 (lanes read a row each)
    double2 Ls[NT * (NT + 1)];  // the inverse of Cg + sigma^2 I (with Cg as its second buffer)
};

template <int NT, int NS, int NR>
__device__ void build_det_sc(const float2 *H, const float2 *y, int nr, int nt, int nsym, int sc,
                             int sym0, int ns, int ld, int ldf, int qtop, double c, double c2,
                             double noise_var, float *Gout, float *fout, signed char *xout,
                             double *ynorm, DetSharedT<NT, NS, NR> &sh, int tid)
{
    const int nthr = blockDim.x;
    const int K = 2 * nt;
    constexpr int LD = NT + 1;          // row stride of Fs and Ls

    const float2 *Hg = H + (size_t)sc * nr * nt;
    for (int e = tid; e < nr * nt; e += nthr) sh.Hs[e] = to_cf32(Hg[e]);
    // The symbols' y go to LDS too when they fit in the inverse's buffer (not
    // used before the factorisation), so that the matrix-core loop below reads
    // no global memory; else it reads y where it needs it.
    cf32 *Ys = reinterpret_cast<cf32 *>(sh.Ls);
    const bool y_lds = NT <= 16 && ns * nr <= (int)(sizeof(sh.Ls) / sizeof(cf32));
    if (y_lds) {
        const float2 *yg = y + ((size_t)sc * nsym + sym0) * nr;
        for (int e = tid; e < ns * nr; e += nthr) Ys[e] = to_cf32(yg[e]);
    }
    __syncthreads();

    for (int e = tid; e < ld * ld; e += nthr) {
        const int r = e / ld, cc = e % ld;
        if (r >= K || cc >= K) Gout[e] = 0.0f;
    }
    // Gram X + iY = H^H H and fields F = H^H y on the matrix cores.  With the
    // stacked real rows A = [Re H; Im H] (2 nr x nt):
    //   X = A^T A,  Y = A^T [Im H; -Re H],
    //   Re F = A^T [Re y; Im y],  Im F = A^T [Im y; -Re y],
    // as 16 x 16 float64 tiles of v_mfma_f64_16x16x4f64 (inner dimension 2 nr in
    // steps of 4), one tile per wavefront in turn: tile 0 -> X, tile 1 -> Y,
    // tile 2 + c -> symbols 8c .. 8c+7 (Re F in columns 0..7, Im F in 8..15).
    // Products of float32 values are exact in float64, so the result differs
    // from a plain float64 loop only by summation order.
    // Operand layout of the instruction: lane l supplies A[l % 16][l / 16] and
    // B[l / 16][l % 16] and receives D[l / 16 + 4 j][l % 16], j = 0..3.
    if constexpr (NT > 16) {
        // more than 16 users: plain float64 sums over the receive antennas
        // (products of float32 values are exact in float64)
        double *Cgd = reinterpret_cast<double *>(sh.Cg);
        double *Fsd = reinterpret_cast<double *>(sh.Fs);
        for (int e = tid; e < nt * nt; e += nthr) {
            const int i = e / nt, j = e % nt;
            double re = 0.0, im = 0.0;
            for (int r = 0; r < nr; ++r) {
                const cf32 hi = sh.Hs[r * nt + i], hj = sh.Hs[r * nt + j];
                re = re + ((double)hi.x * hj.x + (double)hi.y * hj.y);
                im = im + ((double)hi.x * hj.y - (double)hi.y * hj.x);
            }
            Cgd[2 * (i * NT + j)] = re;
            Cgd[2 * (i * NT + j) + 1] = im;
        }
        for (int e = tid; e < ns * nt; e += nthr) {
            const int s0 = e / nt, i = e % nt;
            const float2 *ys = y + ((size_t)sc * nsym + sym0 + s0) * nr;
            double re = 0.0, im = 0.0;
            for (int r = 0; r < nr; ++r) {
                const cf32 h = sh.Hs[r * nt + i];
                const float2 yv = ys[r];
                re = re + ((double)h.x * yv.x + (double)h.y * yv.y);
                im = im + ((double)h.x * yv.y - (double)h.y * yv.x);
            }
            Fsd[2 * (s0 * LD + i)] = re;
            Fsd[2 * (s0 * LD + i) + 1] = im;
        }
    } else
    {
        const int wave = tid >> 6, lane = tid & 63, nwave = nthr >> 6;
        const int lrow = lane & 15, lk = lane >> 4;
        const int n_inner = 2 * nr, ksteps = (n_inner + 3) / 4;
        const int ntiles = 2 + (ns + 7) / 8;
        double *Cgd = reinterpret_cast<double *>(sh.Cg);
        double *Fsd = reinterpret_cast<double *>(sh.Fs);
        for (int t = wave; t < ntiles; t += nwave) {
            mfma_v4d acc = {0.0, 0.0, 0.0, 0.0};
            const int s_col = (t - 2) * 8 + (lrow & 7);     // symbol of this lane's column
#pragma unroll 4
            for (int ks = 0; ks < ksteps; ++ks) {
                const int r2 = ks * 4 + lk;
                const bool top = r2 < nr;
                const int rr = top ? r2 : r2 - nr;
                double a = 0.0, b = 0.0;
                if (r2 < n_inner) {
                    if (lrow < nt) {
                        const cf32 h = sh.Hs[rr * nt + lrow];
                        a = top ? (double)h.x : (double)h.y;
                        if (t == 0) b = a;
                        else if (t == 1) b = top ? (double)h.y : -(double)h.x;
                    }
                    if (t >= 2 && s_col < ns) {
                        const cf32 yv = y_lds ? Ys[s_col * nr + rr]
                                              : to_cf32(y[((size_t)sc * nsym + sym0 + s_col) * nr + rr]);
                        if (lrow < 8) b = top ? (double)yv.x : (double)yv.y;
                        else b = top ? (double)yv.y : -(double)yv.x;
                    }
                }
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
            }
            for (int j = 0; j < 4; ++j) {
                const int row = lk + 4 * j;
                if (row >= nt) continue;
                if (t < 2) {
                    if (lrow < nt) Cgd[2 * (row * NT + lrow) + t] = acc[j];
                } else if (s_col < ns) {
                    Fsd[2 * (s_col * LD + row) + (lrow >= 8 ? 1 : 0)] = acc[j];
                }
            }
        }
    }
    __syncthreads();

    // exactly Hermitian: the upper triangle, mirrored, real diagonal
    const int npair = nt * (nt + 1) / 2;
    for (int p = tid; p < npair; p += nthr) {
        int ia, ib;
        upper_pair(p, nt, ia, ib);
        const double2 v = sh.Cg[ia * NT + ib];
        const double re = v.x;
        const double im = ia == ib ? 0.0 : v.y;
        sh.Cg[ia * NT + ib] = make_double2(re, im);
        sh.Cg[ib * NT + ia] = make_double2(re, 0.0 - im);
        const float gre = (float)(c2 * re);
        const float gim = (float)(c2 * im);
        const float ngim = (float)(c2 * (0.0 - im));
        Gout[ia * ld + ib] = gre;
        Gout[ib * ld + ia] = gre;
        Gout[(nt + ia) * ld + (nt + ib)] = gre;
        Gout[(nt + ib) * ld + (nt + ia)] = gre;
        // upper-right block -Im Cg, lower-left block Im Cg
        Gout[ia * ld + (nt + ib)] = ngim;
        Gout[(nt + ib) * ld + ia] = ngim;
        Gout[(nt + ia) * ld + ib] = gim;
        Gout[ib * ld + (nt + ia)] = gim;
    }
    for (int p = tid; p < ns * nt; p += nthr) {
        const int r0 = p / nt, ia = p % nt;
        const double2 F = sh.Fs[r0 * LD + ia];
        float *fs = fout + (size_t)r0 * ldf;
        fs[ia] = (float)(c * F.x);
        fs[nt + ia] = (float)(c * F.y);
    }
    for (int p = tid; p < ns * (ld - K); p += nthr) {
        const int r0 = p / (ld - K), k = K + p % (ld - K);
        fout[(size_t)r0 * ldf + k] = 0.0f;
    }
    if (ynorm) {
        for (int r0 = tid; r0 < ns; r0 += nthr) {
            const float2 *ys = y + ((size_t)sc * nsym + sym0 + r0) * nr;
            double acc = 0.0;
            for (int r = 0; r < nr; ++r) {
                const double yr = ys[r].x, yi = ys[r].y;
                acc = acc + (yr * yr + yi * yi);
            }
            ynorm[r0] = acc;
        }
    }
    if (!xout) return;   // uniform over the block
    __syncthreads();
    // The inverse is a chain of dependent float64 pivot steps on at most 16
    // rows: the first wavefront does it alone, synchronising through LDS at
    // wavefront level instead of across the block.
    if (tid >= 64) return;

    // (Cg + sigma^2 I)^-1 by Gauss-Jordan (Hermitian positive definite: no
    // pivoting), each pivot step reading one LDS buffer and writing the other
    // (Ls and Cg, rows of NT), so that no element is held in registers across
    // the step's synchronisation
    // (element (i, j) of the NT x NT frame is e = i NT + j, lane e mod 64:
    // compile-time shifts, no integer division in the pivot loop)
    double2 *src = sh.Ls, *dst = sh.Cg;
    for (int e = tid; e < NT * NT; e += 64) {
        const int i = e / NT, j = e % NT;
        if (i >= nt || j >= nt) continue;
        double2 v = sh.Cg[i * NT + j];
        if (i == j) v.x = v.x + noise_var;
        src[i * NT + j] = v;
    }
    wave_sync_lds();
    // Each pivot step reads every operand of this lane's elements first (one
    // round of independent LDS loads), then computes and stores; groups of four
    // elements per lane (all of them for NT <= 16).
    constexpr int kEpl = (NT * NT + 63) / 64;
    constexpr int kGrp = kEpl < 4 ? kEpl : 4;
    for (int k = 0; k < nt; ++k) {
        const cd pk = ld2(src[k * NT + k]);
        const double den = pk.re * pk.re + pk.im * pk.im;
        const cd t{pk.re / den, -pk.im / den};
#pragma unroll 1
        for (int m0 = 0; m0 < kEpl; m0 += kGrp) {
            cd rowk[kGrp], colk[kGrp], old[kGrp];
#pragma unroll
            for (int u = 0; u < kGrp; ++u) {
                const int e = tid + 64 * (m0 + u);
                const int i = e / NT, j = e % NT;
                rowk[u] = cd{0.0, 0.0};
                colk[u] = cd{0.0, 0.0};
                old[u] = cd{0.0, 0.0};
                if (e < NT * NT && i < nt && j < nt) {
                    rowk[u] = ld2(src[k * NT + j]);
                    colk[u] = ld2(src[i * NT + k]);
                    old[u] = ld2(src[i * NT + j]);
                }
            }
#pragma unroll
            for (int u = 0; u < kGrp; ++u) {
                const int e = tid + 64 * (m0 + u);
                const int i = e / NT, j = e % NT;
                if (e >= NT * NT || i >= nt || j >= nt) continue;
                const cd rowv = j == k ? t : cmul(rowk[u], t);
                if (i == k) {
                    dst[i * NT + j] = st2(rowv);
                } else {
                    const cd o = j == k ? cd{0.0, 0.0} : old[u];
                    const cd m = cmul(colk[u], rowv);
                    dst[i * NT + j] = make_double2(o.re - m.re, o.im - m.im);
                }
            }
        }
        wave_sync_lds();
        double2 *tmp = src;
        src = dst;
        dst = tmp;
    }
    const double2 *Ai = src;
    // x = A^-1 F per symbol, one (symbol, user) pair per lane, then slicing
    for (int e = tid; e < ns * NT; e += 64) {
        const int r0 = e / NT, i = e % NT;
        if (i >= nt) continue;
        const double2 *w = sh.Fs + r0 * LD;
        cd acc{0.0, 0.0};
#pragma unroll
        for (int j = 0; j < NT; ++j) {
            if (j >= nt) break;
            const cd v = cmul(ld2(Ai[i * NT + j]), ld2(w[j]));
            acc.re = acc.re + v.re;
            acc.im = acc.im + v.im;
        }
        const double tr = acc.re / c, ti = acc.im / c;
        double lr = 2.0 * floor(tr / 2.0) + 1.0;
        double li = 2.0 * floor(ti / 2.0) + 1.0;
        lr = fmin(fmax(lr, (double)-qtop), (double)qtop);
        li = fmin(fmax(li, (double)-qtop), (double)qtop);
        if (lr != lr) lr = 1.0;   // NaN input: any valid level
        if (li != li) li = 1.0;
        signed char *xo = xout + (size_t)r0 * ld;
        xo[i] = (signed char)(int)lr;
        xo[nt + i] = (signed char)(int)li;
    }
    for (int e = tid; e < ns * (ld - K); e += 64) {
        const int r0 = e / (ld - K), k = K + e % (ld - K);
        xout[(size_t)r0 * ld + k] = 0;
    }
}

// ---------------------------------------------------------------------------
// VPP build of one subcarrier.  A = H H^H, its LDL^H, M = L^-1 and
// A^-1 = M^H D^-1 M in a fixed operation order (so that any implementation of
// the same sequence agrees bit for bit), then
//   G = (tau/2)^2 Re-form(A^-1),  f = -(tau/2) Re-form(A^-1 u).
template <int NU>
struct VppSharedT {
    cf32 Hs[NU * 64];
    double2 As[NU * NU];
    double2 Ls[NU * NU];
    double2 Ms[NU * NU];
    double2 Zs[NU * NU];   // A^-1
    double ds[NU];
};

template <int NU>
__device__ void build_vpp_sc(const float2 *H, const float2 *u, int n, int ntx, int nsym, int sc,
                             int sym0, int ns, int ld, int ldf, double tau, float *Gout, float *fout,
                             signed char *xout, double2 *Ainv_out, double *unorm, VppSharedT<NU> &sh,
                             int tid)
{
    const int nthr = blockDim.x;
    const int K = 2 * n;
    const double ht = 0.5 * tau;
    const double sg = ht * ht;
    const double sf = -ht;

    const float2 *Hg = H + (size_t)sc * n * ntx;
    for (int e = tid; e < n * ntx; e += nthr) sh.Hs[e] = to_cf32(Hg[e]);
    __syncthreads();

    // A_il = sum_j H_ij conj(H_lj), i >= l
    const int npair = n * (n + 1) / 2;
    for (int p = tid; p < npair; p += nthr) {
        int l, i;
        upper_pair(p, n, l, i);   // l <= i
        double re = 0.0, im = 0.0;
        for (int j = 0; j < ntx; ++j) {
            const double ar = sh.Hs[i * ntx + j].x, ai = sh.Hs[i * ntx + j].y;
            const double cr = sh.Hs[l * ntx + j].x, ci = sh.Hs[l * ntx + j].y;
            const double pre = ar * cr + ai * ci;
            const double pim = ai * cr - ar * ci;
            re = re + pre;
            im = im + pim;
        }
        sh.As[i * NU + l] = make_double2(re, im);
        sh.As[l * NU + i] = make_double2(re, -im);
    }
    __syncthreads();

    // LDL^H and M = L^-1: chains of dependent float64 steps on at most 16
    // rows, done by the first wavefront alone with wavefront-level
    // synchronisation through LDS
    if (tid < 64) {
        for (int j = 0; j < n; ++j) {
            if (tid == 0) {
                double dj = sh.As[j * NU + j].x;
                for (int k = 0; k < j; ++k) {
                    const double2 v = sh.Ls[j * NU + k];
                    double t = v.x * v.x + v.y * v.y;
                    t = t * sh.ds[k];
                    dj = dj - t;
                }
                sh.ds[j] = dj;
            }
            wave_sync_lds();
            for (int i = j + 1 + tid; i < n; i += 64) {
                cd s = ld2(sh.As[i * NU + j]);
                for (int k = 0; k < j; ++k) {
                    cd v = cmulc(ld2(sh.Ls[j * NU + k]), ld2(sh.Ls[i * NU + k]));
                    v.re = v.re * sh.ds[k];
                    v.im = v.im * sh.ds[k];
                    s.re = s.re - v.re;
                    s.im = s.im - v.im;
                }
                sh.Ls[i * NU + j] = make_double2(s.re / sh.ds[j], s.im / sh.ds[j]);
            }
            wave_sync_lds();
        }
        // M = L^-1, one column per lane
        for (int m = tid; m < n; m += 64) {
            sh.Ms[m * NU + m] = make_double2(1.0, 0.0);
            for (int i = m + 1; i < n; ++i) {
                cd s{0.0, 0.0};
                for (int k = m; k < i; ++k) {
                    const cd v = cmul(ld2(sh.Ls[i * NU + k]), ld2(sh.Ms[k * NU + m]));
                    s.re = s.re + v.re;
                    s.im = s.im + v.im;
                }
                sh.Ms[i * NU + m] = make_double2(-s.re, -s.im);
            }
        }
    }
    __syncthreads();
    // A^-1_il = sum_{k>=i} conj(M_ki) M_kl / d_k, i >= l
    for (int p = tid; p < npair; p += nthr) {
        int l, i;
        upper_pair(p, n, l, i);
        cd acc{0.0, 0.0};
        for (int k = i; k < n; ++k) {
            cd v = cmulc(ld2(sh.Ms[k * NU + i]), ld2(sh.Ms[k * NU + l]));
            v.re = v.re / sh.ds[k];
            v.im = v.im / sh.ds[k];
            acc.re = acc.re + v.re;
            acc.im = acc.im + v.im;
        }
        sh.Zs[i * NU + l] = st2(acc);
        if (i != l) sh.Zs[l * NU + i] = make_double2(acc.re, -acc.im);
        else sh.Zs[i * NU + i] = make_double2(acc.re, -acc.im);
    }
    __syncthreads();

    if (Ainv_out) {
        for (int e = tid; e < n * n; e += nthr) Ainv_out[e] = sh.Zs[(e / n) * NU + (e % n)];
    }
    for (int e = tid; e < ld * ld; e += nthr) {
        const int r = e / ld, cc = e % ld;
        float v = 0.0f;
        if (r < K && cc < K) {
            const int i = r % n, l = cc % n;
            const double2 z = sh.Zs[i * NU + l];
            if ((r < n) == (cc < n)) v = (float)(sg * z.x);
            else if (r < n) v = (float)(sg * (-z.y));   // upper-right: -Im
            else v = (float)(sg * z.y);                 // lower-left: Im
        }
        Gout[e] = v;
    }
    for (int p = tid; p < ns * n; p += nthr) {
        const int r0 = p / n, i = p % n;
        const float2 *us = u + ((size_t)sc * nsym + sym0 + r0) * n;
        cd z{0.0, 0.0};
        for (int l = 0; l < n; ++l) {
            const cd ul{(double)us[l].x, (double)us[l].y};
            const cd v = cmul(ld2(sh.Zs[i * NU + l]), ul);
            z.re = z.re + v.re;
            z.im = z.im + v.im;
        }
        float *fs = fout + (size_t)r0 * ldf;
        fs[i] = (float)(sf * z.re);
        fs[n + i] = (float)(sf * z.im);
    }
    for (int p = tid; p < ns * (ld - K); p += nthr) {
        const int r0 = p / (ld - K), k = K + p % (ld - K);
        fout[(size_t)r0 * ldf + k] = 0.0f;
    }
    if (xout) {
        for (int p = tid; p < ns * ld; p += nthr) xout[p] = 0;
    }
    if (unorm) {
        for (int r0 = tid; r0 < ns; r0 += nthr) {
            const float2 *us = u + ((size_t)sc * nsym + sym0 + r0) * n;
            double acc = 0.0;
            for (int i = 0; i < n; ++i) {
                cd z{0.0, 0.0};
                for (int l = 0; l < n; ++l) {
                    const cd v = cmul(ld2(sh.Zs[i * NU + l]), cd{(double)us[l].x, (double)us[l].y});
                    z.re = z.re + v.re;
                    z.im = z.im + v.im;
                }
                acc = acc + ((double)us[i].x * z.re + (double)us[i].y * z.im);
            }
            unorm[r0] = acc;
        }
    }
}

// Field entry f_k of this lane's instance: through the scalar cache when the
// instance is wave-uniform, else a vector load whose address is re-derived at
// each use (so that the compiler keeps no row of f in registers); FLDS: the
// row is in LDS (a per-lane LDS address, read with an LDS load).
template <bool PACKED, bool FLDS = false>
__device__ __forceinline__ float load_field(const float *fi, int k)
{
    if constexpr (FLDS) {
        typedef __attribute__((address_space(3))) const float lds_float;
        lds_float *p = (lds_float *)fi;
        asm volatile("" : "+v"(p));
        return p[k];
    } else if constexpr (PACKED) {
        const float *p = fi;
        asm volatile("" : "+v"(p));
        return p[k];
    } else {
        return opaque(fi)[k];
    }
}

// ---------------------------------------------------------------------------
// The anneal of one lane.  G of the instance is wave-uniform: the caller stages
// it in LDS (Gl, KT x KT floats, rows 16-byte aligned) and each row is read
// when the sweep reaches its dimension with 128-bit loads that every lane of
// the wavefront takes from the same address, so the row lands in vector
// registers (products with vector operands issue faster than with scalar
// ones).  f is read through the scalar cache unless several instances share
// the wavefront (PACKED: f per lane, by vector loads).  Per lane the state is the
// flip step of every spin, d_i = -2 w_b s_i (+-2w_b as float) -- or one bit per
// spin (set = spin -1) for large problems, to keep enough wavefronts resident --
// and the levels x[KT]; the local field of a dimension is recomputed from the
// levels when the sweep reaches it (one row of G x - f) and moved by G_kk d
// after an accepted flip inside the dimension.
//
// Per attempt on spin i = k Q + b with h = g_k + (d/2) G_kk:
//   2h = (g_k + g_k) + d G_kk exactly, and 64 beta2 dE = (128 beta2 d) h,
//   the Metropolis threshold index is floor(64 beta2 dE) clamped to [0, 1024],
//   and the flip is accepted iff the 16-bit draw m < T[index] (T in LDS).
// Returns the final energy sum_k x_k (g_k - f_k); `bits` receives the final
// spins (bit set = spin -1).
// Energy sum_k x_k (g_k - f_k) of levels x with fresh fields g = G x - f (G in
// LDS, rows of KT floats), every field a chain of fused multiply-adds from -f_k.
template <int KT>
__device__ __forceinline__ float lane_level_energy(const float *Gl, const float *fi,
                                                   const float (&x)[KT])
{
    float E = 0.0f;
    if constexpr (KT > 32) {
        // Rows in chunks of 8 floats. Each chunk's loads wait for the previous
        // chunk's products (a row's first chunk for the previous row's energy
        // term) through a zero produced from that value, so that the unrolled
        // loop keeps one chunk in flight and the kernel stays within 128
        // registers; the sums are the same chains as below.
#pragma unroll
        for (int k = 0; k < KT; ++k) {
            float acc = -fi[k];
#pragma unroll
            for (int c0 = 0; c0 < KT; c0 += 8) {
                int cz;
                asm volatile("v_mov_b32 %0, 0" : "=v"(cz) : "v"(c0 == 0 ? E : acc));
                const float4 *Gc = reinterpret_cast<const float4 *>(Gl) + cz;
                const float4 v0 = Gc[(k * KT + c0) / 4], v1 = Gc[(k * KT + c0) / 4 + 1];
                const float gr[8] = {v0.x, v0.y, v0.z, v0.w, v1.x, v1.y, v1.z, v1.w};
#pragma unroll
                for (int l = 0; l < 8; ++l) acc = fmaf(gr[l], x[c0 + l], acc);
            }
            const float diff = acc - fi[k];
            E = fmaf(x[k], diff, E);
        }
    } else {
#pragma unroll
        for (int k = 0; k < KT; ++k) {
            float acc = -fi[k];
#pragma unroll
            for (int l = 0; l < KT; ++l) acc = fmaf(Gl[k * KT + l], x[l], acc);
            const float diff = acc - fi[k];
            E = fmaf(x[k], diff, E);
        }
    }
    return E;
}

template <int KT, int Q, bool PACKED = false, bool FLDS = false>
__device__ __forceinline__ float anneal_lane(const float *Gl, const float *fi,
                                             const signed char *xfb_i, const float *beta2,
                                             const uint32_t *T, int sweeps, const int (&wts)[4],
                                             uint32_t key0, uint32_t key1, int init_mode,
                                             uint32_t uch, uint32_t uinst,
                                             uint32_t (&bits)[(KT * Q + 31) / 32])
{
    constexpr int N = KT * Q;
    constexpr int NW = (N + 31) / 32;
    constexpr int NG = (N + 7) / 8;
    constexpr bool kBits = N > 48 || KT >= 32;
    constexpr int ND = kBits ? 1 : N;
    constexpr int NB = kBits ? NW : 1;

    float two_w[Q];
#pragma unroll
    for (int b = 0; b < Q; ++b) two_w[b] = (float)(2 * wts[b]);

    float dv[ND];
    uint32_t sb[NB];
#pragma unroll
    for (int w = 0; w < NB; ++w) sb[w] = 0u;
    auto set_spin = [&](int i, bool negative) {
        if constexpr (kBits) {
            if (negative) sb[i >> 5] |= 1u << (i & 31);
        } else {
            dv[i] = negative ? two_w[i % Q] : -two_w[i % Q];
        }
    };
    if (init_mode == 1 && xfb_i != nullptr) {
#pragma unroll
        for (int k = 0; k < KT; ++k) {
            int rem = xfb_i[k];
#pragma unroll
            for (int b = 0; b < Q; ++b) {
                const int sg = rem > 0 ? 1 : -1;
                rem -= wts[b] * sg;
                set_spin(k * Q + b, sg < 0);
            }
        }
    } else {
#pragma unroll
        for (int j = 0; j < NG; ++j) {
            uint32_t r[4] = {(uint32_t)j, 0xFFFFFFFFu, uch, uinst};
            philox4x32_10(r, key0, key1);
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int i = 8 * j + e;
                if (i < N) {
                    const uint32_t d = (e & 1) ? (r[e >> 1] >> 16) : (r[e >> 1] & 0xFFFFu);
                    set_spin(i, (d & 0x8000u) != 0u);   // spin -1 -> d = +2w
                }
            }
        }
    }
    auto step_of = [&](int i) -> float {
        if constexpr (kBits) {
            uint32_t wd = sb[i >> 5];
            // 64 dimensions: the word is read where the spin is tried, so that
            // the steps of a sweep are not all decoded (into 128 registers) at
            // its start
            if constexpr (KT > 32) asm volatile("" : "+v"(wd));
            return ((wd >> (i & 31)) & 1u) ? two_w[i % Q] : -two_w[i % Q];
        } else {
            return dv[i];
        }
    };
    float x[KT];
#pragma unroll
    for (int k = 0; k < KT; ++k) {
        float lv = 0.0f;
#pragma unroll
        for (int b = 0; b < Q; ++b) lv = lv - 0.5f * step_of(k * Q + b);   // w_b s = -d/2, exact
        x[k] = lv;
    }

    for (int t = 0; t < sweeps; ++t) {
        // the schedule through the scalar cache (wave-uniform)
        const float bd = 128.0f * opaque(beta2)[t];    // exact: power-of-two scale
        uint32_t r[4] = {0u, 0u, 0u, 0u};
        // a row offset the optimiser cannot see through, so that the row loads
        // stay inside the sweep instead of being hoisted into registers
        int roff = 0;
        asm volatile("" : "+v"(roff));
        const float4 *G4 = reinterpret_cast<const float4 *>(Gl) + roff;
#pragma unroll
        for (int k = 0; k < KT; ++k) {
            const float fk = load_field<PACKED, FLDS>(fi, k);
            // local field of dimension k from the current levels; PACKED reads
            // the row in chunks of 8 floats, each issued after the previous
            // chunk's products (the per-lane field loads leave fewer registers)
            constexpr int kChunk = PACKED ? 8 : KT > 32 ? 16 : KT;
            float g = -fk;
            float gkk = 0.0f;
#pragma unroll
            for (int c0 = 0; c0 < KT; c0 += kChunk) {
                int coff = k * (KT / 4) + c0 / 4;
                const float4 *Gc = G4;
                if constexpr (KT > 32) {
                    // a zero made from g: the row offset stays a constant the
                    // loads carry as their immediate (no register per chunk)
                    if (c0 > 0) {
                        int cz;
                        asm volatile("v_mov_b32 %0, 0" : "=v"(cz) : "v"(g));
                        Gc = G4 + cz;
                    }
                } else if (c0 > 0) {
                    asm volatile("" : "+v"(coff) : "v"(g));
                }
                float grow[kChunk];
#pragma unroll
                for (int l4 = 0; l4 < kChunk / 4; ++l4) {
                    const float4 v = Gc[coff + l4];
                    grow[4 * l4 + 0] = v.x;
                    grow[4 * l4 + 1] = v.y;
                    grow[4 * l4 + 2] = v.z;
                    grow[4 * l4 + 3] = v.w;
                }
#pragma unroll
                for (int l = 0; l < kChunk; ++l) {
                    g = fmaf(grow[l], x[c0 + l], g);
                    if (c0 + l == k) gkk = grow[l];
                }
            }
            const float gkh = 0.5f * gkk;                  // exact
#pragma unroll
            for (int b = 0; b < Q; ++b) {
                const int i = k * Q + b;
                if ((i & 7) == 0) {
                    r[0] = (uint32_t)(i >> 3);
                    r[1] = (uint32_t)t;
                    r[2] = uch;
                    r[3] = uinst;
                    philox4x32_10(r, opaque_u32(key0), opaque_u32(key1));
                }
                const int e = i & 7;
                const uint32_t m = (e & 1) ? (r[e >> 1] >> 16) : (r[e >> 1] & 0xFFFFu);
                const float d = step_of(i);
                const float h = fmaf(d, gkh, g);                      // g + (d/2) G_kk
                const float zs = (d * bd) * h;                        // 64 beta2 dE
                const float zc = fminf(fmaxf(zs, 0.0f), (float)kAcceptSteps);
                const uint32_t idx = (uint32_t)zc;
                const bool acc = m < T[idx];
                const float da = acc ? d : 0.0f;
                x[k] = x[k] + da;
                g = fmaf(gkk, da, g);
                if constexpr (kBits) {
                    sb[i >> 5] ^= acc ? (1u << (i & 31)) : 0u;
                } else {
                    dv[i] = acc ? -d : d;
                }
            }
        }
    }

    // the spin words first (the flip steps die here), then the energy
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        uint32_t word = 0u;
        if constexpr (kBits) {
            word = sb[w];
        } else {
#pragma unroll
            for (int bit = 0; bit < 32; ++bit) {
                const int i = 32 * w + bit;
                if (i < N && dv[i] > 0.0f) word |= 1u << bit;   // d > 0 <=> spin -1
            }
        }
        bits[w] = word;
    }
    return lane_level_energy<KT>(Gl, fi, x);
}


// One CIM-CAC anneal per lane (paper §2.3 Eqs. cim1/cim2, Euler steps as in
// §3.2 and Appendix A).  Per lane: the amplitudes and error variables of the
// KT Q spins and of one auxiliary spin carrying the field (index KT Q), and the
// held coupling terms.  The coupling terms go through the structured form --
// levels X_l = sum_b w_b x_(l,b), one row g_k of G X per dimension (G from LDS
// as in anneal_lane), then per spin (-2 w_b)(g_k - G_kk w_b x_i) + 2 w_b f_k x_a
// -- and are recomputed every f_mvm steps.  Padded dimensions have zero
// couplings and fields, so they never reach a real spin.  Returns the energy of
// the final spins sign(x_i) sign(x_a); `bits` receives them (bit set = -1).
template <int KT, int Q, bool PACKED>
__device__ __forceinline__ float cim_lane(const float *Gl, const float *fi,
                                          const signed char *xfb_i, const CimParams &P,
                                          int steps, const int (&wts)[4], uint32_t key0,
                                          uint32_t key1, int init_mode, uint32_t uch,
                                          uint32_t uinst, uint32_t (&bits)[(KT * Q + 31) / 32],
                                          int n_real, bool &diverged)
{
    constexpr int N = KT * Q;
    constexpr int NW = (N + 31) / 32;
    constexpr int NG = (N + 7) / 8;
    float amp[N + 1], err[N + 1], cpl[N + 1];
    float wf[Q];
#pragma unroll
    for (int b = 0; b < Q; ++b) wf[b] = (float)wts[b];
    // the model constants in vector registers: products with vector operands
    // issue faster than with scalar ones
    float dt = P.dt, pm1 = P.pm1, ca0 = P.a, nz = P.nzeta, eps = P.eps;
    asm volatile("" : "+v"(dt), "+v"(pm1), "+v"(ca0), "+v"(nz), "+v"(eps));
    const float inv = 1.0f / 32768.0f;                   // exact
    if (init_mode == 1 && xfb_i != nullptr) {
#pragma unroll
        for (int k = 0; k < KT; ++k) {
            int rem = xfb_i[k];
#pragma unroll
            for (int b = 0; b < Q; ++b) {
                const int sg = rem > 0 ? 1 : -1;
                rem -= wts[b] * sg;
                amp[k * Q + b] = P.amp0 * (float)sg;
            }
        }
        amp[N] = P.amp0;
    } else {
#pragma unroll
        for (int j = 0; j < NG; ++j) {
            uint32_t r[4] = {(uint32_t)j, 0xFFFFFFFFu, uch, uinst};
            philox4x32_10(r, key0, key1);
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int i = 8 * j + e;
                if (i < N) {
                    const uint32_t d = (e & 1) ? (r[e >> 1] >> 16) : (r[e >> 1] & 0xFFFFu);
                    amp[i] = P.amp0 * ((float)((int)d - 32768) * inv);
                }
            }
        }
        uint32_t r[4] = {0x1FFFFFFFu, 0xFFFFFFFFu, uch, uinst};   // draw 0xfffffff8
        philox4x32_10(r, key0, key1);
        amp[N] = P.amp0 * ((float)((int)(r[0] & 0xFFFFu) - 32768) * inv);
    }
#pragma unroll
    for (int i = 0; i <= N; ++i) {
        err[i] = 1.0f;
        cpl[i] = 0.0f;
    }
    const float efloor = 1.0f / 1048576.0f;             // 2^-20
    const int fm = P.f_mvm;
    for (int t = 0; t < steps; ++t) {
        if (t % fm == 0) {
            float X[KT];
#pragma unroll
            for (int l = 0; l < KT; ++l) {
                float v = 0.0f;
#pragma unroll
                for (int b = 0; b < Q; ++b) v = fmaf(wf[b], amp[l * Q + b], v);
                X[l] = v;
            }
            const float xa = amp[N];
            float acc_a = 0.0f;
            int roff = 0;
            asm volatile("" : "+v"(roff));
            const float4 *G4 = reinterpret_cast<const float4 *>(Gl) + roff;
#pragma unroll
            for (int k = 0; k < KT; ++k) {
                float g = 0.0f;
                float gkk = 0.0f;
#pragma unroll
                for (int l4 = 0; l4 < KT / 4; ++l4) {
                    const float4 v = G4[k * (KT / 4) + l4];
                    const float cv[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        g = fmaf(cv[u], X[4 * l4 + u], g);
                        if (4 * l4 + u == k) gkk = cv[u];
                    }
                }
                const float fk = load_field<PACKED>(fi, k);
#pragma unroll
                for (int b = 0; b < Q; ++b) {
                    const int i = k * Q + b;
                    const float self = gkk * (wf[b] * amp[i]);
                    const float inner = g - self;
                    const float t1 = (-2.0f * wf[b]) * inner;
                    const float t2 = ((2.0f * wf[b]) * fk) * xa;
                    cpl[i] = t1 + t2;
                }
                acc_a = fmaf(2.0f * fk, X[k], acc_a);
            }
            cpl[N] = acc_a;
        }
#pragma unroll
        for (int i = 0; i <= N; ++i) {
            const float x = amp[i], e = err[i];
            const float s2 = x * x;
            const float lin = pm1 * x;
            const float cub = s2 * x;
            const float drift = lin - cub;
            const float gain = eps * e;
            const float push = gain * cpl[i];
            const float dx = drift + push;
            const float stp = dt * dx;
            const float t1 = s2 - ca0;
            const float t2 = t1 * e;
            const float de = nz * t2;
            const float estp = dt * de;
            const float en = e + estp;
            amp[i] = x + stp;
            err[i] = en > efloor ? en : efloor;
        }
    }
    // diverged: an amplitude of a real spin or of the auxiliary one beyond the
    // bound or not finite, or such an error variable not finite
    bool div = false;
#pragma unroll
    for (int i = 0; i <= N; ++i) {
        if (i < n_real || i == N)
            div = div || !(fabsf(amp[i]) <= kCimDivergeBound) || !(fabsf(err[i]) <= FLT_MAX);
    }
    diverged = div;
    const bool aneg = amp[N] < 0.0f;
    float x[KT];
#pragma unroll
    for (int w = 0; w < NW; ++w) bits[w] = 0u;
#pragma unroll
    for (int k = 0; k < KT; ++k) {
        int lv = 0;
#pragma unroll
        for (int b = 0; b < Q; ++b) {
            const int i = k * Q + b;
            const bool neg = (amp[i] < 0.0f) != aneg;
            lv += neg ? -wts[b] : wts[b];
            bits[i >> 5] |= neg ? (1u << (i & 31)) : 0u;
        }
        x[k] = (float)lv;
    }
    return lane_level_energy<KT>(Gl, fi, x);
}

// One CIM-CAC anneal per pair of lanes, for 33 to 64 spins (the paper's
// 16-user move problem has 64 spins and the auxiliary one): lane h of the pair
// (h = lane & 1) holds the amplitudes, error variables and held coupling terms
// of dimensions h KT/2 .. (h + 1) KT/2 - 1 (NH = KT Q / 2 spins) and a copy of
// the auxiliary spin's.  At each coupling refresh the pair swaps its levels
// (one cross-lane move per level), so that each lane forms the rows g_k of its
// own dimensions over all KT levels and the auxiliary term over all KT fields,
// in the order of cim_lane; both lanes then hold the same auxiliary values.
// Every spin's update is cim_lane's, so the anneal is the same to the bit.
// Returns the energy of the final spins (both lanes); `bits` receives all
// spin words (both lanes) and `diverged` the flag over all spins.
template <int KT, int Q, bool PACKED>
__device__ __forceinline__ float cim_lane2(const float *Gl, const float *fi,
                                           const signed char *xfb_i, const CimParams &P,
                                           int steps, const int (&wts)[4], uint32_t key0,
                                           uint32_t key1, int init_mode, uint32_t uch,
                                           uint32_t uinst, uint32_t (&bits)[(KT * Q + 31) / 32],
                                           int n_real, bool &diverged, int h)
{
    constexpr int N = KT * Q;
    constexpr int NW = (N + 31) / 32;
    constexpr int KH = KT / 2;                 // dimensions of this lane
    constexpr int NH = KH * Q;                 // spins of this lane
    static_assert(NH % 8 == 0, "whole Philox blocks per lane");
    float amp[NH + 1], err[NH + 1], cpl[NH + 1];
    float wf[Q];
#pragma unroll
    for (int b = 0; b < Q; ++b) wf[b] = (float)wts[b];
    float dt = P.dt, pm1 = P.pm1, ca0 = P.a, nz = P.nzeta, eps = P.eps;
    asm volatile("" : "+v"(dt), "+v"(pm1), "+v"(ca0), "+v"(nz), "+v"(eps));
    const float inv = 1.0f / 32768.0f;                   // exact
    const int k0 = h * KH;                               // first dimension of this lane
    if (init_mode == 1 && xfb_i != nullptr) {
#pragma unroll
        for (int kl = 0; kl < KH; ++kl) {
            int rem = xfb_i[k0 + kl];
#pragma unroll
            for (int b = 0; b < Q; ++b) {
                const int sg = rem > 0 ? 1 : -1;
                rem -= wts[b] * sg;
                amp[kl * Q + b] = P.amp0 * (float)sg;
            }
        }
        amp[NH] = P.amp0;
    } else {
#pragma unroll
        for (int jj = 0; jj < NH / 8; ++jj) {
            // spin i = h NH + 8 jj + e takes draw i: block i / 8, half-word i % 8
            uint32_t r[4] = {(uint32_t)(h * (NH / 8) + jj), 0xFFFFFFFFu, uch, uinst};
            philox4x32_10(r, key0, key1);
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const uint32_t d = (e & 1) ? (r[e >> 1] >> 16) : (r[e >> 1] & 0xFFFFu);
                amp[8 * jj + e] = P.amp0 * ((float)((int)d - 32768) * inv);
            }
        }
        uint32_t r[4] = {0x1FFFFFFFu, 0xFFFFFFFFu, uch, uinst};   // draw 0xfffffff8
        philox4x32_10(r, key0, key1);
        amp[NH] = P.amp0 * ((float)((int)(r[0] & 0xFFFFu) - 32768) * inv);
    }
#pragma unroll
    for (int i = 0; i <= NH; ++i) {
        err[i] = 1.0f;
        cpl[i] = 0.0f;
    }
    const float efloor = 1.0f / 1048576.0f;             // 2^-20
    const int fm = P.f_mvm;
    for (int t = 0; t < steps; ++t) {
        if (t % fm == 0) {
            // the levels of all KT dimensions: this lane's and its partner's
            float X[KT];
#pragma unroll
            for (int kl = 0; kl < KH; ++kl) {
                float v = 0.0f;
#pragma unroll
                for (int b = 0; b < Q; ++b) v = fmaf(wf[b], amp[kl * Q + b], v);
                const float o = __shfl_xor(v, 1, 64);
                X[kl] = h ? o : v;
                X[KH + kl] = h ? v : o;
            }
            const float xa = amp[NH];
            float acc_a = 0.0f;
#pragma unroll
            for (int k = 0; k < KT; ++k) acc_a = fmaf(2.0f * load_field<PACKED>(fi, k), X[k], acc_a);
            int roff = k0 * (KT / 4);
            asm volatile("" : "+v"(roff));
            const float4 *G4 = reinterpret_cast<const float4 *>(Gl) + roff;
#pragma unroll
            for (int kl = 0; kl < KH; ++kl) {
                float g = 0.0f;
#pragma unroll
                for (int l4 = 0; l4 < KT / 4; ++l4) {
                    const float4 v = G4[kl * (KT / 4) + l4];
                    g = fmaf(v.x, X[4 * l4 + 0], g);
                    g = fmaf(v.y, X[4 * l4 + 1], g);
                    g = fmaf(v.z, X[4 * l4 + 2], g);
                    g = fmaf(v.w, X[4 * l4 + 3], g);
                }
                const int k = k0 + kl;
                const float gkk = Gl[k * KT + k];
                const float fk = load_field<PACKED>(fi, k);
#pragma unroll
                for (int b = 0; b < Q; ++b) {
                    const int i = kl * Q + b;
                    const float self = gkk * (wf[b] * amp[i]);
                    const float inner = g - self;
                    const float t1 = (-2.0f * wf[b]) * inner;
                    const float t2 = ((2.0f * wf[b]) * fk) * xa;
                    cpl[i] = t1 + t2;
                }
            }
            cpl[NH] = acc_a;
        }
#pragma unroll
        for (int i = 0; i <= NH; ++i) {
            const float x = amp[i], e = err[i];
            const float s2 = x * x;
            const float lin = pm1 * x;
            const float cub = s2 * x;
            const float drift = lin - cub;
            const float gain = eps * e;
            const float push = gain * cpl[i];
            const float dx = drift + push;
            const float stp = dt * dx;
            const float t1 = s2 - ca0;
            const float t2 = t1 * e;
            const float de = nz * t2;
            const float estp = dt * de;
            const float en = e + estp;
            amp[i] = x + stp;
            err[i] = en > efloor ? en : efloor;
        }
    }
    bool div = !(fabsf(amp[NH]) <= kCimDivergeBound) || !(fabsf(err[NH]) <= FLT_MAX);
#pragma unroll
    for (int il = 0; il < NH; ++il) {
        if (h * NH + il < n_real)
            div = div || !(fabsf(amp[il]) <= kCimDivergeBound) || !(fabsf(err[il]) <= FLT_MAX);
    }
    diverged = div || __shfl_xor(div ? 1 : 0, 1, 64) != 0;
    const bool aneg = amp[NH] < 0.0f;
    uint32_t own[NW];
#pragma unroll
    for (int w = 0; w < NW; ++w) own[w] = 0u;
    float x[KT];
#pragma unroll
    for (int kl = 0; kl < KH; ++kl) {
        int lv = 0;
#pragma unroll
        for (int b = 0; b < Q; ++b) {
            const int il = kl * Q + b;
            const bool neg = (amp[il] < 0.0f) != aneg;
            lv += neg ? -wts[b] : wts[b];
            // global spin h NH + il: word and bit for either half
            const int i0 = il, i1 = NH + il;
            const uint32_t m = neg ? 1u : 0u;
#pragma unroll
            for (int w = 0; w < NW; ++w) {
                const uint32_t b0 = (i0 >> 5) == w ? m << (i0 & 31) : 0u;
                const uint32_t b1 = (i1 >> 5) == w ? m << (i1 & 31) : 0u;
                own[w] |= h ? b1 : b0;
            }
        }
        const float v = (float)lv;
        const float o = __shfl_xor(v, 1, 64);
        x[kl] = h ? o : v;
        x[KH + kl] = h ? v : o;
    }
#pragma unroll
    for (int w = 0; w < NW; ++w) bits[w] = own[w] | __shfl_xor(own[w], 1, 64);
    return lane_level_energy<KT>(Gl, fi, x);
}

// CIM-CAC anneals of 33 to 64 spins, one per pair of lanes (cim_lane2): PACKED
// 64 / gl2 instances per wavefront with gl2 lanes each (gl2 / 2 anneals), or
// 32 anneals of one instance per wavefront (several wavefronts for more).
// Outputs as k_cim.
template <int KT, int Q, bool PACKED>
__global__ void __launch_bounds__(kBlock)
k_cim2(const float *__restrict__ G, int inst_per_G, const float *__restrict__ f,
       const signed char *__restrict__ x_fb, CimParams prm, int steps, int chains, int n_inst,
       int w0, int w1, int w2, int w3, uint32_t key0, uint32_t key1, uint32_t inst_base,
       int init_mode, int gl2, float *__restrict__ chain_E, uint32_t *__restrict__ chain_S,
       unsigned char *__restrict__ chain_div, int n_real)
{
    constexpr int NW = (KT * Q + 31) / 32;
    __shared__ float4 Gw[kWavesPerBlock][KT * KT / 4];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int gw = blockIdx.x * kWavesPerBlock + wave;
    int inst, ch, inst0;
    bool valid = true;
    if constexpr (PACKED) {
        const int per_wave = 64 / gl2;
        inst0 = gw * per_wave;
        if (inst0 >= n_inst) return;
        inst = inst0 + lane / gl2;
        ch = (lane % gl2) >> 1;
        if (inst >= n_inst) {               // tail of the last wavefront: any valid data
            valid = false;
            inst = inst0;
        }
    } else {
        const int wpi = (chains + 31) >> 5;
        inst = gw / wpi;
        if (inst >= n_inst) return;
        inst0 = inst;
        ch = (gw - inst * wpi) * 32 + (lane >> 1);
    }
    const float *Gi = G + (size_t)(inst0 / inst_per_G) * (KT * KT);
    float *Gs = reinterpret_cast<float *>(Gw[wave]);
    for (int e = lane; e < KT * KT; e += 64) Gs[e] = Gi[e];
    wave_sync_lds();
    const float *fi = f + (size_t)inst * KT;
    const signed char *xi = x_fb ? x_fb + (size_t)inst * KT : nullptr;
    const int wts[4] = {w0, w1, w2, w3};
    uint32_t bits[NW];
    bool div;
    uint32_t ginst = (uint32_t)inst + inst_base;
    asm volatile("" : "+v"(ginst));
    const float E = cim_lane2<KT, Q, PACKED>(Gs, fi, xi, prm, steps, wts, key0, key1, init_mode,
                                             (uint32_t)ch, ginst, bits, n_real, div, lane & 1);
    if (valid && ch < chains && (lane & 1) == 0) {
        const size_t o = (size_t)(ginst - inst_base) * chains + ch;
        chain_E[o] = E;
#pragma unroll
        for (int w = 0; w < NW; ++w) chain_S[o * NW + w] = bits[w];
        if (chain_div) chain_div[o] = div ? 1 : 0;
    }
}

// ---------------------------------------------------------------------------
// Selection helpers.
__device__ __forceinline__ uint32_t energy_key(float e)
{
    if (e != e) return 0xFFFFFFFFu;            // NaN after everything
    uint32_t u = __float_as_uint(e);
    if (e == 0.0f) u = 0u;                      // -0 ranks as +0
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ bool energy_less(float a, float b)
{
    if (a != a) return false;
    if (b != b) return true;
    return a < b;
}

__device__ __forceinline__ uint64_t wave_min_u64(uint64_t v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const uint32_t lo = __shfl_xor((uint32_t)v, off, 64);
        const uint32_t hi = __shfl_xor((uint32_t)(v >> 32), off, 64);
        const uint64_t o = ((uint64_t)hi << 32) | lo;
        v = o < v ? o : v;
    }
    return v;
}
__device__ __forceinline__ double wave_sum_f64(double v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Exchanges inside 16-lane rows by DPP (no LDS round trip): CTRL 0xB1 swaps
// neighbours (quad_perm 1,0,3,2), 0x4E swaps lane pairs (quad_perm 2,3,0,1),
// 0x141 mirrors each 8 lanes (lane i <-> 7 - i) and 0x140 each 16 (i <-> 15 - i).
// Applied in that order, each step pairs a lane with one in the other half of
// its 2-, 4-, 8- and 16-lane group, so a commutative combine leaves the same
// value, to the bit, in every lane of the group.
template <int CTRL>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ __forceinline__ uint64_t dpp_u64(uint64_t v)
{
    return ((uint64_t)dpp_u32<CTRL>((uint32_t)(v >> 32)) << 32) | dpp_u32<CTRL>((uint32_t)v);
}
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v)
{
    return __longlong_as_double((long long)dpp_u64<CTRL>((uint64_t)__double_as_longlong(v)));
}
// Sum over aligned groups of g lanes (g a power of two, 1..64), the same in
// every lane of a group (the whole wavefront takes part).
__device__ __forceinline__ double group_sum_f64(double v, int g)
{
    if (g >= 2) v = v + dpp_f64<0xB1>(v);
    if (g >= 4) v = v + dpp_f64<0x4E>(v);
    if (g >= 8) v = v + dpp_f64<0x141>(v);
    if (g >= 16) v = v + dpp_f64<0x140>(v);
    for (int off = 16; off < g; off <<= 1) v = v + __shfl_xor(v, off, 64);
    return v;
}
// Minimum over aligned groups of g lanes (as above).
__device__ __forceinline__ uint64_t group_min_u64(uint64_t v, int g)
{
    uint64_t o;
    if (g >= 2) { o = dpp_u64<0xB1>(v); v = o < v ? o : v; }
    if (g >= 4) { o = dpp_u64<0x4E>(v); v = o < v ? o : v; }
    if (g >= 8) { o = dpp_u64<0x141>(v); v = o < v ? o : v; }
    if (g >= 16) { o = dpp_u64<0x140>(v); v = o < v ? o : v; }
    for (int off = 16; off < g; off <<= 1) {
        const uint32_t lo = __shfl_xor((uint32_t)v, off, 64);
        const uint32_t hi = __shfl_xor((uint32_t)(v >> 32), off, 64);
        o = ((uint64_t)hi << 32) | lo;
        v = o < v ? o : v;
    }
    return v;
}
__device__ __forceinline__ double group_min_f64(double v, int g)
{
    if (g >= 2) v = fmin(v, dpp_f64<0xB1>(v));
    if (g >= 4) v = fmin(v, dpp_f64<0x4E>(v));
    if (g >= 8) v = fmin(v, dpp_f64<0x141>(v));
    if (g >= 16) v = fmin(v, dpp_f64<0x140>(v));
    for (int off = 16; off < g; off <<= 1) v = fmin(v, __shfl_xor(v, off, 64));
    return v;
}

// Energy of the fallback levels with the chains' arithmetic (one wavefront;
// `terms` is this wavefront's LDS scratch of 32 floats).
template <bool TR = false>
__device__ float fallback_energy(const float *Gi, int ldg, int K, const float *fi,
                                 const signed char *xi, float *terms, int lane)
{
    if (lane < K) {
        float acc = -fi[lane];
#pragma unroll 8
        for (int l = 0; l < K; ++l)
            acc = fmaf(TR ? Gi[l * ldg + lane] : Gi[lane * ldg + l], (float)xi[l], acc);
        terms[lane] = acc - fi[lane];
    }
    wave_sync_lds();
    float e = 0.0f;
#pragma unroll 8
    for (int k = 0; k < K; ++k) e = fmaf((float)xi[k], terms[k], e);
    wave_sync_lds();
    return e;
}

// Energy of levels lv (this wavefront's LDS copy, K entries) with the chains'
// arithmetic (one wavefront; `terms` its LDS scratch of 32 floats).
template <bool TR = false>
__device__ float wave_level_energy(const float *Gi, int ldg, int K, const float *fi, const int *lv,
                                   float *terms, int lane)
{
    if (lane < K) {
        float acc = -fi[lane];
#pragma unroll 8
        for (int l = 0; l < K; ++l)
            acc = fmaf(TR ? Gi[l * ldg + lane] : Gi[lane * ldg + l], (float)lv[l], acc);
        terms[lane] = acc - fi[lane];
    }
    wave_sync_lds();
    float e = 0.0f;
#pragma unroll 8
    for (int k = 0; k < K; ++k) e = fmaf((float)lv[k], terms[k], e);
    wave_sync_lds();
    return e;
}

// Applies an instance's winning move (lv: the move levels z in {-2, 0, 2}, this
// wavefront's LDS copy) to its guess xg (a device row of levels): the candidate
// clamp(xg + z, -qtop, qtop) replaces the guess iff its energy with the full
// fields ff is strictly lower.  lv then holds the guess.  cand: LDS scratch of
// 32 ints.
template <bool TR = false>
__device__ void apply_move(int *lv, signed char *xg, const float *Gi, int ldg, int K,
                           const float *ff, int qtop, int *cand, float *terms, int lane)
{
    if (lane < K) {
        const int v = (int)xg[lane] + lv[lane];
        cand[lane] = v < -qtop ? -qtop : (v > qtop ? qtop : v);
        lv[lane] = (int)xg[lane];
    }
    wave_sync_lds();
    const float Ec = wave_level_energy<TR>(Gi, ldg, K, ff, cand, terms, lane);
    const float Eg = wave_level_energy<TR>(Gi, ldg, K, ff, lv, terms, lane);
    if (Ec < Eg && lane < K) {
        xg[lane] = (signed char)cand[lane];
        lv[lane] = cand[lane];
    }
    wave_sync_lds();
}

// Levels of the winning candidate into lv[0..K): the fallback's, or those of
// the spin words S (bit set = spin -1).
__device__ void winning_levels(bool use_fb, const signed char *xi, const uint32_t *S, int K, int q,
                               const int *w, int *lv, int lane)
{
    if (lane < K) {
        int v;
        if (use_fb) {
            v = xi[lane];
        } else {
            v = 0;
            for (int b = 0; b < q; ++b) {
                const int i = lane * q + b;
                v += ((S[i >> 5] >> (i & 31)) & 1u) ? -w[b] : w[b];
            }
        }
        lv[lane] = v;
    }
    wave_sync_lds();
}

// Decode of the winning levels (lv: this wavefront's LDS copy of K levels).
// Hsc: H of the instance's subcarrier, [nr][nt] (device memory or an LDS copy).
__device__ void decode_det(const int *lv, int n, int sc, int sy, int nsym, int nr, int nt, int q,
                           double c, const float2 *Hsc, const float2 *y, unsigned char *sym_out,
                           float *metric_out, int lane)
{
    const int qtop = (1 << q) - 1;
    if (lane < nt) {
        const int pI = (lv[lane] + qtop) >> 1;
        const int pQ = (lv[nt + lane] + qtop) >> 1;
        const int gI = pI ^ (pI >> 1), gQ = pQ ^ (pQ >> 1);
        sym_out[(size_t)n * nt + lane] = (unsigned char)((gI << q) | gQ);
    }
    if (metric_out) {
        double part = 0.0;
        for (int r = lane; r < nr; r += 64) {
            const float2 *Hr = Hsc + (size_t)r * nt;
            const float2 yv = y[((size_t)sc * nsym + sy) * nr + r];
            double re = yv.x, im = yv.y;
#pragma unroll 8
            for (int t = 0; t < nt; ++t) {
                const double xr = c * (double)lv[t];
                const double xi = c * (double)lv[nt + t];
                const double hr = Hr[t].x, hi = Hr[t].y;
                re = re - (hr * xr - hi * xi);
                im = im - (hr * xi + hi * xr);
            }
            part = part + (re * re + im * im);
        }
        const double tot = wave_sum_f64(part);
        if (lane == 0) metric_out[n] = (float)tot;
    }
}

// VPP: v = level / 2; x = H^H A^-1 (u + tau v); gamma = ||x||^2.  Z: A^-1 of
// the subcarrier with row stride ldz; Hsc: its H, [nu][ntx] (device memory or
// LDS copies).  zsh: this wavefront's LDS scratch of 16 double2.
__device__ void decode_vpp(const int *lv, int n, int sc, int sy, int nsym, int nu, int ntx,
                           double tau, const double2 *Z, int ldz, const float2 *Hsc,
                           const float2 *u,
                           signed char *v_out, float2 *x_out, float *gamma_out, double2 *zsh,
                           int lane)
{
    const int K = 2 * nu;
    if (lane < K) v_out[(size_t)n * K + lane] = (signed char)(lv[lane] / 2);
    if (!x_out && !gamma_out) return;
    const float2 *us = u + ((size_t)sc * nsym + sy) * nu;
    if (lane < nu) {
        double zr = 0.0, zi = 0.0;
        for (int l = 0; l < nu; ++l) {
            const double pr = (double)us[l].x + tau * (double)(lv[l] / 2);
            const double pi = (double)us[l].y + tau * (double)(lv[nu + l] / 2);
            const double2 zz = Z[lane * ldz + l];
            zr = zr + (zz.x * pr - zz.y * pi);
            zi = zi + (zz.x * pi + zz.y * pr);
        }
        zsh[lane] = make_double2(zr, zi);
    }
    wave_sync_lds();
    double part = 0.0;
    for (int j = lane; j < ntx; j += 64) {
        double xr = 0.0, xi = 0.0;
        for (int i = 0; i < nu; ++i) {
            const float2 h = Hsc[(size_t)i * ntx + j];
            const double2 z = zsh[i];
            // conj(H_ij) z_i
            xr = xr + ((double)h.x * z.x + (double)h.y * z.y);
            xi = xi + ((double)h.x * z.y - (double)h.y * z.x);
        }
        if (x_out) x_out[(size_t)n * ntx + j] = make_float2((float)xr, (float)xi);
        part = part + (xr * xr + xi * xi);
    }
    const double tot = wave_sum_f64(part);
    if (lane == 0 && gamma_out) gamma_out[n] = (float)tot;
    wave_sync_lds();
}

// ---------------------------------------------------------------------------
// Plain path kernels.
// One wavefront per subcarrier, scratch sized for the problem (NT, NU = 8 or
// 16) and symbols taken 16 at a time: the build is a chain of dependent
// steps, so it pays to have every subcarrier in flight at once rather than
// more threads on each.
constexpr int kBuildBlock = 64;
constexpr int kBuildSyms = 16;

template <int NT, int NR>
__global__ void __launch_bounds__(kBuildBlock) k_det_build(DetBuildArgs a)
{
    // H in LDS for at most NR receive antennas: a smaller frame keeps more
    // subcarriers resident per CU (each is a chain of dependent steps)
    __shared__ DetSharedT<NT, kBuildSyms, NR> sh;
    const int sc = blockIdx.x;
    for (int s0 = 0; s0 < a.n_sym; s0 += kBuildSyms) {
        if (s0 > 0) __syncthreads();
        const int cnt = min(kBuildSyms, a.n_sym - s0);
        const size_t o = (size_t)sc * a.n_sym + s0;
        build_det_sc(a.H, a.y, a.n_r, a.n_t, a.n_sym, sc, s0, cnt, a.ld, a.ld, a.qtop, a.c, a.c2,
                     a.noise_var, a.G + (size_t)sc * a.ld * a.ld, a.f + o * a.ld,
                     a.x_fb ? a.x_fb + o * a.ld : nullptr, a.ynorm ? a.ynorm + o : nullptr, sh,
                     (int)threadIdx.x);
    }
}

template <int NU>
__global__ void __launch_bounds__(kBuildBlock) k_vpp_build(VppBuildArgs a)
{
    __shared__ VppSharedT<NU> sh;
    const int sc = blockIdx.x;
    for (int s0 = 0; s0 < a.n_sym; s0 += kBuildSyms) {
        if (s0 > 0) __syncthreads();
        const int cnt = min(kBuildSyms, a.n_sym - s0);
        const size_t o = (size_t)sc * a.n_sym + s0;
        build_vpp_sc(a.H, a.u, a.n_u, a.n_t, a.n_sym, sc, s0, cnt, a.ld, a.ld, a.tau,
                     a.G + (size_t)sc * a.ld * a.ld, a.f + o * a.ld,
                     a.x_fb ? a.x_fb + o * a.ld : nullptr,
                     a.Ainv ? a.Ainv + (size_t)sc * a.n_u * a.n_u : nullptr,
                     a.unorm ? a.unorm + o : nullptr, sh, (int)threadIdx.x);
    }
}

// One wavefront = 64 chains of one instance; chains > 64 use several
// wavefronts.  PACKED: one wavefront = 64 / glanes instances of glanes lanes
// each (glanes a power of two >= chains, <= 32), all sharing one G -- the host
// guarantees that 64 / glanes divides inst_per_G.  Each wavefront stages its
// G in LDS; with 64 dimensions (16 KB per G) the workgroup instead stages each
// distinct G of its wavefronts once, in g_slots dynamic LDS slots, so that
// four wavefronts per SIMD fit.  Writes every chain's final energy and spin
// words.
template <int KT, int Q, bool PACKED>
constexpr int anneal_min_waves()
{
    return KT <= 8 ? 8 : KT == 16 ? (Q == 3 ? 4 : 6) : KT == 32 ? (Q == 1 || PACKED ? 5 : 4)
                                                                 : (PACKED ? 2 : 4);
}
template <int KT, int Q, bool PACKED>
__global__ void __launch_bounds__(kBlock)
    __attribute__((amdgpu_waves_per_eu(anneal_min_waves<KT, Q, PACKED>(), 8)))
k_anneal(const float *__restrict__ G, int inst_per_G, const float *__restrict__ f,
         const signed char *__restrict__ x_fb, const float *__restrict__ beta2,
         const uint32_t *__restrict__ accept_table, int sweeps, int chains, int n_inst, int w0,
         int w1, int w2, int w3, uint32_t key0, uint32_t key1, uint32_t inst_base,
         int init_mode, int glanes, int g_slots, float *__restrict__ chain_E,
         uint32_t *__restrict__ chain_S)
{
    constexpr int NW = (KT * Q + 31) / 32;
    constexpr bool kSharedG = KT > 32;
    __shared__ uint32_t T[kAcceptSteps + 1];
    // each wavefront's copy of its G (fewer than 64 dimensions)
    __shared__ float4 Gw[kSharedG ? 1 : kWavesPerBlock][kSharedG ? 1 : KT * KT / 4];
    // 64 dimensions: g_slots copies, 16-byte aligned for the 128-bit row loads
    extern __shared__ float4 anneal_gdyn4[];
    float *anneal_gdyn = reinterpret_cast<float *>(anneal_gdyn4);
    for (int e = threadIdx.x; e <= kAcceptSteps; e += kBlock) T[e] = accept_table[e];

    // the first instance of wavefront w and whether it has work
    const int per_wave = PACKED ? 64 / glanes : 1;
    const int wpi = PACKED ? 1 : (chains + 63) >> 6;
    auto first_inst = [&](int w) { return PACKED ? w * per_wave : w / wpi; };
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    // 64 dimensions: the several workgroups of one subcarrier on one XCD, so
    // that its couplings come from HBM once
    const int blk = kSharedG ? xcd_block((int)blockIdx.x, (int)gridDim.x) : (int)blockIdx.x;
    const int gw = blk * kWavesPerBlock + wave;
    int slot = 0;
    if constexpr (kSharedG) {
        // G ids of the block's wavefronts are non-decreasing: stage ids
        // g0 .. g1 (the last wavefront with work), at most g_slots of them
        const int gw0 = blk * kWavesPerBlock;
        const int g0 = first_inst(gw0) / inst_per_G;
        int g1 = g0;
        for (int w = 1; w < kWavesPerBlock; ++w) {
            const int i0 = first_inst(gw0 + w);
            if (i0 < n_inst) g1 = i0 / inst_per_G;
        }
        const int ns = min(g1 - g0 + 1, g_slots);
        const float *Gb = G + (size_t)g0 * (KT * KT);
        for (int e = threadIdx.x; e < ns * KT * KT; e += kBlock) anneal_gdyn[e] = Gb[e];
        slot = __builtin_amdgcn_readfirstlane(first_inst(gw) / inst_per_G - g0);
    }
    __syncthreads();

    int inst, ch, inst0;
    bool valid = true;
    if constexpr (PACKED) {
        inst0 = gw * per_wave;
        if (inst0 >= n_inst) return;
        inst = inst0 + lane / glanes;
        ch = lane % glanes;
        if (inst >= n_inst) {               // tail of the last wavefront: any valid data
            valid = false;
            inst = inst0;
        }
    } else {
        inst = gw / wpi;
        if (inst >= n_inst) return;
        inst0 = inst;
        ch = (gw - inst * wpi) * 64 + lane;
    }
    float *Gs;
    if constexpr (kSharedG) {
        if (slot >= g_slots) return;        // the launcher's slot count covers every block
        Gs = anneal_gdyn + (size_t)slot * (KT * KT);
    } else {
        const float *Gi = G + (size_t)(inst0 / inst_per_G) * (KT * KT);
        Gs = reinterpret_cast<float *>(Gw[wave]);
        for (int e = lane; e < KT * KT; e += 64) Gs[e] = Gi[e];
        wave_sync_lds();
    }
    const float *fi = f + (size_t)inst * KT;
    const signed char *xi = x_fb ? x_fb + (size_t)inst * KT : nullptr;
    const int wts[4] = {w0, w1, w2, w3};
    uint32_t bits[NW];
    // the Philox instance index is the only instance value kept across the
    // anneal (hidden from the optimiser); the output row is re-derived from it
    uint32_t ginst = (uint32_t)inst + inst_base;
    asm volatile("" : "+v"(ginst));
    const float E = anneal_lane<KT, Q, PACKED>(Gs, fi, xi, beta2, T, sweeps, wts, key0, key1,
                                               init_mode, (uint32_t)ch, ginst, bits);
    if (valid && ch < chains) {
        const size_t o = (size_t)(ginst - inst_base) * chains + ch;
        chain_E[o] = E;
#pragma unroll
        for (int w = 0; w < NW; ++w) chain_S[o * NW + w] = bits[w];
    }
}

// CIM-CAC anneals with the layout of k_anneal: one wavefront = 64 chains of
// one instance (several wavefronts for more chains), or PACKED 64 / glanes
// instances per wavefront sharing one G; each wavefront stages its G in LDS.
// Writes every chain's final energy and spin words.
template <int KT, int Q, bool PACKED>
__global__ void __launch_bounds__(kBlock)
k_cim(const float *__restrict__ G, int inst_per_G, const float *__restrict__ f,
      const signed char *__restrict__ x_fb, CimParams prm, int steps, int chains, int n_inst,
      int w0, int w1, int w2, int w3, uint32_t key0, uint32_t key1, uint32_t inst_base,
      int init_mode, int glanes, float *__restrict__ chain_E, uint32_t *__restrict__ chain_S,
      unsigned char *__restrict__ chain_div, int n_real)
{
    constexpr int NW = (KT * Q + 31) / 32;
    __shared__ float4 Gw[kWavesPerBlock][KT * KT / 4];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int gw = blockIdx.x * kWavesPerBlock + wave;
    int inst, ch, inst0;
    bool valid = true;
    if constexpr (PACKED) {
        const int per_wave = 64 / glanes;
        inst0 = gw * per_wave;
        if (inst0 >= n_inst) return;
        inst = inst0 + lane / glanes;
        ch = lane % glanes;
        if (inst >= n_inst) {               // tail of the last wavefront: any valid data
            valid = false;
            inst = inst0;
        }
    } else {
        const int wpi = (chains + 63) >> 6;
        inst = gw / wpi;
        if (inst >= n_inst) return;
        inst0 = inst;
        ch = (gw - inst * wpi) * 64 + lane;
    }
    const float *Gi = G + (size_t)(inst0 / inst_per_G) * (KT * KT);
    float *Gs = reinterpret_cast<float *>(Gw[wave]);
    for (int e = lane; e < KT * KT; e += 64) Gs[e] = Gi[e];
    wave_sync_lds();
    const float *fi = f + (size_t)inst * KT;
    const signed char *xi = x_fb ? x_fb + (size_t)inst * KT : nullptr;
    const int wts[4] = {w0, w1, w2, w3};
    uint32_t bits[NW];
    bool div;
    uint32_t ginst = (uint32_t)inst + inst_base;
    asm volatile("" : "+v"(ginst));
    const float E = cim_lane<KT, Q, PACKED>(Gs, fi, xi, prm, steps, wts, key0, key1, init_mode,
                                            (uint32_t)ch, ginst, bits, n_real, div);
    if (valid && ch < chains) {
        const size_t o = (size_t)(ginst - inst_base) * chains + ch;
        chain_E[o] = E;
#pragma unroll
        for (int w = 0; w < NW; ++w) chain_S[o * NW + w] = bits[w];
        if (chain_div) chain_div[o] = div ? 1 : 0;
    }
}

// Copies an instance's G (KT x KT floats, KT <= GM) into this wavefront's LDS
// slot with rows of KT + 1 floats, so that lanes reading one row each hit
// distinct banks; the loads of each batch of 16 are issued before its stores.
template <int GM>
__device__ __forceinline__ void copy_g_to_lds(float *Gl, const float *Gg, int KT, int lane)
{
    const int n = KT * KT;
#pragma unroll
    for (int j0 = 0; j0 < (GM * GM + 63) / 64; j0 += 16) {
        float v[16];
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const int e = lane + 64 * (j0 + j);
            v[j] = e < n ? Gg[e] : 0.0f;
        }
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const int e = lane + 64 * (j0 + j);
            if (e < n) Gl[(e / KT) * (KT + 1) + e % KT] = v[j];
        }
    }
    wave_sync_lds();
}

// GM: the largest padded dimension count KT the instantiation serves.
template <int GM>
__global__ void __launch_bounds__(kBlock) k_select(SelectArgs a)
{
    __shared__ float terms[kWavesPerBlock][GM];
    __shared__ int lvs[kWavesPerBlock][GM];
    __shared__ double2 zsh[kWavesPerBlock][16];
    __shared__ int cand[kWavesPerBlock][GM];
    __shared__ float Gw[kWavesPerBlock][GM * (GM + 1)];   // each wavefront's copy of its G

    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    // 64 dimensions: the workgroups of one subcarrier on one XCD (its couplings
    // from HBM once)
    const int blk = GM > 32 ? xcd_block((int)blockIdx.x, (int)gridDim.x) : (int)blockIdx.x;
    const int n = blk * kWavesPerBlock + wave;
    if (n >= a.n_inst) return;   // whole wavefront; only wave-level exchange below
    const int C = a.chains, K = a.K, KT = a.KT, q = a.q;
    const int NW = (KT * q + 31) / 32;

    uint64_t best = ~0ull;
    for (int ch = lane; ch < C; ch += 64) {
        const float e = a.chain_E[(size_t)n * C + ch];
        const uint64_t key = ((uint64_t)energy_key(e) << 32) | (uint32_t)ch;
        best = key < best ? key : best;
    }
    best = wave_min_u64(best);
    const int bch = (int)(uint32_t)best;
    const float Eb = a.chain_E[(size_t)n * C + bch];

    const float *Gg = a.G + (size_t)(n / a.inst_per_G) * KT * KT;
    float *Gi = Gw[wave];
    copy_g_to_lds<GM>(Gi, Gg, KT, lane);
    const float *fi = a.f + (size_t)n * KT;
    const signed char *xi = a.x_fb ? a.x_fb + (size_t)n * KT : nullptr;
    bool use_fb = false;
    float Efb = 0.0f;
    if (xi) {
        Efb = fallback_energy(Gi, KT + 1, K, fi, xi, terms[wave], lane);
        use_fb = energy_less(Efb, Eb);
    }
    const uint32_t *S = a.chain_S + ((size_t)n * C + bch) * NW;
    winning_levels(use_fb, xi, S, K, q, a.w, lvs[wave], lane);

    if (a.mode == kSelectSolve) {
        const int N = K * q;
        for (int i = lane; i < N; i += 64) {
            const int k = i / q, b = i % q;
            int s;
            if (use_fb) {
                int rem = lvs[wave][k];
                s = 1;
                for (int bb = 0; bb <= b; ++bb) {
                    s = rem > 0 ? 1 : -1;
                    rem -= a.w[bb] * s;
                }
            } else {
                s = ((S[i >> 5] >> (i & 31)) & 1u) ? -1 : 1;
            }
            a.spins_out[(size_t)n * N + i] = (signed char)s;
        }
        if (lane == 0) {
            a.e_out[n] = use_fb ? Efb : Eb;
            if (a.win_out) a.win_out[n] = use_fb ? C : bch;
        }
        return;
    }
    const int sc = n / a.n_sym, sy = n % a.n_sym;
    if (a.mode == kSelectDelta) {
        apply_move(lvs[wave], a.guess + (size_t)n * KT, Gi, KT + 1, K, a.f_full + (size_t)n * KT,
                   a.qtop, cand[wave], terms[wave], lane);
        if (!a.decode) return;
        decode_det(lvs[wave], n, sc, sy, a.n_sym, a.n_rows, a.n_cols, a.dq, a.c,
                   a.H + (size_t)sc * a.n_rows * a.n_cols, a.y, a.sym_out, a.metric_out, lane);
        return;
    }
    if (a.mode == kSelectDet) {
        decode_det(lvs[wave], n, sc, sy, a.n_sym, a.n_rows, a.n_cols, q, a.c,
                   a.H + (size_t)sc * a.n_rows * a.n_cols, a.y, a.sym_out, a.metric_out, lane);
    } else {
        decode_vpp(lvs[wave], n, sc, sy, a.n_sym, a.n_rows, a.n_cols, a.tau,
                   a.Ainv + (size_t)sc * a.n_rows * a.n_rows, a.n_rows,
                   a.H + (size_t)sc * a.n_rows * a.n_cols, a.y, a.v_out, a.x_out, a.gamma_out,
                   zsh[wave], lane);
    }
}

// ---------------------------------------------------------------------------
// Fused path: persistent launches.  Each workgroup takes work items from a
// device counter; an item is (job, subcarrier, a range of symbols: one per
// 64-chain wavefront, or 64 / glanes per wavefront when packed).  For its item
// the workgroup builds the subcarrier's couplings (into the job's
// per-subcarrier slot; several items of one subcarrier write identical values)
// and the symbols' fields and fallbacks; then each wavefront anneals 64 chains
// of one instance, the chains of an instance are reduced in registers and LDS,
// and the winner's wavefront decodes.  Items come ordered by decreasing cost.
//
// The anneal variants differ in register demand (about 64 VGPRs for KT = 8,
// 73 for KT = 16 with two spins per dimension, up to 128 for the largest), and
// a kernel's register allocation is the maximum over all of its code.  So the
// variants are grouped into three register classes, one persistent kernel each
// with the class's variants inlined, its own queue, its own occupancy target
// and build scratch sized for the problems it takes:
//   class 0: KT = 8 (any q) and KT = 16 with q = 1   <= 64 VGPRs, 8 waves/SIMD
//   class 1: KT = 16, q = 2                          <= 80 VGPRs, 6 waves/SIMD
//   class 2: KT = 16, q = 3 and KT = 32              <= 128 VGPRs, 4 waves/SIMD
constexpr int kFusedBuildSyms = 16;   // symbols per build pass (an item may take several)

// State shared by every class: threshold table, per-wavefront selection and
// decode scratch, the current item.  At namespace scope so that the
// out-of-line variants address it as LDS.
// ---------------------------------------------------------------------------
// Ordered MMSE-SIC of one subcarrier per workgroup of one wavefront.  With
// P = (H_R^H H_R + sigma^2 I)^-1 over the remaining users R, each step takes
// the remaining user i with the smallest Re P_ii (the lowest index among
// equals), its nulling row w = P_i,R H_R^H, and removes i from P by the Schur
// complement P_jl -= P_ji P_il / P_ii.  The ordering and the nulling rows
// depend on H only.  Then the symbols of the subcarrier are detected in
// groups of g = 2^ceil(log2 n_r) lanes, one lane per receive antenna: each
// lane holds one residual entry r_k in registers, the estimate w . r is a
// shuffle reduction over the group, every lane slices it to the nearest odd
// PAM level per real dimension, and subtracts h_ki s_i from its entry.  The
// residual left after the last user is y - H x, whose squared norm is the
// reported metric.  float64 throughout.
//
// Dynamic LDS: H (n_r x n_t complex float32), P (n_t x n_t complex float64),
// the nulling rows W (n_t x n_r complex float64), and the levels of the
// symbols of one pass (64 / g x 2 n_t ints).
__host__ __device__ inline size_t sic_lds_bytes(int nr, int nt)
{
    int g = 1;
    while (g < nr) g <<= 1;
    return (size_t)nr * nt * 8 + (size_t)nt * nt * 16 + (size_t)nt * nr * 16 +
           (size_t)(64 / g) * 2 * nt * 4 + 16 * 4;
}

__device__ __forceinline__ int sic_slice(double x, double rc, int qtop)
{
    // x / c as x times 1 / c (rc); clamped first (no effect on the sliced level)
    // so that the conversion to int stays in range
    const double t = fmin(fmax(x * rc, -(double)(qtop + 2)), (double)(qtop + 2));
    int v = 2 * (int)floor(t * 0.5) + 1;
    return v < -qtop ? -qtop : (v > qtop ? qtop : v);
}

// Ordered MMSE-SIC of one subcarrier by one wavefront (lane 0..63): symbols
// sym0 .. sym0 + ns - 1 of subcarrier sc.  Hs: the subcarrier's H in LDS,
// [nr][nt]; LDS scratch P [nt][nt] and W [nt][nr] (float64 complex), lv
// [spp][2 nt] and order [nt] (int), spp = min(64 / g, spp_cap) symbols per pass
// with g = nr rounded up to a power of two.  Writes the levels (a.levels, row
// stride a.ldl, zero beyond 2 nt), and if asked the symbols, residual metrics
// and the detection order, all indexed by the slot's instance sc n_sym + sym.
__device__ void sic_sc(const SicArgs &a, int sc, int sym0, int ns, const cf32 *Hs, double2 *P,
                       double2 *W, int *lv, int *order, int spp_cap, int lane)
{
    const int nr = a.n_r, nt = a.n_t, qtop = (1 << a.q) - 1;
    const double rc = 1.0 / a.c;
    int g = 1;
    while (g < nr) g <<= 1;
    const int spp = min(64 / g, spp_cap);                   // symbols per pass
    // A = H^H H + sigma^2 I
    for (int e = lane; e < nt * nt; e += 64) {
        const int i = e / nt, j = e % nt;
        cd acc{0.0, 0.0};
#pragma unroll 4
        for (int r = 0; r < nr; ++r) {
            const cf32 hi = Hs[r * nt + i], hj = Hs[r * nt + j];
            const cd v = cmulc(cd{hi.x, hi.y}, cd{hj.x, hj.y});   // conj(h_ri) h_rj
            acc.re = acc.re + v.re;
            acc.im = acc.im + v.im;
        }
        if (i == j) acc.re = acc.re + a.noise_var;
        P[e] = make_double2(acc.re, acc.im);
    }
    wave_sync_lds();
    // in-place Gauss-Jordan inverse (Hermitian positive definite: no pivoting);
    // each lane keeps its elements' row and column factors in registers
    for (int k = 0; k < nt; ++k) {
        const cd pk = ld2(P[k * nt + k]);
        const double rden = 1.0 / (pk.re * pk.re + pk.im * pk.im);
        const cd t{pk.re * rden, -pk.im * rden};
        cd rowv[4], colv[4], old[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int e = lane + 64 * u;
            if (e < nt * nt) {
                const int i = e / nt, j = e % nt;
                rowv[u] = j == k ? t : cmul(ld2(P[k * nt + j]), t);
                colv[u] = ld2(P[i * nt + k]);
                old[u] = ld2(P[e]);
            }
        }
        wave_sync_lds();
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int e = lane + 64 * u;
            if (e < nt * nt) {
                const int i = e / nt, j = e % nt;
                if (i == k) {
                    P[e] = make_double2(rowv[u].re, rowv[u].im);
                } else {
                    const cd o = j == k ? cd{0.0, 0.0} : old[u];
                    const cd m = cmul(colv[u], rowv[u]);
                    P[e] = make_double2(o.re - m.re, o.im - m.im);
                }
            }
        }
        wave_sync_lds();
    }
    // ordering, nulling rows and downdates
    uint32_t rem = nt >= 32 ? 0xFFFFFFFFu : ((1u << nt) - 1u);
    for (int step = 0; step < nt; ++step) {
        const bool mine = lane < nt && ((rem >> lane) & 1u);
        const double d = mine ? P[lane * nt + lane].x : __builtin_inf();
        // the candidates sit in lanes 0 .. nt - 1 <= 15: the minimum over the
        // first 16-lane row reaches each of them
        const double m = group_min_f64(d, 16);
        uint64_t ball = __ballot(mine && d == m);
        if (ball == 0) ball = rem;              // no finite diagonal: the lowest remaining user
        const int i = __builtin_amdgcn_readfirstlane(__ffsll((unsigned long long)ball) - 1);
        if (lane == 0) order[step] = i;
        for (int r = lane; r < nr; r += 64) {
            cd acc{0.0, 0.0};
#pragma unroll 4
            for (int j = 0; j < nt; ++j) {
                if (!((rem >> j) & 1u)) continue;
                const cf32 h = Hs[r * nt + j];
                const cd v = cmulc(cd{h.x, h.y}, ld2(P[i * nt + j]));   // P_ij conj(h_rj)
                acc.re = acc.re + v.re;
                acc.im = acc.im + v.im;
            }
            W[step * nr + r] = make_double2(acc.re, acc.im);
        }
        // Schur complement of user i
        const cd piv = ld2(P[i * nt + i]);
        const double rden = 1.0 / (piv.re * piv.re + piv.im * piv.im);
        const cd ip{piv.re * rden, -piv.im * rden};
        const uint32_t keep = rem & ~(1u << i);
        cd nv[4];
        bool upd[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int e = lane + 64 * u;
            upd[u] = false;
            if (e < nt * nt) {
                const int j = e / nt, l = e % nt;
                if (((keep >> j) & 1u) && ((keep >> l) & 1u)) {
                    const cd mm = cmul(cmul(ld2(P[j * nt + i]), ld2(P[i * nt + l])), ip);
                    const cd o = ld2(P[e]);
                    nv[u] = cd{o.re - mm.re, o.im - mm.im};
                    upd[u] = true;
                }
            }
        }
        wave_sync_lds();
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (upd[u]) P[lane + 64 * u] = make_double2(nv[u].re, nv[u].im);
        rem = keep;
        wave_sync_lds();
    }
    if (a.order_out && lane < nt) a.order_out[(size_t)sc * nt + lane] = order[lane];
    // detection: symbol sl = lane / g of the pass, receive antenna r = lane % g
    const int sl = lane / g, r = lane % g;
    for (int s0 = sym0; s0 < sym0 + ns; s0 += spp) {
        const int sy = s0 + sl;
        const bool act = sl < spp && sy < sym0 + ns && r < nr;
        cd res{0.0, 0.0};
        if (act) {
            const float2 v = a.y[((size_t)sc * a.n_sym + sy) * nr + r];
            res = cd{(double)v.x, (double)v.y};
        }
        for (int k = 0; k < nt; ++k) {
            const int i = order[k];
            cd prod{0.0, 0.0};
            if (act) prod = cmul(ld2(W[k * nr + r]), res);
            prod.re = group_sum_f64(prod.re, g);
            prod.im = group_sum_f64(prod.im, g);
            const int li = sic_slice(prod.re, rc, qtop);
            const int lq = sic_slice(prod.im, rc, qtop);
            if (act && r == 0) {
                lv[sl * 2 * nt + i] = li;
                lv[sl * 2 * nt + nt + i] = lq;
            }
            if (act) {
                const cf32 h = Hs[r * nt + i];
                const cd m = cmul(cd{h.x, h.y}, cd{a.c * (double)li, a.c * (double)lq});
                res.re = res.re - m.re;
                res.im = res.im - m.im;
            }
        }
        // metric: the squared norm of the final residual y - H x
        double e2 = act ? res.re * res.re + res.im * res.im : 0.0;
        e2 = group_sum_f64(e2, g);
        wave_sync_lds();
        const int cnt = min(spp, sym0 + ns - s0);
        const size_t n0 = (size_t)sc * a.n_sym + s0;
        if (a.levels) {
            for (int e = lane; e < cnt * a.ldl; e += 64) {
                const int s = e / a.ldl, k = e % a.ldl;
                a.levels[(n0 + s) * a.ldl + k] = (signed char)(k < 2 * nt ? lv[s * 2 * nt + k] : 0);
            }
        }
        if (a.sym_out) {
            for (int e = lane; e < cnt * nt; e += 64) {
                const int s = e / nt, t = e % nt;
                const int pI = (lv[s * 2 * nt + t] + qtop) >> 1;
                const int pQ = (lv[s * 2 * nt + nt + t] + qtop) >> 1;
                const int gI = pI ^ (pI >> 1), gQ = pQ ^ (pQ >> 1);
                a.sym_out[(n0 + s) * nt + t] = (unsigned char)((gI << a.q) | gQ);
            }
            if (a.metric_out && act && r == 0) a.metric_out[n0 + sl] = (float)e2;
        }
        wave_sync_lds();
    }
}

// Instances of one packed work item: four wavefronts of at most 16 instances.
constexpr int kMaxPackedItem = 64;
struct FusedCommon {
    uint32_t T[kAcceptSteps + 1];
    uint64_t keys[kWavesPerBlock];
    float terms[kWavesPerBlock][32];
    int lvs[kWavesPerBlock][32];
    double2 zsh[kWavesPerBlock][16];
    int cand[kWavesPerBlock][32];
    signed char zmove[32];  // the zero move (fallback of detection around a guess)
    int item;               // the current work item, published by thread 0
    // winning anneal of each instance of a packed item (spin words, energy),
    // left by the wavefront that annealed it for the wavefront that decodes it
    uint32_t wbits[kMaxPackedItem][3];
    float wE[kMaxPackedItem];
};
__shared__ FusedCommon g_fc;

// Build scratch per class: detection with n_t <= NTD, VPP with n_u <= NUV,
// sharing one block of LDS (a job is one or the other), and the couplings G of
// the current item (one subcarrier: KT x KT floats, KT <= 2 max(NTD, NUV)),
// which the build writes here and the anneal reads.
template <int NTD, int NUV>
struct FusedBuildShared {
    using Det = DetSharedT<NTD, kFusedBuildSyms>;
    using Vpp = VppSharedT<NUV>;
    static constexpr size_t kBytes = sizeof(Det) > sizeof(Vpp) ? sizeof(Det) : sizeof(Vpp);
    static constexpr int kGT = 2 * (NTD > NUV ? NTD : NUV);
    alignas(16) unsigned char raw[kBytes];
    alignas(16) float G[kGT * kGT];
    __device__ Det &det() { return *reinterpret_cast<Det *>(raw); }
    __device__ Vpp &vpp() { return *reinterpret_cast<Vpp *>(raw); }
};
template <int CLS> struct FusedClassTraits;
template <> struct FusedClassTraits<0> {
    static constexpr int kNTD = 8, kNUV = 4, kMinWaves = 8;
};
template <> struct FusedClassTraits<1> {
    static constexpr int kNTD = 8, kNUV = 8, kMinWaves = 6;
};
template <> struct FusedClassTraits<2> {
    static constexpr int kNTD = 16, kNUV = 16, kMinWaves = 4;
};
// The class of a variant fixes these bounds: KT = 8 means n_t <= 4 (DET) or
// n_u <= 4 (VPP); KT = 16 means n_t, n_u <= 8; KT = 32 means n_t, n_u <= 16.
template <int CLS>
using FusedBuildSharedOf =
    FusedBuildShared<FusedClassTraits<CLS>::kNTD, FusedClassTraits<CLS>::kNUV>;
__shared__ FusedBuildSharedOf<0> g_fb0;
__shared__ FusedBuildSharedOf<1> g_fb1;
__shared__ FusedBuildSharedOf<2> g_fb2;
template <int CLS>
__device__ __forceinline__ auto &fused_build_shared()
{
    if constexpr (CLS == 0) return g_fb0;
    else if constexpr (CLS == 1) return g_fb1;
    else return g_fb2;
}

// Wave-uniform copies of descriptor fields and item coordinates, so that the
// compiler keeps them (and the addresses derived from them) in scalar registers.
template <typename T>
__device__ __forceinline__ T *uniform_ptr(T *p)
{
    const uint64_t v = (uint64_t)p;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return (T *)(((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ int rfl(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ uint32_t rflu(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ double rfld(double v)
{
    const uint64_t b = (uint64_t)__double_as_longlong(v);
    const uint64_t lo = rflu((uint32_t)b), hi = rflu((uint32_t)(b >> 32));
    return __longlong_as_double((long long)((hi << 32) | lo));
}

// Anneal, select and decode of one work item by variant (KT, Q).  Unpacked:
// wavefront w anneals 64 chains of instance w / wpi.  PACKED: wavefront w
// anneals instances w P .. w P + P - 1 of the item, glanes = 64 / P lanes each,
// reduces each group of lanes to its best chain and decodes its instances one
// after another.
// LDS copies of the current work item's subcarrier data, left by its build:
// couplings G (rows of KT floats), H ([n_rows][n_cols]) and, for VPP, A^-1
// (row stride ldz).
struct FusedItemLds {
    const float *G;
    const float2 *H;
    const double2 *Z;
    int ldz;
    int stage;              // stage of a job of moves around a guess
    int chain;              // 0 the chain from the MMSE guess, 1 from the MMSE-SIC guess
};

// Descriptor fields read after the anneal (through a laundered pointer, so
// that they are loaded when needed instead of being held, and spilled, across
// the anneal loop).
struct FusedPost {
    int kind, K, n_rows, n_cols, n_sym, chains, wpi, ldf, stages, dq;
    int w[4];
    double c, tau;
    const float2 *y;
    const float *ffull, *fbase;
    signed char *xbase, *xsic;
    int guesses;
    void *out0, *out1, *out2;
};

__device__ __forceinline__ FusedPost fused_post(const FusedJob *jp_in)
{
    const FusedJob *jp = jp_in;
    asm volatile("" : "+s"(jp));
    FusedPost p;
    p.kind = rfl(jp->kind);
    p.K = rfl(jp->K);
    p.n_rows = rfl(jp->n_rows);
    p.n_cols = rfl(jp->n_cols);
    p.n_sym = rfl(jp->n_sym);
    p.chains = rfl(jp->chains);
    p.wpi = rfl(jp->wpi);
    p.ldf = rfl(jp->ldf);
    p.stages = rfl(jp->stages);
    p.dq = rfl(jp->dq);
    for (int b = 0; b < 4; ++b) p.w[b] = rfl(jp->w[b]);
    p.c = rfld(jp->c);
    p.tau = rfld(jp->tau);
    p.y = uniform_ptr(jp->y);
    p.ffull = uniform_ptr(jp->f);
    p.fbase = p.stages > 0 ? uniform_ptr(jp->fp) : p.ffull;
    p.xbase = uniform_ptr(jp->x_fb);
    p.xsic = uniform_ptr(jp->x_sic);
    p.guesses = rfl(jp->guesses);
    p.out0 = uniform_ptr(jp->out0);
    p.out1 = uniform_ptr(jp->out1);
    p.out2 = uniform_ptr(jp->out2);
    return p;
}

template <int KT, int Q, bool PACKED>
__device__ __forceinline__ void fused_anneal(const FusedJob *jobs_in, int job_in, int sc_in,
                                             int sym0_in, int ns_in, const FusedItemLds &lds,
                                             int tid)
{
    const float *Gi = lds.G;
    constexpr int NW = (KT * Q + 31) / 32;
    // the descriptor fields the anneal needs, as wave-uniform (scalar) values
    const FusedJob *jp = uniform_ptr(jobs_in) + rfl(job_in);
    const int sc = rfl(sc_in), sym0 = rfl(sym0_in), ns = rfl(ns_in);
    FusedCommon &sh = g_fc;
    const int wave = rfl(tid >> 6);
    const int lane = tid & 63;
    uint32_t bits[NW];
    float E = 0.0f;
    int w[4];
    {
        const int n_sym = rfl(jp->n_sym), ldf = rfl(jp->ldf), wpi = rfl(jp->wpi);
        const int sweeps = rfl(jp->sweeps), init = rfl(jp->init);
        for (int b = 0; b < 4; ++b) w[b] = rfl(jp->w[b]);
        // moves around a guess (stages > 0): the anneal takes the move fields and
        // the zero move as its fallback, Philox key seed + stage; the winning move
        // updates the guess (x_fb) and the last stage decodes the guess
        const bool delta = rfl(jp->stages) > 0;
        uint32_t key0 = rflu(jp->key0), key1 = rflu(jp->key1);
        if (delta) {
            // stage s of the chain from the MMSE guess: key seed + s; of the chain
            // from the MMSE-SIC guess: seed + kMaxStages + s
            const uint64_t kk = (((uint64_t)key1 << 32) | key0) + (uint64_t)rfl(lds.stage) +
                                (uint64_t)(rfl(lds.chain) ? kMaxStages : 0);
            key0 = rflu((uint32_t)kk);
            key1 = rflu((uint32_t)(kk >> 32));
        }
        const float *beta2 = uniform_ptr(jp->beta2);
        const float *fbase = delta ? uniform_ptr(jp->fp) : uniform_ptr(jp->f);
        const signed char *xbase = uniform_ptr(jp->x_fb);
        if constexpr (PACKED) {
            // Wavefront w anneals instances w P .. w P + P - 1 of the item (P =
            // 64 / glanes) and leaves each one's winning anneal in LDS; then
            // the instances' selection tails (fallback, move, decode) are
            // spread over all four wavefronts, instance r on wavefront r mod 4,
            // so that no wavefront decodes a whole subcarrier alone.
            const int gl = rfl(jp->glanes);
            const int lg = __builtin_ctz((unsigned)gl);
            const int per_wave = 64 >> lg;
            const int first = wave * per_wave;
            if (first < ns) {                         // uniform over the wavefront
                const int chains = rfl(jp->chains);
                const int cnt = min(per_wave, ns - first);
                const int grp = lane >> lg;
                const int chn = lane & (gl - 1);
                const bool valid = grp < cnt;
                const int r = first + (valid ? grp : 0);
                const int n = sc * n_sym + sym0 + r;
                const float *fi = fbase + (size_t)n * ldf;
                const signed char *xi = delta ? sh.zmove : xbase + (size_t)n * KT;
                // the Philox instance index of the whole slot
                const uint32_t un = (uint32_t)n + rflu(jp->inst_base);
                E = anneal_lane<KT, Q, true>(Gi, fi, xi, beta2, sh.T, sweeps, w, key0, key1,
                                             init, (uint32_t)chn, un, bits);
                uint64_t key = ~0ull;
                if (valid && chn < chains) key = ((uint64_t)energy_key(E) << 32) | (uint32_t)chn;
                for (int off = gl >> 1; off >= 1; off >>= 1) {   // minimum within each group
                    const uint32_t lo = __shfl_xor((uint32_t)key, off, 64);
                    const uint32_t hi = __shfl_xor((uint32_t)(key >> 32), off, 64);
                    const uint64_t o = ((uint64_t)hi << 32) | lo;
                    key = o < key ? o : key;
                }
                // each group's winning lane publishes its spins and energy
                if (valid && (uint32_t)chn == (uint32_t)key) {
                    for (int ww = 0; ww < NW; ++ww) sh.wbits[r][ww] = bits[ww];
                    sh.wE[r] = E;
                }
            }
        }
        if constexpr (PACKED) {
            __syncthreads();
            // the lane re-derived from a fresh thread index: values made from it
            // before the anneal are not held (spilled) across it
            int tpost = threadIdx.x;
            asm volatile("" : "+v"(tpost));
            const int lanep = tpost & 63;
            const int wavep = rfl(tpost >> 6);
            const FusedPost p = fused_post(jp);
            signed char *xguess = rfl(lds.chain) ? p.xsic : p.xbase;
            for (int r = wavep; r < ns; r += kWavesPerBlock) {
                uint32_t S[NW];
                for (int ww = 0; ww < NW; ++ww) S[ww] = sh.wbits[r][ww];
                const float Ebest = sh.wE[r];
                const int ng = sc * p.n_sym + sym0 + r;
                const float *fg = p.fbase + (size_t)ng * p.ldf;
                const signed char *xg = p.stages > 0 ? sh.zmove : p.xbase + (size_t)ng * KT;
                // detection couplings are exactly symmetric: column reads (lane-contiguous,
                // no LDS bank conflicts) give the row's values
                const float Efb =
                    p.kind == 0 ? fallback_energy<true>(Gi, KT, p.K, fg, xg, sh.terms[wavep], lanep)
                                : fallback_energy<false>(Gi, KT, p.K, fg, xg, sh.terms[wavep], lanep);
                const bool use_fb = energy_less(Efb, Ebest);
                winning_levels(use_fb, xg, S, p.K, Q, p.w, sh.lvs[wavep], lanep);
                if (p.stages > 0) {
                    apply_move<true>(sh.lvs[wavep], xguess + (size_t)ng * KT, Gi, KT, p.K,
                                     p.ffull + (size_t)ng * p.ldf, (1 << p.dq) - 1,
                                     sh.cand[wavep], sh.terms[wavep], lanep);
                } else if (p.kind == 0) {
                    decode_det(sh.lvs[wavep], ng, sc, sym0 + r, p.n_sym, p.n_rows, p.n_cols, Q,
                               p.c, lds.H, p.y, (unsigned char *)p.out0, (float *)p.out1, lanep);
                } else {
                    decode_vpp(sh.lvs[wavep], ng, sc, sym0 + r, p.n_sym, p.n_rows, p.n_cols,
                               p.tau, lds.Z, lds.ldz, lds.H, p.y, (signed char *)p.out0,
                               (float2 *)p.out1, (float *)p.out2, sh.zsh[wavep], lanep);
                }
                wave_sync_lds();
            }
            return;
        }
        const int r0 = wave / wpi;                 // instance of this wavefront within the item
        const int chunk = wave - r0 * wpi;
        const bool active = r0 < ns;               // uniform over the wavefront
        const int n = sc * n_sym + sym0 + (active ? r0 : 0);
        const int ch = chunk * 64 + lane;
        const float *fi = fbase + (size_t)n * ldf;
        const signed char *xi = delta ? sh.zmove : xbase + (size_t)n * KT;
        if (active) {
            // the Philox instance index of the whole slot (wave-uniform)
            const uint32_t un = (uint32_t)n + rflu(jp->inst_base);
            // the move fields are rewritten at every stage, so they are read with
            // vector loads (the scalar cache is not updated by the stores)
            if (delta)
                E = anneal_lane<KT, Q, true>(Gi, fi, xi, beta2, sh.T, sweeps, w, key0, key1, init,
                                             (uint32_t)ch, un, bits);
            else    // the row is wave-uniform (re-read from the first lane for the compiler)
                E = anneal_lane<KT, Q, false>(Gi, uniform_ptr(fi), xi, beta2, sh.T, sweeps, w,
                                              key0, key1, init, (uint32_t)ch, un, bits);
            const int chains = rfl(jp->chains);
            uint64_t key = ~0ull;
            if (ch < chains) key = ((uint64_t)energy_key(E) << 32) | (uint32_t)ch;
            key = wave_min_u64(key);
            if (lane == 0) sh.keys[wave] = key;
        }
    }
    __syncthreads();
    // selection and decode: descriptor fields re-read after the anneal, the lane
    // from a fresh thread index (values made from it before the anneal are not
    // held across it; 32 spins and more, smaller problems keep fewer registers
    // this way)
    int tpost = threadIdx.x;
    if constexpr (KT * Q >= 32) asm volatile("" : "+v"(tpost));
    const int lanep = KT * Q >= 32 ? (tpost & 63) : lane;
    const FusedPost p = fused_post(jp);
    const int r0 = wave / p.wpi;
    const int chunk = wave - r0 * p.wpi;
    const bool active = r0 < ns;
    const int ch = chunk * 64 + lanep;
    int bch = 0;
    if (active) {
        uint64_t best = ~0ull;
        for (int c2 = 0; c2 < p.wpi; ++c2) {
            const uint64_t o = sh.keys[r0 * p.wpi + c2];
            best = o < best ? o : best;
        }
        bch = (int)(uint32_t)best;
        if (ch == bch) {                        // the winning lane publishes its spins
            for (int ww = 0; ww < NW; ++ww) sh.lvs[wave][ww] = (int)bits[ww];
        }
    }
    __syncthreads();
    if (!active || chunk != bch / 64) return;   // the winner's wavefront decodes
    const int n = sc * p.n_sym + sym0 + r0;
    uint32_t S[NW];
    for (int ww = 0; ww < NW; ++ww) S[ww] = (uint32_t)sh.lvs[wave][ww];
    wave_sync_lds();
    const float Ebest = __shfl(E, bch & 63, 64);
    const float *fi = p.fbase + (size_t)n * p.ldf;
    const signed char *xi = p.stages > 0 ? sh.zmove : p.xbase + (size_t)n * KT;
    // detection couplings are exactly symmetric: column reads (lane-contiguous, no
    // LDS bank conflicts) give the row's values
    const float Efb =
        p.kind == 0 ? fallback_energy<true>(Gi, KT, p.K, fi, xi, sh.terms[wave], lanep)
                    : fallback_energy<false>(Gi, KT, p.K, fi, xi, sh.terms[wave], lanep);
    const bool use_fb = energy_less(Efb, Ebest);
    winning_levels(use_fb, xi, S, p.K, Q, p.w, sh.lvs[wave], lanep);
    const int sy = sym0 + r0;
    if (p.stages > 0) {
        apply_move<true>(sh.lvs[wave], (rfl(lds.chain) ? p.xsic : p.xbase) + (size_t)n * KT, Gi,
                         KT, p.K, p.ffull + (size_t)n * p.ldf, (1 << p.dq) - 1, sh.cand[wave],
                         sh.terms[wave], lanep);
    } else if (p.kind == 0) {
        decode_det(sh.lvs[wave], n, sc, sy, p.n_sym, p.n_rows, p.n_cols, Q, p.c, lds.H, p.y,
                   (unsigned char *)p.out0, (float *)p.out1, lanep);
    } else {
        decode_vpp(sh.lvs[wave], n, sc, sy, p.n_sym, p.n_rows, p.n_cols, p.tau, lds.Z, lds.ldz,
                   lds.H, p.y, (signed char *)p.out0, (float2 *)p.out1, (float *)p.out2,
                   sh.zsh[wave], lanep);
    }
}

#define MMGAP_FUSED_CALL(kt, qq)                                                      \
    do {                                                                              \
        if (packed) fused_anneal<kt, qq, true>(jobs, it.job, it.sc, it.sym0, it.ns, lds, tid); \
        else fused_anneal<kt, qq, false>(jobs, it.job, it.sc, it.sym0, it.ns, lds, tid);       \
    } while (0)
template <int CLS>
__device__ __forceinline__ void fused_dispatch(int variant, bool packed, const FusedJob *jobs,
                                               const FusedItem &it, const FusedItemLds &lds,
                                               int tid)
{
    if constexpr (CLS == 0) {
        switch (variant) {
        case 0: MMGAP_FUSED_CALL(8, 1); break;
        case 1: MMGAP_FUSED_CALL(8, 2); break;
        case 2: MMGAP_FUSED_CALL(8, 3); break;
        case 3: MMGAP_FUSED_CALL(16, 1); break;
        default: break;
        }
    } else if constexpr (CLS == 1) {
        if (variant == 4) MMGAP_FUSED_CALL(16, 2);
    } else {
        switch (variant) {
        case 5: MMGAP_FUSED_CALL(16, 3); break;
        case 6: MMGAP_FUSED_CALL(32, 1); break;
        case 7: MMGAP_FUSED_CALL(32, 2); break;
        case 8: MMGAP_FUSED_CALL(32, 3); break;
        default: break;
        }
    }
}
#undef MMGAP_FUSED_CALL

template <int CLS>
__global__ void __launch_bounds__(kBlock)
    __attribute__((amdgpu_waves_per_eu(FusedClassTraits<CLS>::kMinWaves, 8)))
k_fused(const FusedJob *__restrict__ jobs, const FusedItem *__restrict__ items, int n_items,
        unsigned int *__restrict__ counter, const uint32_t *__restrict__ accept_table)
{
    FusedCommon &sh = g_fc;
    auto &bs = fused_build_shared<CLS>();
    for (int e = threadIdx.x; e <= kAcceptSteps; e += kBlock) sh.T[e] = accept_table[e];
    if (threadIdx.x < 32) sh.zmove[threadIdx.x] = 0;
    // the first round of items is taken by block index, the rest through the
    // work counter (which every launch starts at zero)
    bool first = true;
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0)
            sh.item = first ? (int)blockIdx.x : (int)(atomicAdd(counter, 1u) + gridDim.x);
        first = false;
        __syncthreads();
        const int item = __builtin_amdgcn_readfirstlane(sh.item);
        if (item >= n_items) break;           // every wavefront of the block leaves here
        const FusedItem it = items[item];
        const FusedJob &jb = jobs[it.job];
        // The thread index, re-derived per item: every lane-dependent offset
        // of the build, anneal and decode is then recomputed inside the loop
        // rather than hoisted out of it and spilled to scratch memory.
        int tid = threadIdx.x;
        asm volatile("" : "+v"(tid));
        // the couplings of the item's subcarrier go to LDS (rows of KT floats)
        float *Gs = bs.G;
        for (int s0 = 0; s0 < it.ns; s0 += kFusedBuildSyms) {
            const int sym = it.sym0 + s0, cnt = min(kFusedBuildSyms, it.ns - s0);
            float *fs = jb.f + ((size_t)it.sc * jb.n_sym + sym) * jb.ldf;
            signed char *xs = jb.x_fb + ((size_t)it.sc * jb.n_sym + sym) * jb.KT;
            if (s0 > 0) __syncthreads();      // the previous pass is done with the scratch
            if (jb.kind == 0) {
                build_det_sc(jb.H, jb.y, jb.n_rows, jb.n_cols, jb.n_sym, it.sc, sym, cnt, jb.KT,
                             jb.ldf, (1 << jb.dq) - 1, jb.c, jb.c2, jb.noise_var, Gs, fs, xs,
                             nullptr, bs.det(), tid);
            } else {
                build_vpp_sc(jb.H, jb.y, jb.n_rows, jb.n_cols, jb.n_sym, it.sc, sym, cnt, jb.KT,
                             jb.ldf, jb.tau, Gs, fs, xs, nullptr, nullptr, bs.vpp(), tid);
            }
        }
        // The fields were written with vector stores by this workgroup and are
        // read back through the scalar cache, which vector stores do not
        // update.  (1) Every thread waits until its stores are acknowledged by
        // the L2 of this XCD before the barrier (a workgroup-scope release
        // alone emits no such wait; an agent-scope one would also write back
        // and invalidate the L2).  (2) No scalar-cache line can hold a stale
        // copy: a line is read only after this workgroup wrote it -- field rows
        // are padded to 128 bytes (ldf), so that no line holds data of two work
        // items.  The fallback levels are read with vector loads.
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        __syncthreads();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        // Moves around a guess: per stage the move fields f' = f - G x_g of the
        // item's instances (the guesses start as the build's sliced MMSE
        // estimates and are updated by the stage before), then the anneal.
        // The item's descriptors are re-read at every stage through a
        // laundered index, so that only the stage counter and the item index
        // stay live across the anneal (fewer registers spilled per item).
        // MMGaP-E and the chain from the MMSE-SIC guess: that guess (x_sic) was
        // written by the batch's MMSE-SIC launch, which precedes this kernel
        const int guesses = jb.kind == 0 && jb.stages > 0 ? (jb.guesses ? jb.guesses : 1) : 1;
        // anneal steps: per stage, the chain from the MMSE guess, then the one from
        // the MMSE-SIC guess (each as its guess set asks)
        const int nch = guesses == 3 ? 2 : 1;
        const int nst = (jb.stages > 0 ? jb.stages : 1) * nch;
        for (int step = 0; step < nst; ++step) {
            int itm = item;
            asm volatile("" : "+s"(itm));
            const FusedItem its = items[itm];
            const FusedJob &js = jobs[its.job];
            int tds = threadIdx.x;
            asm volatile("" : "+v"(tds));
            const int st = step / nch;
            const int chain = nch == 2 ? step % 2 : (guesses == 2 ? 1 : 0);
            // the decode reads H (and A^-1) from the build's LDS copies
            FusedItemLds lds;
            lds.G = bs.G;
            if (js.kind == 0) {
                lds.H = reinterpret_cast<const float2 *>(bs.det().Hs);
                lds.Z = nullptr;
                lds.ldz = 0;
            } else {
                lds.H = reinterpret_cast<const float2 *>(bs.vpp().Hs);
                lds.Z = bs.vpp().Zs;
                lds.ldz = FusedClassTraits<CLS>::kNUV;
            }
            if (js.stages > 0) {
                if (step > 0) {        // the previous step's guesses are written
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
                    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
                    __syncthreads();
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
                }
                const int KT = js.KT, ldf = js.ldf;
                for (int e = tds; e < its.ns * KT; e += kBlock) {
                    const int r = e / KT, k = e % KT;
                    const size_t n = (size_t)its.sc * js.n_sym + its.sym0 + r;
                    const signed char *xg = (chain ? js.x_sic : js.x_fb) + n * KT;
                    float g = 0.0f;
                    for (int l = 0; l < KT; ++l) g = fmaf(bs.G[k * KT + l], (float)xg[l], g);
                    js.fp[n * ldf + k] = js.f[n * ldf + k] - g;
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
                asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
                __syncthreads();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
            }
            lds.stage = st;
            lds.chain = chain;
            fused_dispatch<CLS>(js.variant, js.glanes > 0, jobs, its, lds, tds);
        }
        // Moves around a guess: the final guesses of the item's instances are
        // decoded, instance r by wavefront r mod 4.  MMGaP-E takes the answer of
        // the chain from the MMSE-SIC guess only if its float32 level energy
        // (full fields) is strictly lower, and writes the choice to out2.
        if (jb.kind == 0 && jb.stages > 0) {
            int itm = item;
            asm volatile("" : "+s"(itm));
            const FusedItem its = items[itm];
            const FusedPost p = fused_post(uniform_ptr(jobs) + rfl(its.job));
            int tds = threadIdx.x;
            asm volatile("" : "+v"(tds));
            const int lane = tds & 63, wave = rfl(tds >> 6);
            const int KT = rfl(jobs[its.job].KT);
            const int g = p.guesses ? p.guesses : 1;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
            __syncthreads();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
            const float2 *Hl = reinterpret_cast<const float2 *>(bs.det().Hs);
            for (int r = wave; r < its.ns; r += kWavesPerBlock) {
                const int sy = its.sym0 + r;
                const int n = its.sc * p.n_sym + sy;
                int *lv = sh.lvs[wave], *cb = sh.cand[wave];
                if (lane < p.K) {
                    lv[lane] = (int)(g == 2 ? p.xsic : p.xbase)[(size_t)n * KT + lane];
                    if (g == 3) cb[lane] = (int)p.xsic[(size_t)n * KT + lane];
                }
                wave_sync_lds();
                bool from_sic = g == 2;
                if (g == 3) {
                    const float *ff = p.ffull + (size_t)n * p.ldf;
                    const float Ea = wave_level_energy<true>(bs.G, KT, p.K, ff, lv, sh.terms[wave],
                                                             lane);
                    const float Eb = wave_level_energy<true>(bs.G, KT, p.K, ff, cb, sh.terms[wave],
                                                             lane);
                    // every lane holds the same energies: the choice is wave-uniform
                    from_sic = __builtin_amdgcn_readfirstlane(Eb < Ea ? 1 : 0) != 0;
                    if (from_sic) {
                        if (lane < p.K) lv[lane] = cb[lane];
                        wave_sync_lds();
                    }
                }
                if (p.out2 && lane == 0 && p.guesses > 0)
                    static_cast<unsigned char *>(p.out2)[n] = from_sic ? 1 : 0;
                decode_det(lv, n, its.sc, sy, p.n_sym, p.n_rows, p.n_cols, p.dq, p.c, Hl, p.y,
                           (unsigned char *)p.out0, (float *)p.out1, lane);
                wave_sync_lds();
            }
        }
    }
}

// f' = f - G x_g, one thread per (instance, dimension); g as a chain of fused
// multiply-adds over l ascending from 0.
template <int KT>
__global__ void __launch_bounds__(kBlock) k_delta_prep(DeltaPrepArgs a)
{
    const size_t t = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (t >= (size_t)a.n_inst * KT) return;
    const int n = (int)(t / KT), k = (int)(t % KT);
    const float *Gk = a.G + ((size_t)(n / a.inst_per_G) * KT + k) * KT;
    const signed char *xg = a.guess + (size_t)n * KT;
    float g = 0.0f;
#pragma unroll
    for (int l = 0; l < KT; ++l) g = fmaf(Gk[l], (float)xg[l], g);
    a.f_out[t] = a.f[t] - g;
}

__global__ void __launch_bounds__(64) k_sic(SicArgs a)
{
    extern __shared__ double2 sic_dyn[];
    const int lane = threadIdx.x;
    const int sc = blockIdx.x;
    const int nr = a.n_r, nt = a.n_t;
    double2 *P = sic_dyn;                                   // [nt][nt]
    double2 *W = P + nt * nt;                               // [nt][nr]
    cf32 *Hs = reinterpret_cast<cf32 *>(W + nt * nr);       // [nr][nt]
    int *lv = reinterpret_cast<int *>(Hs + nr * nt);        // [64 / g][2 nt]
    int g = 1;
    while (g < nr) g <<= 1;
    int *order = lv + (64 / g) * 2 * nt;                    // [nt]
    const float2 *Hg = a.H + (size_t)sc * nr * nt;
    for (int e = lane; e < nr * nt; e += 64) Hs[e] = to_cf32(Hg[e]);
    wave_sync_lds();
    sic_sc(a, sc, 0, a.n_sym, Hs, P, W, lv, order, 64, lane);
}

// The better of two candidates per instance (the second only if its float32
// level energy is strictly lower), then the decode; one wavefront per instance.
__global__ void __launch_bounds__(kBlock) k_pick(PickArgs a)
{
    __shared__ float terms[kWavesPerBlock][32];
    __shared__ int la[kWavesPerBlock][32];
    __shared__ int lb[kWavesPerBlock][32];
    __shared__ float Gw[kWavesPerBlock][32 * 33];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int n = blockIdx.x * kWavesPerBlock + wave;
    if (n >= a.n_inst) return;
    const int K = a.K, KT = a.KT;
    const float *Gg = a.G + (size_t)(n / a.inst_per_G) * KT * KT;
    float *Gi = Gw[wave];
    copy_g_to_lds<32>(Gi, Gg, KT, lane);
    const float *ff = a.f + (size_t)n * KT;
    if (lane < K) {
        la[wave][lane] = a.xa[(size_t)n * KT + lane];
        lb[wave][lane] = a.xb[(size_t)n * KT + lane];
    }
    wave_sync_lds();
    const float Ea = wave_level_energy(Gi, KT + 1, K, ff, la[wave], terms[wave], lane);
    const float Eb = wave_level_energy(Gi, KT + 1, K, ff, lb[wave], terms[wave], lane);
    const bool use_b = Eb < Ea;
    if (a.from_b && lane == 0) a.from_b[n] = use_b ? 1 : 0;
    const int sc = n / a.n_sym, sy = n % a.n_sym;
    decode_det(use_b ? lb[wave] : la[wave], n, sc, sy, a.n_sym, a.n_rows, a.n_cols, a.q, a.c,
               a.H + (size_t)sc * a.n_rows * a.n_cols, a.y, a.sym_out, a.metric_out, lane);
}

// ---------------------------------------------------------------------------
// Detection by moves around a guess (paper §2.3 Fig. 5) and MMGaP-E (§3.2
// Fig. 6) in one launch: the stages that k_delta_prep, k_anneal, k_select
// (kSelectDelta) and k_pick run as separate launches, with the same keys,
// clamp, choices and decode, so the outputs are identical.  A wavefront keeps
// its P = 64 / glanes instances (one subcarrier: one G, staged in LDS once)
// from the first stage to the decode; each instance takes glanes lanes (one
// chain each) and an LDS row for its move fields, guesses and scratch.  The
// chain from guess A (keys seed + s) runs its stages, then the chain from
// guess B (keys seed + kMaxStages + s).  Per stage, per instance:
//   f' = f - G x_g (the move fields),
//   the anneal of the move problem (levels {-2, 0, 2}) with the zero move as
//   fallback, the group's best chain (lowest energy, then lowest index), the
//   zero move instead if its energy is strictly lower,
//   the move applied and clamped, kept iff the float32 energy with the full
//   fields drops.
// Then B's final guess if its energy is strictly lower than A's, and the decode.
// The group reductions and sums keep the operation order of the
// one-wavefront-per-instance kernels; the couplings are read by columns
// (detection couplings are exactly symmetric), which gives the rows' values
// without LDS bank conflicts.

// LDS row of one instance: move fields, energy terms, the energies of the
// current guess and of each chain's final guess (kept here rather than in
// registers across the anneals), guesses A and B, candidate.
template <int KT>
constexpr int search_row_bytes()
{
    return (11 * KT + 16 + 15) / 16 * 16;
}
template <int KT>
struct SearchRow {
    float *fp, *terms, *E;          // E: [0] current guess, [1] chain A's, [2] chain B's
    signed char *xa, *xb, *cand;
    __device__ SearchRow(unsigned char *rows, int row)
    {
        unsigned char *r = rows + (size_t)row * search_row_bytes<KT>();
        fp = reinterpret_cast<float *>(r);
        terms = fp + KT;
        E = terms + KT;
        xa = reinterpret_cast<signed char *>(E + 4);
        xb = xa + KT;
        cand = xb + KT;
    }
};

// The levels of one instance, KT signed bytes in LDS (4-byte aligned), as
// floats (exact small integers), read a word at a time.
template <int KT>
__device__ __forceinline__ void lds_levels(const signed char *lv, float (&x)[KT])
{
    const uint32_t *w = reinterpret_cast<const uint32_t *>(lv);
#pragma unroll
    for (int i = 0; i < KT / 4; ++i) {
        const uint32_t v = w[i];
#pragma unroll
        for (int b = 0; b < 4; ++b) x[4 * i + b] = (float)(int)(int8_t)(v >> (8 * b));
    }
}

// Energy sum_k lv_k (g_k - f_k) with g = G lv - f of each group's instance
// (the operations and order of wave_level_energy): lane j of a group of GL
// lanes forms the terms of dimensions j, j + GL, ..., then every lane sums the
// K terms in order.  Called by the whole wavefront.  With K = KT the levels
// are read once into registers and every loop is unrolled, so the loads of a
// column issue together.
template <int KT>
__device__ __forceinline__ float group_level_energy(const float *Gl, int K, const float *ff,
                                                    const signed char *lv, float *terms, int j,
                                                    int GL)
{
    float e = 0.0f;
    if (K == KT) {
        float x[KT];
        lds_levels<KT>(lv, x);
        for (int k = j; k < KT; k += GL) {
            float acc = -ff[k];
#pragma unroll
            for (int l = 0; l < KT; ++l) acc = fmaf(Gl[l * KT + k], x[l], acc);
            terms[k] = acc - ff[k];
        }
        wave_sync_lds();
        const float4 *t4 = reinterpret_cast<const float4 *>(terms);
#pragma unroll
        for (int k4 = 0; k4 < KT / 4; ++k4) {
            const float4 t = t4[k4];
            e = fmaf(x[4 * k4 + 0], t.x, e);
            e = fmaf(x[4 * k4 + 1], t.y, e);
            e = fmaf(x[4 * k4 + 2], t.z, e);
            e = fmaf(x[4 * k4 + 3], t.w, e);
        }
    } else {
        for (int k = j; k < K; k += GL) {
            float acc = -ff[k];
            for (int l = 0; l < K; ++l) acc = fmaf(Gl[l * KT + k], (float)lv[l], acc);
            terms[k] = acc - ff[k];
        }
        wave_sync_lds();
        for (int k = 0; k < K; ++k) e = fmaf((float)lv[k], terms[k], e);
    }
    wave_sync_lds();
    return e;
}

template <int KT>
constexpr int search_min_waves()
{
    return KT <= 8 ? 8 : KT == 16 ? 6 : 5;
}

template <int KT>
__global__ void __launch_bounds__(kBlock)
    __attribute__((amdgpu_waves_per_eu(search_min_waves<KT>(), 8)))
k_search(SearchArgs a)
{
    constexpr int NW = (2 * KT + 31) / 32;
    __shared__ uint32_t T[kAcceptSteps + 1];
    __shared__ float4 Gw[kWavesPerBlock][KT * KT / 4];
    __shared__ __align__(16) signed char zrow[KT];   // the zero move
    extern __shared__ float4 search_dyn4[];       // the instances' rows
    unsigned char *rows = reinterpret_cast<unsigned char *>(search_dyn4);
    for (int e = threadIdx.x; e <= kAcceptSteps; e += kBlock) T[e] = a.accept_table[e];
    if (threadIdx.x < KT) zrow[threadIdx.x] = 0;
    __syncthreads();

    const int GL = a.glanes;
    const int lg = __builtin_ctz((unsigned)GL);
    const int per_wave = 64 >> lg;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    // a subcarrier's wavefronts (consecutive) in workgroups on one XCD: its
    // couplings, H and y come from HBM once
    const int blk = xcd_block((int)blockIdx.x, (int)gridDim.x);
    const int inst0 = (blk * kWavesPerBlock + wave) * per_wave;
    if (inst0 >= a.n_inst) return;     // whole wavefront; only wave-level exchange below
    const bool use_a = a.guess_a != nullptr, use_b = a.guess_b != nullptr;
    float *Gs = reinterpret_cast<float *>(Gw[wave]);
    bool g_bad;                         // a coupling of the wavefront's G is not finite
    {
        const int lane = threadIdx.x & 63, grp = lane >> lg, j = lane & (GL - 1);
        const int n = inst0 + grp < a.n_inst ? inst0 + grp : inst0;
        const float *Gg = a.G + (size_t)(inst0 / a.inst_per_G) * (KT * KT);
        bool bad = false;
        for (int e = lane; e < KT * KT; e += 64) {
            const float v = Gg[e];
            bad |= !(fabsf(v) <= FLT_MAX);
            Gs[e] = v;
        }
        g_bad = __ballot(bad) != 0;
        const SearchRow<KT> R(rows, wave * per_wave + grp);
        for (int k = j; k < KT; k += GL) {
            if (use_a) R.xa[k] = a.guess_a[(size_t)n * KT + k];
            if (use_b) R.xb[k] = a.guess_b[(size_t)n * KT + k];
        }
        wave_sync_lds();
    }
    const int qtop = (1 << a.dq) - 1;
    const int wts[4] = {1, 1, 0, 0};
    for (int chain = 0; chain < 2; ++chain) {
        if (!(chain ? use_b : use_a)) continue;
        for (int s = 0; s < a.stages; ++s) {
            uint32_t bits[NW];
            float E;
            {
                // lane coordinates from a fresh thread index at every stage, so
                // that nothing derived from it is held across the anneal
                int tid = threadIdx.x;
                asm volatile("" : "+v"(tid));
                const int lane = tid & 63, grp = lane >> lg, j = lane & (GL - 1);
                const int n = inst0 + grp < a.n_inst ? inst0 + grp : inst0;
                const SearchRow<KT> R(rows, wave * per_wave + grp);
                const signed char *xg = chain ? R.xb : R.xa;
                const float *ff = a.f + (size_t)n * KT;
                if (s == 0) {       // the energy of the starting guess (full fields)
                    const float e0 = group_level_energy<KT>(Gs, a.K, ff, xg, R.terms, j, GL);
                    if (j == 0) R.E[0] = e0;
                }
                {                                           // the move fields
                    float xl[KT];
                    lds_levels<KT>(xg, xl);
                    for (int k = j; k < KT; k += GL) {
                        float g = 0.0f;
#pragma unroll
                        for (int l = 0; l < KT; ++l) g = fmaf(Gs[l * KT + k], xl[l], g);
                        R.fp[k] = ff[k] - g;
                    }
                }
                wave_sync_lds();
                const uint64_t kk = (((uint64_t)a.key1 << 32) | a.key0) + (uint64_t)s +
                                    (uint64_t)(chain ? kMaxStages : 0);
                uint32_t ginst = (uint32_t)n + a.inst_base;
                asm volatile("" : "+v"(ginst));
                E = anneal_lane<KT, 2, true, true>(Gs, R.fp, zrow, a.beta2, T, a.sweeps, wts,
                                                   (uint32_t)kk, (uint32_t)(kk >> 32),
                                                   a.init_mode, (uint32_t)j, ginst, bits);
            }
            int tid = threadIdx.x;
            asm volatile("" : "+v"(tid));
            const int lane = tid & 63, grp = lane >> lg, j = lane & (GL - 1);
            const bool valid = inst0 + grp < a.n_inst;
            const int n = valid ? inst0 + grp : inst0;
            const SearchRow<KT> R(rows, wave * per_wave + grp);
            signed char *xg = chain ? R.xb : R.xa;
            const float *ff = a.f + (size_t)n * KT;
            // the group's best chain: lowest energy, then lowest index
            uint64_t key = ~0ull;
            if (valid && j < a.chains) key = ((uint64_t)energy_key(E) << 32) | (uint32_t)j;
            key = group_min_u64(key, GL);
            const int src = (lane & ~(GL - 1)) | (int)((uint32_t)key & (uint32_t)(GL - 1));
            const float Eb = __shfl(E, src, 64);
            uint32_t S[NW];
#pragma unroll
            for (int w = 0; w < NW; ++w) S[w] = __shfl(bits[w], src, 64);
            // the zero move (the fallback): its energy with the move fields sums
            // 0 x (-2 f'_k) over k, which is +0 unless a term is not finite (a
            // coupling or a doubled move field), and then NaN
            bool fbad = false;
            for (int k = j; k < a.K; k += GL) {
                const float fk = R.fp[k];
                fbad |= !(fabsf(-fk - fk) <= FLT_MAX);
            }
            const uint64_t gmask = (GL == 64 ? ~0ull : ((1ull << GL) - 1ull)) << (lane & ~(GL - 1));
            const bool fb_nan = g_bad || (__ballot(fbad) & gmask) != 0;
            const float Efb = fb_nan ? __builtin_nanf("") : 0.0f;
            const bool use_fb = energy_less(Efb, Eb);
            for (int k = j; k < a.K; k += GL) {
                int z = 0;
                if (!use_fb) {
#pragma unroll
                    for (int b = 0; b < 2; ++b) {
                        const int i = 2 * k + b;
                        uint32_t word = S[0];
#pragma unroll
                        for (int w = 1; w < NW; ++w)
                            if ((i >> 5) == w) word = S[w];
                        z += ((word >> (i & 31)) & 1u) ? -1 : 1;
                    }
                }
                const int v = (int)xg[k] + z;
                R.cand[k] = (signed char)(v < -qtop ? -qtop : (v > qtop ? qtop : v));
            }
            wave_sync_lds();
            const float Ec = group_level_energy<KT>(Gs, a.K, ff, R.cand, R.terms, j, GL);
            const float Eg = R.E[0];
            if (Ec < Eg) {
                for (int k = j; k < a.K; k += GL) xg[k] = R.cand[k];
                if (j == 0) R.E[0] = Ec;
            }
            wave_sync_lds();
            if (s == a.stages - 1 && j == 0) R.E[1 + chain] = R.E[0];
            wave_sync_lds();
        }
    }
    // the answer (B's only if its energy is strictly lower) and its decode, as
    // decode_det with the group's lanes: lane j takes receive antennas j and
    // j + GL (n_rows <= 2 GL), and the group's butterfly gives the sum of the
    // wavefront's
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    const int lane = tid & 63, grp = lane >> lg, j = lane & (GL - 1);
    const bool valid = inst0 + grp < a.n_inst;
    const int n = valid ? inst0 + grp : inst0;
    const SearchRow<KT> R(rows, wave * per_wave + grp);
    const bool from_b = use_a && use_b ? R.E[2] < R.E[1] : use_b;
    const signed char *lv = from_b ? R.xb : R.xa;
    const int nt = a.n_cols, nr = a.n_rows;
    const int sc = n / a.n_sym, sy = n - sc * a.n_sym;
    if (valid) {
        for (int t = j; t < nt; t += GL) {
            const int pI = ((int)lv[t] + qtop) >> 1;
            const int pQ = ((int)lv[nt + t] + qtop) >> 1;
            const int gI = pI ^ (pI >> 1), gQ = pQ ^ (pQ >> 1);
            a.sym_out[(size_t)n * nt + t] = (unsigned char)((gI << a.dq) | gQ);
        }
        if (a.from_b && j == 0) a.from_b[n] = from_b ? 1 : 0;
    }
    if (a.metric_out) {
        const float2 *Hsc = a.H + (size_t)sc * nr * nt;
        double part = 0.0;
        for (int r = j; r < nr; r += GL) {
            const float2 *Hr = Hsc + (size_t)r * nt;
            const float2 yv = a.y[((size_t)sc * a.n_sym + sy) * nr + r];
            double re = yv.x, im = yv.y;
            for (int t = 0; t < nt; ++t) {
                const double xr = a.c * (double)lv[t];
                const double xi = a.c * (double)lv[nt + t];
                const double hr = Hr[t].x, hi = Hr[t].y;
                re = re - (hr * xr - hi * xi);
                im = im - (hr * xi + hi * xr);
            }
            part = part + (re * re + im * im);
        }
        for (int off = GL >> 1; off >= 1; off >>= 1) part += __shfl_xor(part, off, 64);
        if (valid && j == 0) a.metric_out[n] = (float)part;
    }
}

__global__ void k_reset_counters(unsigned int *counters, int n)
{
    if (blockIdx.x == 0 && (int)threadIdx.x < n) counters[threadIdx.x] = 0u;
}

// ---------------------------------------------------------------------------
// Dense spin-domain expansion (J, h, constant) of the level-domain form.
__global__ void __launch_bounds__(kBlock) k_expand(ExpandArgs a)
{
    const int N = a.K * a.q;
    const size_t nJ = a.J ? (size_t)a.n_sc * N * N : 0;
    const size_t n_inst = (size_t)a.n_sc * a.n_sym;
    const size_t nh = a.h ? n_inst * N : 0;
    const size_t ne = a.e_const ? n_inst : 0;
    const size_t total = nJ + nh + ne;
    for (size_t e = (size_t)blockIdx.x * kBlock + threadIdx.x; e < total;
         e += (size_t)gridDim.x * kBlock) {
        if (e < nJ) {
            const size_t sc = e / ((size_t)N * N);
            const int i = (int)((e / N) % N), j = (int)(e % N);
            float v = 0.0f;
            if (i != j) {
                const float G = a.G[(sc * a.K + i / a.q) * a.K + j / a.q];
                v = (float)(-2 * a.w[i % a.q] * a.w[j % a.q]) * G;
            }
            a.J[e] = v;
        } else if (e < nJ + nh) {
            const size_t o = e - nJ;
            const size_t n = o / N;
            const int i = (int)(o % N);
            a.h[o] = (float)(2 * a.w[i % a.q]) * a.f[n * a.K + i / a.q];
        } else {
            const size_t n = e - nJ - nh;
            const size_t sc = n / a.n_sym;
            double acc = 0.0;
            for (int i = 0; i < N; ++i) {
                const double w = (double)a.w[i % a.q];
                acc = acc + (w * w) * (double)a.G[(sc * a.K + i / a.q) * a.K + i / a.q];
            }
            a.e_const[n] = (float)(acc + (a.norm ? a.norm[n] : 0.0));
        }
    }
}

__global__ void k_pad_matrix(const float *src, float *dst, int n, int K, int KT)
{
    const size_t total = (size_t)n * KT * KT;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (size_t)gridDim.x * blockDim.x) {
        const size_t m = e / ((size_t)KT * KT);
        const int r = (int)((e / KT) % KT), c = (int)(e % KT);
        dst[e] = (r < K && c < K) ? src[(m * K + r) * K + c] : 0.0f;
    }
}

// Spin words -> int8 spins: out[r][i] = -1 where bit i of word row r is set.
__global__ void k_chain_spins(const uint32_t *S, int NW, int N, size_t n, signed char *out)
{
    const size_t total = n * (size_t)N;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (size_t)gridDim.x * blockDim.x) {
        const size_t r = e / N;
        const int i = (int)(e % N);
        out[e] = ((S[r * NW + (i >> 5)] >> (i & 31)) & 1u) ? (signed char)-1 : (signed char)1;
    }
}

// Byte fill with a kernel (capturable in HIP graphs, unlike a memset node).
__global__ void k_fill_u8(unsigned char *dst, unsigned char v, size_t n)
{
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
         e += (size_t)gridDim.x * blockDim.x)
        dst[e] = v;
}

template <typename T>
__global__ void k_pad_rows(const T *src, T *dst, int m, int K, int KT)
{
    const size_t total = (size_t)m * KT;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (size_t)gridDim.x * blockDim.x) {
        const size_t r = e / KT;
        const int c = (int)(e % KT);
        dst[e] = c < K ? src[r * K + c] : T(0);
    }
}

int grid_for(size_t total)
{
    size_t g = (total + kBlock - 1) / kBlock;
    if (g > 65536) g = 65536;
    return g == 0 ? 1 : (int)g;
}

template <int KT, int Q>
hipError_t launch_anneal_t(const AnnealArgs &a, hipStream_t s)
{
    const int per_wave = a.glanes > 0 ? 64 / a.glanes : 1;
    if (a.glanes > 0 && (a.glanes > 32 || (a.glanes & (a.glanes - 1)) || a.chains > a.glanes ||
                         a.inst_per_G % per_wave != 0))
        return hipErrorInvalidValue;
    const size_t waves = a.glanes > 0 ? ((size_t)a.n_inst + per_wave - 1) / per_wave
                                      : (size_t)a.n_inst * ((a.chains + 63) / 64);
    const size_t blocks = (waves + kWavesPerBlock - 1) / kWavesPerBlock;
    if (blocks == 0) return hipSuccess;
    if (blocks > 0x7FFFFFFFull) return hipErrorInvalidValue;
    // 64 dimensions: LDS slots for the distinct G of a workgroup's wavefronts.
    // Wavefront w takes G floor(w / wpg); four consecutive wavefronts span one
    // G when wpg is a multiple of 4, four when wpg = 1, else at most two.
    int g_slots = 0;
    if (KT > 32) {
        const size_t wpg = a.glanes > 0 ? (size_t)a.inst_per_G / per_wave
                                        : (size_t)a.inst_per_G * ((a.chains + 63) / 64);
        if (wpg == 0) return hipErrorInvalidValue;
        g_slots = wpg % kWavesPerBlock == 0 ? 1 : (wpg == 1 ? kWavesPerBlock : 2);
    }
    const size_t lds = (size_t)g_slots * KT * KT * sizeof(float);
    if (a.glanes > 0)
        hipLaunchKernelGGL((k_anneal<KT, Q, true>), dim3((unsigned)blocks), dim3(kBlock), lds, s,
                           a.G, a.inst_per_G, a.f, a.x_fb, a.beta2, a.accept_table, a.sweeps,
                           a.chains, a.n_inst, a.w[0], a.w[1], a.w[2], a.w[3], a.key0, a.key1,
                           a.inst_base, a.init_mode, a.glanes, g_slots, a.chain_E, a.chain_S);
    else
        hipLaunchKernelGGL((k_anneal<KT, Q, false>), dim3((unsigned)blocks), dim3(kBlock), lds,
                           s, a.G, a.inst_per_G, a.f, a.x_fb, a.beta2, a.accept_table, a.sweeps,
                           a.chains, a.n_inst, a.w[0], a.w[1], a.w[2], a.w[3], a.key0, a.key1,
                           a.inst_base, a.init_mode, 0, g_slots, a.chain_E, a.chain_S);
    return hipGetLastError();
}

// 33 to 64 spins: two lanes per anneal, so an instance takes 2 glanes lanes
// (32 anneals per wavefront when glanes is 0 or 32).
template <int KT, int Q>
hipError_t launch_cim2_t(const AnnealArgs &a, hipStream_t s)
{
    if (a.glanes > 0 && (a.glanes > 32 || (a.glanes & (a.glanes - 1)) || a.chains > a.glanes ||
                         a.inst_per_G % (64 / a.glanes) != 0))
        return hipErrorInvalidValue;
    if (a.cim.f_mvm < 1) return hipErrorInvalidValue;
    const int gl2 = a.glanes > 0 && a.glanes < 32 ? 2 * a.glanes : 0;
    const size_t waves = gl2 > 0 ? ((size_t)a.n_inst + 64 / gl2 - 1) / (64 / gl2)
                                 : (size_t)a.n_inst * ((a.chains + 31) / 32);
    const size_t blocks = (waves + kWavesPerBlock - 1) / kWavesPerBlock;
    if (blocks == 0) return hipSuccess;
    if (blocks > 0x7FFFFFFFull) return hipErrorInvalidValue;
    if (gl2 > 0)
        hipLaunchKernelGGL((k_cim2<KT, Q, true>), dim3((unsigned)blocks), dim3(kBlock), 0, s, a.G,
                           a.inst_per_G, a.f, a.x_fb, a.cim, a.sweeps, a.chains, a.n_inst, a.w[0],
                           a.w[1], a.w[2], a.w[3], a.key0, a.key1, a.inst_base, a.init_mode,
                           gl2, a.chain_E, a.chain_S, a.chain_div, a.n_real);
    else
        hipLaunchKernelGGL((k_cim2<KT, Q, false>), dim3((unsigned)blocks), dim3(kBlock), 0, s,
                           a.G, a.inst_per_G, a.f, a.x_fb, a.cim, a.sweeps, a.chains, a.n_inst,
                           a.w[0], a.w[1], a.w[2], a.w[3], a.key0, a.key1, a.inst_base,
                           a.init_mode, 0, a.chain_E, a.chain_S, a.chain_div, a.n_real);
    return hipGetLastError();
}

template <int KT, int Q>
hipError_t launch_cim_t(const AnnealArgs &a, hipStream_t s)
{
    const int per_wave = a.glanes > 0 ? 64 / a.glanes : 1;
    if (a.glanes > 0 && (a.glanes > 32 || (a.glanes & (a.glanes - 1)) || a.chains > a.glanes ||
                         a.inst_per_G % per_wave != 0))
        return hipErrorInvalidValue;
    if (a.cim.f_mvm < 1) return hipErrorInvalidValue;
    const size_t waves = a.glanes > 0 ? ((size_t)a.n_inst + per_wave - 1) / per_wave
                                      : (size_t)a.n_inst * ((a.chains + 63) / 64);
    const size_t blocks = (waves + kWavesPerBlock - 1) / kWavesPerBlock;
    if (blocks == 0) return hipSuccess;
    if (blocks > 0x7FFFFFFFull) return hipErrorInvalidValue;
    if (a.glanes > 0)
        hipLaunchKernelGGL((k_cim<KT, Q, true>), dim3((unsigned)blocks), dim3(kBlock), 0, s, a.G,
                           a.inst_per_G, a.f, a.x_fb, a.cim, a.sweeps, a.chains, a.n_inst, a.w[0],
                           a.w[1], a.w[2], a.w[3], a.key0, a.key1, a.inst_base, a.init_mode,
                           a.glanes, a.chain_E, a.chain_S, a.chain_div, a.n_real);
    else
        hipLaunchKernelGGL((k_cim<KT, Q, false>), dim3((unsigned)blocks), dim3(kBlock), 0, s, a.G,
                           a.inst_per_G, a.f, a.x_fb, a.cim, a.sweeps, a.chains, a.n_inst, a.w[0],
                           a.w[1], a.w[2], a.w[3], a.key0, a.key1, a.inst_base, a.init_mode, 0,
                           a.chain_E, a.chain_S, a.chain_div, a.n_real);
    return hipGetLastError();
}

}  // namespace

int fused_variant(int KT, int q)
{
    const int kt = KT == 8 ? 0 : (KT == 16 ? 1 : (KT == 32 ? 2 : -1));
    if (kt < 0 || q < 1 || q > 3) return -1;
    return kt * 3 + (q - 1);
}

int fused_kernel_class(int variant)
{
    if (variant < 0 || variant > 8) return -1;
    return variant <= 3 ? 0 : (variant == 4 ? 1 : 2);
}

hipError_t launch_det_build(const DetBuildArgs &a, hipStream_t s)
{
    if (a.n_sc <= 0) return hipSuccess;
    if (a.n_r > 64) return hipErrorInvalidValue;
    const bool r16 = a.n_r <= 16;
    if (a.n_t <= 8) {
        if (r16) hipLaunchKernelGGL((k_det_build<8, 16>), dim3(a.n_sc), dim3(kBuildBlock), 0, s, a);
        else hipLaunchKernelGGL((k_det_build<8, 64>), dim3(a.n_sc), dim3(kBuildBlock), 0, s, a);
    } else if (a.n_t <= 16) {
        if (r16) hipLaunchKernelGGL((k_det_build<16, 16>), dim3(a.n_sc), dim3(kBuildBlock), 0, s, a);
        else hipLaunchKernelGGL((k_det_build<16, 64>), dim3(a.n_sc), dim3(kBuildBlock), 0, s, a);
    } else if (a.n_t <= 32) {
        if (a.n_r <= 32)
            hipLaunchKernelGGL((k_det_build<32, 32>), dim3(a.n_sc), dim3(kBuildBlock), 0, s, a);
        else
            hipLaunchKernelGGL((k_det_build<32, 64>), dim3(a.n_sc), dim3(kBuildBlock), 0, s, a);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_vpp_build(const VppBuildArgs &a, hipStream_t s)
{
    if (a.n_sc <= 0) return hipSuccess;
    if (a.n_u <= 8) hipLaunchKernelGGL(k_vpp_build<8>, dim3(a.n_sc), dim3(kBuildBlock), 0, s, a);
    else hipLaunchKernelGGL(k_vpp_build<16>, dim3(a.n_sc), dim3(kBuildBlock), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_cim(int KT, int q, const AnnealArgs &a, hipStream_t s)
{
#define MMGAP_CIM_CASE(kt, qq) \
    if (KT == kt && q == qq) return launch_cim_t<kt, qq>(a, s);
    MMGAP_CIM_CASE(8, 1)
    MMGAP_CIM_CASE(8, 2)
    MMGAP_CIM_CASE(8, 3)
    MMGAP_CIM_CASE(8, 4)
    MMGAP_CIM_CASE(16, 1)
    MMGAP_CIM_CASE(16, 2)
    MMGAP_CIM_CASE(32, 1)
#undef MMGAP_CIM_CASE
    if (KT == 16 && q == 3) return launch_cim2_t<16, 3>(a, s);
    if (KT == 16 && q == 4) return launch_cim2_t<16, 4>(a, s);
    if (KT == 32 && q == 2) return launch_cim2_t<32, 2>(a, s);
    return hipErrorInvalidValue;
}

hipError_t launch_anneal(int KT, int q, const AnnealArgs &a, hipStream_t s)
{
#define MMGAP_ANNEAL_CASE(kt, qq) \
    if (KT == kt && q == qq) return launch_anneal_t<kt, qq>(a, s);
    MMGAP_ANNEAL_CASE(8, 1)
    MMGAP_ANNEAL_CASE(8, 2)
    MMGAP_ANNEAL_CASE(8, 3)
    MMGAP_ANNEAL_CASE(8, 4)
    MMGAP_ANNEAL_CASE(16, 1)
    MMGAP_ANNEAL_CASE(16, 2)
    MMGAP_ANNEAL_CASE(16, 3)
    MMGAP_ANNEAL_CASE(16, 4)
    MMGAP_ANNEAL_CASE(32, 1)
    MMGAP_ANNEAL_CASE(32, 2)
    MMGAP_ANNEAL_CASE(32, 3)
    MMGAP_ANNEAL_CASE(32, 4)
    MMGAP_ANNEAL_CASE(64, 1)
    MMGAP_ANNEAL_CASE(64, 2)
#undef MMGAP_ANNEAL_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_select(const SelectArgs &a, hipStream_t s)
{
    if (a.n_inst <= 0) return hipSuccess;
    if (a.KT > 64 || a.K > a.KT) return hipErrorInvalidValue;   // G of an instance in LDS
    if (a.mode == kSelectVpp && a.n_rows > 16) return hipErrorInvalidValue;
    const int blocks = (a.n_inst + kWavesPerBlock - 1) / kWavesPerBlock;
    if (a.KT <= 32)
        hipLaunchKernelGGL(k_select<32>, dim3(blocks), dim3(kBlock), 0, s, a);
    else
        hipLaunchKernelGGL(k_select<64>, dim3(blocks), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_delta_prep(const DeltaPrepArgs &a, hipStream_t s)
{
    const size_t total = (size_t)a.n_inst * a.KT;
    if (total == 0) return hipSuccess;
    const size_t blocks = (total + kBlock - 1) / kBlock;
    if (blocks > 0x7FFFFFFFull) return hipErrorInvalidValue;
    if (a.KT == 8)
        hipLaunchKernelGGL(k_delta_prep<8>, dim3((unsigned)blocks), dim3(kBlock), 0, s, a);
    else if (a.KT == 16)
        hipLaunchKernelGGL(k_delta_prep<16>, dim3((unsigned)blocks), dim3(kBlock), 0, s, a);
    else if (a.KT == 32)
        hipLaunchKernelGGL(k_delta_prep<32>, dim3((unsigned)blocks), dim3(kBlock), 0, s, a);
    else if (a.KT == 64)
        hipLaunchKernelGGL(k_delta_prep<64>, dim3((unsigned)blocks), dim3(kBlock), 0, s, a);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_sic(const SicArgs &a, hipStream_t s)
{
    if (a.n_sc <= 0) return hipSuccess;
    if (a.n_r < 1 || a.n_r > 64 || a.n_t < 1 || a.n_t > 16 || a.n_sym < 1 ||
        (a.levels && a.ldl < 2 * a.n_t) || (a.metric_out && !a.sym_out))
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_sic, dim3(a.n_sc), dim3(64), sic_lds_bytes(a.n_r, a.n_t), s, a);
    return hipGetLastError();
}

hipError_t launch_search(int KT, const SearchArgs &a, hipStream_t s)
{
    if (a.n_inst <= 0) return hipSuccess;
    const int gl = a.glanes;
    if (gl < 4 || gl > 64 || (gl & (gl - 1)) || a.chains < 1 || a.chains > gl ||
        a.inst_per_G < 1 || a.inst_per_G % (64 / gl) != 0 || a.n_rows > 2 * gl ||
        a.n_cols < 1 || 2 * a.n_cols != a.K || a.K > KT || a.stages < 1 ||
        (!a.guess_a && !a.guess_b) || a.dq < 1 || a.dq > 3)
        return hipErrorInvalidValue;
    const size_t waves = ((size_t)a.n_inst + 64 / gl - 1) / (64 / gl);
    const size_t blocks = (waves + kWavesPerBlock - 1) / kWavesPerBlock;
    if (blocks > 0x7FFFFFFFull) return hipErrorInvalidValue;
#define MMGAP_SEARCH_CASE(kt)                                                               \
    if (KT == kt) {                                                                        \
        const size_t lds = (size_t)kWavesPerBlock * (64 / gl) * search_row_bytes<kt>();    \
        hipLaunchKernelGGL(k_search<kt>, dim3((unsigned)blocks), dim3(kBlock), lds, s, a); \
        return hipGetLastError();                                                          \
    }
    MMGAP_SEARCH_CASE(8)
    MMGAP_SEARCH_CASE(16)
    MMGAP_SEARCH_CASE(32)
#undef MMGAP_SEARCH_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_pick(const PickArgs &a, hipStream_t s)
{
    if (a.n_inst <= 0) return hipSuccess;
    if (a.K > 32 || a.KT > 32 || a.K > a.KT) return hipErrorInvalidValue;
    const int blocks = (a.n_inst + kWavesPerBlock - 1) / kWavesPerBlock;
    hipLaunchKernelGGL(k_pick, dim3(blocks), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_fused_reset(unsigned int *counters, hipStream_t s)
{
    hipLaunchKernelGGL(k_reset_counters, dim3(1), dim3(64), 0, s, counters, kFusedClasses);
    return hipGetLastError();
}

hipError_t launch_fused(int cls, const FusedJob *jobs, const FusedItem *items, int n_items,
                        unsigned int *counter, const uint32_t *accept_table, int blocks,
                        hipStream_t s)
{
    if (n_items <= 0 || blocks <= 0) return hipSuccess;
    switch (cls) {
    case 0:
        hipLaunchKernelGGL(k_fused<0>, dim3(blocks), dim3(kBlock), 0, s, jobs, items, n_items,
                           counter, accept_table);
        break;
    case 1:
        hipLaunchKernelGGL(k_fused<1>, dim3(blocks), dim3(kBlock), 0, s, jobs, items, n_items,
                           counter, accept_table);
        break;
    case 2:
        hipLaunchKernelGGL(k_fused<2>, dim3(blocks), dim3(kBlock), 0, s, jobs, items, n_items,
                           counter, accept_table);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t fused_blocks_per_cu(int cls, int *blocks)
{
    switch (cls) {
    case 0: return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, k_fused<0>, kBlock, 0);
    case 1: return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, k_fused<1>, kBlock, 0);
    case 2: return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, k_fused<2>, kBlock, 0);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_expand(const ExpandArgs &a, hipStream_t s)
{
    const int N = a.K * a.q;
    const size_t n_inst = (size_t)a.n_sc * a.n_sym;
    const size_t total = (a.J ? (size_t)a.n_sc * N * N : 0) + (a.h ? n_inst * N : 0) +
                         (a.e_const ? n_inst : 0);
    if (total == 0) return hipSuccess;
    hipLaunchKernelGGL(k_expand, dim3(grid_for(total)), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_pad_matrix(const float *src, float *dst, int n, int K, int KT, hipStream_t s)
{
    const size_t total = (size_t)n * KT * KT;
    if (total == 0) return hipSuccess;
    hipLaunchKernelGGL(k_pad_matrix, dim3(grid_for(total)), dim3(kBlock), 0, s, src, dst, n, K,
                       KT);
    return hipGetLastError();
}

hipError_t launch_pad_rows_f32(const float *src, float *dst, int m, int K, int KT, hipStream_t s)
{
    const size_t total = (size_t)m * KT;
    if (total == 0) return hipSuccess;
    hipLaunchKernelGGL(k_pad_rows<float>, dim3(grid_for(total)), dim3(kBlock), 0, s, src, dst, m,
                       K, KT);
    return hipGetLastError();
}

hipError_t launch_chain_spins(const uint32_t *S, int NW, int N, size_t n, signed char *out,
                              hipStream_t s)
{
    if (n == 0 || N == 0) return hipSuccess;
    if (N > NW * 32) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_chain_spins, dim3(grid_for(n * (size_t)N)), dim3(kBlock), 0, s, S, NW, N,
                       n, out);
    return hipGetLastError();
}

hipError_t launch_fill_u8(void *dst, unsigned char v, size_t n, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u8, dim3(grid_for(n)), dim3(kBlock), 0, s, (unsigned char *)dst, v,
                       n);
    return hipGetLastError();
}

hipError_t launch_pad_rows_i8(const signed char *src, signed char *dst, int m, int K, int KT,
                              hipStream_t s)
{
    const size_t total = (size_t)m * KT;
    if (total == 0) return hipSuccess;
    hipLaunchKernelGGL(k_pad_rows<signed char>, dim3(grid_for(total)), dim3(kBlock), 0, s, src,
                       dst, m, K, KT);
    return hipGetLastError();
}

}  // namespace mmgap
