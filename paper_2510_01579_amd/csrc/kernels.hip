// Device code of the Ising hot path (gfx950 / CDNA4, wave64).
//
//  * k_det_build / k_vpp_build -- pre-processing: the Ising couplings G and
//    fields f of every instance (paper §3.2 pre-processing kernel; §3.3 for the
//    vector-perturbation rewriting) and the linear fallback (§2.1 MMSE).
//  * k_anneal<KT,Q>            -- the solver: one single-spin-flip Metropolis
//    anneal per lane, 64 anneals of one instance per wavefront (paper §3.2:
//    one anneal per thread, no synchronisation between anneals).
//  * k_select                  -- post-processing: best anneal per instance,
//    fallback rule, decode and float64 metrics (paper §3.2 post-processing).
//
// Floating point: float32 chain state with round-to-nearest and no implicit
// contraction (this file is compiled with -ffp-contract=off and the pragma
// below).  Fused multiply-adds appear only where written as fmaf(); each one
// is either part of the arithmetic contract (field rows, energies) or has an
// exact product, so that it equals the separately rounded form.
#include <hip/hip_runtime.h>
#include <stdint.h>

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
        const uint32_t n0 = (uint32_t)(pb >> 32) ^ c[1] ^ k0;
        const uint32_t n2 = (uint32_t)(pa >> 32) ^ c[3] ^ k1;
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

// ---------------------------------------------------------------------------
// Detection build: one workgroup per subcarrier.
//   Cg = H^H H (float64, upper triangle, mirrored)      -> G (real form, x c^2)
//   F  = H^H y per symbol                               -> f (real form, x c)
//   MMSE (Cg + sigma^2 I)^-1 F by LDL^H, sliced to the nearest PAM level.
__global__ void __launch_bounds__(kBlock) k_det_build(DetBuildArgs a)
{
    __shared__ float2 Hs[64 * 16];
    __shared__ double2 Cg[16 * 16];
    __shared__ double2 Fs[64 * 16];
    __shared__ double2 Ls[16 * 16];
    __shared__ double ds[16];

    const int sc = blockIdx.x;
    const int tid = threadIdx.x;
    const int nr = a.n_r, nt = a.n_t, K = 2 * nt, ld = a.ld, nsym = a.n_sym;

    const float2 *Hg = a.H + (size_t)sc * nr * nt;
    for (int e = tid; e < nr * nt; e += kBlock) Hs[e] = Hg[e];
    __syncthreads();

    float *Gs = a.G + (size_t)sc * ld * ld;
    // padding rows / columns of G
    for (int e = tid; e < ld * ld; e += kBlock) {
        const int r = e / ld, c = e % ld;
        if (r >= K || c >= K) Gs[e] = 0.0f;
    }
    const int npair = nt * (nt + 1) / 2;
    for (int p = tid; p < npair; p += kBlock) {
        int ia, ib;
        upper_pair(p, nt, ia, ib);
        double re = 0.0, im = 0.0;
        for (int r = 0; r < nr; ++r) {
            const float2 h1 = Hs[r * nt + ia], h2 = Hs[r * nt + ib];
            const double ar = h1.x, ai = h1.y, br = h2.x, bi = h2.y;
            const double pre = ar * br + ai * bi;   // conj(h1) h2
            const double pim = ar * bi - ai * br;
            re = re + pre;
            im = im + pim;
        }
        if (ia == ib) im = 0.0;
        Cg[ia * 16 + ib] = make_double2(re, im);
        Cg[ib * 16 + ia] = make_double2(re, 0.0 - im);
        const float gre = (float)(a.c2 * re);
        const float gim = (float)(a.c2 * im);
        const float ngim = (float)(a.c2 * (0.0 - im));
        Gs[ia * ld + ib] = gre;
        Gs[ib * ld + ia] = gre;
        Gs[(nt + ia) * ld + (nt + ib)] = gre;
        Gs[(nt + ib) * ld + (nt + ia)] = gre;
        // upper-right block -Im Cg, lower-left block Im Cg
        Gs[ia * ld + (nt + ib)] = ngim;
        Gs[(nt + ib) * ld + ia] = ngim;
        Gs[(nt + ia) * ld + ib] = gim;
        Gs[ib * ld + (nt + ia)] = gim;
    }

    // fields
    for (int p = tid; p < nsym * nt; p += kBlock) {
        const int sym = p / nt, ia = p % nt;
        const float2 *ys = a.y + ((size_t)sc * nsym + sym) * nr;
        double re = 0.0, im = 0.0;
        for (int r = 0; r < nr; ++r) {
            const float2 h = Hs[r * nt + ia];
            const float2 yv = ys[r];
            const double pre = (double)h.x * (double)yv.x + (double)h.y * (double)yv.y;
            const double pim = (double)h.x * (double)yv.y - (double)h.y * (double)yv.x;
            re = re + pre;
            im = im + pim;
        }
        Fs[sym * 16 + ia] = make_double2(re, im);
        float *fs = a.f + ((size_t)sc * nsym + sym) * ld;
        fs[ia] = (float)(a.c * re);
        fs[nt + ia] = (float)(a.c * im);
    }
    for (int p = tid; p < nsym * (ld - K); p += kBlock) {
        const int sym = p / (ld - K), k = K + p % (ld - K);
        a.f[((size_t)sc * nsym + sym) * ld + k] = 0.0f;
    }
    if (a.ynorm) {
        for (int sym = tid; sym < nsym; sym += kBlock) {
            const float2 *ys = a.y + ((size_t)sc * nsym + sym) * nr;
            double acc = 0.0;
            for (int r = 0; r < nr; ++r) {
                const double yr = ys[r].x, yi = ys[r].y;
                acc = acc + (yr * yr + yi * yi);
            }
            a.ynorm[(size_t)sc * nsym + sym] = acc;
        }
    }
    if (!a.x_fb) return;   // uniform over the block
    __syncthreads();

    // LDL^H of Cg + sigma^2 I
    for (int j = 0; j < nt; ++j) {
        if (tid == 0) {
            double dj = Cg[j * 16 + j].x + a.noise_var;
            for (int k = 0; k < j; ++k) {
                const double2 v = Ls[j * 16 + k];
                double t = v.x * v.x + v.y * v.y;
                t = t * ds[k];
                dj = dj - t;
            }
            ds[j] = dj;
        }
        __syncthreads();
        for (int i = j + 1 + tid; i < nt; i += kBlock) {
            cd s = ld2(Cg[i * 16 + j]);
            for (int k = 0; k < j; ++k) {
                cd v = cmulc(ld2(Ls[j * 16 + k]), ld2(Ls[i * 16 + k]));
                v.re = v.re * ds[k];
                v.im = v.im * ds[k];
                s.re = s.re - v.re;
                s.im = s.im - v.im;
            }
            Ls[i * 16 + j] = make_double2(s.re / ds[j], s.im / ds[j]);
        }
        __syncthreads();
    }
    // per-symbol solves in place on Fs, then slicing
    for (int sym = tid; sym < nsym; sym += kBlock) {
        double2 *w = Fs + sym * 16;
        for (int i = 0; i < nt; ++i) {
            cd s = ld2(w[i]);
            for (int k = 0; k < i; ++k) {
                const cd v = cmul(ld2(Ls[i * 16 + k]), ld2(w[k]));
                s.re = s.re - v.re;
                s.im = s.im - v.im;
            }
            w[i] = st2(s);
        }
        for (int i = 0; i < nt; ++i) w[i] = make_double2(w[i].x / ds[i], w[i].y / ds[i]);
        for (int i = nt - 1; i >= 0; --i) {
            cd s = ld2(w[i]);
            for (int k = i + 1; k < nt; ++k) {
                const cd v = cmulc(ld2(Ls[k * 16 + i]), ld2(w[k]));
                s.re = s.re - v.re;
                s.im = s.im - v.im;
            }
            w[i] = st2(s);
        }
        signed char *xo = a.x_fb + ((size_t)sc * nsym + sym) * ld;
        for (int i = 0; i < nt; ++i) {
            const double tr = w[i].x / a.c, ti = w[i].y / a.c;
            double lr = 2.0 * floor(tr / 2.0) + 1.0;
            double li = 2.0 * floor(ti / 2.0) + 1.0;
            lr = fmin(fmax(lr, (double)-a.qtop), (double)a.qtop);
            li = fmin(fmax(li, (double)-a.qtop), (double)a.qtop);
            if (lr != lr) lr = 1.0;   // NaN input: any valid level
            if (li != li) li = 1.0;
            xo[i] = (signed char)(int)lr;
            xo[nt + i] = (signed char)(int)li;
        }
        for (int k = K; k < ld; ++k) xo[k] = 0;
    }
}

// ---------------------------------------------------------------------------
// VPP build: one workgroup per subcarrier.  A = H H^H, its LDL^H, M = L^-1 and
// A^-1 = M^H D^-1 M in a fixed operation order (so that any implementation of
// the same sequence agrees bit for bit), then
//   G = (tau/2)^2 Re-form(A^-1),  f = -(tau/2) Re-form(A^-1 u).
__global__ void __launch_bounds__(kBlock) k_vpp_build(VppBuildArgs a)
{
    __shared__ float2 Hs[16 * 64];
    __shared__ double2 As[16 * 16];
    __shared__ double2 Ls[16 * 16];
    __shared__ double2 Ms[16 * 16];
    __shared__ double2 Zs[16 * 16];   // A^-1
    __shared__ double ds[16];

    const int sc = blockIdx.x;
    const int tid = threadIdx.x;
    const int n = a.n_u, ntx = a.n_t, K = 2 * n, ld = a.ld, nsym = a.n_sym;
    const double ht = 0.5 * a.tau;
    const double sg = ht * ht;
    const double sf = -ht;

    const float2 *Hg = a.H + (size_t)sc * n * ntx;
    for (int e = tid; e < n * ntx; e += kBlock) Hs[e] = Hg[e];
    __syncthreads();

    // A_il = sum_j H_ij conj(H_lj), i >= l
    const int npair = n * (n + 1) / 2;
    for (int p = tid; p < npair; p += kBlock) {
        int l, i;
        upper_pair(p, n, l, i);   // l <= i
        double re = 0.0, im = 0.0;
        for (int j = 0; j < ntx; ++j) {
            const double ar = Hs[i * ntx + j].x, ai = Hs[i * ntx + j].y;
            const double cr = Hs[l * ntx + j].x, ci = Hs[l * ntx + j].y;
            const double pre = ar * cr + ai * ci;
            const double pim = ai * cr - ar * ci;
            re = re + pre;
            im = im + pim;
        }
        As[i * 16 + l] = make_double2(re, im);
        As[l * 16 + i] = make_double2(re, -im);
    }
    __syncthreads();

    for (int j = 0; j < n; ++j) {
        if (tid == 0) {
            double dj = As[j * 16 + j].x;
            for (int k = 0; k < j; ++k) {
                const double2 v = Ls[j * 16 + k];
                double t = v.x * v.x + v.y * v.y;
                t = t * ds[k];
                dj = dj - t;
            }
            ds[j] = dj;
        }
        __syncthreads();
        for (int i = j + 1 + tid; i < n; i += kBlock) {
            cd s = ld2(As[i * 16 + j]);
            for (int k = 0; k < j; ++k) {
                cd v = cmulc(ld2(Ls[j * 16 + k]), ld2(Ls[i * 16 + k]));
                v.re = v.re * ds[k];
                v.im = v.im * ds[k];
                s.re = s.re - v.re;
                s.im = s.im - v.im;
            }
            Ls[i * 16 + j] = make_double2(s.re / ds[j], s.im / ds[j]);
        }
        __syncthreads();
    }
    // M = L^-1, one column per thread
    for (int m = tid; m < n; m += kBlock) {
        Ms[m * 16 + m] = make_double2(1.0, 0.0);
        for (int i = m + 1; i < n; ++i) {
            cd s{0.0, 0.0};
            for (int k = m; k < i; ++k) {
                const cd v = cmul(ld2(Ls[i * 16 + k]), ld2(Ms[k * 16 + m]));
                s.re = s.re + v.re;
                s.im = s.im + v.im;
            }
            Ms[i * 16 + m] = make_double2(-s.re, -s.im);
        }
    }
    __syncthreads();
    // A^-1_il = sum_{k>=i} conj(M_ki) M_kl / d_k, i >= l
    for (int p = tid; p < npair; p += kBlock) {
        int l, i;
        upper_pair(p, n, l, i);
        cd acc{0.0, 0.0};
        for (int k = i; k < n; ++k) {
            cd v = cmulc(ld2(Ms[k * 16 + i]), ld2(Ms[k * 16 + l]));
            v.re = v.re / ds[k];
            v.im = v.im / ds[k];
            acc.re = acc.re + v.re;
            acc.im = acc.im + v.im;
        }
        Zs[i * 16 + l] = st2(acc);
        if (i != l) Zs[l * 16 + i] = make_double2(acc.re, -acc.im);
        else Zs[i * 16 + i] = make_double2(acc.re, -acc.im);
    }
    __syncthreads();

    if (a.Ainv) {
        double2 *Ag = a.Ainv + (size_t)sc * n * n;
        for (int e = tid; e < n * n; e += kBlock) Ag[e] = Zs[(e / n) * 16 + (e % n)];
    }
    float *Gs = a.G + (size_t)sc * ld * ld;
    for (int e = tid; e < ld * ld; e += kBlock) {
        const int r = e / ld, c = e % ld;
        float v = 0.0f;
        if (r < K && c < K) {
            const int i = r % n, l = c % n;
            const double2 z = Zs[i * 16 + l];
            if ((r < n) == (c < n)) v = (float)(sg * z.x);
            else if (r < n) v = (float)(sg * (-z.y));   // upper-right: -Im
            else v = (float)(sg * z.y);                 // lower-left: Im
        }
        Gs[e] = v;
    }
    for (int p = tid; p < nsym * n; p += kBlock) {
        const int sym = p / n, i = p % n;
        const float2 *us = a.u + ((size_t)sc * nsym + sym) * n;
        cd z{0.0, 0.0};
        for (int l = 0; l < n; ++l) {
            const cd ul{(double)us[l].x, (double)us[l].y};
            const cd v = cmul(ld2(Zs[i * 16 + l]), ul);
            z.re = z.re + v.re;
            z.im = z.im + v.im;
        }
        float *fs = a.f + ((size_t)sc * nsym + sym) * ld;
        fs[i] = (float)(sf * z.re);
        fs[n + i] = (float)(sf * z.im);
    }
    for (int p = tid; p < nsym * (ld - K); p += kBlock) {
        const int sym = p / (ld - K), k = K + p % (ld - K);
        a.f[((size_t)sc * nsym + sym) * ld + k] = 0.0f;
    }
    if (a.x_fb) {
        for (int p = tid; p < nsym * ld; p += kBlock) a.x_fb[(size_t)sc * nsym * ld + p] = 0;
    }
    if (a.unorm) {
        for (int sym = tid; sym < nsym; sym += kBlock) {
            const float2 *us = a.u + ((size_t)sc * nsym + sym) * n;
            double acc = 0.0;
            for (int i = 0; i < n; ++i) {
                cd z{0.0, 0.0};
                for (int l = 0; l < n; ++l) {
                    const cd v = cmul(ld2(Zs[i * 16 + l]), cd{(double)us[l].x, (double)us[l].y});
                    z.re = z.re + v.re;
                    z.im = z.im + v.im;
                }
                acc = acc + ((double)us[i].x * z.re + (double)us[i].y * z.im);
            }
            a.unorm[(size_t)sc * nsym + sym] = acc;
        }
    }
}

// ---------------------------------------------------------------------------
// The anneal.  One wavefront = 64 anneals (chains) of one instance; chains
// >= 64 use several wavefronts.  G and f of the instance are wave-uniform and
// read through the scalar cache one row ahead of use.  Per lane the state is
// the flip step of every spin, d_i = -2 w_b s_i (+-2w_b as float), and the
// levels x[KT]; the local field of a dimension is recomputed from the levels
// when the sweep reaches it (one row of G x - f) and moved by G_kk d after an
// accepted flip inside the dimension.
//
// Per attempt on spin i = k Q + b with h = g_k + (d/2) G_kk:
//   2h = (g_k + g_k) + d G_kk exactly, and 64 beta2 dE = (128 beta2 d) h,
//   the Metropolis threshold index is floor(64 beta2 dE) clamped to [0, 1024],
//   and the flip is accepted iff the 16-bit draw m < T[index] (T in LDS).

// Hides a pointer's value from the optimiser so that loads through it are
// issued where written (here: one dimension ahead) instead of being hoisted
// out of the sweep loop into registers.  The result lives in the constant
// address space, so wave-uniform loads through it use the scalar cache.
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

template <int KT, int Q>
__global__ void __launch_bounds__(kBlock)
k_anneal(const float *__restrict__ G, int inst_per_G, const float *__restrict__ f,
         const signed char *__restrict__ x_fb, const float *__restrict__ beta2,
         const uint32_t *__restrict__ accept_table, int sweeps, int chains, int n_inst, int w0,
         int w1, int w2, int w3, uint32_t key0, uint32_t key1, int init_mode,
         float *__restrict__ chain_E, uint32_t *__restrict__ chain_S)
{
    constexpr int N = KT * Q;
    constexpr int NW = (N + 31) / 32;
    constexpr int NG = (N + 7) / 8;
    // Spin state: one float flip step per spin when few spins, else one bit per
    // spin (set = spin -1) so that large problems keep enough wavefronts
    // resident; both hold the same values.
    constexpr bool kBits = N > 48 || KT == 32;
    constexpr int ND = kBits ? 1 : N;
    constexpr int NB = kBits ? NW : 1;
    __shared__ uint32_t T[kAcceptSteps + 1];
    for (int e = threadIdx.x; e <= kAcceptSteps; e += kBlock) T[e] = accept_table[e];
    __syncthreads();

    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int wpi = (chains + 63) >> 6;
    const int gw = blockIdx.x * kWavesPerBlock + wave;
    const int inst = gw / wpi;
    if (inst >= n_inst) return;
    const int ch = (gw - inst * wpi) * 64 + lane;
    const float *__restrict__ Gi = G + (size_t)(inst / inst_per_G) * (KT * KT);
    const float *__restrict__ fi = f + (size_t)inst * KT;
    const int wts[4] = {w0, w1, w2, w3};
    float two_w[Q];
#pragma unroll
    for (int b = 0; b < Q; ++b) two_w[b] = (float)(2 * wts[b]);

    const uint32_t uch = (uint32_t)ch;
    const uint32_t uinst = (uint32_t)inst;

    // flip steps d_i = -2 w_b s_i of the initial spins (or their sign bits)
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
    if (init_mode == 1 && x_fb != nullptr) {
        const signed char *xi = x_fb + (size_t)inst * KT;
#pragma unroll
        for (int k = 0; k < KT; ++k) {
            int rem = xi[k];
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
            return ((sb[i >> 5] >> (i & 31)) & 1u) ? two_w[i % Q] : -two_w[i % Q];
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
        const float bd = 128.0f * beta2[t];            // exact: power-of-two scale
        uint32_t r[4] = {0u, 0u, 0u, 0u};
        // rows of G in scalar registers; with KT <= 16 the next row is loaded
        // one dimension ahead, with KT = 32 two rows do not fit the SGPR file
        constexpr bool kPrefetch = KT <= 16;
        float grow[KT];
        float fk = 0.0f;
        if (kPrefetch) {
            cfloat *base = opaque(Gi);
#pragma unroll
            for (int l = 0; l < KT; ++l) grow[l] = base[l];
            fk = opaque(fi)[0];
        }
#pragma unroll
        for (int k = 0; k < KT; ++k) {
            if (!kPrefetch) {
                cfloat *base = opaque(Gi);
#pragma unroll
                for (int l = 0; l < KT; ++l) grow[l] = base[k * KT + l];
                fk = opaque(fi)[k];
            }
            // local field of dimension k from the current levels
            float g = -fk;
#pragma unroll
            for (int l = 0; l < KT; ++l) g = fmaf(grow[l], x[l], g);
            const float gkk = grow[k];
            const float gkh = 0.5f * gkk;                  // exact
            if (kPrefetch && k + 1 < KT) {                 // next row, issued early
                cfloat *base = opaque(Gi);
#pragma unroll
                for (int l = 0; l < KT; ++l) grow[l] = base[(k + 1) * KT + l];
                fk = opaque(fi)[k + 1];
            }
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

    // final state: energy sum_k x_k (g_k - f_k) with fresh fields
    float E = 0.0f;
#pragma unroll
    for (int k = 0; k < KT; ++k) {
        float acc = -fi[k];
#pragma unroll
        for (int l = 0; l < KT; ++l) acc = fmaf(Gi[k * KT + l], x[l], acc);
        const float diff = acc - fi[k];
        E = fmaf(x[k], diff, E);
    }
    if (ch < chains) {
        const size_t o = (size_t)inst * chains + ch;
        chain_E[o] = E;
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
            chain_S[o * NW + w] = word;
        }
    }
}

// ---------------------------------------------------------------------------
// Selection, fallback and decode.  One wavefront per instance.
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

__global__ void __launch_bounds__(kBlock) k_select(SelectArgs a)
{
    __shared__ float terms[kWavesPerBlock][32];
    __shared__ int lvs[kWavesPerBlock][32];
    __shared__ double2 zsh[kWavesPerBlock][16];

    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int n = blockIdx.x * kWavesPerBlock + wave;
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

    const float *Gi = a.G + (size_t)(n / a.inst_per_G) * KT * KT;
    const float *fi = a.f + (size_t)n * KT;
    bool use_fb = false;
    float Efb = 0.0f;
    if (a.x_fb) {
        const signed char *xi = a.x_fb + (size_t)n * KT;
        if (lane < K) {
            float acc = -fi[lane];
            for (int l = 0; l < K; ++l) acc = fmaf(Gi[lane * KT + l], (float)xi[l], acc);
            terms[wave][lane] = acc - fi[lane];
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        float e = 0.0f;
        for (int k = 0; k < K; ++k) e = fmaf((float)xi[k], terms[wave][k], e);
        Efb = e;
        use_fb = energy_less(Efb, Eb);
    }
    // winning levels into LDS
    if (lane < K) {
        int lv;
        if (use_fb) {
            lv = a.x_fb[(size_t)n * KT + lane];
        } else {
            const uint32_t *S = a.chain_S + ((size_t)n * C + bch) * NW;
            lv = 0;
            for (int b = 0; b < q; ++b) {
                const int i = lane * q + b;
                lv += ((S[i >> 5] >> (i & 31)) & 1u) ? -a.w[b] : a.w[b];
            }
        }
        lvs[wave][lane] = lv;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

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
                const uint32_t *S = a.chain_S + ((size_t)n * C + bch) * NW;
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

    const int nsym = a.n_sym;
    const int sc = n / nsym, sy = n % nsym;
    if (a.mode == kSelectDet) {
        const int nt = a.n_cols, nr = a.n_rows;
        const int qtop = (1 << q) - 1;
        if (lane < nt) {
            const int pI = (lvs[wave][lane] + qtop) >> 1;
            const int pQ = (lvs[wave][nt + lane] + qtop) >> 1;
            const int gI = pI ^ (pI >> 1), gQ = pQ ^ (pQ >> 1);
            a.sym_out[(size_t)n * nt + lane] = (unsigned char)((gI << q) | gQ);
        }
        if (a.metric_out) {
            double part = 0.0;
            for (int r = lane; r < nr; r += 64) {
                const float2 *Hr = a.H + ((size_t)sc * nr + r) * nt;
                const float2 yv = a.y[((size_t)sc * nsym + sy) * nr + r];
                double re = yv.x, im = yv.y;
                for (int t = 0; t < nt; ++t) {
                    const double xr = a.c * (double)lvs[wave][t];
                    const double xi = a.c * (double)lvs[wave][nt + t];
                    const double hr = Hr[t].x, hi = Hr[t].y;
                    re = re - (hr * xr - hi * xi);
                    im = im - (hr * xi + hi * xr);
                }
                part = part + (re * re + im * im);
            }
            const double tot = wave_sum_f64(part);
            if (lane == 0) a.metric_out[n] = (float)tot;
        }
        return;
    }

    // VPP: v = level / 2; x = H^H A^-1 (u + tau v); gamma = ||x||^2
    const int nu = a.n_rows, ntx = a.n_cols;
    if (lane < K) a.v_out[(size_t)n * K + lane] = (signed char)(lvs[wave][lane] / 2);
    if (a.x_out || a.gamma_out) {
        const double2 *Z = a.Ainv + (size_t)sc * nu * nu;
        const float2 *us = a.y + ((size_t)sc * nsym + sy) * nu;
        if (lane < nu) {
            double zr = 0.0, zi = 0.0;
            for (int l = 0; l < nu; ++l) {
                const double pr = (double)us[l].x + a.tau * (double)(lvs[wave][l] / 2);
                const double pi = (double)us[l].y + a.tau * (double)(lvs[wave][nu + l] / 2);
                const double2 zz = Z[lane * nu + l];
                zr = zr + (zz.x * pr - zz.y * pi);
                zi = zi + (zz.x * pi + zz.y * pr);
            }
            zsh[wave][lane] = make_double2(zr, zi);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        double part = 0.0;
        for (int j = lane; j < ntx; j += 64) {
            double xr = 0.0, xi = 0.0;
            for (int i = 0; i < nu; ++i) {
                const float2 h = a.H[((size_t)sc * nu + i) * ntx + j];
                const double2 z = zsh[wave][i];
                // conj(H_ij) z_i
                xr = xr + ((double)h.x * z.x + (double)h.y * z.y);
                xi = xi + ((double)h.x * z.y - (double)h.y * z.x);
            }
            if (a.x_out) a.x_out[(size_t)n * ntx + j] = make_float2((float)xr, (float)xi);
            part = part + (xr * xr + xi * xi);
        }
        const double tot = wave_sum_f64(part);
        if (lane == 0 && a.gamma_out) a.gamma_out[n] = (float)tot;
    }
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
    const int wpi = (a.chains + 63) / 64;
    const size_t waves = (size_t)a.n_inst * wpi;
    const size_t blocks = (waves + kWavesPerBlock - 1) / kWavesPerBlock;
    if (blocks == 0) return hipSuccess;
    if (blocks > 0x7FFFFFFFull) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_anneal<KT, Q>), dim3((unsigned)blocks), dim3(kBlock), 0, s, a.G,
                       a.inst_per_G, a.f, a.x_fb, a.beta2, a.accept_table, a.sweeps, a.chains,
                       a.n_inst, a.w[0], a.w[1], a.w[2], a.w[3], a.key0, a.key1, a.init_mode,
                       a.chain_E, a.chain_S);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_det_build(const DetBuildArgs &a, hipStream_t s)
{
    if (a.n_sc <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_det_build, dim3(a.n_sc), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_vpp_build(const VppBuildArgs &a, hipStream_t s)
{
    if (a.n_sc <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_vpp_build, dim3(a.n_sc), dim3(kBlock), 0, s, a);
    return hipGetLastError();
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
#undef MMGAP_ANNEAL_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_select(const SelectArgs &a, hipStream_t s)
{
    if (a.n_inst <= 0) return hipSuccess;
    const int blocks = (a.n_inst + kWavesPerBlock - 1) / kWavesPerBlock;
    hipLaunchKernelGGL(k_select, dim3(blocks), dim3(kBlock), 0, s, a);
    return hipGetLastError();
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
