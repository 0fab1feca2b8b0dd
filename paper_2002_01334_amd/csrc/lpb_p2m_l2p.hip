// lpb_p2m_l2p.hip -- P2M and L2P with the expansion order fixed at compile
// time (FP32 path, 2 <= p <= 15), and their launchers.
#include <hip/hip_runtime.h>

#include "lpb_eval_dev.h"

namespace lpb {

// ---------------------------------------------------------------------------
// P2M and L2P with the order P fixed at compile time (FP32 path, 2 <= P <= 15):
// one lane per charge, half a wave per leaf, the Bessel ratios and every
// solid harmonic in registers (fully unrolled recurrences, table coefficients
// read at uniform addresses); P2M reduces the lanes' coefficient rows through
// LDS once per pair of leaves, 64 coefficients at a time.
template <int P>
__device__ inline void bessel_ratio_reg(double t, const double* __restrict__ tb, const double* __restrict__ ith, float scale,
                                        float (&g)[P + 1])
{
    double a = itilde_series_tab(t, tb + LPB_TB_S1, P + 1), bb = itilde_series_tab(t, tb + LPB_TB_S0, P);
    g[P] = (float)(bb * ith[P]) * scale;
#pragma unroll
    for (int n = P; n >= 1; --n) {
        double c = bb + t * a * tb[LPB_TB_REC + n];
        g[n - 1] = (float)(c * ith[n - 1]) * scale;
        a = bb;
        bb = c;
    }
}

// Recurrence coefficients of the solid harmonics as compile-time constants
// (same definitions as the host tables: A_m, alpha_nm, beta_nm)
constexpr double csqrt(double x)
{
    double r = x > 1.0 ? x : 1.0;
    for (int i = 0; i < 64; ++i) r = 0.5 * (r + x / r);
    return x > 0.0 ? r : 0.0;
}
template <int P>
struct ShTab {
    float amm[P + 1];
    float alpha[(P + 1) * (P + 2) / 2];
    float beta[(P + 1) * (P + 2) / 2];
};
template <int P>
constexpr ShTab<P> make_sh_tab()
{
    ShTab<P> t{};
    double a = 0.28209479177387814;
    for (int m = 0; m <= P; ++m) {
        if (m > 0) a *= csqrt((2.0 * m + 1.0) / (2.0 * m));
        t.amm[m] = (float)a;
        if (m + 1 <= P) t.alpha[ipk(m + 1, m)] = (float)csqrt(2.0 * m + 3.0);
        for (int n = m + 2; n <= P; ++n) {
            double nn = (double)n * n, mm = (double)m * m;
            t.alpha[ipk(n, m)] = (float)csqrt((4.0 * nn - 1.0) / (nn - mm));
            t.beta[ipk(n, m)] = (float)csqrt(((n - 1.0) * (n - 1.0) - mm) * (2.0 * n + 1.0) / ((nn - mm) * (2.0 * n - 3.0)));
        }
    }
    return t;
}

// Calls f(n, m, re, im) for every n <= P, 0 <= m <= n with R_n^m(x, y, z) = re + i im
// (r2 = x^2 + y^2 + z^2)
template <int P, typename F>
__device__ inline void solid_harmonics(float x, float y, float z, F&& f)
{
    constexpr ShTab<P> tab = make_sh_tab<P>();
    const float* amm = tab.amm;
    const float* alpha = tab.alpha;
    const float* beta = tab.beta;
    const float r2 = x * x + y * y + z * z;
    float wr = 1.f, wi = 0.f;
#pragma unroll
    for (int m = 0; m <= P; ++m) {
        if (m > 0) {
            float nr = wr * x - wi * y;
            wi = wr * y + wi * x;
            wr = nr;
        }
        float pr = amm[m] * wr, pi = amm[m] * wi;
        f(m, m, pr, pi);
        if (m + 1 <= P) {
            const float al = alpha[ipk(m + 1, m)];
            float qr = al * z * pr, qi = al * z * pi;
            f(m + 1, m, qr, qi);
#pragma unroll
            for (int n = m + 2; n <= P; ++n) {
                const float a = alpha[ipk(n, m)], b = beta[ipk(n, m)];
                float sr = a * z * qr - b * r2 * pr, si = a * z * qi - b * r2 * pi;
                f(n, m, sr, si);
                pr = qr;
                pi = qi;
                qr = sr;
                qi = si;
            }
        }
    }
}

// NL = 2 or 4 leaves per 64-lane block (a leaf holds about half or a quarter
// of a wave of sources): slot h = lane / (64 / NL) takes leaf NL blockIdx.x + h,
// its sources 64 / NL at a time; lane i then sums coefficient c0 + i of every
// slot's rows.
template <int P, int NL>
__global__ void __launch_bounds__(64) k_p2m_p(EvalArgs<float> A, int n_leaves)
{
    constexpr int K = (P + 1) * (P + 1), LPL = 64 / NL;
    __shared__ float red[64][65];
    const int lane = threadIdx.x, h = lane / LPL, hl = lane % LPL;
    const int w = NL * blockIdx.x + h;
    const bool on = w < n_leaves;
    const int leaf = on ? A.p2m_leaves[w] : A.p2m_leaves[NL * blockIdx.x];
    const FmmDev& F = A.fmm[A.sl_fmm[leaf]];
    const double* __restrict__ ith = A.ith_s + ((size_t)A.sl_fmm[leaf] * (kMaxDepth + 1) + A.sl_lv[leaf]) * (LPB_MAX_P + 1);
    const int s0 = A.sl_start[leaf], s1 = on ? A.sl_start[leaf + 1] : s0;
    const float hinv = (float)(1.0 / A.sl_h[leaf]);
    float acc[K];
#pragma unroll
    for (int k = 0; k < K; ++k) acc[k] = 0.f;
    for (int j = s0 + hl; j < s1; j += LPL) {
        const float ux = A.s_ux[j], uy = A.s_uy[j], uz = A.s_uz[j];
        const double r2d = (double)ux * ux + (double)uy * uy + (double)uz * uz;
        float g[P + 1];
        bessel_ratio_reg<P>(F.lam_s * F.lam_s * r2d, A.bes_tab, ith, A.qs[j], g);
        // Mh_nm += q g_n conj(R_n^m(u/h))
        solid_harmonics<P>(ux * hinv, uy * hinv, uz * hinv,
                           [&](int n, int m, float re, float im) {
                               acc[ire(n, m)] += g[n] * re;
                               if (m > 0) acc[iim(n, m)] -= g[n] * im;
                           });
    }
    int me[NL];
#pragma unroll
    for (int hh = 0; hh < NL; ++hh) {
        const int wh = NL * blockIdx.x + hh;
        me[hh] = wh < n_leaves ? A.sl_me[A.p2m_leaves[wh]] : -1;
    }
#pragma unroll
    for (int c0 = 0; c0 < K; c0 += 64) {
#pragma unroll
        for (int i = 0; i < 64; ++i)
            if (c0 + i < K) red[i][lane] = acc[c0 + i];
        __syncthreads();
        if (c0 + lane < K) {
#pragma unroll
            for (int hh = 0; hh < NL; ++hh) {
                float t = 0.f;
#pragma unroll 16
                for (int jj = 0; jj < LPL; ++jj) t += red[lane][hh * LPL + jj];
                if (me[hh] >= 0) A.me[(size_t)me[hh] * A.KP + c0 + lane] = t;
            }
        }
        __syncthreads();
    }
}

// NL = 2 or 4 leaves per 64-lane block (a leaf holds about half or a quarter
// of a wave of targets): slot h = lane / (64 / NL) takes leaf NL blockIdx.x + h,
// its targets 64 / NL at a time.
template <int P, int NL>
__global__ void __launch_bounds__(64) k_l2p_p(EvalArgs<float> A, int n_leaves)
{
    constexpr int K = (P + 1) * (P + 1), LPL = 64 / NL;
    __shared__ float Ls[NL][K];   // the leaves' local expansions, read at slot-uniform addresses
    const int h = threadIdx.x / LPL, hl = threadIdx.x % LPL;
    const int w = NL * blockIdx.x + h;
    const bool on = w < n_leaves;
    const int leaf = on ? A.l2p_leaves[w] : 0;
    if (on) {
        const int le = A.tl_le[leaf];
        for (int k = hl; k < K; k += LPL) Ls[h][k] = A.le[(size_t)le * A.KP + k];
    }
    __syncthreads();
    if (!on) return;
    const FmmDev& F = A.fmm[A.tl_fmm[leaf]];
    const double* __restrict__ ith = A.ith_t + ((size_t)A.tl_fmm[leaf] * (kMaxDepth + 1) + A.tl_lv[leaf]) * (LPB_MAX_P + 1);
    const int t0 = A.tl_start[leaf], t1 = A.tl_start[leaf + 1];
    const float hinv = (float)(1.0 / A.tl_h[leaf]);
    const float* L = Ls[h];
    for (int j = t0 + hl; j < t1; j += LPL) {
        const float ux = A.t_ux[j], uy = A.t_uy[j], uz = A.t_uz[j];
        const double r2d = (double)ux * ux + (double)uy * uy + (double)uz * uz;
        float g[P + 1];
        bessel_ratio_reg<P>(F.lam_t * F.lam_t * r2d, A.bes_tab, ith, 1.f, g);
        // Phi = far * sum_n g_n [Lh_n0 R_n^0 + 2 sum_{m>0} Re(Lh_nm R_n^m)]
        float phi = 0.f;
        solid_harmonics<P>(ux * hinv, uy * hinv, uz * hinv,
                           [&](int n, int m, float re, float im) {
                               // (a compiler barrier per order m keeps the LDS reads of the
                               // expansion next to their use: hoisted together they held
                               // K registers and cut the waves per SIMD from 8 to 3)
                               if (n == m) asm volatile("" ::: "memory");
                               if (m == 0) phi += g[n] * (L[ire(n, 0)] * re);
                               else phi += 2.f * g[n] * (L[ire(n, m)] * re - L[iim(n, m)] * im);
                           });
        A.parts[A.t_out[j]] = (double)phi * F.far_factor;
    }
}


void launch_p2m_fixed(const EvalArgs<float>& A, int n_leaves, int nl, hipStream_t st)
{
#define LPB_P2M(PP) \
    case PP:                                                                                                     \
        if (nl == 4) hipLaunchKernelGGL((k_p2m_p<PP, 4>), dim3((n_leaves + 3) / 4), dim3(64), 0, st, A, n_leaves); \
        else hipLaunchKernelGGL((k_p2m_p<PP, 2>), dim3((n_leaves + 1) / 2), dim3(64), 0, st, A, n_leaves);         \
        break;
    switch (A.p) {
        LPB_P2M(2) LPB_P2M(3) LPB_P2M(4) LPB_P2M(5) LPB_P2M(6) LPB_P2M(7) LPB_P2M(8) LPB_P2M(9)
        LPB_P2M(10) LPB_P2M(11) LPB_P2M(12) LPB_P2M(13) LPB_P2M(14) LPB_P2M(15)
    default: break;
    }
#undef LPB_P2M
}

void launch_l2p_fixed(const EvalArgs<float>& A, int n_leaves, int nl, hipStream_t st)
{
#define LPB_L2P(PP) \
    case PP:                                                                                                     \
        if (nl == 4) hipLaunchKernelGGL((k_l2p_p<PP, 4>), dim3((n_leaves + 3) / 4), dim3(64), 0, st, A, n_leaves); \
        else hipLaunchKernelGGL((k_l2p_p<PP, 2>), dim3((n_leaves + 1) / 2), dim3(64), 0, st, A, n_leaves);         \
        break;
    switch (A.p) {
        LPB_L2P(2) LPB_L2P(3) LPB_L2P(4) LPB_L2P(5) LPB_L2P(6) LPB_L2P(7) LPB_L2P(8) LPB_L2P(9)
        LPB_L2P(10) LPB_L2P(11) LPB_L2P(12) LPB_L2P(13) LPB_L2P(14) LPB_L2P(15)
    default: break;
    }
#undef LPB_L2P
}

}  // namespace lpb
