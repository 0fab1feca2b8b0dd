// lpb_eval_dev.h -- device helpers shared by the evaluation kernels: Bessel
// ratios (FP64), block -> work schedules, and the 16x16x4 matrix-core
// product of a swizzled operator with a staged source block.
#pragma once
#include <hip/hip_runtime.h>

#include "lpb_eval.h"

namespace lpb {

// Bessel ratios g_n = it_n(lam r) / it_n(lam h), n = 0..p (double)
__device__ inline void bessel_ratio(int p, double lam, double r2, const double* __restrict__ inv_ith, double* g)
{
    itilde_all(p, lam * lam * r2, g);
    for (int n = 0; n <= p; ++n) g[n] *= inv_ith[n];
}

// Bessel-ratio tables (FP64, built on the host): A.bes_tab[LPB_TB_REC + n] =
// 1/((2n+1)(2n+3)), A.bes_tab[LPB_TB_S0 + k] = 1/(2k(2p+2k+1)),
// A.bes_tab[LPB_TB_S1 + k] = 1/(2k(2p+2k+3)), and per FMM and level
// 1/it_n(lam h) (A.ith_s for the source-side lambda, A.ith_t for the target side).
#define LPB_NSER 40
#define LPB_TB_REC 0
#define LPB_TB_S0 (LPB_MAX_P + 2)
#define LPB_TB_S1 (LPB_TB_S0 + LPB_NSER + 1)
#define LPB_TB_SIZE (LPB_TB_S1 + LPB_NSER + 1)

// it_N(x) series with the tabulated factors (t = x^2); large arguments (boxes
// much wider than the Debye length) continue with the explicit factors
__device__ inline double itilde_series_tab(double t, const double* f, int N)
{
    double term = 1.0, sum = 1.0;
    for (int k = 1; k <= LPB_NSER; ++k) {
        term *= t * f[k];
        sum += term;
        if (term <= 1e-17 * sum) return sum;
    }
    for (int k = LPB_NSER + 1; k < 4000; ++k) {
        term *= 0.5 * t / ((double)k * (2.0 * N + 2.0 * k + 1.0));
        sum += term;
        if (term <= 1e-17 * sum) break;
    }
    return sum;
}

// g_n = it_n(lam r)/it_n(lam h) * scale, n = 0..p, written to out[n * stride];
// tb: the p-dependent tables, ith: 1/it_n(lam h) of the box level
template <typename T>
__device__ inline void bessel_ratio_col(int p, double t, const double* __restrict__ tb, const double* __restrict__ ith,
                                        T scale, T* out, int stride)
{
    double a = itilde_series_tab(t, tb + LPB_TB_S1, p + 1), bb = itilde_series_tab(t, tb + LPB_TB_S0, p);
    out[(size_t)p * stride] = (T)(bb * ith[p]) * scale;
    for (int n = p; n >= 1; --n) {
        double c = bb + t * a * tb[LPB_TB_REC + n];
        out[(size_t)(n - 1) * stride] = (T)(c * ith[n - 1]) * scale;
        a = bb;
        bb = c;
    }
}


// ---------------------------------------------------------------------------
// Tiled free-space M2L on the matrix cores.  A tile is 64 target boxes of one
// (FMM, level) that share a child octant inside a 4x4x4 block of parents, so
// all of them have the same 189 V-list offsets d and operators A_d.  For each
// d the tile computes  L[:, tile] += A_d * M[:, tile + d]  as a (KP x KP) x
// (KP x 64) product with 16x16x4 MFMA (FP32 or FP64), the 64 gathered source
// expansions staged in LDS, the operator streamed from memory in the MFMA
// operand layout.  Four waves split the 16-row blocks of the output; results
// accumulate in registers over all 189 offsets and are added to LE once.
// Block -> work item: schedule 0 is linear; schedule 1 gives the blocks of one
// XCD (blocks are dispatched round robin over the 8 XCDs) a contiguous run of
// work items, so items that share operators share that XCD's L2.  Both are
// bijections of [0, n), so results do not depend on the schedule.
__device__ inline int sched_index(int b, int n, int sched)
{
    if (sched == 0) return b;
    const int x = b & 7, k = b >> 3, q = n >> 3, r = n & 7;
    return x * q + min(x, r) + k;
}

template <typename T> struct Vec4;
template <> struct Vec4<float> { typedef float type __attribute__((ext_vector_type(4))); };
template <> struct Vec4<double> { typedef double type __attribute__((ext_vector_type(4))); };
template <typename T> struct Vec2;
template <> struct Vec2<float> { typedef float type __attribute__((ext_vector_type(2))); };
template <> struct Vec2<double> { typedef double type __attribute__((ext_vector_type(2))); };

__device__ inline Vec4<float>::type mfma16(float a, float b, Vec4<float>::type c)
{
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ inline Vec4<double>::type mfma16(double a, double b, Vec4<double>::type c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
// output row (within a 16x16 block) of accumulator element r in lane l
__device__ inline int mfma_row(float, int l, int r) { return 4 * (l >> 4) + r; }
__device__ inline int mfma_row(double, int l, int r) { return (l >> 4) + 4 * r; }

// acc[rb][cb] = A (rows 16 (w RB + rb) ..) x B (LDS, columns 16 cb ..), with
// A in the swizzled operand layout (16-column slabs of A load two slabs
// ahead of the one being multiplied)
template <typename T, int RB, int CB>
__device__ __attribute__((always_inline)) inline void mma_block(const T* __restrict__ Aw, const T* Bs, int NTP, int KB, int w, int l,
                                 typename Vec4<T>::type (&acc)[RB][CB])
{
    typedef typename Vec4<T>::type V4;
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) acc[rb][cb] = V4{0, 0, 0, 0};
    // row blocks past KB (their rows are >= K, never stored) are skipped: the
    // test is wave-uniform
    auto load = [&](V4 (&a)[RB], int s4) {
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
            const int rbg = min(w * RB + rb, KB - 1);
            if (w * RB + rb < KB) a[rb] = *reinterpret_cast<const V4*>(Aw + (((size_t)rbg * KB + min(s4, KB - 1)) * 64 + l) * 4);
        }
    };
    auto slab = [&](const V4 (&a4)[RB], int s4) {
#pragma unroll
        for (int ss = 0; ss < 4; ++ss) {
            const int kk = 16 * s4 + 4 * ss + (l >> 4);
            T b[CB];
#pragma unroll
            for (int cb = 0; cb < CB; ++cb) b[cb] = Bs[kk * NTP + cb * 16 + (l & 15)];
#pragma unroll
            for (int rb = 0; rb < RB; ++rb)
                if (w * RB + rb < KB) {
#pragma unroll
                    for (int cb = 0; cb < CB; ++cb) acc[rb][cb] = mfma16(a4[rb][ss], b[cb], acc[rb][cb]);
                }
        }
    };
    V4 a0[RB], a1[RB];
    load(a0, 0);
    load(a1, 1);
    for (int s4 = 0; s4 < KB; s4 += 2) {
        V4 c[RB];
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) c[rb] = a0[rb];
        load(a0, s4 + 2);
        slab(c, s4);
        if (s4 + 1 < KB) {
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) c[rb] = a1[rb];
            load(a1, s4 + 3);
            slab(c, s4 + 1);
        }
    }
}

// tot += acc, compensated (Kahan) in FP32 so that a sum over many terms keeps
// the error of a single product
template <typename T, int RB, int CB>
__device__ __attribute__((always_inline)) inline void accumulate(const typename Vec4<T>::type (&acc)[RB][CB], typename Vec4<T>::type (&tot)[RB][CB],
                                  typename Vec4<T>::type (&cmp)[RB][CB])
{
    typedef typename Vec4<T>::type V4;
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) {
            if (sizeof(T) == 4) {
                V4 y = acc[rb][cb] - cmp[rb][cb];
                V4 t = tot[rb][cb] + y;
                cmp[rb][cb] = (t - tot[rb][cb]) - y;
                tot[rb][cb] = t;
            } else {
                tot[rb][cb] += acc[rb][cb];
            }
        }
}


}  // namespace lpb
