// lpb_eval.hip -- evaluation kernels of Algorithm 2 (every FMM of every
// system per launch): gather charges, P2M, M2M, M2L, L2L, L2P, near field
// (free-space and reaction), and the component sum.  Templated on the
// arithmetic type T (double for LPB_FP64, float for LPB_MIXED); Bessel
// ratios are always formed in double.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "lpb_eval.h"

namespace lpb {

// ---------------------------------------------------------------------------
// charges of the source slots: qs[k] = q[s_cidx[k]]
template <typename T>
__global__ void k_gather_q(int n, const int* __restrict__ cidx, const double* __restrict__ q, T* __restrict__ qs)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) qs[i] = (T)q[cidx[i]];
}

template <typename T>
__global__ void k_zero(size_t n, T* __restrict__ a)
{
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t st = (size_t)gridDim.x * blockDim.x;
    for (; i < n; i += st) a[i] = T(0);
}

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
// P2M (eqs. melecoeffree, melayerupgoingimage), scaled:
//   Mh_nm = sum_j q_j g_n(r_j) conj(R_n^m(u_j / h)),  u_j = source - box centre.
// One 64-lane block per source leaf; each lane owns a point of the current
// chunk, runs the solid-harmonic recurrence (coefficients from the tables
// sh_amm/sh_alpha/sh_beta, read at wave-uniform addresses) and writes its
// point's weighted coefficient row into LDS; then each lane sums whole
// coefficient rows over the chunk.  The Bessel ratios are formed in FP64.
template <typename T>
__global__ void __launch_bounds__(64) k_p2m(EvalArgs<T> A, int CH)
{
    extern __shared__ unsigned char smem_raw[];
    const int p = A.p, K = A.K;
    const int leaf = A.p2m_leaves[blockIdx.x];
    const int me = A.sl_me[leaf];
    const FmmDev& F = A.fmm[A.sl_fmm[leaf]];
    const double h = A.sl_h[leaf];
    const int CS = CH + 1;                                     // padded row stride
    T* coef = reinterpret_cast<T*>(smem_raw);                  // [K][CH+1]
    T* gl = coef + (size_t)K * CS;                             // [p+1][CH]
    const int lane = threadIdx.x;
    const double* __restrict__ tb = A.bes_tab;
    const double* __restrict__ ith = A.ith_s + ((size_t)A.sl_fmm[leaf] * (kMaxDepth + 1) + F.H) * (LPB_MAX_P + 1);
    const int s0 = A.sl_start[leaf], s1 = A.sl_start[leaf + 1];
    T acc[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) acc[k] = T(0);
    const T hinv = (T)(1.0 / h);
    const T* __restrict__ amm_t = A.sh_amm;
    const T* __restrict__ al_t = A.sh_alpha;
    const T* __restrict__ be_t = A.sh_beta;
    for (int base = s0; base < s1; base += CH) {
        int j = base + lane;
        if (lane < CH && j < s1) {
            T ux = A.s_ux[j], uy = A.s_uy[j], uz = A.s_uz[j], q = A.qs[j];
            double r2d = (double)ux * ux + (double)uy * uy + (double)uz * uz;
            // g_n = it_n(lam r)/it_n(lam h) (FP64), times q, into the lane's LDS column
            bessel_ratio_col<T>(p, F.lam_s * F.lam_s * r2d, tb, ith, q, gl + lane, CH);
            T x = ux * hinv, y = uy * hinv, z = uz * hinv;
            T r2 = x * x + y * y + z * z;
            T wr = T(1), wi = T(0);
            for (int m = 0; m <= p; ++m) {
                if (m > 0) {
                    T nr = wr * x - wi * y;
                    wi = wr * y + wi * x;
                    wr = nr;
                }
                T pr = amm_t[m] * wr, pi = amm_t[m] * wi;
                T gq = gl[(size_t)m * CH + lane];
                coef[(size_t)ire(m, m) * CS + lane] = gq * pr;
                if (m > 0) coef[(size_t)iim(m, m) * CS + lane] = -gq * pi;
                if (m + 1 > p) continue;
                T al = al_t[ipk(m + 1, m)];
                T qr = al * z * pr, qi = al * z * pi;
                gq = gl[(size_t)(m + 1) * CH + lane];
                coef[(size_t)ire(m + 1, m) * CS + lane] = gq * qr;
                if (m > 0) coef[(size_t)iim(m + 1, m) * CS + lane] = -gq * qi;
                for (int n = m + 2; n <= p; ++n) {
                    T a = al_t[ipk(n, m)], b = be_t[ipk(n, m)];
                    T sr = a * z * qr - b * r2 * pr;
                    T si = a * z * qi - b * r2 * pi;
                    gq = gl[(size_t)n * CH + lane];
                    coef[(size_t)ire(n, m) * CS + lane] = gq * sr;
                    if (m > 0) coef[(size_t)iim(n, m) * CS + lane] = -gq * si;
                    pr = qr;
                    pi = qi;
                    qr = sr;
                    qi = si;
                }
            }
        }
        __syncthreads();
        int cnt = min(CH, s1 - base);
#pragma unroll
        for (int kk = 0; kk < 8; ++kk) {
            int k = lane + 64 * kk;
            if (k < K) {
                T sum = T(0);
                for (int jj = 0; jj < cnt; ++jj) sum += coef[(size_t)k * CS + jj];
                acc[kk] += sum;
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int kk = 0; kk < 8; ++kk) {
        int k = lane + 64 * kk;
        if (k < K) A.me[(size_t)me * A.KP + k] = acc[kk];
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
    // row blocks past KB repeat the last one (their rows are >= K, never stored)
    auto load = [&](V4 (&a)[RB], int s4) {
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
            const int rbg = min(w * RB + rb, KB - 1);
            a[rb] = *reinterpret_cast<const V4*>(Aw + (((size_t)rbg * KB + min(s4, KB - 1)) * 64 + l) * 4);
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
#pragma unroll
                for (int cb = 0; cb < CB; ++cb) acc[rb][cb] = mfma16(a4[rb][ss], b[cb], acc[rb][cb]);
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

template <typename T, int RB>
__global__ void __launch_bounds__(256) k_m2l_tile(EvalArgs<T> A)
{
    typedef typename Vec4<T>::type V4;
    constexpr int NT = 64, CB = 4, GMAX = 4 * RB;
    constexpr int NTP = NT + (sizeof(T) == 4 ? 16 : 8);   // padded LDS row (bank spread)
    extern __shared__ unsigned char smem_raw[];
    T* Bs = reinterpret_cast<T*>(smem_raw);               // [KP][NTP]
    __shared__ int s_le[NT];
    const int K = A.K, KP = A.KP, KB = KP / 16;
    const Tile tile = A.tiles[sched_index(blockIdx.x, gridDim.x, A.tile_sched & 1)];
    const TileFL fl = A.tfl[tile.fl];
    const int nside = fl.nside;
    const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
    const int ox = (tile.octant >> 2) & 1, oy = (tile.octant >> 1) & 1, oz = tile.octant & 1;
    // per-offset products accumulate in `acc`; the sum over the 189 offsets is
    // compensated (Kahan, FP32) in `tot`/`cmp`, which keeps the FP32 error at the
    // level of a single offset's product
    V4 acc[RB][CB], tot[RB][CB], cmp[RB][CB];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) tot[rb][cb] = cmp[rb][cb] = V4{0, 0, 0, 0};
    auto tcoord = [&](int j, int& tx, int& ty, int& tz) {
        tx = 2 * (tile.px0 + (j >> 4)) + ox;
        ty = 2 * (tile.py0 + ((j >> 2) & 3)) + oy;
        tz = 2 * (tile.pz0 + (j & 3)) + oz;
    };
    if (tid < NT) {
        int tx, ty, tz;
        tcoord(tid, tx, ty, tz);
        s_le[tid] = (tx < nside && ty < nside && tz < nside)
                        ? A.grid_le[fl.grid_off + ((size_t)tx * nside + ty) * nside + tz] : -1;
    }
    __syncthreads();
    // gather role of this thread: target column gj, rows 16 i + 4 gpart .. +3
    const int gj = tid >> 2, gpart = tid & 3;
    int gtx, gty, gtz;
    tcoord(gj, gtx, gty, gtz);
    const bool gvalid = s_le[gj] >= 0;
    const int* codes = A.oct_codes + tile.octant * kVOffsets;
    V4 greg[GMAX];
    auto fetch = [&](int d) {
        const int code = codes[d];
        const int sx = gtx + code / 49 - 3, sy = gty + (code / 7) % 7 - 3, sz = gtz + code % 7 - 3;
        int me = -1;
        if (gvalid && sx >= 0 && sy >= 0 && sz >= 0 && sx < nside && sy < nside && sz < nside)
            me = A.grid_me[fl.grid_off + ((size_t)sx * nside + sy) * nside + sz];
        const T* src = A.me + (size_t)(me < 0 ? 0 : me) * KP + 4 * gpart;
#pragma unroll
        for (int i = 0; i < GMAX; ++i)
            greg[i] = (me >= 0 && i < KB) ? *reinterpret_cast<const V4*>(src + 16 * i) : V4{0, 0, 0, 0};
    };
    fetch(0);
    for (int d = 0; d < kVOffsets; ++d) {
        __syncthreads();   // every wave is done with the previous offset's B
        const int ent = A.optab[fl.optab_off + codes[d]];
        const int op = ent & ((1 << kReflShift) - 1);
        const T* sg = A.refl_sign + (size_t)(ent >> kReflShift) * KP;
#pragma unroll
        for (int i = 0; i < GMAX; ++i) {
            if (i < KB) {
#pragma unroll
                for (int e = 0; e < 4; ++e) Bs[(16 * i + 4 * gpart + e) * NTP + gj] = greg[i][e] * sg[16 * i + 4 * gpart + e];
            }
        }
        __syncthreads();
        if (d + 1 < kVOffsets) fetch(d + 1);   // next offset's sources load during this offset's products
        const T* Aw = A.pool_swz + (size_t)A.swz_index[op] * KP * KP;
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int cb = 0; cb < CB; ++cb) acc[rb][cb] = V4{0, 0, 0, 0};
        V4 an[RB];
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
            int rbg = w * RB + rb;
            an[rb] = (rbg < KB) ? *reinterpret_cast<const V4*>(Aw + ((size_t)rbg * KB * 64 + l) * 4) : V4{0, 0, 0, 0};
        }
        for (int s4 = 0; s4 < KB; ++s4) {
            V4 a4[RB];
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) {
                a4[rb] = an[rb];
                int rbg = w * RB + rb;
                if (rbg < KB && s4 + 1 < KB)
                    an[rb] = *reinterpret_cast<const V4*>(Aw + (((size_t)rbg * KB + s4 + 1) * 64 + l) * 4);
            }
#pragma unroll
            for (int ss = 0; ss < 4; ++ss) {
                const int kk = 16 * s4 + 4 * ss + (l >> 4);
                T b[CB];
#pragma unroll
                for (int cb = 0; cb < CB; ++cb) b[cb] = Bs[kk * NTP + cb * 16 + (l & 15)];
#pragma unroll
                for (int rb = 0; rb < RB; ++rb) {
                    if (w * RB + rb < KB) {
#pragma unroll
                        for (int cb = 0; cb < CB; ++cb) acc[rb][cb] = mfma16(a4[rb][ss], b[cb], acc[rb][cb]);
                    }
                }
            }
        }
        // result rows: the second sign flip of D A D
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
            V4 sr;
#pragma unroll
            for (int r = 0; r < 4; ++r) sr[r] = sg[min(w * RB + rb, KB - 1) * 16 + mfma_row(T(0), l, r)];
#pragma unroll
            for (int cb = 0; cb < CB; ++cb) acc[rb][cb] *= sr;
        }
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
    // accumulate into the local expansions
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
        int rbg = w * RB + rb;
        if (rbg >= KB) continue;
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) {
            int j = cb * 16 + (l & 15);
            int le = s_le[j];
            if (le < 0) continue;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                int row = rbg * 16 + mfma_row(T(0), l, r);
                if (row < K) A.le[(size_t)le * KP + row] += tot[rb][cb][r];
            }
        }
    }
}

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

// Two leaves per 64-lane block (a leaf holds about half a wave of sources):
// half h = lane >> 5 takes leaf 2 blockIdx.x + h, its sources 32 at a time;
// lane i then sums coefficient c0 + i of both halves' rows.
template <int P>
__global__ void __launch_bounds__(64) k_p2m_p(EvalArgs<float> A, int n_leaves)
{
    constexpr int K = (P + 1) * (P + 1);
    __shared__ float red[64][65];
    const int lane = threadIdx.x, h = lane >> 5, hl = lane & 31;
    const int w = 2 * blockIdx.x + h;
    const bool on = w < n_leaves;
    const int leaf = on ? A.p2m_leaves[w] : A.p2m_leaves[2 * blockIdx.x];
    const FmmDev& F = A.fmm[A.sl_fmm[leaf]];
    const double* __restrict__ ith = A.ith_s + ((size_t)A.sl_fmm[leaf] * (kMaxDepth + 1) + F.H) * (LPB_MAX_P + 1);
    const int s0 = A.sl_start[leaf], s1 = on ? A.sl_start[leaf + 1] : s0;
    const float hinv = (float)(1.0 / A.sl_h[leaf]);
    float acc[K];
#pragma unroll
    for (int k = 0; k < K; ++k) acc[k] = 0.f;
    for (int j = s0 + hl; j < s1; j += 32) {
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
    const int w1 = 2 * blockIdx.x + 1;
    const int me0 = A.sl_me[A.p2m_leaves[2 * blockIdx.x]], me1 = w1 < n_leaves ? A.sl_me[A.p2m_leaves[w1]] : -1;
#pragma unroll
    for (int c0 = 0; c0 < K; c0 += 64) {
#pragma unroll
        for (int i = 0; i < 64; ++i)
            if (c0 + i < K) red[i][lane] = acc[c0 + i];
        __syncthreads();
        if (c0 + lane < K) {
            float t0 = 0.f, t1 = 0.f;
#pragma unroll 16
            for (int jj = 0; jj < 32; ++jj) {
                t0 += red[lane][jj];
                t1 += red[lane][32 + jj];
            }
            A.me[(size_t)me0 * A.KP + c0 + lane] = t0;
            if (me1 >= 0) A.me[(size_t)me1 * A.KP + c0 + lane] = t1;
        }
        __syncthreads();
    }
}

// Two leaves per 64-lane block (a leaf holds about half a wave of targets):
// half h = lane >> 5 takes leaf 2 blockIdx.x + h, its targets 32 at a time.
template <int P>
__global__ void __launch_bounds__(64) k_l2p_p(EvalArgs<float> A, int n_leaves)
{
    constexpr int K = (P + 1) * (P + 1);
    __shared__ float Ls[2][K];   // the leaves' local expansions, read at half-uniform addresses
    const int h = threadIdx.x >> 5, hl = threadIdx.x & 31;
    const int w = 2 * blockIdx.x + h;
    const bool on = w < n_leaves;
    const int leaf = on ? A.l2p_leaves[w] : 0;
    if (on) {
        const int le = A.tl_le[leaf];
        for (int k = hl; k < K; k += 32) Ls[h][k] = A.le[(size_t)le * A.KP + k];
    }
    __syncthreads();
    if (!on) return;
    const FmmDev& F = A.fmm[A.tl_fmm[leaf]];
    const double* __restrict__ ith = A.ith_t + ((size_t)A.tl_fmm[leaf] * (kMaxDepth + 1) + F.H) * (LPB_MAX_P + 1);
    const int t0 = A.tl_start[leaf], t1 = A.tl_start[leaf + 1];
    const float hinv = (float)(1.0 / A.tl_h[leaf]);
    const float* L = Ls[h];
    for (int j = t0 + hl; j < t1; j += 32) {
        const float ux = A.t_ux[j], uy = A.t_uy[j], uz = A.t_uz[j];
        const double r2d = (double)ux * ux + (double)uy * uy + (double)uz * uz;
        float g[P + 1];
        bessel_ratio_reg<P>(F.lam_t * F.lam_t * r2d, A.bes_tab, ith, 1.f, g);
        // Phi = far * sum_n g_n [Lh_n0 R_n^0 + 2 sum_{m>0} Re(Lh_nm R_n^m)]
        float phi = 0.f;
        solid_harmonics<P>(ux * hinv, uy * hinv, uz * hinv,
                           [&](int n, int m, float re, float im) {
                               if (m == 0) phi += g[n] * (L[ire(n, 0)] * re);
                               else phi += 2.f * g[n] * (L[ire(n, m)] * re - L[iim(n, m)] * im);
                           });
        A.parts[A.t_out[j]] = (double)phi * F.far_factor;
    }
}

// ---------------------------------------------------------------------------
// Batched dense translations on the matrix cores: M2M (eq. metome, one term
// per child octant), L2L (one term, 64 children of one octant) and the V-list
// pairs outside the tiled levels (one term, up to 64 pairs of one operator).
// Work item w computes for its 64 columns j
//   y_j = sum_t A_{op_t} x_{src_t[j]}     (x = 0 for a missing source)
// and stores y_j (mode 0) or adds it (mode 1) to row dst[j] of `out`.
// Sources are gathered into LDS as in the tiled M2L, the next term's sources
// load during the current term's products.
// In-LDS per-column transform of a staged block B[k][j] (KP rows, NTP
// stride): reflection signs D (code 0..7) or the rotation of every order-m
// (Re, Im) pair by +m phi (sources) or -m phi (results) (code kXfRotate).
// Every thread of the 256 takes column j = tid & 63 and a quarter of the rows.
// cs[m * 128 + j] = cos(m phi_j), cs[m * 128 + 64 + j] = sin(m phi_j), m = 1..p
template <typename T>
__device__ inline void column_trig(T* cs, int p, int code, double phi)
{
    const int j = threadIdx.x & 63, part = threadIdx.x >> 6;
    if (code != kXfRotate) return;
    for (int m = 1 + part; m <= p; m += 4) {
        double sd, cd;
        sincos((double)m * phi, &sd, &cd);
        cs[m * 128 + j] = (T)cd;
        cs[m * 128 + 64 + j] = (T)sd;
    }
}

template <typename T>
__device__ inline void column_xform(T* Bs, int NTP, int p, int K, int KP, int code, const T* cs, const T* __restrict__ refl,
                                    bool result)
{
    const int j = threadIdx.x & 63, part = threadIdx.x >> 6;
    if (code < 0) return;
    if (code < kXfRotate) {
        const T* sg = refl + (size_t)code * KP;
        for (int k = part; k < K; k += 4) Bs[k * NTP + j] *= sg[k];
        return;
    }
    int q = 0;
    for (int n = 1; n <= p; ++n)
        for (int m = 1; m <= n; ++m, ++q) {
            if ((q & 3) != part) continue;
            const T c = cs[m * 128 + j], sn = result ? -cs[m * 128 + 64 + j] : cs[m * 128 + 64 + j];
            T& re = Bs[ire(n, m) * NTP + j];
            T& im = Bs[iim(n, m) * NTP + j];
            const T a = re, b = im;
            re = a * c - b * sn;
            im = a * sn + b * c;
        }
}

// RBF = ceil(KB / 4): the row blocks per wave of a whole item, which also
// sizes the source staging; GY blocks along y split them (RB per wave each).
template <typename T, int RBF, bool XF, int GY>
__global__ void __launch_bounds__(256) k_batched(const T* __restrict__ in, T* out, const int* __restrict__ term_ptr,
                                                 const int* __restrict__ term_op, const int* __restrict__ term_src,
                                                 const int* __restrict__ dst, int wbase, int mode, int K, int KP,
                                                 const T* __restrict__ pool_swz, int zrow, int sched,
                                                 const int* __restrict__ xcode, const double* __restrict__ xang,
                                                 const T* __restrict__ refl, int p)
{
    typedef typename Vec4<T>::type V4;
    static_assert(GY == 1 || !XF, "results with a transform need whole columns");
    constexpr int RB = (RBF + GY - 1) / GY;
    constexpr int NT = 64, CB = 4, GMAX = 4 * RBF;
    constexpr int NTP = NT + (sizeof(T) == 4 ? 16 : 8);
    extern __shared__ unsigned char smem_raw[];
    T* Bs = reinterpret_cast<T*>(smem_raw);   // [KP][NTP]
    const int KB = KP / 16;
    const int wi = wbase + sched_index(blockIdx.x, gridDim.x, sched);
    const int t0 = term_ptr[wi], t1 = term_ptr[wi + 1];
    const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
    // row-block group of this wave: blocks of a work item along y split the
    // output rows (every block stages all of the sources)
    const int wy = (GY > 1 ? (int)blockIdx.y * 4 : 0) + w;
    const int gj = tid >> 2, gpart = tid & 3;
    V4 acc[RB][CB], tot[RB][CB], cmp[RB][CB];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) tot[rb][cb] = cmp[rb][cb] = V4{0, 0, 0, 0};
    V4 greg[GMAX];
    // XF: per-column transform code and, for rotations, cos / sin (m phi) after B in LDS
    T* trig = Bs + (size_t)KP * NTP;
    const int xc = XF ? xcode[(size_t)wi * NT + (tid & 63)] : -1;
    if (XF) column_trig<T>(trig, p, xc, xang[(size_t)wi * NT + (tid & 63)]);
    auto fetch = [&](int t) {
        const int sidx = term_src[(size_t)t * NT + gj];
        const T* src = in + (size_t)(sidx < 0 ? zrow : sidx) * KP + 4 * gpart;   // missing: the zero row
#pragma unroll
        for (int i = 0; i < GMAX; ++i) greg[i] = (i < KB) ? *reinterpret_cast<const V4*>(src + 16 * i) : V4{0, 0, 0, 0};
    };
    if (t0 < t1) fetch(t0);
    for (int t = t0; t < t1; ++t) {
        __syncthreads();
#pragma unroll
        for (int i = 0; i < GMAX; ++i) {
            if (i < KB) {
#pragma unroll
                for (int e = 0; e < 4; ++e) Bs[(16 * i + 4 * gpart + e) * NTP + gj] = greg[i][e];
            }
        }
        __syncthreads();
        if (XF) {
            // sources into the frame of the stored operator
            column_xform<T>(Bs, NTP, p, K, KP, xc, trig, refl, false);
            __syncthreads();
        }
        const T* Aw = pool_swz + (size_t)term_op[t] * KP * KP;
        if (t + 1 < t1) fetch(t + 1);
        mma_block<T, RB, CB>(Aw, Bs, NTP, KB, wy, l, acc);
        accumulate<T, RB, CB>(acc, tot, cmp);
    }
    if (XF) {
        // results back from the operator's frame, through LDS, then stored row-contiguously
        __syncthreads();
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
            int rbg = w * RB + rb;
            if (rbg >= KB) continue;
#pragma unroll
            for (int cb = 0; cb < CB; ++cb)
#pragma unroll
                for (int r = 0; r < 4; ++r) Bs[(rbg * 16 + mfma_row(T(0), l, r)) * NTP + cb * 16 + (l & 15)] = tot[rb][cb][r];
        }
        __syncthreads();
        column_xform<T>(Bs, NTP, p, K, KP, xc, trig, refl, true);
        __syncthreads();
        for (int e = tid; e < NT * K; e += 256) {
            const int j = e / K, row = e - j * K;
            const int d = dst[(size_t)wi * NT + j];
            if (d < 0) continue;
            if (mode == 0) out[(size_t)d * KP + row] = Bs[row * NTP + j];
            else out[(size_t)d * KP + row] += Bs[row * NTP + j];
        }
        return;
    }
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
        int rbg = wy * RB + rb;
        if (rbg >= KB) continue;
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) {
            const int d = dst[(size_t)wi * NT + cb * 16 + (l & 15)];
            if (d < 0) continue;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                int row = rbg * 16 + mfma_row(T(0), l, r);
                if (row >= K) continue;
                if (mode == 0) out[(size_t)d * KP + row] = tot[rb][cb][r];
                else out[(size_t)d * KP + row] += tot[rb][cb][r];
            }
        }
    }
}

template <typename T, bool XF>
static void launch_batched_x(const EvalArgs<T>& A, int w0, int w1, const T* in, int zrow, T* out, int mode, hipStream_t st)
{
    if (w1 <= w0) return;
    // few work items (coarse levels) leave most CUs idle: split the output
    // row blocks of each item over two blocks (y), each staging the sources
    const int KB = A.KP / 16, n = w1 - w0;
    const int RB = (KB + 3) / 4;
    const int gy = (!XF && n < 512 && RB >= 2) ? 2 : 1;
    const size_t sm = sizeof(T) * ((size_t)A.KP * (64 + (sizeof(T) == 4 ? 16 : 8)) + (XF ? (size_t)(A.p + 1) * 128 : 0));
    dim3 g(n, gy), b(256);
#define LPB_BATCHED(R)                                                                                                      \
    if constexpr (!XF) {                                                                                                    \
        if (gy == 2) {                                                                                                      \
            hipLaunchKernelGGL((k_batched<T, R, XF, 2>), g, b, sm, st, in, out, A.bw_term_ptr, A.bw_op, A.bw_src, A.bw_dst, \
                               w0, mode, A.K, A.KP, A.pool_swz, zrow, A.batch_sched, A.bw_xc, A.bw_xa, A.refl_sign, A.p);   \
            break;                                                                                                          \
        }                                                                                                                   \
    }                                                                                                                       \
    hipLaunchKernelGGL((k_batched<T, R, XF, 1>), g, b, sm, st, in, out, A.bw_term_ptr, A.bw_op, A.bw_src, A.bw_dst, w0, mode, \
                       A.K, A.KP, A.pool_swz, zrow, A.batch_sched, A.bw_xc, A.bw_xa, A.refl_sign, A.p)
    switch (RB) {
    case 1: LPB_BATCHED(1); break;
    case 2: LPB_BATCHED(2); break;
    case 3: LPB_BATCHED(3); break;
    case 4: LPB_BATCHED(4); break;
    case 5: LPB_BATCHED(5); break;
    case 6: LPB_BATCHED(6); break;
    default: LPB_BATCHED(7); break;
    }
#undef LPB_BATCHED
}
template <typename T>
static void launch_batched(const EvalArgs<T>& A, int w0, int w1, const T* in, int zrow, T* out, int mode, hipStream_t st)
{
    launch_batched_x<T, false>(A, w0, w1, in, zrow, out, mode, st);
}

// V-list pairs outside the tiled levels: LE[box] += sum of the box's pair rows
// of the scratch, in list order (deterministic)
template <typename T>
__global__ void k_m2l_reduce(EvalArgs<T> A)
{
    const int le = A.m2l_boxes[blockIdx.x];
    const int k0 = A.m2l_ptr[le], k1 = A.m2l_ptr[le + 1];
    for (int row = threadIdx.x; row < A.K; row += blockDim.x) {
        // four rows' loads in flight at a time; the sum keeps list order
        T s = T(0);
        int k = k0;
        for (; k + 4 <= k1; k += 4) {
            const T a0 = A.m2l_scratch[(size_t)k * A.KP + row], a1 = A.m2l_scratch[(size_t)(k + 1) * A.KP + row],
                    a2 = A.m2l_scratch[(size_t)(k + 2) * A.KP + row], a3 = A.m2l_scratch[(size_t)(k + 3) * A.KP + row];
            s += a0;
            s += a1;
            s += a2;
            s += a3;
        }
        for (; k < k1; ++k) s += A.m2l_scratch[(size_t)k * A.KP + row];
        A.le[(size_t)le * A.KP + row] += s;
    }
}

// The same product with the number of 16-row blocks KB fixed at compile
// time (p <= 15): the 16-column slabs of the operator stream through a ring
// of D register slabs, so every load is issued D slabs (D * RB * 4 MFMAs)
// ahead of its use, continuing across offsets into the next operator.
// RBW = 0: four waves, each owning ceil(KB/4) row blocks; RBW = 1: KB waves
// of one row block each (more waves per CU to hide latency, same arithmetic
// per output element in the same order, so both give identical results).
template <typename T, int KB, int RBW>
__global__ void __launch_bounds__(RBW == 1 ? 64 * KB : 256) k_m2l_tile_kb(EvalArgs<T> A)
{
    typedef typename Vec4<T>::type V4;
    constexpr int NWT = (RBW == 1) ? KB : 4;              // waves per block
    constexpr int RB = (RBW == 1) ? 1 : (KB + 3) / 4;     // row blocks per wave
    constexpr int NWACT = (KB + RB - 1) / RB;   // waves that own row blocks (the others only gather)
    constexpr int NV = 4 * KB / NWT;                       // staged 4-vectors per thread and offset
    constexpr int D = (RBW == 0 && sizeof(T) == 4 && RB <= 2) ? ((KB % 4 == 0) ? 4 : ((KB % 2 == 0) ? 2 : 1))
                                                               : ((KB % 2 == 0) ? 2 : 1);
    constexpr int NT = 64, CB = 4, KP = 16 * KB;
    constexpr int NTP = NT + (sizeof(T) == 4 ? 16 : 8);   // padded LDS row (bank spread)
    extern __shared__ unsigned char smem_raw[];
    T* Bs = reinterpret_cast<T*>(smem_raw);               // [KP][NTP]
    __shared__ int s_le[NT];
    const int K = A.K;
    const Tile tile = A.tiles[sched_index(blockIdx.x, gridDim.x, A.tile_sched & 1)];
    const TileFL fl = A.tfl[tile.fl];
    const int nside = fl.nside;
    const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
    const int ox = (tile.octant >> 2) & 1, oy = (tile.octant >> 1) & 1, oz = tile.octant & 1;
    V4 acc[RB][CB], tot[RB][CB], cmp[RB][CB];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) tot[rb][cb] = cmp[rb][cb] = V4{0, 0, 0, 0};
    auto tcoord = [&](int j, int& tx, int& ty, int& tz) {
        tx = 2 * (tile.px0 + (j >> 4)) + ox;
        ty = 2 * (tile.py0 + ((j >> 2) & 3)) + oy;
        tz = 2 * (tile.pz0 + (j & 3)) + oz;
    };
    if (tid < NT) {
        int tx, ty, tz;
        tcoord(tid, tx, ty, tz);
        s_le[tid] = (tx < nside && ty < nside && tz < nside)
                        ? A.grid_le[fl.grid_off + ((size_t)tx * nside + ty) * nside + tz] : -1;
    }
    __syncthreads();
    const int gj = tid / NWT, gpart = tid % NWT;   // column and 4-vector part of the gather
    int gtx, gty, gtz;
    tcoord(gj, gtx, gty, gtz);
    const bool gvalid = s_le[gj] >= 0;
    const int* codes = A.oct_codes + tile.octant * kVOffsets;
    V4 greg[NV];
    auto fetch = [&](int d) {
        const int code = codes[d];
        const int sx = gtx + code / 49 - 3, sy = gty + (code / 7) % 7 - 3, sz = gtz + code % 7 - 3;
        int me = -1;
        if (gvalid && sx >= 0 && sy >= 0 && sz >= 0 && sx < nside && sy < nside && sz < nside)
            me = A.grid_me[fl.grid_off + ((size_t)sx * nside + sy) * nside + sz];
        // a missing source reads the zero row
        const T* src = A.me + (size_t)(me < 0 ? A.n_me : me) * KP + 4 * gpart;
#pragma unroll
        for (int i = 0; i < NV; ++i) greg[i] = *reinterpret_cast<const V4*>(src + 4 * NWT * i);
    };
    auto opent = [&](int d) { return A.optab[fl.optab_off + codes[d]]; };
    auto opA = [&](int d) {
        return A.pool_swz + (size_t)A.swz_index[opent(d) & ((1 << kReflShift) - 1)] * KP * KP;
    };
    V4 ring[D][RB];
    // row blocks past KB (last active wave only) repeat the last block; their
    // rows are >= K and never stored
    auto loadA = [&](const T* Aw, int s4, V4 (&dst)[RB]) {
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
            const int rbg = min(w * RB + rb, KB - 1);
            dst[rb] = *reinterpret_cast<const V4*>(Aw + (((size_t)rbg * KB + s4) * 64 + l) * 4);
        }
    };
    const T* Aw = opA(0);
    if (w < NWACT) {
#pragma unroll
        for (int i = 0; i < D; ++i) loadA(Aw, i, ring[i]);
    }
    fetch(0);
    // products of up to GRP consecutive offsets of one reflection class chain in
    // the MFMA accumulators; the row signs and the compensated sum follow per run
    constexpr int GRP = (sizeof(T) == 4) ? 4 : 1;
    int run = 0;
    for (int d = 0; d < kVOffsets; ++d) {
        const int cls = opent(d) >> kReflShift;
        const T* sg = A.refl_sign + (size_t)cls * KP;
        __syncthreads();   // every wave is done with the previous offset's B
#pragma unroll
        for (int i = 0; i < NV; ++i) {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int k = 4 * (NWT * i + gpart) + e;
                Bs[k * NTP + gj] = greg[i][e] * sg[k];
            }
        }
        __syncthreads();
        const bool more = d + 1 < kVOffsets;
        const T* Awn = more ? opA(d + 1) : Aw;
        if (more) fetch(d + 1);   // next offset's sources load during this offset's products
        const bool flush = !more || run + 1 == GRP || (opent(d + 1) >> kReflShift) != cls;
        if (w < NWACT) {          // wave-uniform; the product loop itself has no branches
            if (run == 0) {
#pragma unroll
                for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                    for (int cb = 0; cb < CB; ++cb) acc[rb][cb] = V4{0, 0, 0, 0};
            }
#pragma unroll
            for (int s4 = 0; s4 < KB; ++s4) {
                V4 a4[RB];
#pragma unroll
                for (int rb = 0; rb < RB; ++rb) a4[rb] = ring[s4 % D][rb];
                if (s4 + D < KB) loadA(Aw, s4 + D, ring[s4 % D]);
                else loadA(Awn, s4 + D - KB, ring[s4 % D]);   // (the last offset reloads its own operator)
#pragma unroll
                for (int ss = 0; ss < 4; ++ss) {
                    const int kk = 16 * s4 + 4 * ss + (l >> 4);
                    T b[CB];
#pragma unroll
                    for (int cb = 0; cb < CB; ++cb) b[cb] = Bs[kk * NTP + cb * 16 + (l & 15)];
#pragma unroll
                    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                        for (int cb = 0; cb < CB; ++cb) acc[rb][cb] = mfma16(a4[rb][ss], b[cb], acc[rb][cb]);
                }
            }
            if (flush) {
                // result rows: the second sign flip of D A D
#pragma unroll
                for (int rb = 0; rb < RB; ++rb) {
                    V4 sr;
#pragma unroll
                    for (int r = 0; r < 4; ++r) sr[r] = sg[min(w * RB + rb, KB - 1) * 16 + mfma_row(T(0), l, r)];
#pragma unroll
                    for (int cb = 0; cb < CB; ++cb) acc[rb][cb] *= sr;
                }
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
        }
        run = flush ? 0 : run + 1;
        Aw = Awn;
    }
    if (w >= NWACT) return;
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
        int rbg = w * RB + rb;
        if (rbg >= KB) continue;
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) {
            int j = cb * 16 + (l & 15);
            int le = s_le[j];
            if (le < 0) continue;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                int row = rbg * 16 + mfma_row(T(0), l, r);
                if (row < K) A.le[(size_t)le * KP + row] += tot[rb][cb][r];
            }
        }
    }
}

// Tiled M2L by reflection orbits (FP32, p >= kOrbitMinP).  The 189 V-list
// offsets of a child octant fall into 56 orbits {sigma d} of the canonical
// offset d = (|dx|,|dy|,|dz|) under the reflections sigma of the axes, and
// A_{sigma d} = D_sigma A_d D_sigma with D_sigma = diag(chi_sigma(e_k)), e_k the
// sign class of coefficient k and chi_sigma(e) = (-1)^|sigma & e|.  For the
// result rows of class c therefore
//   sum_sigma (D_sigma A_d D_sigma x_sigma)_c = A_d[c, :] B^(c),
//   B^(c) = sum_sigma chi_sigma(c) x'_sigma,   x'_sigma = D_sigma x_sigma:
// one product per orbit instead of one per member.  With the members
// sigma_j = deposit(j, both) | minus (see kOrbits),
//   B^(c) = (-1)^|c & minus| Wc[extract(c, both)],
//   Wc[m] = D_minus sum_j (-1)^|j & m| prod_{axes b of j} D_b x_j,
// a Walsh-Hadamard transform over the nb both-axes whose butterflies carry
// the per-coefficient axis signs (t v for the upper input); the class sign
// (-1)^|c & minus| multiplies the orbit's product before it is added.  The
// operands hold the result rows in class order (orb_rows), so every 16-row
// block has one class.
// Each wave owns 16 targets of the tile (a 16-column block of the product)
// and every row block: per (orbit, 16-coefficient slab) step each lane loads
// four consecutive coefficients of its target's member sources (the B
// operand of four products, the operand layout arranged to match), forms the
// transforms in registers and issues the products; loads run two steps
// ahead.  The orbits come in groups of one both-axes mask (kOrbGroupMask), so
// each gather loads exactly the members its orbit has.  No data is shared between waves, so the waves never wait for each
// other.  Each orbit's products go to the result with Kahan compensation.
template <int P, int MASK>
__device__ __forceinline__ void orbit_step(const Vec4<float>::type (&xs)[8], const int __attribute__((ext_vector_type(4))) ek, int minus,
                                           const Vec4<float>::type (&ra)[class_row_blocks(P)],
                                           Vec4<float>::type (&acc)[class_row_blocks(P)])
{
    typedef Vec4<float>::type V4;
    typedef int I4 __attribute__((ext_vector_type(4)));
    constexpr int NRB = class_row_blocks(P);
    constexpr int NB = (MASK & 1) + ((MASK >> 1) & 1) + ((MASK >> 2) & 1);
    constexpr int M = 1 << NB;
    constexpr int AX[3] = {(MASK & 1) ? 0 : ((MASK & 2) ? 1 : 2), (MASK & 1) ? ((MASK & 2) ? 1 : 2) : 2, 2};
    V4 y[M];
#pragma unroll
    for (int j = 0; j < M; ++j) y[j] = xs[j];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        // sign of the 4 coefficients under the reflection of axis AX[b]
        I4 t;
#pragma unroll
        for (int e = 0; e < 4; ++e) t[e] = ((ek[e] >> AX[b]) & 1) << 31;
#pragma unroll
        for (int j = 0; j < M; ++j)
            if (!((j >> b) & 1)) {
                const V4 u = y[j];
                V4 v = y[j | (1 << b)];
#pragma unroll
                for (int e = 0; e < 4; ++e) v[e] = __int_as_float(__float_as_int(v[e]) ^ t[e]);
                y[j] = u + v;
                y[j | (1 << b)] = u - v;
            }
    }
    if (minus) {
        I4 t;
#pragma unroll
        for (int e = 0; e < 4; ++e) t[e] = (__builtin_popcount(ek[e] & minus) & 1) << 31;
#pragma unroll
        for (int j = 0; j < M; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) y[j][e] = __int_as_float(__float_as_int(y[j][e]) ^ t[e]);
    }
    // class c of row block rb reads Wc[extract(c, both)]
    auto ext = [](int c) {
        int m = 0, o = 0;
        for (int bit = 0; bit < 3; ++bit)
            if ((MASK >> bit) & 1) m |= ((c >> bit) & 1) << o++;
        return m;
    };
#pragma unroll
    for (int ss = 0; ss < 4; ++ss)
#pragma unroll
        for (int rb = 0; rb < NRB; ++rb) acc[rb] = mfma16(ra[rb][ss], y[ext(class_of_row_block(P, rb))][ss], acc[rb]);
}

template <int P>
__global__ void __launch_bounds__(256) k_m2l_orbit(EvalArgs<float> A)
{
    typedef Vec4<float>::type V4;
    constexpr int K = (P + 1) * (P + 1), KB = (K + 15) / 16, KP = 16 * KB;
    constexpr int NRB = class_row_blocks(P);
    constexpr int OPSZ = NRB * KB * 256;     // floats of one operator
    constexpr int NIT = kOrbits * KB;        // steps (even: kOrbits is)
    constexpr int NG = kOrbGrid * kOrbGrid * kOrbGrid;
    __shared__ int s_grid[NG];               // ME row of each local source box
    __shared__ int s_tab[kOrbits * kOrbTab]; // the octant's orbit table
    __shared__ int s_kcls[KP];               // sign class of each coefficient
    __shared__ int s_le[64];                 // LE row of each target (-1 none)
    __shared__ int s_aoff[kOrbits];          // operator of each orbit
    const Tile tile = A.tiles[sched_index(blockIdx.x, gridDim.x, A.tile_sched & 1)];
    const TileFL fl = A.tfl[tile.fl];
    const int nside = fl.nside;
    const int tid = threadIdx.x, l = tid & 63;
    const int ox = (tile.octant >> 2) & 1, oy = (tile.octant >> 1) & 1, oz = tile.octant & 1;
    const int* tab = A.orb_tab + tile.octant * (kOrbits * kOrbTab);
    {
        // every gather of the set-up is issued before the first LDS store, so
        // the independent loads are in flight together
        constexpr int NTH = 256, NGL = (NG + NTH - 1) / NTH, NTL = (kOrbits * kOrbTab + NTH - 1) / NTH;
        static_assert(KP <= NTH, "one coefficient class per thread");
        const int gx0 = 2 * tile.px0 + ox - 3, gy0 = 2 * tile.py0 + oy - 3, gz0 = 2 * tile.pz0 + oz - 3;
        int gv[NGL], tv[NTL];
#pragma unroll
        for (int k = 0; k < NGL; ++k) {
            const int i = tid + k * NTH;
            const int sx = gx0 + i / (kOrbGrid * kOrbGrid), sy = gy0 + (i / kOrbGrid) % kOrbGrid, sz = gz0 + i % kOrbGrid;
            gv[k] = -1;
            if (i < NG && sx >= 0 && sy >= 0 && sz >= 0 && sx < nside && sy < nside && sz < nside)
                gv[k] = A.grid_me[fl.grid_off + ((size_t)sx * nside + sy) * nside + sz];
        }
#pragma unroll
        for (int k = 0; k < NTL; ++k) {
            const int i = tid + k * NTH;
            tv[k] = (i < kOrbits * kOrbTab) ? tab[i] : 0;
        }
        const int kv = (tid < KP) ? A.orb_kcls[tid] : 0;
        int lv = -1;
        if (tid < 64) {
            const int tx = 2 * (tile.px0 + (tid >> 4)) + ox, ty = 2 * (tile.py0 + ((tid >> 2) & 3)) + oy,
                      tz = 2 * (tile.pz0 + (tid & 3)) + oz;
            if (tx < nside && ty < nside && tz < nside)
                lv = A.grid_le[fl.grid_off + ((size_t)tx * nside + ty) * nside + tz];
        } else if (tid < 64 + kOrbits) {
            const int q = tid - 64;
            const int op = A.optab[fl.optab_off + tab[q * kOrbTab + 17]] & ((1 << kReflShift) - 1);
            lv = A.orb_index[op];
        }
#pragma unroll
        for (int k = 0; k < NGL; ++k) {
            const int i = tid + k * NTH;
            if (i < NG) s_grid[i] = gv[k] < 0 ? A.n_me : gv[k];   // a missing source reads the zero row
        }
#pragma unroll
        for (int k = 0; k < NTL; ++k) {
            const int i = tid + k * NTH;
            if (i < kOrbits * kOrbTab) s_tab[i] = tv[k];
        }
        if (tid < KP) s_kcls[tid] = kv;
        if (tid < 64) s_le[tid] = lv;
        else if (tid < 64 + kOrbits) s_aoff[tid - 64] = lv;
    }
    __syncthreads();
    const int cb = tid >> 6, g = l >> 4, jj = l & 15, j = 16 * cb + jj;
    const int tli = ((2 * (j >> 4)) * kOrbGrid + 2 * ((j >> 2) & 3)) * kOrbGrid + 2 * (j & 3);
    // the expansions (with the zero row) span under 2^32 bytes: the launch checks it
    const __amdgpu_buffer_rsrc_t rme =
        __builtin_amdgcn_make_buffer_rsrc(A.me, 0, (int)((unsigned)(A.n_me + 1) * (unsigned)(KP * 4)), 0x00020000);
    const unsigned zoff = (unsigned)A.n_me * (unsigned)(KP * 4) + 16u * g;
    // member row byte offsets of the orbit being gathered, its first CNT
    // members: the orbit groups fix the member count at compile time, and the
    // last orbit of a group also gathers the first steps of the next group's
    // first orbit, which has no more members (its absent ones read the zero row)
    unsigned off[8];
    auto lorbit = [&](auto cntc, int q) {
        constexpr int CNT = decltype(cntc)::value;
        const int* row = s_tab + q * kOrbTab;
        const int nm = 1 << (__builtin_amdgcn_readfirstlane(row[0]) & 15);
#pragma unroll
        for (int m = 0; m < CNT; ++m)
            off[m] = (m < nm) ? (unsigned)s_grid[tli + row[1 + m]] * (unsigned)(KP * 4) + 16u * g : zoff;
    };
    typedef int I4 __attribute__((ext_vector_type(4)));
    // operand slabs: gathered two steps ahead (DA = 2) while the registers
    // allow, one step ahead for the larger orders (they come mostly from L2)
    constexpr int DA = (NRB <= 9) ? 2 : 1;
    V4 xr[2][8], ra[DA][NRB];
    I4 er[2];
    // operand and member gathers are buffer loads: wave-uniform bases and
    // offsets in scalar registers, one fixed 32-bit lane offset, so a gather
    // costs no vector address arithmetic
    const unsigned lane16 = 16u * l;
    auto load_a = [&](int t, V4 (&as)[NRB]) {
        const int q = t / KB, s = t % KB;
        const float* Ao = A.pool_orb + (size_t)__builtin_amdgcn_readfirstlane(s_aoff[q]) * OPSZ;
        const __amdgpu_buffer_rsrc_t ra_ = __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(Ao), 0, OPSZ * 4, 0x00020000);
#pragma unroll
        for (int rb = 0; rb < NRB; ++rb)
            as[rb] = __builtin_bit_cast(V4, __builtin_amdgcn_raw_buffer_load_b128(ra_, lane16, (rb * KB + s) * 1024, 0));
    };
    // gather step t: its first CNT member sources and the coefficient classes
    // (and, with DA = 2, its operand slab)
    auto load = [&](auto cntc, int t, V4 (&xs)[8], V4 (&as)[NRB], I4& ek) {
        constexpr int CNT = decltype(cntc)::value;
        const int s = t % KB;
        if (s == 0) lorbit(cntc, t / KB);
        if constexpr (DA == 2) load_a(t, as);
#pragma unroll
        for (int m = 0; m < CNT; ++m) xs[m] = __builtin_bit_cast(V4, __builtin_amdgcn_raw_buffer_load_b128(rme, off[m], 64 * s, 0));
        ek = *reinterpret_cast<const I4*>(s_kcls + 16 * s + 4 * g);
    };
    V4 acc[NRB], tot[NRB], cmp[NRB];
#pragma unroll
    for (int rb = 0; rb < NRB; ++rb) acc[rb] = tot[rb] = cmp[rb] = V4{0, 0, 0, 0};
    typedef std::integral_constant<int, 1 << __builtin_popcount(kOrbGroupMask[0])> NM0;
    load(NM0{}, 0, xr[0], ra[0], er[0]);
    load(NM0{}, 1, xr[1], ra[DA - 1], er[1]);
    if constexpr (DA == 1) load_a(0, ra[0]);
    // one orbit: its KB steps with the transform specialised for its both-axes
    // (steps of one orbit form one straight code path, so the transforms of a
    // step can overlap the products of the previous one); step t uses register
    // slot t & 1 and refills it with step t + 2 (the last steps re-gather a
    // valid step)
    auto run = [&](auto maskc, auto parc, int q, int minus) {
        constexpr int MASK = decltype(maskc)::value, PAR = decltype(parc)::value;
        typedef std::integral_constant<int, 1 << __builtin_popcount(MASK)> NM;
        const int t0 = q * KB;
        // (the scheduling fences keep each step's transforms after its own loads'
        // wait: hoisted into the previous step they would wait for the loads
        // just issued)
        constexpr int A0 = (DA == 2) ? PAR : 0, A1 = (DA == 2) ? (PAR ^ 1) : 0;
        for (int s = 0; s < KB; s += 2) {
            orbit_step<P, MASK>(xr[PAR], er[PAR], minus, ra[A0], acc);
            if constexpr (DA == 1) load_a(min(t0 + s + 1, NIT - 1), ra[0]);
            load(NM{}, min(t0 + s + 2, NIT - 1), xr[PAR], ra[A0], er[PAR]);
            __builtin_amdgcn_sched_barrier(0);
            if (s + 1 < KB) {
                orbit_step<P, MASK>(xr[PAR ^ 1], er[PAR ^ 1], minus, ra[A1], acc);
                if constexpr (DA == 1) load_a(min(t0 + s + 2, NIT - 1), ra[0]);
                load(NM{}, min(t0 + s + 3, NIT - 1), xr[PAR ^ 1], ra[A1], er[PAR ^ 1]);
                __builtin_amdgcn_sched_barrier(0);
            }
        }
    };
    auto orbit = [&](auto maskc, auto parc, int q) {
        // negative one-sign axes of the orbit
        const int minus = (__builtin_amdgcn_readfirstlane(s_tab[q * kOrbTab]) >> 7) & 7;
        run(maskc, parc, q, minus);
#pragma unroll
        for (int rb = 0; rb < NRB; ++rb) {
            // class sign (-1)^|c & minus| of the orbit's product
            const bool neg = __builtin_popcount(class_of_row_block(P, rb) & minus) & 1;
            const V4 pr = neg ? -acc[rb] : acc[rb];
            const V4 yk = pr - cmp[rb];
            const V4 tk = tot[rb] + yk;
            cmp[rb] = (tk - tot[rb]) - yk;
            tot[rb] = tk;
            acc[rb] = V4{0, 0, 0, 0};
        }
    };
    // the orbit groups in table order; with odd KB the first step of orbit q
    // uses slot q & 1
    auto group = [&](auto gic) {
        constexpr int GI = decltype(gic)::value;
        typedef std::integral_constant<int, kOrbGroupMask[GI]> MC;
        const int q0 = GI * kOrbGroup;
        if constexpr (KB & 1) {
            constexpr int P0 = (GI * kOrbGroup) & 1;
            for (int k = 0;; ++k) {
                orbit(MC{}, std::integral_constant<int, P0>{}, q0 + 2 * k);
                if (2 * k + 1 >= kOrbGroup) break;
                orbit(MC{}, std::integral_constant<int, P0 ^ 1>{}, q0 + 2 * k + 1);
            }
        } else {
            for (int k = 0; k < kOrbGroup; ++k) orbit(MC{}, std::integral_constant<int, 0>{}, q0 + k);
        }
    };
    static_assert(kOrbits == 8 * kOrbGroup, "eight orbit groups");
    group(std::integral_constant<int, 0>{});
    group(std::integral_constant<int, 1>{});
    group(std::integral_constant<int, 2>{});
    group(std::integral_constant<int, 3>{});
    group(std::integral_constant<int, 4>{});
    group(std::integral_constant<int, 5>{});
    group(std::integral_constant<int, 6>{});
    group(std::integral_constant<int, 7>{});
    const int le = s_le[j];
    if (le < 0) return;
    // all row indices, then all current LE values, then the stores (loads in
    // flight together)
    int nat[NRB][4];
    float cur[NRB][4];
    float* lr = A.le + (size_t)le * KP;
#pragma unroll
    for (int rb = 0; rb < NRB; ++rb)
#pragma unroll
        for (int r = 0; r < 4; ++r) nat[rb][r] = A.orb_rows[16 * rb + 4 * g + r];
#pragma unroll
    for (int rb = 0; rb < NRB; ++rb)
#pragma unroll
        for (int r = 0; r < 4; ++r) cur[rb][r] = nat[rb][r] >= 0 ? lr[nat[rb][r]] : 0.0f;
#pragma unroll
    for (int rb = 0; rb < NRB; ++rb)
#pragma unroll
        for (int r = 0; r < 4; ++r)
            if (nat[rb][r] >= 0) lr[nat[rb][r]] = cur[rb][r] + (tot[rb][r] - cmp[rb][r]);
}

template <typename T>
static void launch_m2l_tile(const EvalArgs<T>& A, hipStream_t st)
{
    const int KB = A.KP / 16, RB = (KB + 3) / 4;
    const size_t sm = sizeof(T) * (size_t)A.KP * (64 + (sizeof(T) == 4 ? 16 : 8));
    dim3 g(A.n_tiles), b(256);
    // variant bit of the schedule: KB waves of one row block each
    const bool wide = (A.tile_sched >> 1) & 1;
    if constexpr (sizeof(T) == 4) {
        // (row byte offsets of the expansions are 32-bit in the orbit kernel)
        if (A.pool_orb && A.p >= kOrbitMinP && A.p <= kOrbitMaxP &&
            (size_t)(A.n_me + 1) * A.KP * sizeof(float) < ((size_t)1 << 32)) {
#define LPB_ORB(PP)                                                                                                \
    case PP:                                                                                                       \
        hipLaunchKernelGGL((k_m2l_orbit<PP>), g, dim3(256), 0, st, A);                                             \
        return;
            switch (A.p) {
                LPB_ORB(5) LPB_ORB(6) LPB_ORB(7) LPB_ORB(8) LPB_ORB(9) LPB_ORB(10)
                LPB_ORB(11) LPB_ORB(12) LPB_ORB(13) LPB_ORB(14) LPB_ORB(15)
            default: break;
            }
#undef LPB_ORB
        }
    }
#define LPB_TKB(N)                                                                                  \
    case N:                                                                                         \
        if (wide) hipLaunchKernelGGL((k_m2l_tile_kb<T, N, 1>), g, dim3(64 * N), sm, st, A);         \
        else hipLaunchKernelGGL((k_m2l_tile_kb<T, N, 0>), g, b, sm, st, A);                         \
        return;
    switch (KB) {
        LPB_TKB(1) LPB_TKB(2) LPB_TKB(3) LPB_TKB(4) LPB_TKB(5) LPB_TKB(6)
        LPB_TKB(7) LPB_TKB(8) LPB_TKB(9) LPB_TKB(10) LPB_TKB(11) LPB_TKB(12)
    default: break;
    }
    // FP64 at KB > 12 would spill registers: it takes the generic kernel below
    if constexpr (sizeof(T) == 4) {
        switch (KB) {
            LPB_TKB(13) LPB_TKB(14) LPB_TKB(15) LPB_TKB(16)
        default: break;
        }
    }
#undef LPB_TKB
    switch (RB) {
    case 1: hipLaunchKernelGGL((k_m2l_tile<T, 1>), g, b, sm, st, A); break;
    case 2: hipLaunchKernelGGL((k_m2l_tile<T, 2>), g, b, sm, st, A); break;
    case 3: hipLaunchKernelGGL((k_m2l_tile<T, 3>), g, b, sm, st, A); break;
    case 4: hipLaunchKernelGGL((k_m2l_tile<T, 4>), g, b, sm, st, A); break;
    case 5: hipLaunchKernelGGL((k_m2l_tile<T, 5>), g, b, sm, st, A); break;
    case 6: hipLaunchKernelGGL((k_m2l_tile<T, 6>), g, b, sm, st, A); break;
    default: hipLaunchKernelGGL((k_m2l_tile<T, 7>), g, b, sm, st, A); break;
    }
}

// ---------------------------------------------------------------------------
// L2P (eqs. freespace3dlocexp, lelayerimage), scaled:
//   Phi = far_factor * sum_n g_n(r) [Lh_n0 R_n^0 + 2 sum_{m>0} Re(Lh_nm R_n^m)](u/h)
// One 64-lane block per target leaf, a lane per target; the leaf's local
// expansion is read at wave-uniform addresses, the Bessel ratios (FP64) sit
// in the lane's LDS column.
template <typename T>
__global__ void __launch_bounds__(64) k_l2p(EvalArgs<T> A, int CH)
{
    extern __shared__ unsigned char smem_raw[];
    const int p = A.p;
    const int leaf = A.l2p_leaves[blockIdx.x];
    const int le = A.tl_le[leaf];
    const FmmDev& F = A.fmm[A.tl_fmm[leaf]];
    const double h = A.tl_h[leaf];
    T* gl = reinterpret_cast<T*>(smem_raw);                       // [p+1][CH]
    const int lane = threadIdx.x;
    if (lane >= CH) return;
    const double* __restrict__ tb = A.bes_tab;
    const double* __restrict__ ith = A.ith_t + ((size_t)A.tl_fmm[leaf] * (kMaxDepth + 1) + F.H) * (LPB_MAX_P + 1);
    const T* __restrict__ Ls = A.le + (size_t)le * A.KP;
    const T* __restrict__ amm_t = A.sh_amm;
    const T* __restrict__ al_t = A.sh_alpha;
    const T* __restrict__ be_t = A.sh_beta;
    const int t0 = A.tl_start[leaf], t1 = A.tl_start[leaf + 1];
    const T hinv = (T)(1.0 / h);
    for (int j = t0 + lane; j < t1; j += CH) {
        T ux = A.t_ux[j], uy = A.t_uy[j], uz = A.t_uz[j];
        double r2d = (double)ux * ux + (double)uy * uy + (double)uz * uz;
        bessel_ratio_col<T>(p, F.lam_t * F.lam_t * r2d, tb, ith, T(1), gl + lane, CH);
        T x = ux * hinv, y = uy * hinv, z = uz * hinv;
        T r2 = x * x + y * y + z * z;
        T wr = T(1), wi = T(0);
        T phi = T(0);
        for (int m = 0; m <= p; ++m) {
            if (m > 0) {
                T nr = wr * x - wi * y;
                wi = wr * y + wi * x;
                wr = nr;
            }
            const T two = (m > 0) ? T(2) : T(1);
            T pr = amm_t[m] * wr, pi = amm_t[m] * wi;
            T sm = gl[(size_t)m * CH + lane] * (Ls[ire(m, m)] * pr - (m > 0 ? Ls[iim(m, m)] * pi : T(0)));
            if (m + 1 <= p) {
                T al = al_t[ipk(m + 1, m)];
                T qr = al * z * pr, qi = al * z * pi;
                sm += gl[(size_t)(m + 1) * CH + lane] * (Ls[ire(m + 1, m)] * qr - (m > 0 ? Ls[iim(m + 1, m)] * qi : T(0)));
                for (int n = m + 2; n <= p; ++n) {
                    T a = al_t[ipk(n, m)], b = be_t[ipk(n, m)];
                    T sr = a * z * qr - b * r2 * pr;
                    T si = a * z * qi - b * r2 * pi;
                    sm += gl[(size_t)n * CH + lane] * (Ls[ire(n, m)] * sr - (m > 0 ? Ls[iim(n, m)] * si : T(0)));
                    pr = qr;
                    pi = qi;
                    qr = sr;
                    qi = si;
                }
            }
            phi += two * sm;
        }
        A.parts[A.t_out[j]] = (double)phi * F.far_factor;
    }
}

// ---------------------------------------------------------------------------
// Free-space near field (eq. freereactioncomponents, j != i):
//   Phi_i += sum_{j in U(i), j != i} q_j e^{-lam r}/(4 pi eps r)
// (the self term is the pair at distance 0; charges must be distinct points)
// One 64-lane block per work item of up to 64 targets of one leaf (dense
// leaves span several items).  All U-list sources (up to SMAX at a time)
// are staged in LDS with their offset from the target leaf centre; two lanes
// share a target and split the sources, and combine at the end.  This is the
// FP64 form (the FP32 one follows).
__device__ inline double pair_kernel(double r2, double lam) { double r = sqrt(r2); return exp(-lam * r) / r; }

template <typename T>
__global__ void __launch_bounds__(64) k_p2p_free(EvalArgs<T> A)
{
    constexpr int SMAX = 512;
    __shared__ T sx[SMAX], sy[SMAX], sz[SMAX], sq[SMAX];
    const int leaf = A.p2p_free_leaves[blockIdx.x];
    const FmmDev& F = A.fmm[A.tl_fmm[leaf]];
    const T lamk = (sizeof(T) == 4) ? (T)(F.lam_t * 1.4426950408889634) : (T)F.lam_t;
    const int t0 = A.p2p_free_t0[blockIdx.x], t1 = min(A.tl_start[leaf + 1], t0 + 64);
    const double tcx = A.tl_ctr[3 * leaf], tcy = A.tl_ctr[3 * leaf + 1], tcz = A.tl_ctr[3 * leaf + 2];
    const int lane = threadIdx.x, half = lane >> 5, tl = lane & 31;
    const int k0 = A.p2p_ptr[leaf], k1 = A.p2p_ptr[leaf + 1];
    for (int base = t0; base < t1; base += 32) {
        int j = base + tl;
        bool act = j < t1;
        T x = act ? A.t_ux[j] : T(0), y = act ? A.t_uy[j] : T(0), z = act ? A.t_uz[j] : T(0);
        T sum = T(0), comp = T(0);
        int k = k0, s = (k0 < k1) ? A.sl_start[A.p2p_src[k0]] : 0;
        while (k < k1) {
            // stage up to SMAX sources, continuing across source leaves
            int n = 0;
            __syncthreads();
            while (k < k1 && n < SMAX) {
                int sl = A.p2p_src[k];
                int se = A.sl_start[sl + 1];
                int take = min(se - s, SMAX - n);
                T ox = (T)(A.sl_ctr[3 * sl] - tcx), oy = (T)(A.sl_ctr[3 * sl + 1] - tcy), oz = (T)(A.sl_ctr[3 * sl + 2] - tcz);
                for (int i = lane; i < take; i += 64) {
                    sx[n + i] = A.s_ux[s + i] + ox;
                    sy[n + i] = A.s_uy[s + i] + oy;
                    sz[n + i] = A.s_uz[s + i] + oz;
                    sq[n + i] = A.qs[s + i];
                }
                n += take;
                s += take;
                if (s >= se) {
                    ++k;
                    if (k < k1) s = A.sl_start[A.p2p_src[k]];
                }
            }
            __syncthreads();
            if (act) {
                for (int jj = half; jj < n; jj += 2) {
                    T dx = x - sx[jj], dy = y - sy[jj], dz = z - sz[jj];
                    T r2 = dx * dx + dy * dy + dz * dz;
                    // the target itself (r = 0) is the only coincident source of a free-space FMM
                    T v = (r2 > T(0)) ? sq[jj] * pair_kernel(r2, lamk) : T(0);
                    if (sizeof(T) == 4) {
                        T yk = v - comp;
                        T tk = sum + yk;
                        comp = (tk - sum) - yk;
                        sum = tk;
                    } else {
                        sum += v;
                    }
                }
            }
        }
        // combine the two halves (lane l and l+32 share a target)
        T other = __shfl_xor(sum - comp, 32, 64);
        if (act && half == 0) A.parts[A.t_out[j]] += ((double)(sum - comp) + (double)other) / (4.0 * LPB_PI * F.eps_t);
    }
}

// FP32 form.  Every position relative to the target leaf centre is carried as
// hi + lo (two FP32 numbers; sources formed in FP64 while staging), so the
// difference of two close points keeps its relative accuracy: FP32 positions
// alone would lose eps32 * h / r of it for a pair at distance r in a leaf of
// side h.  The first U-list leaf is the target's own (the r = 0 self pair is
// excluded there only); terms are summed in groups of eight or four and the group
// sums are added with Kahan compensation.
// positions are pre-scaled by s = lambda log2(e): with r' = s r the term is
// q e^{-lambda r} / r = s q 2^{-r'} / r' (the factor s is applied once per
// target); the hardware 2^x is used directly (terms below 2^-126 relative to
// q / r' are negligible, so its flush of denormal results does not matter)
// The hi parts alone (offsets below 1.5 h per axis, h the leaf side) give a
// distance to within 3.1e-7 h, i.e. 5e-6 of r at worst for r >= h/16, where
// such rounding errors of independent pairs largely cancel in the sum; only a
// pair closer than h/16 takes the lo parts.  Sources are taken eight (then four) at a time: hi-part distances
// first, and the lo parts only in the (rare) groups holding such a pair.
__device__ inline float p2p_term32(float w, float r2)
{
    const float ri = __frsqrt_rn(r2);
    return w * __builtin_amdgcn_exp2f(-(r2 * ri)) * ri;
}

// acc + the same term, as one fused multiply-add (w / r' times 2^{-r'})
__device__ inline float p2p_fma32(float w, float r2, float acc)
{
    const float ri = __frsqrt_rn(r2);
    return fmaf(w * ri, __builtin_amdgcn_exp2f(-(r2 * ri)), acc);
}

// The hi/lo splits of targets and sources must round identically (a pair at
// one point must give exactly zero): the scaled position is rounded to FP64
// on its own, never fused into the subtraction that forms the lo part.
__device__ inline double mul_rn(double a, double b)
{
#pragma clang fp contract(off)
    return a * b;
}

__global__ void __launch_bounds__(64) k_p2p_free32(EvalArgs<float> A)
{
    constexpr int SMAX = 256;
    __shared__ float4 sh[SMAX];   // x, y, z (hi) and q
    __shared__ float4 sl[SMAX];   // x, y, z (lo)
    const int leaf = A.p2p_free_leaves[blockIdx.x];
    const FmmDev& F = A.fmm[A.tl_fmm[leaf]];
    const double sc = F.lam_t * 1.4426950408889634;   // lambda log2(e)
    const int t0 = A.p2p_free_t0[blockIdx.x], t1 = min(A.tl_start[leaf + 1], t0 + 64);
    const float thr2 = (float)((A.tl_h[leaf] * sc / 16.0) * (A.tl_h[leaf] * sc / 16.0));
    const double tcx = A.tl_ctr[3 * leaf], tcy = A.tl_ctr[3 * leaf + 1], tcz = A.tl_ctr[3 * leaf + 2];
    const int lane = threadIdx.x, half = lane >> 5, tl = lane & 31;
    const int k0 = A.p2p_ptr[leaf], k1 = A.p2p_ptr[leaf + 1];
    const int nself = A.sl_start[A.p2p_src[k0] + 1] - A.sl_start[A.p2p_src[k0]];
    for (int base = t0; base < t1; base += 32) {
        const int j = base + tl;
        const bool act = j < t1;
        // target offset (hi + lo), scaled in FP64 and split again
        const double TX = act ? mul_rn((double)A.t_ux[j] + (double)A.t_lx[j], sc) : 0.0;
        const double TY = act ? mul_rn((double)A.t_uy[j] + (double)A.t_ly[j], sc) : 0.0;
        const double TZ = act ? mul_rn((double)A.t_uz[j] + (double)A.t_lz[j], sc) : 0.0;
        const float xh = (float)TX, yh = (float)TY, zh = (float)TZ;
        const float xl = (float)(TX - (double)xh), yl = (float)(TY - (double)yh), zl = (float)(TZ - (double)zh);
        float sum = 0.f, comp = 0.f;
        auto kahan = [&](float v) {
            float y = v - comp;
            float t = sum + y;
            comp = (t - sum) - y;
            sum = t;
        };
        int k = k0, s = A.sl_start[A.p2p_src[k0]], staged = 0;
        while (k < k1) {
            // stage up to SMAX sources, continuing across source leaves
            int n = 0;
            __syncthreads();
            while (k < k1 && n < SMAX) {
                const int sl_i = A.p2p_src[k];
                const int se = A.sl_start[sl_i + 1];
                const int take = min(se - s, SMAX - n);
                const double ox = A.sl_ctr[3 * sl_i] - tcx, oy = A.sl_ctr[3 * sl_i + 1] - tcy,
                             oz = A.sl_ctr[3 * sl_i + 2] - tcz;
                for (int i = lane; i < take; i += 64) {
                    const double X = mul_rn(((double)A.s_ux[s + i] + (double)A.s_lx[s + i]) + ox, sc);
                    const double Y = mul_rn(((double)A.s_uy[s + i] + (double)A.s_ly[s + i]) + oy, sc);
                    const double Z = mul_rn(((double)A.s_uz[s + i] + (double)A.s_lz[s + i]) + oz, sc);
                    const float hx = (float)X, hy = (float)Y, hz = (float)Z;
                    sh[n + i] = make_float4(hx, hy, hz, A.qs[s + i]);
                    sl[n + i] = make_float4((float)(X - (double)hx), (float)(Y - (double)hy), (float)(Z - (double)hz), 0.f);
                }
                n += take;
                s += take;
                if (s >= se) {
                    ++k;
                    if (k < k1) s = A.sl_start[A.p2p_src[k]];
                }
            }
            __syncthreads();
            if (act) {
                // staged sources below nself belong to the target's own leaf
                const int ns = min(max(nself - staged, 0), n);
                auto full_r2 = [&](int i) {
                    const float4 hs = sh[i], ls = sl[i];
                    const float dx = (xh - hs.x) + (xl - ls.x), dy = (yh - hs.y) + (yl - ls.y),
                                dz = (zh - hs.z) + (zl - ls.z);
                    return dx * dx + dy * dy + dz * dz;
                };
                for (int jj = half; jj < ns; jj += 2) {
                    const float r2 = full_r2(jj);
                    if (r2 > 0.f) kahan(p2p_term32(sh[jj].w, r2));
                }
                // the main loop's counter is wave-uniform (each half starts at
                // its own parity within it); the tails continue per lane
                const int par = (half - ns) & 1;
                const float4* shp = sh + par;
                int ju = ns;
                for (; ju + 15 < n; ju += 16) {
                    float w[8], r2[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        const float4 hs = shp[ju + 2 * u];
                        const float dx = xh - hs.x, dy = yh - hs.y, dz = zh - hs.z;
                        w[u] = hs.w;
                        r2[u] = dx * dx + dy * dy + dz * dz;
                    }
                    const float mn = fminf(fminf(fminf(r2[0], r2[1]), fminf(r2[2], r2[3])),
                                           fminf(fminf(r2[4], r2[5]), fminf(r2[6], r2[7])));
                    if (mn < thr2) {
#pragma unroll
                        for (int u = 0; u < 8; ++u) r2[u] = full_r2(ju + par + 2 * u);
                    }
                    float s8 = 0.f;
#pragma unroll
                    for (int u = 0; u < 8; ++u) s8 = p2p_fma32(w[u], r2[u], s8);
                    kahan(s8);
                }
                int jj = ju + par;
                for (; jj + 6 < n; jj += 8) {
                    float w[4], r2[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const float4 hs = sh[jj + 2 * u];
                        const float dx = xh - hs.x, dy = yh - hs.y, dz = zh - hs.z;
                        w[u] = hs.w;
                        r2[u] = dx * dx + dy * dy + dz * dz;
                    }
                    if (fminf(fminf(r2[0], r2[1]), fminf(r2[2], r2[3])) < thr2) {
#pragma unroll
                        for (int u = 0; u < 4; ++u) r2[u] = full_r2(jj + 2 * u);
                    }
                    kahan((p2p_term32(w[0], r2[0]) + p2p_term32(w[1], r2[1])) +
                          (p2p_term32(w[2], r2[2]) + p2p_term32(w[3], r2[3])));
                }
                for (; jj < n; jj += 2) kahan(p2p_term32(sh[jj].w, full_r2(jj)));
            }
            staged += n;
        }
        // combine the two halves (lane l and l+32 share a target)
        const float other = __shfl_xor(sum - comp, 32, 64);
        if (act && half == 0) A.parts[A.t_out[j]] += ((double)(sum - comp) + (double)other) * sc / (4.0 * LPB_PI * F.eps_t);
    }
}

// ---------------------------------------------------------------------------
// Reaction near field (Algorithm 1, last step): every pair is the integral
//   u~ = (1/4pi) int_0^inf lrho J_0(lrho rho) e^{-l_z zt + l'_z zs} sigma(lrho) / l_z dlrho
// (canonical frame: zt > 0 target height, zs < 0 image depth), by composite
// 20-point Gauss-Legendre on panels chosen as for the M2L initial values.
// FP64 always.  One thread per target, over the (component, source leaf)
// pairs of its leaf (every component of the leaf's target tree).
template <typename T>
__global__ void k_p2p_react(EvalArgs<T> A)
{
    int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= A.n_react_targets) return;
    const int leaf = A.react_tgt_leaf[idx];
    const int j = A.react_tgt_slot[idx];
    const double tx = A.tl_ctr[3 * leaf] + (double)A.t_ux[j];
    const double ty = A.tl_ctr[3 * leaf + 1] + (double)A.t_uy[j];
    const double tz = A.tl_ctr[3 * leaf + 2] + (double)A.t_uz[j];
    const double lt_tol = log(A.quad_tol);
    double total = 0.0;
    for (int k = A.rp_ptr[leaf]; k < A.rp_ptr[leaf + 1]; ++k) {
        const FmmDev& F = A.fmm[A.rp_fmm[k]];
        const Medium& Md = A.media[F.medium];
        double lmin = Md.lam[0], dmax = 0.0;
        for (int kk = 1; kk <= Md.L; ++kk) lmin = fmin(lmin, Md.lam[kk]);
        for (int kk = 1; kk < Md.L; ++kk) dmax = fmax(dmax, Md.d[kk - 1] - Md.d[kk]);
        double w0 = lmin;
        if (dmax > 0.0 && LPB_PI / (2.0 * dmax) < w0) w0 = LPB_PI / (2.0 * dmax);
        const double lt = F.lam_t, ls = F.lam_s;
        int sl = A.rp_src[k];
        for (int s = A.sl_start[sl]; s < A.sl_start[sl + 1]; ++s) {
            double sxp = A.sl_ctr[3 * sl] + (double)A.s_ux[s];
            double syp = A.sl_ctr[3 * sl + 1] + (double)A.s_uy[s];
            double szp = A.sl_ctr[3 * sl + 2] + (double)A.s_uz[s];
            double rho = sqrt((tx - sxp) * (tx - sxp) + (ty - syp) * (ty - syp));
            double c = tz - szp;
            // envelope lrho e^{-c lrho}: X from 1 * log(X/x*) - c (X - x*) = log(tol)
            double xs = 1.0 / c, hi = xs + 1.0 / c, step = 1.0 / c;
            while (log(hi / xs) - c * (hi - xs) > lt_tol) { step *= 2.0; hi = xs + step; }
            double lo = xs;
            for (int it = 0; it < 80; ++it) {
                double mid = 0.5 * (lo + hi);
                if (log(mid / xs) - c * (mid - xs) > lt_tol) lo = mid; else hi = mid;
            }
            double X = hi, a = 0.0, acc = 0.0;
            while (a < X) {
                double w = fmax(w0, 0.8 * a);
                w = fmin(w, 4.5 / c);
                if (rho > 0.0) w = fmin(w, 1.1 * LPB_PI / rho);
                for (int q = 0; q < 20; ++q) {
                    double t = a + 0.5 * w * (A.gl_x[q] + 1.0);
                    double lz = sqrt(lt * lt + t * t), lzp = sqrt(ls * ls + t * t);
                    double sg = sigma_transmission(Md.L, Md.eps, Md.lam, Md.d, F.l, F.lp, F.a, F.b, t);
                    acc += 0.5 * w * A.gl_w[q] * t * j0(t * rho) * exp(-lz * tz + lzp * szp) * sg / lz;
                }
                a += w;
            }
            total += (double)A.qs[s] * acc;
        }
    }
    A.parts[A.t_out[j]] += total / (4.0 * LPB_PI);
}

// ---------------------------------------------------------------------------
// Component sum (eq. totalinteraction): phi[i] = sum_slot parts[slot][i]
__global__ void k_sum(int64_t n, int nslots, const double* __restrict__ parts, double* __restrict__ phi)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    for (int k = 0; k < nslots; ++k) s += parts[(size_t)k * n + i];
    phi[i] = s;
}

// ---------------------------------------------------------------------------
template <typename T>
hipError_t eval_run(const EvalArgs<T>& A, const EvalSched& S, int stages, hipStream_t st, hipEvent_t* ev)
{
#define LPB_MARK(k) \
    if (ev) (void)hipEventRecord(ev[k], st)
    const int K = A.K, p = A.p;
    LPB_MARK(0);
    if (A.n_src > 0) hipLaunchKernelGGL(k_gather_q<T>, dim3((A.n_src + 255) / 256), dim3(256), 0, st, A.n_src, A.s_cidx, A.q, A.qs);
    hipLaunchKernelGGL(k_zero<double>, dim3(1024), dim3(256), 0, st, (size_t)A.nslots * A.ncharges, A.parts);
    if (A.n_le > 0) hipLaunchKernelGGL(k_zero<T>, dim3(1024), dim3(256), 0, st, (size_t)A.n_le * A.KP, A.le);
    const bool far = stages & 1, near = stages & 2;
    LPB_MARK(1);
    // upward pass
    // point chunks sized so that a block's LDS stays under 24 KB (several blocks per CU)
    auto pick_ch = [&](size_t per_ch, size_t fixed) {
        int ch = 64;
        while (ch > 8 && fixed + per_ch * ch > 24u * 1024u) ch >>= 1;
        return ch;
    };
    // P2M / L2P with the order fixed at compile time where it is specialised
    bool p_fixed = false;
    if constexpr (sizeof(T) == 4) p_fixed = p >= 2 && p <= 15;
    if (far && S.n_p2m > 0) {
        if constexpr (sizeof(T) == 4) {
            if (p_fixed) {
#define LPB_P2M(PP) \
    case PP: hipLaunchKernelGGL(k_p2m_p<PP>, dim3((S.n_p2m + 1) / 2), dim3(64), 0, st, A, S.n_p2m); break;
                switch (p) {
                    LPB_P2M(2) LPB_P2M(3) LPB_P2M(4) LPB_P2M(5) LPB_P2M(6) LPB_P2M(7) LPB_P2M(8) LPB_P2M(9)
                    LPB_P2M(10) LPB_P2M(11) LPB_P2M(12) LPB_P2M(13) LPB_P2M(14) LPB_P2M(15)
                default: break;
                }
#undef LPB_P2M
            }
        }
        if (!p_fixed) {
            int ch = pick_ch(sizeof(T) * ((size_t)K + p + 1), sizeof(T) * (size_t)K);
            size_t sm = sizeof(T) * ((size_t)K * (ch + 1) + (size_t)(p + 1) * ch);
            hipLaunchKernelGGL(k_p2m<T>, dim3(S.n_p2m), dim3(64), sm, st, A, ch);
        }
    }
    LPB_MARK(2);
    for (int l = kMaxDepth; l >= 0 && far; --l) launch_batched<T>(A, S.bm2m_lv[l], S.bm2m_lv[l + 1], A.me, A.n_me, A.me, 0, st);
    // V-list translations (all levels), then the downward pass
    LPB_MARK(3);
    if (far && A.n_tiles > 0) launch_m2l_tile<T>(A, st);
    LPB_MARK(4);
    if (far && S.bm2l_w1 > S.bm2l_w0) {
        launch_batched_x<T, true>(A, S.bm2l_w0, S.bm2l_w1, A.me, A.n_me, A.m2l_scratch, 0, st);
        hipLaunchKernelGGL(k_m2l_reduce<T>, dim3(S.n_m2l_boxes), dim3(128), 0, st, A);
    }
    LPB_MARK(5);
    for (int l = 0; l <= kMaxDepth && far; ++l) launch_batched<T>(A, S.bl2l_lv[l], S.bl2l_lv[l + 1], A.le, A.n_le, A.le, 1, st);
    LPB_MARK(6);
    if (far && S.n_l2p > 0) {
        if constexpr (sizeof(T) == 4) {
            if (p_fixed) {
#define LPB_L2P(PP) \
    case PP: hipLaunchKernelGGL(k_l2p_p<PP>, dim3((S.n_l2p + 1) / 2), dim3(64), 0, st, A, S.n_l2p); break;
                switch (p) {
                    LPB_L2P(2) LPB_L2P(3) LPB_L2P(4) LPB_L2P(5) LPB_L2P(6) LPB_L2P(7) LPB_L2P(8) LPB_L2P(9)
                    LPB_L2P(10) LPB_L2P(11) LPB_L2P(12) LPB_L2P(13) LPB_L2P(14) LPB_L2P(15)
                default: break;
                }
#undef LPB_L2P
            }
        }
        if (!p_fixed) {
            size_t sm = sizeof(T) * (size_t)(p + 1) * 64;
            hipLaunchKernelGGL(k_l2p<T>, dim3(S.n_l2p), dim3(64), sm, st, A, 64);
        }
    }
    // near field
    LPB_MARK(7);
    if (near && S.n_p2p_free > 0) {
        if constexpr (sizeof(T) == 4) hipLaunchKernelGGL(k_p2p_free32, dim3(S.n_p2p_free), dim3(64), 0, st, A);
        else hipLaunchKernelGGL(k_p2p_free<T>, dim3(S.n_p2p_free), dim3(64), 0, st, A);
    }
    LPB_MARK(8);
    if (near && A.n_react_targets > 0)
        hipLaunchKernelGGL(k_p2p_react<T>, dim3((A.n_react_targets + 63) / 64), dim3(64), 0, st, A);
    LPB_MARK(9);
    if (A.ncharges > 0)
        hipLaunchKernelGGL(k_sum, dim3((unsigned)((A.ncharges + 255) / 256)), dim3(256), 0, st, A.ncharges, A.nslots, A.parts, A.phi);
    LPB_MARK(10);
#undef LPB_MARK
    return hipGetLastError();
}

template hipError_t eval_run<double>(const EvalArgs<double>&, const EvalSched&, int, hipStream_t, hipEvent_t*);
template hipError_t eval_run<float>(const EvalArgs<float>&, const EvalSched&, int, hipStream_t, hipEvent_t*);

template <typename T>
hipError_t stage_run(const EvalArgs<T>& A, const EvalSched& S, int which, hipStream_t st)
{
    if (which == 0) {
        if (A.n_tiles > 0) launch_m2l_tile<T>(A, st);
    } else {
        for (int l = kMaxDepth; l >= 0; --l) launch_batched<T>(A, S.bm2m_lv[l], S.bm2m_lv[l + 1], A.me, A.n_me, A.me, 0, st);
        launch_batched_x<T, true>(A, S.bm2l_w0, S.bm2l_w1, A.me, A.n_me, A.m2l_scratch, 0, st);
        for (int l = 0; l <= kMaxDepth; ++l) launch_batched<T>(A, S.bl2l_lv[l], S.bl2l_lv[l + 1], A.le, A.n_le, A.le, 1, st);
    }
    return hipGetLastError();
}
template hipError_t stage_run<double>(const EvalArgs<double>&, const EvalSched&, int, hipStream_t);
template hipError_t stage_run<float>(const EvalArgs<float>&, const EvalSched&, int, hipStream_t);

}  // namespace lpb
