// lpb_eval.hip -- evaluation kernels of Algorithm 2 (every FMM of every
// system per launch): gather charges, P2M, M2M, M2L, L2L, L2P, near field
// (free-space and reaction), and the component sum.  Templated on the
// arithmetic type T (double for LPB_FP64, float for LPB_MIXED); Bessel
// ratios are always formed in double.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "lpb_eval_dev.h"

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
    const double* __restrict__ ith = A.ith_s + ((size_t)A.sl_fmm[leaf] * (kMaxDepth + 1) + A.sl_lv[leaf]) * (LPB_MAX_P + 1);
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
// (Re, Im) pair by +m phi (sources) or -m phi (results) (code kXfRotate +
// dir, phi the azimuth of the V-list direction dir).
// Every thread of the 256 takes column j = tid & 63 and a quarter of the rows.
// cs[m * 128 + j] = cos(m phi_j), cs[m * 128 + 64 + j] = sin(m phi_j), m = 1..p,
// copied from the direction table rot[dir][m][cos, sin]
template <typename T>
__device__ inline void column_trig(T* cs, int p, int code, const T* __restrict__ rot)
{
    const int j = threadIdx.x & 63, part = threadIdx.x >> 6;
    if (code < kXfRotate) return;
    const T* r = rot + (size_t)(code - kXfRotate) * (p + 1) * 2;
    for (int m = 1 + part; m <= p; m += 4) {
        cs[m * 128 + j] = r[2 * m];
        cs[m * 128 + 64 + j] = r[2 * m + 1];
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
    // the (n, m >= 1) pairs in order n = 1.., m = 1..n; this thread takes
    // every fourth, starting at number `part`
    int n = 1, m = 1;
    for (int k = 0; k < part; ++k)
        if (++m > n) { ++n; m = 1; }
    while (n <= p) {
        const T c = cs[m * 128 + j], sn = result ? -cs[m * 128 + 64 + j] : cs[m * 128 + 64 + j];
        T& re = Bs[ire(n, m) * NTP + j];
        T& im = Bs[iim(n, m) * NTP + j];
        const T a = re, b = im;
        re = a * c - b * sn;
        im = a * sn + b * c;
        for (int k = 0; k < 4; ++k)
            if (++m > n) { ++n; m = 1; }
    }
}

// RBF = ceil(KB / (4 / WC)): the row blocks per wave of a whole item, which
// also sizes the source staging; GY blocks along y split them (RB per wave
// each).  WC = 2 arranges the four waves as 2 x 2 (row blocks x halves of
// the 64 columns), so that KB = 2 or 6 row blocks give every wave the same
// number of products (with WC = 1 one wave of four would idle); FP32 only.
// XF (untiled V-list pairs): the sources are brought into the frame of the
// stored operator here; the results stay in that frame (the reduction over a
// box's pairs applies the inverse transform).
// A block takes the work items it, it + gridDim.x, ... of the launch (one
// each when the grid covers them all; a smaller grid keeps its blocks
// resident and gathers the next item's first sources during the current
// item's last product and write-back).  Items are independent, so results
// do not depend on the grid or the order.
// MT: items of several terms (M2M: one per child octant), summed with Kahan
// compensation; single-term items (L2L, untiled M2L) store the product as is
template <typename T, int RBF, bool XF, int GY, bool MT, int WC>
__global__ void __launch_bounds__(256) k_batched(const T* __restrict__ in, T* out, const int* __restrict__ term_ptr,
                                                 const int* __restrict__ term_op, const int* __restrict__ term_src,
                                                 const int* __restrict__ dst, int wbase, int nitems, int mode, int K,
                                                 int KP, const T* __restrict__ pool_swz, int zrow, int sched,
                                                 const int* __restrict__ xcode, const T* __restrict__ rot,
                                                 const T* __restrict__ refl, int p)
{
    typedef typename Vec4<T>::type V4;
    static_assert(GY == 1 || !XF, "results with a transform need whole columns");
    static_assert(WC == 1 || (WC == 2 && GY == 1), "column halves only with whole items per block");
    constexpr int RB = (RBF + GY - 1) / GY;
    constexpr int NT = 64, CB = 4 / WC, GMAX = (4 / WC) * RBF;
    constexpr int NTP = NT + (sizeof(T) == 4 ? 16 : 8);
    extern __shared__ unsigned char smem_raw[];
    T* Bs = reinterpret_cast<T*>(smem_raw);   // [KP][NTP]
    const int KB = KP / 16;
    const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
    // row-block group of this wave: blocks of a work item along y split the
    // output rows (every block stages all of the sources)
    const int wy = (GY > 1 ? (int)blockIdx.y * 4 : 0) + w / WC, wc = w % WC;
    // source staging: thread (column gj, part gpart) moves coefficients
    // 16 i + 4 gpart + e of column gj; the lanes of a wave take 64 columns, so
    // their LDS stores fall in distinct banks
    const int gj = tid & 63, gpart = tid >> 6;
    V4 acc[RB][CB], tot[RB][CB], cmp[RB][CB];
    V4 greg[GMAX];
    // XF: per-column transform code and, for rotations, cos / sin (m phi) after B in LDS
    T* trig = Bs + (size_t)KP * NTP;
    auto fetch = [&](int t) {
        const int sidx = term_src[(size_t)t * NT + gj];
        const T* src = in + (size_t)(sidx < 0 ? zrow : sidx) * KP + 4 * gpart;   // missing: the zero row
#pragma unroll
        for (int i = 0; i < GMAX; ++i) greg[i] = (i < KB) ? *reinterpret_cast<const V4*>(src + 16 * i) : V4{0, 0, 0, 0};
    };
    auto item = [&](int it) { return wbase + sched_index(it, nitems, sched & 1); };
    bool staged_next = false;
    for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
        const int wi = item(it);
        const int t0 = term_ptr[wi], t1 = term_ptr[wi + 1];
        const int nit = it + (int)gridDim.x;
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int cb = 0; cb < CB; ++cb) {
                if constexpr (MT) tot[rb][cb] = cmp[rb][cb] = V4{0, 0, 0, 0};
                else acc[rb][cb] = V4{0, 0, 0, 0};
            }
        const int xc = XF ? xcode[(size_t)wi * NT + (tid & 63)] : -1;
        if (XF) column_trig<T>(trig, p, xc, rot);
        if (t0 < t1 && !staged_next) fetch(t0);
        staged_next = false;
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
            if (t + 1 < t1) {
                fetch(t + 1);
            } else if (nit < nitems) {
                // the next item's first sources load during this product
                const int nwi = item(nit);
                if (term_ptr[nwi] < term_ptr[nwi + 1]) {
                    fetch(term_ptr[nwi]);
                    staged_next = true;
                }
            }
            mma_block<T, RB, CB>(Aw, Bs + wc * CB * 16, NTP, KB, wy, l, acc);
            if constexpr (MT) accumulate<T, RB, CB>(acc, tot, cmp);
        }
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
            int rbg = wy * RB + rb;
            if (rbg >= KB) continue;
#pragma unroll
            for (int cb = 0; cb < CB; ++cb) {
                const int d = dst[(size_t)wi * NT + (wc * CB + cb) * 16 + (l & 15)];
                if (d < 0) continue;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    int row = rbg * 16 + mfma_row(T(0), l, r);
                    if (row >= K) continue;
                    const T v = MT ? tot[rb][cb][r] : acc[rb][cb][r];
                    // (the untiled M2L's scratch rows are K long, the expansions KP)
                    const size_t o = (size_t)d * (XF ? K : KP) + row;
                    if (mode == 0) out[o] = v;
                    else out[o] += v;
                }
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
    int RB = (KB + 3) / 4;
    const int gy = (!XF && n < 512 && RB >= 2) ? 2 : 1;
    // FP32, KB = 2 or 6: waves as 2 x 2 (rows x column halves), KB / 2 row
    // blocks each (in FP64 the three blocks' registers cost occupancy)
    const bool wc2 = sizeof(T) == 4 && gy == 1 && (KB == 2 || KB == 6);
    if (wc2) RB = (KB + 1) / 2;
    const size_t sm = sizeof(T) * ((size_t)A.KP * (64 + (sizeof(T) == 4 ? 16 : 8)) + (XF ? (size_t)(A.p + 1) * 128 : 0));
    // schedule bits 1-2: 0 one block per item, else 256 CUs x {2, 4, 8} resident blocks looping over the items
    const int pers = (A.batch_sched >> 1) & 3;
    const int gx = pers == 0 ? n : std::min(n, 256 * (1 << pers));
    dim3 g(gx, gy), b(256);
#define LPB_BATCHED_MT(R, MT)                                                                                               \
    if constexpr (!XF) {                                                                                                    \
        if (gy == 2) {                                                                                                      \
            hipLaunchKernelGGL((k_batched<T, R, XF, 2, MT, 1>), g, b, sm, st, in, out, A.bw_term_ptr, A.bw_op, A.bw_src,     \
                               A.bw_dst, w0, n, mode, A.K, A.KP, A.pool_swz, zrow, A.batch_sched, A.bw_xc, A.rot_tab,      \
                               A.refl_sign, A.p);                                                                           \
            break;                                                                                                          \
        }                                                                                                                   \
    }                                                                                                                       \
    if constexpr (sizeof(T) == 4 && (R == 1 || R == 3)) {                                                                   \
        if (wc2) {                                                                                                          \
            hipLaunchKernelGGL((k_batched<T, R, XF, 1, MT, 2>), g, b, sm, st, in, out, A.bw_term_ptr, A.bw_op, A.bw_src,     \
                               A.bw_dst, w0, n, mode, A.K, A.KP, A.pool_swz, zrow, A.batch_sched, A.bw_xc, A.rot_tab,      \
                               A.refl_sign, A.p);                                                                           \
            break;                                                                                                          \
        }                                                                                                                   \
    }                                                                                                                       \
    hipLaunchKernelGGL((k_batched<T, R, XF, 1, MT, 1>), g, b, sm, st, in, out, A.bw_term_ptr, A.bw_op, A.bw_src, A.bw_dst,  \
                       w0, n, mode, A.K, A.KP, A.pool_swz, zrow, A.batch_sched, A.bw_xc, A.rot_tab, A.refl_sign, A.p)
    // M2M items sum eight terms (mode 0 without a transform); L2L and untiled
    // M2L items have one
#define LPB_BATCHED(R)                \
    if (!XF && mode == 0) {           \
        LPB_BATCHED_MT(R, true);      \
    } else {                          \
        LPB_BATCHED_MT(R, false);     \
    }
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
#undef LPB_BATCHED_MT
}
template <typename T>
static void launch_batched(const EvalArgs<T>& A, int w0, int w1, const T* in, int zrow, T* out, int mode, hipStream_t st)
{
    launch_batched_x<T, false>(A, w0, w1, in, zrow, out, mode, st);
}

// V-list pairs outside the tiled levels: LE[box] += sum of the box's pair rows
// of the scratch, each brought back from the frame of its stored operator
// (reflection signs, or the rotation of every order-m (Re, Im) pair by
// -m phi): row' = a row + b partner row with (a, b) from a table per
// transform code and row.  A 256-thread block per box: lane l of wave w
// takes row 64 c + l (c = 0, 1, ... over the rows) and the chunks of eight
// consecutive pairs w, w + 4, ... of the box's list in order (the last
// pairs one by one), a chunk's loads in flight together; the
// partner row (the neighbouring row, always in the same 64-row chunk for
// p <= 20) comes from the neighbouring lane.  Wave 0 then adds the other
// waves' sums in wave order, so the result does not depend on timing.  In
// FP32 the sums are compensated (Kahan), so they keep the error of a single
// pair's product.
template <typename T>
__global__ void __launch_bounds__(256) k_m2l_reduce(EvalArgs<T> A)
{
    typedef typename Vec2<T>::type V2;
    constexpr int G = 4, U = 8;
    __shared__ T part[2][G - 1][64];
    const int le = A.m2l_boxes[blockIdx.x];
    const int k0 = A.m2l_ptr[le], k1 = A.m2l_ptr[le + 1];
    const int K = A.K;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), l = threadIdx.x & 63;
    const V2* __restrict__ xf = reinterpret_cast<const V2*>(A.xf_ab);
    for (int rc = 0; rc < K; rc += 64) {
        const int row = rc + l;
        const bool live = row < K;
        // the partner row of an order-m (Re, Im) pair: (n^2 + 2m - 1, n^2 + 2m)
        int n = 0;
        while ((n + 1) * (n + 1) <= row) ++n;
        const int idx = row - n * n;
        const int plane = idx == 0 ? l : ((idx & 1) ? l + 1 : l - 1);
        const int rr = live ? row : 0;
        T s = T(0), c = T(0);
        auto add = [&](T a) {
            if constexpr (sizeof(T) == 4) {
                const T y = a - c, t = s + y;
                c = (t - s) - y;
                s = t;
            } else {
                s += a;
            }
        };
        // chunks of U consecutive pairs, chunk i to wave i mod G; then the
        // last pairs one by one, pair j to wave j mod G
        const int nfull = (k1 - k0) / U;
        for (int ci = w; ci < nfull; ci += G) {
            const int k = k0 + ci * U;
            int code[U];
            T own[U];
            V2 ab[U];
#pragma unroll
            for (int u = 0; u < U; ++u) code[u] = A.m2l_xc[k + u];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                own[u] = A.m2l_scratch[(size_t)(k + u) * K + rr];
                ab[u] = xf[(size_t)code[u] * K + rr];
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (!live) own[u] = T(0);
                const T other = __shfl(own[u], plane);
                add(own[u] * ab[u].x + other * ab[u].y);
            }
        }
        for (int k = k0 + nfull * U + w; k < k1; k += G) {
            const V2 ab = xf[(size_t)A.m2l_xc[k] * K + rr];
            T own = A.m2l_scratch[(size_t)k * K + rr];
            if (!live) own = T(0);
            const T other = __shfl(own, plane);
            add(own * ab.x + other * ab.y);
        }
        if (w > 0) {
            part[0][w - 1][l] = s;
            part[1][w - 1][l] = c;
        }
        __syncthreads();
        if (w == 0 && live) {
            // a wave's compensated sum is s - c
#pragma unroll
            for (int g = 0; g < G - 1; ++g) {
                add(part[0][g][l]);
                if constexpr (sizeof(T) == 4) add(-part[1][g][l]);
            }
            A.le[(size_t)le * A.KP + row] += s;
        }
        __syncthreads();
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
    const double* __restrict__ ith = A.ith_t + ((size_t)A.tl_fmm[leaf] * (kMaxDepth + 1) + A.tl_lv[leaf]) * (LPB_MAX_P + 1);
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
    const int t0 = A.p2p_free_t0[blockIdx.x], t1 = min(A.tl_start[leaf + 1], t0 + (A.p2p_free_ts[blockIdx.x] & 255));
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
        if (act && half == 0) A.parts[A.near_off + A.t_out[j]] += ((double)(sum - comp) + (double)other) / (4.0 * LPB_PI * F.eps_t);
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
    // T targets on T x S lanes: lane = target tl + T * split s; split s takes
    // the staged sources j = s (mod S)
    const int ts = A.p2p_free_ts[blockIdx.x], T = ts & 255, S = ts >> 8;
    const int t0 = A.p2p_free_t0[blockIdx.x], t1 = min(A.tl_start[leaf + 1], t0 + T);
    const float thr2 = (float)((A.tl_h[leaf] * sc / 16.0) * (A.tl_h[leaf] * sc / 16.0));
    const double tcx = A.tl_ctr[3 * leaf], tcy = A.tl_ctr[3 * leaf + 1], tcz = A.tl_ctr[3 * leaf + 2];
    const int lane = threadIdx.x, s = lane / T, tl = lane - s * T;
    const int k0 = A.p2p_ptr[leaf], k1 = A.p2p_ptr[leaf + 1];
    const int nself = A.sl_start[A.p2p_src[k0] + 1] - A.sl_start[A.p2p_src[k0]];
    const int j = t0 + tl;
    const bool act = s < S && j < t1;
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
    int k = k0, src = A.sl_start[A.p2p_src[k0]], staged = 0;
    while (k < k1) {
        // stage up to SMAX sources, continuing across source leaves
        int n = 0;
        __syncthreads();
        while (k < k1 && n < SMAX) {
            const int sl_i = A.p2p_src[k];
            const int se = A.sl_start[sl_i + 1];
            const int take = min(se - src, SMAX - n);
            const double ox = A.sl_ctr[3 * sl_i] - tcx, oy = A.sl_ctr[3 * sl_i + 1] - tcy, oz = A.sl_ctr[3 * sl_i + 2] - tcz;
            for (int i = lane; i < take; i += 64) {
                const double X = mul_rn(((double)A.s_ux[src + i] + (double)A.s_lx[src + i]) + ox, sc);
                const double Y = mul_rn(((double)A.s_uy[src + i] + (double)A.s_ly[src + i]) + oy, sc);
                const double Z = mul_rn(((double)A.s_uz[src + i] + (double)A.s_lz[src + i]) + oz, sc);
                const float hx = (float)X, hy = (float)Y, hz = (float)Z;
                sh[n + i] = make_float4(hx, hy, hz, A.qs[src + i]);
                sl[n + i] = make_float4((float)(X - (double)hx), (float)(Y - (double)hy), (float)(Z - (double)hz), 0.f);
            }
            n += take;
            src += take;
            if (src >= se) {
                ++k;
                if (k < k1) src = A.sl_start[A.p2p_src[k]];
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
            for (int jj = s; jj < ns; jj += S) {
                const float r2 = full_r2(jj);
                if (r2 > 0.f) kahan(p2p_term32(sh[jj].w, r2));
            }
            // the main loop's counter is wave-uniform (each split starts at its
            // own residue within it); the tails continue per lane
            const int par = ((s - ns) % S + S) % S;
            const float4* shp = sh + par;
            int ju = ns;
            for (; ju + 8 * S - 1 < n; ju += 8 * S) {
                float w[8], r2[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const float4 hs = shp[ju + S * u];
                    const float dx = xh - hs.x, dy = yh - hs.y, dz = zh - hs.z;
                    w[u] = hs.w;
                    r2[u] = dx * dx + dy * dy + dz * dz;
                }
                const float mn = fminf(fminf(fminf(r2[0], r2[1]), fminf(r2[2], r2[3])),
                                       fminf(fminf(r2[4], r2[5]), fminf(r2[6], r2[7])));
                if (mn < thr2) {
#pragma unroll
                    for (int u = 0; u < 8; ++u) r2[u] = full_r2(ju + par + S * u);
                }
                float s8 = 0.f;
#pragma unroll
                for (int u = 0; u < 8; ++u) s8 = p2p_fma32(w[u], r2[u], s8);
                kahan(s8);
            }
            int jj = ju + par;
            for (; jj + 3 * S < n; jj += 4 * S) {
                float w[4], r2[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const float4 hs = sh[jj + S * u];
                    const float dx = xh - hs.x, dy = yh - hs.y, dz = zh - hs.z;
                    w[u] = hs.w;
                    r2[u] = dx * dx + dy * dy + dz * dz;
                }
                if (fminf(fminf(r2[0], r2[1]), fminf(r2[2], r2[3])) < thr2) {
#pragma unroll
                    for (int u = 0; u < 4; ++u) r2[u] = full_r2(jj + S * u);
                }
                kahan((p2p_term32(w[0], r2[0]) + p2p_term32(w[1], r2[1])) +
                      (p2p_term32(w[2], r2[2]) + p2p_term32(w[3], r2[3])));
            }
            for (; jj < n; jj += S) kahan(p2p_term32(sh[jj].w, full_r2(jj)));
        }
        staged += n;
    }
    // the S partial sums of a target, added in split order (FP64)
    const float mine = sum - comp;
    double tot = (double)mine;
    for (int q = 1; q < 4; ++q) {
        const float other = __shfl(mine, min(tl + q * T, 63), 64);
        if (q < S) tot += (double)other;
    }
    if (act && s == 0) A.parts[A.near_off + A.t_out[j]] += tot * sc / (4.0 * LPB_PI * F.eps_t);
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
hipError_t eval_run(const EvalArgs<T>& A, const EvalSched& S, int stages, hipStream_t st, hipEvent_t* ev,
                    const EvalFork* fk)
{
#define LPB_MARK(k) \
    if (ev) (void)hipEventRecord(ev[k], st)
    const int K = A.K, p = A.p;
    LPB_MARK(0);
    if (A.n_src > 0) hipLaunchKernelGGL(k_gather_q<T>, dim3((A.n_src + 255) / 256), dim3(256), 0, st, A.n_src, A.s_cidx, A.q, A.qs);
    hipLaunchKernelGGL(k_zero<double>, dim3(1024), dim3(256), 0, st, (size_t)A.nslots * A.ncharges, A.parts);
    if (A.n_le > 0) hipLaunchKernelGGL(k_zero<T>, dim3(1024), dim3(256), 0, st, (size_t)A.n_le * A.KP, A.le);
    const bool far = stages & 1, near = stages & 2;
    // the free-space near field (its own slot) on the third stream beside the far field
    const bool near_split = near && S.n_p2p_free > 0 && far && fk && fk->near && !ev;
    auto run_near_free = [&](hipStream_t s) {
        if constexpr (sizeof(T) == 4) hipLaunchKernelGGL(k_p2p_free32, dim3(S.n_p2p_free), dim3(64), 0, s, A);
        else hipLaunchKernelGGL(k_p2p_free<T>, dim3(S.n_p2p_free), dim3(64), 0, s, A);
    };
    if (near_split) {
        hipError_t e = hipEventRecord(fk->near_fork, st);
        if (e == hipSuccess) e = hipStreamWaitEvent(fk->near, fk->near_fork, 0);
        if (e != hipSuccess) return e;
        run_near_free(fk->near);
        if ((e = hipEventRecord(fk->near_join, fk->near)) != hipSuccess) return e;
    }
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
            if (p_fixed) launch_p2m_fixed(A, S.n_p2m, S.p2m_nl, st);
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
    // the untiled V-list pairs write LE boxes of other levels or trees than
    // the tiled M2L: with a fork they run on the side stream beside it
    const bool list = far && S.bm2l_w1 > S.bm2l_w0;
    const bool split = list && fk && fk->side && !ev && A.n_tiles > 0;
    auto run_list = [&](hipStream_t s) {
        launch_batched_x<T, true>(A, S.bm2l_w0, S.bm2l_w1, A.me, A.n_me, A.m2l_scratch, 0, s);
        hipLaunchKernelGGL(k_m2l_reduce<T>, dim3(S.n_m2l_boxes), dim3(256), 0, s, A);
    };
    if (split) {
        hipError_t e = hipEventRecord(fk->fork, st);
        if (e == hipSuccess) e = hipStreamWaitEvent(fk->side, fk->fork, 0);
        if (e != hipSuccess) return e;
        run_list(fk->side);
        if ((e = hipEventRecord(fk->join, fk->side)) != hipSuccess) return e;
    }
    if (far && A.n_tiles > 0) launch_m2l_tile<T>(A, st);
    LPB_MARK(4);
    if (list && !split) run_list(st);
    if (split) {
        hipError_t e = hipStreamWaitEvent(st, fk->join, 0);
        if (e != hipSuccess) return e;
    }
    // X-lists of adaptive trees: local expansions from coarser leaves' sources
    if (far) launch_p2l<T>(A, st);
    LPB_MARK(5);
    for (int l = 0; l <= kMaxDepth && far; ++l) launch_batched<T>(A, S.bl2l_lv[l], S.bl2l_lv[l + 1], A.le, A.n_le, A.le, 1, st);
    LPB_MARK(6);
    if (far && S.n_l2p > 0) {
        if constexpr (sizeof(T) == 4) {
            if (p_fixed) launch_l2p_fixed(A, S.n_l2p, S.l2p_nl, st);
        }
        if (!p_fixed) {
            size_t sm = sizeof(T) * (size_t)(p + 1) * 64;
            hipLaunchKernelGGL(k_l2p<T>, dim3(S.n_l2p), dim3(64), sm, st, A, 64);
        }
    }
    // W-lists of adaptive trees: finer boxes' expansions at the leaves' targets
    if (far) launch_m2p<T>(A, st);
    // near field
    LPB_MARK(7);
    if (near && S.n_p2p_free > 0 && !near_split) run_near_free(st);
    LPB_MARK(8);
    if (near && A.n_react_targets > 0)
        hipLaunchKernelGGL(k_p2p_react<T>, dim3((A.n_react_targets + 63) / 64), dim3(64), 0, st, A);
    LPB_MARK(9);
    if (near_split) {
        hipError_t e = hipStreamWaitEvent(st, fk->near_join, 0);
        if (e != hipSuccess) return e;
    }
    if (A.ncharges > 0)
        hipLaunchKernelGGL(k_sum, dim3((unsigned)((A.ncharges + 255) / 256)), dim3(256), 0, st, A.ncharges, A.nslots, A.parts, A.phi);
    LPB_MARK(10);
#undef LPB_MARK
    return hipGetLastError();
}

template hipError_t eval_run<double>(const EvalArgs<double>&, const EvalSched&, int, hipStream_t, hipEvent_t*,
                                     const EvalFork*);
template hipError_t eval_run<float>(const EvalArgs<float>&, const EvalSched&, int, hipStream_t, hipEvent_t*,
                                    const EvalFork*);

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
