// lpb_adaptive.hip -- the W- and X-lists of adaptive trees (Sec. 3.5, closing
// remarks on adaptive trees): a source box's multipole expansion evaluated at
// the targets of a coarser leaf directly (M2P), and a target box's local
// expansion formed from the sources of a coarser leaf directly (P2L).
//
// Free space (eqs. freespace3dmulexp, melecoeffree), in the scaled real form
// of the expansions (Mh = M / (4 pi i_n(lam h)), Lh = i_n(lam h) L):
//   M2P:  Phi(r) += far * sum_n 4 pi i_n(lam h_s) k_n(lam |v|) [Mh_n0 Y_n^0 + 2 sum_{m>0} Re(Mh_nm Y_n^m)](v^),
//         v = r - c_s;
//   P2L:  Lh_nm += q i_n(lam h_t) 4 pi k_n(lam |v|) conj(Y_n^m(v^)),  v = r' - c_t.
// Reaction components: the precomputed point operators of the operator
// generator (one K-vector per point and box): M2P dots it with Mh, P2L adds
// q times it to Lh.  All arithmetic in FP64; the expansions are read and
// written in the evaluation type.
#include <hip/hip_runtime.h>

#include "lpb_eval_dev.h"

namespace lpb {

#define LPB_KMAX ((LPB_MAX_P + 1) * (LPB_MAX_P + 1))

// Calls f(n, m, re, im) with Y_n^m(v) = re + i im for every n <= p, 0 <= m <= n,
// at a unit vector v = (x, y, z), by the solid-harmonic recurrence
// (coefficients amm[m], al / be at the packed index, FP64, in LDS)
template <int P, typename Fn>
__device__ __attribute__((always_inline)) inline void unit_harmonics(int p_rt, const double* amm, const double* al,
                                                                     const double* be, double x, double y, double z,
                                                                     Fn&& f)
{
    const int p = P > 0 ? P : p_rt;
    double wr = 1.0, wi = 0.0;
#pragma unroll
    for (int m = 0; m <= p; ++m) {
        if (m > 0) {
            const double nr = wr * x - wi * y;
            wi = wr * y + wi * x;
            wr = nr;
        }
        double pr = amm[m] * wr, pi = amm[m] * wi;
        f(m, m, pr, pi);
        if (m + 1 > p) continue;
        double qr = al[ipk(m + 1, m)] * z * pr, qi = al[ipk(m + 1, m)] * z * pi;
        f(m + 1, m, qr, qi);
#pragma unroll
        for (int n = m + 2; n <= p; ++n) {
            const double a = al[ipk(n, m)], b = be[ipk(n, m)];
            const double sr = a * z * qr - b * pr, si = a * z * qi - b * pi;
            f(n, m, sr, si);
            pr = qr;
            pi = qi;
            qr = sr;
            qi = si;
        }
    }
}

// k_n(x), n = 0..p (forward recurrence as bessel_k_all), unrolled for a
// compile-time P so that the values stay in registers
template <int P>
__device__ __attribute__((always_inline)) inline void bessel_k_fixed(int p_rt, double x, double* out)
{
    const int p = P > 0 ? P : p_rt;
    const double e = 0.5 * LPB_PI * exp(-x) / x, xi = 1.0 / x;
    out[0] = e;
    if (p >= 1) out[1] = e * (1.0 + xi);
#pragma unroll
    for (int n = 1; n < p; ++n) out[n + 1] = out[n - 1] + (2.0 * n + 1.0) * xi * out[n];
}

// M2P: one 256-thread block per target leaf with W-list entries, one lane
// per target (64 at a time); wave w takes the entries w, w + 4, ... in
// order, every lane reading the entry's expansion itself, and wave 0 adds
// the other waves' sums in wave order.
template <typename T, int P>
__global__ void __launch_bounds__(256) k_m2p(EvalArgs<T> A)
{
    constexpr int G = 4;
    extern __shared__ double sm_m2p[];
    const int p = P > 0 ? P : A.p, K = (p + 1) * (p + 1), Kp = (p + 1) * (p + 2) / 2;
    double* tab = sm_m2p;                        // amm[p+1], alpha[Kp], beta[Kp]
    double* part = sm_m2p + p + 1 + 2 * Kp;      // [G - 1][64]: the other waves' sums
    const int leaf = A.w_leaves[blockIdx.x];
    const int t0 = A.tl_start[leaf], t1 = A.tl_start[leaf + 1];
    const int e0 = A.w_ptr[leaf], e1 = A.w_ptr[leaf + 1];
    const double tcx = A.tl_ctr[3 * leaf], tcy = A.tl_ctr[3 * leaf + 1], tcz = A.tl_ctr[3 * leaf + 2];
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    for (int k = threadIdx.x; k < p + 1 + 2 * Kp; k += 64 * G) tab[k] = A.sh64[k];
    __syncthreads();
    const double *amm = tab, *al = tab + p + 1, *be = tab + p + 1 + Kp;
    for (int base = t0; base < t1; base += 64) {
        const int j = base + lane;
        const bool act = j < t1;
        double acc = 0.0;
        if (act) {
            const double ux = (double)A.t_ux[j] + (A.t_lx ? (double)A.t_lx[j] : 0.0);
            const double uy = (double)A.t_uy[j] + (A.t_ly ? (double)A.t_ly[j] : 0.0);
            const double uz = (double)A.t_uz[j] + (A.t_lz ? (double)A.t_lz[j] : 0.0);
            for (int e = e0 + w; e < e1; e += G) {
                const int fid = A.w_fmm[e];
                const FmmDev& F = A.fmm[fid];
                // the entry's expansion: the same addresses in every lane
                // (read through the caches, no staging or barriers)
                const T* __restrict__ M = A.me + (size_t)A.w_me[e] * A.KP;
                if (F.kind == 1) {
                    const double* v = A.pt_vec + A.w_vec[e] + (int64_t)(j - t0) * K;
                    double s = 0.0;
                    for (int k = 0; k < K; ++k) s += v[k] * (double)M[k];
                    acc += s;
                    continue;
                }
                // free space: the target's offset from the source box centre
                const double vx = ux + (tcx - A.w_ctr[3 * e]), vy = uy + (tcy - A.w_ctr[3 * e + 1]),
                             vz = uz + (tcz - A.w_ctr[3 * e + 2]);
                const double r = sqrt(vx * vx + vy * vy + vz * vz);
                double kn[(P > 0 ? P : LPB_MAX_P) + 1];
                bessel_k_fixed<P>(p, F.lam_s * r, kn);
                const double* sc = A.fin_s + ((size_t)fid * (kMaxDepth + 1) + A.w_lv[e]) * (LPB_MAX_P + 1);
                double s = 0.0;
                unit_harmonics<P>(p, amm, al, be, vx / r, vy / r, vz / r, [&](int n, int m, double cr, double ci) {
                    const double re = (double)M[ire(n, m)], im = m ? (double)M[iim(n, m)] : 0.0;
                    s += (m ? 2.0 : 1.0) * sc[n] * kn[n] * (re * cr - im * ci);
                });
                acc += F.far_factor * s;
            }
        }
        if (w > 0) part[(w - 1) * 64 + lane] = acc;
        __syncthreads();
        if (w == 0 && act) {
#pragma unroll
            for (int g = 0; g < G - 1; ++g) acc += part[g * 64 + lane];
            A.parts[A.t_out[j]] += acc;
        }
        __syncthreads();
    }
}

// P2L: one 64-lane block per target box with X-list entries.  Free space:
// the sources of all the box's free-space entries in one sequence, per chunk
// of CH of them each lane forms its source's scaled row in LDS (FP64
// arithmetic, the row stored in the precision of the expansions), then lanes
// sum rows in FP64; reaction: each lane takes coefficients k and sums q
// times the point operators over the leaf's sources.
template <typename T, int P>
__global__ void __launch_bounds__(64) k_p2l(EvalArgs<T> A, int CH)
{
    extern __shared__ double sm_p2l[];
    const int p = P > 0 ? P : A.p, K = (p + 1) * (p + 1), Kp = (p + 1) * (p + 2) / 2;
    double* tab = sm_p2l;                                        // amm, alpha, beta
    T* rows = reinterpret_cast<T*>(sm_p2l + p + 1 + 2 * Kp);     // [K][CH + 1], in the precision of the expansions
    const int b = blockIdx.x;
    const int le = A.x_box_le[b];
    const double cx = A.x_box_ctr[3 * b], cy = A.x_box_ctr[3 * b + 1], cz = A.x_box_ctr[3 * b + 2];
    const int lane = threadIdx.x;
    for (int k = lane; k < p + 1 + 2 * Kp; k += 64) tab[k] = A.sh64[k];
    const double *amm = tab, *al = tab + p + 1, *be = tab + p + 1 + Kp;
    double acc[(LPB_KMAX + 63) / 64];
#pragma unroll
    for (int kk = 0; kk < (LPB_KMAX + 63) / 64; ++kk) acc[kk] = 0.0;
    const int e0 = A.x_box_ptr[b], e1 = A.x_box_ptr[b + 1];
    // free-space entries: their sources as one sequence (entry order), CH at
    // a time, so that the lanes stay busy across entries with few sources
    int tot = 0;
    for (int e = e0; e < e1; ++e)
        if (A.fmm[A.x_fmm[e]].kind != 1) tot += A.sl_start[A.x_sl[e] + 1] - A.sl_start[A.x_sl[e]];
    for (int base = 0; base < tot; base += CH) {
        __syncthreads();
        if (lane < CH && base + lane < tot) {
            // the entry and source of position base + lane
            // (always found: base + lane < tot)
            int e = e0, off = base + lane, sl = 0, fid = 0;
            for (; e < e1; ++e) {
                fid = A.x_fmm[e];
                if (A.fmm[fid].kind == 1) continue;
                sl = A.x_sl[e];
                const int n = A.sl_start[sl + 1] - A.sl_start[sl];
                if (off < n) break;
                off -= n;
            }
            const FmmDev& F = A.fmm[fid];
            const int j = A.sl_start[sl] + off;
            const double* sc = A.fin_t + ((size_t)fid * (kMaxDepth + 1) + A.x_box_lv[b]) * (LPB_MAX_P + 1);
            const double vx = (double)A.s_ux[j] + (A.s_lx ? (double)A.s_lx[j] : 0.0) + (A.sl_ctr[3 * sl] - cx);
            const double vy = (double)A.s_uy[j] + (A.s_ly ? (double)A.s_ly[j] : 0.0) + (A.sl_ctr[3 * sl + 1] - cy);
            const double vz = (double)A.s_uz[j] + (A.s_lz ? (double)A.s_lz[j] : 0.0) + (A.sl_ctr[3 * sl + 2] - cz);
            const double r = sqrt(vx * vx + vy * vy + vz * vz);
            double kn[(P > 0 ? P : LPB_MAX_P) + 1];
            bessel_k_fixed<P>(p, F.lam_t * r, kn);
            const double q = (double)A.qs[j];
            T* row = rows + lane;
            unit_harmonics<P>(p, amm, al, be, vx / r, vy / r, vz / r, [&](int n, int m, double cr, double ci) {
                // Lh_nm += q i_n(lam h) 4 pi k_n conj(Y_n^m)
                const double g = q * sc[n] * kn[n];
                row[(size_t)ire(n, m) * (CH + 1)] = (T)(g * cr);
                if (m > 0) row[(size_t)iim(n, m) * (CH + 1)] = (T)(-g * ci);
            });
        }
        __syncthreads();
        const int cnt = min(CH, tot - base);
#pragma unroll
        for (int kk = 0; kk < (LPB_KMAX + 63) / 64; ++kk) {
            const int k = lane + 64 * kk;
            if (k < K) {
                double s = 0.0;
                for (int jj = 0; jj < cnt; ++jj) s += (double)rows[(size_t)k * (CH + 1) + jj];
                acc[kk] += s;
            }
        }
    }
    // reaction entries: each lane takes coefficients k over the leaf's sources
    for (int e = e0; e < e1; ++e) {
        const FmmDev& F = A.fmm[A.x_fmm[e]];
        if (F.kind != 1) continue;
        const int sl = A.x_sl[e];
        const int s0 = A.sl_start[sl], s1 = A.sl_start[sl + 1];
        const double* v = A.pt_vec + A.x_vec[e];
        for (int j = s0; j < s1; ++j) {
            const double q = (double)A.qs[j];
#pragma unroll
            for (int kk = 0; kk < (LPB_KMAX + 63) / 64; ++kk) {
                const int k = lane + 64 * kk;
                if (k < K) acc[kk] += q * v[(int64_t)(j - s0) * K + k];
            }
        }
    }
#pragma unroll
    for (int kk = 0; kk < (LPB_KMAX + 63) / 64; ++kk) {
        const int k = lane + 64 * kk;
        if (k < K) A.le[(size_t)le * A.KP + k] += (T)acc[kk];
    }
}

template <typename T>
void launch_m2p(const EvalArgs<T>& A, hipStream_t st)
{
    const int Kp = (A.p + 1) * (A.p + 2) / 2;
    if (A.n_w_leaves <= 0) return;
    const size_t sm = sizeof(double) * (A.p + 1 + 2 * Kp + 3 * 64);
#define LPB_M2P(PP) \
    case PP: hipLaunchKernelGGL((k_m2p<T, PP>), dim3(A.n_w_leaves), dim3(256), sm, st, A); break;
    switch (A.p) {
        LPB_M2P(2) LPB_M2P(3) LPB_M2P(4) LPB_M2P(5) LPB_M2P(6) LPB_M2P(7) LPB_M2P(8) LPB_M2P(9) LPB_M2P(10)
        LPB_M2P(11) LPB_M2P(12) LPB_M2P(13) LPB_M2P(14) LPB_M2P(15)
    default: hipLaunchKernelGGL((k_m2p<T, 0>), dim3(A.n_w_leaves), dim3(256), sm, st, A); break;
    }
#undef LPB_M2P
}

template <typename T>
void launch_p2l(const EvalArgs<T>& A, hipStream_t st)
{
    // sources per row chunk: as many lanes as the LDS rows allow (<= 48 KiB)
    const int Kp = (A.p + 1) * (A.p + 2) / 2;
    if (A.n_x_boxes <= 0) return;
    int ch = 64;
    while (ch > 8 && sizeof(T) * (size_t)A.K * (ch + 1) > 48u * 1024u) ch >>= 1;
    const size_t sm = sizeof(T) * (size_t)A.K * (ch + 1) + sizeof(double) * (A.p + 1 + 2 * Kp);
#define LPB_P2L(PP) \
    case PP: hipLaunchKernelGGL((k_p2l<T, PP>), dim3(A.n_x_boxes), dim3(64), sm, st, A, ch); break;
    switch (A.p) {
        LPB_P2L(2) LPB_P2L(3) LPB_P2L(4) LPB_P2L(5) LPB_P2L(6) LPB_P2L(7) LPB_P2L(8) LPB_P2L(9) LPB_P2L(10)
        LPB_P2L(11) LPB_P2L(12) LPB_P2L(13) LPB_P2L(14) LPB_P2L(15)
    default: hipLaunchKernelGGL((k_p2l<T, 0>), dim3(A.n_x_boxes), dim3(64), sm, st, A, ch); break;
    }
#undef LPB_P2L
}

template void launch_m2p<float>(const EvalArgs<float>&, hipStream_t);
template void launch_m2p<double>(const EvalArgs<double>&, hipStream_t);
template void launch_p2l<float>(const EvalArgs<float>&, hipStream_t);
template void launch_p2l<double>(const EvalArgs<double>&, hipStream_t);

}  // namespace lpb
