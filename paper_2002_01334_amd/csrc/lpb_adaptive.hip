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

// M2P: one 64-lane block per target leaf with W-list entries, one lane per
// target (64 at a time); the entry's expansion is staged in LDS in FP64.
template <typename T>
__global__ void __launch_bounds__(64) k_m2p(EvalArgs<T> A)
{
    extern __shared__ double sm_m2p[];
    double* M = sm_m2p;                 // K
    double* sc = sm_m2p + A.K;          // p + 1: 4 pi i_n(lam h_s)
    const int p = A.p, K = A.K;
    const int leaf = A.w_leaves[blockIdx.x];
    const int t0 = A.tl_start[leaf], t1 = A.tl_start[leaf + 1];
    const int e0 = A.w_ptr[leaf], e1 = A.w_ptr[leaf + 1];
    const double tcx = A.tl_ctr[3 * leaf], tcy = A.tl_ctr[3 * leaf + 1], tcz = A.tl_ctr[3 * leaf + 2];
    const int lane = threadIdx.x;
    for (int base = t0; base < t1; base += 64) {
        const int j = base + lane;
        const bool act = j < t1;
        double acc = 0.0;
        for (int e = e0; e < e1; ++e) {
            const FmmDev& F = A.fmm[A.w_fmm[e]];
            const int me = A.w_me[e];
            __syncthreads();
            for (int k = lane; k < K; k += 64) M[k] = (double)A.me[(size_t)me * A.KP + k];
            if (lane == 0 && F.kind == 0) {
                double buf[LPB_MAX_P + 2];
                bessel_i_all(p, F.lam_s * (2.0 * F.R / (double)(1 << A.w_lv[e])), buf);
                for (int n = 0; n <= p; ++n) sc[n] = 4.0 * LPB_PI * buf[n];
            }
            __syncthreads();
            if (!act) continue;
            if (F.kind == 1) {
                const double* v = A.pt_vec + A.w_vec[e] + (int64_t)(j - t0) * K;
                double s = 0.0;
                for (int k = 0; k < K; ++k) s += v[k] * M[k];
                acc += s;
                continue;
            }
            // target offset from the source box centre
            const double ux = (double)A.t_ux[j] + (A.t_lx ? (double)A.t_lx[j] : 0.0);
            const double uy = (double)A.t_uy[j] + (A.t_ly ? (double)A.t_ly[j] : 0.0);
            const double uz = (double)A.t_uz[j] + (A.t_lz ? (double)A.t_lz[j] : 0.0);
            const double vx = ux + (tcx - A.w_ctr[3 * e]), vy = uy + (tcy - A.w_ctr[3 * e + 1]),
                         vz = uz + (tcz - A.w_ctr[3 * e + 2]);
            const double r = sqrt(vx * vx + vy * vy + vz * vz);
            double kn[LPB_MAX_P + 1];
            bessel_k_all(p, F.lam_s * r, kn);
            const double x = vx / r, y = vy / r, z = vz / r;
            // Y_n^m(v^) = R_n^m(x, y, z) on the unit sphere, by the solid-harmonic recurrence
            double s = 0.0, wr = 1.0, wi = 0.0, amm = 0.28209479177387814;
            for (int m = 0; m <= p; ++m) {
                if (m > 0) {
                    const double nr = wr * x - wi * y;
                    wi = wr * y + wi * x;
                    wr = nr;
                    amm *= sqrt((2.0 * m + 1.0) / (2.0 * m));
                }
                double pr = amm * wr, pi = amm * wi, qr = 0.0, qi = 0.0;
                const double f = m ? 2.0 : 1.0;
                for (int n = m; n <= p; ++n) {
                    double cr, ci;
                    if (n == m) {
                        cr = pr;
                        ci = pi;
                    } else if (n == m + 1) {
                        qr = sqrt(2.0 * m + 3.0) * z * pr;
                        qi = sqrt(2.0 * m + 3.0) * z * pi;
                        cr = qr;
                        ci = qi;
                    } else {
                        const double nn = (double)n * n, mm = (double)m * m;
                        const double a = sqrt((4.0 * nn - 1.0) / (nn - mm));
                        const double b = sqrt(((n - 1.0) * (n - 1.0) - mm) * (2.0 * n + 1.0) / ((nn - mm) * (2.0 * n - 3.0)));
                        cr = a * z * qr - b * pr;
                        ci = a * z * qi - b * pi;
                        pr = qr;
                        pi = qi;
                        qr = cr;
                        qi = ci;
                    }
                    const double re = M[ire(n, m)], im = m ? M[iim(n, m)] : 0.0;
                    s += f * sc[n] * kn[n] * (re * cr - im * ci);
                }
            }
            acc += F.far_factor * s;
        }
        if (act) A.parts[A.t_out[j]] += acc;
    }
}

// P2L: one 64-lane block per target box with X-list entries.  Free space:
// per chunk of CH sources each lane forms its source's scaled row in LDS,
// then lanes sum rows; reaction: each lane takes coefficients k and sums
// q times the point operators over the leaf's sources.
template <typename T>
__global__ void __launch_bounds__(64) k_p2l(EvalArgs<T> A)
{
    constexpr int CH = 16;
    extern __shared__ double sm_p2l[];
    const int p = A.p, K = A.K;
    double* rows = sm_p2l;                        // [K][CH + 1]
    double* sc = sm_p2l + (size_t)K * (CH + 1);   // p + 1: 4 pi i_n(lam h_t)
    const int b = blockIdx.x;
    const int le = A.x_box_le[b];
    const double cx = A.x_box_ctr[3 * b], cy = A.x_box_ctr[3 * b + 1], cz = A.x_box_ctr[3 * b + 2];
    const int lane = threadIdx.x;
    double acc[(LPB_KMAX + 63) / 64];
#pragma unroll
    for (int kk = 0; kk < (LPB_KMAX + 63) / 64; ++kk) acc[kk] = 0.0;
    for (int e = A.x_box_ptr[b]; e < A.x_box_ptr[b + 1]; ++e) {
        const FmmDev& F = A.fmm[A.x_fmm[e]];
        const int sl = A.x_sl[e];
        const int s0 = A.sl_start[sl], s1 = A.sl_start[sl + 1];
        if (F.kind == 1) {
            const double* v = A.pt_vec + A.x_vec[e];
            for (int j = s0; j < s1; ++j) {
                const double q = (double)A.qs[j];
#pragma unroll
                for (int kk = 0; kk < (LPB_KMAX + 63) / 64; ++kk) {
                    const int k = lane + 64 * kk;
                    if (k < K) acc[kk] += q * v[(int64_t)(j - s0) * K + k];
                }
            }
            continue;
        }
        __syncthreads();
        if (lane == 0) {
            double buf[LPB_MAX_P + 2];
            bessel_i_all(p, F.lam_t * (2.0 * F.R / (double)(1 << A.x_box_lv[b])), buf);
            for (int n = 0; n <= p; ++n) sc[n] = 4.0 * LPB_PI * buf[n];
        }
        const double ox = A.sl_ctr[3 * sl] - cx, oy = A.sl_ctr[3 * sl + 1] - cy, oz = A.sl_ctr[3 * sl + 2] - cz;
        for (int base = s0; base < s1; base += CH) {
            __syncthreads();
            const int j = base + lane;
            if (lane < CH && j < s1) {
                const double vx = (double)A.s_ux[j] + (A.s_lx ? (double)A.s_lx[j] : 0.0) + ox;
                const double vy = (double)A.s_uy[j] + (A.s_ly ? (double)A.s_ly[j] : 0.0) + oy;
                const double vz = (double)A.s_uz[j] + (A.s_lz ? (double)A.s_lz[j] : 0.0) + oz;
                const double r = sqrt(vx * vx + vy * vy + vz * vz);
                double kn[LPB_MAX_P + 1];
                bessel_k_all(p, F.lam_t * r, kn);
                const double q = (double)A.qs[j];
                const double x = vx / r, y = vy / r, z = vz / r;
                double wr = 1.0, wi = 0.0, amm = 0.28209479177387814;
                for (int m = 0; m <= p; ++m) {
                    if (m > 0) {
                        const double nr = wr * x - wi * y;
                        wi = wr * y + wi * x;
                        wr = nr;
                        amm *= sqrt((2.0 * m + 1.0) / (2.0 * m));
                    }
                    double pr = amm * wr, pi = amm * wi, qr = 0.0, qi = 0.0;
                    for (int n = m; n <= p; ++n) {
                        double cr, ci;
                        if (n == m) {
                            cr = pr;
                            ci = pi;
                        } else if (n == m + 1) {
                            qr = sqrt(2.0 * m + 3.0) * z * pr;
                            qi = sqrt(2.0 * m + 3.0) * z * pi;
                            cr = qr;
                            ci = qi;
                        } else {
                            const double nn = (double)n * n, mm = (double)m * m;
                            const double a = sqrt((4.0 * nn - 1.0) / (nn - mm));
                            const double bb = sqrt(((n - 1.0) * (n - 1.0) - mm) * (2.0 * n + 1.0) / ((nn - mm) * (2.0 * n - 3.0)));
                            cr = a * z * qr - bb * pr;
                            ci = a * z * qi - bb * pi;
                            pr = qr;
                            pi = qi;
                            qr = cr;
                            qi = ci;
                        }
                        const double g = q * sc[n] * kn[n];
                        rows[(size_t)ire(n, m) * (CH + 1) + lane] = g * cr;
                        if (m > 0) rows[(size_t)iim(n, m) * (CH + 1) + lane] = -g * ci;
                    }
                }
            }
            __syncthreads();
            const int cnt = min(CH, s1 - base);
#pragma unroll
            for (int kk = 0; kk < (LPB_KMAX + 63) / 64; ++kk) {
                const int k = lane + 64 * kk;
                if (k < K) {
                    double s = 0.0;
                    for (int jj = 0; jj < cnt; ++jj) s += rows[(size_t)k * (CH + 1) + jj];
                    acc[kk] += s;
                }
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
    if (A.n_w_leaves > 0)
        hipLaunchKernelGGL(k_m2p<T>, dim3(A.n_w_leaves), dim3(64), sizeof(double) * (A.K + A.p + 1), st, A);
}

template <typename T>
void launch_p2l(const EvalArgs<T>& A, hipStream_t st)
{
    if (A.n_x_boxes > 0)
        hipLaunchKernelGGL(k_p2l<T>, dim3(A.n_x_boxes), dim3(64), sizeof(double) * ((size_t)A.K * 17 + A.p + 1), st, A);
}

template void launch_m2p<float>(const EvalArgs<float>&, hipStream_t);
template void launch_m2p<double>(const EvalArgs<double>&, hipStream_t);
template void launch_p2l<float>(const EvalArgs<float>&, hipStream_t);
template void launch_p2l<double>(const EvalArgs<double>&, hipStream_t);

}  // namespace lpb
