// lpb_eval.hip -- evaluation kernels of Algorithm 2 (every FMM of every
// system per launch): gather charges, P2M, M2M, M2L, L2L, L2P, near field
// (free-space and reaction), and the component sum.  Templated on the
// arithmetic type T (double for LPB_FP64, float for LPB_MIXED); Bessel
// ratios are always formed in double.
#include <hip/hip_runtime.h>

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

// ---------------------------------------------------------------------------
// P2M (eqs. melecoeffree, melayerupgoingimage), scaled:
//   Mh_nm = sum_j q_j g_n(r_j) conj(R_n^m(u_j / h)),  u_j = source - box centre.
// One 64-lane block per source leaf; lanes own points, the per-point
// coefficient rows are staged in LDS and summed per coefficient.
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
    T* rre = coef + (size_t)K * CS;                            // [Kp][CH]
    T* rim = rre + (size_t)((p + 1) * (p + 2) / 2) * CH;
    __shared__ double inv_ith[LPB_MAX_P + 1];
    const int lane = threadIdx.x;
    if (lane == 0) {
        double t[LPB_MAX_P + 2];
        itilde_all(p, F.lam_s * F.lam_s * h * h, t);
        for (int n = 0; n <= p; ++n) inv_ith[n] = 1.0 / t[n];
    }
    __syncthreads();
    const int s0 = A.sl_start[leaf], s1 = A.sl_start[leaf + 1];
    T acc[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) acc[k] = T(0);
    const T hinv = (T)(1.0 / h);
    for (int base = s0; base < s1; base += CH) {
        int j = base + lane;
        if (lane < CH && j < s1) {
            T ux = A.s_ux[j], uy = A.s_uy[j], uz = A.s_uz[j], q = A.qs[j];
            double r2 = (double)ux * ux + (double)uy * uy + (double)uz * uz;
            double g[LPB_MAX_P + 2];
            bessel_ratio(p, F.lam_s, r2, inv_ith, g);
            // solid harmonics R_n^m(u/h) into per-lane LDS columns
            solid_harmonics_lds<T>(p, ux * hinv, uy * hinv, uz * hinv, rre + lane, rim + lane, CH);
            for (int n = 0; n <= p; ++n) {
                T gq = (T)g[n] * q;
                for (int m = 0; m <= n; ++m) {
                    coef[(size_t)ire(n, m) * CS + lane] = gq * rre[(size_t)ipk(n, m) * CH + lane];
                    if (m > 0) coef[(size_t)iim(n, m) * CS + lane] = -gq * rim[(size_t)ipk(n, m) * CH + lane];
                }
            }
        }
        __syncthreads();
        int cnt = min(CH, s1 - base);
#pragma unroll
        for (int kk = 0; kk < 8; ++kk) {
            int k = lane + 64 * kk;
            if (k < K) {
                T s = T(0);
                for (int jj = 0; jj < cnt; ++jj) s += coef[(size_t)k * CS + jj];
                acc[kk] += s;
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int kk = 0; kk < 8; ++kk) {
        int k = lane + 64 * kk;
        if (k < K) A.me[(size_t)me * K + k] = acc[kk];
    }
}

// ---------------------------------------------------------------------------
// Dense real-form operator application, one block per output box:
//   out[row] (+)= sum_pairs sum_c Op[c*K + row] * in[c]
// used for M2M (CSR by parent), M2L (CSR by target) and L2L (one pair).
template <typename T>
__device__ inline void apply_pairs(int K, const T* __restrict__ pool, const T* __restrict__ invec, const int* __restrict__ src,
                                   const int* __restrict__ op, int b, int e, T* xs, T& acc)
{
    const int row = threadIdx.x;
    for (int k = b; k < e; ++k) {
        const T* v = invec + (size_t)src[k] * K;
        for (int c = threadIdx.x; c < K; c += blockDim.x) xs[c] = v[c];
        __syncthreads();
        if (row < K) {
            const T* O = pool + (size_t)op[k] * K * K;
            T s0 = T(0), s1 = T(0);
            int c = 0;
            for (; c + 1 < K; c += 2) {
                s0 += O[(size_t)c * K + row] * xs[c];
                s1 += O[(size_t)(c + 1) * K + row] * xs[c + 1];
            }
            if (c < K) s0 += O[(size_t)c * K + row] * xs[c];
            acc += s0 + s1;
        }
        __syncthreads();
    }
}

template <typename T>
__global__ void k_m2m(EvalArgs<T> A, int pbeg)
{
    extern __shared__ unsigned char smem_raw[];
    T* xs = reinterpret_cast<T*>(smem_raw);
    const int pi = pbeg + blockIdx.x;
    T acc = T(0);
    apply_pairs<T>(A.K, A.pool, A.me, A.m2m_child, A.m2m_op, A.m2m_ptr[pi], A.m2m_ptr[pi + 1], xs, acc);
    if ((int)threadIdx.x < A.K) A.me[(size_t)A.m2m_parent[pi] * A.K + threadIdx.x] = acc;
}

template <typename T>
__global__ void k_m2l(EvalArgs<T> A)
{
    extern __shared__ unsigned char smem_raw[];
    T* xs = reinterpret_cast<T*>(smem_raw);
    const int le = A.m2l_boxes[blockIdx.x];
    T acc = T(0);
    apply_pairs<T>(A.K, A.pool, A.me, A.m2l_src, A.m2l_op, A.m2l_ptr[le], A.m2l_ptr[le + 1], xs, acc);
    if ((int)threadIdx.x < A.K) A.le[(size_t)le * A.K + threadIdx.x] = acc;
}

template <typename T>
__global__ void k_l2l(EvalArgs<T> A, int cbeg)
{
    extern __shared__ unsigned char smem_raw[];
    T* xs = reinterpret_cast<T*>(smem_raw);
    const int ci = cbeg + blockIdx.x;
    T acc = T(0);
    apply_pairs<T>(A.K, A.pool, A.le, A.l2l_parent + ci, A.l2l_op + ci, 0, 1, xs, acc);
    if ((int)threadIdx.x < A.K) A.le[(size_t)A.l2l_child[ci] * A.K + threadIdx.x] += acc;
}

// ---------------------------------------------------------------------------
// L2P (eqs. freespace3dlocexp, lelayerimage), scaled:
//   Phi = far_factor * sum_n g_n(r) [Lh_n0 R_n^0 + 2 sum_{m>0} Re(Lh_nm R_n^m)](u/h)
template <typename T>
__global__ void __launch_bounds__(64) k_l2p(EvalArgs<T> A, int CH)
{
    extern __shared__ unsigned char smem_raw[];
    const int p = A.p, K = A.K;
    const int leaf = A.l2p_leaves[blockIdx.x];
    const int le = A.tl_le[leaf];
    const FmmDev& F = A.fmm[A.tl_fmm[leaf]];
    const double h = A.tl_h[leaf];
    T* Ls = reinterpret_cast<T*>(smem_raw);                       // [K]
    T* rre = Ls + K;                                              // [Kp][CH]
    T* rim = rre + (size_t)((p + 1) * (p + 2) / 2) * CH;
    __shared__ double inv_ith[LPB_MAX_P + 1];
    const int lane = threadIdx.x;
    if (lane == 0) {
        double t[LPB_MAX_P + 2];
        itilde_all(p, F.lam_t * F.lam_t * h * h, t);
        for (int n = 0; n <= p; ++n) inv_ith[n] = 1.0 / t[n];
    }
    for (int k = lane; k < K; k += 64) Ls[k] = A.le[(size_t)le * K + k];
    __syncthreads();
    const int t0 = A.tl_start[leaf], t1 = A.tl_start[leaf + 1];
    const T hinv = (T)(1.0 / h);
    if (lane >= CH) return;
    for (int j = t0 + lane; j < t1; j += CH) {
        T ux = A.t_ux[j], uy = A.t_uy[j], uz = A.t_uz[j];
        double r2 = (double)ux * ux + (double)uy * uy + (double)uz * uz;
        double g[LPB_MAX_P + 2];
        bessel_ratio(p, F.lam_t, r2, inv_ith, g);
        solid_harmonics_lds<T>(p, ux * hinv, uy * hinv, uz * hinv, rre + lane, rim + lane, CH);
        T phi = T(0);
        for (int n = 0; n <= p; ++n) {
            T s = Ls[ire(n, 0)] * rre[(size_t)ipk(n, 0) * CH + lane];
            T s2 = T(0);
            for (int m = 1; m <= n; ++m)
                s2 += Ls[ire(n, m)] * rre[(size_t)ipk(n, m) * CH + lane] - Ls[iim(n, m)] * rim[(size_t)ipk(n, m) * CH + lane];
            phi += (T)g[n] * (s + T(2) * s2);
        }
        A.parts[A.t_out[j]] = (double)phi * F.far_factor;
    }
}

// ---------------------------------------------------------------------------
// Free-space near field (eq. freereactioncomponents, j != i):
//   Phi_i += sum_{j in U(i), j != i} q_j e^{-lam r}/(4 pi eps r)
// One 64-lane block per target leaf; lanes own targets, sources staged in LDS.
// FP32 sums use Kahan compensation.
template <typename T>
__global__ void __launch_bounds__(64) k_p2p_free(EvalArgs<T> A)
{
    __shared__ T sx[64], sy[64], sz[64], sq[64];
    __shared__ int sc[64];
    const int leaf = A.p2p_free_leaves[blockIdx.x];
    const FmmDev& F = A.fmm[A.tl_fmm[leaf]];
    const T lam = (T)F.lam_t;
    const int t0 = A.tl_start[leaf], t1 = A.tl_start[leaf + 1];
    const double tcx = A.tl_ctr[3 * leaf], tcy = A.tl_ctr[3 * leaf + 1], tcz = A.tl_ctr[3 * leaf + 2];
    for (int base = t0; base < t1; base += 64) {
        int j = base + threadIdx.x;
        bool act = j < t1;
        T x = act ? A.t_ux[j] : T(0), y = act ? A.t_uy[j] : T(0), z = act ? A.t_uz[j] : T(0);
        int ci = act ? A.t_cidx[j] : -1;
        T sum = T(0), comp = T(0);
        for (int k = A.p2p_ptr[leaf]; k < A.p2p_ptr[leaf + 1]; ++k) {
            int sl = A.p2p_src[k];
            // offset of the source leaf centre from the target leaf centre
            T ox = (T)(A.sl_ctr[3 * sl] - tcx), oy = (T)(A.sl_ctr[3 * sl + 1] - tcy), oz = (T)(A.sl_ctr[3 * sl + 2] - tcz);
            const int s0 = A.sl_start[sl], s1 = A.sl_start[sl + 1];
            for (int sb = s0; sb < s1; sb += 64) {
                int s = sb + threadIdx.x;
                __syncthreads();
                if (s < s1) {
                    sx[threadIdx.x] = A.s_ux[s] + ox;
                    sy[threadIdx.x] = A.s_uy[s] + oy;
                    sz[threadIdx.x] = A.s_uz[s] + oz;
                    sq[threadIdx.x] = A.qs[s];
                    sc[threadIdx.x] = A.s_cidx[s];
                }
                __syncthreads();
                int cnt = min(64, s1 - sb);
                if (act) {
                    for (int jj = 0; jj < cnt; ++jj) {
                        T dx = x - sx[jj], dy = y - sy[jj], dz = z - sz[jj];
                        T r2 = dx * dx + dy * dy + dz * dz;
                        T ri = (sc[jj] == ci) ? T(0) : T(1) / sqrt(r2);
                        T v = sq[jj] * exp(-lam * (r2 * ri)) * ri;
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
        }
        if (act) A.parts[A.t_out[j]] += (double)sum / (4.0 * LPB_PI * F.eps_t);
    }
}

// ---------------------------------------------------------------------------
// Reaction near field (Algorithm 1, last step): every pair is the integral
//   u~ = (1/4pi) int_0^inf lrho J_0(lrho rho) e^{-l_z zt + l'_z zs} sigma(lrho) / l_z dlrho
// (canonical frame: zt > 0 target height, zs < 0 image depth), by composite
// 20-point Gauss-Legendre on panels chosen as for the M2L initial values.
// FP64 always.  One thread per target.
template <typename T>
__global__ void k_p2p_react(EvalArgs<T> A)
{
    int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= A.n_react_targets) return;
    const int leaf = A.react_tgt_leaf[idx];
    const int j = A.react_tgt_slot[idx];
    const FmmDev& F = A.fmm[A.tl_fmm[leaf]];
    const Medium& Md = A.media[F.medium];
    double lmin = Md.lam[0], dmax = 0.0;
    for (int k = 1; k <= Md.L; ++k) lmin = fmin(lmin, Md.lam[k]);
    for (int k = 1; k < Md.L; ++k) dmax = fmax(dmax, Md.d[k - 1] - Md.d[k]);
    double w0 = lmin;
    if (dmax > 0.0 && LPB_PI / (2.0 * dmax) < w0) w0 = LPB_PI / (2.0 * dmax);
    const double tx = A.tl_ctr[3 * leaf] + (double)A.t_ux[j];
    const double ty = A.tl_ctr[3 * leaf + 1] + (double)A.t_uy[j];
    const double tz = A.tl_ctr[3 * leaf + 2] + (double)A.t_uz[j];
    const double lt = F.lam_t, ls = F.lam_s;
    const double lt_tol = log(A.quad_tol);
    double total = 0.0;
    for (int k = A.p2p_ptr[leaf]; k < A.p2p_ptr[leaf + 1]; ++k) {
        int sl = A.p2p_src[k];
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
    const int Kp = (p + 1) * (p + 2) / 2;
    const int bsz = ((K + 63) / 64) * 64;
    LPB_MARK(0);
    if (A.n_src > 0) hipLaunchKernelGGL(k_gather_q<T>, dim3((A.n_src + 255) / 256), dim3(256), 0, st, A.n_src, A.s_cidx, A.q, A.qs);
    hipLaunchKernelGGL(k_zero<double>, dim3(1024), dim3(256), 0, st, (size_t)A.nslots * A.ncharges, A.parts);
    if (A.n_le > 0) hipLaunchKernelGGL(k_zero<T>, dim3(1024), dim3(256), 0, st, (size_t)A.n_le * K, A.le);
    const bool far = stages & 1, near = stages & 2;
    LPB_MARK(1);
    // upward pass
    // point chunks sized so that a block's LDS stays under 40 KB (several blocks per CU)
    auto pick_ch = [&](size_t per_ch, size_t fixed) {
        int ch = 64;
        while (ch > 8 && fixed + per_ch * ch > 40u * 1024u) ch >>= 1;
        return ch;
    };
    if (far && S.n_p2m > 0) {
        int ch = pick_ch(sizeof(T) * ((size_t)K + 2 * Kp), sizeof(T) * (size_t)K);
        size_t sm = sizeof(T) * ((size_t)K * (ch + 1) + 2 * (size_t)Kp * ch);
        hipLaunchKernelGGL(k_p2m<T>, dim3(S.n_p2m), dim3(64), sm, st, A, ch);
    }
    LPB_MARK(2);
    for (int l = kMaxDepth; l >= 0; --l) {
        int b = S.m2m_level_ptr[l], e = S.m2m_level_ptr[l + 1];
        if (far && e > b) hipLaunchKernelGGL(k_m2m<T>, dim3(e - b), dim3(bsz), sizeof(T) * K, st, A, b);
    }
    // V-list translations (all levels), then the downward pass
    LPB_MARK(3);
    if (far && S.n_m2l_boxes > 0) hipLaunchKernelGGL(k_m2l<T>, dim3(S.n_m2l_boxes), dim3(bsz), sizeof(T) * K, st, A);
    LPB_MARK(4);
    for (int l = 0; l <= kMaxDepth; ++l) {
        int b = S.l2l_level_ptr[l], e = S.l2l_level_ptr[l + 1];
        if (far && e > b) hipLaunchKernelGGL(k_l2l<T>, dim3(e - b), dim3(bsz), sizeof(T) * K, st, A, b);
    }
    LPB_MARK(5);
    if (far && S.n_l2p > 0) {
        int ch = pick_ch(2 * sizeof(T) * (size_t)Kp, sizeof(T) * (size_t)K);
        size_t sm = sizeof(T) * ((size_t)K + 2 * (size_t)Kp * ch);
        hipLaunchKernelGGL(k_l2p<T>, dim3(S.n_l2p), dim3(64), sm, st, A, ch);
    }
    // near field
    LPB_MARK(6);
    if (near && S.n_p2p_free > 0) hipLaunchKernelGGL(k_p2p_free<T>, dim3(S.n_p2p_free), dim3(64), 0, st, A);
    LPB_MARK(7);
    if (near && A.n_react_targets > 0)
        hipLaunchKernelGGL(k_p2p_react<T>, dim3((A.n_react_targets + 63) / 64), dim3(64), 0, st, A);
    LPB_MARK(8);
    if (A.ncharges > 0)
        hipLaunchKernelGGL(k_sum, dim3((unsigned)((A.ncharges + 255) / 256)), dim3(256), 0, st, A.ncharges, A.nslots, A.parts, A.phi);
    LPB_MARK(9);
#undef LPB_MARK
    return hipGetLastError();
}

template hipError_t eval_run<double>(const EvalArgs<double>&, const EvalSched&, int, hipStream_t, hipEvent_t*);
template hipError_t eval_run<float>(const EvalArgs<float>&, const EvalSched&, int, hipStream_t, hipEvent_t*);

}  // namespace lpb
