// lpb_opgen.hip -- FP64 generation of the translation operators on the GPU.
//
// Every operator is stored as a real K x K matrix (K = (p+1)^2), column-major,
// acting on the real-form coefficient vectors of lpb_math.h (Re/Im of the
// m >= 0 coefficients; the m < 0 ones follow from conjugate symmetry of real
// charges).  The complex operator A maps a vector with M_{n,-m} =
// (-1)^m conj(M_nm) to one with the same symmetry, so
//   L = A M  ->  Re L = Re(A+ + B) a - Im(A+ - B) b,  Im L = Im(A+ + B) a + Re(A+ - B) b
// with A+ = A_{nm,nu mu}, B = (-1)^mu A_{nm,nu,-mu}, M_{nu mu} = a + i b.
//
// Free space (Theorems 3.1-3.3, eqs. metole and metome), with
// G(n,m;nu,mu;q) = int Y_n^m conj(Y_nu^mu) conj(Y_q^{m-mu}) dOmega:
//   Sh_{n nu}^{m mu}(b) = 4 pi sum_q i_q(lam b) Y_q^{m-mu}(b^) G(n,m;nu,mu;q)
//   S_{n nu}^{m mu}(b)  = 4 pi sum_q (-1)^{n+q} k_q(lam b) Y_q^{m-mu}(b^) G(n,m;nu,mu;q)
//   M2M: A_{nm,nu mu} = conj(Sh_{n nu}^{m mu}(c_child - c_parent))
//   L2L: A_{nm,nu mu} = Sh_{nu n}^{mu m}(c_child - c_parent)
//   M2L: A_{nm,nu mu} = S_{nu n}^{mu m}(c_t - c_s)
// (sums over nu, mu; the printed prefactors of eqs. spmhat3d and
// singularseparation are replaced by these forms, which satisfy the addition
// theorems.)
//
// Reaction components (Sec. 3.5), in the canonical frame (interface at z = 0,
// targets above, images below) every component has the a = 1 form
//   T_{nm,nu mu} = (-1)^n e^{i(mu-m) phi} I_{nm,nu mu}(rho, zt, zs)      (eq. coefintable)
//   I = sum_s D_s Sc_{|m|+|mu|+2s+1, mu-m, ij}                            (eq. metoletableform)
// with D_s = i^{mu-m} C~^s (real for the rows m >= 0 kept here), the scaled
// integrals S^n Sc_{nm,ij} (eq. M2Ltable) from composite Gauss-Legendre
// quadrature for m = 0, 1 and the forward recurrence (eq. recurrence1) for
// m >= 2, and sigma^{ab} from the transmission conditions.
//
// Scaling: operators act on Mh = M / (4 pi i_n(lam h)) and Lh = L i_n(lam h)
// (h = box side of the level), so each operator is multiplied by the
// matching diagonal factors.
#include <hip/hip_runtime.h>

#include "lpb_opgen.h"

namespace lpb {

__constant__ double c_fact[171];
__constant__ double c_gl_x[20];
__constant__ double c_gl_w[20];

#define LPB_NGL 20
#define LPB_MAXN (2 * LPB_MAX_P + 4)
#define LPB_MAXPANEL 4096
#define LPB_YW (4 * LPB_MAX_P + 1)

__device__ inline double dsgn(int k) { return (k & 1) ? -1.0 : 1.0; }
__device__ inline int jk(int n, int m) { return n * n + n + m; }

// ---- coefficient table D_s(n,m,nu,mu) of one reaction FMM -----------------
// D_s = (-1)^{m+s} sqrt((N+M)! (N-M)!) sum_t b^t_{nm} b^{s-t}_{nu|mu|}
//       lam_t^{-m-2t} lam_s^{-|mu|-2(s-t)},  N = m+|mu|+2s+1, M = mu-m  (m >= 0),
// where b^t_{nm} are the coefficients of the Legendre-product expansion
// (P^_n^m(l_z/l) = (l/l_z)^i sum_t tau b^t (-i)^{m+2t}... l_rho^{m+2t} / l^{m+2t}),
// so that i^{mu-m} C~^s = D_s for the rows m >= 0.
__global__ void k_dtable(int p, int nrf, const int* __restrict__ rf_list, const FmmDev* __restrict__ fmms,
                         const double* __restrict__ btab, double* __restrict__ dtab)
{
    const int K = (p + 1) * (p + 1);
    const int Kp = (p + 1) * (p + 2) / 2;
    const int SM = p + 2;
    long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    long long total = (long long)nrf * Kp * K;
    if (idx >= total) return;
    int col = (int)(idx % K);
    int row = (int)((idx / K) % Kp);
    int r = (int)(idx / ((long long)K * Kp));
    const FmmDev& F = fmms[rf_list[r]];
    int n = 0;
    while ((n + 1) * (n + 2) / 2 <= row) ++n;
    int m = row - n * (n + 1) / 2;
    int nu = 0;
    while ((nu + 1) * (nu + 1) <= col) ++nu;
    int mu = col - nu * nu - nu;
    int amu = mu < 0 ? -mu : mu;
    int rn = (n + m) / 2, rnu = (nu + amu) / 2;
    const int BT = p + 1;   // t stride of btab
    double* out = dtab + ((size_t)r * Kp * K + (size_t)row * K + col) * SM;
    for (int s = 0; s < SM; ++s) out[s] = 0.0;
    int smax = (n - rn) + (nu - rnu);
    for (int s = 0; s <= smax; ++s) {
        int t0 = s - (nu - rnu);
        if (t0 < 0) t0 = 0;
        int t1 = s < (n - rn) ? s : (n - rn);
        double acc = 0.0;
        for (int t = t0; t <= t1; ++t) {
            double bt = btab[((size_t)(n * (n + 1) / 2 + m)) * BT + t];
            double bs = btab[((size_t)(nu * (nu + 1) / 2 + amu)) * BT + (s - t)];
            acc += bt * bs * pow(F.lam_t, -(double)(m + 2 * t)) * pow(F.lam_s, -(double)(amu + 2 * (s - t)));
        }
        int N = m + amu + 2 * s + 1, M = mu - m;
        out[s] = dsgn(m + s) * sqrt(c_fact[N + M] * c_fact[N - M]) * acc;
    }
}

// ---- quadrature of the initial values S^n Sc_{n0,ij} (n odd), S^n Sc_{n1,ij} (n even)
__device__ double xmax_envelope(double c, int npow, double tol)
{
    double lt = log(tol);
    double xs = npow / c;
    double step = 1.0 / c, hi = xs + step;
    while (npow * log(hi / xs) - c * (hi - xs) > lt) {
        step *= 2.0;
        hi = xs + step;
    }
    double lo = xs;
    for (int it = 0; it < 100; ++it) {
        double mid = 0.5 * (lo + hi);
        if (npow * log(mid / xs) - c * (mid - xs) > lt) lo = mid;
        else hi = mid;
    }
    return hi;
}

// Panel boundaries on [0, X]: width = min(1.1 pi/rho, 4.5/c, max(w0, 0.8 a)),
// w0 = min(lambda_min, pi/(2 D_max)).  Returns -1 if the budget is exceeded.
__device__ int make_panels(double rho, double c, int npow, double lam_min, double dmax, double tol, double* a,
                           int maxp)
{
    double X = (npow > 0) ? xmax_envelope(c, npow, tol) : -log(tol) / c;
    double w0 = lam_min;
    if (dmax > 0.0 && LPB_PI / (2.0 * dmax) < w0) w0 = LPB_PI / (2.0 * dmax);
    int np = 0;
    double x = 0.0;
    a[0] = 0.0;
    while (x < X) {
        double w = fmax(w0, 0.8 * x);
        w = fmin(w, 4.5 / c);
        if (rho > 0.0) w = fmin(w, 1.1 * LPB_PI / rho);
        x += w;
        if (np >= maxp) return -1;
        a[++np] = x;
    }
    return np;
}

__device__ inline double medium_lam_min(const Medium& M)
{
    double v = M.lam[0];
    for (int k = 1; k <= M.L; ++k) v = fmin(v, M.lam[k]);
    return v;
}

__device__ inline double medium_dmax(const Medium& M)
{
    double v = 0.0;
    for (int k = 1; k < M.L; ++k) v = fmax(v, M.d[k - 1] - M.d[k]);
    return v;
}

__global__ void __launch_bounds__(256) k_quad(int p, const RKey* __restrict__ rkeys, const FmmDev* __restrict__ fmms,
                                              const Medium* __restrict__ media, double tol,
                                              double* __restrict__ stab, int* __restrict__ flag)
{
    __shared__ double panels[LPB_MAXPANEL + 1];
    __shared__ int s_np;
    __shared__ double red[256];
    const int g = blockIdx.x, ij = blockIdx.y;
    const int i = ij >> 1, j = ij & 1;
    const RKey& rk = rkeys[g];
    const FmmDev& F = fmms[rk.fmm];
    const Medium& Md = media[F.medium];
    const int nmax = 2 * p + 3;
    const int N1 = nmax + 1;
    const double c = rk.zt - rk.zs;
    if (threadIdx.x == 0) {
        s_np = make_panels(rk.rho, c, nmax, medium_lam_min(Md), medium_dmax(Md), tol, panels, LPB_MAXPANEL);
        if (s_np < 0) atomicOr(flag, 1);
    }
    __syncthreads();
    const int np = s_np;
    double acc[LPB_MAXN];
#pragma unroll
    for (int n = 0; n < LPB_MAXN; ++n) acc[n] = 0.0;
    if (np > 0) {
        const double lt = F.lam_t, ls = F.lam_s;
        for (int k = threadIdx.x; k < np * LPB_NGL; k += blockDim.x) {
            int pn = k / LPB_NGL, q = k % LPB_NGL;
            double a0 = panels[pn], a1 = panels[pn + 1];
            double t = a0 + 0.5 * (a1 - a0) * (c_gl_x[q] + 1.0);
            double w = 0.5 * (a1 - a0) * c_gl_w[q];
            double lz = sqrt(lt * lt + t * t), lzp = sqrt(ls * ls + t * t);
            double sg = sigma_transmission(Md.L, Md.eps, Md.lam, Md.d, F.l, F.lp, F.a, F.b, t);
            double f = w * exp(-lz * rk.zt + lzp * rk.zs) * sg / lz;
            if (i) f *= lt / lz;
            if (j) f *= ls / lzp;
            double j0v = j0(t * rk.rho), j1v = j1(t * rk.rho);
            double ts = t * rk.S, pw = 1.0;
#pragma unroll
            for (int n = 0; n < LPB_MAXN; ++n) {
                if (n <= nmax) {
                    if (n & 1) acc[n] += f * pw * j0v / c_fact[n];
                    else if (n >= 2) acc[n] += f * pw * j1v / sqrt(c_fact[n + 1] * c_fact[n - 1]);
                }
                pw *= ts;
            }
        }
    }
    double* T = stab + ((size_t)g * 4 + ij) * N1 * N1;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int n = 0; n < LPB_MAXN; ++n) {
        if (n > nmax) break;
        double v = acc[n];
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        if (lane == 0) red[wv] = v;
        __syncthreads();
        if (threadIdx.x == 0) {
            double sum = 0.0;
            for (int k = 0; k < (int)(blockDim.x >> 6); ++k) sum += red[k];
            if (n & 1) T[n * N1 + 0] = sum;
            else if (n >= 2) T[n * N1 + 1] = sum;
        }
        __syncthreads();
    }
}

// forward recurrence (eq. recurrence1) on the entries with n - m odd:
//   S^n Sc_{n,m+1} = (2m/a_{n+m}) (S/rho) S^{n-1} Sc_{n-1,m} - (a_{n-m}/a_{n+m}) S^n Sc_{n,m-1}
__global__ void k_recur(int p, int nkeys, const RKey* __restrict__ rkeys, double* __restrict__ stab,
                        int* __restrict__ flag)
{
    int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= nkeys * 4) return;
    int g = idx / 4;
    const RKey& rk = rkeys[g];
    const int nmax = 2 * p + 3, N1 = nmax + 1;
    double* T = stab + (size_t)idx * N1 * N1;
    if (rk.rho == 0.0) {
        for (int n = 0; n <= nmax; ++n)
            for (int m = 1; m <= n; ++m) T[n * N1 + m] = 0.0;
        return;
    }
    const double sr = rk.S / rk.rho;
    for (int m = 1; m < nmax; ++m)
        for (int n = m + 1; n <= nmax; ++n) {
            if (((n - m - 1) & 1) == 0) continue;   // keep n - (m+1) odd
            double anm = sqrt((double)(n + m) * (n + m + 1));
            double amn = sqrt((double)(n - m) * (n - m + 1));
            if (2.0 * m / anm >= rk.rho / rk.S) atomicOr(flag, 2);
            T[n * N1 + m + 1] = 2.0 * m / anm * sr * T[(n - 1) * N1 + m] - amn / anm * T[n * N1 + m - 1];
        }
}

// scaled diagonal factors i_n(lam h), n = 0..p (local array)
__device__ inline void scale_in(int p, double lam, double h, double* out) { bessel_i_all(p, lam * h, out); }

// write the real-form entries of one (n, m>=0) x (nu, mu>=0) block
__device__ inline void store_real(double* __restrict__ R, int K, int n, int m, int nu, int mu, double2 Ap, double2 Am)
{
    // R column-major: R[col*K + row]
    if (mu == 0) {
        R[(size_t)ire(nu, 0) * K + ire(n, m)] = Ap.x;
        if (m > 0) R[(size_t)ire(nu, 0) * K + iim(n, m)] = Ap.y;
        return;
    }
    double sg = dsgn(mu);
    double Bx = sg * Am.x, By = sg * Am.y;
    R[(size_t)ire(nu, mu) * K + ire(n, m)] = Ap.x + Bx;
    R[(size_t)iim(nu, mu) * K + ire(n, m)] = -(Ap.y - By);
    if (m > 0) {
        R[(size_t)ire(nu, mu) * K + iim(n, m)] = Ap.y + By;
        R[(size_t)iim(nu, mu) * K + iim(n, m)] = Ap.x - Bx;
    }
}

// ---- reaction M2L operators -----------------------------------------------
__global__ void __launch_bounds__(256) k_react_op(int p, const int* __restrict__ op_list, const OpDesc* __restrict__ ops,
                                                  const RKey* __restrict__ rkeys, const FmmDev* __restrict__ fmms,
                                                  const int* __restrict__ rf_index, const double* __restrict__ dtab,
                                                  const double* __restrict__ stab, double* __restrict__ pool)
{
    const int K = (p + 1) * (p + 1), Kp = (p + 1) * (p + 2) / 2, SM = p + 2;
    const int nmax = 2 * p + 3, N1 = nmax + 1;
    const int oi = op_list[blockIdx.x];
    const OpDesc& od = ops[oi];
    const RKey& rk = rkeys[od.rkey];
    const FmmDev& F = fmms[od.fmm];
    __shared__ double in_t[LPB_MAX_P + 1], in_s[LPB_MAX_P + 1], sinv[LPB_MAXN];
    if (threadIdx.x == 0) {
        scale_in(p, F.lam_t, rk.S, in_t);
        scale_in(p, F.lam_s, rk.S, in_s);
        for (int N = 0; N <= nmax; ++N) sinv[N] = pow(rk.S, -(double)N);
    }
    __syncthreads();
    const double* D = dtab + (size_t)rf_index[od.fmm] * Kp * K * SM;
    const double* tab = stab + (size_t)od.rkey * 4 * N1 * N1;
    double* R = pool + (size_t)oi * K * K;
    for (int e = threadIdx.x; e < Kp * Kp; e += blockDim.x) {
        int row = e / Kp, colp = e % Kp;
        int n = 0;
        while ((n + 1) * (n + 2) / 2 <= row) ++n;
        int m = row - n * (n + 1) / 2;
        int nu = 0;
        while ((nu + 1) * (nu + 2) / 2 <= colp) ++nu;
        int mu0 = colp - nu * (nu + 1) / 2;
        double2 A[2];
        for (int sgn = 0; sgn < 2; ++sgn) {
            int mu = sgn ? -mu0 : mu0;
            A[sgn] = make_double2(0.0, 0.0);
            if (sgn && mu0 == 0) continue;
            int amu = mu0;
            int ii = (n + m) & 1, jj = (nu + amu) & 1;
            const double* Tb = tab + (size_t)(ii * 2 + jj) * N1 * N1;
            const double* Ds = D + ((size_t)row * K + jk(nu, mu)) * SM;
            int rn = (n + m) / 2, rnu = (nu + amu) / 2;
            int smax = (n - rn) + (nu - rnu);
            int M = mu - m, aM = M < 0 ? -M : M;
            double sgM = (M < 0) ? dsgn(aM) : 1.0;
            double I = 0.0;
            for (int s = 0; s <= smax; ++s) {
                int N = m + amu + 2 * s + 1;
                I += Ds[s] * Tb[N * N1 + aM] * sinv[N];
            }
            I *= sgM;
            double f = dsgn(n) * I * in_t[n] * 4.0 * LPB_PI * in_s[nu];
            double ang = (double)(mu - m) * od.phi;
            A[sgn] = make_double2(f * cos(ang), f * sin(ang));
        }
        store_real(R, K, n, m, nu, mu0, A[0], A[1]);
    }
}

// ---- free-space operators (M2M, L2L, M2L) ----------------------------------
__global__ void __launch_bounds__(256) k_free_op(int p, const int* __restrict__ op_list, const OpDesc* __restrict__ ops,
                                                 const FmmDev* __restrict__ fmms, const double* __restrict__ gtab,
                                                 double* __restrict__ pool)
{
    const int K = (p + 1) * (p + 1), Kp = (p + 1) * (p + 2) / 2, NQ = 2 * p + 1;
    const int oi = op_list[blockIdx.x];
    const OpDesc& od = ops[oi];
    const FmmDev& F = fmms[od.fmm];
    __shared__ double rad[2 * LPB_MAX_P + 1];
    __shared__ double2 Yb[(2 * LPB_MAX_P + 1) * LPB_YW];
    __shared__ double sc_row[LPB_MAX_P + 1], sc_col[LPB_MAX_P + 1];
    const double b = sqrt(od.bx * od.bx + od.by * od.by + od.bz * od.bz);
    const double lam = (od.type == OP_M2M) ? F.lam_s : F.lam_t;
    const double h = 2.0 * F.R / (double)(1 << od.level);   // side of the written level
    if (threadIdx.x == 0) {
        double tmp[2 * LPB_MAX_P + 1];
        if (od.type == OP_M2L_FREE) bessel_k_all(2 * p, lam * b, tmp);
        else bessel_i_all(2 * p, lam * b, tmp);
        for (int q = 0; q <= 2 * p; ++q) rad[q] = tmp[q];
        double a1[LPB_MAX_P + 1], a2[LPB_MAX_P + 1];
        if (od.type == OP_M2M) {          // rows: parent (h), cols: child (h/2)
            scale_in(p, lam, h, a1);
            scale_in(p, lam, 0.5 * h, a2);
            for (int n = 0; n <= p; ++n) { sc_row[n] = 1.0 / a1[n]; sc_col[n] = a2[n]; }
        } else if (od.type == OP_L2L) {   // rows: child (h), cols: parent (2h)
            scale_in(p, lam, h, a1);
            scale_in(p, lam, 2.0 * h, a2);
            for (int n = 0; n <= p; ++n) { sc_row[n] = a1[n]; sc_col[n] = 1.0 / a2[n]; }
        } else {                          // M2L: rows target (lam_t, h), cols source (lam_s, h)
            scale_in(p, F.lam_t, h, a1);
            scale_in(p, F.lam_s, h, a2);
            for (int n = 0; n <= p; ++n) { sc_row[n] = a1[n]; sc_col[n] = 4.0 * LPB_PI * a2[n]; }
        }
    }
    // harmonics of b^ for q <= 2p
    {
        const int Q = 2 * p;
        double ct = b > 0 ? od.bz / b : 1.0;
        double ph = (od.bx == 0.0 && od.by == 0.0) ? 0.0 : atan2(od.by, od.bx);
        for (int e = threadIdx.x; e < (Q + 1) * (Q + 2) / 2; e += blockDim.x) {
            int q = 0;
            while ((q + 1) * (q + 2) / 2 <= e) ++q;
            int s = e - q * (q + 1) / 2;
            // P^_q^s(ct) by the normalised recurrence in q for fixed s
            double sn = sqrt(fmax(0.0, 1.0 - ct * ct));
            double amm = 0.28209479177387814, sm = 1.0;
            for (int k = 1; k <= s; ++k) { amm *= sqrt((2.0 * k + 1.0) / (2.0 * k)); sm *= sn; }
            double p0 = amm * sm, val = p0;
            if (q > s) {
                double p1 = sqrt(2.0 * s + 3.0) * ct * p0;
                val = p1;
                for (int nn = s + 2; nn <= q; ++nn) {
                    double n2 = (double)nn * nn, m2 = (double)s * s;
                    double a = sqrt((4.0 * n2 - 1.0) / (n2 - m2));
                    double bb = sqrt(((nn - 1.0) * (nn - 1.0) - m2) * (2.0 * nn + 1.0) / ((n2 - m2) * (2.0 * nn - 3.0)));
                    double p2 = a * ct * p1 - bb * p0;
                    p0 = p1;
                    p1 = p2;
                    val = p2;
                }
            }
            double cs = cos(s * ph), sn2 = sin(s * ph);
            Yb[q * LPB_YW + (Q + s)] = make_double2(val * cs, val * sn2);
            if (s > 0) Yb[q * LPB_YW + (Q - s)] = make_double2(dsgn(s) * val * cs, -dsgn(s) * val * sn2);
        }
    }
    __syncthreads();
    const int Q = 2 * p;
    double* R = pool + (size_t)oi * K * K;
    for (int e = threadIdx.x; e < Kp * Kp; e += blockDim.x) {
        int row = e / Kp, colp = e % Kp;
        int n = 0;
        while ((n + 1) * (n + 2) / 2 <= row) ++n;
        int m = row - n * (n + 1) / 2;
        int nu = 0;
        while ((nu + 1) * (nu + 2) / 2 <= colp) ++nu;
        int mu0 = colp - nu * (nu + 1) / 2;
        double2 A[2];
        for (int sgn = 0; sgn < 2; ++sgn) {
            int mu = sgn ? -mu0 : mu0;
            A[sgn] = make_double2(0.0, 0.0);
            if (sgn && mu0 == 0) continue;
            const double* G = gtab + ((size_t)row * K + jk(nu, mu)) * NQ;
            double sr = 0.0, si = 0.0;
            int qlo = n > nu ? n - nu : nu - n;
            for (int q = qlo; q <= n + nu; q += 2) {
                double gq = G[q];
                if (gq == 0.0) continue;
                double2 y;
                double f;
                if (od.type == OP_M2M) {          // conj(Sh_{n nu}^{m mu}) : Y_q^{m-mu}
                    y = Yb[q * LPB_YW + (Q + m - mu)];
                    f = rad[q] * gq;
                    sr += f * y.x;
                    si -= f * y.y;
                } else if (od.type == OP_L2L) {   // Sh_{nu n}^{mu m} = ... Y_q^{mu-m} (-1)^{mu-m} G(n,m;nu,mu;q)
                    y = Yb[q * LPB_YW + (Q + mu - m)];
                    f = rad[q] * gq * dsgn(mu - m);
                    sr += f * y.x;
                    si += f * y.y;
                } else {                          // S_{nu n}^{mu m}: (-1)^{nu+q} k_q Y_q^{mu-m} (-1)^{mu-m} G
                    y = Yb[q * LPB_YW + (Q + mu - m)];
                    f = rad[q] * gq * dsgn(nu + q + mu - m);
                    sr += f * y.x;
                    si += f * y.y;
                }
            }
            double sc = 4.0 * LPB_PI * sc_row[n] * sc_col[nu];
            A[sgn] = make_double2(sc * sr, sc * si);
        }
        store_real(R, K, n, m, nu, mu0, A[0], A[1]);
    }
}

// Free-space M2L operators in the operand layout of the 16x16x4 MFMA:
//   out[((rb*KB + s4)*64 + lane)*4 + ss] = A[row = 16 rb + lane%16][k = 16 s4 + 4 ss + lane/16]
// (zero outside K x K), KB = KP/16.  A is the column-major FP64 operator.
template <typename T>
__global__ void k_swizzle(int K, int KP, int nsw, const int* __restrict__ ops, const double* __restrict__ pool,
                          T* __restrict__ out)
{
    const int KB = KP / 16;
    size_t per = (size_t)KP * KP;
    size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= per * nsw) return;
    int o = (int)(idx / per);
    size_t e = idx % per;
    int ss = (int)(e & 3), lane = (int)((e >> 2) & 63);
    size_t rest = e >> 8;
    int s4 = (int)(rest % KB), rb = (int)(rest / KB);
    int row = 16 * rb + (lane & 15), k = 16 * s4 + 4 * ss + (lane >> 4);
    double v = (row < K && k < K) ? pool[(size_t)ops[o] * K * K + (size_t)k * K + row] : 0.0;
    out[idx] = (T)v;
}

// The same layout with the rows permuted (rowmap: operand row -> result
// coefficient, -1 for a zero padding row), NRB row blocks, and the four
// coefficients a lane holds for the four products of a 16-coefficient slab
// consecutive (product ss, lane l: coefficient 16 s4 + 4 (l / 16) + ss).
__global__ void k_swizzle_rows(int K, int KP, int NRB, int nsw, const int* __restrict__ ops,
                               const int* __restrict__ rowmap, const double* __restrict__ pool, float* __restrict__ out)
{
    const int KB = KP / 16;
    size_t per = (size_t)NRB * 16 * KP;
    size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= per * nsw) return;
    int o = (int)(idx / per);
    size_t e = idx % per;
    int ss = (int)(e & 3), lane = (int)((e >> 2) & 63);
    size_t rest = e >> 8;
    int s4 = (int)(rest % KB), rb = (int)(rest / KB);
    int row = rowmap[16 * rb + (lane & 15)], k = 16 * s4 + 4 * (lane >> 4) + ss;
    double v = (row >= 0 && k < K) ? pool[(size_t)ops[o] * K * K + (size_t)k * K + row] : 0.0;
    out[idx] = (float)v;
}

// ---- reaction point operators of adaptive trees ---------------------------
// (Sec. 3.5, closing remarks on adaptive trees.)  In the canonical frame (a =
// 1 form) for one point and one box of side S:
//   M2P (W-list; target r, source box centre c):  u~(r) = sum M_{nu mu} F~_{nu mu},
//     F~_{nu mu} = e^{i mu phi} I_{00,nu mu}(rho, z, z_c) / sqrt(4 pi),  (rho, phi) of r - c;
//   P2L (X-list; image r', target box centre c):  L_nm = sqrt(4 pi) (-1)^n e^{-i m phi} I_{nm,00}(rho, z_c, z'),
//     (rho, phi) of c - r'  (the F~ and L rows of eq. coefintable, the L row being
//     the T row of a unit charge at r': its ME about r' is M_00 = sqrt(4 pi)).
// I from the D table (eq. metoletableform) and the scaled integrals
// S^n Sc_{nm,ij} up to n = p + 2 (the largest index the rows (0,0) and
// columns (0,0) reach).  rho may be below S here, so the table mixes the two
// recurrences: initial values by quadrature for m = 0 and 1 (all n) and for
// the row n = p + 2, the forward recurrence (eq. recurrence1) wherever its
// bound 2m/a_{n+m} < rho/S holds, the backward recurrence (eq.
// backwardrecurrence1) for the other entries, row by row down; only entries
// with n - m odd enter I.  Output in the real form of the expansions (the
// scaled ME Mh = M / (4 pi i_nu(lam_s S)) is dotted with the M2P row; the
// P2L vector is the scaled Lh = i_n(lam_t S) L of a unit charge).
#define LPB_PTN (LPB_MAX_P + 3)
#define LPB_PTH ((LPB_PTN + 1) / 2)
template <typename T>
__global__ void __launch_bounds__(64) k_point_ops(int p, const PointOp* __restrict__ pops, const FmmDev* __restrict__ fmms,
                                                  const Medium* __restrict__ media, const int* __restrict__ rf_index,
                                                  const double* __restrict__ dtab, const T* __restrict__ tx,
                                                  const T* __restrict__ ty, const T* __restrict__ tz,
                                                  const T* __restrict__ tlx, const T* __restrict__ tly,
                                                  const T* __restrict__ tlz, const T* __restrict__ sx,
                                                  const T* __restrict__ sy, const T* __restrict__ sz,
                                                  const T* __restrict__ slx, const T* __restrict__ sly,
                                                  const T* __restrict__ slz, const double* __restrict__ tl_ctr,
                                                  const double* __restrict__ sl_ctr, double tol,
                                                  double* __restrict__ out, int* __restrict__ flag)
{
    __shared__ double panels[LPB_MAXPANEL + 1];
    __shared__ int s_np;
    __shared__ double tab[2][LPB_PTN][LPB_PTN];
    __shared__ double sc[LPB_MAX_P + 1], sinv[LPB_PTN];
    const PointOp& op = pops[blockIdx.x];
    const FmmDev& F = fmms[op.fmm];
    const Medium& Md = media[F.medium];
    const int K = (p + 1) * (p + 1), Kp = (p + 1) * (p + 2) / 2, SM = p + 2;
    const int N = p + 2;
    const int lane = threadIdx.x;
    // the point (canonical frame) and the geometry of the pair
    double px, py, pz;
    if (op.kind == 0) {
        px = tl_ctr[3 * op.leaf] + (double)tx[op.pt] + (tlx ? (double)tlx[op.pt] : 0.0);
        py = tl_ctr[3 * op.leaf + 1] + (double)ty[op.pt] + (tly ? (double)tly[op.pt] : 0.0);
        pz = tl_ctr[3 * op.leaf + 2] + (double)tz[op.pt] + (tlz ? (double)tlz[op.pt] : 0.0);
    } else {
        px = sl_ctr[3 * op.leaf] + (double)sx[op.pt] + (slx ? (double)slx[op.pt] : 0.0);
        py = sl_ctr[3 * op.leaf + 1] + (double)sy[op.pt] + (sly ? (double)sly[op.pt] : 0.0);
        pz = sl_ctr[3 * op.leaf + 2] + (double)sz[op.pt] + (slz ? (double)slz[op.pt] : 0.0);
    }
    const double dx = op.kind == 0 ? px - op.bx : op.bx - px, dy = op.kind == 0 ? py - op.by : op.by - py;
    const double rho = sqrt(dx * dx + dy * dy);
    const double phi = rho > 0.0 ? atan2(dy, dx) : 0.0;
    const double zt = op.kind == 0 ? pz : op.bz, zs = op.kind == 0 ? op.bz : pz;
    const double S = op.h, c = zt - zs;
    if (lane == 0) {
        s_np = make_panels(rho, c, N, medium_lam_min(Md), medium_dmax(Md), tol, panels, LPB_MAXPANEL);
        if (s_np < 0) atomicOr(flag, 1);
    }
    __syncthreads();
    const int np = s_np;
    // per lane: initial values of two tables (ij = 00 and, for M2P, 01; for
    // P2L, 10): m = 0 at odd n, m = 1 at even n >= 2, row N at m >= 2 with N - m odd
    double a0[2][LPB_PTH], a1[2][LPB_PTH], ar[2][LPB_PTH];
    for (int q = 0; q < 2; ++q)
        for (int k = 0; k < LPB_PTH; ++k) a0[q][k] = a1[q][k] = ar[q][k] = 0.0;
    const double lt = F.lam_t, ls = F.lam_s;
    for (int k = lane; k < (np > 0 ? np : 0) * LPB_NGL; k += 64) {
        const int pn = k / LPB_NGL, qd = k % LPB_NGL;
        const double x0 = panels[pn], x1 = panels[pn + 1];
        const double t = x0 + 0.5 * (x1 - x0) * (c_gl_x[qd] + 1.0);
        const double w = 0.5 * (x1 - x0) * c_gl_w[qd];
        const double lz = sqrt(lt * lt + t * t), lzp = sqrt(ls * ls + t * t);
        const double sg = sigma_transmission(Md.L, Md.eps, Md.lam, Md.d, F.l, F.lp, F.a, F.b, t);
        const double f0 = w * exp(-lz * zt + lzp * zs) * sg / lz;
        const double f[2] = {f0, op.kind == 0 ? f0 * ls / lzp : f0 * lt / lz};
        const double j0v = j0(t * rho), j1v = j1(t * rho);
        const double ts = t * S;
        double pw = 1.0;
        for (int n = 0; n <= N; ++n) {
            for (int q = 0; q < 2; ++q) {
                if (n & 1) a0[q][n >> 1] += f[q] * pw * j0v / c_fact[n];
                else if (n >= 2) a1[q][(n >> 1) - 1] += f[q] * pw * j1v / sqrt(c_fact[n + 1] * c_fact[n - 1]);
            }
            if (n < N) pw *= ts;
        }
        if (rho > 0.0)
            for (int m = 2; m <= N; ++m) {
                if (((N - m) & 1) == 0) continue;
                const double jm = jn(m, t * rho) * pw / sqrt(c_fact[N + m] * c_fact[N - m]);
                for (int q = 0; q < 2; ++q) ar[q][m >> 1] += f[q] * jm;
            }
    }
    // wave reductions (one wave per block), in a fixed order
    for (int q = 0; q < 2; ++q)
        for (int k = 0; k < LPB_PTH; ++k)
            for (int off = 32; off > 0; off >>= 1) {
                a0[q][k] += __shfl_xor(a0[q][k], off, 64);
                a1[q][k] += __shfl_xor(a1[q][k], off, 64);
                ar[q][k] += __shfl_xor(ar[q][k], off, 64);
            }
    if (lane == 0) {
        for (int q = 0; q < 2; ++q) {
            double(*Tq)[LPB_PTN] = tab[q];
            bool done[LPB_PTN][LPB_PTN];
            for (int n = 0; n <= N; ++n)
                for (int m = 0; m <= N; ++m) {
                    Tq[n][m] = 0.0;
                    done[n][m] = false;
                }
            for (int n = 1; n <= N; n += 2) { Tq[n][0] = a0[q][n >> 1]; done[n][0] = true; }
            for (int n = 2; n <= N; n += 2) { Tq[n][1] = a1[q][(n >> 1) - 1]; done[n][1] = true; }
            if (rho > 0.0) {
                for (int m = 2; m <= N; ++m)
                    if ((N - m) & 1) { Tq[N][m] = ar[q][m >> 1]; done[N][m] = true; }
                const double x = rho / S;
                // forward, increasing m: (n, m+1) from (n-1, m) and (n, m-1), n - m even
                for (int m = 1; m < N; ++m)
                    for (int n = m + 1; n < N; ++n) {
                        if (((n - m) & 1) != 0) continue;
                        const double anm = sqrt((double)(n + m) * (n + m + 1));
                        if (!(2.0 * m / anm < x) || !done[n - 1][m] || !done[n][m - 1]) continue;
                        const double amn = sqrt((double)(n - m) * (n - m + 1));
                        Tq[n][m + 1] = 2.0 * m / anm / x * Tq[n - 1][m] - amn / anm * Tq[n][m - 1];
                        done[n][m + 1] = true;
                    }
                // backward, down from the row N: (n-1, m) from (n, m+1) and (n, m-1)
                for (int n = N; n >= 2; --n)
                    for (int m = 1; m <= n - 1; ++m) {
                        if ((((n - 1) - m) & 1) == 0 || done[n - 1][m]) continue;
                        const double anm = sqrt((double)(n + m) * (n + m + 1));
                        const double amn = sqrt((double)(n - m) * (n - m + 1));
                        Tq[n - 1][m] = anm / (2.0 * m) * x * Tq[n][m + 1] + amn / (2.0 * m) * x * Tq[n][m - 1];
                        done[n - 1][m] = true;
                    }
            }
        }
        double buf[LPB_MAX_P + 2];
        bessel_i_all(p, (op.kind == 0 ? ls : lt) * S, buf);
        for (int n = 0; n <= p; ++n) sc[n] = buf[n];
        for (int n = 0; n <= N; ++n) sinv[n] = pow(S, -(double)n);
    }
    __syncthreads();
    const double* D = dtab + (size_t)rf_index[op.fmm] * Kp * K * SM;
    double* o = out + op.out;
    const double r4pi = 1.0 / sqrt(4.0 * LPB_PI);
    if (op.kind == 0) {
        // row (0,0) of D; columns (nu, +-mu); q = table of parity j = (nu + mu) & 1
        for (int e = lane; e < Kp; e += 64) {
            int nu = 0;
            while ((nu + 1) * (nu + 2) / 2 <= e) ++nu;
            const int mu = e - nu * (nu + 1) / 2;
            const int q = (nu + mu) & 1;
            const int rn = (nu + mu) / 2, smax = nu - rn;
            double Fr[2] = {0.0, 0.0}, Fi[2] = {0.0, 0.0};
            for (int sgn = 0; sgn < 2; ++sgn) {
                if (sgn && mu == 0) continue;
                const int m2 = sgn ? -mu : mu;
                const double* Ds = D + ((size_t)0 * K + jk(nu, m2)) * SM;
                double I = 0.0;
                for (int s = 0; s <= smax; ++s) {
                    const int Nn = mu + 2 * s + 1;
                    I += Ds[s] * tab[q][Nn][mu] * sinv[Nn];
                }
                if (m2 < 0) I *= dsgn(mu);
                Fr[sgn] = cos(m2 * phi) * I * r4pi;
                Fi[sgn] = sin(m2 * phi) * I * r4pi;
            }
            const double f = 4.0 * LPB_PI * sc[nu];
            if (mu == 0) {
                o[ire(nu, 0)] = f * Fr[0];
            } else {
                o[ire(nu, mu)] = f * (Fr[0] + dsgn(mu) * Fr[1]);
                o[iim(nu, mu)] = f * (-Fi[0] + dsgn(mu) * Fi[1]);
            }
        }
    } else {
        // rows (n, m >= 0) of D, column (0,0); q = table of parity i = (n + m) & 1
        for (int e = lane; e < Kp; e += 64) {
            int n = 0;
            while ((n + 1) * (n + 2) / 2 <= e) ++n;
            const int m = e - n * (n + 1) / 2;
            const int q = (n + m) & 1;
            const int rn = (n + m) / 2, smax = n - rn;
            const double* Ds = D + ((size_t)e * K + jk(0, 0)) * SM;
            double I = 0.0;
            for (int s = 0; s <= smax; ++s) {
                const int Nn = m + 2 * s + 1;
                I += Ds[s] * tab[q][Nn][m] * sinv[Nn];
            }
            I *= dsgn(m);   // Sc_{N,-m} = (-1)^m Sc_{N,m}
            const double f = sqrt(4.0 * LPB_PI) * dsgn(n) * I * sc[n];
            o[ire(n, m)] = f * cos(m * phi);
            if (m > 0) o[iim(n, m)] = -f * sin(m * phi);
        }
    }
}

__global__ void k_to_float(size_t n, const double* __restrict__ a, float* __restrict__ b)
{
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) b[i] = (float)a[i];
}

// Host driver ----------------------------------------------------------------
// 20-point Gauss-Legendre nodes and weights on [-1,1] by Newton iteration on P_20
void gauss_legendre20(double* x, double* w)
{
    const int n = 20;
    for (int i = 0; i < n; ++i) {
        double z = cos(LPB_PI * (i + 0.75) / (n + 0.5));
        for (int it = 0; it < 100; ++it) {
            double p1 = 1.0, p2 = 0.0;
            for (int j = 1; j <= n; ++j) {
                double p3 = p2;
                p2 = p1;
                p1 = ((2.0 * j - 1.0) * z * p2 - (j - 1.0) * p3) / j;
            }
            double dp = n * (z * p1 - p2) / (z * z - 1.0);
            double dz = p1 / dp;
            z -= dz;
            if (fabs(dz) < 1e-16) break;
        }
        double p1 = 1.0, p2 = 0.0;
        for (int j = 1; j <= n; ++j) {
            double p3 = p2;
            p2 = p1;
            p1 = ((2.0 * j - 1.0) * z * p2 - (j - 1.0) * p3) / j;
        }
        double dp = n * (z * p1 - p2) / (z * z - 1.0);
        x[i] = z;
        w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

hipError_t opgen_upload_constants()
{
    double f[171];
    f[0] = 1.0;
    for (int k = 1; k <= 170; ++k) f[k] = f[k - 1] * (double)k;
    hipError_t e = hipMemcpyToSymbol(HIP_SYMBOL(c_fact), f, sizeof(f));
    if (e != hipSuccess) return e;
    double x[20], w[20];
    gauss_legendre20(x, w);
    e = hipMemcpyToSymbol(HIP_SYMBOL(c_gl_x), x, sizeof(x));
    if (e != hipSuccess) return e;
    return hipMemcpyToSymbol(HIP_SYMBOL(c_gl_w), w, sizeof(w));
}

hipError_t opgen_run(const OpgenInputs& in, hipStream_t st)
{
    const int p = in.p, K = (p + 1) * (p + 1), Kp = (p + 1) * (p + 2) / 2;
    if (in.n_rf > 0) {
        long long total = (long long)in.n_rf * Kp * K;
        int blocks = (int)((total + 255) / 256);
        hipLaunchKernelGGL(k_dtable, dim3(blocks), dim3(256), 0, st, p, in.n_rf, in.d_rf_list, in.d_fmm, in.d_btab,
                           in.d_dtab);
    }
    if (in.n_pt > 0) {
        if (in.pt_f32)
            hipLaunchKernelGGL(k_point_ops<float>, dim3(in.n_pt), dim3(64), 0, st, p, in.d_pt_ops, in.d_fmm, in.d_media,
                               in.d_rf_index, in.d_dtab, (const float*)in.t_u[0], (const float*)in.t_u[1],
                               (const float*)in.t_u[2], (const float*)in.t_u[3], (const float*)in.t_u[4],
                               (const float*)in.t_u[5], (const float*)in.s_u[0], (const float*)in.s_u[1],
                               (const float*)in.s_u[2], (const float*)in.s_u[3], (const float*)in.s_u[4],
                               (const float*)in.s_u[5], in.tl_ctr, in.sl_ctr, in.quad_tol, in.d_pt_vec, in.d_flag);
        else
            hipLaunchKernelGGL(k_point_ops<double>, dim3(in.n_pt), dim3(64), 0, st, p, in.d_pt_ops, in.d_fmm, in.d_media,
                               in.d_rf_index, in.d_dtab, (const double*)in.t_u[0], (const double*)in.t_u[1],
                               (const double*)in.t_u[2], (const double*)in.t_u[3], (const double*)in.t_u[4],
                               (const double*)in.t_u[5], (const double*)in.s_u[0], (const double*)in.s_u[1],
                               (const double*)in.s_u[2], (const double*)in.s_u[3], (const double*)in.s_u[4],
                               (const double*)in.s_u[5], in.tl_ctr, in.sl_ctr, in.quad_tol, in.d_pt_vec, in.d_flag);
    }
    if (in.n_rkeys > 0) {
        hipLaunchKernelGGL(k_quad, dim3(in.n_rkeys, 4), dim3(256), 0, st, p, in.d_rkeys, in.d_fmm, in.d_media,
                           in.quad_tol, in.d_stab, in.d_flag);
        int thr = in.n_rkeys * 4;
        hipLaunchKernelGGL(k_recur, dim3((thr + 63) / 64), dim3(64), 0, st, p, in.n_rkeys, in.d_rkeys, in.d_stab,
                           in.d_flag);
    }
    if (in.n_react > 0)
        hipLaunchKernelGGL(k_react_op, dim3(in.n_react), dim3(256), 0, st, p, in.d_react_list, in.d_ops, in.d_rkeys,
                           in.d_fmm, in.d_rf_index, in.d_dtab, in.d_stab, in.d_pool);
    if (in.n_free > 0)
        hipLaunchKernelGGL(k_free_op, dim3(in.n_free), dim3(256), 0, st, p, in.d_free_list, in.d_ops, in.d_fmm,
                           in.d_gtab, in.d_pool);
    if (in.d_pool32) {
        size_t n = (size_t)in.n_ops * K * K;
        hipLaunchKernelGGL(k_to_float, dim3(2048), dim3(256), 0, st, n, in.d_pool, in.d_pool32);
    }
    if (in.n_swz > 0) {
        size_t n = (size_t)in.KP * in.KP * in.n_swz;
        unsigned blocks = (unsigned)((n + 255) / 256);
        if (in.d_swz32)
            hipLaunchKernelGGL(k_swizzle<float>, dim3(blocks), dim3(256), 0, st, K, in.KP, in.n_swz, in.d_swz_ops,
                               in.d_pool, in.d_swz32);
        else
            hipLaunchKernelGGL(k_swizzle<double>, dim3(blocks), dim3(256), 0, st, K, in.KP, in.n_swz, in.d_swz_ops,
                               in.d_pool, in.d_swz64);
    }
    if (in.n_orb > 0 && in.d_orb32) {
        size_t n = (size_t)in.NRB * 16 * in.KP * in.n_orb;
        unsigned blocks = (unsigned)((n + 255) / 256);
        hipLaunchKernelGGL(k_swizzle_rows, dim3(blocks), dim3(256), 0, st, K, in.KP, in.NRB, in.n_orb, in.d_orb_ops,
                           in.d_rowmap, in.d_pool, in.d_orb32);
    }
    return hipGetLastError();
}

}  // namespace lpb
