// lpb_math.h -- special functions and expansion bases of the GPU library
// (host + device).  Written for the library; shares nothing with the oracle.
//
// Bases (Sec. 3.1 of Wang, Zhang, Cai): Y_n^m = P^_n^m(cos t) e^{i m p} with
// P^_n^m = sqrt((2n+1)/(4 pi) (n-m)!/(n+m)!) (1-x^2)^{m/2} d^m P_n/dx^m (m >= 0,
// no Condon-Shortley phase) and Y_n^{-m} = (-1)^m conj(Y_n^m); modified
// spherical Bessel functions i_n(x) = sqrt(pi/(2x)) I_{n+1/2}(x) and
// k_n(x) = sqrt(pi/(2x)) K_{n+1/2}(x), so k_0(x) = (pi/2) e^{-x}/x.
//
// The expansions are stored scaled per tree level (box side h):
//   Mh_nm = M_nm / (4 pi i_n(lam h)),   Lh_nm = L_nm i_n(lam h),
// which turns P2M and L2P into sums of q * g_n(r) * R_n^m(u/h) with the
// regular solid harmonic R_n^m(v) = |v|^n Y_n^m(v^) and the Bessel ratio
// g_n(r) = it_n(lam r) / it_n(lam h), where it_n(x) = i_n(x) (2n+1)!! / x^n
// is an even power series in x with it_n(0) = 1.
#pragma once
#include <math.h>

#ifdef __HIPCC__
#define LPB_HD __host__ __device__ inline
#else
#define LPB_HD inline
#endif

#define LPB_PI 3.14159265358979323846

namespace lpb {

// it_n(x) for n = 0..nmax as a function of t = x^2.  The two highest orders
// come from the series  it_n = sum_k (t/2)^k / (k! prod_{j=1..k} (2n+2j+1));
// the rest from the backward recurrence
//   it_{n-1} = it_n + t it_{n+1} / ((2n+1)(2n+3))
// (from i_{n-1} - i_{n+1} = (2n+1) i_n / x), which needs no division by x.
LPB_HD double itilde_series(int n, double t)
{
    double term = 1.0, sum = 1.0;
    for (int k = 1; k < 4000; ++k) {
        term *= 0.5 * t / ((double)k * (2.0 * n + 2.0 * k + 1.0));
        sum += term;
        if (term <= 1e-17 * sum) break;
    }
    return sum;
}

LPB_HD void itilde_all(int nmax, double t, double* out)
{
    double a = itilde_series(nmax + 1, t);
    double b = itilde_series(nmax, t);
    out[nmax] = b;
    for (int n = nmax; n >= 1; --n) {
        double c = b + t * a / ((2.0 * n + 1.0) * (2.0 * n + 3.0));
        out[n - 1] = c;
        a = b;
        b = c;
    }
}

// i_n(x), n = 0..nmax (x >= 0)
LPB_HD void bessel_i_all(int nmax, double x, double* out)
{
    itilde_all(nmax, x * x, out);
    double f = 1.0;
    for (int n = 0; n <= nmax; ++n) {
        out[n] *= f;               // f = x^n / (2n+1)!!
        f *= x / (2.0 * n + 3.0);
    }
}

// k_n(x), n = 0..nmax (x > 0) by the forward recurrence
// k_{n+1} = k_{n-1} + (2n+1)/x k_n, which is stable for the growing k_n.
LPB_HD void bessel_k_all(int nmax, double x, double* out)
{
    double e = 0.5 * LPB_PI * exp(-x) / x;
    out[0] = e;
    if (nmax >= 1) out[1] = e * (1.0 + 1.0 / x);
    for (int n = 1; n < nmax; ++n) out[n + 1] = out[n - 1] + (2.0 * n + 1.0) / x * out[n];
}

// Index of the real-form coefficient vector: degree n occupies [n^2, n^2+2n];
// Re of order m at n^2 + (m ? 2m-1 : 0), Im of order m > 0 at n^2 + 2m.
LPB_HD constexpr int ire(int n, int m) { return n * n + (m ? 2 * m - 1 : 0); }
LPB_HD constexpr int iim(int n, int m) { return n * n + 2 * m; }
// packed (n, m >= 0) index
LPB_HD constexpr int ipk(int n, int m) { return n * (n + 1) / 2 + m; }

// Sign class of a real-form coefficient under the reflections of the axes:
// bit 0 set if it changes sign under x -> -x (Re: m odd, Im: m even), bit 1
// under y -> -y (the Im parts), bit 2 under z -> -z (n + m odd).
LPB_HD constexpr int coef_class(int n, int m, int im)
{
    return (im ? 1 - (m & 1) : (m & 1)) | (im ? 2 : 0) | (((n + m) & 1) << 2);
}
LPB_HD constexpr int class_size(int p, int c)
{
    int s = 0;
    for (int n = 0; n <= p; ++n)
        for (int m = 0; m <= n; ++m) {
            s += coef_class(n, m, 0) == c;
            if (m > 0) s += coef_class(n, m, 1) == c;
        }
    return s;
}
// Rows ordered by sign class, each class padded to a multiple of 16: the
// number of 16-row blocks, and the class of block rb.
LPB_HD constexpr int class_row_blocks(int p)
{
    int b = 0;
    for (int c = 0; c < 8; ++c) b += (class_size(p, c) + 15) / 16;
    return b;
}
LPB_HD constexpr int class_of_row_block(int p, int rb)
{
    for (int c = 0; c < 8; ++c) {
        rb -= (class_size(p, c) + 15) / 16;
        if (rb < 0) return c;
    }
    return 7;
}

// Regular solid harmonics R_n^m(v) = |v|^n Y_n^m(v^), 0 <= m <= n <= p,
// written to re/im at packed index ipk(n,m), from
//   R_m^m = A_m (x + i y)^m,  A_m = A_{m-1} sqrt((2m+1)/(2m)), A_0 = 1/sqrt(4 pi),
//   R_n^m = al_nm z R_{n-1}^m - be_nm |v|^2 R_{n-2}^m,
//   al_nm = sqrt((4n^2-1)/(n^2-m^2)),
//   be_nm = sqrt(((n-1)^2-m^2)(2n+1)/((n^2-m^2)(2n-3))).
template <typename T>
LPB_HD void solid_harmonics(int p, T x, T y, T z, T* re, T* im)
{
    T r2 = x * x + y * y + z * z;
    T wr = T(1), wi = T(0);          // (x + i y)^m
    T amm = T(0.28209479177387814);  // 1/sqrt(4 pi)
    for (int m = 0; m <= p; ++m) {
        if (m > 0) {
            T nr = wr * x - wi * y;
            wi = wr * y + wi * x;
            wr = nr;
            amm *= (T)sqrt((2.0 * m + 1.0) / (2.0 * m));
        }
        T pr = amm * wr, pi = amm * wi;   // R_m^m
        re[ipk(m, m)] = pr;
        im[ipk(m, m)] = pi;
        if (m + 1 > p) continue;
        T al = (T)sqrt(2.0 * m + 3.0);   // al_{m+1,m} = sqrt((4(m+1)^2-1)/(2m+1))
        T qr = al * z * pr, qi = al * z * pi;
        re[ipk(m + 1, m)] = qr;
        im[ipk(m + 1, m)] = qi;
        for (int n = m + 2; n <= p; ++n) {
            double nn = (double)n * n, mm = (double)m * m;
            T a = (T)sqrt((4.0 * nn - 1.0) / (nn - mm));
            T b = (T)sqrt(((n - 1.0) * (n - 1.0) - mm) * (2.0 * n + 1.0) / ((nn - mm) * (2.0 * n - 3.0)));
            T sr = a * z * qr - b * r2 * pr;
            T si = a * z * qi - b * r2 * pi;
            re[ipk(n, m)] = sr;
            im[ipk(n, m)] = si;
            pr = qr;
            pi = qi;
            qr = sr;
            qi = si;
        }
    }
}

// Normalised associated Legendre P^_n^m(x), 0 <= m <= n <= nmax, packed index.
LPB_HD void legendre_norm(int nmax, double x, double* out)
{
    double s = sqrt(fmax(0.0, 1.0 - x * x));
    double amm = 0.28209479177387814;
    double sm = 1.0;
    for (int m = 0; m <= nmax; ++m) {
        if (m > 0) {
            amm *= sqrt((2.0 * m + 1.0) / (2.0 * m));
            sm *= s;
        }
        double p0 = amm * sm;
        out[ipk(m, m)] = p0;
        if (m + 1 > nmax) continue;
        double p1 = sqrt(2.0 * m + 3.0) * x * p0;
        out[ipk(m + 1, m)] = p1;
        for (int n = m + 2; n <= nmax; ++n) {
            double nn = (double)n * n, mm = (double)m * m;
            double a = sqrt((4.0 * nn - 1.0) / (nn - mm));
            double b = sqrt(((n - 1.0) * (n - 1.0) - mm) * (2.0 * n + 1.0) / ((nn - mm) * (2.0 * n - 3.0)));
            double p2 = a * x * p1 - b * p0;
            out[ipk(n, m)] = p2;
            p0 = p1;
            p1 = p2;
        }
    }
}

// Reaction density sigma^{ab}_{l lp}(lrho) of an (L+1)-layer medium from the
// transmission conditions (Sec. 2.1: continuity of u and eps du/dz at each
// interface, decay at +-inf).  In layer k the spectral field is
//   [k == lp] e^{-lz_lp |z - z'|}/(eps_lp lz_lp)
//   + A_k e^{-lz_k (z - d_k)}/lz_k + B_k e^{-lz_k (d_{k-1} - z)}/lz_k,
// with A_L = B_0 = 0; A_k, B_k are linear in X_1 = e^{-lz_lp (z'-d_lp)} and
// X_2 = e^{-lz_lp (d_{lp-1}-z')}, and sigma^{1b} (sigma^{2b}) is the
// coefficient of X_b in A_l (B_l) (eqs. greenfuncomponent, totaldensity).
// Every basis function is 1/lz at its own interface and decays away from it,
// so no entry overflows.  Unknowns: A_0..A_{L-1}, B_1..B_L.
#define LPB_MAXL 8
LPB_HD double sigma_transmission(int L, const double* eps, const double* lam, const double* d, int l, int lp, int a,
                                 int b, double lrho)
{
    const int n = 2 * L;
    double M[2 * LPB_MAXL][2 * LPB_MAXL + 1];
    double lz[LPB_MAXL + 1];
    for (int k = 0; k <= L; ++k) lz[k] = sqrt(lam[k] * lam[k] + lrho * lrho);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j <= n; ++j) M[i][j] = 0.0;
    for (int i = 0; i < L; ++i) {
        int rv = 2 * i, rf = 2 * i + 1;
        // layer i (above interface i)
        M[rv][i] += 1.0 / lz[i];
        M[rf][i] -= eps[i];
        if (i >= 1) {
            double e = exp(-lz[i] * (d[i - 1] - d[i]));
            M[rv][L + i - 1] += e / lz[i];
            M[rf][L + i - 1] += eps[i] * e;
        }
        // layer i+1 (below interface i)
        if (i + 1 < L) {
            double e = exp(-lz[i + 1] * (d[i] - d[i + 1]));
            M[rv][i + 1] -= e / lz[i + 1];
            M[rf][i + 1] += eps[i + 1] * e;
        }
        M[rv][L + i] -= 1.0 / lz[i + 1];
        M[rf][L + i] -= eps[i + 1];
        // free-space part of the source, coefficient of X_b
        if (lp == i && b == 1) {
            M[rv][n] -= 1.0 / (eps[lp] * lz[lp]);
            M[rf][n] -= eps[i] / eps[lp];
        }
        if (lp == i + 1 && b == 2) {
            M[rv][n] += 1.0 / (eps[lp] * lz[lp]);
            M[rf][n] -= eps[i + 1] / eps[lp];
        }
    }
    // Gaussian elimination with partial pivoting
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int r = c + 1; r < n; ++r)
            if (fabs(M[r][c]) > fabs(M[piv][c])) piv = r;
        if (piv != c)
            for (int j = c; j <= n; ++j) {
                double t = M[c][j];
                M[c][j] = M[piv][j];
                M[piv][j] = t;
            }
        double inv = 1.0 / M[c][c];
        for (int r = c + 1; r < n; ++r) {
            double f = M[r][c] * inv;
            if (f == 0.0) continue;
            for (int j = c; j <= n; ++j) M[r][j] -= f * M[c][j];
        }
    }
    double x[2 * LPB_MAXL];
    for (int r = n - 1; r >= 0; --r) {
        double s = M[r][n];
        for (int j = r + 1; j < n; ++j) s -= M[r][j] * x[j];
        x[r] = s / M[r][r];
    }
    return (a == 1) ? x[l] : x[L + l - 1];
}

}  // namespace lpb

namespace lpb {
// R_n^m(v) as in solid_harmonics, written with a stride (LDS columns).
template <typename T>
LPB_HD void solid_harmonics_lds(int p, T x, T y, T z, T* re, T* im, int stride)
{
    T r2 = x * x + y * y + z * z;
    T wr = T(1), wi = T(0);
    T amm = T(0.28209479177387814);
    for (int m = 0; m <= p; ++m) {
        if (m > 0) {
            T nr = wr * x - wi * y;
            wi = wr * y + wi * x;
            wr = nr;
            amm *= (T)sqrt((2.0 * m + 1.0) / (2.0 * m));
        }
        T pr = amm * wr, pi = amm * wi;
        re[(size_t)ipk(m, m) * stride] = pr;
        im[(size_t)ipk(m, m) * stride] = pi;
        if (m + 1 > p) continue;
        T al = (T)sqrt(2.0 * m + 3.0);
        T qr = al * z * pr, qi = al * z * pi;
        re[(size_t)ipk(m + 1, m) * stride] = qr;
        im[(size_t)ipk(m + 1, m) * stride] = qi;
        for (int n = m + 2; n <= p; ++n) {
            double nn = (double)n * n, mm = (double)m * m;
            T a = (T)sqrt((4.0 * nn - 1.0) / (nn - mm));
            T b = (T)sqrt(((n - 1.0) * (n - 1.0) - mm) * (2.0 * n + 1.0) / ((nn - mm) * (2.0 * n - 3.0)));
            T sr = a * z * qr - b * r2 * pr;
            T si = a * z * qi - b * r2 * pi;
            re[(size_t)ipk(n, m) * stride] = sr;
            im[(size_t)ipk(n, m) * stride] = si;
            pr = qr;
            pi = qi;
            qr = sr;
            qi = si;
        }
    }
}
}  // namespace lpb
