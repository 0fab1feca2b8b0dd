/*
 * lpb_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, FP64 CPU oracle for the layered-media linearized
 * Poisson-Boltzmann (screened Coulomb / Yukawa) potential and its fast
 * multipole method, written from B. Wang, W. Z. Zhang, W. Cai, "Fast Multipole
 * Method for 3-D Linearized Poisson-Boltzmann Equation in Layered Media"
 * (arXiv 2002.01334).  Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library; the GPU product path
 * never does.  It shares no code, header, table or constant generator with
 * the GPU library.
 *
 * Contents (paper section / equation each function follows):
 *   - special functions: modified spherical Bessel i_n, k_n (Sec. 3.1),
 *     normalised associated Legendre P^_n^m, spherical harmonics Y_n^m
 *     (Sec. 3.1 definition), Gaunt integrals of three harmonics (Thm 3.2/3.3),
 *     Gauss-Legendre nodes.
 *   - reaction densities sigma^{ab}_{ll'} of the three-layer medium
 *     (eqs. densitythreelayer1-3), in an overflow-free scaled form.
 *   - direct O(N^2) sum of the layered Green's function (eqs. potential1,
 *     totalinteraction, generalcomponents, zexponential), reaction parts by
 *     composite Gauss-Legendre quadrature of the Sommerfeld integrals after
 *     the angular integral is done with the J_n identity (Sec. 3.5).
 *   - CPU FMM (Algorithms 1 and 2): free-space Yukawa FMM with the addition
 *     theorem operators (eqs. melecoeffree, metole, metome), and one FMM per
 *     reaction component over equivalent polarization sources
 *     (eqs. equivpolarcoord, melayerupgoingimage, lelayerimage) whose M2L
 *     operators come from quadrature of the initial values, the forward
 *     recurrence (eq. recurrence1), the Legendre-product expansion
 *     (eq. metoletableform) and eq. coefintable.
 *   - adaptive trees (Sec. 3.5, closing remarks): boxes divided while they
 *     hold more than the leaf cap, U/V/W/X lists by a dual traversal of the
 *     target and source trees, and the point forms on the W- and X-lists:
 *     free-space M2P / P2L (eqs. freespace3dmulexp, melecoeffree) and
 *     reaction M2P / P2L from the F~ and L rows of eq. coefintable, whose
 *     Sommerfeld tables mix the forward and backward
 *     (eq. backwardrecurrence1) recurrences.
 *
 * Readings of places where the printed text is garbled or silent are listed
 * at each use (sigma typos, index order of the translation sums, Gaunt
 * prefactors, the spurious factorial in C^s, the garbled factorial in C~^s).
 *
 * Parity pins: every function here is checked by tests/test_oracle_*.py
 * against closed forms, identities or library routines; see the test files.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

#define ORC_PI 3.14159265358979323846
#define ORC_HMAX 16        /* bits per dimension of the fine cell code       */
#define ORC_MAXDEPTH 12    /* deepest tree level the oracle builds           */
#define ORC_PMAX 20        /* largest expansion order supported              */
#define ORC_NGL 16         /* Gauss-Legendre points per quadrature panel     */
#define ORC_MAXL 8         /* most interfaces                                */

/* ------------------------------------------------------------------------ */
/* factorials and small helpers                                             */
/* ------------------------------------------------------------------------ */

static double g_fact[171];
static double g_gl16_x[ORC_NGL], g_gl16_w[ORC_NGL];
#define ORC_NGAUNT 64
static double g_gl64_x[ORC_NGAUNT], g_gl64_w[ORC_NGAUNT];

void orc_gauss_legendre(int n, double* x, double* w);

#define ORC_GNMAX (2 * ORC_PMAX)
static double g_plm64[ORC_NGAUNT][(ORC_GNMAX + 1) * (ORC_GNMAX + 2) / 2];
void orc_plm(int nmax, double x, double* out);

__attribute__((constructor)) static void orc_init(void)
{
    g_fact[0] = 1.0;
    for (int k = 1; k <= 170; ++k) g_fact[k] = g_fact[k - 1] * (double)k;
    orc_gauss_legendre(ORC_NGL, g_gl16_x, g_gl16_w);
    orc_gauss_legendre(ORC_NGAUNT, g_gl64_x, g_gl64_w);
    for (int k = 0; k < ORC_NGAUNT; ++k) orc_plm(ORC_GNMAX, g_gl64_x[k], g_plm64[k]);
}

static double fact(int n) { return (n < 0 || n > 170) ? NAN : g_fact[n]; }
static double sgn_pow(int k) { return (k % 2 == 0) ? 1.0 : -1.0; } /* (-1)^k */
static int iabs(int k) { return k < 0 ? -k : k; }
static int idx_nm(int n, int m) { return n * n + n + m; } /* m = -n..n */

/* i^k for integer k */
static cplx ipow(int k)
{
    int r = ((k % 4) + 4) % 4;
    if (r == 0) return 1.0;
    if (r == 1) return I;
    if (r == 2) return -1.0;
    return -I;
}

/* ------------------------------------------------------------------------ */
/* Gauss-Legendre nodes on [-1,1] by Newton iteration on P_n                */
/* ------------------------------------------------------------------------ */
void orc_gauss_legendre(int n, double* x, double* w)
{
    for (int i = 0; i < n; ++i) {
        double z = cos(ORC_PI * (i + 0.75) / (n + 0.5));
        double p1 = 0, p2 = 0, dp = 0;
        for (int it = 0; it < 100; ++it) {
            p1 = 1.0;
            p2 = 0.0;
            for (int j = 1; j <= n; ++j) {
                double p3 = p2;
                p2 = p1;
                p1 = ((2.0 * j - 1.0) * z * p2 - (j - 1.0) * p3) / j;
            }
            dp = n * (z * p1 - p2) / (z * z - 1.0);
            double dz = p1 / dp;
            z -= dz;
            if (fabs(dz) < 1e-16) break;
        }
        p1 = 1.0;
        p2 = 0.0;
        for (int j = 1; j <= n; ++j) {
            double p3 = p2;
            p2 = p1;
            p1 = ((2.0 * j - 1.0) * z * p2 - (j - 1.0) * p3) / j;
        }
        dp = n * (z * p1 - p2) / (z * z - 1.0);
        x[i] = z;
        w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

/* ------------------------------------------------------------------------ */
/* Modified spherical Bessel functions (Sec. 3.1: i_n(z) = i^{-n} j_n(iz),  */
/* k_n(z) = -(pi/2) i^n h_n^(1)(iz), so k_0(x) = (pi/2) e^{-x}/x).          */
/* ------------------------------------------------------------------------ */

/* i_n(x) from its power series sum_k x^{n+2k} / (2^k k! (2n+2k+1)!!);
 * all terms are positive, so the sum has no cancellation. */
double orc_bessel_i(int n, double x)
{
    if (x == 0.0) return n == 0 ? 1.0 : 0.0;
    double term = 1.0;
    for (int k = 1; k <= n; ++k) term *= x / (2.0 * k + 1.0);
    double sum = term;
    for (int k = 1; k < 2000; ++k) {
        term *= x * x / (2.0 * k * (2.0 * n + 2.0 * k + 1.0));
        sum += term;
        if (term < 1e-18 * sum) break;
    }
    return sum;
}

/* k_n(x) = (pi/(2x)) e^{-x} sum_{k=0}^n (n+k)! / (k! (n-k)!) (2x)^{-k}. */
double orc_bessel_k(int n, double x)
{
    double s = 0.0;
    for (int k = 0; k <= n; ++k) s += fact(n + k) / (fact(k) * fact(n - k)) * pow(2.0 * x, -k);
    return ORC_PI / (2.0 * x) * exp(-x) * s;
}

/* ------------------------------------------------------------------------ */
/* Normalised associated Legendre functions and spherical harmonics         */
/* (Sec. 3.1): Y_n^m = P^_n^m(cos t) e^{i m p},                             */
/* P^_n^m = sqrt((2n+1)/(4 pi) (n-m)!/(n+m)!) (1-x^2)^{m/2} d^m P_n / dx^m  */
/* for m >= 0, and P^_n^{-m} = (-1)^m P^_n^m, so Y_n^{-m} = (-1)^m conj Y.  */
/* The paper's (-1)^m convention factor cancels in every product used by    */
/* the method (an expansion coefficient always meets its conjugate).        */
/* ------------------------------------------------------------------------ */
static double cnm(int n, int m) { return sqrt((2.0 * n + 1.0) / (4.0 * ORC_PI) * fact(n - m) / fact(n + m)); }

/* out[n(n+1)/2 + m] = P^_n^m(x), 0 <= m <= n <= nmax, |x| <= 1 */
void orc_plm(int nmax, double x, double* out)
{
    double s = sqrt(fmax(0.0, 1.0 - x * x));
    double pmm = 1.0; /* (2m-1)!! s^m */
    for (int m = 0; m <= nmax; ++m) {
        if (m > 0) pmm *= (2.0 * m - 1.0) * s;
        double p0 = pmm, p1 = 0.0;
        out[m * (m + 1) / 2 + m] = cnm(m, m) * p0;
        if (m + 1 <= nmax) {
            p1 = (2.0 * m + 1.0) * x * p0;
            out[(m + 1) * (m + 2) / 2 + m] = cnm(m + 1, m) * p1;
        }
        for (int n = m + 2; n <= nmax; ++n) {
            double pn = ((2.0 * n - 1.0) * x * p1 - (n + m - 1.0) * p0) / (double)(n - m);
            p0 = p1;
            p1 = pn;
            out[n * (n + 1) / 2 + m] = cnm(n, m) * pn;
        }
    }
}

/* Y_n^m at the direction of (vx,vy,vz) for n <= nmax, all m; index n^2+n+m.
 * The zero vector is given theta = phi = 0. */
void orc_ylm(int nmax, double vx, double vy, double vz, double* re, double* im)
{
    double r = sqrt(vx * vx + vy * vy + vz * vz);
    double ct = r > 0 ? vz / r : 1.0;
    double ph = (vx == 0.0 && vy == 0.0) ? 0.0 : atan2(vy, vx);
    double* P = (double*)malloc(sizeof(double) * (nmax + 1) * (nmax + 2) / 2);
    orc_plm(nmax, ct, P);
    for (int n = 0; n <= nmax; ++n)
        for (int m = 0; m <= n; ++m) {
            double v = P[n * (n + 1) / 2 + m];
            re[idx_nm(n, m)] = v * cos(m * ph);
            im[idx_nm(n, m)] = v * sin(m * ph);
            if (m > 0) {
                re[idx_nm(n, -m)] = sgn_pow(m) * v * cos(m * ph);
                im[idx_nm(n, -m)] = -sgn_pow(m) * v * sin(m * ph);
            }
        }
    free(P);
}

static void ylm_c(int nmax, double vx, double vy, double vz, cplx* Y)
{
    int K = (nmax + 1) * (nmax + 1);
    double* re = (double*)malloc(sizeof(double) * 2 * K);
    orc_ylm(nmax, vx, vy, vz, re, re + K);
    for (int k = 0; k < K; ++k) Y[k] = re[k] + I * re[K + k];
    free(re);
}

/* Gaunt integral G = int Y_{n1}^{m1} Y_{n2}^{m2} Y_{n3}^{m3} dOmega (no
 * conjugations, the harmonics above).  The azimuthal integral is 2 pi when
 * m1+m2+m3 = 0 and zero otherwise; the polar integrand is then a polynomial
 * of degree n1+n2+n3 in cos(theta), integrated exactly by 64-point
 * Gauss-Legendre (exact to degree 127). */
double orc_gaunt(int n1, int m1, int n2, int m2, int n3, int m3)
{
    if (m1 + m2 + m3 != 0) return 0.0;
    if (iabs(m1) > n1 || iabs(m2) > n2 || iabs(m3) > n3) return 0.0;
    if (n1 > ORC_GNMAX || n2 > ORC_GNMAX || n3 > ORC_GNMAX || n1 + n2 + n3 > 2 * ORC_NGAUNT - 1) return NAN;
    double f1 = m1 < 0 ? sgn_pow(-m1) : 1.0, f2 = m2 < 0 ? sgn_pow(-m2) : 1.0, f3 = m3 < 0 ? sgn_pow(-m3) : 1.0;
    int i1 = n1 * (n1 + 1) / 2 + iabs(m1), i2 = n2 * (n2 + 1) / 2 + iabs(m2), i3 = n3 * (n3 + 1) / 2 + iabs(m3);
    double s = 0.0;
    for (int k = 0; k < ORC_NGAUNT; ++k) s += g_gl64_w[k] * g_plm64[k][i1] * g_plm64[k][i2] * g_plm64[k][i3];
    return 2.0 * ORC_PI * f1 * f2 * f3 * s;
}

/* ------------------------------------------------------------------------ */
/* Layered medium                                                           */
/* ------------------------------------------------------------------------ */
typedef struct {
    int L;                      /* number of interfaces; layers 0..L      */
    double eps[ORC_MAXL + 1];
    double lam[ORC_MAXL + 1];
    double d[ORC_MAXL];         /* d_0 > d_1 > ... > d_{L-1}              */
} layers_t;

static int layer_of(const layers_t* Ly, double z)
{
    int l = 0;
    for (int k = 0; k < Ly->L; ++k)
        if (Ly->d[k] > z) l = k + 1;
    return l;
}

/* Reaction densities sigma^{ab}_{l lp}(lrho) of the three-layer medium,
 * eqs. densitythreelayer1-3, with these readings of the printed text:
 *  - the closed forms assume d_0 = 0; written here with the middle-layer
 *    thickness D = d_0 - d_1 (cosh(-d_1 t) -> cosh(D t), e^{-d_1 t} -> e^{D t});
 *  - sigma^{11}_{10}: the numerator factor printed lambda_1 lambda_1z is read
 *    eps_1 lambda_1z (matches the transmission conditions);
 *  - sigma^{21}_{11}: the printed '+' in (eps1 l1z + eps0 l0z) is read '-',
 *    which makes it equal to sigma^{12}_{11} as the transmission conditions
 *    require;
 *  - every numerator and kappa are multiplied by 2 e^{-D l1z} so nothing
 *    overflows for large lrho (cosh -> 1+x^2, sinh -> 1-x^2, e^{D l1z} -> 2,
 *    no exponential -> 2x with x = e^{-D l1z}).
 * Returns NAN for an invalid (l, lp, a, b). */
double orc_sigma3(const double* eps, const double* lam, double d0, double d1, int l, int lp, int a, int b,
                  double lrho)
{
    double D = d0 - d1;
    double e0 = eps[0], e1 = eps[1], e2 = eps[2];
    double z0 = sqrt(lam[0] * lam[0] + lrho * lrho);
    double z1 = sqrt(lam[1] * lam[1] + lrho * lrho);
    double z2 = sqrt(lam[2] * lam[2] + lrho * lrho);
    double x = exp(-D * z1);
    double x2 = x * x;
    double kap = e1 * z1 * (e0 * z0 + e2 * z2) * (1.0 + x2) + (e1 * e1 * z1 * z1 + e0 * e2 * z0 * z2) * (1.0 - x2);
    int key = ((l * 3 + lp) * 2 + (a - 1)) * 2 + (b - 1);
#define SKEY(L_, LP_, A_, B_) ((((L_)*3 + (LP_)) * 2 + ((A_)-1)) * 2 + ((B_)-1))
    switch (key) {
    /* source in the top layer */
    case SKEY(0, 0, 1, 1):
        return (e1 * z1 * (e0 * z0 - e2 * z2) * (1.0 + x2) - (e1 * e1 * z1 * z1 - e0 * e2 * z0 * z2) * (1.0 - x2)) /
               (e0 * kap);
    case SKEY(1, 0, 1, 1): return 2.0 * x * e0 * z1 * (e1 * z1 - e2 * z2) / (e0 * kap);
    case SKEY(1, 0, 2, 1): return 2.0 * e0 * z1 * (e1 * z1 + e2 * z2) / (e0 * kap);
    case SKEY(2, 0, 2, 1): return 2.0 * x * 2.0 * e0 * e1 * z1 * z2 / (e0 * kap);
    /* source in the middle layer */
    case SKEY(0, 1, 1, 1): return 2.0 * x * e1 * z0 * (e1 * z1 - e2 * z2) / (e1 * kap);
    case SKEY(0, 1, 1, 2): return 2.0 * e1 * z0 * (e1 * z1 + e2 * z2) / (e1 * kap);
    case SKEY(1, 1, 1, 1): return 2.0 * (e1 * z1 - e2 * z2) * (e1 * z1 + e0 * z0) / (2.0 * e1 * kap);
    case SKEY(1, 1, 1, 2): return 2.0 * x * (e1 * z1 - e2 * z2) * (e1 * z1 - e0 * z0) / (2.0 * e1 * kap);
    case SKEY(1, 1, 2, 1): return 2.0 * x * (e1 * z1 - e2 * z2) * (e1 * z1 - e0 * z0) / (2.0 * e1 * kap);
    case SKEY(1, 1, 2, 2): return 2.0 * (e1 * z1 + e2 * z2) * (e1 * z1 - e0 * z0) / (2.0 * e1 * kap);
    case SKEY(2, 1, 2, 1): return 2.0 * e1 * z2 * (e0 * z0 + e1 * z1) / (e1 * kap);
    case SKEY(2, 1, 2, 2): return 2.0 * x * e1 * z2 * (e1 * z1 - e0 * z0) / (e1 * kap);
    /* source in the bottom layer */
    case SKEY(0, 2, 1, 2): return 2.0 * x * 2.0 * e1 * z1 * e2 * z0 / (e2 * kap);
    case SKEY(1, 2, 2, 2): return 2.0 * x * e2 * z1 * (e1 * z1 - e0 * z0) / (e2 * kap);
    case SKEY(1, 2, 1, 2): return 2.0 * e2 * z1 * (e0 * z0 + e1 * z1) / (e2 * kap);
    case SKEY(2, 2, 2, 2):
        return (e1 * z1 * (e2 * z2 - e0 * z0) * (1.0 + x2) - (e1 * e1 * z1 * z1 - e0 * e2 * z0 * z2) * (1.0 - x2)) /
               (e2 * kap);
    default: return NAN;
    }
#undef SKEY
}

/* Reaction densities of a general stack (Sec. 2.1: eqs. greenfuncomponent,
 * totaldensity; the paper writes sigma out only for three layers) by
 * generalized reflection and transmission coefficients.  For one lrho, with
 * zeta_k = sqrt(lam_k^2 + lrho^2), Y_k = eps_k zeta_k and h_k = d_{k-1} - d_k,
 * the spectral field in layer k is the source term (k = lp)
 * e^{-zeta |z - z'|} / (eps_lp zeta_lp) plus an up-going wave
 * P_k e^{-zeta_k (z - d_k)} and a down-going wave Q_k e^{-zeta_k (d_{k-1} - z)};
 * sigma^{1b}_{l lp} and sigma^{2b}_{l lp} are the coefficients of the source
 * exponentials X_1 = e^{-zeta_lp (z' - d_lp)}, X_2 = e^{-zeta_lp (d_{lp-1} - z')}
 * in zeta_l P_l and zeta_l Q_l.  Continuity of u and eps du/dz at each
 * interface gives, looking down from layer k at d_k (a down-going wave of unit
 * amplitude there), the reflected amplitude
 *   Rd_k = (Y_k - W) / (Y_k + W),  W = Y_{k+1} (1 - g) / (1 + g),
 *   g = e^{-2 zeta_{k+1} h_{k+1}} Rd_{k+1}   (Rd_L = 0, g = 0 into layer L),
 * and the transmitted down-going amplitude Td_k = (1 + Rd_k) / (1 + g) in
 * layer k+1; looking up at d_{k-1} the same with the layers above (Ru_0 = 0).
 * In the source layer P = Rd (x1 + Q E), Q = Ru (x2 + P E), E = e^{-zeta h},
 * x_b = X_b / (eps zeta); the waves leaving it are carried through the
 * layers below (down-going amplitude at the top of each, times Td) and above
 * (up-going amplitude at the bottom of each, times Tu).  Every factor is at
 * most 1 in modulus, so nothing overflows at large lrho.  Returns NAN for an
 * invalid (l, lp, a, b). */
static int comp_valid(const layers_t* Ly, int l, int lp, int a, int b);

static double sigma_stack(const layers_t* Ly, int l, int lp, int a, int b, double lrho)
{
    const int L = Ly->L;
    double zt[ORC_MAXL + 1], Y[ORC_MAXL + 1], E[ORC_MAXL + 1];
    double Rd[ORC_MAXL + 1], Td[ORC_MAXL + 1], Ru[ORC_MAXL + 1], Tu[ORC_MAXL + 1];
    if (!comp_valid(Ly, l, lp, a, b)) return NAN;
    for (int k = 0; k <= L; ++k) {
        zt[k] = sqrt(Ly->lam[k] * Ly->lam[k] + lrho * lrho);
        Y[k] = Ly->eps[k] * zt[k];
        /* attenuation across layer k (unbounded top and bottom layers: 0) */
        E[k] = (k == 0 || k == L) ? 0.0 : exp(-zt[k] * (Ly->d[k - 1] - Ly->d[k]));
    }
    Rd[L] = 0.0;
    Td[L] = 0.0;
    for (int k = L - 1; k >= 0; --k) {
        double g = E[k + 1] * E[k + 1] * Rd[k + 1];
        double W = Y[k + 1] * (1.0 - g) / (1.0 + g);
        Rd[k] = (Y[k] - W) / (Y[k] + W);
        Td[k] = (1.0 + Rd[k]) / (1.0 + g);
    }
    Ru[0] = 0.0;
    Tu[0] = 0.0;
    for (int k = 1; k <= L; ++k) {
        double g = E[k - 1] * E[k - 1] * Ru[k - 1];
        double W = Y[k - 1] * (1.0 - g) / (1.0 + g);
        Ru[k] = (Y[k] - W) / (Y[k] + W);
        Tu[k] = (1.0 + Ru[k]) / (1.0 + g);
    }
    /* unit source exponential of side b */
    double x1 = (b == 1) ? 1.0 / Y[lp] : 0.0, x2 = (b == 2) ? 1.0 / Y[lp] : 0.0;
    double Es = E[lp], den = 1.0 - Rd[lp] * Ru[lp] * Es * Es;
    double P = (Rd[lp] * x1 + Rd[lp] * Ru[lp] * Es * x2) / den;
    double Q = (Ru[lp] * x2 + Ru[lp] * Rd[lp] * Es * x1) / den;
    double Pl = 0.0, Ql = 0.0;
    if (l == lp) {
        Pl = P;
        Ql = Q;
    } else if (l > lp) {
        /* down-going amplitude at the top of layer lp+1, then layer by layer */
        double t = Td[lp] * (x1 + Q * Es);
        for (int k = lp + 1; k < l; ++k) t = Td[k] * t * E[k];
        Ql = t;
        Pl = Rd[l] * t * E[l];
    } else {
        /* up-going amplitude at the bottom of layer lp-1, then layer by layer */
        double u = Tu[lp] * (x2 + P * Es);
        for (int k = lp - 1; k > l; --k) u = Tu[k] * u * E[k];
        Pl = u;
        Ql = Ru[l] * u * E[l];
    }
    return zt[l] * (a == 1 ? Pl : Ql);
}


static double sigma(const layers_t* Ly, int l, int lp, int a, int b, double lrho)
{
    /* three layers: the paper's closed forms; any other stack: the recursion */
    if (Ly->L == 2) return orc_sigma3(Ly->eps, Ly->lam, Ly->d[0], Ly->d[1], l, lp, a, b, lrho);
    return sigma_stack(Ly, l, lp, a, b, lrho);
}

/* A reaction component (l, lp, a, b) exists iff a=1 -> l<L, a=2 -> l>0,
 * b=1 -> lp<L, b=2 -> lp>0 (eqs. reactioncomponent, decomposition2). */
static int comp_valid(const layers_t* Ly, int l, int lp, int a, int b)
{
    if (a == 1 && l >= Ly->L) return 0;
    if (a == 2 && l <= 0) return 0;
    if (b == 1 && lp >= Ly->L) return 0;
    if (b == 2 && lp <= 0) return 0;
    return 1;
}

/* distance of a target at height z from the interface its component uses,
 * tau_1(z) = z - d_l, tau_2(z) = d_{l-1} - z (eq. zexponential) */
static double tau_t(const layers_t* Ly, int l, int a, double z) { return a == 1 ? z - Ly->d[l] : Ly->d[l - 1] - z; }
/* tau'_1(z') = z' - d_lp, tau'_2(z') = d_{lp-1} - z' */
static double tau_s(const layers_t* Ly, int lp, int b, double zp) { return b == 1 ? zp - Ly->d[lp] : Ly->d[lp - 1] - zp; }

/* ------------------------------------------------------------------------ */
/* Composite Gauss-Legendre quadrature on [0, X_max] for the Sommerfeld-    */
/* type integrals of Sec. 3.5.  The integrands behave like                  */
/* lrho^npow J_m(lrho rho) e^{-c lrho} times smooth factors; X_max is where */
/* the envelope lrho^npow e^{-c lrho} has fallen to tol of its peak.  Panel */
/* widths resolve half a Bessel period (pi/rho), the exponential (4/c), the */
/* branch points of sqrt(lambda^2 + lrho^2) near the origin (lam_min) and   */
/* the poles of sigma at |lrho| ~ pi/(2 D) (D = thickest finite layer).     */
/* ------------------------------------------------------------------------ */
typedef struct {
    int n;
    double* x;
    double* w;
} nodes_t;

static double xmax_envelope(double c, int npow, double tol)
{
    double lt = log(tol);
    if (npow == 0) return -lt / c;
    double xs = npow / c;
    double step = 1.0 / c;
    double hi = xs + step;
    while (npow * log(hi / xs) - c * (hi - xs) > lt) {
        step *= 2.0;
        hi = xs + step;
    }
    double lo = xs;
    for (int it = 0; it < 200; ++it) {
        double mid = 0.5 * (lo + hi);
        if (npow * log(mid / xs) - c * (mid - xs) > lt) lo = mid;
        else hi = mid;
    }
    return hi;
}

static void build_nodes(nodes_t* nd, double rho, double c, int npow, double lam_min, double dmax, double tol)
{
    double X = xmax_envelope(c, npow, tol);
    double w0 = lam_min;
    if (dmax > 0 && ORC_PI / (2.0 * dmax) < w0) w0 = ORC_PI / (2.0 * dmax);
    int cap = 1024;
    nd->x = (double*)malloc(sizeof(double) * cap * ORC_NGL);
    nd->w = (double*)malloc(sizeof(double) * cap * ORC_NGL);
    nd->n = 0;
    double a = 0.0;
    int np = 0;
    while (a < X) {
        double w = a > w0 ? a : w0;
        if (4.0 / c < w) w = 4.0 / c;
        if (rho > 0 && ORC_PI / rho < w) w = ORC_PI / rho;
        if (np == cap) {
            cap *= 2;
            nd->x = (double*)realloc(nd->x, sizeof(double) * cap * ORC_NGL);
            nd->w = (double*)realloc(nd->w, sizeof(double) * cap * ORC_NGL);
        }
        for (int k = 0; k < ORC_NGL; ++k) {
            nd->x[nd->n] = a + 0.5 * w * (g_gl16_x[k] + 1.0);
            nd->w[nd->n] = 0.5 * w * g_gl16_w[k];
            nd->n++;
        }
        a += w;
        np++;
    }
}

static void free_nodes(nodes_t* nd)
{
    free(nd->x);
    free(nd->w);
}

static double layers_lam_min(const layers_t* Ly)
{
    double m = Ly->lam[0];
    for (int k = 1; k <= Ly->L; ++k) m = fmin(m, Ly->lam[k]);
    return m;
}

static double layers_dmax(const layers_t* Ly)
{
    double m = 0.0;
    for (int k = 1; k < Ly->L; ++k) m = fmax(m, Ly->d[k - 1] - Ly->d[k]);
    return m;
}

#define ORC_TOL 1e-16

/* ------------------------------------------------------------------------ */
/* Green's function components                                              */
/* ------------------------------------------------------------------------ */

/* free space part e^{-lambda r} / (4 pi eps r) (eq. layeredGreensfun) */
static double green_free(double lam, double eps, double r) { return exp(-lam * r) / (4.0 * ORC_PI * eps * r); }

/* Reaction component u^{ab}_{l lp}(r, r') (eq. generalcomponents) with the
 * angular integral done by the J_n identity (Sec. 3.5):
 *   u = (1/4pi) int_0^inf lrho J_0(lrho rho) e^{-l_z tau_a(z) - l'_z tau'_b(z')}
 *                         sigma^{ab}_{l lp}(lrho) / l_z dlrho. */
double orc_reaction_u(const double* eps, const double* lam, const double* d, int L, int l, int lp, int a, int b,
                      double x, double y, double z, double xp, double yp, double zp)
{
    layers_t Ly;
    if (L < 1 || L > ORC_MAXL) return NAN;
    Ly.L = L;
    for (int k = 0; k <= L; ++k) {
        Ly.eps[k] = eps[k];
        Ly.lam[k] = lam[k];
    }
    for (int k = 0; k < L; ++k) Ly.d[k] = d[k];
    if (!comp_valid(&Ly, l, lp, a, b)) return NAN;
    double rho = hypot(x - xp, y - yp);
    double tt = tau_t(&Ly, l, a, z), ts = tau_s(&Ly, lp, b, zp);
    nodes_t nd;
    build_nodes(&nd, rho, tt + ts, 1, layers_lam_min(&Ly), layers_dmax(&Ly), ORC_TOL);
    double s = 0.0;
    for (int k = 0; k < nd.n; ++k) {
        double t = nd.x[k];
        double lz = sqrt(lam[l] * lam[l] + t * t), lzp = sqrt(lam[lp] * lam[lp] + t * t);
        s += nd.w[k] * t * jn(0, t * rho) * exp(-lz * tt - lzp * ts) * sigma(&Ly, l, lp, a, b, t) / lz;
    }
    free_nodes(&nd);
    return s / (4.0 * ORC_PI);
}

/* ------------------------------------------------------------------------ */
/* Direct O(N^2) summation (eqs. potential1 / totalinteraction):             */
/*   Phi_l(r_i) = sum_{j != i, j in layer l} Q_j e^{-lam_l r}/(4 pi eps_l r)  */
/*              + sum_{all j} Q_j sum_{valid (a,b)} u^{ab}_{l l_j}(r_i, r_j)  */
/* The free part excludes j = i; the reaction part includes it (the image   */
/* of a charge is never at the charge).                                     */
/* ------------------------------------------------------------------------ */
static int fill_layers(layers_t* Ly, int nlayers, const double* eps, const double* lam, const double* d)
{
    if (nlayers < 1 || nlayers > ORC_MAXL + 1) return -1;
    Ly->L = nlayers - 1;
    for (int k = 0; k < nlayers; ++k) {
        Ly->eps[k] = eps[k];
        Ly->lam[k] = lam[k];
    }
    for (int k = 0; k < Ly->L; ++k) Ly->d[k] = d[k];
    return 0;
}

/* sigma^{ab}_{l lp}(lrho) of a stack of nlayers layers by the generalized
 * reflection recursion (any number of layers, three included). */
double orc_sigma_stack(int nlayers, const double* eps, const double* lam, const double* d, int l, int lp, int a,
                       int b, double lrho)
{
    layers_t Ly;
    if (fill_layers(&Ly, nlayers, eps, lam, d) || Ly.L < 1) return NAN;
    return sigma_stack(&Ly, l, lp, a, b, lrho);
}

int orc_direct_sum(int nlayers, const double* eps, const double* lam, const double* d, int64_t n, const double* x,
                   const double* y, const double* z, const double* q, int64_t nt, const int64_t* tidx, double* phi,
                   int nthreads)
{
    layers_t Ly;
    if (fill_layers(&Ly, nlayers, eps, lam, d)) return -1;
    int* lay = (int*)malloc(sizeof(int) * n);
    for (int64_t j = 0; j < n; ++j) lay[j] = layer_of(&Ly, z[j]);
    double lmin = layers_lam_min(&Ly), dmax = layers_dmax(&Ly);
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (int64_t ti = 0; ti < nt; ++ti) {
        int64_t i = tidx ? tidx[ti] : ti;
        int l = lay[i];
        double acc = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            int lp = lay[j];
            double rho = hypot(x[i] - x[j], y[i] - y[j]);
            if (lp == l && j != i) {
                double r = sqrt(rho * rho + (z[i] - z[j]) * (z[i] - z[j]));
                acc += q[j] * green_free(lam[l], eps[l], r);
            }
            if (Ly.L == 0) continue;
            /* all valid reaction components of this (target, source) pair */
            double tt[4], ts[4], cmin = INFINITY;
            int ab[4][2], nc = 0;
            for (int a = 1; a <= 2; ++a)
                for (int b = 1; b <= 2; ++b)
                    if (comp_valid(&Ly, l, lp, a, b)) {
                        ab[nc][0] = a;
                        ab[nc][1] = b;
                        tt[nc] = tau_t(&Ly, l, a, z[i]);
                        ts[nc] = tau_s(&Ly, lp, b, z[j]);
                        cmin = fmin(cmin, tt[nc] + ts[nc]);
                        nc++;
                    }
            nodes_t nd;
            build_nodes(&nd, rho, cmin, 1, lmin, dmax, ORC_TOL);
            double s = 0.0;
            for (int k = 0; k < nd.n; ++k) {
                double t = nd.x[k];
                double lz = sqrt(lam[l] * lam[l] + t * t), lzp = sqrt(lam[lp] * lam[lp] + t * t);
                double g = 0.0;
                for (int c = 0; c < nc; ++c)
                    g += exp(-lz * tt[c] - lzp * ts[c]) * sigma(&Ly, l, lp, ab[c][0], ab[c][1], t);
                s += nd.w[k] * t * jn(0, t * rho) * g / lz;
            }
            free_nodes(&nd);
            acc += q[j] * s / (4.0 * ORC_PI);
        }
        phi[ti] = acc;
    }
    free(lay);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Free-space translation operators (Theorems 3.1-3.3).                     */
/* With the harmonics above, for |r| < |b|:                                 */
/*   i_n Y_n^m(r+b) = sum_{nu,mu} Sh_{n nu}^{m mu}(b) i_nu Y_nu^mu(r),      */
/*   k_n Y_n^m(r+b) = sum_{nu,mu} S_{n nu}^{m mu}(b) i_nu Y_nu^mu(r),       */
/*   Sh = 4 pi sum_q          i_q(lam b) Y_q^{m-mu}(b^) G_q,                */
/*   S  = 4 pi sum_q (-1)^{n+q} k_q(lam b) Y_q^{m-mu}(b^) G_q,              */
/*   G_q = int Y_n^m conj(Y_nu^mu) conj(Y_q^{m-mu}) dOmega.                 */
/* The printed prefactors of the separation matrices (4pi(-1)^{nu-n+m+q}    */
/* and 2 pi^2 (-1)^{m+nu+1}) hold only under an unstated Gaunt convention;  */
/* these forms are pinned by the addition-theorem tests instead.            */
/* Translations (eqs. metole, metome; the sums run over nu, mu):            */
/*   M2L: L_nm  = sum S_{nu n}^{mu m}(rc_t - rc_s) M_{nu mu}                */
/*   M2M: M~_nm = sum conj(Sh_{n nu}^{m mu}(rc_s - rc~_s)) M_{nu mu}        */
/*   L2L: L~_nm = sum Sh_{nu n}^{mu m}(rc~_t - rc_t) L_{nu mu}              */
/* ------------------------------------------------------------------------ */
typedef struct {
    int p, K;
    double* G; /* G[(row*K + col)*(2p+1) + q] = G_q(n,m; nu,mu), row = idx(n,m), col = idx(nu,mu) */
} gaunt_tab_t;

static void gaunt_tab_init(gaunt_tab_t* T, int p)
{
    T->p = p;
    T->K = (p + 1) * (p + 1);
    int nq = 2 * p + 1;
    T->G = (double*)calloc((size_t)T->K * T->K * nq, sizeof(double));
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (int n = 0; n <= p; ++n)
        for (int m = -n; m <= n; ++m)
            for (int nu = 0; nu <= p; ++nu)
                for (int mu = -nu; mu <= nu; ++mu)
                    for (int q = 0; q <= 2 * p; ++q) {
                        if (q < iabs(n - nu) || q > n + nu || (n + nu + q) % 2) continue;
                        if (iabs(m - mu) > q) continue;
                        /* conj(Y_nu^mu) = (-1)^mu Y_nu^{-mu}; conj(Y_q^{m-mu}) = (-1)^{m-mu} Y_q^{mu-m} */
                        double g = sgn_pow(iabs(m)) * orc_gaunt(n, m, nu, -mu, q, mu - m);
                        T->G[((size_t)idx_nm(n, m) * T->K + idx_nm(nu, mu)) * nq + q] = g;
                    }
}

static void gaunt_tab_free(gaunt_tab_t* T) { free(T->G); }

/* Dense operator A (K x K complex, row-major, A[row*K+col]) for one of:
 *   kind 0: M2M, A_{(n,m),(nu,mu)} = conj(Sh_{n nu}^{m mu}(b))
 *   kind 1: L2L, A_{(n,m),(nu,mu)} = Sh_{nu n}^{mu m}(b)
 *   kind 2: M2L, A_{(n,m),(nu,mu)} = S_{nu n}^{mu m}(b)                    */
static void free_operator(const gaunt_tab_t* T, int kind, double lam, double bx, double by, double bz, cplx* A)
{
    int p = T->p, K = T->K, nq = 2 * p + 1;
    double b = sqrt(bx * bx + by * by + bz * bz);
    int K2 = (2 * p + 1) * (2 * p + 1);
    cplx* Yb = (cplx*)malloc(sizeof(cplx) * K2);
    ylm_c(2 * p, bx, by, bz, Yb);
    double rad[2 * ORC_PMAX + 1];
    for (int q = 0; q <= 2 * p; ++q) rad[q] = (kind == 2) ? orc_bessel_k(q, lam * b) : orc_bessel_i(q, lam * b);
    for (int n = 0; n <= p; ++n)
        for (int m = -n; m <= n; ++m)
            for (int nu = 0; nu <= p; ++nu)
                for (int mu = -nu; mu <= nu; ++mu) {
                    /* (N,Mm) is the first index pair of Sh/S, (V,U) the second */
                    int N, Mm, V, U;
                    if (kind == 0) { N = n; Mm = m; V = nu; U = mu; }
                    else { N = nu; Mm = mu; V = n; U = m; }
                    cplx s = 0.0;
                    const double* G = &T->G[((size_t)idx_nm(N, Mm) * K + idx_nm(V, U)) * nq];
                    for (int q = iabs(N - V); q <= N + V; q += 2) {
                        if (iabs(Mm - U) > q || G[q] == 0.0) continue;
                        double f = (kind == 2) ? sgn_pow(N + q) : 1.0;
                        s += f * rad[q] * Yb[idx_nm(q, Mm - U)] * G[q];
                    }
                    s *= 4.0 * ORC_PI;
                    A[(size_t)idx_nm(n, m) * K + idx_nm(nu, mu)] = (kind == 0) ? conj(s) : s;
                }
    free(Yb);
}

static void apply_op(int K, const cplx* A, const cplx* x, cplx* y /* += */)
{
    for (int r = 0; r < K; ++r) {
        cplx s = 0.0;
        for (int c = 0; c < K; ++c) s += A[(size_t)r * K + c] * x[c];
        y[r] += s;
    }
}

/* P2M (eq. melecoeffree): M_nm += q 4 pi i_n(lam |r'-c|) conj(Y_n^m(r'-c)) */
static void p2m_one(int p, double lam, double q, double dx, double dy, double dz, cplx* M)
{
    int K = (p + 1) * (p + 1);
    cplx* Y = (cplx*)malloc(sizeof(cplx) * K);
    ylm_c(p, dx, dy, dz, Y);
    double r = sqrt(dx * dx + dy * dy + dz * dz);
    for (int n = 0; n <= p; ++n) {
        double in = orc_bessel_i(n, lam * r);
        for (int m = -n; m <= n; ++m) M[idx_nm(n, m)] += q * 4.0 * ORC_PI * in * conj(Y[idx_nm(n, m)]);
    }
    free(Y);
}

/* L2P (eq. freespace3dlocexp / lelayerimage): sum_nm L_nm i_n(lam|r-c|) Y_n^m(r-c) */
static double l2p_one(int p, double lam, const cplx* L, double dx, double dy, double dz)
{
    int K = (p + 1) * (p + 1);
    cplx* Y = (cplx*)malloc(sizeof(cplx) * K);
    ylm_c(p, dx, dy, dz, Y);
    double r = sqrt(dx * dx + dy * dy + dz * dz);
    cplx s = 0.0;
    for (int n = 0; n <= p; ++n) {
        double in = orc_bessel_i(n, lam * r);
        for (int m = -n; m <= n; ++m) s += L[idx_nm(n, m)] * in * Y[idx_nm(n, m)];
    }
    free(Y);
    return creal(s);
}

/* ------------------------------------------------------------------------ */
/* Reaction M2L operators (Sec. 3.5).                                       */
/* ------------------------------------------------------------------------ */

/* a^j_{nm} (m >= 0): coefficient of x^{2j-n-m} in c_nm d^m P_n/dx^m */
static double a_coef(int n, int m, int j)
{
    if (2 * j - n - m < 0) return 0.0;
    return sgn_pow(n - j) * fact(2 * j) * cnm(n, m) / (pow(2.0, n) * fact(j) * fact(n - j) * fact(2 * j - n - m));
}

/* b^s_{nm} = sum_{j=q}^{n} (-1)^s a^j_{nm} (j-r)! / (s! (j-r-s)!),
 * r = floor((n+m)/2), q = max(ceil((n+m)/2), s+r)  (m >= 0) */
static double b_coef(int n, int m, int s)
{
    int r = (n + m) / 2;
    int q = (n + m + 1) / 2;
    if (s + r > q) q = s + r;
    double acc = 0.0;
    for (int j = q; j <= n; ++j) acc += sgn_pow(s) * a_coef(n, m, j) * fact(j - r) / (fact(s) * fact(j - r - s));
    return acc;
}

static double tau_sign(int m) { return m >= 0 ? 1.0 : sgn_pow(-m); }

/* C^s_{n nu m mu} of the Legendre-product expansion
 *   P^_n^m(l_z/l) P^_nu^mu(l'_z/l') = sum_s C^s lrho^{|m|+|mu|+2s} (l/l_z)^i (l'/l'_z)^j,
 * with the printed extra factor (|m|+|mu|+2s)! dropped: with it the
 * expansion does not reproduce the product (pinned by a test). */
static cplx c_coef(int n, int nu, int m, int mu, int s, double lam, double lamp)
{
    int am = iabs(m), amu = iabs(mu);
    int r = (n + am) / 2, rp = (nu + amu) / 2;
    int t0 = s - nu + rp;
    if (t0 < 0) t0 = 0;
    int t1 = s < n - r ? s : n - r;
    cplx acc = 0.0;
    for (int t = t0; t <= t1; ++t) {
        cplx den = ipow(am + 2 * t) * pow(lam, am + 2 * t) * ipow(amu + 2 * (s - t)) * pow(lamp, amu + 2 * (s - t));
        acc += tau_sign(m) * tau_sign(mu) * b_coef(n, am, t) * b_coef(nu, amu, s - t) / den;
    }
    return acc;
}

/* C~^s = sqrt((|m|-m+|mu|+mu+2s+1)! (|m|+m+|mu|-mu+2s+1)!) C^s
 * (the printed "\pounds!" is read as a factorial sign). */
static cplx ct_coef(int n, int nu, int m, int mu, int s, double lam, double lamp)
{
    int am = iabs(m), amu = iabs(mu);
    return sqrt(fact(am - m + amu + mu + 2 * s + 1) * fact(am + m + amu - mu + 2 * s + 1)) *
           c_coef(n, nu, m, mu, s, lam, lamp);
}

typedef struct {
    layers_t Ly;
    int l, lp, a, b;
} rcomp_t;

/* Z^+(z,z') = e^{-l_z (z - d_l) - l'_z (d_l - z')}           (a = 1)
 * Z^-(z,z') = e^{-l_z (d_{l-1} - z) - l'_z (z' - d_{l-1})}   (a = 2)     (eq. zexpkernel) */
static double zkern(const rcomp_t* C, double lz, double lzp, double zt, double zs)
{
    const layers_t* Ly = &C->Ly;
    if (C->a == 1) return exp(-lz * (zt - Ly->d[C->l]) - lzp * (Ly->d[C->l] - zs));
    return exp(-lz * (Ly->d[C->l - 1] - zt) - lzp * (zs - Ly->d[C->l - 1]));
}

static double zsep(const rcomp_t* C, double zt, double zs)
{
    const layers_t* Ly = &C->Ly;
    if (C->a == 1) return (zt - Ly->d[C->l]) + (Ly->d[C->l] - zs);
    return (Ly->d[C->l - 1] - zt) + (zs - Ly->d[C->l - 1]);
}

static double a_n(int n) { return sqrt((double)n * (n + 1.0)); }

/* Scaled Sommerfeld integrals S^n Sc_{n m, ij}(rho, zt, zs) (eq. M2Ltable and
 * its scaled form) for 0 <= m <= n <= nmax, i, j in {0,1}:
 *   tab[((i*2+j)*(nmax+1) + n)*(nmax+1) + m].
 * Initial values m = 0 (n = 0..nmax) and m = 1 (n = 1..nmax) by composite
 * Gauss-Legendre quadrature; the rest by the forward recurrence
 * (eq. recurrence1):
 *   S^n Sc_{n,m+1} = (2m / a_{n+m}) (S/rho) S^{n-1} Sc_{n-1,m}
 *                    - (a_{n-m}/a_{n+m}) S^n Sc_{n,m-1},  n >= m+1,
 * with a_k = sqrt(k(k+1)).  For rho = 0, Sc_{n,m>0} = 0.  The recurrence is
 * used only where the stability bound 2m/a_{n+m} < rho/S holds, as it does
 * for every M2L pair of the tree (rho = 0 or rho >= S).  Returns 1 if that
 * bound was violated somewhere. */
static int sommerfeld_table(const rcomp_t* C, double rho, double zt, double zs, double S, int nmax, double* tab)
{
    const layers_t* Ly = &C->Ly;
    int N1 = nmax + 1;
    double lt = Ly->lam[C->l], ls = Ly->lam[C->lp];
    memset(tab, 0, sizeof(double) * 4 * N1 * N1);
    nodes_t nd;
    build_nodes(&nd, rho, zsep(C, zt, zs), nmax, layers_lam_min(Ly), layers_dmax(Ly), ORC_TOL);
    for (int k = 0; k < nd.n; ++k) {
        double t = nd.x[k];
        double lz = sqrt(lt * lt + t * t), lzp = sqrt(ls * ls + t * t);
        double base = nd.w[k] * zkern(C, lz, lzp, zt, zs) * sigma(Ly, C->l, C->lp, C->a, C->b, t) / lz;
        double j0 = jn(0, t * rho), j1 = jn(1, t * rho);
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 2; ++j) {
                double f = base * (i ? lt / lz : 1.0) * (j ? ls / lzp : 1.0);
                double* T = tab + (size_t)(i * 2 + j) * N1 * N1;
                double pw = 1.0; /* (t S)^n */
                for (int n = 0; n <= nmax; ++n) {
                    T[n * N1 + 0] += f * pw * j0 / fact(n); /* sqrt(n! n!) = n! */
                    if (n >= 1) T[n * N1 + 1] += f * pw * j1 / sqrt(fact(n + 1) * fact(n - 1));
                    pw *= t * S;
                }
            }
    }
    free_nodes(&nd);
    int unstable = 0;
    for (int ij = 0; ij < 4; ++ij) {
        double* T = tab + (size_t)ij * N1 * N1;
        if (rho == 0.0) {
            for (int n = 0; n <= nmax; ++n)
                for (int m = 1; m <= n; ++m) T[n * N1 + m] = 0.0;
            continue;
        }
        for (int m = 1; m < nmax; ++m)
            for (int n = m + 1; n <= nmax; ++n) {
                if (2.0 * m / a_n(n + m) >= rho / S) unstable = 1;
                T[n * N1 + m + 1] = 2.0 * m / a_n(n + m) * (S / rho) * T[(n - 1) * N1 + m] -
                                    a_n(n - m) / a_n(n + m) * T[n * N1 + m - 1];
            }
    }
    return unstable;
}

/* Table of C~^s for all (n,m,nu,mu,s) of one component. */
typedef struct {
    int p, smax;
    cplx* v; /* [(idx(n,m)*K + idx(nu,mu))*(smax+1) + s] */
} ctab_t;

static void ctab_init(ctab_t* T, int p, double lam, double lamp)
{
    int K = (p + 1) * (p + 1);
    T->p = p;
    T->smax = 2 * p + 2;
    T->v = (cplx*)calloc((size_t)K * K * (T->smax + 1), sizeof(cplx));
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (int n = 0; n <= p; ++n)
        for (int m = -n; m <= n; ++m)
            for (int nu = 0; nu <= p; ++nu)
                for (int mu = -nu; mu <= nu; ++mu) {
                    int r = (n + iabs(m)) / 2, rp = (nu + iabs(mu)) / 2;
                    for (int s = 0; s <= (n - r) + (nu - rp); ++s)
                        T->v[((size_t)idx_nm(n, m) * K + idx_nm(nu, mu)) * (T->smax + 1) + s] =
                            ct_coef(n, nu, m, mu, s, lam, lamp);
                }
}

/* I_{nm,nu mu} (eq. uniformintegral) assembled from the scaled table by
 * eq. metoletableform: I = i^{mu-m} sum_s C~^s Sc_{|m|+|mu|+2s+1, mu-m, ij},
 * i = (n+|m|) mod 2, j = (nu+|mu|) mod 2, Sc_{N,-M} = (-1)^M Sc_{N,M}. */
static cplx assemble_I(const ctab_t* CT, const double* tab, int nmax, double S, int n, int m, int nu, int mu)
{
    int K = (CT->p + 1) * (CT->p + 1);
    int N1 = nmax + 1;
    int i = (n + iabs(m)) % 2, j = (nu + iabs(mu)) % 2;
    int r = (n + iabs(m)) / 2, rp = (nu + iabs(mu)) / 2;
    const double* T = tab + (size_t)(i * 2 + j) * N1 * N1;
    const cplx* cv = &CT->v[((size_t)idx_nm(n, m) * K + idx_nm(nu, mu)) * (CT->smax + 1)];
    cplx acc = 0.0;
    for (int s = 0; s <= (n - r) + (nu - rp); ++s) {
        int Nn = iabs(m) + iabs(mu) + 2 * s + 1;
        int M = mu - m;
        double sc = T[Nn * N1 + iabs(M)] * (M < 0 ? sgn_pow(-M) : 1.0) / pow(S, Nn);
        acc += cv[s] * sc;
    }
    return ipow(mu - m) * acc;
}

/* Reaction M2L operator (eq. coefintable):
 *   T^{1b}_{nm,nu mu} = (-1)^n          e^{i(mu-m) phi_st} I^{1b}_{nm,nu mu}(rho_st, zc_t, zc_s)
 *   T^{2b}_{nm,nu mu} = (-1)^{nu+m+mu}  e^{i(mu-m) phi_st} I^{2b}_{nm,nu mu}(rho_st, zc_t, zc_s)
 * given the phi-independent part I (K x K). */
static void reaction_T_from_I(const rcomp_t* C, int p, const cplx* Imat, double phi, cplx* A)
{
    int K = (p + 1) * (p + 1);
    for (int n = 0; n <= p; ++n)
        for (int m = -n; m <= n; ++m)
            for (int nu = 0; nu <= p; ++nu)
                for (int mu = -nu; mu <= nu; ++mu) {
                    double sg = (C->a == 1) ? sgn_pow(n) : sgn_pow(nu + iabs(m) + iabs(mu));
                    int r = idx_nm(n, m), c = idx_nm(nu, mu);
                    A[(size_t)r * K + c] = sg * cexp(I * (mu - m) * phi) * Imat[(size_t)r * K + c];
                }
}

static void reaction_I_matrix(const rcomp_t* C, const ctab_t* CT, int p, double rho, double zt, double zs, double S,
                              cplx* Imat, int* unstable)
{
    int nmax = 2 * p + 3, K = (p + 1) * (p + 1);
    double* tab = (double*)malloc(sizeof(double) * 4 * (nmax + 1) * (nmax + 1));
    int u = sommerfeld_table(C, rho, zt, zs, S, nmax, tab);
    if (unstable) *unstable |= u;
    for (int n = 0; n <= p; ++n)
        for (int m = -n; m <= n; ++m)
            for (int nu = 0; nu <= p; ++nu)
                for (int mu = -nu; mu <= nu; ++mu)
                    Imat[(size_t)idx_nm(n, m) * K + idx_nm(nu, mu)] = assemble_I(CT, tab, nmax, S, n, m, nu, mu);
    free(tab);
}

/* Test-only cross-check: I_{nm,nu mu} by direct quadrature of eq.
 * uniformintegral with Q = P^_n^m(l_z/l) P^_nu^mu(l'_z/l') evaluated as the
 * associated Legendre function beyond [-1,1] on the branch
 * (1-w^2)^{1/2} = -i sqrt(w^2-1) (Prop. 3.2 and eq. branch). */
static cplx plm_big(int n, int m, double w, double lrho_over_lam)
{
    int am = iabs(m);
    /* d^am P_n / dw^am by the three-term recurrence in n */
    double p0 = 1.0;
    for (int k = 1; k <= am; ++k) p0 *= (2.0 * k - 1.0);
    double val;
    if (n == am) val = p0;
    else {
        double p1 = (2.0 * am + 1.0) * w * p0;
        for (int k = am + 2; k <= n; ++k) {
            double pk = ((2.0 * k - 1.0) * w * p1 - (k + am - 1.0) * p0) / (double)(k - am);
            p0 = p1;
            p1 = pk;
        }
        val = p1;
    }
    cplx root = cpow(-I * lrho_over_lam, am);
    return tau_sign(m) * cnm(n, am) * root * val;
}

static cplx reaction_I_direct_one(const rcomp_t* C, int n, int m, int nu, int mu, double rho, double zt, double zs,
                                  double* absint)
{
    const layers_t* Ly = &C->Ly;
    double lt = Ly->lam[C->l], ls = Ly->lam[C->lp];
    nodes_t nd;
    build_nodes(&nd, rho, zsep(C, zt, zs), n + nu + 2, layers_lam_min(Ly), layers_dmax(Ly), ORC_TOL);
    cplx acc = 0.0;
    for (int k = 0; k < nd.n; ++k) {
        double t = nd.x[k];
        double lz = sqrt(lt * lt + t * t), lzp = sqrt(ls * ls + t * t);
        cplx Q = plm_big(n, m, lz / lt, t / lt) * plm_big(nu, mu, lzp / ls, t / ls);
        double f = nd.w[k] * t * jn(mu - m, t * rho) * zkern(C, lz, lzp, zt, zs) *
                   sigma(Ly, C->l, C->lp, C->a, C->b, t) / lz;
        acc += f * Q;
        if (absint) *absint += fabs(f) * cabs(Q);
    }
    free_nodes(&nd);
    return ipow(mu - m) * acc;
}

/* ------------------------------------------------------------------------ */
/* Point forms of the expansions, used by adaptive trees (Sec. 3.5, closing */
/* remarks on adaptive trees): a multipole expansion evaluated at a target  */
/* directly (M2P, W-list) and a local expansion formed from a source        */
/* directly (P2L, X-list).                                                  */
/* ------------------------------------------------------------------------ */

/* free space, eq. freespace3dmulexp: sum_nm M_nm k_n(lam r_s) Y_n^m(r - c) */
static double m2p_free_one(int p, double lam, const cplx* M, double dx, double dy, double dz)
{
    int K = (p + 1) * (p + 1);
    cplx* Y = (cplx*)malloc(sizeof(cplx) * K);
    ylm_c(p, dx, dy, dz, Y);
    double r = sqrt(dx * dx + dy * dy + dz * dz);
    cplx s = 0.0;
    for (int n = 0; n <= p; ++n) {
        double kn = orc_bessel_k(n, lam * r);
        for (int m = -n; m <= n; ++m) s += M[idx_nm(n, m)] * kn * Y[idx_nm(n, m)];
    }
    free(Y);
    return creal(s);
}

/* free space, eq. melecoeffree with the conjugate reading of Y_n^{-m}:
 * L_nm += q 4 pi k_n(lam r'_t) conj(Y_n^m(r' - c)) */
static void p2l_free_one(int p, double lam, double q, double dx, double dy, double dz, cplx* L)
{
    int K = (p + 1) * (p + 1);
    cplx* Y = (cplx*)malloc(sizeof(cplx) * K);
    ylm_c(p, dx, dy, dz, Y);
    double r = sqrt(dx * dx + dy * dy + dz * dz);
    for (int n = 0; n <= p; ++n) {
        double kn = orc_bessel_k(n, lam * r);
        for (int m = -n; m <= n; ++m) L[idx_nm(n, m)] += q * 4.0 * ORC_PI * kn * conj(Y[idx_nm(n, m)]);
    }
    free(Y);
}

/* Scaled Sommerfeld table S^n Sc_{nm,ij}(rho, zt, zs), 0 <= m <= n <= nmax, of
 * a point and a box centre (layout as sommerfeld_table).  Here rho can take
 * any value from 0 up, also below the box side S, so each entry is reached
 * by the recurrence that is stable for it:
 *   - initial values by quadrature: m = 0 (n = 0..nmax), m = 1 (n = 1..nmax)
 *     and the whole row n = nmax;
 *   - the forward recurrence (eq. recurrence1) for S^n Sc_{n,m+1} wherever
 *     its bound 2m/a_{n+m} < rho/S holds, in increasing m;
 *   - the backward recurrence (eq. backwardrecurrence1)
 *       S^{n-1} Sc_{n-1,m} = (a_{n+m}/(2m)) (rho/S) S^n Sc_{n,m+1}
 *                          + (a_{n-m}/(2m)) (rho/S) S^n Sc_{n,m-1}
 *     for every other entry, row by row down from n = nmax.
 * rho = 0: Sc_{n,m>0} = 0. */
static void sommerfeld_table_pt(const rcomp_t* C, double rho, double zt, double zs, double S, int nmax, double* tab)
{
    const layers_t* Ly = &C->Ly;
    int N1 = nmax + 1;
    double lt = Ly->lam[C->l], ls = Ly->lam[C->lp];
    memset(tab, 0, sizeof(double) * 4 * N1 * N1);
    char* done = (char*)calloc((size_t)N1 * N1, 1);
    nodes_t nd;
    build_nodes(&nd, rho, zsep(C, zt, zs), nmax, layers_lam_min(Ly), layers_dmax(Ly), ORC_TOL);
    for (int k = 0; k < nd.n; ++k) {
        double t = nd.x[k];
        double lz = sqrt(lt * lt + t * t), lzp = sqrt(ls * ls + t * t);
        double base = nd.w[k] * zkern(C, lz, lzp, zt, zs) * sigma(Ly, C->l, C->lp, C->a, C->b, t) / lz;
        double j0 = jn(0, t * rho), j1 = jn(1, t * rho);
        double pwN = pow(t * S, nmax);
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 2; ++j) {
                double f = base * (i ? lt / lz : 1.0) * (j ? ls / lzp : 1.0);
                double* T = tab + (size_t)(i * 2 + j) * N1 * N1;
                double pw = 1.0; /* (t S)^n */
                for (int n = 0; n <= nmax; ++n) {
                    T[n * N1 + 0] += f * pw * j0 / fact(n);
                    if (n >= 1) T[n * N1 + 1] += f * pw * j1 / sqrt(fact(n + 1) * fact(n - 1));
                    pw *= t * S;
                }
                if (rho > 0.0)
                    for (int m = 2; m <= nmax; ++m)
                        T[nmax * N1 + m] += f * pwN * jn(m, t * rho) / sqrt(fact(nmax + m) * fact(nmax - m));
            }
    }
    free_nodes(&nd);
    for (int n = 0; n <= nmax; ++n) {
        done[n * N1 + 0] = 1;
        if (n >= 1) done[n * N1 + 1] = 1;
    }
    if (rho == 0.0) {
        free(done);
        return; /* the m >= 1 entries stay 0 (J_m(0) = 0) */
    }
    for (int m = 0; m <= nmax; ++m) done[nmax * N1 + m] = 1;
    double x = rho / S;
    /* forward, increasing m */
    for (int m = 1; m < nmax; ++m)
        for (int n = m + 1; n < nmax; ++n) {
            if (!(2.0 * m / a_n(n + m) < x)) continue;
            if (!done[(n - 1) * N1 + m] || !done[n * N1 + m - 1]) continue;
            for (int ij = 0; ij < 4; ++ij) {
                double* T = tab + (size_t)ij * N1 * N1;
                T[n * N1 + m + 1] =
                    2.0 * m / a_n(n + m) / x * T[(n - 1) * N1 + m] - a_n(n - m) / a_n(n + m) * T[n * N1 + m - 1];
            }
            done[n * N1 + m + 1] = 1;
        }
    /* backward, down from the row nmax */
    for (int n = nmax; n >= 2; --n)
        for (int m = 1; m <= n - 1; ++m) {
            if (done[(n - 1) * N1 + m]) continue;
            for (int ij = 0; ij < 4; ++ij) {
                double* T = tab + (size_t)ij * N1 * N1;
                T[(n - 1) * N1 + m] = a_n(n + m) / (2.0 * m) * x * T[n * N1 + m + 1] +
                                      a_n(n - m) / (2.0 * m) * x * T[n * N1 + m - 1];
            }
            done[(n - 1) * N1 + m] = 1;
        }
    free(done);
}

/* Reaction ME evaluated at a target r (eq. melayerupgoingimage with the F~
 * rows of eq. coefintable):
 *   u~(r) = sum_{nu mu} M_{nu mu} F~_{nu mu}(r, c),
 *   F~^{1b}_{nu mu} = e^{i mu phi} I^{1b}_{00,nu mu}(rho, z, z_c) / sqrt(4 pi),
 *   F~^{2b}_{nu mu} = (-1)^{nu+mu} e^{i mu phi} I^{2b}_{00,nu mu}(rho, z, z_c) / sqrt(4 pi),
 * (rho, phi) the polar coordinates of (x - c_x, y - c_y).  I_{00,nu mu} needs
 * the table up to n = p + 2; S is the source box side. */
static double m2p_react_one(const rcomp_t* C, const ctab_t* CT, int p, const cplx* M, double x, double y, double z,
                            const double* c, double S)
{
    int nmax = p + 2;
    double* tab = (double*)malloc(sizeof(double) * 4 * (nmax + 1) * (nmax + 1));
    double rho = hypot(x - c[0], y - c[1]);
    double phi = rho > 0.0 ? atan2(y - c[1], x - c[0]) : 0.0;
    sommerfeld_table_pt(C, rho, z, c[2], S, nmax, tab);
    cplx s = 0.0;
    for (int nu = 0; nu <= p; ++nu)
        for (int mu = -nu; mu <= nu; ++mu) {
            double sg = (C->a == 1) ? 1.0 : sgn_pow(nu + iabs(mu));
            s += sg * cexp(I * mu * phi) * assemble_I(CT, tab, nmax, S, 0, 0, nu, mu) * M[idx_nm(nu, mu)];
        }
    free(tab);
    return creal(s) / sqrt(4.0 * ORC_PI);
}

/* Reaction LE about a target centre c from one image source at (x, y, z)
 * with charge q (the L rows of eq. coefintable):
 *   L^{1b}_nm += q (-1)^n sqrt(4 pi) e^{-i m phi} I^{1b}_{nm,00}(rho, z_c, z'),
 *   L^{2b}_nm += q (-1)^m sqrt(4 pi) e^{-i m phi} I^{2b}_{nm,00}(rho, z_c, z'),
 * (rho, phi) the polar coordinates of (c_x - x, c_y - y).  The 2b line is
 * printed with the heights in the other order; every I takes the target-side
 * height first, as in its definition and in the T rows. */
static void p2l_react_one(const rcomp_t* C, const ctab_t* CT, int p, double q, double x, double y, double z,
                          const double* c, double S, cplx* L)
{
    int nmax = p + 2;
    double* tab = (double*)malloc(sizeof(double) * 4 * (nmax + 1) * (nmax + 1));
    double rho = hypot(c[0] - x, c[1] - y);
    double phi = rho > 0.0 ? atan2(c[1] - y, c[0] - x) : 0.0;
    sommerfeld_table_pt(C, rho, c[2], z, S, nmax, tab);
    for (int n = 0; n <= p; ++n)
        for (int m = -n; m <= n; ++m) {
            double sg = (C->a == 1) ? sgn_pow(n) : sgn_pow(iabs(m));
            L[idx_nm(n, m)] +=
                q * sg * sqrt(4.0 * ORC_PI) * cexp(-I * m * phi) * assemble_I(CT, tab, nmax, S, n, m, 0, 0);
        }
    free(tab);
}

/* ------------------------------------------------------------------------ */
/* Tree (shared definition with the GPU library, written separately):      */
/*  root cube (cx,cy,cz) +- R; fine cell of a point                         */
/*    t = ((x - cx) + R) / (2R),  ix = clamp(floor(t * 2^16), 0, 2^16-1),   */
/*  level-l cell = fine cell >> (16 - l).  Uniform trees: depth H = the    */
/*  smallest l with N_src <= cap * #non-empty source boxes(l) and the same  */
/*  for targets (H <= 12).  Adaptive trees: each point set divides a box    */
/*  while it holds more than cap points (down to level 12), a reaction      */
/*  component's sets also while a box is wider than its nearest point's    */
/*  distance from the interface (see divide_box).  V-list at                */
/*  level l >= 2: existing source boxes that are children of the            */
/*  neighbours of the target's parent and not adjacent to the target;       */
/*  U-, W- and X-lists by the dual traversal (traverse() below); on uniform */
/*  trees the U-list is the adjacent or equal boxes at level H.             */
/* ------------------------------------------------------------------------ */
static uint32_t fine_cell(double x, double c, double R)
{
    double t = ((x - c) + R) / (2.0 * R);
    double f = floor(t * 65536.0);
    if (f < 0) f = 0;
    if (f > 65535) f = 65535;
    return (uint32_t)f;
}

static uint64_t morton_key(uint32_t ix, uint32_t iy, uint32_t iz, int level)
{
    uint64_t k = 0;
    for (int bit = level - 1; bit >= 0; --bit) {
        k = (k << 3) | (uint64_t)(((ix >> bit) & 1u) << 2) | (uint64_t)(((iy >> bit) & 1u) << 1) |
            (uint64_t)((iz >> bit) & 1u);
    }
    return k;
}

typedef struct {
    int n;
    uint32_t *cx, *cy, *cz; /* fine cells */
} cells_t;

typedef struct {
    int nb;
    uint64_t* key;          /* sorted distinct box keys at this level */
    int* start;             /* for the leaf level: point list offsets (nb+1) */
} boxlev_t;

static int cmp_u64(const void* a, const void* b)
{
    uint64_t x = *(const uint64_t*)a, y = *(const uint64_t*)b;
    return x < y ? -1 : (x > y ? 1 : 0);
}

static void distinct_boxes(const cells_t* C, int level, boxlev_t* B)
{
    uint64_t* k = (uint64_t*)malloc(sizeof(uint64_t) * (C->n > 0 ? C->n : 1));
    int sh = ORC_HMAX - level;
    for (int i = 0; i < C->n; ++i) k[i] = morton_key(C->cx[i] >> sh, C->cy[i] >> sh, C->cz[i] >> sh, level);
    qsort(k, C->n, sizeof(uint64_t), cmp_u64);
    int nb = 0;
    for (int i = 0; i < C->n; ++i)
        if (i == 0 || k[i] != k[i - 1]) k[nb++] = k[i];
    B->nb = nb;
    B->key = k;
    B->start = NULL;
}

static int find_box(const boxlev_t* B, uint64_t key)
{
    int lo = 0, hi = B->nb - 1;
    while (lo <= hi) {
        int mid = (lo + hi) / 2;
        if (B->key[mid] == key) return mid;
        if (B->key[mid] < key) lo = mid + 1;
        else hi = mid - 1;
    }
    return -1;
}

static void key_coords(uint64_t key, int level, int* ix, int* iy, int* iz)
{
    int x = 0, y = 0, z = 0;
    for (int bit = 0; bit < level; ++bit) {
        z |= (int)((key >> (3 * bit)) & 1u) << bit;
        y |= (int)((key >> (3 * bit + 1)) & 1u) << bit;
        x |= (int)((key >> (3 * bit + 2)) & 1u) << bit;
    }
    *ix = x;
    *iy = y;
    *iz = z;
}

/* ------------------------------------------------------------------------ */
/* One FMM (Algorithm 1 for a reaction component, the classic Yukawa FMM   */
/* for a free-space component) on the tree above: uniform, or adaptive.    */
/* ------------------------------------------------------------------------ */
typedef struct {
    int kind; /* 0 free, 1 reaction */
    rcomp_t rc;
    double lam_s, lam_t, far_factor; /* far_factor multiplies L2P */
    double eps_t;
} fmmspec_t;

typedef struct {
    int depth;
    int nleaf_t, nleaf_s;
    long long m2l_pairs, p2p_pairs, w_pairs, x_pairs;
    int unstable;
} fmmstat_t;

static int sort_by_key_cmp_idx(const void* a, const void* b)
{
    const uint64_t* x = (const uint64_t*)a;
    const uint64_t* y = (const uint64_t*)b;
    if (x[0] != y[0]) return x[0] < y[0] ? -1 : 1;
    return x[1] < y[1] ? -1 : (x[1] > y[1] ? 1 : 0);
}

/* Points sorted by (fine key, index): order[k] and key[k] = the fine-cell
 * Morton key (level ORC_HMAX) of the k-th point. */
static void sort_points(const cells_t* C, int* order, uint64_t* key)
{
    uint64_t* kv = (uint64_t*)malloc(sizeof(uint64_t) * 2 * (C->n > 0 ? C->n : 1));
    for (int i = 0; i < C->n; ++i) {
        kv[2 * i] = morton_key(C->cx[i], C->cy[i], C->cz[i], ORC_HMAX);
        kv[2 * i + 1] = (uint64_t)i;
    }
    qsort(kv, C->n, 2 * sizeof(uint64_t), sort_by_key_cmp_idx);
    for (int i = 0; i < C->n; ++i) {
        key[i] = kv[2 * i];
        order[i] = (int)kv[2 * i + 1];
    }
    free(kv);
}

/* Adaptive rule: a box (above ORC_MAXDEPTH) is divided while it holds more
 * than cap points; with sep != 0 (the sets of a reaction component, whose
 * root is halved by the interface plane: fine z cells 32767 | 32768) a box
 * is also divided while it is wider than the distance of its nearest point
 * from the plane, both in fine cells, down to 3 levels below the level at
 * which the occupancy rule stopped.  lv[i] = leaf level of point i (key,
 * order: the sorted points). */
static uint32_t plane_dist(uint64_t key)
{
    uint32_t cz = 0;
    for (int bit = 0; bit < ORC_HMAX; ++bit) cz |= (uint32_t)((key >> (3 * bit)) & 1u) << bit;
    return cz >= 32768u ? cz - 32768u : 32767u - cz;
}

static void divide_box(int k0, int k1, int l, int locc, const int* order, const uint64_t* key, int cap, int sep,
                       int* lv)
{
    int split = 0;
    if (l < ORC_MAXDEPTH) {
        if (k1 - k0 > cap) {
            split = 1;
            locc = -1;
        } else {
            if (locc < 0) locc = l;
            if (sep && l < locc + 3) {
                uint32_t dmin = 0xffffffffu;
                for (int k = k0; k < k1; ++k) {
                    uint32_t d = plane_dist(key[k]);
                    if (d < dmin) dmin = d;
                }
                split = (1u << (ORC_HMAX - l)) > dmin;
            }
        }
    }
    if (!split) {
        for (int k = k0; k < k1; ++k) lv[order[k]] = l;
        return;
    }
    int sh = 3 * (ORC_HMAX - l - 1);
    for (int a = k0; a < k1;) {
        int b = a + 1;
        while (b < k1 && (key[b] >> sh) == (key[a] >> sh)) ++b;
        divide_box(a, b, l + 1, locc, order, key, cap, sep, lv);
        a = b;
    }
}

static void leaf_levels(int n, const int* order, const uint64_t* key, int cap, int sep, int* lv)
{
    if (n > 0) divide_box(0, n, 0, -1, order, key, cap, sep, lv);
}

/* distinct level-l cells of the points whose leaf level is at least l */
static void level_boxes(const cells_t* C, const int* lv, int level, boxlev_t* B)
{
    uint64_t* k = (uint64_t*)malloc(sizeof(uint64_t) * (C->n > 0 ? C->n : 1));
    int sh = ORC_HMAX - level, m = 0;
    for (int i = 0; i < C->n; ++i)
        if (lv[i] >= level) k[m++] = morton_key(C->cx[i] >> sh, C->cy[i] >> sh, C->cz[i] >> sh, level);
    qsort(k, m, sizeof(uint64_t), cmp_u64);
    int nb = 0;
    for (int i = 0; i < m; ++i)
        if (i == 0 || k[i] != k[i - 1]) k[nb++] = k[i];
    B->nb = nb;
    B->key = k;
    B->start = NULL;
}

static int box_child(const boxlev_t* B, int H, int l, int b, int o)
{
    if (l >= H) return -1;
    return find_box(&B[l + 1], (B[l].key[b] << 3) | (uint64_t)o);
}

static int box_is_leaf(const boxlev_t* B, int H, int l, int b)
{
    for (int o = 0; o < 8; ++o)
        if (box_child(B, H, l, b, o) >= 0) return 0;
    return 1;
}

/* the closed cubes of box (la, A[la].key[ia]) and box (lb, B[lb].key[ib])
 * touch or overlap */
static int boxes_adjacent(const boxlev_t* A, int la, int ia, const boxlev_t* B, int lb, int ib)
{
    int a[3], c[3];
    key_coords(A[la].key[ia], la, &a[0], &a[1], &a[2]);
    key_coords(B[lb].key[ib], lb, &c[0], &c[1], &c[2]);
    int L = la > lb ? la : lb;
    for (int k = 0; k < 3; ++k) {
        long alo = (long)a[k] << (L - la), ahi = ((long)(a[k] + 1) << (L - la)) - 1;
        long clo = (long)c[k] << (L - lb), chi = ((long)(c[k] + 1) << (L - lb)) - 1;
        if (alo > chi + 1 || clo > ahi + 1) return 0;
    }
    return 1;
}

/* box pairs (target level, target box, source level, source box) */
typedef struct {
    int n, cap;
    int* v;
} plist_t;

static void plist_push(plist_t* P, int tl, int tb, int sl, int sb)
{
    if (P->n == P->cap) {
        P->cap = P->cap ? 2 * P->cap : 256;
        P->v = (int*)realloc(P->v, sizeof(int) * 4 * P->cap);
    }
    int* e = P->v + 4 * P->n++;
    e[0] = tl;
    e[1] = tb;
    e[2] = sl;
    e[3] = sb;
}

/* Dual traversal of the target and source trees from a pair of adjacent
 * boxes (levels below 2 count as adjacent: they carry no expansions).  Two
 * leaves: U-list (direct).  A target leaf and a source box with children:
 * the children that are not adjacent to the leaf go to its W-list (their
 * multipole expansions are evaluated at its targets, M2P), the others are
 * traversed further.  A source leaf and a target box with children:
 * symmetrically the X-list (local expansions formed from the leaf's sources,
 * P2L).  Two boxes with children (same level): child pairs that are not
 * adjacent are the V-list (M2L, listed level by level from the box sets), the
 * others are traversed further. */
static void traverse(const boxlev_t* TB, const boxlev_t* SB, int H, int tl, int tb, int sl, int sb, plist_t* U,
                     plist_t* W, plist_t* X)
{
    int tleaf = box_is_leaf(TB, H, tl, tb), sleaf = box_is_leaf(SB, H, sl, sb);
    if (tleaf && sleaf) {
        plist_push(U, tl, tb, sl, sb);
        return;
    }
    if (tleaf) {
        for (int o = 0; o < 8; ++o) {
            int c = box_child(SB, H, sl, sb, o);
            if (c < 0) continue;
            if (sl + 1 < 2 || boxes_adjacent(TB, tl, tb, SB, sl + 1, c)) traverse(TB, SB, H, tl, tb, sl + 1, c, U, W, X);
            else plist_push(W, tl, tb, sl + 1, c);
        }
        return;
    }
    if (sleaf) {
        for (int o = 0; o < 8; ++o) {
            int c = box_child(TB, H, tl, tb, o);
            if (c < 0) continue;
            if (tl + 1 < 2 || boxes_adjacent(TB, tl + 1, c, SB, sl, sb)) traverse(TB, SB, H, tl + 1, c, sl, sb, U, W, X);
            else plist_push(X, tl + 1, c, sl, sb);
        }
        return;
    }
    for (int ot = 0; ot < 8; ++ot) {
        int tc = box_child(TB, H, tl, tb, ot);
        if (tc < 0) continue;
        for (int os = 0; os < 8; ++os) {
            int sc = box_child(SB, H, sl, sb, os);
            if (sc < 0) continue;
            if (tl + 1 < 2 || boxes_adjacent(TB, tl + 1, tc, SB, sl + 1, sc))
                traverse(TB, SB, H, tl + 1, tc, sl + 1, sc, U, W, X);
        }
    }
}

/* first and one-past-last sorted point of box (l, k) */
static void box_range(int n, const uint64_t* key, int l, uint64_t k, int* lo, int* hi)
{
    int sh = 3 * (ORC_HMAX - l);
    uint64_t a = k << sh, b = (k + 1) << sh;
    int x = 0, y = n;
    while (x < y) {
        int m = (x + y) / 2;
        if (key[m] < a) x = m + 1;
        else y = m;
    }
    *lo = x;
    y = n;
    while (x < y) {
        int m = (x + y) / 2;
        if (key[m] < b) x = m + 1;
        else y = m;
    }
    *hi = x;
}

/* CSR of a pair list by (level, box) of its first pair of fields: the
 * entries of target box (l, b) are idx[ptr[off[l] + b] .. ptr[off[l] + b + 1]),
 * in list order. */
static void plist_csr(const plist_t* P, const boxlev_t* TB, int H, int* off, int** ptr, int** idx)
{
    int tot = 0;
    for (int l = 0; l <= H; ++l) {
        off[l] = tot;
        tot += TB[l].nb;
    }
    *ptr = (int*)calloc((size_t)tot + 1, sizeof(int));
    *idx = (int*)malloc(sizeof(int) * (P->n > 0 ? P->n : 1));
    for (int k = 0; k < P->n; ++k) (*ptr)[off[P->v[4 * k]] + P->v[4 * k + 1] + 1]++;
    for (int k = 0; k < tot; ++k) (*ptr)[k + 1] += (*ptr)[k];
    int* fill = (int*)malloc(sizeof(int) * (tot + 1));
    memcpy(fill, *ptr, sizeof(int) * (tot + 1));
    for (int k = 0; k < P->n; ++k) (*idx)[fill[off[P->v[4 * k]] + P->v[4 * k + 1]]++] = k;
    free(fill);
}

static void box_center(double cx, double cy, double cz, double R, int level, int ix, int iy, int iz, double* c)
{
    double h = 2.0 * R / (double)(1 << level);
    c[0] = (cx - R) + (ix + 0.5) * h;
    c[1] = (cy - R) + (iy + 0.5) * h;
    c[2] = (cz - R) + (iz + 0.5) * h;
}

static void key_center(double cx, double cy, double cz, double R, int level, uint64_t key, double* c)
{
    int ix, iy, iz;
    key_coords(key, level, &ix, &iy, &iz);
    box_center(cx, cy, cz, R, level, ix, iy, iz, c);
}

/* direct part of one target from the sources [k0, k1) of the sorted order
 * (free: the Green's function without the self term; reaction: u~^{ab} by
 * quadrature of I_00, Algorithm 1's last step) */
static double near_sum(const fmmspec_t* F, int i, const double* tx, const double* ty, const double* tz,
                       const int64_t* tid, int k0, int k1, const int* sorder, const double* sx, const double* sy,
                       const double* sz, const double* sq, const int64_t* sid, long long* npp)
{
    const layers_t* Ly = &F->rc.Ly;
    double lmin = layers_lam_min(Ly), dmax = layers_dmax(Ly);
    double acc = 0.0;
    for (int ks = k0; ks < k1; ++ks) {
        int j = sorder[ks];
        if (F->kind == 0) {
            if (sid[j] == tid[i]) continue;
            double r = sqrt((tx[i] - sx[j]) * (tx[i] - sx[j]) + (ty[i] - sy[j]) * (ty[i] - sy[j]) +
                            (tz[i] - sz[j]) * (tz[i] - sz[j]));
            acc += sq[j] * green_free(F->lam_t, F->eps_t, r);
        } else {
            /* u~^{ab}(r, r'_ab) = I_00 with Q_00 = 1/(4 pi) (Algorithm 1, last step) */
            const rcomp_t* C = &F->rc;
            double rho = hypot(tx[i] - sx[j], ty[i] - sy[j]);
            double lt = Ly->lam[C->l], ls = Ly->lam[C->lp];
            nodes_t nd;
            build_nodes(&nd, rho, zsep(C, tz[i], sz[j]), 1, lmin, dmax, ORC_TOL);
            double s = 0.0;
            for (int k = 0; k < nd.n; ++k) {
                double t = nd.x[k];
                double lz = sqrt(lt * lt + t * t), lzp = sqrt(ls * ls + t * t);
                s += nd.w[k] * t * jn(0, t * rho) * zkern(C, lz, lzp, tz[i], sz[j]) *
                     sigma(Ly, C->l, C->lp, C->a, C->b, t) / lz;
            }
            free_nodes(&nd);
            acc += sq[j] * s / (4.0 * ORC_PI);
        }
        (*npp)++;
    }
    return acc;
}

/* pre_s, pre_t: fine cells of the sources and targets (computed here from the
 * coordinates and the root cube when NULL); Hfix >= 0 imposes the depth of a
 * uniform tree; adaptive = 1 builds the adaptive trees instead (leaf rule
 * above, separately for sources and targets; a reaction component's sets
 * with the separation rule) with W- and X-lists, adaptive = 2 the adaptive
 * trees by occupancy alone. */
static int run_fmm(const fmmspec_t* F, int p, int cap, int adaptive, int ns, const double* sx, const double* sy,
                   const double* sz, const double* sq, const int64_t* sid, int nt, const double* tx,
                   const double* ty, const double* tz, const int64_t* tid, double cx, double cy, double cz, double R,
                   const cells_t* pre_s, const cells_t* pre_t, int Hfix,
                   const gaunt_tab_t* GT, const ctab_t* CT, double* phi, fmmstat_t* st)
{
    int K = (p + 1) * (p + 1);
    memset(phi, 0, sizeof(double) * nt);
    memset(st, 0, sizeof(*st));
    if (nt == 0 || ns == 0) return 0;
    cells_t Cs, Ct;
    Cs.n = ns;
    Ct.n = nt;
    Cs.cx = (uint32_t*)malloc(sizeof(uint32_t) * 3 * ns);
    Cs.cy = Cs.cx + ns;
    Cs.cz = Cs.cy + ns;
    Ct.cx = (uint32_t*)malloc(sizeof(uint32_t) * 3 * nt);
    Ct.cy = Ct.cx + nt;
    Ct.cz = Ct.cy + nt;
    for (int i = 0; i < ns; ++i) {
        Cs.cx[i] = pre_s ? pre_s->cx[i] : fine_cell(sx[i], cx, R);
        Cs.cy[i] = pre_s ? pre_s->cy[i] : fine_cell(sy[i], cy, R);
        Cs.cz[i] = pre_s ? pre_s->cz[i] : fine_cell(sz[i], cz, R);
    }
    for (int i = 0; i < nt; ++i) {
        Ct.cx[i] = pre_t ? pre_t->cx[i] : fine_cell(tx[i], cx, R);
        Ct.cy[i] = pre_t ? pre_t->cy[i] : fine_cell(ty[i], cy, R);
        Ct.cz[i] = pre_t ? pre_t->cz[i] : fine_cell(tz[i], cz, R);
    }
    int* sorder = (int*)malloc(sizeof(int) * ns);
    int* torder = (int*)malloc(sizeof(int) * nt);
    uint64_t* skey = (uint64_t*)malloc(sizeof(uint64_t) * ns);
    uint64_t* tkey = (uint64_t*)malloc(sizeof(uint64_t) * nt);
    sort_points(&Cs, sorder, skey);
    sort_points(&Ct, torder, tkey);
    /* leaf level of every point */
    int* slv = (int*)malloc(sizeof(int) * ns);
    int* tlv = (int*)malloc(sizeof(int) * nt);
    int H = -1;
    if (adaptive) {
        leaf_levels(ns, sorder, skey, cap, adaptive == 1 && F->kind == 1, slv);
        leaf_levels(nt, torder, tkey, cap, adaptive == 1 && F->kind == 1, tlv);
        for (int i = 0; i < ns; ++i) H = slv[i] > H ? slv[i] : H;
        for (int i = 0; i < nt; ++i) H = tlv[i] > H ? tlv[i] : H;
    } else {
        for (int l = 0; l <= ORC_MAXDEPTH && H < 0; ++l) {
            boxlev_t a, b;
            distinct_boxes(&Cs, l, &a);
            distinct_boxes(&Ct, l, &b);
            if (Hfix >= 0 ? l == Hfix : ((long long)ns <= (long long)cap * a.nb && (long long)nt <= (long long)cap * b.nb))
                H = l;
            free(a.key);
            free(b.key);
        }
        if (H < 0) H = ORC_MAXDEPTH;
        for (int i = 0; i < ns; ++i) slv[i] = H;
        for (int i = 0; i < nt; ++i) tlv[i] = H;
    }
    st->depth = H;
    boxlev_t SB[ORC_MAXDEPTH + 1], TB[ORC_MAXDEPTH + 1];
    for (int l = 0; l <= H; ++l) {
        level_boxes(&Cs, slv, l, &SB[l]);
        level_boxes(&Ct, tlv, l, &TB[l]);
    }
    /* leaves (level, box) of each tree, by level then Morton order */
    int *sleaf = (int*)malloc(sizeof(int) * 2 * ns), *tleaf = (int*)malloc(sizeof(int) * 2 * nt);
    int nsl = 0, ntl = 0;
    for (int l = 0; l <= H; ++l) {
        for (int b = 0; b < SB[l].nb; ++b)
            if (box_is_leaf(SB, H, l, b)) {
                sleaf[2 * nsl] = l;
                sleaf[2 * nsl++ + 1] = b;
            }
        for (int b = 0; b < TB[l].nb; ++b)
            if (box_is_leaf(TB, H, l, b)) {
                tleaf[2 * ntl] = l;
                tleaf[2 * ntl++ + 1] = b;
            }
    }
    st->nleaf_s = nsl;
    st->nleaf_t = ntl;
    /* U-, W- and X-lists */
    plist_t U = {0, 0, NULL}, W = {0, 0, NULL}, X = {0, 0, NULL};
    traverse(TB, SB, H, 0, 0, 0, 0, &U, &W, &X);
    st->w_pairs = W.n;
    st->x_pairs = X.n;
    int toff[ORC_MAXDEPTH + 1];
    int *uptr, *uidx, *wptr, *widx, *xptr, *xidx;
    plist_csr(&U, TB, H, toff, &uptr, &uidx);
    plist_csr(&W, TB, H, toff, &wptr, &widx);
    plist_csr(&X, TB, H, toff, &xptr, &xidx);

    /* ---------------- far field (levels >= 2) ---------------- */
    if (H >= 2) {
        cplx* ME[ORC_MAXDEPTH + 1];
        cplx* LE[ORC_MAXDEPTH + 1];
        for (int l = 0; l <= H; ++l) {
            ME[l] = (l >= 2) ? (cplx*)calloc((size_t)SB[l].nb * K, sizeof(cplx)) : NULL;
            LE[l] = (l >= 2) ? (cplx*)calloc((size_t)TB[l].nb * K, sizeof(cplx)) : NULL;
        }
        /* P2M at the leaves (eq. melecoeffree / melayerupgoingimage) */
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 4)
#endif
        for (int e = 0; e < nsl; ++e) {
            int l = sleaf[2 * e], b = sleaf[2 * e + 1];
            if (l < 2) continue;
            double c[3];
            int k0, k1;
            key_center(cx, cy, cz, R, l, SB[l].key[b], c);
            box_range(ns, skey, l, SB[l].key[b], &k0, &k1);
            for (int k = k0; k < k1; ++k) {
                int j = sorder[k];
                p2m_one(p, F->lam_s, sq[j], sx[j] - c[0], sy[j] - c[1], sz[j] - c[2], &ME[l][(size_t)b * K]);
            }
        }
        /* M2M, levels H-1 .. 2 (eq. metome) */
        cplx* Aop = (cplx*)malloc(sizeof(cplx) * (size_t)K * K * 8);
        for (int l = H - 1; l >= 2; --l) {
            double hc = 2.0 * R / (double)(1 << (l + 1));
            for (int o = 0; o < 8; ++o) {
                /* child octant o = (ox,oy,oz) bits; b = c_child - c_parent */
                int ox = (o >> 2) & 1, oy = (o >> 1) & 1, oz = o & 1;
                free_operator(GT, 0, F->lam_s, (ox - 0.5) * hc, (oy - 0.5) * hc, (oz - 0.5) * hc,
                              &Aop[(size_t)o * K * K]);
            }
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 4)
#endif
            for (int b = 0; b < SB[l].nb; ++b) {
                for (int o = 0; o < 8; ++o) {
                    int c = find_box(&SB[l + 1], (SB[l].key[b] << 3) | (uint64_t)o);
                    if (c < 0) continue;
                    apply_op(K, &Aop[(size_t)o * K * K], &ME[l + 1][(size_t)c * K], &ME[l][(size_t)b * K]);
                }
            }
        }
        /* downward pass: L2L from the parent, the V-list M2L, the X-list P2L */
        for (int l = 2; l <= H; ++l) {
            double h = 2.0 * R / (double)(1 << l);
            if (l >= 3) {
                for (int o = 0; o < 8; ++o) {
                    int ox = (o >> 2) & 1, oy = (o >> 1) & 1, oz = o & 1;
                    /* b = c~_t (child) - c_t (parent) */
                    free_operator(GT, 1, F->lam_t, (ox - 0.5) * h, (oy - 0.5) * h, (oz - 0.5) * h,
                                  &Aop[(size_t)o * K * K]);
                }
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 4)
#endif
                for (int b = 0; b < TB[l].nb; ++b) {
                    int pb = find_box(&TB[l - 1], TB[l].key[b] >> 3);
                    int o = (int)(TB[l].key[b] & 7u);
                    apply_op(K, &Aop[(size_t)o * K * K], &LE[l - 1][(size_t)pb * K], &LE[l][(size_t)b * K]);
                }
            }
            /* V-list M2L.  Pass 1 lists the pairs of this level; pass 2
             * builds each distinct operator once (free: per offset; reaction:
             * the phi-independent part per (dx^2+dy^2, target z-row, source
             * z-row), then the phase per (dx, dy)); pass 3 applies them. */
            int nside = 1 << l;
            int nkeys = (F->kind == 1) ? 49 * nside * nside : 343;
            int nikeys = (F->kind == 1) ? 19 * nside * nside : 0;
            int cap_p = 1024, np_ = 0;
            int* pt = (int*)malloc(sizeof(int) * cap_p);
            int* ps = (int*)malloc(sizeof(int) * cap_p);
            int* pk = (int*)malloc(sizeof(int) * cap_p);
            int* tfirst = (int*)malloc(sizeof(int) * (TB[l].nb + 1));
            double* krep = (double*)malloc(sizeof(double) * 6 * nkeys); /* representative centres */
            char* kused = (char*)calloc((size_t)nkeys, 1);
            char* iused = (char*)calloc((size_t)(nikeys > 0 ? nikeys : 1), 1);
            for (int b = 0; b < TB[l].nb; ++b) {
                tfirst[b] = np_;
                int tx_, ty_, tz_;
                key_coords(TB[l].key[b], l, &tx_, &ty_, &tz_);
                double ct[3];
                box_center(cx, cy, cz, R, l, tx_, ty_, tz_, ct);
                int px = tx_ >> 1, py = ty_ >> 1, pz = tz_ >> 1;
                for (int qx = px - 1; qx <= px + 1; ++qx)
                    for (int qy = py - 1; qy <= py + 1; ++qy)
                        for (int qz = pz - 1; qz <= pz + 1; ++qz) {
                            if (qx < 0 || qy < 0 || qz < 0 || qx >= nside / 2 || qy >= nside / 2 || qz >= nside / 2)
                                continue;
                            for (int o = 0; o < 8; ++o) {
                                int sx_ = 2 * qx + ((o >> 2) & 1), sy_ = 2 * qy + ((o >> 1) & 1),
                                    sz_ = 2 * qz + (o & 1);
                                int dx = sx_ - tx_, dy = sy_ - ty_, dz = sz_ - tz_;
                                if (iabs(dx) <= 1 && iabs(dy) <= 1 && iabs(dz) <= 1) continue;
                                int sb = find_box(&SB[l], morton_key(sx_, sy_, sz_, l));
                                if (sb < 0) continue;
                                int key;
                                if (F->kind == 0) key = ((dx + 3) * 7 + (dy + 3)) * 7 + (dz + 3);
                                else key = (((dx + 3) * 7 + (dy + 3)) * nside + tz_) * nside + sz_;
                                if (!kused[key]) {
                                    double cs[3];
                                    box_center(cx, cy, cz, R, l, sx_, sy_, sz_, cs);
                                    kused[key] = 1;
                                    for (int k = 0; k < 3; ++k) {
                                        krep[6 * key + k] = ct[k];
                                        krep[6 * key + 3 + k] = cs[k];
                                    }
                                    if (F->kind == 1) iused[((dx * dx + dy * dy) * nside + tz_) * nside + sz_] = 1;
                                }
                                if (np_ == cap_p) {
                                    cap_p *= 2;
                                    pt = (int*)realloc(pt, sizeof(int) * cap_p);
                                    ps = (int*)realloc(ps, sizeof(int) * cap_p);
                                    pk = (int*)realloc(pk, sizeof(int) * cap_p);
                                }
                                pt[np_] = b;
                                ps[np_] = sb;
                                pk[np_] = key;
                                np_++;
                            }
                        }
            }
            tfirst[TB[l].nb] = np_;
            st->m2l_pairs += np_;
            cplx** ops = (cplx**)calloc((size_t)nkeys, sizeof(cplx*));
            cplx** iops = (cplx**)calloc((size_t)(nikeys > 0 ? nikeys : 1), sizeof(cplx*));
            int unstable = 0;
            if (F->kind == 1) {
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 1) reduction(| : unstable)
#endif
                for (int ik = 0; ik < nikeys; ++ik) {
                    if (!iused[ik]) continue;
                    int sz_ = ik % nside, tz_ = (ik / nside) % nside, d2 = ik / (nside * nside);
                    double zt = (cz - R) + (tz_ + 0.5) * h, zs = (cz - R) + (sz_ + 0.5) * h;
                    double rho = h * sqrt((double)d2);
                    iops[ik] = (cplx*)malloc(sizeof(cplx) * (size_t)K * K);
                    int uu = 0;
                    reaction_I_matrix(&F->rc, CT, p, rho, zt, zs, h, iops[ik], &uu);
                    unstable |= uu;
                }
            }
            st->unstable |= unstable;
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 1)
#endif
            for (int key = 0; key < nkeys; ++key) {
                if (!kused[key]) continue;
                const double* ct = &krep[6 * key];
                const double* cs = ct + 3;
                ops[key] = (cplx*)malloc(sizeof(cplx) * (size_t)K * K);
                if (F->kind == 0) {
                    free_operator(GT, 2, F->lam_t, ct[0] - cs[0], ct[1] - cs[1], ct[2] - cs[2], ops[key]);
                } else {
                    int sz_ = key % nside, tz_ = (key / nside) % nside, dxy = key / (nside * nside);
                    int dx = dxy / 7 - 3, dy = dxy % 7 - 3;
                    double ph = (dx == 0 && dy == 0) ? 0.0 : atan2(ct[1] - cs[1], ct[0] - cs[0]);
                    reaction_T_from_I(&F->rc, p, iops[((dx * dx + dy * dy) * nside + tz_) * nside + sz_], ph,
                                      ops[key]);
                }
            }
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 4)
#endif
            for (int b = 0; b < TB[l].nb; ++b)
                for (int k = tfirst[b]; k < tfirst[b + 1]; ++k)
                    apply_op(K, ops[pk[k]], &ME[l][(size_t)ps[k] * K], &LE[l][(size_t)b * K]);
            for (int k = 0; k < nkeys; ++k) free(ops[k]);
            for (int k = 0; k < nikeys; ++k) free(iops[k]);
            free(ops);
            free(iops);
            free(pt);
            free(ps);
            free(pk);
            free(tfirst);
            free(krep);
            free(kused);
            free(iused);
            /* X-list: local expansions formed from the sources of coarser
             * leaves directly (eq. melecoeffree; reaction: the L rows of eq.
             * coefintable with the point table, S = this box's side) */
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 1)
#endif
            for (int b = 0; b < TB[l].nb; ++b) {
                double c[3];
                key_center(cx, cy, cz, R, l, TB[l].key[b], c);
                for (int e = xptr[toff[l] + b]; e < xptr[toff[l] + b + 1]; ++e) {
                    const int* v = X.v + 4 * xidx[e];
                    int k0, k1;
                    box_range(ns, skey, v[2], SB[v[2]].key[v[3]], &k0, &k1);
                    for (int k = k0; k < k1; ++k) {
                        int j = sorder[k];
                        if (F->kind == 0)
                            p2l_free_one(p, F->lam_t, sq[j], sx[j] - c[0], sy[j] - c[1], sz[j] - c[2],
                                         &LE[l][(size_t)b * K]);
                        else
                            p2l_react_one(&F->rc, CT, p, sq[j], sx[j], sy[j], sz[j], c, h, &LE[l][(size_t)b * K]);
                    }
                }
            }
        }
        /* L2P at the leaves, then the W-list: multipole expansions of finer
         * boxes evaluated at the leaf's targets directly (eq.
         * freespace3dmulexp; reaction: the F~ rows of eq. coefintable with the
         * point table, S = the source box's side) */
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 4)
#endif
        for (int e = 0; e < ntl; ++e) {
            int l = tleaf[2 * e], b = tleaf[2 * e + 1];
            int k0, k1;
            box_range(nt, tkey, l, TB[l].key[b], &k0, &k1);
            if (l >= 2) {
                double c[3];
                key_center(cx, cy, cz, R, l, TB[l].key[b], c);
                for (int k = k0; k < k1; ++k) {
                    int i = torder[k];
                    phi[i] += F->far_factor *
                              l2p_one(p, F->lam_t, &LE[l][(size_t)b * K], tx[i] - c[0], ty[i] - c[1], tz[i] - c[2]);
                }
            }
            for (int w = wptr[toff[l] + b]; w < wptr[toff[l] + b + 1]; ++w) {
                const int* v = W.v + 4 * widx[w];
                int sl = v[2], sb = v[3];
                double c[3];
                key_center(cx, cy, cz, R, sl, SB[sl].key[sb], c);
                const cplx* M = &ME[sl][(size_t)sb * K];
                for (int k = k0; k < k1; ++k) {
                    int i = torder[k];
                    if (F->kind == 0)
                        phi[i] += F->far_factor * m2p_free_one(p, F->lam_s, M, tx[i] - c[0], ty[i] - c[1], tz[i] - c[2]);
                    else
                        phi[i] += m2p_react_one(&F->rc, CT, p, M, tx[i], ty[i], tz[i], c,
                                                2.0 * R / (double)(1 << sl));
                }
            }
        }
        free(Aop);
        for (int l = 0; l <= H; ++l) {
            free(ME[l]);
            free(LE[l]);
        }
    }

    /* ---------------- near field (U-list) ---------------- */
    long long npp = 0;
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : npp)
#endif
    for (int e = 0; e < ntl; ++e) {
        int l = tleaf[2 * e], b = tleaf[2 * e + 1];
        int k0, k1;
        box_range(nt, tkey, l, TB[l].key[b], &k0, &k1);
        for (int u = uptr[toff[l] + b]; u < uptr[toff[l] + b + 1]; ++u) {
            const int* v = U.v + 4 * uidx[u];
            int s0, s1;
            box_range(ns, skey, v[2], SB[v[2]].key[v[3]], &s0, &s1);
            for (int k = k0; k < k1; ++k) {
                int i = torder[k];
                phi[i] += near_sum(F, i, tx, ty, tz, tid, s0, s1, sorder, sx, sy, sz, sq, sid, &npp);
            }
        }
    }
    st->p2p_pairs = npp;

    for (int l = 0; l <= H; ++l) {
        free(SB[l].key);
        free(TB[l].key);
    }
    free(U.v);
    free(W.v);
    free(X.v);
    free(uptr);
    free(uidx);
    free(wptr);
    free(widx);
    free(xptr);
    free(xidx);
    free(sleaf);
    free(tleaf);
    free(slv);
    free(tlv);
    free(sorder);
    free(torder);
    free(skey);
    free(tkey);
    free(Cs.cx);
    free(Ct.cx);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Algorithm 2: all free-space and reaction components, summed.             */
/* Components are enumerated as: free l = 0..L; then (a,b) = (1,1) for      */
/* l = 0..L-1, l' = 0..L-1; (1,2) for l = 0..L-1, l' = 1..L; (2,1) for      */
/* l = 1..L, l' = 0..L-1; (2,2) for l = 1..L, l' = 1..L.                    */
/* ------------------------------------------------------------------------ */
int orc_num_components(int nlayers)
{
    int L = nlayers - 1;
    return (L + 1) + 4 * L * L;
}

/* Describe component c: out[0]=kind, out[1]=l, out[2]=lp, out[3]=a, out[4]=b */
int orc_component(int nlayers, int c, int* out)
{
    int L = nlayers - 1;
    if (c < 0) return -1;
    if (c <= L) {
        out[0] = 0;
        out[1] = c;
        out[2] = c;
        out[3] = 0;
        out[4] = 0;
        return 0;
    }
    c -= L + 1;
    for (int a = 1; a <= 2; ++a)
        for (int b = 1; b <= 2; ++b) {
            int l0 = (a == 1) ? 0 : 1, lp0 = (b == 1) ? 0 : 1;
            for (int l = l0; l < l0 + L; ++l)
                for (int lp = lp0; lp < lp0 + L; ++lp) {
                    if (c == 0) {
                        out[0] = 1;
                        out[1] = l;
                        out[2] = lp;
                        out[3] = a;
                        out[4] = b;
                        return 0;
                    }
                    c--;
                }
        }
    return -1;
}

/* Root cube of a free-space component: the bounding cube of the layer's
 * charges. */
static void root_free(int n, const double* x, const double* y, const double* z, double* c, double* R)
{
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int i = 0; i < n; ++i) {
        double v[3] = {x[i], y[i], z[i]};
        for (int k = 0; k < 3; ++k) {
            lo[k] = fmin(lo[k], v[k]);
            hi[k] = fmax(hi[k], v[k]);
        }
    }
    double r = 0.0;
    for (int k = 0; k < 3; ++k) {
        c[k] = 0.5 * (lo[k] + hi[k]);
        r = fmax(r, 0.5 * (hi[k] - lo[k]));
    }
    *R = r > 0 ? r : 0.5;
}

/* Common grid of the reaction components of one medium.  In the frame of a
 * reaction component whose interface is z = 0 with the targets above it
 * (mirrored in z when the interface is the upper one, a = 2), every target
 * sits at height tau_a of its own layer and every equivalent source at depth
 * -tau'_b of its layer (eq. equivpolarcoord), independently of the other
 * layer of the component.  One root cube and one depth therefore serve all
 * of them (Sec. 3.5: the largest box is halved by the interface):
 *   centre x, y: middle of the bounding box of all charges; z: the interface;
 *   half side R: the largest of the half x and y extents and of every
 *     distance tau of a charge to an interface of its own layer;
 *   depth: the smallest l <= 12 at which every point set (layer, side) with
 *     N charges, placed at +tau (targets) and at -tau (images), has
 *     N <= cap * (non-empty boxes at level l); then raised (by at most 3
 *     levels, to at most 12) until the box side 2R/2^l is <= the smallest tau.
 * Cells: fine_cell(x, cx, R), fine_cell(y, cy, R), fine_cell(+-tau, 0, R);
 * for a = 2 the z cell is mirrored (65535 - c) into the original orientation. */
typedef struct {
    double cx, cy, R;
    int H;
} rgrid_t;

static int side_valid(const layers_t* Ly, int l, int s) { return s == 1 ? l < Ly->L : l > 0; }

static void reaction_grid(const layers_t* Ly, int64_t n, const double* x, const double* y, const double* z,
                          const int* lay, int cap, rgrid_t* G)
{
    double lo[2] = {INFINITY, INFINITY}, hi[2] = {-INFINITY, -INFINITY}, r = 0.0, tmin = INFINITY;
    for (int64_t i = 0; i < n; ++i) {
        lo[0] = fmin(lo[0], x[i]);
        hi[0] = fmax(hi[0], x[i]);
        lo[1] = fmin(lo[1], y[i]);
        hi[1] = fmax(hi[1], y[i]);
        for (int sd = 1; sd <= 2; ++sd)
            if (side_valid(Ly, lay[i], sd)) {
                double t = fabs(tau_s(Ly, lay[i], sd, z[i]));
                r = fmax(r, t);
                tmin = fmin(tmin, t);
            }
    }
    G->cx = 0.5 * (lo[0] + hi[0]);
    G->cy = 0.5 * (lo[1] + hi[1]);
    r = fmax(r, 0.5 * (hi[0] - lo[0]));
    r = fmax(r, 0.5 * (hi[1] - lo[1]));
    G->R = r > 0 ? r : 0.5;
    G->H = 0;
    /* depth: every (layer, side) set, as targets (+tau) and as images (-tau) */
    for (int l = 0; l <= Ly->L; ++l)
        for (int sd = 1; sd <= 2; ++sd) {
            if (!side_valid(Ly, l, sd)) continue;
            int m = 0;
            for (int64_t i = 0; i < n; ++i) m += lay[i] == l;
            if (m == 0) continue;
            for (int sg = -1; sg <= 1; sg += 2) {
                cells_t C;
                C.n = m;
                C.cx = (uint32_t*)malloc(sizeof(uint32_t) * 3 * m);
                C.cy = C.cx + m;
                C.cz = C.cy + m;
                int k = 0;
                for (int64_t i = 0; i < n; ++i)
                    if (lay[i] == l) {
                        C.cx[k] = fine_cell(x[i], G->cx, G->R);
                        C.cy[k] = fine_cell(y[i], G->cy, G->R);
                        C.cz[k++] = fine_cell(sg * tau_s(Ly, l, sd, z[i]), 0.0, G->R);
                    }
                int lv = 0;
                for (; lv < ORC_MAXDEPTH; ++lv) {
                    boxlev_t B;
                    distinct_boxes(&C, lv, &B);
                    int ok = (long long)m <= (long long)cap * B.nb;
                    free(B.key);
                    if (ok) break;
                }
                if (lv > G->H) G->H = lv;
                free(C.cx);
            }
        }
    /* separation: with leaves no wider than the smallest distance tau of a
     * charge to an interface of its layer, every target and every image lies
     * at least one box away from the interface plane, so no reaction U-list
     * pair remains (Remark 1: the reaction near field is rare).  At most 3
     * levels are added to the occupancy depth for this. */
    int hs = 0;
    while (hs < ORC_MAXDEPTH && 2.0 * G->R / (double)(1 << hs) > tmin) ++hs;
    int hcap = G->H + 3 < ORC_MAXDEPTH ? G->H + 3 : ORC_MAXDEPTH;
    if (hs > hcap) hs = hcap;
    if (hs > G->H) G->H = hs;
}

/* Fine cells of the targets (layer l, side a) and images (layer lp, side b)
 * of a reaction component on the common grid, in the original orientation. */
static void reaction_cells(const layers_t* Ly, const rgrid_t* G, int l, int lp, int a, int b, int nt,
                           const double* tx, const double* ty, const double* tz, int ns, const double* sx,
                           const double* sy, const double* sz_orig, cells_t* Ct, cells_t* Cs)
{
    Ct->n = nt;
    Ct->cx = (uint32_t*)malloc(sizeof(uint32_t) * 3 * (nt + 1));
    Ct->cy = Ct->cx + nt;
    Ct->cz = Ct->cy + nt;
    Cs->n = ns;
    Cs->cx = (uint32_t*)malloc(sizeof(uint32_t) * 3 * (ns + 1));
    Cs->cy = Cs->cx + ns;
    Cs->cz = Cs->cy + ns;
    for (int i = 0; i < nt; ++i) {
        Ct->cx[i] = fine_cell(tx[i], G->cx, G->R);
        Ct->cy[i] = fine_cell(ty[i], G->cy, G->R);
        uint32_t c = fine_cell(tau_t(Ly, l, a, tz[i]), 0.0, G->R);
        Ct->cz[i] = (a == 2) ? 65535u - c : c;
    }
    for (int i = 0; i < ns; ++i) {
        Cs->cx[i] = fine_cell(sx[i], G->cx, G->R);
        Cs->cy[i] = fine_cell(sy[i], G->cy, G->R);
        uint32_t c = fine_cell(-tau_s(Ly, lp, b, sz_orig[i]), 0.0, G->R);
        Cs->cz[i] = (a == 2) ? 65535u - c : c;
    }
}

/* Full layered FMM (Algorithm 2).  phi[n] receives the potential at every
 * charge in input order; comp_phi (nullable) [ncomp][n] receives each
 * component's contribution; stats (nullable) [ncomp][6] receives
 * depth, target leaves, source leaves, M2L pairs, P2P pairs, recurrence
 * stability violation flag. */
int orc_fmm(int nlayers, const double* eps, const double* lam, const double* d, int64_t n, const double* x,
            const double* y, const double* z, const double* q, int p, int leaf_cap, int adaptive, int nthreads,
            double* phi, double* comp_phi, double* stats)
{
    layers_t Ly;
    if (fill_layers(&Ly, nlayers, eps, lam, d)) return -1;
    if (p < 0 || p > ORC_PMAX || leaf_cap < 1) return -3;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
    int ncomp = orc_num_components(nlayers);
    int* lay = (int*)malloc(sizeof(int) * (n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) lay[i] = layer_of(&Ly, z[i]);
    memset(phi, 0, sizeof(double) * n);
    if (comp_phi) memset(comp_phi, 0, sizeof(double) * n * ncomp);
    gaunt_tab_t GT;
    gaunt_tab_init(&GT, p);
    rgrid_t G;
    memset(&G, 0, sizeof(G));
    if (Ly.L > 0) reaction_grid(&Ly, n, x, y, z, lay, leaf_cap, &G);
    for (int c = 0; c < ncomp; ++c) {
        int desc[5];
        orc_component(nlayers, c, desc);
        int kind = desc[0], l = desc[1], lp = desc[2], a = desc[3], b = desc[4];
        /* gather targets (layer l) and sources (layer lp) */
        int nt = 0, ns = 0;
        for (int64_t i = 0; i < n; ++i) {
            if (lay[i] == l) nt++;
            if (lay[i] == lp) ns++;
        }
        double* buf = (double*)malloc(sizeof(double) * (3 * nt + 5 * ns + nt + 1));
        double *tx = buf, *ty = tx + nt, *tz = ty + nt, *sx = tz + nt, *sy = sx + ns, *sz = sy + ns, *sq = sz + ns;
        double* ph = sq + ns;
        double* szo = ph + nt;   /* sources' own z */
        int64_t* tid = (int64_t*)malloc(sizeof(int64_t) * (nt + ns + 1));
        int64_t* sid = tid + nt;
        int it = 0, is = 0;
        double zi = 0.0;
        if (kind == 1) zi = (a == 1) ? Ly.d[l] : Ly.d[l - 1];
        for (int64_t i = 0; i < n; ++i) {
            if (lay[i] == l) {
                tx[it] = x[i];
                ty[it] = y[i];
                tz[it] = z[i];
                tid[it++] = i;
            }
            if (lay[i] == lp) {
                sx[is] = x[i];
                sy[is] = y[i];
                szo[is] = z[i];
                if (kind == 0) sz[is] = z[i];
                else {
                    /* equivalent polarization coordinate (eq. equivpolarcoord, with the
                     * source's own z in place of the printed z_{lj}) */
                    double ts = tau_s(&Ly, lp, b, z[i]);
                    sz[is] = (a == 1) ? Ly.d[l] - ts : Ly.d[l - 1] + ts;
                }
                sq[is] = q[i];
                sid[is++] = i;
            }
        }
        fmmspec_t F;
        memset(&F, 0, sizeof(F));
        F.kind = kind;
        F.rc.Ly = Ly;
        F.rc.l = l;
        F.rc.lp = lp;
        F.rc.a = a;
        F.rc.b = b;
        F.lam_t = Ly.lam[l];
        F.lam_s = Ly.lam[lp];
        F.eps_t = Ly.eps[l];
        /* free space: e^{-lam r}/(4 pi eps r) = (lam / (2 pi^2 eps)) k_0(lam r) */
        F.far_factor = (kind == 0) ? Ly.lam[l] / (2.0 * ORC_PI * ORC_PI * Ly.eps[l]) : 1.0;
        double ctr[3], R;
        cells_t Cs, Ct;
        Cs.cx = Ct.cx = NULL;
        if (kind == 0) root_free(nt, tx, ty, tz, ctr, &R);
        else {
            ctr[0] = G.cx;
            ctr[1] = G.cy;
            ctr[2] = zi;
            R = G.R;
            reaction_cells(&Ly, &G, l, lp, a, b, nt, tx, ty, tz, ns, sx, sy, szo, &Ct, &Cs);
        }
        ctab_t CT;
        CT.v = NULL;
        if (kind == 1) ctab_init(&CT, p, Ly.lam[l], Ly.lam[lp]);
        fmmstat_t st;
        run_fmm(&F, p, leaf_cap, adaptive, ns, sx, sy, sz, sq, sid, nt, tx, ty, tz, tid, ctr[0], ctr[1], ctr[2], R,
                kind == 1 ? &Cs : NULL, kind == 1 ? &Ct : NULL, kind == 1 ? G.H : -1, &GT,
                kind == 1 ? &CT : NULL, ph, &st);
        if (CT.v) free(CT.v);
        free(Cs.cx);
        free(Ct.cx);
        for (int k = 0; k < nt; ++k) {
            phi[tid[k]] += ph[k];
            if (comp_phi) comp_phi[(size_t)c * n + tid[k]] = ph[k];
        }
        if (stats) {
            double* s = stats + (size_t)c * 8;
            s[0] = st.depth;
            s[1] = st.nleaf_t;
            s[2] = st.nleaf_s;
            s[3] = (double)st.m2l_pairs;
            s[4] = (double)st.p2p_pairs;
            s[5] = st.unstable;
            s[6] = (double)st.w_pairs;
            s[7] = (double)st.x_pairs;
        }
        free(buf);
        free(tid);
    }
    gaunt_tab_free(&GT);
    free(lay);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Single-source expansion chains used by the operator pins.                */
/* ------------------------------------------------------------------------ */

/* Free space: source r', ME centre cs, (optional) M2M to cs2, M2L to LE
 * centre ct, (optional) L2L to ct2, evaluate at r; returns the expansion of
 * k_0(lam |r - r'|).  mode bit 0: do M2M (cs -> cs2); bit 1: do L2L. */
double orc_free_chain(int p, double lam, const double* rs, const double* cs, const double* cs2, const double* ct,
                      const double* ct2, const double* r, int mode)
{
    int K = (p + 1) * (p + 1);
    gaunt_tab_t GT;
    gaunt_tab_init(&GT, p);
    cplx* M = (cplx*)calloc(K, sizeof(cplx));
    cplx* M2 = (cplx*)calloc(K, sizeof(cplx));
    cplx* L = (cplx*)calloc(K, sizeof(cplx));
    cplx* L2 = (cplx*)calloc(K, sizeof(cplx));
    cplx* A = (cplx*)malloc(sizeof(cplx) * K * K);
    p2m_one(p, lam, 1.0, rs[0] - cs[0], rs[1] - cs[1], rs[2] - cs[2], M);
    const double* c_me = cs;
    if (mode & 1) {
        free_operator(&GT, 0, lam, cs[0] - cs2[0], cs[1] - cs2[1], cs[2] - cs2[2], A);
        apply_op(K, A, M, M2);
        memcpy(M, M2, sizeof(cplx) * K);
        c_me = cs2;
    }
    free_operator(&GT, 2, lam, ct[0] - c_me[0], ct[1] - c_me[1], ct[2] - c_me[2], A);
    apply_op(K, A, M, L);
    const double* c_le = ct;
    if (mode & 2) {
        free_operator(&GT, 1, lam, ct2[0] - ct[0], ct2[1] - ct[1], ct2[2] - ct[2], A);
        apply_op(K, A, L, L2);
        memcpy(L, L2, sizeof(cplx) * K);
        c_le = ct2;
    }
    double v = l2p_one(p, lam, L, r[0] - c_le[0], r[1] - c_le[1], r[2] - c_le[2]);
    free(M);
    free(M2);
    free(L);
    free(L2);
    free(A);
    gaunt_tab_free(&GT);
    return v;
}

/* Free-space addition theorems evaluated directly (pins for the operators):
 * which = 0: returns sum_{nu<=p,mu} Sh_{n nu}^{m mu}(b) i_nu Y_nu^mu(r) (complex, out[2])
 * which = 1: returns sum_{nu<=p,mu} S_{n nu}^{m mu}(b) i_nu Y_nu^mu(r)                  */
void orc_addition_sum(int p, int pq, double lam, int n, int m, const double* b, const double* r, int which,
                      double* out)
{
    /* build the operators at order pq >= n for the rows, truncating columns at p */
    int P = pq > p ? pq : p;
    int K = (P + 1) * (P + 1);
    gaunt_tab_t GT;
    gaunt_tab_init(&GT, P);
    cplx* A = (cplx*)malloc(sizeof(cplx) * K * K);
    /* kind 1 gives A_{(n,m),(nu,mu)} = Sh_{nu n}^{mu m}; take the transpose entries */
    free_operator(&GT, which == 0 ? 1 : 2, lam, b[0], b[1], b[2], A);
    cplx* Y = (cplx*)malloc(sizeof(cplx) * K);
    ylm_c(P, r[0], r[1], r[2], Y);
    double rr = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
    cplx s = 0.0;
    for (int nu = 0; nu <= p; ++nu)
        for (int mu = -nu; mu <= nu; ++mu)
            s += A[(size_t)idx_nm(nu, mu) * K + idx_nm(n, m)] * orc_bessel_i(nu, lam * rr) * Y[idx_nm(nu, mu)];
    out[0] = creal(s);
    out[1] = cimag(s);
    free(A);
    free(Y);
    gaunt_tab_free(&GT);
}

/* Reaction component, single source: the image of r' (equivalent
 * polarization coordinate), ME about the image centre cs (which must lie on
 * the image side), M2L to the target centre ct, LE evaluated at r.  Returns
 * the expansion value of u^{ab}_{l lp}(r, r'). */
double orc_reaction_chain(const double* eps, const double* lam, const double* d, int L, int l, int lp, int a, int b,
                          int p, const double* rs, const double* cs, const double* ct, const double* r, int* unstable)
{
    rcomp_t C;
    fill_layers(&C.Ly, L + 1, eps, lam, d);
    C.l = l;
    C.lp = lp;
    C.a = a;
    C.b = b;
    if (L < 1 || L > ORC_MAXL || !comp_valid(&C.Ly, l, lp, a, b)) return NAN;
    int K = (p + 1) * (p + 1);
    double ts = tau_s(&C.Ly, lp, b, rs[2]);
    double zimg = (a == 1) ? C.Ly.d[l] - ts : C.Ly.d[l - 1] + ts;
    cplx* M = (cplx*)calloc(K, sizeof(cplx));
    cplx* Lc = (cplx*)calloc(K, sizeof(cplx));
    cplx* Im = (cplx*)malloc(sizeof(cplx) * K * K);
    cplx* A = (cplx*)malloc(sizeof(cplx) * K * K);
    p2m_one(p, lam[lp], 1.0, rs[0] - cs[0], rs[1] - cs[1], zimg - cs[2], M);
    ctab_t CT;
    ctab_init(&CT, p, lam[l], lam[lp]);
    double rho = hypot(ct[0] - cs[0], ct[1] - cs[1]);
    double ph = (ct[0] == cs[0] && ct[1] == cs[1]) ? 0.0 : atan2(ct[1] - cs[1], ct[0] - cs[0]);
    /* the scaling length S only rescales intermediate values; use the centre separation */
    double S = fmin(fabs(ct[2] - cs[2]), rho > 0 ? rho : INFINITY);
    int uu = 0;
    reaction_I_matrix(&C, &CT, p, rho, ct[2], cs[2], S, Im, &uu);
    if (unstable) *unstable = uu;
    reaction_T_from_I(&C, p, Im, ph, A);
    apply_op(K, A, M, Lc);
    double v = l2p_one(p, lam[l], Lc, r[0] - ct[0], r[1] - ct[1], r[2] - ct[2]);
    free(M);
    free(Lc);
    free(Im);
    free(A);
    free(CT.v);
    return v;
}

/* Recurrence-versus-direct-quadrature pin: I_{nm,nu mu} of a component at
 * (rho, zt, zs) from the recurrence path (eq. metoletableform) and from
 * direct quadrature with Q = P^ P^.  out: [re_rec, im_rec, re_dir, im_dir]. */
void orc_reaction_I_pair(const double* eps, const double* lam, const double* d, int L, int l, int lp, int a, int b,
                         int p, double rho, double zt, double zs, double S, int n, int m, int nu, int mu, double* out)
{
    rcomp_t C;
    fill_layers(&C.Ly, L + 1, eps, lam, d);
    C.l = l;
    C.lp = lp;
    C.a = a;
    C.b = b;
    int nmax = 2 * p + 3;
    double* tab = (double*)malloc(sizeof(double) * 4 * (nmax + 1) * (nmax + 1));
    sommerfeld_table(&C, rho, zt, zs, S, nmax, tab);
    ctab_t CT;
    ctab_init(&CT, p, lam[l], lam[lp]);
    cplx v = assemble_I(&CT, tab, nmax, S, n, m, nu, mu);
    cplx w = reaction_I_direct_one(&C, n, m, nu, mu, rho, zt, zs, NULL);
    out[0] = creal(v);
    out[1] = cimag(v);
    out[2] = creal(w);
    out[3] = cimag(w);
    free(tab);
    free(CT.v);
}

/* Rounding scale of the recurrence path (running error analysis): the same
 * steps as sommerfeld_table and assemble_I applied to moduli, |a - b| ->
 * |a| + |b|, starting from the quadrature of the moduli of the initial-value
 * integrands.  The rounding error of every table entry and of every I entry
 * is a modest multiple of 1e-16 times this scale; it grows where the forward
 * recurrence in m amplifies earlier entries (large m at small rho / S). */
static void reaction_I_bound(const rcomp_t* C, const ctab_t* CT, int p, double rho, double zt, double zs, double S,
                             double* B)
{
    const layers_t* Ly = &C->Ly;
    int nmax = 2 * p + 3, N1 = nmax + 1, K = (p + 1) * (p + 1);
    double lt = Ly->lam[C->l], ls = Ly->lam[C->lp];
    double* tab = (double*)calloc((size_t)4 * N1 * N1, sizeof(double));
    nodes_t nd;
    build_nodes(&nd, rho, zsep(C, zt, zs), nmax, layers_lam_min(Ly), layers_dmax(Ly), ORC_TOL);
    for (int k = 0; k < nd.n; ++k) {
        double t = nd.x[k];
        double lz = sqrt(lt * lt + t * t), lzp = sqrt(ls * ls + t * t);
        double base = fabs(nd.w[k] * zkern(C, lz, lzp, zt, zs) * sigma(Ly, C->l, C->lp, C->a, C->b, t) / lz);
        double j0 = fabs(jn(0, t * rho)), j1 = fabs(jn(1, t * rho));
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 2; ++j) {
                double f = base * (i ? lt / lz : 1.0) * (j ? ls / lzp : 1.0);
                double* T = tab + (size_t)(i * 2 + j) * N1 * N1;
                double pw = 1.0;
                for (int n = 0; n <= nmax; ++n) {
                    T[n * N1 + 0] += f * pw * j0 / fact(n);
                    if (n >= 1) T[n * N1 + 1] += f * pw * j1 / sqrt(fact(n + 1) * fact(n - 1));
                    pw *= t * S;
                }
            }
    }
    free_nodes(&nd);
    for (int ij = 0; ij < 4 && rho > 0.0; ++ij) {
        double* T = tab + (size_t)ij * N1 * N1;
        for (int m = 1; m < nmax; ++m)
            for (int n = m + 1; n <= nmax; ++n)
                T[n * N1 + m + 1] = 2.0 * m / a_n(n + m) * (S / rho) * T[(n - 1) * N1 + m] +
                                    a_n(n - m) / a_n(n + m) * T[n * N1 + m - 1];
    }
    for (int n = 0; n <= p; ++n)
        for (int m = -n; m <= n; ++m)
            for (int nu = 0; nu <= p; ++nu)
                for (int mu = -nu; mu <= nu; ++mu) {
                    int i = (n + iabs(m)) % 2, j = (nu + iabs(mu)) % 2;
                    int r = (n + iabs(m)) / 2, rp = (nu + iabs(mu)) / 2;
                    const double* T = tab + (size_t)(i * 2 + j) * N1 * N1;
                    const cplx* cv = &CT->v[((size_t)idx_nm(n, m) * K + idx_nm(nu, mu)) * (CT->smax + 1)];
                    double acc = 0.0;
                    for (int s = 0; s <= (n - r) + (nu - rp); ++s) {
                        int Nn = iabs(m) + iabs(mu) + 2 * s + 1;
                        acc += cabs(cv[s]) * T[Nn * N1 + iabs(mu - m)] / pow(S, Nn);
                    }
                    B[(size_t)idx_nm(n, m) * K + idx_nm(nu, mu)] = acc;
                }
    free(tab);
}

/* The same cross-check for the whole K x K matrix, K = (p+1)^2, rows (n,m)
 * and columns (nu,mu) in the order n^2+n+m: rec = the recurrence path
 * (eqs. M2Ltable, recurrence1, metoletableform), dir = direct quadrature of
 * eq. uniformintegral with Q = P^_n^m P^_nu^mu, each [K*K] re then [K*K] im;
 * dabs[K*K] = the same quadrature of the integrand's modulus (the scale of
 * the rounding error of an oscillatory quadrature); rbound[K*K] = the
 * rounding scale of the recurrence path (reaction_I_bound).  Returns 1 if
 * the recurrence stability bound was violated. */
int orc_reaction_I_both(const double* eps, const double* lam, const double* d, int L, int l, int lp, int a, int b,
                        int p, double rho, double zt, double zs, double S, double* rec, double* dir, double* dabs,
                        double* rbound)
{
    rcomp_t C;
    fill_layers(&C.Ly, L + 1, eps, lam, d);
    C.l = l;
    C.lp = lp;
    C.a = a;
    C.b = b;
    int K = (p + 1) * (p + 1);
    cplx* Im = (cplx*)malloc(sizeof(cplx) * (size_t)K * K);
    ctab_t CT;
    ctab_init(&CT, p, lam[l], lam[lp]);
    int unstable = 0;
    reaction_I_matrix(&C, &CT, p, rho, zt, zs, S, Im, &unstable);
    reaction_I_bound(&C, &CT, p, rho, zt, zs, S, rbound);
    for (int k = 0; k < K * K; ++k) {
        rec[k] = creal(Im[k]);
        rec[(size_t)K * K + k] = cimag(Im[k]);
    }
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (int r = 0; r < K; ++r) {
        int n = (int)sqrt((double)r), m = r - n * n - n;
        for (int nu = 0; nu <= p; ++nu)
            for (int mu = -nu; mu <= nu; ++mu) {
                int c = idx_nm(nu, mu);
                double ab = 0.0;
                cplx w = reaction_I_direct_one(&C, n, m, nu, mu, rho, zt, zs, &ab);
                dabs[(size_t)r * K + c] = ab;
                dir[(size_t)r * K + c] = creal(w);
                dir[(size_t)K * K + (size_t)r * K + c] = cimag(w);
            }
    }
    free(Im);
    free(CT.v);
    return unstable;
}

/* Raw scaled Sommerfeld table (for the recurrence pins):
 * out[((i*2+j)*(nmax+1)+n)*(nmax+1)+m] = S^n Sc_{nm,ij}; mode 0 = recurrence
 * path of the M2L operators, mode 1 = every entry by direct quadrature of
 * eq. M2Ltable, mode 2 = the point table (forward and backward recurrences). */
int orc_sommerfeld_table(const double* eps, const double* lam, const double* d, int L, int l, int lp, int a, int b,
                         double rho, double zt, double zs, double S, int nmax, int mode, double* out)
{
    rcomp_t C;
    fill_layers(&C.Ly, L + 1, eps, lam, d);
    C.l = l;
    C.lp = lp;
    C.a = a;
    C.b = b;
    if (mode == 0) return sommerfeld_table(&C, rho, zt, zs, S, nmax, out);
    if (mode == 2) {
        sommerfeld_table_pt(&C, rho, zt, zs, S, nmax, out);
        return 0;
    }
    const layers_t* Ly = &C.Ly;
    int N1 = nmax + 1;
    double lt = Ly->lam[l], ls = Ly->lam[lp];
    memset(out, 0, sizeof(double) * 4 * N1 * N1);
    nodes_t nd;
    build_nodes(&nd, rho, zsep(&C, zt, zs), nmax, layers_lam_min(Ly), layers_dmax(Ly), ORC_TOL);
    for (int k = 0; k < nd.n; ++k) {
        double t = nd.x[k];
        double lz = sqrt(lt * lt + t * t), lzp = sqrt(ls * ls + t * t);
        double base = nd.w[k] * zkern(&C, lz, lzp, zt, zs) * sigma(Ly, l, lp, a, b, t) / lz;
        for (int m = 0; m <= nmax; ++m) {
            double jm = jn(m, t * rho);
            for (int i = 0; i < 2; ++i)
                for (int j = 0; j < 2; ++j) {
                    double f = base * (i ? lt / lz : 1.0) * (j ? ls / lzp : 1.0) * jm;
                    for (int n = m; n <= nmax; ++n)
                        out[((i * 2 + j) * N1 + n) * N1 + m] +=
                            f * pow(t * S, n) / sqrt(fact(n + m) * fact(n - m));
                }
        }
    }
    free_nodes(&nd);
    return 0;
}

/* Legendre-product expansion pin: returns sum_s C^s lrho^{|m|+|mu|+2s}
 * (l/l_z)^i (l'/l'_z)^j and the product P^_n^m(l_z/l) P^_nu^mu(l'_z/l')
 * evaluated directly; out = [re_exp, im_exp, re_dir, im_dir]. */
void orc_legendre_product(int n, int m, int nu, int mu, double lam, double lamp, double lrho, double* out)
{
    double lz = sqrt(lam * lam + lrho * lrho), lzp = sqrt(lamp * lamp + lrho * lrho);
    int i = (n + iabs(m)) % 2, j = (nu + iabs(mu)) % 2;
    int r = (n + iabs(m)) / 2, rp = (nu + iabs(mu)) / 2;
    cplx s = 0.0;
    for (int k = 0; k <= (n - r) + (nu - rp); ++k)
        s += c_coef(n, nu, m, mu, k, lam, lamp) * pow(lrho, iabs(m) + iabs(mu) + 2 * k);
    s *= pow(lam / lz, i) * pow(lamp / lzp, j);
    cplx dct = plm_big(n, m, lz / lam, lrho / lam) * plm_big(nu, mu, lzp / lamp, lrho / lamp);
    out[0] = creal(s);
    out[1] = cimag(s);
    out[2] = creal(dct);
    out[3] = cimag(dct);
}

/* Associated Legendre beyond [-1,1] on the paper's branch (for Prop. 3.2 pin) */
void orc_plm_beyond(int n, int m, double w, double* out)
{
    cplx v = plm_big(n, m, w, sqrt(w * w - 1.0));
    out[0] = creal(v);
    out[1] = cimag(v);
}

/* Tree summary of one component, for the tree-equality parity test:
 * out_depth, and for every target / source point its leaf Morton key. */
int orc_component_tree(int nlayers, const double* eps, const double* lam, const double* d, int64_t n,
                       const double* x, const double* y, const double* z, int comp, int leaf_cap, int adaptive,
                       int* depth, int64_t* nt_out, int64_t* ns_out, uint64_t* tkeys, uint64_t* skeys, int* tlev,
                       int* slev, double* root)
{
    layers_t Ly;
    if (fill_layers(&Ly, nlayers, eps, lam, d)) return -1;
    int desc[5];
    if (orc_component(nlayers, comp, desc)) return -1;
    int kind = desc[0], l = desc[1], lp = desc[2], a = desc[3], b = desc[4];
    int nt = 0, ns = 0;
    double* buf = (double*)malloc(sizeof(double) * 7 * (n + 1));
    double *tx = buf, *ty = tx + n, *tz = ty + n, *sx = tz + n, *sy = sx + n, *sz = sy + n, *szo = sz + n;
    int* lay = (int*)malloc(sizeof(int) * (n + 1));
    for (int64_t i = 0; i < n; ++i) {
        int li = layer_of(&Ly, z[i]);
        lay[i] = li;
        if (li == l) {
            tx[nt] = x[i];
            ty[nt] = y[i];
            tz[nt++] = z[i];
        }
        if (li == lp) {
            sx[ns] = x[i];
            sy[ns] = y[i];
            szo[ns] = z[i];
            if (kind == 0) sz[ns] = z[i];
            else {
                double ts = tau_s(&Ly, lp, b, z[i]);
                sz[ns] = (a == 1) ? Ly.d[l] - ts : Ly.d[l - 1] + ts;
            }
            ns++;
        }
    }
    double c[3], R;
    cells_t Cs, Ct;
    int H = ORC_MAXDEPTH;
    if (kind == 0) {
        root_free(nt, tx, ty, tz, c, &R);
        Cs.n = ns;
        Ct.n = nt;
        Cs.cx = (uint32_t*)malloc(sizeof(uint32_t) * 3 * (ns + 1));
        Cs.cy = Cs.cx + ns;
        Cs.cz = Cs.cy + ns;
        Ct.cx = (uint32_t*)malloc(sizeof(uint32_t) * 3 * (nt + 1));
        Ct.cy = Ct.cx + nt;
        Ct.cz = Ct.cy + nt;
        for (int i = 0; i < ns; ++i) {
            Cs.cx[i] = fine_cell(sx[i], c[0], R);
            Cs.cy[i] = fine_cell(sy[i], c[1], R);
            Cs.cz[i] = fine_cell(sz[i], c[2], R);
        }
        for (int i = 0; i < nt; ++i) {
            Ct.cx[i] = fine_cell(tx[i], c[0], R);
            Ct.cy[i] = fine_cell(ty[i], c[1], R);
            Ct.cz[i] = fine_cell(tz[i], c[2], R);
        }
        for (int lv = 0; lv <= ORC_MAXDEPTH; ++lv) {
            boxlev_t SB, TB;
            distinct_boxes(&Cs, lv, &SB);
            distinct_boxes(&Ct, lv, &TB);
            int ok = (long long)ns <= (long long)leaf_cap * SB.nb && (long long)nt <= (long long)leaf_cap * TB.nb;
            free(SB.key);
            free(TB.key);
            if (ok) {
                H = lv;
                break;
            }
        }
    } else {
        rgrid_t G;
        reaction_grid(&Ly, n, x, y, z, lay, leaf_cap, &G);
        c[0] = G.cx;
        c[1] = G.cy;
        c[2] = (a == 1) ? Ly.d[l] : Ly.d[l - 1];
        R = G.R;
        H = G.H;
        reaction_cells(&Ly, &G, l, lp, a, b, nt, tx, ty, tz, ns, sx, sy, szo, &Ct, &Cs);
    }
    free(lay);
    /* leaf level of each point: H (uniform) or the adaptive rule per set */
    for (int i = 0; i < nt; ++i) tlev[i] = H;
    for (int i = 0; i < ns; ++i) slev[i] = H;
    if (adaptive) {
        const cells_t* sets[2] = {&Ct, &Cs};
        int* lvs[2] = {tlev, slev};
        H = 0;
        for (int t = 0; t < 2; ++t) {
            int m = sets[t]->n;
            int* order = (int*)malloc(sizeof(int) * (m + 1));
            uint64_t* key = (uint64_t*)malloc(sizeof(uint64_t) * (m + 1));
            sort_points(sets[t], order, key);
            leaf_levels(m, order, key, leaf_cap, adaptive == 1 && kind == 1, lvs[t]);
            for (int i = 0; i < m; ++i) H = lvs[t][i] > H ? lvs[t][i] : H;
            free(order);
            free(key);
        }
    }
    for (int i = 0; i < nt; ++i) {
        int sh = ORC_HMAX - tlev[i];
        tkeys[i] = morton_key(Ct.cx[i] >> sh, Ct.cy[i] >> sh, Ct.cz[i] >> sh, tlev[i]);
    }
    for (int i = 0; i < ns; ++i) {
        int sh = ORC_HMAX - slev[i];
        skeys[i] = morton_key(Cs.cx[i] >> sh, Cs.cy[i] >> sh, Cs.cz[i] >> sh, slev[i]);
    }
    *depth = H;
    *nt_out = nt;
    *ns_out = ns;
    root[0] = c[0];
    root[1] = c[1];
    root[2] = c[2];
    root[3] = R;
    free(buf);
    free(Cs.cx);
    free(Ct.cx);
    return 0;
}

/* Point-form pins.  Free space: mode 0 forms the ME of a unit source rs about
 * c and evaluates it at r (M2P); mode 1 forms the LE about c from rs (P2L)
 * and evaluates it at r.  Returns the expansion value of k_0(lam |r - rs|). */
double orc_free_point_chain(int p, double lam, const double* rs, const double* c, const double* r, int mode)
{
    int K = (p + 1) * (p + 1);
    cplx* E = (cplx*)calloc(K, sizeof(cplx));
    double v;
    if (mode == 0) {
        p2m_one(p, lam, 1.0, rs[0] - c[0], rs[1] - c[1], rs[2] - c[2], E);
        v = m2p_free_one(p, lam, E, r[0] - c[0], r[1] - c[1], r[2] - c[2]);
    } else {
        p2l_free_one(p, lam, 1.0, rs[0] - c[0], rs[1] - c[1], rs[2] - c[2], E);
        v = l2p_one(p, lam, E, r[0] - c[0], r[1] - c[1], r[2] - c[2]);
    }
    free(E);
    return v;
}

/* Reaction component, single source rs (original coordinates; its image is
 * formed here): mode 0 = ME about the image-side centre c evaluated at r
 * (M2P); mode 1 = LE about the target-side centre c formed from the image
 * (P2L), evaluated at r.  S is the box side that scales the table.  Returns
 * the expansion value of u~^{ab}_{l lp}(r, r'). */
double orc_reaction_point_chain(const double* eps, const double* lam, const double* d, int L, int l, int lp, int a,
                                int b, int p, const double* rs, const double* c, const double* r, double S, int mode)
{
    rcomp_t C;
    fill_layers(&C.Ly, L + 1, eps, lam, d);
    C.l = l;
    C.lp = lp;
    C.a = a;
    C.b = b;
    if (L < 1 || L > ORC_MAXL || !comp_valid(&C.Ly, l, lp, a, b)) return NAN;
    int K = (p + 1) * (p + 1);
    double ts = tau_s(&C.Ly, lp, b, rs[2]);
    double zimg = (a == 1) ? C.Ly.d[l] - ts : C.Ly.d[l - 1] + ts;
    ctab_t CT;
    ctab_init(&CT, p, lam[l], lam[lp]);
    cplx* E = (cplx*)calloc(K, sizeof(cplx));
    double v;
    if (mode == 0) {
        p2m_one(p, lam[lp], 1.0, rs[0] - c[0], rs[1] - c[1], zimg - c[2], E);
        v = m2p_react_one(&C, &CT, p, E, r[0], r[1], r[2], c, S);
    } else {
        p2l_react_one(&C, &CT, p, 1.0, rs[0], rs[1], zimg, c, S, E);
        v = l2p_one(p, lam[l], E, r[0] - c[0], r[1] - c[1], r[2] - c[2]);
    }
    free(E);
    free(CT.v);
    return v;
}

/* Point-table pin: I_{nm,nu mu} at (rho, zt, zs) assembled from the point
 * table (forward and backward recurrences, table up to n = p + 2, so (n, m)
 * or (nu, mu) must be (0, 0)) and by direct quadrature with Q = P^ P^.
 * out = [re_tab, im_tab, re_dir, im_dir]. */
void orc_reaction_I_point(const double* eps, const double* lam, const double* d, int L, int l, int lp, int a, int b,
                          int p, double rho, double zt, double zs, double S, int n, int m, int nu, int mu, double* out)
{
    rcomp_t C;
    fill_layers(&C.Ly, L + 1, eps, lam, d);
    C.l = l;
    C.lp = lp;
    C.a = a;
    C.b = b;
    int nmax = p + 2;
    double* tab = (double*)malloc(sizeof(double) * 4 * (nmax + 1) * (nmax + 1));
    sommerfeld_table_pt(&C, rho, zt, zs, S, nmax, tab);
    ctab_t CT;
    ctab_init(&CT, p, lam[l], lam[lp]);
    cplx v = assemble_I(&CT, tab, nmax, S, n, m, nu, mu);
    cplx w = reaction_I_direct_one(&C, n, m, nu, mu, rho, zt, zs, NULL);
    out[0] = creal(v);
    out[1] = cimag(v);
    out[2] = creal(w);
    out[3] = cimag(w);
    free(tab);
    free(CT.v);
}

/* List pin: builds the trees (uniform at depth Hfix when adaptive = 0, else
 * adaptive with leaf cap `cap`, sep as for a reaction component's sets) and
 * lists of run_fmm for sources and targets
 * given by their fine cells (cx, cy, cz per point, 0..65535), and counts for
 * every (target, source) pair how many list entries cover it: V (all targets
 * under the target box and all sources under the source box), U, W and X.
 * cover[i * ns + j] (sorted-order independent: indices are the inputs').
 * counts[0..3] = number of V, U, W, X box pairs. */
int orc_list_coverage(int ns, const uint32_t* scell, int nt, const uint32_t* tcell, int cap, int adaptive, int sep,
                      int Hfix, int* cover, long long* counts)
{
    cells_t Cs, Ct;
    Cs.n = ns;
    Ct.n = nt;
    Cs.cx = (uint32_t*)scell;
    Cs.cy = Cs.cx + ns;
    Cs.cz = Cs.cy + ns;
    Ct.cx = (uint32_t*)tcell;
    Ct.cy = Ct.cx + nt;
    Ct.cz = Ct.cy + nt;
    memset(cover, 0, sizeof(int) * (size_t)nt * ns);
    memset(counts, 0, sizeof(long long) * 4);
    if (ns == 0 || nt == 0) return 0;
    int* sorder = (int*)malloc(sizeof(int) * ns);
    int* torder = (int*)malloc(sizeof(int) * nt);
    uint64_t* skey = (uint64_t*)malloc(sizeof(uint64_t) * ns);
    uint64_t* tkey = (uint64_t*)malloc(sizeof(uint64_t) * nt);
    sort_points(&Cs, sorder, skey);
    sort_points(&Ct, torder, tkey);
    int* slv = (int*)malloc(sizeof(int) * ns);
    int* tlv = (int*)malloc(sizeof(int) * nt);
    int H = 0;
    if (adaptive) {
        leaf_levels(ns, sorder, skey, cap, sep, slv);
        leaf_levels(nt, torder, tkey, cap, sep, tlv);
        for (int i = 0; i < ns; ++i) H = slv[i] > H ? slv[i] : H;
        for (int i = 0; i < nt; ++i) H = tlv[i] > H ? tlv[i] : H;
    } else {
        H = Hfix;
        for (int i = 0; i < ns; ++i) slv[i] = H;
        for (int i = 0; i < nt; ++i) tlv[i] = H;
    }
    boxlev_t SB[ORC_MAXDEPTH + 1], TB[ORC_MAXDEPTH + 1];
    for (int l = 0; l <= H; ++l) {
        level_boxes(&Cs, slv, l, &SB[l]);
        level_boxes(&Ct, tlv, l, &TB[l]);
    }
    plist_t U = {0, 0, NULL}, W = {0, 0, NULL}, X = {0, 0, NULL}, V = {0, 0, NULL};
    traverse(TB, SB, H, 0, 0, 0, 0, &U, &W, &X);
    /* V-list as run_fmm lists it: level l >= 2, children of the neighbours
     * of the target's parent that are not adjacent to the target */
    for (int l = 2; l <= H; ++l) {
        int nside = 1 << l;
        for (int b = 0; b < TB[l].nb; ++b) {
            int tx_, ty_, tz_;
            key_coords(TB[l].key[b], l, &tx_, &ty_, &tz_);
            int px = tx_ >> 1, py = ty_ >> 1, pz = tz_ >> 1;
            for (int qx = px - 1; qx <= px + 1; ++qx)
                for (int qy = py - 1; qy <= py + 1; ++qy)
                    for (int qz = pz - 1; qz <= pz + 1; ++qz) {
                        if (qx < 0 || qy < 0 || qz < 0 || qx >= nside / 2 || qy >= nside / 2 || qz >= nside / 2)
                            continue;
                        for (int o = 0; o < 8; ++o) {
                            int sx_ = 2 * qx + ((o >> 2) & 1), sy_ = 2 * qy + ((o >> 1) & 1), sz_ = 2 * qz + (o & 1);
                            if (iabs(sx_ - tx_) <= 1 && iabs(sy_ - ty_) <= 1 && iabs(sz_ - tz_) <= 1) continue;
                            int sb = find_box(&SB[l], morton_key(sx_, sy_, sz_, l));
                            if (sb >= 0) plist_push(&V, l, b, l, sb);
                        }
                    }
        }
    }
    plist_t* lists[4] = {&V, &U, &W, &X};
    for (int t = 0; t < 4; ++t) {
        counts[t] = lists[t]->n;
        for (int e = 0; e < lists[t]->n; ++e) {
            const int* v = lists[t]->v + 4 * e;
            int t0, t1, s0, s1;
            box_range(nt, tkey, v[0], TB[v[0]].key[v[1]], &t0, &t1);
            box_range(ns, skey, v[2], SB[v[2]].key[v[3]], &s0, &s1);
            for (int a = t0; a < t1; ++a)
                for (int c = s0; c < s1; ++c) cover[(size_t)torder[a] * ns + sorder[c]]++;
        }
        free(lists[t]->v);
    }
    for (int l = 0; l <= H; ++l) {
        free(SB[l].key);
        free(TB[l].key);
    }
    free(sorder);
    free(torder);
    free(skey);
    free(tkey);
    free(slv);
    free(tlv);
    return 0;
}
