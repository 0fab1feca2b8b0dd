/* Sanitizer driver for the oracle (test infrastructure; built with
 * AddressSanitizer and UndefinedBehaviorSanitizer by tests/test_sanitizers.py):
 * small runs of every exported entry point, uniform and adaptive trees. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int orc_fmm(int nlayers, const double* eps, const double* lam, const double* d, int64_t n, const double* x,
            const double* y, const double* z, const double* q, int p, int leaf_cap, int adaptive, int nthreads,
            double* phi, double* comp_phi, double* stats);
int orc_direct_sum(int nlayers, const double* eps, const double* lam, const double* d, int64_t n, const double* x,
                   const double* y, const double* z, const double* q, int64_t nt, const int64_t* targets, double* phi,
                   int nthreads);
int orc_list_coverage(int ns, const uint32_t* scell, int nt, const uint32_t* tcell, int cap, int adaptive, int sep,
                      int Hfix, int* cover, long long* counts);
int orc_component_tree(int nlayers, const double* eps, const double* lam, const double* d, int64_t n,
                       const double* x, const double* y, const double* z, int comp, int leaf_cap, int adaptive,
                       int* depth, int64_t* nt_out, int64_t* ns_out, uint64_t* tkeys, uint64_t* skeys, int* tlev,
                       int* slev, double* root);
int orc_num_components(int nlayers);
double orc_reaction_point_chain(const double* eps, const double* lam, const double* d, int L, int l, int lp, int a,
                                int b, int p, const double* rs, const double* c, const double* r, double S, int mode);
double orc_free_point_chain(int p, double lam, const double* rs, const double* c, const double* r, int mode);
int orc_sommerfeld_table(const double* eps, const double* lam, const double* d, int L, int l, int lp, int a, int b,
                         double rho, double zt, double zs, double S, int nmax, int mode, double* out);

static double urand(uint64_t* s)
{
    *s = *s * 6364136223846793005ULL + 1442695040888963407ULL;
    return (double)(*s >> 11) * (1.0 / 9007199254740992.0);
}

int main(void)
{
    const double eps[3] = {1, 2, 4}, lam[3] = {1.2, 1.5, 2.0}, d[2] = {0.0, -1.2};
    const double zlo[3] = {0.03, -1.17, -2.2}, zhi[3] = {1.0, -0.03, -1.23}, zc[3] = {0.08, -0.08, -1.28};
    enum { PER = 40, N = 3 * PER };
    double x[N], y[N], z[N], q[N], phi[N], ref[N];
    uint64_t s = 7;
    for (int l = 0; l < 3; ++l)
        for (int i = 0; i < PER; ++i) {
            int k = l * PER + i;
            if (i % 2) {
                x[k] = urand(&s) - 0.5;
                y[k] = urand(&s) - 0.5;
                z[k] = zlo[l] + (zhi[l] - zlo[l]) * urand(&s);
            } else {
                x[k] = 0.1 + 0.02 * (urand(&s) - 0.5);
                y[k] = -0.1 + 0.02 * (urand(&s) - 0.5);
                z[k] = zc[l] + 0.01 * (urand(&s) - 0.5);
            }
            q[k] = 2.0 * urand(&s) - 1.0;
        }
    int bad = 0;
    if (orc_direct_sum(3, eps, lam, d, N, x, y, z, q, N, NULL, ref, 2)) bad++;
    int nc = orc_num_components(3);
    double* cphi = malloc(sizeof(double) * N * nc);
    double* st = malloc(sizeof(double) * 8 * nc);
    for (int ad = 0; ad <= 2; ++ad)
        for (int cap = 10; cap <= 10; ++cap) {
            if (orc_fmm(3, eps, lam, d, N, x, y, z, q, 2, cap, ad, 2, phi, cphi, st)) bad++;
            double e = 0, r = 0;
            for (int i = 0; i < N; ++i) {
                e += (phi[i] - ref[i]) * (phi[i] - ref[i]);
                r += ref[i] * ref[i];
            }
            if (!(sqrt(e / r) < 5e-2)) {
                bad++;
                fprintf(stderr, "fmm adaptive %d cap %d: rel err %.3e\n", ad, cap, sqrt(e / r));
            }
            for (int c = 0; c < nc; ++c) {
                int depth;
                int64_t nt, ns;
                uint64_t tk[N], sk[N];
                int tl[N], sl[N];
                double root[4];
                if (orc_component_tree(3, eps, lam, d, N, x, y, z, c, cap, ad, &depth, &nt, &ns, tk, sk, tl, sl, root))
                    bad++;
            }
        }
    uint32_t sc[3 * N], tc[3 * N];
    for (int i = 0; i < N; ++i) {
        sc[i] = (uint32_t)(65535.0 * urand(&s));
        sc[N + i] = (uint32_t)(30000 + 2000 * urand(&s));
        sc[2 * N + i] = (uint32_t)(32768 + 3000 * urand(&s));
        tc[i] = (uint32_t)(65535.0 * urand(&s));
        tc[N + i] = (uint32_t)(30000 + 2000 * urand(&s));
        tc[2 * N + i] = (uint32_t)(32767 - 3000 * urand(&s));
    }
    int* cover = malloc(sizeof(int) * N * N);
    long long cnt[4];
    for (int sep = 0; sep <= 1; ++sep) {
        if (orc_list_coverage(N, sc, N, tc, 5, 1, sep, 0, cover, cnt)) bad++;
        for (int i = 0; i < N * N; ++i)
            if (cover[i] != 1) {
                bad++;
                break;
            }
    }
    const double rs[3] = {0.625, 0.5, -0.1}, cs[3] = {0.6, 0.52, -0.3}, ct[3] = {0.63, 0.5, 0.25},
                 rt[3] = {0.66, 0.48, 0.27}, c0[3] = {0, 0, 0}, r0[3] = {0.3, 0.1, 0.25}, s0[3] = {0.05, 0.02, -0.03};
    for (int mode = 0; mode <= 1; ++mode) {
        double v = orc_reaction_point_chain(eps, lam, d, 2, 1, 1, 1, 1, 6, rs, mode ? ct : cs, mode ? rt : ct, 0.1, mode);
        if (!isfinite(v)) bad++;
        if (!isfinite(orc_free_point_chain(6, 1.2, mode ? r0 : s0, c0, mode ? s0 : r0, mode))) bad++;
    }
    double* tab = malloc(sizeof(double) * 4 * 12 * 12);
    for (int mode = 0; mode <= 2; ++mode)
        orc_sommerfeld_table(eps, lam, d, 2, 1, 1, 1, 1, 0.003, 0.04, -0.06, 0.1, 11, mode, tab);
    free(tab);
    free(cover);
    free(cphi);
    free(st);
    printf("oracle sanitizer driver: %d failures\n", bad);
    return bad ? 1 : 0;
}
