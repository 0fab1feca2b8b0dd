"""Independent reference for the reaction densities: solve the transmission
conditions of the layered problem (Sec. 2.1: continuity of u and of
eps du/dz at every interface, decay at +-infinity) in the spectral domain,
for one lambda_rho, as a dense linear system.

In layer l the spectral field is
    u_l(z) = [l == l'] e^{-lz_l' |z - z'|} / (eps_l' lz_l')
             + A_l e^{-lz_l (z - d_l)} / lz_l + B_l e^{-lz_l (d_{l-1} - z)} / lz_l
(A_L = 0, B_0 = 0), and A_l, B_l are linear in the two source exponentials
X_1 = e^{-lz_l'(z' - d_l')} and X_2 = e^{-lz_l'(d_{l'-1} - z')}; sigma^{1b}_{l l'}
is the coefficient of X_b in A_l and sigma^{2b}_{l l'} the one in B_l."""
import numpy as np


def solve(eps, lam, d, lrho, lp, b):
    L = len(d)
    lz = np.sqrt(np.asarray(lam, float) ** 2 + lrho ** 2)
    nu = 2 * L

    def iA(l):
        return l

    def iB(l):
        return L + l - 1

    M = np.zeros((nu, nu))
    rhs = np.zeros(nu)
    for i in range(L):
        rv, rf = 2 * i, 2 * i + 1
        M[rv, iA(i)] += 1 / lz[i]
        M[rf, iA(i)] += -eps[i]
        if i >= 1:
            e = np.exp(-lz[i] * (d[i - 1] - d[i]))
            M[rv, iB(i)] += e / lz[i]
            M[rf, iB(i)] += eps[i] * e
        if i + 1 < L:
            e = np.exp(-lz[i + 1] * (d[i] - d[i + 1]))
            M[rv, iA(i + 1)] -= e / lz[i + 1]
            M[rf, iA(i + 1)] += eps[i + 1] * e
        M[rv, iB(i + 1)] -= 1 / lz[i + 1]
        M[rf, iB(i + 1)] -= eps[i + 1]
        if lp == i and b == 1:
            rhs[rv] -= 1 / (eps[lp] * lz[lp])
            rhs[rf] -= eps[i] / eps[lp]
        if lp == i + 1 and b == 2:
            rhs[rv] += 1 / (eps[lp] * lz[lp])
            rhs[rf] -= eps[i + 1] / eps[lp]
    sol = np.linalg.solve(M, rhs)
    A = {l: sol[iA(l)] for l in range(L)}
    B = {l: sol[iB(l)] for l in range(1, L + 1)}
    return A, B
