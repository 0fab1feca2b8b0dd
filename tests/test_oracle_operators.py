"""Pins of the oracle's expansion operators: free-space addition theorems
(Thm 3.1-3.3) against direct evaluation, the modified Funk-Hecke expansion
(Prop. 3.2), the Legendre-product expansion behind C^s, the forward
recurrence (eq. recurrence1) against direct quadrature of every entry, and
the reaction ME -> M2L -> LE chain against direct Sommerfeld quadrature of
the reaction component."""
import numpy as np
import pytest
from scipy import special as sp

LAM = 1.3


def _iY(orc, n, m, v):
    return orc.bessel_i(n, LAM * np.linalg.norm(v)) * orc.ylm(n, v)[n * n + n + m]


def _kY(orc, n, m, v):
    return orc.bessel_k(n, LAM * np.linalg.norm(v)) * orc.ylm(n, v)[n * n + n + m]


@pytest.mark.parametrize("nm", [(0, 0), (2, 1), (3, -2), (4, 4), (5, -1)])
def test_regular_addition_theorem(orc, nm):
    n, m = nm
    b = np.array([0.3, -0.2, 0.5])
    r = np.array([0.1, 0.15, -0.05])
    s = orc.addition_sum(12, 12, LAM, n, m, b, r, 0)
    assert abs(s - _iY(orc, n, m, r + b)) < 1e-15


@pytest.mark.parametrize("nm", [(0, 0), (2, 1), (3, -2), (4, 4), (5, -1)])
def test_singular_addition_theorem_converges(orc, nm):
    n, m = nm
    b = np.array([0.8, -0.5, 0.6])
    r = np.array([0.1, 0.15, -0.05])
    ex = _kY(orc, n, m, r + b)
    errs = [abs(orc.addition_sum(p, max(p, n), LAM, n, m, b, r, 1) - ex) / abs(ex) for p in (6, 10, 14)]
    assert errs[0] < 1e-2 and errs[1] < errs[0] / 50 and errs[2] < errs[1] / 50 and errs[2] < 1e-8


def test_k0_addition_theorem_thm31(orc):
    # Thm 3.1, eq. sphbessel00: k0(lam|r1+b|) = 4pi sum (-1)^n k_n(lam b) conj(Y(b)) i_n(lam r1) Y(r1)
    b = np.array([0.7, 0.2, -0.4])
    r1 = np.array([0.05, -0.1, 0.12])
    Yb = orc.ylm(30, b)
    Yr = orc.ylm(30, r1)
    s = 0.0
    for n in range(31):
        kn = orc.bessel_k(n, LAM * np.linalg.norm(b))
        inn = orc.bessel_i(n, LAM * np.linalg.norm(r1))
        for m in range(-n, n + 1):
            s += 4 * np.pi * (-1) ** n * kn * np.conj(Yb[n * n + n + m]) * inn * Yr[n * n + n + m]
    assert s.real == pytest.approx(sp.spherical_kn(0, LAM * np.linalg.norm(r1 + b)), rel=1e-14)


def test_modified_funk_hecke_prop32(orc):
    # Prop 3.2: e^{lambda_vec . r} = sum conj(B_n^m(r)) P^_n^m(lz/lam) e^{i m alpha},
    # B = 4 pi (-1)^n i_n(lam r) Y_n^m, lambda_vec = (i lr cos a, i lr sin a, -lz)
    lam, lr, al = 1.1, 0.8, 0.7
    lz = np.hypot(lam, lr)
    r = np.array([0.12, -0.2, 0.15])
    lhs = np.exp(1j * lr * (r[0] * np.cos(al) + r[1] * np.sin(al)) - lz * r[2])
    Y = orc.ylm(40, r)
    s = 0.0
    for n in range(41):
        inn = orc.bessel_i(n, lam * np.linalg.norm(r))
        for m in range(-n, n + 1):
            B = 4 * np.pi * (-1) ** n * inn * Y[n * n + n + m]
            s += np.conj(B) * orc.plm_beyond(n, m, lz / lam) * np.exp(1j * m * al)
    assert abs(s - lhs) < 1e-13 * abs(lhs)


def test_legendre_product_expansion(orc):
    # P^_n^m(lz/l) P^_nu^mu(lz'/l') = sum_s C^s lr^{|m|+|mu|+2s} (l/lz)^i (l'/lz')^j
    worst = 0.0
    for n in range(0, 8):
        for m in range(-n, n + 1):
            for nu in range(0, 8, 3):
                for mu in range(-nu, nu + 1):
                    for lr in (0.05, 0.7, 3.0):
                        e, d = orc.legendre_product(n, m, nu, mu, 1.2, 0.5, lr)
                        worst = max(worst, abs(e - d) / abs(d))
    assert worst < 1e-12


MED = ((1.0, 8.6, 20.5), (1.2, 0.5, 2.1), (0.0, -1.2))


@pytest.mark.parametrize("geom", [(1, 3), (2, 3), (3, 1), (2, 2), (0, 2)])
@pytest.mark.parametrize("comp", [(1, 1, 1, 1), (1, 1, 2, 2), (0, 2, 1, 2), (2, 0, 2, 1)])
def test_recurrence_matches_direct_quadrature(orc, geom, comp):
    # V-list geometry of a level with box side S: rho = dx*S, centres (j+1/2) S and (k+1/2) S
    # from the interface.  Both sides are oscillatory integrals, so each is exact only to
    # ~1e-16 of the integral of |integrand|, which the largest entry of the rows n' <= n
    # stands in for: the recurrence must agree with direct quadrature of every Sc_{nm,ij}
    # to 1e-13 of that scale, and every entry at least 1e-3 of its row's largest must agree
    # to 1e-5 relative (a wrong recurrence coefficient fails both).
    ly = orc.Layers(*MED)
    l, lp, a, b = comp
    S = 0.1
    dx, dz = geom
    iface = ly.d[l] if a == 1 else ly.d[l - 1]
    sgn = 1 if a == 1 else -1
    zt = iface + sgn * (dz - 0.5) * S
    zs = iface - sgn * 0.5 * S
    nmax = 2 * 8 + 3
    rec, rc = orc.sommerfeld_table(ly, l, lp, a, b, dx * S, zt, zs, S, nmax, 0)
    dirt, _ = orc.sommerfeld_table(ly, l, lp, a, b, dx * S, zt, zs, S, nmax, 1)
    assert rc == 0
    for i in range(2):
        for j in range(2):
            upto = 0.0
            for n in range(nmax + 1):
                row = np.abs(dirt[i, j, n, : n + 1]).max()
                upto = max(upto, row)
                err = np.abs(rec[i, j, n, : n + 1] - dirt[i, j, n, : n + 1]).max()
                assert err <= 1e-13 * upto, (i, j, n, err, upto)
                d = dirt[i, j, n, : n + 1]
                sig = np.abs(d) >= 1e-3 * row
                rel = np.abs(rec[i, j, n, : n + 1] - d)[sig] / np.abs(d[sig])
                assert rel.max() <= 1e-5, (i, j, n, rel.max())


@pytest.mark.parametrize("geom", [(2, 2), (3, 1), (0, 3), (1, 3), (2, 3)])
@pytest.mark.parametrize("comp", [(1, 1, 1, 1), (1, 1, 2, 2), (0, 1, 1, 1), (2, 1, 2, 2), (0, 2, 1, 2),
                                  (2, 0, 2, 1)])
def test_reaction_I_recurrence_matches_direct_Q(orc, geom, comp):
    # The whole matrix I_{nm,nu mu}, n, nu <= 8, of a reaction M2L at a V-list geometry (box
    # side S, rho = dx S, target centre (dz - 1/2) S above the interface, image centre S/2
    # below; a = 1 and a = 2): the recurrence path (initial values by quadrature, eq.
    # recurrence1, C~^s assembly of eq. metoletableform) against direct quadrature of eq.
    # uniformintegral with Q = P^_n^m P^_nu^mu on the branch of eq. branch.  Both are exact up
    # to rounding, whose scale is the quadrature of the integrand's modulus (direct side) plus
    # the same recurrence run on moduli (recurrence side; it grows where the forward recurrence
    # in m amplifies earlier entries, at large |mu - m| and small rho / S).  Every entry must
    # agree within 1e-13 of that scale (observed <= 1.3e-15); entries with rho = 0 and mu != m
    # vanish on both sides.  A wrong coefficient, sign or index anywhere in either path leaves
    # errors of the order of |I| on the well-conditioned entries.
    ly = orc.Layers(*MED)
    l, lp, a, b = comp
    S = 0.1
    dx, dz = geom
    iface = ly.d[l] if a == 1 else ly.d[l - 1]
    sgn = 1 if a == 1 else -1
    zt = iface + sgn * (dz - 0.5) * S
    zs = iface - sgn * 0.5 * S
    rec, dirq, dabs, rbound, unstable = orc.reaction_I_both(ly, l, lp, a, b, 8, dx * S, zt, zs, S)
    assert unstable == 0
    scale = dabs + rbound
    zero = scale == 0
    assert np.all(rec[zero] == 0) and np.all(dirq[zero] == 0)
    err = np.abs(rec - dirq)[~zero] / scale[~zero]
    assert err.max() <= 1e-13, err.max()
    # and the well-conditioned entries (scale within 1e6 of |I|) agree to 1e-6 relative
    good = ~zero & (scale <= 1e6 * np.abs(dirq))
    assert good.sum() >= 0.5 * (~zero).sum()
    rel = np.abs(rec - dirq)[good] / np.abs(dirq[good])
    assert rel.max() <= 1e-6, rel.max()
    # the single-entry cross-check agrees with the matrix form
    for (n, m, nu, mu) in ((3, 1, 2, -2), (8, -3, 5, 4)):
        v, w = orc.reaction_I_pair(ly, l, lp, a, b, 8, dx * S, zt, zs, S, n, m, nu, mu)
        r, c = n * n + n + m, nu * nu + nu + mu
        assert v == rec[r, c] and w == dirq[r, c]


@pytest.mark.parametrize("comp", [(1, 1, 1, 1), (1, 1, 2, 2), (0, 1, 1, 1), (2, 1, 2, 2), (0, 2, 1, 2)])
def test_reaction_chain_converges_to_quadrature(orc, comp):
    # Sec. 3.4 example medium and source r' = (0.625, 0.5, -0.1) (middle layer where lp = 1);
    # ME about an image-side centre, M2L (eq. coefintable via the recurrence) to a target-side
    # centre, LE at r: error decays geometrically in p.
    ly = orc.Layers(*MED)
    l, lp, a, b = comp
    zsrc = {0: 0.4, 1: -0.1, 2: -1.5}[lp]
    rs = np.array([0.625, 0.5, zsrc])
    ts = (rs[2] - ly.d[lp]) if b == 1 else (ly.d[lp - 1] - rs[2])
    zimg = ly.d[l] - ts if a == 1 else ly.d[l - 1] + ts
    iface = ly.d[l] if a == 1 else ly.d[l - 1]
    sgn = 1 if a == 1 else -1
    cs = np.array([0.6, 0.6, zimg - sgn * 0.05])
    ct = np.array([0.3, 0.7, iface + sgn * 0.3])
    r = ct + np.array([0.05, -0.04, 0.03])
    ex = orc.reaction_u(ly, l, lp, a, b, r, rs)
    errs = []
    for p in (2, 5, 8, 11):
        v, unstable = orc.reaction_chain(ly, l, lp, a, b, p, rs, cs, ct, r)
        assert unstable == 0
        errs.append(abs(v - ex) / abs(ex))
    assert errs[3] < 1e-7 and errs[1] < errs[0] and errs[3] < errs[1] / 100, errs


def test_free_chain_p2m_m2l_l2p_and_shifts(orc):
    rs = np.array([0.05, 0.02, -0.03])
    cs = np.zeros(3)
    ct = np.array([1.0, 0.5, -0.5])
    r = ct + np.array([0.04, -0.05, 0.06])
    ex = sp.spherical_kn(0, LAM * np.linalg.norm(r - rs))
    e = [abs(orc.free_chain(p, LAM, rs, cs, ct, r) - ex) / ex for p in (2, 6, 10)]
    assert e[0] < 1e-3 and e[1] < e[0] / 1e3 and e[2] < 1e-11
    cs2 = np.array([0.1, 0.1, 0.1])
    ct2 = ct + np.array([-0.06, 0.06, 0.06])
    e = [abs(orc.free_chain(p, LAM, rs, cs, ct, r, cs2=cs2, ct2=ct2) - ex) / ex for p in (4, 8, 12)]
    assert e[1] < e[0] / 100 and e[2] < 1e-10
