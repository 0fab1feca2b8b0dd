"""Pins of the oracle's point forms for adaptive trees (Sec. 3.5, closing
remarks): the multipole expansion evaluated at a target (M2P, W-list) and the
local expansion formed from a source (P2L, X-list), free space
(eqs. freespace3dmulexp, melecoeffree) and reaction (the F~ and L rows of eq.
coefintable), and the point table of scaled Sommerfeld integrals that mixes
the forward (eq. recurrence1) and backward (eq. backwardrecurrence1)
recurrences, against direct quadrature of every entry."""
import numpy as np
import pytest
from scipy import special as sp

MED = ([1.0, 8.6, 20.5], [1.2, 0.5, 2.1], [0.0, -1.2])
COMPS = [(1, 1, 1, 1), (1, 1, 2, 2), (0, 1, 1, 1), (2, 1, 2, 2), (0, 2, 1, 2)]


def test_free_point_forms_converge_to_k0(orc):
    lam = 1.2
    rs = np.array([0.05, 0.02, -0.03])
    r = np.array([0.3, 0.1, 0.25])
    c = np.zeros(3)
    ex = sp.spherical_kn(0, lam * np.linalg.norm(r - rs))
    for mode, (a, b) in ((0, (rs, r)), (1, (r, rs))):
        # mode 0: ME about c of a source near c, evaluated at a far target;
        # mode 1: LE about c of a far source, evaluated near c
        e = [abs(orc.free_point_chain(p, lam, a, c, b, mode) - ex) / ex for p in (2, 5, 8, 11)]
        assert e[0] < 1e-2 and e[1] < e[0] / 100 and e[2] < e[1] / 100 and e[3] < 1e-11, (mode, e)


def _geom(ly, comp):
    l, lp, a, b = comp
    zsrc = {0: 0.4, 1: -0.1, 2: -1.5}[lp]
    rs = np.array([0.625, 0.5, zsrc])
    ts = (rs[2] - ly.d[lp]) if b == 1 else (ly.d[lp - 1] - rs[2])
    zimg = ly.d[l] - ts if a == 1 else ly.d[l - 1] + ts
    iface = ly.d[l] if a == 1 else ly.d[l - 1]
    sgn = 1 if a == 1 else -1
    return rs, zimg, iface, sgn


@pytest.mark.parametrize("geo", [(0.125, 0.02), (0.125, 0.2), (0.25, 0.0)])
@pytest.mark.parametrize("comp", COMPS)
def test_reaction_point_forms_converge_to_quadrature(orc, comp, geo):
    # Sec. 3.4 medium, source r' in layer lp.  M2P: ME about an image-side centre c, evaluated
    # at a target whose horizontal distance from c is 0.02 (below the box side S: backward
    # recurrence), 0.2 (above: forward) or 0 (J_m(0) = 0).  P2L: LE about a target-side
    # centre at the same horizontal distances from the image, evaluated near the centre.  Both
    # must converge geometrically in p to the direct Sommerfeld quadrature of u~^{ab} (a wrong
    # sign of the 2b rows, a swapped height pair or a wrong recurrence leaves O(1) errors).
    ly = orc.Layers(*MED)
    l, lp, a, b = comp
    S, dxy = geo
    rs, zimg, iface, sgn = _geom(ly, comp)
    c = np.array([0.6, 0.52, zimg - sgn * 0.03])
    r = np.array([0.6 + dxy, 0.52, iface + sgn * 0.25])
    ex = orc.reaction_u(ly, l, lp, a, b, r, rs)
    e = [abs(orc.reaction_point_chain(ly, l, lp, a, b, p, rs, c, r, S, 0) - ex) / abs(ex) for p in (2, 5, 8, 11)]
    assert e[0] < 1e-2 and e[1] < e[0] / 100 and e[3] < e[1] / 1e4 and e[3] < 1e-10, ("m2p", e)
    ct = np.array([0.625 + dxy, 0.5, iface + sgn * 0.25])
    rt = ct + np.array([0.03, -0.02, 0.02])
    ex = orc.reaction_u(ly, l, lp, a, b, rt, rs)
    e = [abs(orc.reaction_point_chain(ly, l, lp, a, b, p, rs, ct, rt, S, 1) - ex) / abs(ex) for p in (2, 5, 8, 11)]
    assert e[0] < 1e-2 and e[1] < e[0] / 100 and e[3] < e[1] / 1e4 and e[3] < 1e-10, ("p2l", e)


@pytest.mark.parametrize("frac", [0.0, 0.01, 0.3, 0.9, 1.5])
@pytest.mark.parametrize("comp", [(1, 1, 1, 1), (2, 1, 2, 2), (0, 2, 1, 2)])
def test_point_table_matches_direct_quadrature(orc, comp, frac):
    # Every entry S^n Sc_{nm,ij}, n <= p + 2 = 10, of the point table (initial values m = 0, 1
    # and the row n = 10 by quadrature; forward recurrence where 2m/a_{n+m} < rho/S, backward
    # elsewhere) against direct quadrature of eq. M2Ltable: within 1e-13 of the largest entry
    # of the rows up to it, and entries at least 1e-3 of their row's largest within 1e-6
    # relative.  rho = 0.01 S is where the forward recurrence alone loses every digit.
    ly = orc.Layers(*MED)
    l, lp, a, b = comp
    S = 0.1
    iface = ly.d[l] if a == 1 else ly.d[l - 1]
    sgn = 1 if a == 1 else -1
    zt, zs = iface + sgn * 0.4 * S, iface - sgn * 0.6 * S
    nmax = 10
    pt, _ = orc.sommerfeld_table(ly, l, lp, a, b, frac * S, zt, zs, S, nmax, 2)
    dirt, _ = orc.sommerfeld_table(ly, l, lp, a, b, frac * S, zt, zs, S, nmax, 1)
    for i in range(2):
        for j in range(2):
            upto = 0.0
            for n in range(nmax + 1):
                row = np.abs(dirt[i, j, n, : n + 1]).max()
                upto = max(upto, row)
                err = np.abs(pt[i, j, n, : n + 1] - dirt[i, j, n, : n + 1]).max()
                assert err <= 1e-13 * upto, (i, j, n, err, upto)
                d = dirt[i, j, n, : n + 1]
                sig = np.abs(d) >= 1e-3 * row
                rel = np.abs(pt[i, j, n, : n + 1] - d)[sig] / np.abs(d[sig])
                assert rel.max() <= 1e-6, (i, j, n, rel.max())
    if frac == 0.01:
        fwd, unstable = orc.sommerfeld_table(ly, l, lp, a, b, frac * S, zt, zs, S, nmax, 0)
        assert unstable == 1
        # the forward recurrence alone misses the bound the point table meets by far
        assert np.abs(fwd - dirt).max() > 1e-3 * np.abs(dirt).max()


@pytest.mark.parametrize("frac", [0.0, 0.05, 0.5, 2.0])
def test_point_I_rows_match_direct_Q(orc, frac):
    # The I entries the point forms use, I_{00,nu mu} (M2P) and I_{nm,00} (P2L), n, nu <= 8,
    # assembled from the point table (eq. metoletableform) against direct quadrature of eq.
    # uniformintegral with Q = P^ P^, within 1e-10 of the largest entry of the row (the direct
    # side rounds at up to ~1e-11 of it where its integrand cancels; observed <= 7e-12).
    ly = orc.Layers(*MED)
    for comp in ((1, 1, 1, 1), (2, 1, 2, 2)):
        l, lp, a, b = comp
        S = 0.1
        iface = ly.d[l] if a == 1 else ly.d[l - 1]
        sgn = 1 if a == 1 else -1
        zt, zs = iface + sgn * 0.5 * S, iface - sgn * 0.5 * S
        for which in (0, 1):
            vals = []
            for n in range(9):
                for m in range(-n, n + 1):
                    idx = (0, 0, n, m) if which == 0 else (n, m, 0, 0)
                    vals.append(orc.reaction_I_point(ly, l, lp, a, b, 8, frac * S, zt, zs, S, *idx))
            v = np.array([x[0] for x in vals])
            w = np.array([x[1] for x in vals])
            assert np.abs(v - w).max() <= 1e-10 * np.abs(w).max(), (comp, which, np.abs(v - w).max() / np.abs(w).max())
