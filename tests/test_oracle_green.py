"""Pins of the oracle's layered Green's function: reaction densities
(eqs. densitythreelayer1-3) against an independent transmission-condition
solve, the Sommerfeld identity (eq. sommerfeldid) through the homogeneous
medium, and the equal-lambda image series."""
import numpy as np
import pytest

from tests import transmission

MEDIA = [
    ((1.0, 2.0, 4.0), (1.2, 1.5, 2.0), (0.0, -1.2)),
    ((1.0, 8.6, 20.5), (1.2, 0.5, 2.1), (0.0, -1.2)),       # the paper's Sec. 4 medium
    ((70.0, 3.0, 30.0), (0.6, 2.4, 1.1), (0.5, -0.3)),      # thin middle layer, d_0 != 0
]

COMPS = [(l, lp, a, b) for l in range(3) for lp in range(3) for a in (1, 2) for b in (1, 2)
         if not ((a == 1 and l >= 2) or (a == 2 and l <= 0) or (b == 1 and lp >= 2) or (b == 2 and lp <= 0))]


def test_sixteen_components():
    assert len(COMPS) == 16


@pytest.mark.parametrize("medium", MEDIA)
def test_sigma_matches_transmission_solve(orc, medium):
    ly = orc.Layers(*medium)
    for lrho in (0.0, 0.05, 0.7, 3.0, 25.0):
        for (l, lp, a, b) in COMPS:
            A, B = transmission.solve(ly.eps, ly.lam, ly.d, lrho, lp, b)
            ref = A[l] if a == 1 else B[l]
            assert orc.sigma3(ly, l, lp, a, b, lrho) == pytest.approx(ref, rel=1e-12, abs=1e-300)


def test_sigma_no_overflow_at_large_lrho(orc):
    ly = orc.Layers(*MEDIA[1])
    for (l, lp, a, b) in COMPS:
        v = orc.sigma3(ly, l, lp, a, b, 5000.0)
        assert np.isfinite(v)


def test_sommerfeld_identity_through_homogeneous_medium(orc):
    # identical layers: sigma = 1/eps for the cross-layer transmission components and 0 for
    # same-layer reflection, so the reaction parts of a cross-layer pair add up to
    # e^{-lam r}/(4 pi eps r) (eq. sommerfeldid) and a same-layer reaction vanishes.
    hom = orc.Layers((3.0, 3.0, 3.0), (1.3, 1.3, 1.3), (0.0, -1.2))
    rng = np.random.default_rng(0)
    zr = {0: (0.05, 1.0), 1: (-1.15, -0.05), 2: (-2.5, -1.25)}
    for l in range(3):
        for lp in range(3):
            r = np.r_[rng.uniform(-0.5, 0.5, 2), rng.uniform(*zr[l])]
            rp = np.r_[rng.uniform(-0.5, 0.5, 2), rng.uniform(*zr[lp])]
            tot = sum(orc.reaction_u(hom, l, lp, a, b, r, rp) for (L_, LP_, a, b) in COMPS if (L_, LP_) == (l, lp))
            R = np.linalg.norm(r - rp)
            ref = np.exp(-1.3 * R) / (4 * np.pi * 3.0 * R) if l != lp else 0.0
            assert tot == pytest.approx(ref, rel=1e-13, abs=1e-17)


def test_equal_lambda_image_series(orc):
    # equal lambda, different eps: u^{11}_{11} = sum_k (R2/eps1) (R0 R2)^k e^{-lam R_k}/(4 pi R_k),
    # R_k^2 = rho^2 + (tau + tau' + 2kD)^2, R0 = (e1-e0)/(e1+e0), R2 = (e1-e2)/(e1+e2)
    e0, e1, e2, lam, D = 1.0, 5.0, 2.0, 1.1, 1.2
    ly = orc.Layers((e0, e1, e2), (lam, lam, lam), (0.0, -D))
    R0 = (e1 - e0) / (e1 + e0)
    R2 = (e1 - e2) / (e1 + e2)
    for r, rp in [((0.1, 0.05, -0.4), (-0.2, 0.1, -0.9)), ((0.0, 0.0, -0.2), (0.0, 0.0, -0.2))]:
        r, rp = np.array(r), np.array(rp)
        tau, taup = r[2] + D, rp[2] + D
        rho = np.hypot(*(r[:2] - rp[:2]))
        k = np.arange(300)
        Rk = np.sqrt(rho ** 2 + (tau + taup + 2 * k * D) ** 2)
        ref = np.sum((R2 / e1) * (R0 * R2) ** k * np.exp(-lam * Rk) / (4 * np.pi * Rk))
        assert orc.reaction_u(ly, 1, 1, 1, 1, r, rp) == pytest.approx(ref, rel=1e-13)


def test_direct_sum_homogeneous_equals_free_space(orc):
    # whole-problem pin: with identical layers the layered potential equals the
    # free-space screened Coulomb sum over all charges
    from paper_2002_01334_amd import inputs

    pr = inputs.three_layer(12, seed=5)
    hom = orc.Layers((2.5, 2.5, 2.5), (0.9, 0.9, 0.9), pr.d)
    phi = orc.direct_sum(hom, pr.x, pr.y, pr.z, pr.q)
    P = np.stack([pr.x, pr.y, pr.z], 1)
    R = np.linalg.norm(P[:, None] - P[None], axis=2)
    np.fill_diagonal(R, np.inf)
    ref = (np.exp(-0.9 * R) / (4 * np.pi * 2.5 * R)) @ pr.q
    assert np.allclose(phi, ref, rtol=1e-12, atol=1e-15)
