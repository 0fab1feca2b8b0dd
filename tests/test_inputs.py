"""Host checks of the seeded workload recipes (no GPU): the paper's test
problem of Sec. 4 (P_4-shaped bodies in three layers)."""
import numpy as np

from paper_2002_01334_amd import inputs


def test_p4_body_volume_closed_forms():
    # a = 0: the sphere of radius 1/2
    assert abs(inputs.p4_volume(0.0) - np.pi / 6.0) < 1e-15
    # the polar radius is 1/2 for every a (P_4(1) = 1), the equatorial one 1/2 - 5a/8 (P_4(0) = 3/8)
    for a in inputs.PAPER_A:
        assert abs(inputs.p4_radius(a, 1.0) - 0.5) < 1e-15
        assert abs(inputs.p4_radius(a, 0.0) - (0.5 - 5.0 * a / 8.0)) < 1e-15
    # volume against a midpoint rule in cos(theta) (independent of the Gauss rule)
    c = (np.arange(200_000) + 0.5) / 100_000 - 1.0
    for a in inputs.PAPER_A:
        mid = 2.0 * np.pi / 3.0 * np.sum(inputs.p4_radius(a, c) ** 3) * (2.0 / len(c))
        assert abs(mid - inputs.p4_volume(a)) < 1e-9


def test_paper_domains_counts_geometry_and_seed():
    n = 30_000
    prob = inputs.paper_domains(n, seed=0)
    assert prob.n == n and list(prob.eps) == [1.0, 8.6, 20.5] and list(prob.lam) == [1.2, 0.5, 2.1]
    counts = np.bincount(prob.layer, minlength=3)
    vol = np.array([inputs.p4_volume(a) for a in inputs.PAPER_A])
    assert np.all(np.abs(counts - n * vol / vol.sum()) <= 3)
    for l, (a, zc) in enumerate(zip(inputs.PAPER_A, inputs.PAPER_ZC)):
        m = prob.layer == l
        dx, dy, dz = prob.x[m], prob.y[m], prob.z[m] - zc
        rho = np.sqrt(dx * dx + dy * dy + dz * dz)
        assert np.all(rho < inputs.p4_radius(a, dz / rho) + 1e-15)
        # inside the layer, clear of the interfaces z = 0 and -1.2 by 0.1 - rounding
        lo, hi = zc - 0.5, zc + 0.5
        assert prob.z[m].min() >= lo - 1e-12 and prob.z[m].max() <= hi + 1e-12
        assert np.all(np.abs(prob.q[m]) <= 1.0)
        # uniform in the body: the mean offset is near the centre
        assert abs(dx.mean()) < 0.02 and abs(dy.mean()) < 0.02 and abs(dz.mean()) < 0.02
    again = inputs.paper_domains(n, seed=0)
    assert np.array_equal(prob.x, again.x) and np.array_equal(prob.q, again.q)
    other = inputs.paper_domains(n, seed=1)
    assert not np.array_equal(prob.x, other.x)
    fixed = inputs.paper_domains(per_layer=(912, 640, 1296))
    assert list(np.bincount(fixed.layer)) == [912, 640, 1296]
