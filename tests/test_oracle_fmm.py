"""Pins of the oracle FMM (Algorithms 1 and 2) against the oracle direct sum,
which is itself pinned by tests/test_oracle_green.py: geometric decay of the
error in p, the homogeneous-medium limit against a numpy free-space sum, and
the bookkeeping of the 3 + 16 components."""
import numpy as np
import pytest

from paper_2002_01334_amd import inputs


def _err2(phi, ref, layer):
    return [np.linalg.norm(phi[layer == l] - ref[layer == l]) / np.linalg.norm(ref[layer == l]) for l in range(3)]


@pytest.fixture(scope="module")
def small(orc):
    pr = inputs.three_layer(40, seed=0)
    ly = orc.Layers(pr.eps, pr.lam, pr.d)
    ref = orc.direct_sum(ly, pr.x, pr.y, pr.z, pr.q)
    return pr, ly, ref


def test_fmm_error_decays_geometrically_in_p(orc, small):
    pr, ly, ref = small
    errs = []
    for p in (2, 5, 8, 11):
        phi, cphi, st = orc.fmm(ly, pr.x, pr.y, pr.z, pr.q, p, leaf_cap=4, components=True)
        errs.append(max(_err2(phi, ref, pr.layer)))
        assert np.all(st[:, 5] == 0)           # recurrence stability bound never violated
        assert np.all(st[:, 0] >= 2)           # the far field is exercised in every component
        assert np.all(st[3:, 3] > 0)           # every reaction component has M2L pairs
    assert errs[0] < 5e-2
    for a, b in zip(errs, errs[1:]):
        assert b < a / 8
    assert errs[-1] < 5e-6


def test_fmm_components_sum_and_targets(orc, small):
    pr, ly, ref = small
    phi, cphi, st = orc.fmm(ly, pr.x, pr.y, pr.z, pr.q, 6, leaf_cap=8, components=True)
    assert np.allclose(cphi.sum(0), phi, rtol=0, atol=1e-15)
    for c in range(cphi.shape[0]):
        kind, l, lp, a, b = orc.component(3, c)
        assert np.all(cphi[c][pr.layer != l] == 0.0)


def test_fmm_without_far_field_equals_direct_sum(orc):
    # every charge 0.625 from the interfaces of its layer and x, y within +-0.3:
    # the reaction grid's half side equals the smallest tau, so with a leaf cap
    # above every layer's size every tree has depth <= 1, every interaction is
    # near field and the FMM reduces to the direct sum
    rng = np.random.default_rng(3)
    n = 40
    x, y = rng.uniform(-0.3, 0.3, (2, 3 * n))
    z = np.repeat([0.625, -0.625, -1.875], n)
    q = rng.uniform(-1, 1, 3 * n)
    ly = orc.Layers((1.0, 2.0, 4.0), (1.2, 1.5, 2.0), (0.0, -1.25))
    ref = orc.direct_sum(ly, x, y, z, q)
    phi, cphi, st = orc.fmm(ly, x, y, z, q, 4, leaf_cap=1000, components=True)
    assert np.all(st[:, 0] <= 1)
    assert np.allclose(phi, ref, rtol=1e-12, atol=1e-14)


def test_fmm_homogeneous_medium_equals_free_space(orc):
    pr = inputs.three_layer(30, seed=7)
    hom = orc.Layers((2.0, 2.0, 2.0), (1.4, 1.4, 1.4), pr.d)
    P = np.stack([pr.x, pr.y, pr.z], 1)
    R = np.linalg.norm(P[:, None] - P[None], axis=2)
    np.fill_diagonal(R, np.inf)
    ref = (np.exp(-1.4 * R) / (4 * np.pi * 2.0 * R)) @ pr.q
    phi = orc.fmm(hom, pr.x, pr.y, pr.z, pr.q, 10, leaf_cap=6)
    assert max(_err2(phi, ref, pr.layer)) < 5e-6


def test_tree_depth_rule(orc):
    pr = inputs.three_layer(200, seed=0)
    ly = orc.Layers(pr.eps, pr.lam, pr.d)
    d0, tk, sk, root = orc.component_tree(ly, pr.x, pr.y, pr.z, 0, leaf_cap=50)
    assert d0 == 1 and len(tk) == 200                     # 200 charges, 8 boxes of <= 50 on average
    d3, tk, sk, root = orc.component_tree(ly, pr.x, pr.y, pr.z, 3, leaf_cap=50)
    assert root[2] == 0.0                                 # reaction root centred on the interface
    assert abs(root[3] - np.max(np.abs(pr.z[pr.layer == 0]))) < 1e-15
