"""Pins of the oracle's adaptive trees (Sec. 3.5, closing remarks on adaptive
trees): the U-, V-, W- and X-lists cover every (target, source) pair exactly
once, and the FMM on adaptive trees (point forms M2P / P2L on the W- and
X-lists) converges geometrically in p to the direct sum on clustered input,
component by component in agreement with the FMM on uniform trees."""
import numpy as np
import pytest

from paper_2002_01334_amd import inputs


def _cells(rng, n, centre, spread):
    a = rng.integers(0, 65536, (n // 2, 3))
    b = np.clip(rng.normal(centre, spread, (n - n // 2, 3)), 0, 65535).astype(np.int64)
    return np.vstack([a, b])


@pytest.mark.parametrize("sep", [False, True])
@pytest.mark.parametrize("cap", [1, 6, 30])
@pytest.mark.parametrize("same", [False, True])
def test_lists_cover_every_pair_exactly_once(orc, cap, same, sep):
    # Clustered sources and targets (half uniform, half a tight Gaussian cluster, a different
    # cluster for the targets) on the fine grid: every pair must be covered by exactly one V,
    # U, W or X entry; a dropped or doubled list entry anywhere breaks this (also with the
    # reaction sets' extra division near the plane z cell 32767 | 32768, sep).  The uniform
    # tree at a fixed depth is covered too (no W or X entries).
    rng = np.random.default_rng(cap)
    s = _cells(rng, 600, 20000, 1500)
    t = s if same else _cells(rng, 450, 26000, 2500)
    cov, cnt = orc.list_coverage(s, t, cap, adaptive=True, sep=sep)
    assert cov.min() == 1 and cov.max() == 1
    assert cnt[1] > 0 and cnt[2] > 0 and cnt[3] > 0, cnt
    if same:
        assert cnt[2] == cnt[3]
    for H in (2, 4):
        cov, cnt = orc.list_coverage(s, t, cap, adaptive=False, H=H)
        assert cov.min() == 1 and cov.max() == 1 and cnt[2] == 0 and cnt[3] == 0


def test_adaptive_fmm_converges_to_direct_sum(orc):
    # Three layers, 120 charges each, half of them in a tight cluster next to an interface.
    # Trees by occupancy alone (mode 2, leaf cap 10): W- and X-lists in the free-space and in
    # the reaction components, so the reaction point forms carry much of the potential; the FMM
    # must decay geometrically in p to the direct sum, and agree with the uniform-tree FMM
    # component by component at p = 9 (both within truncation error of the same sum).  Mode 1
    # (reaction sets also divided near the interface) converges to the same sum.
    pr = inputs.three_layer_interface_clusters(120, seed=5)
    ly = orc.Layers(pr.eps, pr.lam, pr.d)
    d = orc.direct_sum(ly, pr.x, pr.y, pr.z, pr.q)
    errs = []
    for p in (3, 6, 9):
        phi, cphi, st = orc.fmm(ly, pr.x, pr.y, pr.z, pr.q, p, leaf_cap=10, components=True, adaptive=2)
        errs.append(np.linalg.norm(phi - d) / np.linalg.norm(d))
    assert errs[0] < 1e-2 and errs[1] < errs[0] / 10 and errs[2] < errs[1] / 5 and errs[2] < 1e-5, errs
    assert st[0, 6] > 0 and st[0, 7] > 0
    react = st[3:]
    assert (react[:, 6] > 0).sum() >= 4 and (react[:, 7] > 0).sum() >= 4
    uphi, ucphi, ust = orc.fmm(ly, pr.x, pr.y, pr.z, pr.q, 9, leaf_cap=10, components=True)
    assert ust[:, 6].sum() == 0 and ust[:, 7].sum() == 0
    for c in range(cphi.shape[0]):
        nrm = np.linalg.norm(ucphi[c])
        if nrm > 0:
            assert np.linalg.norm(cphi[c] - ucphi[c]) <= 1e-4 * nrm, (c, np.linalg.norm(cphi[c] - ucphi[c]) / nrm)
    phi1, _, st1 = orc.fmm(ly, pr.x, pr.y, pr.z, pr.q, 9, leaf_cap=10, components=True, adaptive=1)
    assert np.linalg.norm(phi1 - d) / np.linalg.norm(d) < 1e-5
    # the separation rule removes most reaction near-field pairs
    assert st1[3:, 4].sum() < react[:, 4].sum() / 10
