"""Pins of the oracle on stacks of any number of layers (Sec. 2.1: the
paper gives the Green's function of a general stack, eqs. greenfuncomponent
and totaldensity, but writes the reaction densities out only for three
layers).  The oracle's densities come from a generalized reflection
recursion; here they meet (i) the paper's three-layer closed forms, (ii) an
independent dense solve of the transmission conditions for 2, 4 and 5
layers, and the full layered Green's function meets (iii) the homogeneous
stack, where the reaction parts must rebuild or cancel the free-space kernel
(eq. sommerfeldid), and (iv) a stack with an interface between two identical
layers, which must equal the stack without it.  The oracle FMM on a 4-layer
and a 2-layer problem then converges geometrically in p to the oracle's
direct sum."""
import itertools

import numpy as np
import pytest

import transmission

MED3 = ((1.0, 8.6, 20.5), (1.2, 0.5, 2.1), (0.0, -1.2))


def comps(nl):
    L = nl - 1
    for l, lp, a, b in itertools.product(range(nl), range(nl), (1, 2), (1, 2)):
        if (a == 1 and l >= L) or (a == 2 and l <= 0) or (b == 1 and lp >= L) or (b == 2 and lp <= 0):
            continue
        yield l, lp, a, b


def test_recursion_equals_three_layer_closed_forms(orc):
    ly = orc.Layers(*MED3)
    worst = 0.0
    for l, lp, a, b in comps(3):
        for lr in (0.0, 0.3, 2.0, 17.0, 300.0, 5000.0):
            s3 = orc.sigma3(ly, l, lp, a, b, lr)
            sr = orc.sigma_stack(ly, l, lp, a, b, lr)
            assert np.isfinite(sr)
            worst = max(worst, abs(sr - s3) / max(abs(s3), 1e-300) if s3 != 0 else abs(sr))
    assert worst <= 1e-12, worst


@pytest.mark.parametrize("nl", [2, 4, 5])
def test_recursion_equals_dense_transmission_solve(orc, nl):
    rng = np.random.default_rng(nl)
    eps = rng.uniform(1, 30, nl)
    lam = rng.uniform(0.4, 2.5, nl)
    d = -np.cumsum(np.concatenate([[0.0], rng.uniform(0.5, 1.5, nl - 2)]))
    ly = orc.Layers(eps, lam, d)
    for lr in (0.0, 0.4, 1.5, 3.0):
        for lp in range(nl):
            for b in (1, 2):
                if (b == 1 and lp >= nl - 1) or (b == 2 and lp == 0):
                    continue
                A, B = transmission.solve(eps, lam, d, lr, lp, b)
                scale = max(max(abs(v) for v in A.values()), max(abs(v) for v in B.values()))
                for l in range(nl):
                    for a, ref in ((1, A.get(l)), (2, B.get(l))):
                        if ref is None:
                            continue
                        got = orc.sigma_stack(ly, l, lp, a, b, lr)
                        assert abs(got - ref) <= 1e-12 * abs(ref) + 1e-14 * scale, (l, lp, a, b, lr, got, ref)


def _layered_green(orc, ly, r, rp):
    """u_{l l'}(r, r') of eq. layeredGreensfun: reaction components summed,
    plus the free-space kernel when source and target share a layer."""
    nl = ly.nlayers
    bounds = [np.inf] + list(ly.d) + [-np.inf]
    l = next(k for k in range(nl) if bounds[k + 1] < r[2] < bounds[k])
    lp = next(k for k in range(nl) if bounds[k + 1] < rp[2] < bounds[k])
    g = sum(orc.reaction_u(ly, l, lp, a, b, r, rp) for (ll, llp, a, b) in comps(nl) if (ll, llp) == (l, lp))
    if l == lp:
        R = np.linalg.norm(np.subtract(r, rp))
        g += np.exp(-ly.lam[l] * R) / (4 * np.pi * ly.eps[l] * R)
    return g


PTS = [((0.1, -0.2, 0.3), (-0.3, 0.25, 0.6)), ((0.2, 0.1, 0.4), (0.0, -0.1, -0.5)),
       ((0.3, 0.0, -0.8), (-0.2, 0.2, -2.9)), ((-0.1, 0.4, -1.7), (0.2, 0.1, -1.4)),
       ((0.05, 0.05, -3.2), (0.3, -0.3, 0.9))]


def test_homogeneous_stack_is_free_space(orc):
    # identical layers: the layered kernel is e^{-lam r}/(4 pi eps r) for every pair of layers
    ly = orc.Layers([2.5] * 4, [1.3] * 4, [0.0, -1.2, -2.4])
    for r, rp in PTS:
        R = np.linalg.norm(np.subtract(r, rp))
        ref = np.exp(-1.3 * R) / (4 * np.pi * 2.5 * R)
        assert abs(_layered_green(orc, ly, r, rp) - ref) <= 1e-12 * ref, (r, rp)


def test_interface_between_identical_layers_is_invisible(orc):
    # layers 1 and 2 of the 4-layer stack are the same material: its kernel equals the
    # 3-layer stack without the interface at z = -1.2 (middle layer -2.4 < z < 0)
    eps4, lam4 = (1.0, 3.0, 3.0, 7.0), (1.2, 0.9, 0.9, 2.0)
    ly4 = orc.Layers(eps4, lam4, [0.0, -1.2, -2.4])
    ly3 = orc.Layers((1.0, 3.0, 7.0), (1.2, 0.9, 2.0), [0.0, -2.4])
    for r, rp in PTS + [((0.0, 0.1, -0.3), (0.2, 0.0, -2.0)), ((0.1, 0.1, -1.9), (0.0, 0.3, -0.7))]:
        g4 = _layered_green(orc, ly4, r, rp)
        g3 = _layered_green(orc, ly3, r, rp)
        assert abs(g4 - g3) <= 1e-12 * abs(g3), (r, rp, g4, g3)


@pytest.mark.parametrize("nl", [2, 4])
def test_fmm_on_stacks_converges_to_direct_sum(orc, nl):
    from paper_2002_01334_amd import inputs

    prob = inputs.stack(120, nl, seed=5)
    ly = orc.Layers(prob.eps, prob.lam, prob.d)
    direct = orc.direct_sum(ly, prob.x, prob.y, prob.z, prob.q)
    errs = []
    for p in (3, 6, 10):
        phi = orc.fmm(ly, prob.x, prob.y, prob.z, prob.q, p, leaf_cap=8)
        errs.append(max(np.linalg.norm(phi[prob.layer == l] - direct[prob.layer == l]) /
                        np.linalg.norm(direct[prob.layer == l]) for l in range(nl)))
    assert errs[0] < 1e-2 and errs[1] < errs[0] / 10 and errs[2] < errs[1] / 10 and errs[2] < 1e-5, errs
