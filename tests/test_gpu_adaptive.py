"""GPU parity of adaptive trees (Sec. 3.5, closing remarks on adaptive trees):
the leaves (levels and keys) against the oracle's, the FP64 path against the
oracle FMM on the same adaptive trees per output slot (<= 1e-10, which covers
the W-list M2P and X-list P2L point forms, free-space and reaction, and the
reaction point operators with their forward/backward recurrence tables), and
mixed precision against FP64 (<= 1e-6)."""
import numpy as np
import pytest

import oracle as O
from lpbtest import err2, run, slot_errors
from paper_2002_01334_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lpb():
    import torch

    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    from paper_2002_01334_amd import lpb as m

    m.load()
    return m


@pytest.fixture(scope="module")
def clustered():
    # 120 charges per layer, half in tight clusters next to the interfaces
    return inputs.three_layer_interface_clusters(120, seed=5)


@pytest.mark.parametrize("mode", [1, 2])
def test_adaptive_leaves_match_oracle(lpb, clustered, mode):
    prob = clustered
    ly = O.Layers(prob.eps, prob.lam, prob.d)
    ctx = lpb.Context(p=2, leaf_cap=10, adaptive=mode)
    ctx.set_layers(prob.eps, prob.lam, prob.d)
    ctx.build_tree(prob.x, prob.y, prob.z)
    for c in range(O.num_components(3)):
        info = ctx.fmm_info(c, keys=True)
        d, tk, sk, root, tl, sl = O.component_tree(ly, prob.x, prob.y, prob.z, c, leaf_cap=10, adaptive=mode)
        assert np.array_equal(info["root"], root), c
        tkey = tk | (tl.astype(np.uint64) << np.uint64(58))
        skey = sk | (sl.astype(np.uint64) << np.uint64(58))
        assert np.array_equal(info["tkeys"], tkey) and np.array_equal(info["skeys"], skey), c
    ctx.close()


@pytest.mark.parametrize("p,mode", [(4, 2), (7, 2), (7, 1)])
def test_adaptive_fp64_matches_oracle_fmm_per_slot(lpb, clustered, p, mode):
    # mode 2 (occupancy alone) puts thousands of reaction (point, box) pairs on the W- and
    # X-lists; mode 1 (reaction sets also divided near the interface) few or none
    prob = clustered
    ly = O.Layers(prob.eps, prob.lam, prob.d)
    ctx, phi = run(lpb, prob, p, 10, adaptive=mode)
    parts = ctx.debug_parts()
    st = ctx.stats()
    ctx.close()
    print(f"adaptive {mode} p={p}: W {st['n_w_pairs']} X {st['n_x_pairs']} point ops {st['n_point_ops']}",
          flush=True)
    assert st["n_w_pairs"] > 0 and st["n_x_pairs"] > 0
    if mode == 2:
        assert st["n_point_ops"] > 1000
    ref, cphi, ost = O.fmm(ly, prob.x, prob.y, prob.z, prob.q, p, leaf_cap=10, components=True, adaptive=mode)
    assert st["n_w_pairs"] == int(ost[:, 6].sum()) and st["n_x_pairs"] == int(ost[:, 7].sum())
    assert st["n_m2l_pairs"] == int(ost[:, 3].sum())
    assert st["n_p2p_pairs"] == int(ost[:, 4].sum()) + prob.n
    assert err2(phi, ref, prob.layer) <= 1e-10
    for key, e in slot_errors(parts, cphi, prob.layer, 3).items():
        assert e <= 1e-10, (key, e)


@pytest.mark.parametrize("mode", [1, 2])
def test_adaptive_mixed_matches_fp64_and_oracle(lpb, clustered, mode):
    prob = clustered
    ly = O.Layers(prob.eps, prob.lam, prob.d)
    ctx, phi64 = run(lpb, prob, 7, 10, adaptive=mode)
    ctx.close()
    ctx, phi32 = run(lpb, prob, 7, 10, precision=lpb.LPB_MIXED, adaptive=mode)
    ctx.close()
    assert err2(phi32, phi64, prob.layer) <= 1e-6
    ref = O.fmm(ly, prob.x, prob.y, prob.z, prob.q, 7, leaf_cap=10, adaptive=mode)
    assert err2(phi32, ref, prob.layer) <= 1e-6


def test_adaptive_free_space_tiled_levels(lpb):
    # one medium, 2e4 charges, 70 % in a tight cluster: adaptive leaves down to
    # levels the tiled M2L covers, with W- and X-lists between them
    rng = np.random.default_rng(11)
    n = 20000
    m = int(0.7 * n)
    P = np.vstack([rng.uniform(-1, 1, (n - m, 3)), np.clip(rng.normal(0.3, 0.03, (m, 3)), -1, 1)])
    x, y, z = P[:, 0].copy(), P[:, 1].copy(), P[:, 2].copy()
    q = rng.uniform(-1, 1, n)
    ly = O.Layers([2.0], [0.8], [])
    out = {}
    for prec in (lpb.LPB_FP64, lpb.LPB_MIXED):
        ctx = lpb.Context(p=8, leaf_cap=12, precision=prec, adaptive=1)
        ctx.set_layers([2.0], [0.8], [])
        ctx.build_tree(x, y, z)
        out[prec] = ctx.evaluate(q)
        st = ctx.stats()
        ctx.close()
        assert st["n_m2l_tile_pairs"] > 0 and st["n_w_pairs"] > 0 and st["n_x_pairs"] > 0
    ref = O.fmm(ly, x, y, z, q, 8, leaf_cap=12, adaptive=1)
    layer = np.zeros(n, dtype=int)
    assert err2(out[lpb.LPB_FP64], ref, layer, 1) <= 1e-10
    assert err2(out[lpb.LPB_MIXED], out[lpb.LPB_FP64], layer, 1) <= 1e-6


@pytest.mark.parametrize("mode", [1, 2])
def test_adaptive_batch_matches_single_systems_bitwise(lpb, mode):
    # three interface-clustered systems with different media in one batched
    # evaluation on adaptive trees: each system's potential bit for bit that
    # of its own context (the W/X lists and point operators of every system
    # share the stage launches)
    probs = [inputs.three_layer_interface_clusters(n, seed=s) for n, s in ((90, 3), (60, 4), (120, 5))]
    probs[1].eps = np.array([2.0, 30.0, 5.0])
    probs[1].lam = np.array([0.7, 2.5, 1.1])
    singles = []
    for pr in probs:
        ctx, phi = run(lpb, pr, 6, 8, adaptive=mode)
        ctx.close()
        singles.append(phi)
    ctx = lpb.Context(p=6, leaf_cap=8, adaptive=mode)
    ctx.set_systems([p.eps for p in probs], [p.lam for p in probs], [p.d for p in probs])
    ctx.build_trees([p.x for p in probs], [p.y for p in probs], [p.z for p in probs])
    outs = ctx.evaluate_batch([p.q for p in probs])
    st = ctx.stats()
    ctx.close()
    assert st["n_w_pairs"] > 0 and st["n_x_pairs"] > 0
    for a, b in zip(outs, singles):
        assert np.array_equal(a, b)


def test_adaptive_four_layer_stack_fp64_matches_oracle(lpb):
    # general L (Sec. 2.1): a 4-layer stack on adaptive trees (occupancy alone, so the
    # reaction W/X lists of all 4 L^2 = 36 components are busy), FP64 against the oracle
    prob = inputs.stack(70, 4, seed=2)
    ly = O.Layers(prob.eps, prob.lam, prob.d)
    ctx, phi = run(lpb, prob, 5, 6, adaptive=2)
    st = ctx.stats()
    ctx.close()
    assert st["n_w_pairs"] > 0 and st["n_x_pairs"] > 0
    ref = O.fmm(ly, prob.x, prob.y, prob.z, prob.q, 5, leaf_cap=6, adaptive=2)
    assert err2(phi, ref, prob.layer, 4) <= 1e-10


def test_adaptive_orders_beyond_the_fixed_kernels(lpb):
    # p = 17 (mixed only): the W/X kernels with the order read at run time, one medium
    rng = np.random.default_rng(12)
    n = 6000
    P = np.vstack([rng.uniform(-1, 1, (n // 2, 3)), np.clip(rng.normal(-0.2, 0.04, (n - n // 2, 3)), -1, 1)])
    x, y, z = P[:, 0].copy(), P[:, 1].copy(), P[:, 2].copy()
    q = rng.uniform(-1, 1, n)
    ctx = lpb.Context(p=17, leaf_cap=10, precision=lpb.LPB_MIXED, adaptive=1)
    ctx.set_layers([2.0], [0.8], [])
    ctx.build_tree(x, y, z)
    phi = ctx.evaluate(q)
    st = ctx.stats()
    ctx.close()
    assert st["n_w_pairs"] > 0 and st["n_x_pairs"] > 0
    ref = O.fmm(O.Layers([2.0], [0.8], []), x, y, z, q, 17, leaf_cap=10, adaptive=1)
    assert err2(phi, ref, np.zeros(n, dtype=int), 1) <= 1e-6
