"""Parity of the tiled free-space M2L against the oracle FMM.

Free-space trees of depth >= 4 send their V-list pairs at levels 4..8 through
the tiled matrix-core kernels: in FP64 the per-offset product over 56
canonical operators with reflection sign flips, in mixed precision the
reflection-orbit form (5 <= p <= 15) or the per-offset form in FP32 (other
p).  Here those paths meet the oracle FMM (Algorithm 2, eq. metole) on the
same tree: FP64 per output slot within 1e-10 (rounding only), mixed per
layer within 1e-6 (FP32 bulk).  Inputs follow the benchmark recipe at
sizes where the free trees reach depth 4 (1e4 charges per layer, leaf cap 8)
and depth 5 (1e5 per layer, leaf cap 8)."""
import numpy as np
import pytest

import oracle as O
from lpbtest import err2, run, slot_errors
from paper_2002_01334_amd import inputs

pytestmark = pytest.mark.gpu

DEEP = {"depth4": (10_000, 8), "depth5": (100_000, 8)}
# (tree, p): p = 10 the benchmark order, 7 an odd order, 15 the largest orbit
# order, 5 the smallest orbit order, 4 the FP32 per-offset form
CASES = [("depth4", 10), ("depth4", 7), ("depth4", 15), ("depth5", 5), ("depth5", 4)]


@pytest.fixture(scope="module")
def lpb():
    import torch

    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    from paper_2002_01334_amd import lpb as m

    m.load()
    return m


_PROBS = {}


def deep_problem(name):
    if name not in _PROBS:
        n, cap = DEEP[name]
        prob = inputs.three_layer(n, seed=0)
        _PROBS[name] = (prob, O.Layers(prob.eps, prob.lam, prob.d), cap)
    return _PROBS[name]


@pytest.mark.parametrize("tree,p", CASES)
def test_tiled_m2l_fp64_and_mixed_vs_oracle_fmm(lpb, tree, p):
    prob, ly, cap = deep_problem(tree)
    want_depth = int(tree[-1])
    print(f"[tiled parity] {tree} n={prob.n} cap={cap} p={p}", flush=True)
    ref, cphi, ost = O.fmm(ly, prob.x, prob.y, prob.z, prob.q, p, leaf_cap=cap, components=True)
    ctx, phi64 = run(lpb, prob, p, cap, device=True)
    st = ctx.stats()
    parts = ctx.debug_parts()
    depths = [ctx.fmm_info(c)["depth"] for c in range(3)]   # the three free-space FMMs come first
    ctx.close()
    assert depths == [want_depth] * 3, depths
    assert st["n_m2l_tile_pairs"] > 0 and st["n_m2l_tiles"] > 0
    assert st["n_m2l_pairs"] == int(ost[:, 3].sum())
    e64 = err2(phi64, ref, prob.layer)
    es = slot_errors(parts, cphi, prob.layer, 3)
    print(f"  FP64 vs oracle FMM {e64:.2e}, worst slot {max(es.values()):.2e}", flush=True)
    assert e64 <= 1e-10
    for key, e in es.items():
        assert e <= 1e-10, (key, e)
    ctx, phi32 = run(lpb, prob, p, cap, precision=lpb.LPB_MIXED, device=True)
    st32 = ctx.stats()
    ctx.close()
    assert st32["n_m2l_tile_pairs"] == st["n_m2l_tile_pairs"]
    e32 = err2(phi32, ref, prob.layer)
    print(f"  mixed vs oracle FMM {e32:.2e}", flush=True)
    assert e32 <= 1e-6


def sparse_lattice(seed, n=400):
    """One charge near the centre of each of n random cells of the 8^3 corner
    block of a 16^3 lattice over [-1, 1]^3 (plus the far corner cell, which
    with the near one fixes the bounding cube): with leaf cap 1 no two charges
    share a level-4 box, so the tree has depth 4 with few V-list pairs, and the
    8^3 block's M2L tiles hold about 50 of their 64 target boxes (tiles of
    fewer than 16 give their pairs to the batched list)."""
    rng = np.random.default_rng(seed)
    blk = rng.choice(8**3, n, replace=False)
    cells = np.unique(np.concatenate([(blk // 64) * 256 + ((blk // 8) % 8) * 16 + blk % 8, [0, 16**3 - 1]]))
    ijk = (cells // 256, (cells // 16) % 16, cells % 16)
    x, y, z = [-1 + (2 * i + 1) / 16.0 + rng.uniform(-0.01, 0.01, len(cells)) for i in ijk]
    return x, y, z, rng.uniform(-1, 1, len(cells))


@pytest.mark.parametrize("p", [16, 20])
def test_mixed_high_orders_vs_oracle_fmm(lpb, p):
    """Orders above the FP64 limit run in mixed precision only (per-offset
    FP32 tiled M2L, generic P2M/L2P): against the oracle FMM on a depth-4
    free-space tree."""
    x, y, z, q = sparse_lattice(p)
    ly = O.Layers([2.0], [0.8], [])
    ref = O.fmm(ly, x, y, z, q, p, leaf_cap=1)
    ctx = lpb.Context(p=p, leaf_cap=1, precision=lpb.LPB_MIXED)
    ctx.set_layers([2.0], [0.8], [])
    ctx.build_tree(x, y, z)
    phi = ctx.evaluate(q)
    st = ctx.stats()
    depth = ctx.fmm_info(0)["depth"]
    ctx.close()
    assert depth == 4 and st["n_m2l_tile_pairs"] > 0
    e = float(np.linalg.norm(phi - ref) / np.linalg.norm(ref))
    print(f"p={p} mixed vs oracle FMM {e:.2e}")
    assert e <= 1e-6
    with pytest.raises(lpb.LpbError) as ex:
        lpb.Context(p=p, precision=lpb.LPB_FP64)
    assert ex.value.status == lpb.LPB_ERANGE
