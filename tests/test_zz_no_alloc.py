"""lpb_evaluate_noalloc (the entry point for callers that cannot allocate)
against lpb_evaluate through the C ABI: bit-identical potentials on two
calls in a row, the second on a smaller system (the GPU's shared scratch
array still holds the first call's partial potentials), in mixed precision
and FP64; and its error paths (unprepared context, size beyond the array)."""
import numpy as np
import pytest

from paper_2002_01334_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lpb():
    import torch

    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    from paper_2002_01334_amd import lpb as m

    m.load()
    return m


def _dev(prob):
    import torch

    return {k: torch.tensor(getattr(prob, k), dtype=torch.float64, device="cuda:0") for k in "xyzq"}


@pytest.mark.parametrize("precision", [1, 0])
def test_noalloc_matches_evaluate_bitwise(lpb, precision):
    import torch

    for n, seed in ((10_000, 0), (3_000, 7)):
        prob = inputs.three_layer(n, seed=seed)
        t = _dev(prob)
        ctx = lpb.Context(p=8, leaf_cap=30, precision=precision)
        ctx.set_layers(prob.eps, prob.lam, prob.d)
        ctx.build_tree(t["x"], t["y"], t["z"])
        out = torch.empty_like(t["q"])
        with pytest.raises(lpb.LpbError) as e:
            ctx.evaluate_noalloc(t["q"], out)
        assert e.value.status == lpb.LPB_ESTATE
        ctx.evaluate(t["q"])   # generates the operators and picks the schedules
        for q in (t["q"], 2.0 * t["q"]):
            got = ctx.evaluate_noalloc(q, out).cpu().numpy()
            want = ctx.evaluate(q).cpu().numpy()
            assert np.array_equal(got, want), (n, precision)
        ctx.close()


def test_noalloc_rejects_sizes_beyond_the_scratch_array(lpb):
    import torch

    prob = inputs.three_layer(1_400_000, seed=0)   # 3 slots x 4.2e6 charges > 12 Mi partial potentials
    t = _dev(prob)
    ctx = lpb.Context(p=4, leaf_cap=50, precision=lpb.LPB_MIXED)
    ctx.set_layers(prob.eps, prob.lam, prob.d)
    ctx.build_tree(t["x"], t["y"], t["z"])
    ctx.evaluate(t["q"])
    out = torch.empty_like(t["q"])
    with pytest.raises(lpb.LpbError) as e:
        ctx.evaluate_noalloc(t["q"], out)
    assert e.value.status == lpb.LPB_ERANGE
    ctx.close()
