"""The device-memory hook of lpb_options (alloc / free / alloc_user): a
context backed by PyTorch's caching allocator gives bit-identical results
and returns every buffer it took; an allocator that refuses at any point
(context tables, tree, operators) makes that call fail with LPB_ENOMEM, with
no abort and no buffer left behind."""
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


class Counting:
    """torch's caching allocator, recording live buffers; refuses every
    request from number `refuse_from` on (None: never)."""

    def __init__(self, lpb, refuse_from=None):
        import torch

        self.torch = torch
        self.live = {}
        self.calls = 0
        self.refuse_from = refuse_from
        self.hook = lpb.Allocator(self.alloc, self.free)

    def alloc(self, n):
        self.calls += 1
        if self.refuse_from is not None and self.calls > self.refuse_from:
            return 0
        ptr = self.torch.cuda.caching_allocator_alloc(n, device=0)
        assert ptr % 256 == 0
        self.live[ptr] = n
        return ptr

    def free(self, ptr):
        assert ptr in self.live, "freed a pointer it was not given"
        del self.live[ptr]
        self.torch.cuda.caching_allocator_delete(ptr)


def _setup_and_eval(lpb, prob, allocator, precision):
    ctx = lpb.Context(p=8, leaf_cap=30, precision=precision, allocator=allocator.hook if allocator else None)
    ctx.set_layers(prob.eps, prob.lam, prob.d)
    ctx.build_tree(prob.x, prob.y, prob.z)
    return ctx, ctx.evaluate(prob.q)


@pytest.mark.parametrize("precision", [1, 0])
def test_torch_caching_allocator_backs_the_context(lpb, precision):
    import torch

    prob = inputs.three_layer(10_000, seed=0)
    base = torch.cuda.memory_allocated(0)
    al = Counting(lpb)
    ctx, phi = _setup_and_eval(lpb, prob, al, precision)
    assert len(al.live) > 20 and torch.cuda.memory_allocated(0) > base
    ref_ctx, ref = _setup_and_eval(lpb, prob, None, precision)
    ref_ctx.close()
    assert np.array_equal(phi, ref)
    # a new tree drops the plan's buffers through the hook and takes new ones
    prob2 = inputs.three_layer(4_000, seed=3)
    ctx.build_tree(prob2.x, prob2.y, prob2.z)
    ctx.evaluate(prob2.q)
    ctx.close()
    assert al.live == {}
    assert torch.cuda.memory_allocated(0) == base


def test_refusing_allocator_gives_enomem_without_leaks(lpb):
    prob = inputs.three_layer(3_000, seed=1)
    # count the requests of each phase with an allocator that never refuses
    al = Counting(lpb)
    ctx = lpb.Context(p=6, leaf_cap=30, allocator=al.hook)
    n_create = al.calls
    ctx.set_layers(prob.eps, prob.lam, prob.d)
    ctx.build_tree(prob.x, prob.y, prob.z)
    n_build = al.calls - n_create
    ctx.evaluate(prob.q)
    n_eval = al.calls - n_create - n_build
    ctx.close()
    assert al.live == {} and n_create > 0 and n_build > 2 and n_eval > 0
    # refuse in lpb_create
    al = Counting(lpb, refuse_from=n_create - 1)
    with pytest.raises(lpb.LpbError) as e:
        lpb.Context(p=6, leaf_cap=30, allocator=al.hook)
    assert e.value.status == lpb.LPB_ENOMEM and al.live == {}
    # refuse in lpb_build_tree, then in the operator generation of the first evaluate
    for k in (n_create + n_build // 2, n_create + n_build + n_eval // 2):
        al = Counting(lpb, refuse_from=k)
        ctx = lpb.Context(p=6, leaf_cap=30, allocator=al.hook)
        ctx.set_layers(prob.eps, prob.lam, prob.d)
        with pytest.raises(lpb.LpbError) as e:
            ctx.build_tree(prob.x, prob.y, prob.z)
            ctx.evaluate(prob.q)
        assert e.value.status == lpb.LPB_ENOMEM
        # what the failed call took is back; the context still holds only its tables
        assert len(al.live) <= n_create + (n_build if k > n_create + n_build else 0)
        ctx.close()
        assert al.live == {}, k


def test_memory_the_library_does_not_write_is_never_read(lpb):
    """Every buffer of these contexts starts as 0xFF bytes (NaN in FP32 and
    FP64): results must equal those of fresh hipMalloc memory bit for bit, in
    both precisions, captured and eager, on a tree with tiled levels and on
    one with reaction near-field pairs."""
    import ctypes

    import torch

    hip = ctypes.CDLL("libamdhip64.so")
    hip.hipMemset.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_size_t]

    def poisoned(n):
        ptr = torch.cuda.caching_allocator_alloc(n, device=0)
        assert hip.hipMemset(ptr, 0xFF, n) == 0 and hip.hipDeviceSynchronize() == 0
        return ptr

    hook = lpb.Allocator(poisoned, torch.cuda.caching_allocator_delete)
    near = inputs.three_layer(150, seed=11)
    for i, zz in {0: 0.002, 150: -0.003, 151: -1.198, 300: -1.202}.items():
        near.z[i] = zz
    for prob, p, cap in ((inputs.three_layer(10_000, seed=0), 7, 8), (near, 6, 8)):
        for precision in (0, 1):
            for graph in (1, 0):
                out = []
                for alloc in (None, hook):
                    ctx = lpb.Context(p=p, leaf_cap=cap, precision=precision, graph=graph, autotune=graph,
                                      allocator=alloc)
                    ctx.set_layers(prob.eps, prob.lam, prob.d)
                    ctx.build_tree(prob.x, prob.y, prob.z)
                    out.append(ctx.evaluate(prob.q))
                    ctx.close()
                assert np.all(np.isfinite(out[1])) and np.array_equal(out[0], out[1]), (p, precision, graph)
