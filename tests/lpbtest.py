"""Helpers shared by the GPU tests: per-layer relative l2 errors (the paper's
Err_2 of Sec. 4), the output slot of each oracle component, and one
evaluation through the C ABI."""
import numpy as np

import oracle as O


def err2(a, b, layer, nl=3):
    """max over layers of ||a - b|| / ||b|| restricted to the layer."""
    out = []
    for l in range(nl):
        m = layer == l
        if m.sum() == 0:
            continue
        nb = np.linalg.norm(b[m])
        out.append(np.linalg.norm(a[m] - b[m]) / nb if nb > 0 else np.linalg.norm(a[m]))
    return max(out)


def slot_map(nl):
    """Output slot of each component: 0 free space, a (1 or 2) for the reaction
    components through the lower / upper interface of the target's layer, whose
    target trees (and local expansions) the library shares."""
    m = {}
    for c in range(O.num_components(nl)):
        kind, l, lp, a, b = O.component(nl, c)
        m[c] = (l, 0 if kind == 0 else a)
    return m


def slot_errors(parts, cphi, layer, nl):
    """Relative l2 error of every (layer, slot) partial potential of the
    library against the sum of the oracle's components feeding that slot."""
    sm = slot_map(nl)
    out = {}
    for l in range(nl):
        m = layer == l
        if not m.any():
            continue
        for s in range(parts.shape[0]):
            comps = [c for c in range(cphi.shape[0]) if sm[c] == (l, s)]
            if not comps:
                continue
            ref = cphi[comps].sum(axis=0)[m]
            nr = np.linalg.norm(ref)
            out[(l, s)] = np.linalg.norm(parts[s][m] - ref) / nr if nr > 0 else np.linalg.norm(parts[s][m])
    return out


def run(lpb, prob, p, leaf_cap, precision=0, device=False, **kw):
    ctx = lpb.Context(p=p, leaf_cap=leaf_cap, precision=precision, **kw)
    ctx.set_layers(prob.eps, prob.lam, prob.d)
    if device:
        import torch

        t = {k: torch.tensor(getattr(prob, k), dtype=torch.float64, device="cuda:0") for k in "xyzq"}
        ctx.build_tree(t["x"], t["y"], t["z"])
        phi = ctx.evaluate(t["q"]).cpu().numpy()
    else:
        ctx.build_tree(prob.x, prob.y, prob.z)
        phi = ctx.evaluate(prob.q)
    return ctx, phi
