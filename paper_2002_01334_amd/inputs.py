"""Seeded synthetic inputs for the layered-media workloads.

This module holds only random-number generation and geometry recipes (no
arithmetic of the method); tests, the benchmark and the oracle checks all
draw their charges from here.

Generator: SplitMix64 (Steele, Lea, Flood 2014).  Draw k (k = 0, 1, ...) of a
stream seeded with s is mix(s + (k+1) * 0x9E3779B97F4A7C15) with the
published finaliser; a uniform double is (draw >> 11) * 2^-53.  Gaussians use
Box-Muller on two consecutive uniforms.

Workload recipe (the paper's three-layer test problem, Sec. 4, re-centred
in unit cubes): interfaces z = 0 and z = -1.2; layer 0 charges uniform in
[-0.5,0.5]^2 x [0.1,1.1], layer 1 in [-0.5,0.5]^2 x [-1.1,-0.1], layer 2 in
[-0.5,0.5]^2 x [-2.3,-1.3] (centres (0,0,0.6), (0,0,-0.6), (0,0,-1.8) as in
the paper, 0.1 clearance from every interface); charges q ~ U[-1,1].
Per layer the draws are x, y, z, q for charge 0, then charge 1, and so on;
layers are drawn in order 0, 1, 2 from one stream.
"""
from __future__ import annotations

import dataclasses

import numpy as np

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


class SplitMix64:
    """Counter form of SplitMix64: draw k = mix(seed + (k+1)*gamma)."""

    def __init__(self, seed: int):
        self.seed = np.uint64(seed & 0xFFFFFFFFFFFFFFFF)
        self.k = 0

    def draws(self, count: int) -> np.ndarray:
        with np.errstate(over="ignore"):
            idx = np.arange(self.k + 1, self.k + 1 + count, dtype=np.uint64)
            z = self.seed + idx * _GAMMA
            z = (z ^ (z >> np.uint64(30))) * _M1
            z = (z ^ (z >> np.uint64(27))) * _M2
            z = z ^ (z >> np.uint64(31))
        self.k += count
        return z

    def uniform(self, count: int) -> np.ndarray:
        return (self.draws(count) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


@dataclasses.dataclass
class LayeredProblem:
    eps: np.ndarray
    lam: np.ndarray
    d: np.ndarray        # interfaces, strictly decreasing
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    q: np.ndarray
    layer: np.ndarray    # layer index of each charge

    @property
    def n(self) -> int:
        return len(self.x)


EPS3 = (1.0, 2.0, 4.0)
LAM3 = (1.2, 1.5, 2.0)
D3 = (0.0, -1.2)
# z-ranges of the unit cubes of the three layers
ZBOX3 = ((0.1, 1.1), (-1.1, -0.1), (-2.3, -1.3))


def _uniform_block(rng: SplitMix64, n: int, lo, hi):
    u = rng.uniform(4 * n).reshape(n, 4)
    x = lo[0] + (hi[0] - lo[0]) * u[:, 0]
    y = lo[1] + (hi[1] - lo[1]) * u[:, 1]
    z = lo[2] + (hi[2] - lo[2]) * u[:, 2]
    q = -1.0 + 2.0 * u[:, 3]
    return x, y, z, q


def _gauss_block(rng: SplitMix64, n: int, lo, hi, sigma: float, centre=None):
    """Gaussian about the cube centre (or `centre`), redrawn until inside the cube."""
    lo = np.asarray(lo, float)
    hi = np.asarray(hi, float)
    c = 0.5 * (lo + hi) if centre is None else np.asarray(centre, float)
    out = np.empty((n, 3))
    filled = 0
    while filled < n:
        need = n - filled
        u = rng.uniform(6 * need).reshape(need, 6)
        r1 = np.sqrt(-2.0 * np.log(np.maximum(u[:, 0::2], 2.0 ** -53)))
        g = r1 * np.cos(2.0 * np.pi * u[:, 1::2])
        pts = c + sigma * g
        ok = np.all((pts >= lo) & (pts <= hi), axis=1)
        k = int(ok.sum())
        out[filled:filled + k] = pts[ok]
        filled += k
    q = -1.0 + 2.0 * rng.uniform(n)
    return out[:, 0], out[:, 1], out[:, 2], q


def three_layer(per_layer, seed: int = 0, clustered_fraction: float = 0.0, sigma: float = 0.1,
                eps=EPS3, lam=LAM3) -> LayeredProblem:
    """Charges in the three unit cubes (per_layer an int or 3 ints)."""
    if np.isscalar(per_layer):
        per_layer = (int(per_layer),) * 3
    rng = SplitMix64(seed)
    xs, ys, zs, qs, ls = [], [], [], [], []
    for l, n in enumerate(per_layer):
        lo = (-0.5, -0.5, ZBOX3[l][0])
        hi = (0.5, 0.5, ZBOX3[l][1])
        nc = int(round(clustered_fraction * n))
        x, y, z, q = _uniform_block(rng, n - nc, lo, hi)
        if nc:
            gx, gy, gz, gq = _gauss_block(rng, nc, lo, hi, sigma)
            x, y, z, q = (np.concatenate(a) for a in ((x, gx), (y, gy), (z, gz), (q, gq)))
        xs.append(x); ys.append(y); zs.append(z); qs.append(q); ls.append(np.full(n, l, np.int32))
    return LayeredProblem(np.array(eps, float), np.array(lam, float), np.array(D3, float),
                          np.concatenate(xs), np.concatenate(ys), np.concatenate(zs), np.concatenate(qs),
                          np.concatenate(ls))


def three_layer_interface_clusters(per_layer, seed: int = 0, sigma: float = 0.04, gap: float = 0.02,
                                   eps=EPS3, lam=LAM3) -> LayeredProblem:
    """Strongly clustered charges next to the interfaces (adaptive-tree
    inputs): per layer half uniform in the layer's slab of the unit square
    column, |x|, |y| <= 1/2, kept `gap` away from every interface (the top
    and bottom slabs 1.08 thick), half Gaussian (sigma) about (0.1, -0.1,
    z_c) with z_c = 0.05 + gap/2 from the interface below the top layer,
    above and below the middle layer's nearest interface, redrawn until
    inside the slab."""
    if np.isscalar(per_layer):
        per_layer = (int(per_layer),) * 3
    rng = SplitMix64(seed)
    top, mid = D3[0], D3[1]
    slabs = [(top + gap, top + 1.1), (mid + gap, top - gap), (mid - 1.1, mid - gap)]
    centres = [top + 0.05 + gap / 2, top - 0.05 - gap / 2, mid - 0.05 - gap / 2]
    xs, ys, zs, qs, ls = [], [], [], [], []
    for l, n in enumerate(per_layer):
        lo = (-0.5, -0.5, slabs[l][0])
        hi = (0.5, 0.5, slabs[l][1])
        nc = n // 2
        x, y, z, q = _uniform_block(rng, n - nc, lo, hi)
        if nc:
            gx, gy, gz, gq = _gauss_block(rng, nc, lo, hi, sigma, centre=(0.1, -0.1, centres[l]))
            x, y, z, q = (np.concatenate(a) for a in ((x, gx), (y, gy), (z, gz), (q, gq)))
        xs.append(x); ys.append(y); zs.append(z); qs.append(q); ls.append(np.full(n, l, np.int32))
    return LayeredProblem(np.array(eps, float), np.array(lam, float), np.array(D3, float),
                          np.concatenate(xs), np.concatenate(ys), np.concatenate(zs), np.concatenate(qs),
                          np.concatenate(ls))


# A stack of up to five layers (general L, Sec. 2.1): interfaces every 1.2
# below z = 0; the first three layers are the three-layer medium above.
STACK_EPS = (1.0, 2.0, 4.0, 8.0, 3.0)
STACK_LAM = (1.2, 1.5, 2.0, 0.8, 1.1)


def stack(per_layer, nlayers: int, seed: int = 0) -> LayeredProblem:
    """nlayers layers, interfaces z = 0, -1.2, -2.4, ...; eps and lambda the
    first nlayers of STACK_EPS / STACK_LAM; per layer (an int or nlayers ints)
    charges uniform in x, y in [-0.5, 0.5] and z in the 1.0-thick slab of the
    layer at 0.1 clearance from its interfaces (the unbounded top and bottom
    layers: 0.1 to 1.1 away from their interface); q ~ U[-1, 1], draws x, y,
    z, q per charge, layers in order from one stream (three layers give
    three_layer's charges)."""
    if np.isscalar(per_layer):
        per_layer = (int(per_layer),) * nlayers
    d = np.array([round(-1.2 * k, 12) + 0.0 for k in range(nlayers - 1)])
    rng = SplitMix64(seed)
    xs, ys, zs, qs, ls = [], [], [], [], []
    for l, n in enumerate(per_layer):
        hi = 1.1 if l == 0 else round(d[l - 1] - 0.1, 12)
        lo = round(hi - 1.0, 12)
        x, y, z, q = _uniform_block(rng, n, (-0.5, -0.5, lo), (0.5, 0.5, hi))
        xs.append(x); ys.append(y); zs.append(z); qs.append(q); ls.append(np.full(n, l, np.int32))
    return LayeredProblem(np.array(STACK_EPS[:nlayers], float), np.array(STACK_LAM[:nlayers], float), d,
                          np.concatenate(xs), np.concatenate(ys), np.concatenate(zs), np.concatenate(qs),
                          np.concatenate(ls))


def batch_system(k: int, nmin: float = 1e3, nmax: float = 5e4) -> LayeredProblem:
    """System k of the batched workload: seed 1000+k; N_total log-uniform in
    [nmin, nmax], split floor(N/3) per layer with the remainder in layer 0;
    eps ~ U[1,80], lambda ~ U[0.5,3] per layer; middle thickness D ~ U[0.8,2],
    interfaces (0, -D); middle cube side min(1, D-0.2) centred at -D/2; top and
    bottom unit cubes at 0.1 clearance."""
    rng = SplitMix64(1000 + k)
    u = rng.uniform(8)
    ntot = int(np.exp(np.log(nmin) + (np.log(nmax) - np.log(nmin)) * u[0]))
    eps = 1.0 + 79.0 * u[1:4]
    lam = 0.5 + 2.5 * u[4:7]
    D = 0.8 + 1.2 * u[7]
    per = [ntot // 3] * 3
    per[0] += ntot - 3 * (ntot // 3)
    side = min(1.0, D - 0.2)
    boxes = [((-0.5, -0.5, 0.1), (0.5, 0.5, 1.1)),
             ((-side / 2, -side / 2, -D / 2 - side / 2), (side / 2, side / 2, -D / 2 + side / 2)),
             ((-0.5, -0.5, -D - 1.1), (0.5, 0.5, -D - 0.1))]
    xs, ys, zs, qs, ls = [], [], [], [], []
    for l in range(3):
        x, y, z, q = _uniform_block(rng, per[l], boxes[l][0], boxes[l][1])
        xs.append(x); ys.append(y); zs.append(z); qs.append(q); ls.append(np.full(per[l], l, np.int32))
    return LayeredProblem(eps, lam, np.array([0.0, -D]), np.concatenate(xs), np.concatenate(ys),
                          np.concatenate(zs), np.concatenate(qs), np.concatenate(ls))


# The paper's own test problem (Sec. 4): three layers with interfaces z = 0 and
# -1.2, eps = (1, 8.6, 20.5), lambda = (1.2, 0.5, 2.1); charges uniform inside
# the bodies r(theta) = 0.5 - a + (a/8)(35 cos^4 - 30 cos^2 + 3)(theta) (a
# P_4-modulated sphere of polar radius 0.5) with a = 0.1, 0.15, 0.05, shifted
# to the centres (0, 0, 0.6), (0, 0, -0.6), (0, 0, -1.8).
PAPER_EPS = (1.0, 8.6, 20.5)
PAPER_LAM = (1.2, 0.5, 2.1)
PAPER_A = (0.1, 0.15, 0.05)
PAPER_ZC = (0.6, -0.6, -1.8)
# total charge counts of the paper's timing table
PAPER_N = (618_256, 1_128_556, 1_862_568, 2_861_288)


def p4_radius(a: float, c):
    """Radius of the body at cos(theta) = c."""
    c2 = np.asarray(c, float) ** 2
    return 0.5 - a + (a / 8.0) * (35.0 * c2 * c2 - 30.0 * c2 + 3.0)


def p4_volume(a: float) -> float:
    """Volume (2 pi / 3) int_{-1}^{1} r(c)^3 dc (a polynomial of degree 12 in
    c, exact with 8 Gauss-Legendre nodes; 16 are used)."""
    c, w = np.polynomial.legendre.leggauss(16)
    return float(2.0 * np.pi / 3.0 * np.sum(w * p4_radius(a, c) ** 3))


def paper_domains(n_total=None, seed: int = 0, per_layer=None) -> LayeredProblem:
    """Charges of the paper's test problem: n_total split over the layers in
    proportion to the body volumes (equal density; the remainder goes to
    layer 0), or the per-layer counts given.  Candidates uniform in the cube
    of side 1 about each centre (draws x, y, z, q per candidate, layers in
    order from one stream) are kept when inside the body; q ~ U[-1, 1] (the
    paper does not state the charges)."""
    if per_layer is None:
        vol = [p4_volume(a) for a in PAPER_A]
        per_layer = [int(n_total * v / sum(vol)) for v in vol]
        per_layer[0] += n_total - sum(per_layer)
    rng = SplitMix64(seed)
    xs, ys, zs, qs, ls = [], [], [], [], []
    for l, n in enumerate(per_layer):
        a, zc = PAPER_A[l], PAPER_ZC[l]
        frac = p4_volume(a)             # the cube has volume 1
        out = np.empty((n, 4))
        filled = 0
        while filled < n:
            need = n - filled
            m = int(need / frac * 1.05) + 16
            u = rng.uniform(4 * m).reshape(m, 4) - 0.5
            rho = np.sqrt(u[:, 0] ** 2 + u[:, 1] ** 2 + u[:, 2] ** 2)
            ok = rho < p4_radius(a, u[:, 2] / np.maximum(rho, 1e-300))
            acc = u[ok][:need]
            out[filled:filled + len(acc)] = acc
            filled += len(acc)
        xs.append(out[:, 0]); ys.append(out[:, 1]); zs.append(zc + out[:, 2]); qs.append(2.0 * out[:, 3])
        ls.append(np.full(n, l, np.int32))
    return LayeredProblem(np.array(PAPER_EPS), np.array(PAPER_LAM), np.array(D3, float),
                          np.concatenate(xs), np.concatenate(ys), np.concatenate(zs), np.concatenate(qs),
                          np.concatenate(ls))


def sample_targets(prob: LayeredProblem, per_layer: int, seed: int = 1) -> np.ndarray:
    """per_layer distinct charge indices from each layer (sorted)."""
    rng = SplitMix64(seed)
    out = []
    for l in range(len(prob.eps)):
        idx = np.nonzero(prob.layer == l)[0]
        k = min(per_layer, len(idx))
        keys = rng.draws(len(idx))
        out.append(idx[np.argsort(keys, kind="stable")[:k]])
    return np.sort(np.concatenate(out))
