"""FP64 CPU oracle for the layered-media linearized Poisson-Boltzmann FMM.

TEST INFRASTRUCTURE ONLY.  This package binds ``lpb_oracle.c`` (plain C,
FP64) with ctypes.  Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU
baseline leg of ``bench.py`` may import it; the GPU product library never
loads it and shares no code with it.

Every function cites the passage of Wang, Zhang & Cai (arXiv 2002.01334) it
follows in the C source; the pins that check it live in
``tests/test_oracle_*.py``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(_HERE, "lpb_oracle.c")
LIB = os.path.join(_HERE, "liblpb_oracle.so")

_lib = None

_D = ctypes.c_double
_I = ctypes.c_int
_L = ctypes.c_int64
_PD = ctypes.POINTER(ctypes.c_double)
_PI = ctypes.POINTER(ctypes.c_int)
_PU32 = ctypes.POINTER(ctypes.c_uint32)
_PLL = ctypes.POINTER(ctypes.c_longlong)
_PL = ctypes.POINTER(ctypes.c_int64)
_PU = ctypes.POINTER(ctypes.c_uint64)


def build(verbose: bool = False) -> str:
    """Compile the oracle with gcc (plain C, OpenMP for independent loops)."""
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", LIB, SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    return LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        L = ctypes.CDLL(LIB)
        sig = {
            "orc_bessel_i": (_D, [_I, _D]),
            "orc_bessel_k": (_D, [_I, _D]),
            "orc_plm": (None, [_I, _D, _PD]),
            "orc_ylm": (None, [_I, _D, _D, _D, _PD, _PD]),
            "orc_gaunt": (_D, [_I, _I, _I, _I, _I, _I]),
            "orc_gauss_legendre": (None, [_I, _PD, _PD]),
            "orc_sigma3": (_D, [_PD, _PD, _D, _D, _I, _I, _I, _I, _D]),
            "orc_sigma_stack": (_D, [_I, _PD, _PD, _PD, _I, _I, _I, _I, _D]),
            "orc_reaction_u": (_D, [_PD, _PD, _PD, _I, _I, _I, _I, _I, _D, _D, _D, _D, _D, _D]),
            "orc_direct_sum": (_I, [_I, _PD, _PD, _PD, _L, _PD, _PD, _PD, _PD, _L, _PL, _PD, _I]),
            "orc_fmm": (_I, [_I, _PD, _PD, _PD, _L, _PD, _PD, _PD, _PD, _I, _I, _I, _I, _PD, _PD, _PD]),
            "orc_num_components": (_I, [_I]),
            "orc_component": (_I, [_I, _I, _PI]),
            "orc_free_chain": (_D, [_I, _D, _PD, _PD, _PD, _PD, _PD, _PD, _I]),
            "orc_addition_sum": (None, [_I, _I, _D, _I, _I, _PD, _PD, _I, _PD]),
            "orc_reaction_chain": (_D, [_PD, _PD, _PD, _I, _I, _I, _I, _I, _I, _PD, _PD, _PD, _PD, _PI]),
            "orc_reaction_I_pair": (None, [_PD, _PD, _PD, _I, _I, _I, _I, _I, _I, _D, _D, _D, _D,
                                           _I, _I, _I, _I, _PD]),
            "orc_reaction_I_both": (_I, [_PD, _PD, _PD, _I, _I, _I, _I, _I, _I, _D, _D, _D, _D, _PD, _PD, _PD, _PD]),
            "orc_sommerfeld_table": (_I, [_PD, _PD, _PD, _I, _I, _I, _I, _I, _D, _D, _D, _D, _I, _I, _PD]),
            "orc_free_point_chain": (_D, [_I, _D, _PD, _PD, _PD, _I]),
            "orc_list_coverage": (_I, [_I, _PU32, _I, _PU32, _I, _I, _I, _I, _PI, _PLL]),
            "orc_reaction_point_chain": (_D, [_PD, _PD, _PD, _I, _I, _I, _I, _I, _I, _PD, _PD, _PD, _D, _I]),
            "orc_reaction_I_point": (None, [_PD, _PD, _PD, _I, _I, _I, _I, _I, _I, _D, _D, _D, _D,
                                            _I, _I, _I, _I, _PD]),
            "orc_legendre_product": (None, [_I, _I, _I, _I, _D, _D, _D, _PD]),
            "orc_plm_beyond": (None, [_I, _I, _D, _PD]),
            "orc_component_tree": (_I, [_I, _PD, _PD, _PD, _L, _PD, _PD, _PD, _I, _I, _I, _PI, _PL, _PL,
                                        _PU, _PU, _PI, _PI, _PD]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(_PD)


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


class Layers:
    """eps, lam per layer (top to bottom) and interfaces d_0 > ... > d_{L-1}."""

    def __init__(self, eps, lam, d):
        self.eps = _f64(eps)
        self.lam = _f64(lam)
        self.d = _f64(d) if len(d) else np.zeros(1)
        self.nlayers = len(self.eps)
        assert len(self.lam) == self.nlayers and len(d) == self.nlayers - 1

    @property
    def L(self):
        return self.nlayers - 1


# --- special functions -----------------------------------------------------

def bessel_i(n, x):
    return lib().orc_bessel_i(int(n), float(x))


def bessel_k(n, x):
    return lib().orc_bessel_k(int(n), float(x))


def plm(nmax, x):
    out = np.zeros((nmax + 1) * (nmax + 2) // 2)
    lib().orc_plm(nmax, float(x), _p(out))
    return out


def ylm(nmax, v):
    K = (nmax + 1) ** 2
    re = np.zeros(K)
    im = np.zeros(K)
    lib().orc_ylm(nmax, float(v[0]), float(v[1]), float(v[2]), _p(re), _p(im))
    return re + 1j * im


def gaunt(n1, m1, n2, m2, n3, m3):
    return lib().orc_gaunt(n1, m1, n2, m2, n3, m3)


def gauss_legendre(n):
    x = np.zeros(n)
    w = np.zeros(n)
    lib().orc_gauss_legendre(n, _p(x), _p(w))
    return x, w


def sigma3(ly: Layers, l, lp, a, b, lrho):
    return lib().orc_sigma3(_p(ly.eps), _p(ly.lam), float(ly.d[0]), float(ly.d[1]), l, lp, a, b, float(lrho))


def sigma_stack(ly: Layers, l, lp, a, b, lrho):
    """sigma^{ab}_{l lp}(lrho) of any stack by the generalized reflection recursion."""
    return lib().orc_sigma_stack(ly.nlayers, _p(ly.eps), _p(ly.lam), _p(ly.d), l, lp, a, b, float(lrho))


def plm_beyond(n, m, w):
    out = np.zeros(2)
    lib().orc_plm_beyond(n, m, float(w), _p(out))
    return out[0] + 1j * out[1]


def legendre_product(n, m, nu, mu, lam, lamp, lrho):
    out = np.zeros(4)
    lib().orc_legendre_product(n, m, nu, mu, float(lam), float(lamp), float(lrho), _p(out))
    return out[0] + 1j * out[1], out[2] + 1j * out[3]


# --- Green's function ------------------------------------------------------

def reaction_u(ly: Layers, l, lp, a, b, r, rp):
    return lib().orc_reaction_u(_p(ly.eps), _p(ly.lam), _p(ly.d), ly.L, l, lp, a, b,
                                float(r[0]), float(r[1]), float(r[2]),
                                float(rp[0]), float(rp[1]), float(rp[2]))


def direct_sum(ly: Layers, x, y, z, q, targets=None, nthreads=0):
    x, y, z, q = map(_f64, (x, y, z, q))
    n = len(x)
    if targets is None:
        nt = n
        tp = None
    else:
        targets = np.ascontiguousarray(np.asarray(targets, dtype=np.int64))
        nt = len(targets)
        tp = targets.ctypes.data_as(_PL)
    phi = np.zeros(nt)
    rc = lib().orc_direct_sum(ly.nlayers, _p(ly.eps), _p(ly.lam), _p(ly.d), n, _p(x), _p(y), _p(z), _p(q),
                              nt, tp, _p(phi), int(nthreads))
    if rc != 0:
        raise RuntimeError(f"orc_direct_sum failed: {rc}")
    return phi


def num_components(nlayers):
    return lib().orc_num_components(nlayers)


def component(nlayers, c):
    out = (ctypes.c_int * 5)()
    if lib().orc_component(nlayers, c, out) != 0:
        raise IndexError(c)
    return tuple(out)


def fmm(ly: Layers, x, y, z, q, p, leaf_cap=50, nthreads=0, components=False, adaptive=0):
    """CPU FMM (Algorithm 2) on uniform trees (adaptive 0), or on adaptive
    trees with W- and X-lists (1: the reaction sets also divided near the
    interface; 2: by occupancy alone).  Returns phi, and with components=True also (comp_phi
    [ncomp, n], stats [ncomp, 8]: depth, target leaves, source leaves, V-list
    pairs, direct point pairs, unstable flag, W-list pairs, X-list pairs)."""
    x, y, z, q = map(_f64, (x, y, z, q))
    n = len(x)
    nc = num_components(ly.nlayers)
    phi = np.zeros(n)
    cphi = np.zeros((nc, n)) if components else None
    stats = np.zeros((nc, 8))
    rc = lib().orc_fmm(ly.nlayers, _p(ly.eps), _p(ly.lam), _p(ly.d), n, _p(x), _p(y), _p(z), _p(q),
                       int(p), int(leaf_cap), int(adaptive), int(nthreads), _p(phi),
                       _p(cphi) if components else None, _p(stats))
    if rc != 0:
        raise RuntimeError(f"orc_fmm failed: {rc}")
    if components:
        return phi, cphi, stats
    return phi


def component_tree(ly: Layers, x, y, z, comp, leaf_cap=50, adaptive=0):
    """Depth, each target's and source's leaf key and the root (centre, half
    side) of one component; adaptive=True also returns the leaf levels
    (keys are then at each point's own leaf level)."""
    x, y, z = map(_f64, (x, y, z))
    n = len(x)
    depth = ctypes.c_int()
    nt = ctypes.c_int64()
    ns = ctypes.c_int64()
    tk = np.zeros(n, dtype=np.uint64)
    sk = np.zeros(n, dtype=np.uint64)
    tl = np.zeros(n + 1, dtype=np.int32)
    sl = np.zeros(n + 1, dtype=np.int32)
    root = np.zeros(4)
    rc = lib().orc_component_tree(ly.nlayers, _p(ly.eps), _p(ly.lam), _p(ly.d), n, _p(x), _p(y), _p(z),
                                  comp, leaf_cap, int(adaptive), ctypes.byref(depth), ctypes.byref(nt),
                                  ctypes.byref(ns), tk.ctypes.data_as(_PU), sk.ctypes.data_as(_PU),
                                  tl.ctypes.data_as(_PI), sl.ctypes.data_as(_PI), _p(root))
    if rc != 0:
        raise RuntimeError("orc_component_tree failed")
    if adaptive:
        return (depth.value, tk[:nt.value].copy(), sk[:ns.value].copy(), root, tl[:nt.value].copy(),
                sl[:ns.value].copy())
    return depth.value, tk[:nt.value].copy(), sk[:ns.value].copy(), root


# --- operator pins ---------------------------------------------------------

def free_chain(p, lam, rs, cs, ct, r, cs2=None, ct2=None):
    mode = (1 if cs2 is not None else 0) | (2 if ct2 is not None else 0)
    cs2 = _f64(cs2 if cs2 is not None else cs)
    ct2 = _f64(ct2 if ct2 is not None else ct)
    return lib().orc_free_chain(p, float(lam), _p(_f64(rs)), _p(_f64(cs)), _p(cs2), _p(_f64(ct)), _p(ct2),
                                _p(_f64(r)), mode)


def addition_sum(p, pq, lam, n, m, b, r, which):
    out = np.zeros(2)
    lib().orc_addition_sum(p, pq, float(lam), n, m, _p(_f64(b)), _p(_f64(r)), which, _p(out))
    return out[0] + 1j * out[1]


def reaction_chain(ly: Layers, l, lp, a, b, p, rs, cs, ct, r):
    unstable = ctypes.c_int()
    v = lib().orc_reaction_chain(_p(ly.eps), _p(ly.lam), _p(ly.d), ly.L, l, lp, a, b, p,
                                 _p(_f64(rs)), _p(_f64(cs)), _p(_f64(ct)), _p(_f64(r)), ctypes.byref(unstable))
    return v, unstable.value


def reaction_I_pair(ly: Layers, l, lp, a, b, p, rho, zt, zs, S, n, m, nu, mu):
    out = np.zeros(4)
    lib().orc_reaction_I_pair(_p(ly.eps), _p(ly.lam), _p(ly.d), ly.L, l, lp, a, b, p, float(rho), float(zt),
                              float(zs), float(S), n, m, nu, mu, _p(out))
    return out[0] + 1j * out[1], out[2] + 1j * out[3]


def list_coverage(scells, tcells, cap, adaptive=True, H=0, sep=False):
    """(cover [nt, ns], counts [V, U, W, X]) of the oracle's lists between
    sources and targets given by fine cells ([n, 3] ints in 0..65535); sep:
    the reaction sets' separation rule."""
    sc = np.ascontiguousarray(np.asarray(scells, dtype=np.uint32).T)
    tc = np.ascontiguousarray(np.asarray(tcells, dtype=np.uint32).T)
    ns, nt = sc.shape[1], tc.shape[1]
    cover = np.zeros((nt, ns), dtype=np.int32)
    counts = np.zeros(4, dtype=np.int64)
    lib().orc_list_coverage(ns, sc.ctypes.data_as(_PU32), nt, tc.ctypes.data_as(_PU32), int(cap),
                            1 if adaptive else 0, 1 if sep else 0, int(H), cover.ctypes.data_as(_PI),
                            counts.ctypes.data_as(_PLL))
    return cover, counts


def free_point_chain(p, lam, rs, c, r, mode):
    """mode 0: ME of a unit source rs about c evaluated at r (M2P); mode 1: LE
    about c formed from rs (P2L) evaluated at r."""
    return lib().orc_free_point_chain(p, float(lam), _p(_f64(rs)), _p(_f64(c)), _p(_f64(r)), mode)


def reaction_point_chain(ly: Layers, l, lp, a, b, p, rs, c, r, S, mode):
    """Reaction component of a unit source rs: mode 0 = ME about the image-side
    centre c evaluated at r (M2P); mode 1 = LE about the target-side centre c
    formed from the image (P2L), evaluated at r."""
    return lib().orc_reaction_point_chain(_p(ly.eps), _p(ly.lam), _p(ly.d), ly.L, l, lp, a, b, p, _p(_f64(rs)),
                                          _p(_f64(c)), _p(_f64(r)), float(S), mode)


def reaction_I_point(ly: Layers, l, lp, a, b, p, rho, zt, zs, S, n, m, nu, mu):
    out = np.zeros(4)
    lib().orc_reaction_I_point(_p(ly.eps), _p(ly.lam), _p(ly.d), ly.L, l, lp, a, b, p, float(rho), float(zt),
                               float(zs), float(S), n, m, nu, mu, _p(out))
    return out[0] + 1j * out[1], out[2] + 1j * out[3]


def reaction_I_both(ly: Layers, l, lp, a, b, p, rho, zt, zs, S):
    """Whole I matrix of a reaction M2L (rows (n,m), columns (nu,mu)) by the
    recurrence path and by direct quadrature, the quadrature of the direct
    integrand's modulus and the rounding scale of the recurrence path;
    returns (rec, dir, dabs, rbound, unstable)."""
    K = (p + 1) ** 2
    rec = np.zeros(2 * K * K)
    dr = np.zeros(2 * K * K)
    da = np.zeros(K * K)
    rb = np.zeros(K * K)
    u = lib().orc_reaction_I_both(_p(ly.eps), _p(ly.lam), _p(ly.d), ly.L, l, lp, a, b, p, float(rho), float(zt),
                                  float(zs), float(S), _p(rec), _p(dr), _p(da), _p(rb))
    c = lambda v: (v[:K * K] + 1j * v[K * K:]).reshape(K, K)
    return c(rec), c(dr), da.reshape(K, K), rb.reshape(K, K), u


def sommerfeld_table(ly: Layers, l, lp, a, b, rho, zt, zs, S, nmax, mode):
    out = np.zeros((2, 2, nmax + 1, nmax + 1))
    rc = lib().orc_sommerfeld_table(_p(ly.eps), _p(ly.lam), _p(ly.d), ly.L, l, lp, a, b, float(rho), float(zt),
                                    float(zs), float(S), nmax, mode, _p(out))
    return out, rc
