"""ctypes binding of liblpbfmm.so (declarations in include/lpb.h).

Argument marshalling only: every step of the computation runs in the HIP
library.  Arrays may be numpy (host) or torch CUDA tensors (device; their
data pointers are passed with on_device=1).  Loading fails loudly when the
library has not been built.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblpbfmm.so")

LPB_OK, LPB_EINVAL, LPB_ERANGE, LPB_ENOMEM, LPB_EDEVICE, LPB_ESTATE, LPB_ENUMERIC = 0, -1, -2, -3, -4, -5, -6
LPB_FP64, LPB_MIXED = 0, 1

_D = ctypes.c_double
_I = ctypes.c_int
_L = ctypes.c_int64
_P = ctypes.c_void_p
_PD = ctypes.POINTER(ctypes.c_double)


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class Options(ctypes.Structure):
    _fields_ = [("p", _I), ("leaf_cap", _I), ("precision", _I), ("quad_tol", _D), ("iface_tol", _D),
                ("device", _I), ("stream", _P), ("stages", _I), ("timing", _I), ("graph", _I), ("autotune", _I),
                ("schedule", _I), ("alloc", ALLOC_FN), ("free", FREE_FN), ("alloc_user", _P), ("adaptive", _I)]


class Allocator:
    """Device-memory hook of lpb_options: alloc(nbytes) -> int pointer (0 when
    it cannot) and free(ptr), wrapped as C callbacks (kept alive with the
    context that uses them)."""

    def __init__(self, alloc, free):
        self.c_alloc = ALLOC_FN(lambda n, user: alloc(int(n)) or None)
        self.c_free = FREE_FN(lambda ptr, user: free(int(ptr)))


def torch_allocator(device=0, stream=None):
    """An Allocator backed by PyTorch's caching allocator on `device`."""
    import torch

    return Allocator(lambda n: torch.cuda.caching_allocator_alloc(n, device=device, stream=stream),
                     torch.cuda.caching_allocator_delete)


class Stats(ctypes.Structure):
    _fields_ = [("n_fmm", _I), ("max_depth", _I), ("n_m2l_pairs", _L), ("n_m2l_tile_pairs", _L), ("n_p2p_pairs", _L),
                ("n_react_p2p_pairs", _L), ("n_operators", _L), ("operator_bytes", _L),
                ("t_build_ms", _D), ("t_opgen_ms", _D), ("t_eval_ms", _D), ("t_stage_ms", _D * 10),
                ("tile_schedule", _I), ("batch_schedule", _I), ("t_tune_ms", _D), ("n_m2l_tiles", _L),
                ("n_p2m_points", _L), ("n_l2p_points", _L), ("n_m2m_links", _L), ("n_l2l_links", _L),
                ("n_m2l_list_ops", _L), ("n_w_pairs", _L), ("n_x_pairs", _L), ("n_w_points", _L),
                ("n_x_points", _L), ("n_point_ops", _L)]

    STAGES = ["setup", "p2m", "m2m", "m2l_tile", "m2l_list", "l2l", "l2p", "p2p_free", "p2p_react", "sum"]

    def as_dict(self):
        d = {f: getattr(self, f) for f, _ in self._fields_ if f != "t_stage_ms"}
        d["t_stage_ms"] = dict(zip(self.STAGES, list(self.t_stage_ms)))
        return d


EXPORTS = ["lpb_default_options", "lpb_create", "lpb_set_layers", "lpb_build_tree", "lpb_evaluate",
           "lpb_set_systems", "lpb_build_trees", "lpb_evaluate_batch", "lpb_get_stats", "lpb_fmm_info",
           "lpb_debug_parts", "lpb_last_error", "lpb_destroy", "lpb_host_gaunt", "lpb_evaluate_noalloc"]

_lib = None


class LpbError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"lpb status {status}: {msg}")
        self.status = status


def load():
    """Load liblpbfmm.so (built by paper_2002_01334_amd/build.py)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2002_01334_amd/build.py")
    L = ctypes.CDLL(LIB_PATH)
    L.lpb_default_options.argtypes = [ctypes.POINTER(Options)]
    L.lpb_default_options.restype = None
    L.lpb_create.argtypes = [ctypes.POINTER(Options), ctypes.POINTER(_P)]
    L.lpb_create.restype = _I
    L.lpb_set_layers.argtypes = [_P, _I, _PD, _PD, _PD]
    L.lpb_set_layers.restype = _I
    L.lpb_build_tree.argtypes = [_P, _L, _P, _P, _P, _I]
    L.lpb_build_tree.restype = _I
    L.lpb_evaluate.argtypes = [_P, _P, _P, _I]
    L.lpb_evaluate.restype = _I
    L.lpb_set_systems.argtypes = [_P, _I, ctypes.POINTER(_I), ctypes.POINTER(_P), ctypes.POINTER(_P), ctypes.POINTER(_P)]
    L.lpb_set_systems.restype = _I
    L.lpb_build_trees.argtypes = [_P, _I, ctypes.POINTER(_L), ctypes.POINTER(_P), ctypes.POINTER(_P),
                                  ctypes.POINTER(_P), _I]
    L.lpb_build_trees.restype = _I
    L.lpb_evaluate_batch.argtypes = [_P, _I, ctypes.POINTER(_P), ctypes.POINTER(_P), _I]
    L.lpb_evaluate_batch.restype = _I
    L.lpb_get_stats.argtypes = [_P, ctypes.POINTER(Stats)]
    L.lpb_get_stats.restype = _I
    L.lpb_fmm_info.argtypes = [_P, _I, _I, ctypes.POINTER(_I), _PD, ctypes.POINTER(_L), ctypes.POINTER(_L), _P, _P]
    L.lpb_fmm_info.restype = _I
    L.lpb_debug_parts.argtypes = [_P, _P, ctypes.POINTER(_I)]
    L.lpb_debug_parts.restype = _I
    L.lpb_last_error.argtypes = [_P]
    L.lpb_last_error.restype = ctypes.c_char_p
    L.lpb_destroy.argtypes = [_P]
    L.lpb_destroy.restype = None
    L.lpb_evaluate_noalloc.argtypes = [_P, _P, _P]
    L.lpb_evaluate_noalloc.restype = _I
    L.lpb_host_gaunt.argtypes = [_I] * 6
    L.lpb_host_gaunt.restype = _D
    _lib = L
    return L


def _ptr(a):
    """(pointer, on_device, keepalive) of a numpy array or torch tensor of float64."""
    if isinstance(a, np.ndarray):
        a = np.ascontiguousarray(a, dtype=np.float64)
        return a.ctypes.data, 0, a
    import torch

    if isinstance(a, torch.Tensor):
        if a.dtype != torch.float64:
            raise TypeError("tensors must be float64")
        a = a.contiguous()
        return a.data_ptr(), (1 if a.is_cuda else 0), a
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    return a.ctypes.data, 0, a


class Context:
    """One lpb context (one GPU, one stream)."""

    def __init__(self, p=10, leaf_cap=50, precision=LPB_FP64, quad_tol=1e-16, iface_tol=1e-9, device=0,
                 stream=None, stages=3, timing=0, graph=1, autotune=1, schedule=0, allocator=None, adaptive=0):
        L = load()
        opt = Options()
        L.lpb_default_options(ctypes.byref(opt))
        self._allocator = allocator
        if allocator is not None:
            opt.alloc = allocator.c_alloc
            opt.free = allocator.c_free
        opt.p = p
        opt.leaf_cap = leaf_cap
        opt.precision = precision
        opt.quad_tol = quad_tol
        opt.iface_tol = iface_tol
        opt.device = device
        opt.stream = stream
        opt.stages = stages
        opt.timing = timing
        opt.graph = graph
        opt.autotune = autotune
        opt.schedule = schedule
        opt.adaptive = int(adaptive)
        h = _P()
        rc = L.lpb_create(ctypes.byref(opt), ctypes.byref(h))
        if rc != LPB_OK:
            raise LpbError(rc, L.lpb_last_error(None).decode())
        self._h = h
        self._L = L
        self.p = p
        self.n = 0

    def _check(self, rc):
        if rc != LPB_OK:
            raise LpbError(rc, self._L.lpb_last_error(self._h).decode())

    def set_layers(self, eps, lam, interfaces):
        eps = np.ascontiguousarray(eps, dtype=np.float64)
        lam = np.ascontiguousarray(lam, dtype=np.float64)
        d = np.ascontiguousarray(interfaces, dtype=np.float64)
        if d.size == 0:
            d = np.zeros(1)
        self._check(self._L.lpb_set_layers(self._h, len(eps), eps.ctypes.data_as(_PD), lam.ctypes.data_as(_PD),
                                           d.ctypes.data_as(_PD)))

    def build_tree(self, x, y, z):
        (px, dx, kx), (py, dy, ky), (pz, dz, kz) = _ptr(x), _ptr(y), _ptr(z)
        n = len(kx)
        self._check(self._L.lpb_build_tree(self._h, n, px, py, pz, dx))
        self.n = n

    def evaluate(self, q, out=None):
        pq, dq, kq = _ptr(q)
        if out is None:
            if dq:
                import torch

                out = torch.empty(self.n, dtype=torch.float64, device=kq.device)
            else:
                out = np.empty(self.n, dtype=np.float64)
        po, do, ko = _ptr(out)
        if do != dq:
            raise ValueError("q and phi must both be host or both be device arrays")
        self._check(self._L.lpb_evaluate(self._h, pq, po, dq))
        return ko

    def evaluate_noalloc(self, q, out):
        """lpb_evaluate_noalloc: q and out are float64 device tensors of n."""
        pq, dq, kq = _ptr(q)
        po, do, ko = _ptr(out)
        if not (dq and do):
            raise ValueError("evaluate_noalloc takes device tensors")
        self._check(self._L.lpb_evaluate_noalloc(self._h, pq, po))
        return ko

    def set_systems(self, eps_list, lam_list, d_list):
        n = len(eps_list)
        self._keep = [np.ascontiguousarray(a, dtype=np.float64) for a in (*eps_list, *lam_list, *d_list)]
        e = self._keep[:n]
        l = self._keep[n:2 * n]
        d = [a if a.size else np.zeros(1) for a in self._keep[2 * n:]]
        self._keep += d
        nl = (_I * n)(*[len(a) for a in e])
        arr = lambda xs: (_P * n)(*[a.ctypes.data for a in xs])
        self._check(self._L.lpb_set_systems(self._h, n, nl, arr(e), arr(l), arr(d)))
        self.nsys = n

    def build_trees(self, xs, ys, zs):
        n = len(xs)
        keep = [_ptr(a) for a in (*xs, *ys, *zs)]
        on_dev = keep[0][1]
        ns = (_L * n)(*[len(k[2]) for k in keep[:n]])
        arr = lambda ks: (_P * n)(*[k[0] for k in ks])
        self._check(self._L.lpb_build_trees(self._h, n, ns, arr(keep[:n]), arr(keep[n:2 * n]), arr(keep[2 * n:]),
                                            on_dev))
        self.sizes = [len(k[2]) for k in keep[:n]]

    def evaluate_batch(self, qs, outs=None):
        n = len(qs)
        kq = [_ptr(a) for a in qs]
        on_dev = kq[0][1]
        if outs is None:
            if on_dev:
                import torch

                outs = [torch.empty(len(k[2]), dtype=torch.float64, device=k[2].device) for k in kq]
            else:
                outs = [np.empty(len(k[2])) for k in kq]
        ko = [_ptr(a) for a in outs]
        self._check(self._L.lpb_evaluate_batch(self._h, n, (_P * n)(*[k[0] for k in kq]),
                                               (_P * n)(*[k[0] for k in ko]), on_dev))
        return [k[2] for k in ko]

    def stats(self):
        s = Stats()
        self._check(self._L.lpb_get_stats(self._h, ctypes.byref(s)))
        return s.as_dict()

    def fmm_info(self, fmm, sys=0, keys=False):
        desc = (_I * 6)()
        root = np.zeros(4)
        nt = _L()
        ns = _L()
        rc = self._L.lpb_fmm_info(self._h, sys, fmm, desc, root.ctypes.data_as(_PD), ctypes.byref(nt),
                                  ctypes.byref(ns), None, None)
        if rc != LPB_OK:
            return None
        out = {"kind": desc[0], "l": desc[1], "lp": desc[2], "a": desc[3], "b": desc[4], "depth": desc[5],
               "root": root, "nt": nt.value, "ns": ns.value}
        if keys:
            tk = np.zeros(nt.value, dtype=np.uint64)
            sk = np.zeros(ns.value, dtype=np.uint64)
            self._check(self._L.lpb_fmm_info(self._h, sys, fmm, desc, root.ctypes.data_as(_PD), ctypes.byref(nt),
                                             ctypes.byref(ns), tk.ctypes.data, sk.ctypes.data))
            out["tkeys"] = tk
            out["skeys"] = sk
        return out

    def debug_parts(self):
        ns = _I()
        self._check(self._L.lpb_debug_parts(self._h, None, ctypes.byref(ns)))
        total = sum(self.sizes) if hasattr(self, "sizes") and self.sizes else self.n
        out = np.zeros((ns.value, total))
        self._check(self._L.lpb_debug_parts(self._h, out.ctypes.data, ctypes.byref(ns)))
        return out

    def close(self):
        if getattr(self, "_h", None):
            self._L.lpb_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def host_gaunt(n1, m1, n2, m2, n3, m3):
    return load().lpb_host_gaunt(n1, m1, n2, m2, n3, m3)
