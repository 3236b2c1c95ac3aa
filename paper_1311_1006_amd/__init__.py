"""MI355X (gfx950) fast multipole method for the 2D harmonic kernel.

Python binding of the C ABI declared in ``include/fmm.h`` (argument
marshalling only; every step of the method runs in the HIP library
``libfmm_hip.so``).  Device arrays are torch tensors on the current HIP
device; complex arrays are ``torch.complex128``.  Calls are ordered on the
current torch stream.

    tree = build_tree(z, n_levels=9)                      # Sec. 2.2
    pl = plan(tree, p=16, theta=0.5, precision="mixed")    # Sec. 2.1 lists
    phi = evaluate(pl, m)                                  # phi_i = sum m_j/(z_i - z_j)
    g_m, g_z = evaluate_adjoint(pl, m, g_phi)              # transposed chain

The library must be built (``python -m paper_1311_1006_amd.build`` or
``__graft_entry__.build()``); there is no fallback.
"""
import ctypes as C
import os
import re

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfmm_hip.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "fmm.h")

FMM_FP64, FMM_MIXED = 0, 1
FMM_FLAG_GRAPH, FMM_FLAG_PHASE_TIMING, FMM_FLAG_LEVELWISE = 1, 2, 4
_PREC = {"fp64": FMM_FP64, "mixed": FMM_MIXED, FMM_FP64: FMM_FP64, FMM_MIXED: FMM_MIXED}


class FmmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("fmm error %d: %s" % (code, msg))
        self.code = code


class _Tuning(C.Structure):
    _fields_ = [("p2p_split", C.c_int), ("m2l_batch", C.c_int), ("flags", C.c_int), ("p2p_targets", C.c_int),
                ("smooth_delta", C.c_double), ("p2p_src_tile", C.c_int), ("reserved", C.c_int)]


class _Stats(C.Structure):
    _fields_ = [("n_points", C.c_int64), ("n_boxes", C.c_int64), ("n_leaves", C.c_int64),
                ("n_p2p_pairs", C.c_int64), ("n_m2l_pairs", C.c_int64), ("n_strong_entries", C.c_int64),
                ("p", C.c_int), ("precision", C.c_int), ("max_levels", C.c_int), ("nprob", C.c_int),
                ("theta", C.c_double),
                ("t_upward_us", C.c_double), ("t_m2l_us", C.c_double), ("t_downward_us", C.c_double),
                ("t_p2p_us", C.c_double), ("t_total_us", C.c_double), ("t_tree_us", C.c_double),
                ("t_plan_us", C.c_double), ("t_l2l_us", C.c_double), ("static_bytes", C.c_int64)]


class _TunerParams(C.Structure):
    _fields_ = [("n_levels", C.c_int), ("p2p_split", C.c_int), ("m2l_batch", C.c_int), ("p", C.c_int),
                ("theta", C.c_double)]


class _TunerConfig(C.Structure):
    _fields_ = [("init", _TunerParams), ("min_levels", C.c_int), ("max_levels", C.c_int),
                ("cap", C.c_double), ("window", C.c_int), ("knob_interval", C.c_int),
                ("algorithm", C.c_int), ("level_interval", C.c_int), ("theta_interval", C.c_int),
                ("fib_length", C.c_int), ("theta_min", C.c_double), ("theta_max", C.c_double),
                ("theta_unit", C.c_double), ("tol", C.c_double), ("seed", C.c_ulonglong)]


_ALGORITHMS = {"at3b": 0, "at2": 1, "at1": 2}


_lib = None


def lib():
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libfmm_hip.so is not built (run python -m paper_1311_1006_amd.build)")
    L = C.CDLL(LIB_PATH)
    vp, dp, i64p, ip = C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int64), C.POINTER(C.c_int)
    sig = {
        "fmm_build_tree": (C.c_int, [vp, i64p, C.c_int, ip, vp, C.POINTER(vp)]),
        "fmm_tree_update_positions": (C.c_int, [vp, vp, vp]),
        "fmm_tree_destroy": (None, [vp]),
        "fmm_plan": (C.c_int, [vp, C.c_int, C.c_double, C.c_int, C.POINTER(_Tuning), vp, C.POINTER(vp)]),
        "fmm_plan_destroy": (None, [vp]),
        "fmm_evaluate": (C.c_int, [vp, vp, vp, vp]),
        "fmm_evaluate_parts": (C.c_int, [vp, vp, vp, vp, vp]),
        "fmm_evaluate_static": (C.c_int, [vp, vp, vp, vp]),
        "fmm_evaluate_adjoint": (C.c_int, [vp, vp, vp, vp, vp, vp]),
        "fmm_plan_stats": (C.c_int, [vp, C.POINTER(_Stats)]),
        "fmm_tree_layout": (C.c_int, [vp, C.c_int, ip, i64p, i64p]),
        "fmm_tree_download": (C.c_int, [vp, C.c_int, i64p, i64p, dp, vp]),
        "fmm_plan_list_size": (C.c_int, [vp, C.c_int, C.c_int, C.c_int, i64p]),
        "fmm_plan_download_list": (C.c_int, [vp, C.c_int, C.c_int, C.c_int, i64p, i64p, vp]),
        "fmm_tuner_create": (C.c_int, [C.POINTER(_TunerConfig), C.POINTER(vp)]),
        "fmm_tuner_next": (C.c_int, [vp, C.POINTER(_TunerParams)]),
        "fmm_tuner_observe": (C.c_int, [vp, C.c_double]),
        "fmm_tuner_best": (C.c_int, [vp, C.POINTER(_TunerParams), dp, dp]),
        "fmm_tuner_destroy": (None, [vp]),
        "fmm_evaluate_field": (C.c_int, [vp, vp, vp, vp, vp]),
        "fmm_evaluate_log": (C.c_int, [vp, vp, vp, vp]),
        "fmm_p_from_tol": (C.c_int, [C.c_double, C.c_double]),
        "fmm_choose_order": (C.c_int, [vp, vp, C.c_double, C.c_double, C.c_int, C.c_int, vp,
                                       C.POINTER(C.c_int), dp]),
        "fmm_last_error": (C.c_char_p, []),
        "fmm_evaluate_points": (C.c_int, [vp, vp, vp, C.c_int64, vp, vp, vp]),
        "fmm_debug_fail_alloc": (C.c_int, [C.c_int64]),
        "fmm_debug_live_blocks": (C.c_int, [i64p]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def header_functions():
    """Names of the functions declared in include/fmm.h."""
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fmm_[a-z0-9_]+)\s*\(", src)))


def _check(rc):
    if rc != 0:
        raise FmmError(rc, lib().fmm_last_error().decode())


def debug_fail_alloc(after):
    """Make the device allocation `after` allocations from now fail once
    with FMM_ENOMEM (after < 0: cancel)."""
    _check(lib().fmm_debug_fail_alloc(int(after)))


def debug_live_blocks():
    """Device blocks held by live trees, plans and schedules."""
    n = C.c_int64()
    _check(lib().fmm_debug_live_blocks(C.byref(n)))
    return n.value


def _stream(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def _dev_complex(t, name):
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.complex128):
        raise TypeError("%s must be a complex128 tensor on the HIP device" % name)
    return t.contiguous()


def p_from_tol(tol, theta):
    r = lib().fmm_p_from_tol(tol, theta)
    if r < 0:
        _check(r)
    return r


def choose_order(tree, m, theta=0.5, tol=5e-7, p_lo=8, p_hi=24, stream=None):
    """Smallest expansion order p in [p_lo, p_hi] whose FP64 and mixed results
    agree with an FP64 evaluation at a higher order (p = 32 for p_hi <= 24) to `tol` (relative 2-norm over all
    targets); returns (p, (err_fp64, err_mixed)), p = -1 when none does."""
    m = _dev_complex(m, "m")
    p = C.c_int(-1)
    err = (C.c_double * 2)()
    _check(lib().fmm_choose_order(tree._h, C.c_void_p(m.data_ptr()), float(theta), float(tol), int(p_lo),
                                  int(p_hi), _stream(stream), C.byref(p), err))
    return p.value, (err[0], err[1])


class Tree:
    """Balanced median-split tree of one or more problems (Sec. 2.2)."""

    def __init__(self, handle, offsets, n_levels, z):
        self._h = handle
        self.offsets = list(offsets)
        self.n_levels = list(n_levels)
        self.n = self.offsets[-1]
        self.device = z.device

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.fmm_tree_destroy(self._h)
            self._h = None

    def update_positions(self, z, stream=None):
        z = _dev_complex(z, "z")
        _check(lib().fmm_tree_update_positions(self._h, C.c_void_p(z.data_ptr()), _stream(stream)))

    def download(self, prob=0):
        import numpy as np
        L = lib()
        nl, n, nb = C.c_int(), C.c_int64(), C.c_int64()
        _check(L.fmm_tree_layout(self._h, prob, C.byref(nl), C.byref(n), C.byref(nb)))
        perm = np.zeros(n.value, np.int64)
        rng = np.zeros((nb.value, 2), np.int64)
        geom = np.zeros((nb.value, 7), np.float64)
        _check(L.fmm_tree_download(self._h, prob, perm.ctypes.data_as(C.POINTER(C.c_int64)),
                                   rng.ctypes.data_as(C.POINTER(C.c_int64)),
                                   geom.ctypes.data_as(C.POINTER(C.c_double)), _stream(None)))
        return perm, rng, geom


def build_tree(z, n_levels, offsets=None, stream=None):
    """z: complex128 device tensor of all problems' positions (concatenated);
    offsets: problem boundaries (default: one problem); n_levels: int or
    per-problem list."""
    z = _dev_complex(z, "z")
    if offsets is None:
        offsets = [0, z.numel()]
    nprob = len(offsets) - 1
    if isinstance(n_levels, int):
        n_levels = [n_levels] * nprob
    off = (C.c_int64 * (nprob + 1))(*offsets)
    lv = (C.c_int * nprob)(*n_levels)
    h = C.c_void_p()
    _check(lib().fmm_build_tree(C.c_void_p(z.data_ptr()), off, nprob, lv, _stream(stream), C.byref(h)))
    return Tree(h, offsets, n_levels, z)


class Plan:
    """Connectivity lists and launch structures for (p, theta, precision)."""

    def __init__(self, handle, tree, p, theta, precision):
        self._h = handle
        self.tree = tree
        self.p, self.theta, self.precision = p, theta, precision

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.fmm_plan_destroy(self._h)
            self._h = None

    def stats(self):
        st = _Stats()
        _check(lib().fmm_plan_stats(self._h, C.byref(st)))
        return {k: getattr(st, k) for k, _ in _Stats._fields_}

    def download_list(self, prob, level, kind):
        """CSR (off, ids) of the strong (kind 0) or weak (kind 1) list."""
        import numpy as np
        n = C.c_int64()
        _check(lib().fmm_plan_list_size(self._h, prob, level, kind, C.byref(n)))
        off = np.zeros(4 ** level + 1, np.int64)
        ids = np.zeros(max(n.value, 1), np.int64)
        _check(lib().fmm_plan_download_list(self._h, prob, level, kind, off.ctypes.data_as(C.POINTER(C.c_int64)),
                                            ids.ctypes.data_as(C.POINTER(C.c_int64)), _stream(None)))
        return off, ids[:n.value]


def plan(tree, p, theta, precision="fp64", p2p_split=0, m2l_batch=0, graph=False, timing=False, smooth_delta=0.0,
         stream=None, levelwise=False, p2p_targets=0, p2p_src_tile=0):
    """levelwise: the far field's upward and downward passes level by level
    (FMM_FLAG_LEVELWISE) instead of by subtrees.  p2p_split, p2p_targets,
    p2p_src_tile, m2l_batch: the launch-shape knobs of fmm_tuning (0: auto)."""
    flags = ((FMM_FLAG_GRAPH if graph else 0) | (FMM_FLAG_PHASE_TIMING if timing else 0) |
             (FMM_FLAG_LEVELWISE if levelwise else 0))
    tn = _Tuning(p2p_split, m2l_batch, flags, p2p_targets, float(smooth_delta), p2p_src_tile, 0)
    h = C.c_void_p()
    _check(lib().fmm_plan(tree._h, p, float(theta), _PREC[precision], C.byref(tn), _stream(stream), C.byref(h)))
    return Plan(h, tree, p, theta, precision)


def evaluate(pl, m, out=None, stream=None):
    import torch
    m = _dev_complex(m, "m")
    if out is None:
        out = torch.empty_like(m)
    _check(lib().fmm_evaluate(pl._h, C.c_void_p(m.data_ptr()), C.c_void_p(out.data_ptr()), _stream(stream)))
    return out


def evaluate_static(pl, m, out, stream=None):
    """fmm_evaluate_static: phi = FMM(m) into the caller's `out`, the
    evaluation's working memory taken from the library's fixed device array
    (the call allocates nothing).  The plan's lists must be final (one
    evaluate() or stats() first)."""
    m = _dev_complex(m, "m")
    if not out.is_contiguous():
        raise TypeError("out must be contiguous")
    out = _dev_complex(out, "out")
    _check(lib().fmm_evaluate_static(pl._h, C.c_void_p(m.data_ptr()), C.c_void_p(out.data_ptr()), _stream(stream)))
    return out


def evaluate_field(pl, m, phi=None, dphi=None, stream=None):
    """phi and its derivative dphi/dz at every point of the plan's tree."""
    import torch
    m = _dev_complex(m, "m")
    if phi is None:
        phi = torch.empty_like(m)
    if dphi is None:
        dphi = torch.empty_like(m)
    _check(lib().fmm_evaluate_field(pl._h, C.c_void_p(m.data_ptr()), C.c_void_p(phi.data_ptr()),
                                    C.c_void_p(dphi.data_ptr()), _stream(stream)))
    return phi, dphi


def evaluate_log(pl, q, out=None, stream=None):
    """The logarithmic potential u_i = sum over z_j != z_i of q_j log|z_i - z_j|
    for real strengths q (float64 device tensor, input order); returns u."""
    import torch
    if not (isinstance(q, torch.Tensor) and q.is_cuda and q.dtype == torch.float64):
        raise TypeError("q must be a float64 tensor on the HIP device")
    q = q.contiguous()
    if out is None:
        out = torch.empty_like(q)
    _check(lib().fmm_evaluate_log(pl._h, C.c_void_p(q.data_ptr()), C.c_void_p(out.data_ptr()), _stream(stream)))
    return out


def evaluate_points(pl, m, y, field=False, out=None, stream=None):
    """The field of the plan's sources (strengths m) at evaluation points y
    apart from them (eq. 2.2; fmm_evaluate_points).  Returns phi at y, or
    (phi, dphi) with field=True."""
    import torch
    m, y = _dev_complex(m, "m"), _dev_complex(y, "y")
    phi = torch.empty_like(y) if out is None else out
    dphi = torch.empty_like(y) if field else None
    _check(lib().fmm_evaluate_points(pl._h, C.c_void_p(m.data_ptr()), C.c_void_p(y.data_ptr()), y.numel(),
                                     C.c_void_p(phi.data_ptr()), C.c_void_p(dphi.data_ptr() if field else None),
                                     _stream(stream)))
    return (phi, dphi) if field else phi


def evaluate_at(z, m, y, p=16, theta=0.5, n_levels=None, precision="fp64", field=False, stream=None):
    """The field of the sources (z, m) at separate evaluation points y (eq.
    2.2): a tree and a plan over the sources alone, then fmm_evaluate_points.
    Returns phi at y, or (phi, dphi) with field=True."""
    z, m, y = _dev_complex(z, "z"), _dev_complex(m, "m"), _dev_complex(y, "y")
    if n_levels is None:
        from .driver import default_levels
        n_levels = default_levels(z.numel())
    tr = build_tree(z, n_levels, stream=stream)
    pl = plan(tr, p, theta, precision, stream=stream)
    return evaluate_points(pl, m, y, field=field, stream=stream)


def evaluate_parts(pl, m, stream=None):
    import torch
    m = _dev_complex(m, "m")
    near = torch.empty_like(m)
    far = torch.empty_like(m)
    _check(lib().fmm_evaluate_parts(pl._h, C.c_void_p(m.data_ptr()), C.c_void_p(near.data_ptr()),
                                    C.c_void_p(far.data_ptr()), _stream(stream)))
    return near, far


def evaluate_adjoint(pl, m, g_phi, stream=None):
    import torch
    m = _dev_complex(m, "m")
    g_phi = _dev_complex(g_phi, "g_phi")
    gm = torch.empty_like(m)
    gz = torch.empty_like(m)
    _check(lib().fmm_evaluate_adjoint(pl._h, C.c_void_p(m.data_ptr()), C.c_void_p(g_phi.data_ptr()),
                                      C.c_void_p(gm.data_ptr()), C.c_void_p(gz.data_ptr()), _stream(stream)))
    return gm, gz


class Tuner:
    """Online autotuner (Sec. 4.2; host only): the AT3b, AT2 or AT1 walk over
    N_levels and, with theta_interval > 0, theta (p following theta by
    Table 4.1's rule when tol > 0); AT3b also walks the P2P split and M2L
    batch knobs."""

    def __init__(self, n_levels, min_levels, max_levels, p2p_split=4, m2l_batch=4, cap=0.1, window=3,
                 knob_interval=6, algorithm="at3b", level_interval=6, theta=0.5, theta_interval=0,
                 theta_min=0.3, theta_max=0.7, theta_unit=0.01, fib_length=4, tol=0.0, p=0, seed=0):
        cfg = _TunerConfig(_TunerParams(n_levels, p2p_split, m2l_batch, p, theta), min_levels, max_levels, cap,
                           window, knob_interval, _ALGORITHMS[algorithm], level_interval, theta_interval,
                           fib_length, theta_min, theta_max, theta_unit, tol, seed)
        self._h = C.c_void_p()
        rc = lib().fmm_tuner_create(C.byref(cfg), C.byref(self._h))
        if rc != 0:
            raise FmmError(rc, "invalid tuner configuration")
        self.tunes_theta = theta_interval > 0 or tol > 0.0   # its parameters carry theta and p

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.fmm_tuner_destroy(self._h)
            self._h = None

    def next(self):
        p = _TunerParams()
        _check(lib().fmm_tuner_next(self._h, C.byref(p)))
        return _params_dict(p)

    def observe(self, seconds):
        _check(lib().fmm_tuner_observe(self._h, float(seconds)))

    def best(self):
        p = _TunerParams()
        cost, run = C.c_double(), C.c_double()
        _check(lib().fmm_tuner_best(self._h, C.byref(p), C.byref(cost), C.byref(run)))
        return _params_dict(p), cost.value, run.value


def _params_dict(p):
    return {"n_levels": p.n_levels, "p2p_split": p.p2p_split, "m2l_batch": p.m2l_batch, "p": p.p,
            "theta": p.theta}


def update_positions(tree, z, stream=None):
    """Replace the tree's positions, keeping its geometry frozen."""
    tree.update_positions(z, stream)


class _Potential:
    """torch.autograd.Function: phi = FMM(z, m); backward runs the adjoint
    FMM (fmm_evaluate_adjoint) with the geometry of the forward frozen."""

    _fn = None

    @classmethod
    def fn(cls):
        if cls._fn is None:
            import torch

            class PotentialFn(torch.autograd.Function):
                @staticmethod
                def forward(ctx, z, m, p, theta, n_levels, precision):
                    tree = build_tree(z.detach(), n_levels)
                    pl = plan(tree, p, theta, precision)
                    md = m.detach().contiguous()
                    phi = evaluate(pl, md)
                    ctx.pl = pl
                    ctx.tree = tree
                    ctx.save_for_backward(md)
                    return phi

                @staticmethod
                def backward(ctx, g_phi):
                    (md,) = ctx.saved_tensors
                    # torch's gradient of a real loss w.r.t. a complex tensor is
                    # dL/dRe + i dL/dIm, the convention of fmm_evaluate_adjoint
                    g_m, g_z = evaluate_adjoint(ctx.pl, md, g_phi.contiguous())
                    return g_z, g_m, None, None, None, None

            cls._fn = PotentialFn
        return cls._fn


def potential(z, m, p=16, theta=0.5, n_levels=None, precision="fp64"):
    """phi_i = sum_{z_j != z_i} m_j / (z_i - z_j) by the FMM, differentiable in
    z and m (complex128 device tensors).  n_levels defaults to about 16
    points per leaf."""
    import math
    if n_levels is None:
        n_levels = max(1, int(math.log(max(z.numel(), 1) / 16.0, 4)) + 1)
        while 4 ** (n_levels - 1) > z.numel():
            n_levels -= 1
    return _Potential.fn().apply(z, m, p, theta, n_levels, precision)
