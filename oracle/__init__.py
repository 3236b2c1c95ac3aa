"""Python shim over the FP64 CPU oracle (``fmm_oracle.c``).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import this package; the product library
never does.  Arrays are numpy: complex values as ``complex128`` (interleaved
re/im in memory), indices as ``int64``.

Functions (each follows the paper passage named in the C source):
  direct(z, m, targets=None)           O1, eq. (2.1)/(2.2), exclusion by position
  direct_points(z, m, y)               eq. (2.2), separate evaluation points
  direct_deriv_points(z, m, y)         the y-derivative of (2.2)'s field
  direct_smoothed(z, m, delta, targets=None)   O1 with the smoother of Sec. 5.1
  direct_log_points(z, q, y)           the logarithmic potential, real strengths
  direct_compensated(z, m)             O1 with Neumaier summation
  grad_direct(z, m, g)                 O3, gradient through the direct sum
  tree(z, L)                           balanced median-split pyramid, Sec. 2.2
  lists(geom, L, theta)                strong / weak connectivity, Sec. 2.1
  well_separated(gb, gc, theta)        theta-criterion (2.3)
  fmm(z, m, p, theta, L)               O2, the serial FMM
  p2m / m2m / m2l / l2l / l2p / mpole_eval   single expansion operators
  p_from_tol(tol, theta)               expansion order rule, Table 4.1
"""
import ctypes as C
import numpy as np

from . import build as _build

_lib = None


def lib():
    global _lib
    if _lib is None:
        path = _build.build()
        L = C.CDLL(path)
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int64)
        i64 = C.c_int64
        L.oracle_direct.argtypes = [i64, dp, dp, i64, ip, dp]
        L.oracle_direct_points.argtypes = [i64, dp, dp, i64, dp, dp]
        L.oracle_direct_deriv_points.argtypes = [i64, dp, dp, i64, dp, dp]
        L.oracle_direct_smoothed.argtypes = [i64, dp, dp, C.c_double, i64, ip, dp]
        L.oracle_direct_log_points.argtypes = [i64, dp, dp, i64, dp, dp]
        L.oracle_direct_compensated.argtypes = [i64, dp, dp, dp]
        L.oracle_grad_direct.argtypes = [i64, dp, dp, dp, dp, dp]
        L.oracle_p2m.argtypes = [dp, i64, dp, dp, C.c_int, dp]
        L.oracle_mpole_eval.argtypes = [dp, C.c_int, dp, i64, dp, dp]
        L.oracle_m2m.argtypes = [dp, dp, C.c_int, dp, dp]
        L.oracle_m2l.argtypes = [dp, dp, C.c_int, dp, dp]
        L.oracle_l2l.argtypes = [dp, dp, C.c_int, dp, dp]
        L.oracle_l2p.argtypes = [dp, C.c_int, dp, i64, dp, dp]
        L.oracle_tree.argtypes = [i64, dp, C.c_int, ip, ip, dp]
        L.oracle_tree.restype = C.c_int
        L.oracle_well_separated.argtypes = [dp, dp, C.c_double]
        L.oracle_well_separated.restype = C.c_int
        L.oracle_list_counts.argtypes = [C.c_int, dp, C.c_double, ip, ip]
        L.oracle_lists.argtypes = [C.c_int, dp, C.c_double, ip, ip, ip, ip]
        L.oracle_fmm.argtypes = [i64, dp, dp, C.c_int, C.c_double, C.c_int, dp, dp, dp]
        L.oracle_fmm.restype = C.c_int
        L.oracle_p_from_tol.argtypes = [C.c_double, C.c_double]
        L.oracle_p_from_tol.restype = C.c_int
        L.oracle_threads.argtypes = []
        L.oracle_threads.restype = C.c_int
        _lib = L
    return _lib


def _c(a):
    """complex128 contiguous view"""
    return np.ascontiguousarray(a, dtype=np.complex128)


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _ip(a):
    return a.ctypes.data_as(C.POINTER(C.c_int64))


def direct(z, m, targets=None):
    z, m = _c(z), _c(m)
    n = z.size
    if targets is None:
        out = np.zeros(n, np.complex128)
        lib().oracle_direct(n, _dp(z), _dp(m), n, None, _dp(out))
    else:
        t = np.ascontiguousarray(targets, dtype=np.int64)
        out = np.zeros(t.size, np.complex128)
        lib().oracle_direct(n, _dp(z), _dp(m), t.size, _ip(t), _dp(out))
    return out


def direct_points(z, m, y):
    z, m, y = _c(z), _c(m), _c(y)
    out = np.zeros(y.size, np.complex128)
    lib().oracle_direct_points(z.size, _dp(z), _dp(m), y.size, _dp(y), _dp(out))
    return out


def direct_smoothed(z, m, delta, targets=None):
    z, m = _c(z), _c(m)
    n = z.size
    if targets is None:
        out = np.zeros(n, np.complex128)
        lib().oracle_direct_smoothed(n, _dp(z), _dp(m), float(delta), n, None, _dp(out))
    else:
        t = np.ascontiguousarray(targets, dtype=np.int64)
        out = np.zeros(t.size, np.complex128)
        lib().oracle_direct_smoothed(n, _dp(z), _dp(m), float(delta), t.size, _ip(t), _dp(out))
    return out


def direct_log_points(z, q, y):
    """u_i = sum over z_j != y_i of q_j log|y_i - z_j| (real q, real u)."""
    z, y = _c(z), _c(y)
    q = np.ascontiguousarray(q, dtype=np.float64)
    assert q.shape == (z.size,)
    out = np.zeros(y.size, np.float64)
    lib().oracle_direct_log_points(z.size, _dp(z), _dp(q), y.size, _dp(y), _dp(out))
    return out


def direct_deriv_points(z, m, y):
    z, m, y = _c(z), _c(m), _c(y)
    out = np.zeros(y.size, np.complex128)
    lib().oracle_direct_deriv_points(z.size, _dp(z), _dp(m), y.size, _dp(y), _dp(out))
    return out


def direct_compensated(z, m):
    z, m = _c(z), _c(m)
    out = np.zeros(z.size, np.complex128)
    lib().oracle_direct_compensated(z.size, _dp(z), _dp(m), _dp(out))
    return out


def grad_direct(z, m, g):
    z, m, g = _c(z), _c(m), _c(g)
    gm = np.zeros(z.size, np.complex128)
    gz = np.zeros(z.size, np.complex128)
    lib().oracle_grad_direct(z.size, _dp(z), _dp(m), _dp(g), _dp(gm), _dp(gz))
    return gm, gz


def nbox(L):
    return (4 ** L - 1) // 3


def level_base(l):
    return (4 ** l - 1) // 3


def tree(z, L):
    """Returns (perm, range[nbox,2], geom[nbox,7]); raises on invalid L."""
    z = _c(z)
    n = z.size
    nb = nbox(L)
    perm = np.zeros(n, np.int64)
    rng = np.zeros((nb, 2), np.int64)
    geom = np.zeros((nb, 7), np.float64)
    rc = lib().oracle_tree(n, _dp(z), L, _ip(perm), _ip(rng), _dp(geom))
    if rc != 0:
        raise ValueError("invalid tree parameters")
    return perm, rng, geom


def well_separated(gb, gc, theta):
    gb = np.ascontiguousarray(gb, np.float64)
    gc = np.ascontiguousarray(gc, np.float64)
    return bool(lib().oracle_well_separated(_dp(gb), _dp(gc), theta))


def lists(geom, L, theta):
    """Per level l: (strong_off, strong_ids, weak_off, weak_ids) with
    level-local box indices; returns a list of L such tuples."""
    geom = np.ascontiguousarray(geom, np.float64)
    ns = np.zeros(L, np.int64)
    nw = np.zeros(L, np.int64)
    lib().oracle_list_counts(L, _dp(geom), theta, _ip(ns), _ip(nw))
    noff = nbox(L) + L
    soff = np.zeros(noff, np.int64)
    woff = np.zeros(noff, np.int64)
    sid = np.zeros(int(ns.sum()) + 1, np.int64)
    wid = np.zeros(int(nw.sum()) + 1, np.int64)
    lib().oracle_lists(L, _dp(geom), theta, _ip(soff), _ip(sid), _ip(woff), _ip(wid))
    out = []
    s0 = w0 = 0
    for l in range(L):
        o = level_base(l) + l
        nb = 4 ** l
        so = soff[o:o + nb + 1].copy()
        wo = woff[o:o + nb + 1].copy()
        out.append((so, sid[s0:s0 + so[-1]].copy(), wo, wid[w0:w0 + wo[-1]].copy()))
        s0 += so[-1]
        w0 += wo[-1]
    return out


def fmm(z, m, p, theta, L, parts=False):
    z, m = _c(z), _c(m)
    n = z.size
    phi = np.zeros(n, np.complex128)
    near = np.zeros(n, np.complex128)
    far = np.zeros(n, np.complex128)
    rc = lib().oracle_fmm(n, _dp(z), _dp(m), p, theta, L, _dp(phi), _dp(near), _dp(far))
    if rc != 0:
        raise ValueError("invalid FMM parameters")
    return (phi, near, far) if parts else phi


def p2m(c, z, m, p):
    c = _c(np.atleast_1d(c))
    z, m = _c(z), _c(m)
    a = np.zeros(p, np.complex128)
    lib().oracle_p2m(_dp(c), z.size, _dp(z), _dp(m), p, _dp(a))
    return a


def mpole_eval(c, a, z):
    c = _c(np.atleast_1d(c))
    a, z = _c(a), _c(z)
    out = np.zeros(z.size, np.complex128)
    lib().oracle_mpole_eval(_dp(c), a.size, _dp(a), z.size, _dp(z), _dp(out))
    return out


def m2m(cc, cp, a):
    cc, cp, a = _c(np.atleast_1d(cc)), _c(np.atleast_1d(cp)), _c(a)
    out = np.zeros(a.size, np.complex128)
    lib().oracle_m2m(_dp(cc), _dp(cp), a.size, _dp(a), _dp(out))
    return out


def m2l(cs, ct, a):
    cs, ct, a = _c(np.atleast_1d(cs)), _c(np.atleast_1d(ct)), _c(a)
    out = np.zeros(a.size, np.complex128)
    lib().oracle_m2l(_dp(cs), _dp(ct), a.size, _dp(a), _dp(out))
    return out


def l2l(cp, cc, b):
    cp, cc, b = _c(np.atleast_1d(cp)), _c(np.atleast_1d(cc)), _c(b)
    out = np.zeros(b.size, np.complex128)
    lib().oracle_l2l(_dp(cp), _dp(cc), b.size, _dp(b), _dp(out))
    return out


def l2p(c, b, z):
    c, b, z = _c(np.atleast_1d(c)), _c(b), _c(z)
    out = np.zeros(z.size, np.complex128)
    lib().oracle_l2p(_dp(c), b.size, _dp(b), z.size, _dp(z), _dp(out))
    return out


def p_from_tol(tol, theta):
    return int(lib().oracle_p_from_tol(tol, theta))


def threads():
    """OpenMP threads the oracle's parallel loops use."""
    return int(lib().oracle_threads())


def rel_err2(phi, ref):
    """e_2 = ||phi - ref||_2 / ||ref||_2 (the paper does not define its
    relative error; this 2-norm reading is the primary metric)."""
    return float(np.linalg.norm(phi - ref) / np.linalg.norm(ref))


def rel_errinf(phi, ref):
    return float(np.max(np.abs(phi - ref)) / np.max(np.abs(ref)))
