"""Time stepping with online tuning: every step rebuilds the tree (positions
move), plans, evaluates, and reports the device time to the tuner, which
proposes the next N_levels and launch shapes (Sec. 4.2: the FMM is used in a
time-marching loop, each call is timed, moves are accepted or rejected on
the timings that follow).

Vortex-style advection dz/dt = conj(phi)/(2 pi i) with explicit Euler; the
update itself is an elementwise torch operation, not part of the FMM.
"""
import math

from . import Tuner, build_tree, evaluate, plan


def default_levels(n, per_leaf=16):
    """N_levels with about per_leaf points per leaf (4^(L-1) <= n)."""
    L = max(1, int(math.log(max(n, 1) / per_leaf, 4)) + 1)
    while L > 1 and 4 ** (L - 1) > n:
        L -= 1
    return L


def advect(z, m, steps, dt, p=16, theta=0.5, precision="mixed", tuner=None, n_levels=None, callback=None,
           smooth_delta=0.0):
    """Advance positions z (complex128 device tensor) by `steps` Euler steps.
    tuner: a Tuner (or None for fixed parameters).  callback(step, z, phi,
    params, seconds) is called after every evaluation.  smooth_delta > 0:
    the near field takes the Gaussian smoother of the vortex application
    (Sec. 5.1).  Returns the final z and the list of per-step (params,
    seconds)."""
    import torch
    L0 = n_levels or default_levels(z.numel())
    hist = []
    for step in range(steps):
        if tuner is not None:
            prm = tuner.next()
        else:
            prm = {"n_levels": L0, "p2p_split": 0, "m2l_batch": 0}
        L = min(prm["n_levels"], default_levels(z.numel(), per_leaf=1))
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        tree = build_tree(z, L)
        # a tuner that walks theta also carries the order for it (p from its tolerance)
        pp, th = (prm["p"], prm["theta"]) if getattr(tuner, "tunes_theta", False) else (p, theta)
        pl = plan(tree, pp, th, precision, p2p_split=prm["p2p_split"], m2l_batch=prm["m2l_batch"],
                  smooth_delta=smooth_delta)
        phi = evaluate(pl, m)
        e1.record()
        e1.synchronize()
        sec = e0.elapsed_time(e1) * 1e-3
        if tuner is not None:
            tuner.observe(sec)
        hist.append((dict(prm, n_levels=L), sec))
        if callback is not None:
            callback(step, z, phi, prm, sec)
        z = z + dt * torch.conj(phi) / (2j * math.pi)
    return z, hist


def make_tuner(n, **kw):
    """An AT3b-style tuner started at about 16 points per leaf."""
    L = default_levels(n)
    return Tuner(n_levels=L, min_levels=max(1, L - 3), max_levels=default_levels(n, per_leaf=1), **kw)
