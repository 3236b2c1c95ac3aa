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


def batch_levels(sizes, offset=0, per_leaf=16):
    """Per-problem N_levels of a batch: about per_leaf points per leaf, all
    moved by a common offset, each kept within 1 .. one point per leaf."""
    return [max(1, min(default_levels(n, per_leaf) + offset, default_levels(n, per_leaf=1))) for n in sizes]


def tune_batch(z, m, offsets, p, theta, precision, iterations=60, out=None, **kw):
    """Online autotuning of one batch of problems (CSR offsets, one tree) for
    repeated graph launches: the AT3b walk (Sec. 4.2, Algorithm 4) over a
    level offset shared by every problem (batch_levels; the tuner's N_levels
    3 is offset 0, its range 1 .. 5 offsets -2 .. +2) and the two launch-shape
    knobs (P2P split, M2L pair slots).  Every iteration replays the graph of
    the proposed configuration once (trees and plans are kept per
    configuration; a plan's first call captures its graph and is not timed)
    and reports the replay's device time.  Returns (best parameters with the
    level offset and the per-problem levels, per-iteration (parameters,
    seconds))."""
    import torch
    sizes = [int(offsets[b + 1] - offsets[b]) for b in range(len(offsets) - 1)]
    if out is None:
        out = torch.empty_like(m)
    kw.setdefault("window", 2)
    kw.setdefault("knob_interval", 4)
    tu = Tuner(n_levels=3, min_levels=1, max_levels=5, p2p_split=4, m2l_batch=4, **kw)
    trees, plans, hist = {}, {}, []
    for _ in range(iterations):
        prm = tu.next()
        off = prm["n_levels"] - 3
        Ls = tuple(batch_levels(sizes, off))
        if Ls not in trees:
            trees[Ls] = build_tree(z, list(Ls), offsets=list(offsets))
        key = (Ls, prm["p2p_split"], prm["m2l_batch"])
        if key not in plans:
            plans[key] = plan(trees[Ls], p, theta, precision, p2p_split=prm["p2p_split"],
                              m2l_batch=prm["m2l_batch"], graph=True)
            evaluate(plans[key], m, out)             # captures the graph
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        evaluate(plans[key], m, out)
        e1.record()
        e1.synchronize()
        sec = e0.elapsed_time(e1) * 1e-3
        tu.observe(sec)
        hist.append((dict(prm, level_offset=off), sec))
    best = tu.best()[0]
    off = best["n_levels"] - 3
    return dict(best, level_offset=off, levels=batch_levels(sizes, off)), hist


def make_tuner(n, **kw):
    """An AT3b-style tuner started at about 16 points per leaf."""
    L = default_levels(n)
    return Tuner(n_levels=L, min_levels=max(1, L - 3), max_levels=default_levels(n, per_leaf=1), **kw)
