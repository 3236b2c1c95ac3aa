"""Seeded synthetic inputs for the FMM workloads.

This module holds random-number recipes only, none of the method's
arithmetic; both the HIP path's tests/benchmark and the CPU oracle are fed
from it.  All generators use ``numpy.random.default_rng(seed)`` (PCG64) and
return complex128 arrays ``z`` (positions x + iy) and ``m`` (strengths).

The paper's experiments are time-stepping simulations described in prose
(Sec. 3.3: a million points uniform in the unit square; Sec. 4.1: a
line-like distribution; Sec. 5: vortex sheets and galaxies that cluster over
time).  There is no dataset; these recipes stand in for them.
"""
import math

import numpy as np


def uniform(n, seed=0, nsub=10000):
    """n points uniform in [0,1)^2, complex N(0,1) strengths (real and
    imaginary parts i.i.d.), plus a subsample of evaluation indices drawn
    without replacement (all indices when n <= nsub).  Draw order: positions,
    strengths, subsample."""
    rng = np.random.default_rng(seed)
    xy = rng.random((n, 2))
    g = rng.standard_normal((n, 2))
    z = xy[:, 0] + 1j * xy[:, 1]
    m = g[:, 0] + 1j * g[:, 1]
    if n > nsub:
        sub = np.sort(rng.choice(n, nsub, replace=False))
    else:
        sub = np.arange(n)
    return z, m, sub


def clustered(n=1_000_000, seed=0, nclusters=32, frac_clustered=0.9, sigma=1e-3):
    """Non-uniform case: 90% of the points in isotropic Gaussian clusters of
    width sigma around centres uniform in [0,1)^2, 10% uniform; real
    strengths +1/-1 in equal numbers, randomly placed; then a global random
    permutation of the points.  Draw order: centres, clustered offsets,
    uniform points, strength permutation, point permutation."""
    rng = np.random.default_rng(seed)
    centres = rng.random((nclusters, 2))
    nc = int(round(n * frac_clustered))
    per = nc // nclusters
    nc = per * nclusters
    nu = n - nc
    pts_c = rng.standard_normal((nc, 2)) * sigma + np.repeat(centres, per, axis=0)
    pts_u = rng.random((nu, 2))
    xy = np.concatenate([pts_c, pts_u], axis=0)
    s = np.concatenate([np.ones(n // 2), -np.ones(n - n // 2)])
    s = s[rng.permutation(n)]
    perm = rng.permutation(n)
    xy = xy[perm]
    z = xy[:, 0] + 1j * xy[:, 1]
    m = s.astype(np.complex128)
    return z, m


def line_like(n, seed=0, width=1e-3):
    """Points scattered approximately along a line (Sec. 4.1 studies such a
    distribution): x uniform in [0,1), y = 0.5 + 0.25*x + width*N(0,1);
    complex N(0,1) strengths."""
    rng = np.random.default_rng(seed)
    x = rng.random(n)
    y = 0.5 + 0.25 * x + width * rng.standard_normal(n)
    g = rng.standard_normal((n, 2))
    return x + 1j * y, g[:, 0] + 1j * g[:, 1]


def clusters4(n, rng, sigma=1e-3):
    """4 Gaussian clusters of width sigma, centres uniform in [0,1)^2, equal
    split (the remainder goes to the last cluster)."""
    centres = rng.random((4, 2))
    counts = [n // 4] * 3 + [n - 3 * (n // 4)]
    parts = [rng.standard_normal((c, 2)) * sigma + centres[i] for i, c in enumerate(counts)]
    xy = np.concatenate(parts, axis=0)
    return xy[:, 0] + 1j * xy[:, 1]


def batch(nprob=128, seed=0, nmin=1_000, nmax=200_000):
    """Many independent problems of uneven size: per problem, in order,
    N_b = round(exp(U(ln nmin, ln nmax))), kind = uniform if U < 0.5 else
    4-cluster, then positions, then complex N(0,1) strengths.  Returns lists
    (zs, ms, kinds)."""
    rng = np.random.default_rng(seed)
    zs, ms, kinds = [], [], []
    for _ in range(nprob):
        nb = int(round(math.exp(rng.uniform(math.log(nmin), math.log(nmax)))))
        kind = "uniform" if rng.uniform() < 0.5 else "clusters4"
        if kind == "uniform":
            xy = rng.random((nb, 2))
            z = xy[:, 0] + 1j * xy[:, 1]
        else:
            z = clusters4(nb, rng)
        g = rng.standard_normal((nb, 2))
        zs.append(z)
        ms.append(g[:, 0] + 1j * g[:, 1])
        kinds.append(kind)
    return zs, ms, kinds


def kelvin_helmholtz(n, seed=0, aspect=20.0, amp=1e-3):
    """The vortex-sheet start of Sec. 5.1: about n vortices on a regular grid
    in a long thin rectangle [0, 1] x [-h/2, h/2], h = 1/aspect, the upper
    half of the rows with strength +1/N and the lower half -1/N (total
    circulation zero), displaced by amp*h*sin(2 pi x) in y to seed the
    instability, plus a seeded jitter of 1e-6 of the spacing.  Returns
    (z, m, spacing); spacing = grid spacing in x (about that in y)."""
    ny = max(2, 2 * int(round(math.sqrt(n / aspect) / 2)))
    nx = max(1, n // ny)
    h = 1.0 / aspect
    xs = (np.arange(nx) + 0.5) / nx
    ys = ((np.arange(ny) + 0.5) / ny - 0.5) * h
    X, Y = np.meshgrid(xs, ys)
    X, Y = X.ravel(), Y.ravel()
    N = X.size
    m = np.where(Y > 0, 1.0, -1.0) / N + 0j
    rng = np.random.default_rng(seed)
    sp = 1.0 / nx
    Y = Y + amp * h * np.sin(2 * np.pi * X) + 1e-6 * sp * rng.standard_normal(N)
    X = X + 1e-6 * sp * rng.standard_normal(N)
    return X + 1j * Y, m, sp


def roots_of_unity(n, centre=0.0 + 0.0j, radius=1.0, phase=0.0):
    """n points equally spaced on a circle (closed-form test input)."""
    k = np.arange(n)
    return centre + radius * np.exp(1j * (2 * np.pi * k / n + phase))


def subsample(n, nsub, seed):
    """Sorted evaluation indices, drawn without replacement."""
    rng = np.random.default_rng(seed)
    if n <= nsub:
        return np.arange(n)
    return np.sort(rng.choice(n, nsub, replace=False))
