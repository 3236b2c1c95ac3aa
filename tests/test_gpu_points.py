"""Evaluation points apart from the sources (eq. 2.2, fmm_evaluate_points)
through the C ABI, against the oracle's FP64 direct sums at the points.
Bars: FP64 at p = 40 within 1e-12 (a point takes a multipole expansion at a
distance of at least 1/theta of its radius, so the truncation is below
0.5^40 ~ 1e-12 there),
mixed precision within 1e-6 in e2 and e_inf; every point placement the
method distinguishes: inside the leaves' discs, outside them (they stop at an
upper level), outside the root's box, on a source (left out, as (2.2) says),
and not finite."""
import numpy as np
import pytest

from paper_1311_1006_amd import workloads as W

from gpu_util import dev, e2, einf, host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_1311_1006_amd as F
    F.lib()
    return F


@pytest.fixture(scope="module")
def orc():
    import oracle
    return oracle


def _points(z, n, seed):
    """uniform points over the sources' extent and beyond, some on sources,
    some far outside, some on the corners of the sources' bounding square"""
    rng = np.random.default_rng(seed)
    x0, x1, y0, y1 = z.real.min(), z.real.max(), z.imag.min(), z.imag.max()
    y = (x0 - 0.1 + (x1 - x0 + 0.2) * rng.random(n)) + 1j * (y0 - 0.1 + (y1 - y0 + 0.2) * rng.random(n))
    y[:16] = z[rng.choice(z.size, 16, replace=False)]
    y[16:24] = 5.0 + 3j + rng.random(8)
    y[24:28] = [x0 + 1j * y0, x1 + 1j * y0, x0 + 1j * y1, x1 + 1j * y1]
    return y


@pytest.mark.parametrize("kind", ["uniform", "clustered"])
def test_points_fp64_and_derivative_match_direct_sum(F, orc, kind):
    if kind == "uniform":
        z, m, _ = W.uniform(40000, seed=21)
        L = 6
    else:
        z, m = W.clustered(40000, seed=22, nclusters=8)
        L = 7
    y = _points(z, 6000, seed=23)
    pl = F.plan(F.build_tree(dev(z), L), 40, 0.5, "fp64")
    phi, dphi = F.evaluate_points(pl, dev(m), dev(y), field=True)
    assert e2(host(phi), orc.direct_points(z, m, y)) <= 1e-12
    assert e2(host(dphi), orc.direct_deriv_points(z, m, y)) <= 1e-12
    # without the derivative the near field of points in leaves is summed by
    # the near-field kernel instead of one lane per point: the same values up
    # to rounding
    assert e2(host(F.evaluate_points(pl, dev(m), dev(y))), host(phi)) <= 1e-14


@pytest.mark.parametrize("kind", ["uniform", "clustered"])
def test_points_mixed_within_1e6(F, orc, kind):
    if kind == "uniform":
        z, m, _ = W.uniform(60000, seed=31)
        L = 7
    else:
        z, m = W.clustered(60000, seed=32, nclusters=16)
        L = 7
    y = _points(z, 8000, seed=33)
    pl = F.plan(F.build_tree(dev(z), L), 16, 0.5, "mixed")
    phi, dphi = F.evaluate_points(pl, dev(m), dev(y), field=True)
    ref = orc.direct_points(z, m, y)
    assert e2(host(phi), ref) <= 1e-6 and einf(host(phi), ref) <= 1e-6
    refd = orc.direct_deriv_points(z, m, y)
    assert e2(host(dphi), refd) <= 1e-6


def test_points_leave_the_sources_evaluation_alone(F, orc):
    z, m, _ = W.uniform(20000, seed=41)
    y = _points(z, 3000, seed=42)
    for prec in ("fp64", "mixed"):
        pl = F.plan(F.build_tree(dev(z), 5), 16, 0.5, prec)
        before = host(F.evaluate(pl, dev(m)))
        a = host(F.evaluate_points(pl, dev(m), dev(y)))
        # the plan now holds the far field of m, not a forward evaluation
        with pytest.raises(F.FmmError) as ex:
            F.evaluate_adjoint(pl, dev(m), dev(np.ones(z.size, complex)))
        assert ex.value.code == -4
        b = host(F.evaluate_points(pl, dev(m), dev(y)))
        assert np.array_equal(a, b)                              # deterministic
        assert np.array_equal(host(F.evaluate(pl, dev(m))), before)


def test_points_one_level_and_not_finite(F, orc):
    z, m, _ = W.uniform(3000, seed=51)
    y = _points(z, 500, seed=52)
    y[100] = complex(np.nan, 0.5)
    pl = F.plan(F.build_tree(dev(z), 1), 40, 0.5, "fp64")    # the root is the only box
    phi = host(F.evaluate_points(pl, dev(m), dev(y)))
    assert np.isnan(phi[100])
    keep = np.arange(y.size) != 100
    assert e2(phi[keep], orc.direct_points(z, m, y[keep])) <= 1e-13


def test_points_arguments(F):
    import ctypes as C
    import torch
    z, m, _ = W.uniform(4000, seed=61)
    md = dev(m)
    pl = F.plan(F.build_tree(dev(z), 3), 8, 0.5, "fp64")
    empty = torch.empty(0, dtype=torch.complex128, device="cuda")
    assert F.evaluate_points(pl, md, empty).numel() == 0
    rc = F.lib().fmm_evaluate_points(pl._h, C.c_void_p(md.data_ptr()), None, 5, None, None, None)
    assert rc == -1
    # a batch of two problems
    tb = F.build_tree(dev(np.concatenate([z, z])), [3, 3], offsets=[0, z.size, 2 * z.size])
    pb = F.plan(tb, 8, 0.5, "fp64")
    with pytest.raises(F.FmmError) as ex:
        F.evaluate_points(pb, dev(np.concatenate([m, m])), dev(z[:10]))
    assert ex.value.code == -1
    # a smoothed near field
    ps = F.plan(F.build_tree(dev(z), 3), 8, 0.5, "fp64", smooth_delta=1e-3)
    with pytest.raises(F.FmmError) as ex:
        F.evaluate_points(ps, md, dev(z[:10]))
    assert ex.value.code == -1


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-6), ("mixed", 1e-6)])
def test_points_full_size(F, orc, prec, tol):
    """N = 1e6 sources, N_levels 9, p = 13 (the headline configuration), and
    1e6 separate uniform points: 2000 of them against the direct sum."""
    z, m, _ = W.uniform(1_000_000, seed=0)
    rng = np.random.default_rng(71)
    y = rng.random(1_000_000) + 1j * rng.random(1_000_000)
    pl = F.plan(F.build_tree(dev(z), 9), 13, 0.5, prec)
    phi = host(F.evaluate_points(pl, dev(m), dev(y)))
    sub = rng.choice(y.size, 2000, replace=False)
    ref = orc.direct_points(z, m, y[sub])
    assert e2(phi[sub], ref) <= tol and einf(phi[sub], ref) <= tol
