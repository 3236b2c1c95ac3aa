"""The smoothed near field of the vortex application (Sec. 5.1, eq. 5.2)
through the C ABI, against the oracle's smoothed direct sum.  The far field
is left unsmoothed, exact to exp(-R^2/delta^2) with R the smallest leaf
radius; the inputs keep delta well below the leaf radii.  Bars: FP64 at
p = 30 within 1e-12, mixed precision within 1e-6."""
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


@pytest.mark.parametrize("n,L", [(20000, 5), (50001, 6)])
def test_smoothed_field_matches_direct_sum(F, orc, n, L):
    z, m, sp = W.kelvin_helmholtz(n, seed=1)
    delta = sp / 2
    tree = F.build_tree(dev(z), L)
    sub = np.arange(0, z.size, 7)
    ref = orc.direct_smoothed(z, m, delta, targets=sub)
    for prec, p, bar in (("fp64", 30, 1e-12), ("mixed", 16, 1e-6)):
        phi = F.evaluate(F.plan(tree, p, 0.5, prec, smooth_delta=delta), dev(m))
        assert e2(host(phi)[sub], ref) <= bar and einf(host(phi)[sub], ref) <= bar, prec
    # the smoothing matters at this delta: the unsmoothed field differs
    plain = F.evaluate(F.plan(tree, 30, 0.5, "fp64"), dev(m))
    assert e2(host(plain)[sub], ref) > 1e-6


def test_vanishing_delta_is_the_plain_field(F):
    z, m, _ = W.uniform(30000, seed=2)
    tree = F.build_tree(dev(z), 6)
    for prec in ("fp64", "mixed"):
        a = F.evaluate(F.plan(tree, 16, 0.5, prec, smooth_delta=1e-12), dev(m))
        b = F.evaluate(F.plan(tree, 16, 0.5, prec), dev(m))
        np.testing.assert_array_equal(host(a), host(b))


def test_smoothing_is_refused_where_it_is_not_implemented(F):
    z, m, sp = W.kelvin_helmholtz(4000, seed=3)
    tree = F.build_tree(dev(z), 4)
    pl = F.plan(tree, 12, 0.5, "fp64", smooth_delta=sp / 2)
    phi = F.evaluate(pl, dev(m))
    with pytest.raises(F.FmmError):
        F.evaluate_field(pl, dev(m))
    with pytest.raises(F.FmmError):
        F.evaluate_adjoint(pl, dev(m), phi)
    for bad in (-1.0, float("inf"), float("nan")):
        with pytest.raises(F.FmmError):
            F.plan(tree, 12, 0.5, "fp64", smooth_delta=bad)


def test_kelvin_helmholtz_steps(F, orc):
    """A few Euler steps of the vortex sheet with the smoothed kernel and the
    tuner; the field of the evolving points stays within the mixed bar."""
    import torch
    from paper_1311_1006_amd.driver import advect, make_tuner
    z, m, sp = W.kelvin_helmholtz(40000, seed=4)
    delta = sp / 2
    tu = make_tuner(z.size, cap=0.1, window=2, knob_interval=3)
    errs = {}

    def check(step, zt, phi, prm, sec):
        if step in (0, 5):
            zh = host(zt)
            sub = np.arange(0, zh.size, 13)
            ref = orc.direct_smoothed(zh, m, delta, targets=sub)
            errs[step] = max(e2(host(phi)[sub], ref), einf(host(phi)[sub], ref))

    zf, hist = advect(dev(z), dev(m), 6, 1e-3, p=16, precision="mixed", tuner=tu, callback=check,
                      smooth_delta=delta)
    assert errs[0] <= 1e-6 and errs[5] <= 1e-6, errs
    assert torch.isfinite(zf.real).all() and torch.isfinite(zf.imag).all()
