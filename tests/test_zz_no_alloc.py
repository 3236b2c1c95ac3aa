"""fmm_evaluate_static (the evaluation that allocates nothing, its working
memory in the library's fixed device array) against fmm_evaluate on the same
plans, through the C ABI: two calls in a row, the second on a smaller
problem, in both precisions.  The two run the same kernels, so the results
must be identical bit for bit."""
import ctypes as C

import numpy as np
import pytest

from paper_1311_1006_amd import workloads as W

from gpu_util import dev, host

pytestmark = pytest.mark.gpu

STATIC_BYTES = 64 << 20
FMM_EINVAL, FMM_ESTATE = -1, -4


@pytest.fixture(scope="module")
def F():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_1311_1006_amd as F
    F.lib()
    return F


def _static(F, pl, m, out):
    return F.lib().fmm_evaluate_static(pl._h, C.c_void_p(m.data_ptr()), C.c_void_p(out.data_ptr()),
                                       F._stream(None))


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_static_matches_evaluate_two_calls(F, prec):
    import torch
    for n, L, seed in ((300000, 8, 21), (70001, 6, 22)):     # the second call smaller
        z, m, _ = W.uniform(n, seed=seed)
        pl = F.plan(F.build_tree(dev(z), L), 13, 0.5, prec)
        md = dev(m)
        ref = F.evaluate(pl, md)                            # also makes the plan's lists final
        assert 0 < pl.stats()["static_bytes"] <= STATIC_BYTES
        out = torch.full_like(md, float("nan"))
        assert _static(F, pl, md, out) == 0, F.lib().fmm_last_error()
        np.testing.assert_array_equal(host(out), host(ref))


def test_static_leaves_the_plan_state_alone(F):
    # the adjoint reads the plan's last fmm_evaluate: a static evaluation of
    # other strengths in between must not change it
    import torch
    z, m, _ = W.uniform(50000, seed=23)
    pl = F.plan(F.build_tree(dev(z), 6), 13, 0.5, "fp64")
    md, g = dev(m), dev(np.conj(m))
    F.evaluate(pl, md)
    gm0, gz0 = (host(t) for t in F.evaluate_adjoint(pl, md, g))
    F.evaluate(pl, md)
    other = dev(2.0 * m[::-1])
    out = torch.empty_like(md)
    assert _static(F, pl, other, out) == 0, F.lib().fmm_last_error()
    ref = F.evaluate(F.plan(F.build_tree(dev(z), 6), 13, 0.5, "fp64"), other)
    np.testing.assert_array_equal(host(out), host(ref))
    gm1, gz1 = (host(t) for t in F.evaluate_adjoint(pl, md, g))
    np.testing.assert_array_equal(gm1, gm0)
    np.testing.assert_array_equal(gz1, gz0)


def test_static_refuses_what_does_not_fit(F):
    import torch
    z, m, _ = W.uniform(1000000, seed=24)
    pl = F.plan(F.build_tree(dev(z), 9), 13, 0.5, "fp64")
    md = dev(m)
    F.evaluate(pl, md)
    assert pl.stats()["static_bytes"] > STATIC_BYTES
    out = torch.zeros_like(md)
    assert _static(F, pl, md, out) == FMM_EINVAL
    assert "more than the fixed" in F.lib().fmm_last_error().decode()
    assert not bool(torch.any(out != 0))                     # no partial output
