"""The derivative of the field (fmm_evaluate_field) and evaluation points
apart from the sources (eq. 2.2), through the C ABI, against the FP64 direct
sums of the oracle.  Bars: FP64 at p = 30 within 1e-12 (the FP64 bar of the
FMM; the truncation error there is ~1e-14), mixed precision within 1e-6;
phi from fmm_evaluate_field equals fmm_evaluate's bit for bit."""
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


@pytest.mark.parametrize("n,L", [(20000, 5), (7777, 4)])
def test_field_derivative_matches_direct_sum(F, orc, n, L):
    z, m, _ = W.uniform(n, seed=n)
    tree = F.build_tree(dev(z), L)
    sub = np.arange(0, n, 3)
    refd = orc.direct_deriv_points(z, m, z[sub])
    for prec, p, bar in (("fp64", 30, 1e-12), ("mixed", 16, 1e-6)):
        pl = F.plan(tree, p, 0.5, prec)
        phi, dphi = F.evaluate_field(pl, dev(m))
        assert e2(host(dphi)[sub], refd) <= bar and einf(host(dphi)[sub], refd) <= bar, prec
        plain = F.evaluate(F.plan(tree, p, 0.5, prec), dev(m))
        np.testing.assert_array_equal(host(phi), host(plain))


def test_field_derivative_converges_with_p(F, orc):
    n, L = 20000, 5
    z, m, _ = W.uniform(n, seed=3)
    tree = F.build_tree(dev(z), L)
    sub = np.arange(0, n, 5)
    refd = orc.direct_deriv_points(z, m, z[sub])
    errs = []
    for p in (8, 12, 16, 20, 24):
        _, dphi = F.evaluate_field(F.plan(tree, p, 0.5, "fp64"), dev(m))
        errs.append(e2(host(dphi)[sub], refd))
    assert all(b < a / 5 for a, b in zip(errs, errs[1:])), errs


def test_clustered_and_ragged_inputs(F, orc):
    z, _ = W.clustered(30001, seed=4, nclusters=6)
    m = np.random.default_rng(5).standard_normal(z.size) + 0j
    tree = F.build_tree(dev(z), 6)
    sub = np.arange(0, z.size, 7)
    _, dphi = F.evaluate_field(F.plan(tree, 30, 0.5, "fp64"), dev(m))
    assert e2(host(dphi)[sub], orc.direct_deriv_points(z, m, z[sub])) <= 1e-12


@pytest.mark.parametrize("prec,p,tol", [("fp64", 40, 1e-11), ("mixed", 16, 1e-6)])
def test_field_with_split_source_lists_then_adjoint(F, orc, prec, p, tol):
    # four tight clusters: boxes between clusters have strong lists of
    # hundreds of leaves, so the derivative's near field is summed in work
    # chunks whose partial sums are combined in order.  The adjoint on the
    # same plan shares the near-field buffer and the chunk partials (of which
    # the derivative writes only its own two sums): it must not see them, and
    # the derivative evaluated again after it must be the same bit for bit.
    z, m = W.clustered(20000, seed=3, nclusters=4, sigma=1e-5)
    L = 6
    pl = F.plan(F.build_tree(dev(z), L), p, 0.5, prec)
    off, _ = pl.download_list(0, L - 1, 0)
    assert np.diff(off).max() > 4 * (2048 // (20000 // 4 ** (L - 1) + 2))
    sub = np.arange(0, z.size, 7)
    refd = orc.direct_deriv_points(z, m, z[sub])
    phi, dphi = F.evaluate_field(pl, dev(m))
    assert e2(host(dphi)[sub], refd) <= tol and einf(host(dphi)[sub], refd) <= tol
    gm, gz = F.evaluate_adjoint(pl, dev(m), 2 * phi)
    rgm, rgz = orc.grad_direct(z, m, 2 * orc.direct(z, m))
    assert e2(host(gm), rgm) <= tol and e2(host(gz), rgz) <= tol
    _, dphi2 = F.evaluate_field(pl, dev(m))
    np.testing.assert_array_equal(host(dphi2), host(dphi))


def test_tiny_problems(F):
    # one point: no field; two points: dphi_0 = -m_1/(z_0 - z_1)^2 exactly enough
    _, d1 = F.evaluate_field(F.plan(F.build_tree(dev(np.array([0.3 + 0.4j])), 1), 8, 0.5), dev(np.array([2.0 + 1j])))
    assert np.all(host(d1) == 0)
    z = np.array([0.1 + 0.2j, 0.7 - 0.3j])
    m = np.array([1.5 - 0.5j, -0.25 + 2j])
    _, d2 = F.evaluate_field(F.plan(F.build_tree(dev(z), 1), 8, 0.5), dev(m))
    ref = np.array([-m[1] / (z[0] - z[1]) ** 2, -m[0] / (z[1] - z[0]) ** 2])
    assert e2(host(d2), ref) <= 1e-14


def test_separate_evaluation_points(F, orc):
    """Eq. 2.2: the field of the sources at points y; points placed on sources
    leave those sources out."""
    z, m, _ = W.uniform(30000, seed=6)
    rng = np.random.default_rng(7)
    y = rng.random(5000) + 1j * rng.random(5000)
    y[:10] = z[:10]
    y[10:20] = 2.0 + 1j * rng.random(10)          # outside the sources' square
    phi, dphi = F.evaluate_at(dev(z), dev(m), dev(y), p=40, field=True)
    assert e2(host(phi), orc.direct_points(z, m, y)) <= 1e-12
    assert e2(host(dphi), orc.direct_deriv_points(z, m, y)) <= 1e-12
    phim = F.evaluate_at(dev(z), dev(m), dev(y), p=16, precision="mixed")
    refm = orc.direct_points(z, m, y)
    assert e2(host(phim), refm) <= 1e-6 and einf(host(phim), refm) <= 1e-6


def test_field_rejects_null_arguments(F):
    import ctypes as C
    z, m, _ = W.uniform(100, seed=1)
    pl = F.plan(F.build_tree(dev(z), 2), 8, 0.5)
    md = dev(m)
    rc = F.lib().fmm_evaluate_field(pl._h, C.c_void_p(md.data_ptr()), C.c_void_p(md.data_ptr()), None, None)
    assert rc == -1
