"""The adjoint FMM (fmm_evaluate_adjoint) against finite differences of the
same FMM with its geometry frozen, against the analytic gradient of the
direct sum (CPU oracle), and against the transposition identity
G_m = -conj(FMM[conj(g)]); plus the torch.autograd wrapper."""
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


def _loss(phi):
    return float(np.sum(np.abs(phi) ** 2))


def _separated(n, seed, dmin):
    """Uniform points in the unit square, a candidate closer than dmin to an
    accepted point is drawn again: a central difference with step h is only
    accurate when h is small against every pair distance."""
    rng = np.random.default_rng(seed)
    pts = np.empty(n, dtype=np.complex128)
    k = 0
    while k < n:
        c = rng.random() + 1j * rng.random()
        if k == 0 or np.min(np.abs(pts[:k] - c)) >= dmin:
            pts[k] = c
            k += 1
    m = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    return pts, m


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_adjoint_matches_direct_gradient(orc, F, prec):
    z, m, _ = W.uniform(2000, seed=1)
    pl = F.plan(F.build_tree(dev(z), 4), 16, 0.5, prec)
    phi = F.evaluate(pl, dev(m))
    g = 2 * phi                              # L = sum |phi|^2
    gm, gz = F.evaluate_adjoint(pl, dev(m), g)
    rgm, rgz = orc.grad_direct(z, m, 2 * orc.direct(z, m))
    # measured (N = 2000, p = 16): FP64 2e-9 / 7e-11, mixed 1.2e-7 / 1.6e-7
    # (the mixed error is that of the FP32 forward phi fed in as the cotangent
    # plus the adjoint's own FP32 sums, each ~1e-7)
    tol = 1e-6
    assert e2(host(gm), rgm) <= tol and einf(host(gm), rgm) <= tol
    assert e2(host(gz), rgz) <= tol and einf(host(gz), rgz) <= tol


@pytest.mark.parametrize("prec,p,tol", [("fp64", 40, 1e-11), ("mixed", 16, 1e-6)])
def test_adjoint_with_split_source_lists(orc, F, prec, p, tol):
    # four tight clusters: boxes that straddle two clusters have strong lists
    # of hundreds of leaves, so the adjoint near field is summed in work
    # chunks of whole list entries whose partial sums are combined in order
    z, m = W.clustered(20000, seed=3, nclusters=4, sigma=1e-5)
    L = 6
    pl = F.plan(F.build_tree(dev(z), L), p, 0.5, prec)
    off, _ = pl.download_list(0, L - 1, 0)
    assert np.diff(off).max() > 4 * (2048 // (20000 // 4 ** (L - 1) + 2))
    phi = F.evaluate(pl, dev(m))
    gm, gz = F.evaluate_adjoint(pl, dev(m), 2 * phi)
    rgm, rgz = orc.grad_direct(z, m, 2 * orc.direct(z, m))
    assert e2(host(gm), rgm) <= tol
    assert e2(host(gz), rgz) <= tol


def test_adjoint_matches_frozen_geometry_fd(F):
    # directional central differences (h = 1e-6, FP64) of L = sum |phi|^2 with
    # the tree geometry frozen (fmm_tree_update_positions).  The O(h^2) error
    # of the difference is about (h/d)^2 * 20/6 relative for the closest pair
    # distance d, so pairs are kept >= 1e-2 apart (uniform points put some
    # pairs within ~1e-6 of each other); then it is ~1e-7
    z, m = _separated(2000, seed=2, dmin=1e-2)
    tree = F.build_tree(dev(z), 4)
    pl = F.plan(tree, 16, 0.5, "fp64")
    md = dev(m)
    phi = F.evaluate(pl, md)
    gm, gz = F.evaluate_adjoint(pl, md, 2 * phi)
    gm, gz = host(gm), host(gz)
    rng = np.random.default_rng(3)
    h = 1e-6
    for _ in range(3):
        v = rng.standard_normal(2000) + 1j * rng.standard_normal(2000)
        tree.update_positions(dev(z + h * v))
        lp = _loss(host(F.evaluate(pl, md)))
        tree.update_positions(dev(z - h * v))
        lm = _loss(host(F.evaluate(pl, md)))
        fd = (lp - lm) / (2 * h)
        an = float(np.sum(np.real(np.conj(gz) * v)))
        assert abs(fd - an) <= 1e-6 * abs(an)
        tree.update_positions(dev(z))
        lp = _loss(host(F.evaluate(pl, dev(m + h * v))))
        lm = _loss(host(F.evaluate(pl, dev(m - h * v))))
        fd = (lp - lm) / (2 * h)
        an = float(np.sum(np.real(np.conj(gm) * v)))
        assert abs(fd - an) <= 1e-6 * abs(an)


def test_transposition_identity(F):
    # with symmetric lists the FMM operator is antisymmetric: A^T = -A, so
    # G_m = conj(A^T conj(g)) = -conj(FMM[conj(g)])
    z, m, _ = W.uniform(5000, seed=4)
    g = W.uniform(5000, seed=5)[1]
    pl = F.plan(F.build_tree(dev(z), 5), 16, 0.5, "fp64")
    F.evaluate(pl, dev(m))
    gm, _ = F.evaluate_adjoint(pl, dev(m), dev(g))
    ref = -np.conj(host(F.evaluate(pl, dev(np.conj(g)))))
    assert e2(host(gm), ref) <= 1e-12


def test_gradient_identities(F):
    z, m, _ = W.uniform(3000, seed=6)
    pl = F.plan(F.build_tree(dev(z), 4), 16, 0.5, "fp64")
    phi = F.evaluate(pl, dev(m))
    Lv = _loss(host(phi))
    gm, gz = F.evaluate_adjoint(pl, dev(m), 2 * phi)
    gm, gz = host(gm), host(gz)
    scale = np.sum(np.abs(gz * z)) + np.sum(np.abs(gm * m))
    # scaling of m: dL/de = 2L exactly (phi is linear in m)
    assert abs(np.sum(np.real(np.conj(gm) * m)) - 2 * Lv) <= 1e-12 * scale
    # rotations of m leave |phi| unchanged
    assert abs(np.sum(np.real(np.conj(gm) * 1j * m))) <= 1e-12 * scale
    # translation and scaling of z hold up to the FMM's truncation (frozen geometry)
    assert abs(np.sum(gz)) <= 1e-6 * np.sum(np.abs(gz))
    assert abs(np.sum(np.real(np.conj(gz) * z)) + 2 * Lv) <= 1e-6 * scale


def test_autograd_function(orc, F):
    import torch
    z, m, _ = W.uniform(2000, seed=7)
    zt = dev(z).requires_grad_(True)
    mt = dev(m).requires_grad_(True)
    phi = F.potential(zt, mt, p=16, theta=0.5, n_levels=4, precision="fp64")
    loss = (phi.abs() ** 2).sum()
    loss.backward()
    rgm, rgz = orc.grad_direct(z, m, 2 * orc.direct(z, m))
    assert e2(zt.grad.cpu().numpy(), rgz) <= 1e-6
    assert e2(mt.grad.cpu().numpy(), rgm) <= 1e-6
    # torch's own complex-gradient convention on a holomorphic map of m
    w = torch.tensor([1.0 + 2.0j], dtype=torch.complex128, requires_grad=True)
    (w.abs() ** 2).sum().backward()
    assert complex(w.grad[0]) == 2.0 + 4.0j
