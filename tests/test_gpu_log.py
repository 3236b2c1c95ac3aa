"""The logarithmic potential (fmm_evaluate_log; the paper's second kernel,
Sec. 3.3, with the a_0 log term of the multipole expansion, Sec. 2.1)
through the C ABI, against the FP64 direct sum of the oracle.  Bars: FP64 at
p = 30 within 1e-12 (relative 2-norm), mixed precision at p = 16 within 1e-6;
real strengths, u_i = sum over z_j != z_i of q_j log|z_i - z_j|."""
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


def devr(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda")


@pytest.mark.parametrize("n,L", [(20000, 5), (7777, 4), (30001, 6)])
def test_log_matches_direct_sum(F, orc, n, L):
    z, _, _ = W.uniform(n, seed=n)
    q = np.random.default_rng(n).standard_normal(n)
    tree = F.build_tree(dev(z), L)
    sub = np.arange(0, n, 3)
    ref = orc.direct_log_points(z, q, z[sub])
    for prec, p, bar in (("fp64", 30, 1e-12), ("mixed", 16, 1e-6)):
        u = host(F.evaluate_log(F.plan(tree, p, 0.5, prec), devr(q)))
        assert e2(u[sub], ref) <= bar, (prec, e2(u[sub], ref))


def test_log_clustered_and_line(F, orc):
    for z in (W.clustered(40000, seed=7, nclusters=8)[0], W.line_like(30000, seed=8)[0]):
        q = np.random.default_rng(9).standard_normal(z.size)
        tree = F.build_tree(dev(z), 6)
        sub = np.arange(0, z.size, 11)
        ref = orc.direct_log_points(z, q, z[sub])
        u = host(F.evaluate_log(F.plan(tree, 30, 0.5, "fp64"), devr(q)))
        assert e2(u[sub], ref) <= 1e-12
        um = host(F.evaluate_log(F.plan(tree, 16, 0.5, "mixed"), devr(q)))
        assert e2(um[sub], ref) <= 1e-6 and einf(um[sub], ref) <= 1e-6


def test_log_converges_with_p(F, orc):
    n = 20000
    z, _, _ = W.uniform(n, seed=5)
    q = np.random.default_rng(6).standard_normal(n)
    tree = F.build_tree(dev(z), 5)
    sub = np.arange(0, n, 7)
    ref = orc.direct_log_points(z, q, z[sub])
    errs = [e2(host(F.evaluate_log(F.plan(tree, p, 0.5, "fp64"), devr(q)))[sub], ref) for p in (6, 10, 14, 18)]
    assert all(b < a / 5 for a, b in zip(errs, errs[1:])), errs


def test_log_tiny_problems_and_one_box(F, orc):
    u1 = host(F.evaluate_log(F.plan(F.build_tree(dev(np.array([0.3 + 0.4j])), 1), 8, 0.5), devr(np.array([2.0]))))
    assert np.all(u1 == 0)
    z = np.array([0.1 + 0.2j, 0.7 - 0.3j, 0.1 + 0.2j])       # a coincident pair is left out
    q = np.array([1.5, -0.25, 2.0])
    u = host(F.evaluate_log(F.plan(F.build_tree(dev(z), 1), 8, 0.5), devr(q)))
    np.testing.assert_allclose(u, orc.direct_log_points(z, q, z), rtol=1e-14)
    z, _, _ = W.uniform(3000, seed=2)                           # N_levels = 1: all near field
    q = np.random.default_rng(2).standard_normal(z.size)
    u = host(F.evaluate_log(F.plan(F.build_tree(dev(z), 1), 8, 0.5), devr(q)))
    assert e2(u, orc.direct_log_points(z, q, z)) <= 1e-14


def test_log_batch_of_problems(F, orc):
    zs, _, _ = W.batch(nprob=5, seed=11, nmin=1000, nmax=20000)
    from paper_1311_1006_amd.driver import default_levels
    Ls = [default_levels(len(z)) for z in zs]
    off = np.concatenate([[0], np.cumsum([len(z) for z in zs])]).tolist()
    q = np.random.default_rng(12).standard_normal(off[-1])
    tree = F.build_tree(dev(np.concatenate(zs)), Ls, offsets=off)
    u = host(F.evaluate_log(F.plan(tree, 30, 0.5, "fp64"), devr(q)))
    for b in range(len(zs)):
        ref = orc.direct_log_points(zs[b], q[off[b]:off[b + 1]], zs[b])
        assert e2(u[off[b]:off[b + 1]], ref) <= 1e-12, b


def test_log_at_separate_points(F, orc):
    """Evaluation points with zero strength in the same tree (as for eq. 2.2)."""
    z, _, _ = W.uniform(20000, seed=13)
    rng = np.random.default_rng(14)
    y = rng.random(3000) + 1j * rng.random(3000)
    y[:5] = z[:5]                                              # on a source: that source is left out
    q = rng.standard_normal(z.size)
    zz = np.concatenate([z, y])
    qq = np.concatenate([q, np.zeros(y.size)])
    tree = F.build_tree(dev(zz), 5)
    u = host(F.evaluate_log(F.plan(tree, 30, 0.5, "fp64"), devr(qq)))[z.size:]
    assert e2(u, orc.direct_log_points(z, q, y)) <= 1e-12


def test_log_leaves_the_harmonic_evaluation_unchanged(F):
    z, m, _ = W.uniform(20000, seed=15)
    q = np.random.default_rng(16).standard_normal(z.size)
    tree = F.build_tree(dev(z), 5)
    for prec in ("fp64", "mixed"):
        pl = F.plan(tree, 16, 0.5, prec)
        ref = host(F.evaluate(F.plan(tree, 16, 0.5, prec), dev(m)))
        F.evaluate_log(pl, devr(q))
        np.testing.assert_array_equal(host(F.evaluate(pl, dev(m))), ref)
        F.evaluate_log(pl, devr(q))
        with pytest.raises(F.FmmError):                        # the adjoint needs a harmonic evaluation first
            F.evaluate_adjoint(pl, dev(m), dev(m))


def test_log_rejects_bad_arguments(F):
    import ctypes as C
    z, _, _ = W.uniform(500, seed=1)
    tree = F.build_tree(dev(z), 2)
    pl = F.plan(tree, 8, 0.5)
    q = devr(np.ones(z.size))
    assert F.lib().fmm_evaluate_log(pl._h, None, C.c_void_p(q.data_ptr()), None) == -1
    with pytest.raises(F.FmmError):
        F.evaluate_log(F.plan(tree, 8, 0.5, smooth_delta=0.01), q)
    with pytest.raises(TypeError):
        F.evaluate_log(pl, dev(np.ones(z.size)))               # complex strengths
