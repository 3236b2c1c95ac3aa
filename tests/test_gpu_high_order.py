"""Expansion orders above 32 terms (1 <= p <= 64), through the C ABI.

Table 4.1 asks for p = 33 (TOL 1e-8, theta 0.6), p = 34 (1e-7, 0.65) and
p = 39 (1e-8, 0.65).  Above 32 terms P2M runs in two blocks of 32 terms,
L2P holds the local expansions in LDS, and M2L takes three (p <= 48) or
four (p <= 64) 16-row MFMA blocks.  Checks:
  * FP64 FMM vs the oracle's serial FMM at equal (p, theta, N_levels):
    relative 2-norm <= 1e-12, near and far parts separately;
  * FP64 FMM vs the direct sum within Table 4.1's TOL at the table's p;
  * mixed precision within 1e-6 of the direct sum;
  * the derivative field, the logarithmic kernel and the adjoint at p > 32.
"""
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


# (N, N_levels): leaves of about 78 (64 lanes per leaf), 20 (32 lanes) and
# 7 points (16 lanes, where P2M would also form the leaves' parents at p <= 32)
SHAPES = [(20000, 5), (20000, 6), (30000, 7)]


@pytest.mark.parametrize("p,theta", [(33, 0.6), (34, 0.65), (39, 0.65), (48, 0.5), (49, 0.5), (64, 0.5)])
@pytest.mark.parametrize("n,L", SHAPES)
def test_fp64_high_order_matches_oracle_fmm(orc, F, p, theta, n, L):
    z, m, _ = W.uniform(n, seed=n + p)
    pl = F.plan(F.build_tree(dev(z), L), p, theta, "fp64")
    phi = host(F.evaluate(pl, dev(m)))
    ref, rnear, rfar = orc.fmm(z, m, p, theta, L, parts=True)
    assert e2(phi, ref) <= 1e-12
    near, far = F.evaluate_parts(pl, dev(m))
    assert e2(host(near), rnear) <= 1e-12
    assert e2(host(far), rfar) <= 1e-12


@pytest.mark.parametrize("tol,theta,p", [(1e-8, 0.6, 33), (1e-7, 0.65, 34), (1e-8, 0.65, 39)])
def test_fp64_table_4_1_entries_above_32_terms(orc, F, tol, theta, p):
    z, m, _ = W.uniform(20000, seed=31)
    assert F.p_from_tol(tol, theta) == p
    pl = F.plan(F.build_tree(dev(z), 5), p, theta, "fp64")
    assert e2(host(F.evaluate(pl, dev(m))), orc.direct(z, m)) <= tol


@pytest.mark.parametrize("p", [40, 64])
def test_mixed_high_order_within_1e6(orc, F, p):
    z, m, _ = W.uniform(20000, seed=32)
    pl = F.plan(F.build_tree(dev(z), 6), p, 0.5, "mixed")
    phi = host(F.evaluate(pl, dev(m)))
    ref = orc.direct(z, m)
    assert e2(phi, ref) <= 1e-6
    assert einf(phi, ref) <= 1e-6


def test_high_order_field_log_and_adjoint(orc, F):
    import torch
    z, m, _ = W.uniform(6000, seed=33)
    sub = W.subsample(z.size, 1000, seed=2)
    pl = F.plan(F.build_tree(dev(z), 5), 40, 0.5, "fp64")
    phi, dphi = F.evaluate_field(pl, dev(m))
    assert e2(host(phi)[sub], orc.direct(z, m, sub)) <= 1e-12
    assert e2(host(dphi)[sub], orc.direct_deriv_points(z, m, z[sub])) <= 1e-11
    q = np.random.default_rng(5).standard_normal(z.size)
    u = host(F.evaluate_log(pl, torch.from_numpy(q).cuda()))
    assert e2(u[sub], orc.direct_log_points(z, q, z[sub])) <= 1e-12
    phi = F.evaluate(pl, dev(m))
    gm, gz = F.evaluate_adjoint(pl, dev(m), 2 * phi)
    rgm, rgz = orc.grad_direct(z, m, 2 * orc.direct(z, m))
    assert e2(host(gm), rgm) <= 1e-12
    assert e2(host(gz), rgz) <= 1e-11


def test_choose_order_above_32_terms(F):
    # p_hi above 24: the reference evaluation takes p_hi + 16 = 56 terms
    z, m, _ = W.uniform(20000, seed=34)
    tree = F.build_tree(dev(z), 5)
    p, (e64, emx) = F.choose_order(tree, dev(m), 0.65, 1e-5, p_lo=8, p_hi=40)
    assert 8 <= p <= 40 and e64 <= 1e-5 and emx <= 1e-5
