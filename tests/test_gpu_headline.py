"""Parity at the benchmark's own shape: N = 1e6 uniform points in the unit
square, complex N(0,1) strengths (seed 0), N_levels = 9 (65,536 leaves of
15-16 points), p = 13, theta = 0.5 -- the configuration whose throughput
the benchmark reports.

This shape reaches code that the smaller parity cases do not: eight global
split stages of the tree build before the in-LDS stage, the FP64
instantiation of P2M / L2P for leaves of at most 16 points and p <= 16 with
the leaves' M2M and L2L folded in, and the M2L of the top levels (0..5) on
its own stream beside the deeper levels.

Checks (through the C ABI):
  * tree: identical ranges and point sets per box, bit-identical geometry
    against the oracle's tree (Sec. 2.2);
  * lists: strong and weak lists identical at every level (Sec. 2.1);
  * FP64 FMM: relative 2-norm error <= 1e-12 against the oracle's serial
    FMM at equal (p, theta, N_levels), for the whole result and for the
    near and far parts separately, in every launch shape the benchmark
    may pick (P2P subgroups, M2L pair slots);
  * mixed precision: e2 <= 1e-6 and e_inf <= 1e-6 against the FP64 direct
    sum on a 10,000-target subsample, and within 1e-6 of the FP64 FMM over
    all points.
"""
import numpy as np
import pytest

from paper_1311_1006_amd import workloads as W

from gpu_util import dev, e2, einf, host, same_tree

pytestmark = pytest.mark.gpu

N, L, P, THETA = 1_000_000, 9, 13, 0.5


@pytest.fixture(scope="module")
def F():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_1311_1006_amd as F
    F.lib()
    return F


@pytest.fixture(scope="module")
def work(orc):
    z, m, sub = W.uniform(N, seed=0)
    perm, rng, geom = orc.tree(z, L)
    ref, rnear, rfar = orc.fmm(z, m, P, THETA, L, parts=True)
    return dict(z=z, m=m, sub=sub, geom=geom, ref=ref, rnear=rnear, rfar=rfar)


@pytest.fixture(scope="module")
def tree(F, orc, work):
    print("headline: tree N=%d L=%d" % (N, L), flush=True)
    return same_tree(orc, F, work["z"], L)


def test_headline_lists_match_oracle(F, orc, work, tree):
    lo = orc.lists(work["geom"], L, THETA)
    pl = F.plan(tree, P, THETA, "fp64")
    for l in range(L):
        so, sid, wo, wid = lo[l]
        gso, gsid = pl.download_list(0, l, 0)
        gwo, gwid = pl.download_list(0, l, 1)
        assert np.array_equal(gso, so) and np.array_equal(gsid, sid), "strong list level %d" % l
        assert np.array_equal(gwo, wo) and np.array_equal(gwid, wid), "weak list level %d" % l
    st = pl.stats()
    assert st["n_m2l_pairs"] == sum(int(lo[l][2][-1]) for l in range(L))


@pytest.mark.parametrize("split,batch", [(0, 0), (2, 0), (0, 8), (0, 16)])
def test_headline_fp64_matches_oracle_fmm(F, work, tree, split, batch):
    print("headline: fp64 split=%d batch=%d" % (split, batch), flush=True)
    pl = F.plan(tree, P, THETA, "fp64", p2p_split=split, m2l_batch=batch)
    m = dev(work["m"])
    phi = host(F.evaluate(pl, m))
    assert e2(phi, work["ref"]) <= 1e-12
    near, far = F.evaluate_parts(pl, m)
    assert e2(host(near), work["rnear"]) <= 1e-12
    assert e2(host(far), work["rfar"]) <= 1e-12


def test_headline_mixed_within_1e6(F, orc, work, tree):
    print("headline: mixed", flush=True)
    z, m, sub = work["z"], work["m"], work["sub"]
    pl = F.plan(tree, P, THETA, "mixed")
    phi = host(F.evaluate(pl, dev(m)))
    direct = orc.direct(z, m, sub)
    assert e2(phi[sub], direct) <= 1e-6
    assert einf(phi[sub], direct) <= 1e-6
    # and against the FP64 FMM of the same tree over every point
    assert e2(phi, work["ref"]) <= 1e-6
    assert einf(phi, work["ref"]) <= 1e-6
