"""Parity of the HIP path against the CPU oracle, called through the C ABI.

Tree: same boxes and bit-identical geometry (the split rule and the
geometry are evaluated with individually rounded IEEE operations on both
sides).  Lists: identical.  FP64 FMM: relative 2-norm error <= 1e-12 against
the serial FMM oracle at equal (p, theta, N_levels).  Mixed precision:
<= 1e-6 against the FP64 direct sum.  Edge cases: one level, one point per
leaf, ragged sizes, ties, clustered and line-like inputs, a batch of
problems, the exact-selection fallback for heavy ties.
"""
import numpy as np
import pytest

from paper_1311_1006_amd import workloads as W

from gpu_util import dev, e2, einf, host, same_tree

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_1311_1006_amd as F
    F.lib()
    return F


def _lists_equal(orc, F, pl, geom, L, theta, prob=0):
    lo = orc.lists(geom, L, theta)
    for l in range(L):
        so, sid, wo, wid = lo[l]
        gso, gsid = pl.download_list(prob, l, 0)
        gwo, gwid = pl.download_list(prob, l, 1)
        assert np.array_equal(gso, so) and np.array_equal(gsid, sid), "strong list level %d" % l
        assert np.array_equal(gwo, wo) and np.array_equal(gwid, wid), "weak list level %d" % l


@pytest.mark.parametrize("n,L", [(10000, 5), (10007, 4), (16, 3), (1, 1), (777, 1), (50000, 6), (200000, 7)])
def test_tree_and_lists_match_oracle(orc, F, n, L):
    z, m, _ = W.uniform(n, seed=n)
    tree = same_tree(orc, F, z, L)
    pl = F.plan(tree, 12, 0.5)
    _lists_equal(orc, F, pl, orc.tree(z, L)[2], L, 0.5)


@pytest.mark.parametrize("kind", ["clustered", "line", "ties"])
def test_tree_nonuniform(orc, F, kind):
    n, L = 30000, 6
    if kind == "clustered":
        z, _ = W.clustered(n, seed=1, nclusters=8)
    elif kind == "line":
        z, _ = W.line_like(n, seed=1)
    else:
        rng = np.random.default_rng(2)
        z = np.round(rng.random(n) * 64) / 64 + 1j * np.round(rng.random(n) * 64) / 64
    tree = same_tree(orc, F, z, L)
    pl = F.plan(tree, 10, 0.5)
    _lists_equal(orc, F, pl, orc.tree(z, L)[2], L, 0.5)


def test_clustered_long_lists_match_oracle(orc, F):
    # four tight clusters: strong lists of up to ~2000 boxes one level above
    # the leaves and ~8000 at the leaves (longer than a wavefront's LDS
    # frontier, and too long for fixed per-box pools)
    z, m = W.clustered(100000, seed=3, nclusters=4, sigma=1e-5)
    L = 8
    tree = same_tree(orc, F, z, L)
    geom = orc.tree(z, L)[2]
    for _ in range(2):   # the first plan learns the layout, the second uses it
        pl = F.plan(tree, 12, 0.5, "fp64")
        _lists_equal(orc, F, pl, geom, L, 0.5)
    # the longest leaf lists are cut into several work chunks (chunks of
    # 2048 / (points per leaf + 1) entries)
    off, _ = pl.download_list(0, L - 1, 0)
    npl = 100000 // 4 ** (L - 1)
    assert np.diff(off).max() > 4 * (2048 // (npl + 2))
    phi = host(F.evaluate(pl, dev(m)))
    assert e2(phi, orc.fmm(z, m, 12, 0.5, L)) <= 1e-12
    # a fresh plan evaluated at once: the upward pass is enqueued before the
    # plan's list and work-chunk kernels, and the near field must wait for them
    for prec in ("fp64", "mixed"):
        ref = host(F.evaluate(F.plan(tree, 12, 0.5, prec), dev(m)))
        for _ in range(3):
            assert np.array_equal(host(F.evaluate(F.plan(tree, 12, 0.5, prec), dev(m))), ref)


def test_far_point_long_lists_match_oracle(orc, F):
    # one point far from a uniform cloud: every box that holds it stretches
    # to it and is strong with nearly every box of its level, so parent lists
    # reach about 4^(N_levels - 2) boxes (65536 here): their sibling groups
    # are split over several workgroups of several loop trips each
    z, m, _ = W.uniform(270000, seed=91)
    z[123] = 1000.0 + 1000.0j
    L = 10
    tree = same_tree(orc, F, z, L)
    geom = orc.tree(z, L)[2]
    pl = F.plan(tree, 8, 0.5, "fp64")
    _lists_equal(orc, F, pl, geom, L, 0.5)
    off, _ = pl.download_list(0, L - 2, 0)
    assert np.diff(off).max() > 16384          # a parent list of more than 16 loop trips
    phi = host(F.evaluate(pl, dev(m)))
    assert e2(phi, orc.fmm(z, m, 8, 0.5, L)) <= 1e-12


def test_tree_exact_select_fallback(orc, F):
    # a segment whose median bucket holds > 2048 points with identical
    # coordinates cannot be resolved by bucketing: the exact radix select runs
    rng = np.random.default_rng(3)
    n = 40000
    x = rng.choice([0.25, 0.5, 0.75], n)
    y = rng.random(n) * 0.1
    same_tree(orc, F, x + 1j * y, 5)


def test_tree_many_tied_coordinates(orc, F):
    # 64 distinct x values with 200 points each: every x split meets runs of
    # tied coordinates, ordered by input index
    rng = np.random.default_rng(13)
    x = np.repeat(np.arange(64) / 64.0, 200)
    rng.shuffle(x)
    z = x + 1j * rng.random(x.size)
    same_tree(orc, F, z, 5)


@pytest.mark.parametrize("levelwise", [False, True])
@pytest.mark.parametrize("n,L,p", [(10000, 5, 17), (10007, 4, 12), (50000, 6, 16), (4096, 6, 20), (3000, 3, 9),
                                   (70000, 7, 30)])
def test_fp64_fmm_matches_oracle_fmm(orc, F, n, L, p, levelwise):
    # levelwise False: the far field by subtrees (P2M with two M2M levels,
    # three-level M2M subtrees, L2P shifting every ancestor's M2L sum into the
    # leaves); True: one launch per level of M2M and L2L
    z, m, _ = W.uniform(n, seed=n + 1)
    tree = F.build_tree(dev(z), L)
    pl = F.plan(tree, p, 0.5, "fp64", levelwise=levelwise)
    phi = host(F.evaluate(pl, dev(m)))
    ref, rnear, rfar = orc.fmm(z, m, p, 0.5, L, parts=True)
    assert e2(phi, ref) <= 1e-12
    near, far = F.evaluate_parts(pl, dev(m))
    assert e2(host(near), rnear) <= 1e-12
    assert e2(host(far), rfar) <= 1e-12


@pytest.mark.parametrize("n,L,p", [(20000, 5, 16), (60000, 7, 13), (30000, 6, 28)])
def test_mixed_subtree_matches_levelwise(orc, F, n, L, p):
    # the two forms of the far field in mixed precision: both within 1e-6 of
    # the direct sum, and within 1e-6 of each other (e2 and e_inf)
    z, m, _ = W.uniform(n, seed=n + 2)
    tree = F.build_tree(dev(z), L)
    md = dev(m)
    a = host(F.evaluate(F.plan(tree, p, 0.5, "mixed"), md))
    b = host(F.evaluate(F.plan(tree, p, 0.5, "mixed", levelwise=True), md))
    ref = orc.direct(z, m)
    for phi in (a, b):
        assert e2(phi, ref) <= 1e-6
        assert einf(phi, ref) <= 1e-6
    assert e2(a, b) <= 1e-6 and einf(a, b) <= 1e-6


@pytest.mark.parametrize("batch,p", [(4, 16), (8, 16), (16, 16), (8, 20), (16, 24)])
def test_m2l_batch_shapes_match_oracle(orc, F, batch, p):
    # M2L with one, two or four boxes sharing a wavefront's 16 pair slots
    z, m, _ = W.uniform(30000, seed=14)
    tree = F.build_tree(dev(z), 6)
    pl = F.plan(tree, p, 0.5, "fp64", m2l_batch=batch)
    assert e2(host(F.evaluate(pl, dev(m))), orc.fmm(z, m, p, 0.5, 6)) <= 1e-12
    plm = F.plan(tree, p, 0.5, "mixed", m2l_batch=batch)
    phim, ref = host(F.evaluate(plm, dev(m))), orc.direct(z, m)
    assert e2(phim, ref) <= 1e-6 and einf(phim, ref) <= 1e-6


def test_fp64_fmm_clustered_matches_oracle(orc, F):
    z, m = W.clustered(20000, seed=4, nclusters=8)
    tree = F.build_tree(dev(z), 6)
    pl = F.plan(tree, 16, 0.5, "fp64")
    phi = host(F.evaluate(pl, dev(m)))
    assert e2(phi, orc.fmm(z, m, 16, 0.5, 6)) <= 1e-12


def test_fp64_single_level_is_direct_sum(orc, F):
    z, m, _ = W.uniform(700, seed=5)
    pl = F.plan(F.build_tree(dev(z), 1), 8, 0.5, "fp64")
    assert e2(host(F.evaluate(pl, dev(m))), orc.direct(z, m)) <= 1e-13


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-13), ("mixed", 1e-6)])
def test_split_source_lists_match_direct_sum(orc, F, prec, tol):
    # one leaf of 5000 points: every near-field work item sums over a strong
    # list of one entry with 5000 sources (a list is cut into chunks of whole
    # entries, so this one is not cut)
    z, m, _ = W.uniform(5000, seed=6)
    pl = F.plan(F.build_tree(dev(z), 1), 8, 0.5, prec)
    phi = host(F.evaluate(pl, dev(m)))
    assert e2(phi, orc.direct(z, m)) <= tol
    assert np.array_equal(phi, host(F.evaluate(pl, dev(m))))   # deterministic


def test_fp64_within_table_tolerance_of_direct(orc, F):
    # Table 4.1: p = 17 for TOL = 1e-6 at theta = 0.5
    z, m, _ = W.uniform(10000, seed=0)
    pl = F.plan(F.build_tree(dev(z), 5), 17, 0.5, "fp64")
    assert e2(host(F.evaluate(pl, dev(m))), orc.direct(z, m)) <= 1e-6


@pytest.mark.parametrize("n,L,p", [(10000, 5, 17), (60000, 6, 16), (20000, 7, 16)])
def test_mixed_within_1e6_of_direct(orc, F, n, L, p):
    z, m, _ = W.uniform(n, seed=n + 2)
    pl = F.plan(F.build_tree(dev(z), L), p, 0.5, "mixed")
    phi = host(F.evaluate(pl, dev(m)))
    ref = orc.direct(z, m)
    assert e2(phi, ref) <= 1e-6 and einf(phi, ref) <= 1e-6


def test_coincident_points_are_excluded(orc, F):
    z, m, _ = W.uniform(3000, seed=6)
    z[100:110] = z[5]            # ten duplicates of one position
    for prec, tol in (("fp64", 1e-12), ("mixed", 1e-6)):
        pl = F.plan(F.build_tree(dev(z), 4), 14, 0.5, prec)
        phi = host(F.evaluate(pl, dev(m)))
        assert np.all(np.isfinite(phi))
        ref = orc.fmm(z, m, 14, 0.5, 4)
        assert e2(phi, ref) <= tol and einf(phi, ref) <= tol


def test_batch_equals_single_problems(orc, F):
    zs, ms, _ = W.batch(nprob=6, seed=7, nmin=500, nmax=30000)
    Ls = [max(1, min(6, int(np.log(len(z) / 20) / np.log(4)) + 1)) for z in zs]
    off = np.concatenate([[0], np.cumsum([len(z) for z in zs])]).tolist()
    zc, mc = np.concatenate(zs), np.concatenate(ms)
    tree = F.build_tree(dev(zc), Ls, offsets=off)
    for b in range(len(zs)):
        same_tree(orc, F, zs[b], Ls[b], prob=b, tree=tree)
    pl = F.plan(tree, 16, 0.5, "fp64")
    phi = host(F.evaluate(pl, dev(mc)))
    for b in range(len(zs)):
        # problems of different depths: the far field level by level, as a
        # single problem planned with levelwise=True
        single = F.plan(F.build_tree(dev(zs[b]), Ls[b]), 16, 0.5, "fp64", levelwise=True)
        one = host(F.evaluate(single, dev(ms[b])))
        np.testing.assert_array_equal(phi[off[b]:off[b + 1]], one)
        assert e2(one, orc.fmm(zs[b], ms[b], 16, 0.5, Ls[b])) <= 1e-12


def test_deterministic_bitwise(F):
    z, m, _ = W.uniform(100000, seed=8)
    outs = []
    for prec in ("fp64", "mixed", "fp64", "mixed"):
        pl = F.plan(F.build_tree(dev(z), 7), 16, 0.5, prec)
        outs.append(host(F.evaluate(pl, dev(m))))
    assert np.array_equal(outs[0], outs[2]) and np.array_equal(outs[1], outs[3])


def test_invalid_arguments_raise(F):
    z, m, _ = W.uniform(100, seed=9)
    with pytest.raises(F.FmmError):
        F.build_tree(dev(z), 5)           # 256 leaves > 100 points
    bad = z.copy()
    bad[3] = np.nan
    # neither the build nor the plan waits for the device: the first call
    # that needs the lists reports it, and so does every later call
    pl = F.plan(F.build_tree(dev(bad), 2), 8, 0.5)
    with pytest.raises(F.FmmError):
        F.evaluate(pl, dev(m))
    with pytest.raises(F.FmmError):
        pl.stats()
    with pytest.raises(F.FmmError):
        F.build_tree(dev(bad), 2).download(0)
    tree = F.build_tree(dev(z), 2)
    for p, th in ((0, 0.5), (65, 0.5), (10, 0.0), (10, 1.0)):
        with pytest.raises(F.FmmError):
            F.plan(tree, p, th)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_near_field_launch_shapes(orc, F, prec):
    # every near-field launch shape (targets per lane x lane subgroups) and
    # staging tile sums what the default shape sums: bit for bit across tiles
    # (each lane meets its sources in the same order), to rounding across
    # shapes (the lane reductions differ)
    z, m, _ = W.uniform(60000, seed=81)
    tree = F.build_tree(dev(z), 7)
    md = dev(m)
    ref = host(F.evaluate(F.plan(tree, 12, 0.5, prec), md))
    assert e2(ref, orc.fmm(z, m, 12, 0.5, 7)) <= (1e-12 if prec == "fp64" else 1e-6)
    for tile in (64, 128, 256):
        assert np.array_equal(host(F.evaluate(F.plan(tree, 12, 0.5, prec, p2p_src_tile=tile), md)), ref), tile
    tol = 1e-14 if prec == "fp64" else 1e-6
    shapes = [(1, 4), (2, 4), (4, 4), (2, 2), (4, 2), (8, 2), (4, 1), (8, 1), (8, 0)]
    if prec == "mixed":
        shapes += [(16, 2), (16, 1), (16, 0)]
    for tg, split in shapes:
        phi = host(F.evaluate(F.plan(tree, 12, 0.5, prec, p2p_targets=tg, p2p_split=split, p2p_src_tile=128), md))
        assert e2(phi, ref) <= tol, (tg, split)
    for bad in (dict(p2p_targets=8, p2p_split=4), dict(p2p_targets=1, p2p_split=2), dict(p2p_targets=3),
                dict(p2p_src_tile=100)):
        with pytest.raises(F.FmmError) as ex:
            F.plan(tree, 12, 0.5, prec, **bad)
        assert ex.value.code == -1, bad
    if prec == "fp64":
        with pytest.raises(F.FmmError):
            F.plan(tree, 12, 0.5, prec, p2p_targets=16)
