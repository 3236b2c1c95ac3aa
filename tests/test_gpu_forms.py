"""The batched / graph-replayed form and the time-stepping driver with the
tuner, through the C ABI.  Graph replays are checked against eager
evaluations after every replay, with eager work in between."""
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


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_graph_replays_match_eager(F, prec):
    import torch
    zs, ms, _ = W.batch(nprob=24, seed=3, nmin=1000, nmax=20000)
    from paper_1311_1006_amd.driver import default_levels
    Ls = [default_levels(len(z)) for z in zs]
    off = np.concatenate([[0], np.cumsum([len(z) for z in zs])]).tolist()
    zc = np.concatenate(zs)
    tree = F.build_tree(dev(zc), Ls, offsets=off)
    pg = F.plan(tree, 16, 0.5, prec, graph=True)
    pe = F.plan(tree, 16, 0.5, prec)
    m_buf = dev(np.concatenate(ms))
    out = torch.empty_like(m_buf)
    rng = np.random.default_rng(4)
    for it in range(4):
        mv = rng.standard_normal(zc.size) + 1j * rng.standard_normal(zc.size)
        m_buf.copy_(dev(mv))
        F.evaluate(pg, m_buf, out)              # first call captures, later calls replay
        ref = F.evaluate(pe, m_buf)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(host(out), host(ref))
        _ = (m_buf * 2).sum().item()            # eager work between replays


def test_batch_of_many_problems_matches_single_problems(F, orc):
    zs, ms, kinds = W.batch(nprob=40, seed=5, nmin=1000, nmax=30000)
    from paper_1311_1006_amd.driver import default_levels
    Ls = [default_levels(len(z)) for z in zs]
    off = np.concatenate([[0], np.cumsum([len(z) for z in zs])]).tolist()
    tree = F.build_tree(dev(np.concatenate(zs)), Ls, offsets=off)
    pl = F.plan(tree, 16, 0.5, "mixed", graph=True)
    phi = host(F.evaluate(pl, dev(np.concatenate(ms))))
    for b in (0, 7, 21, 39):
        # problems of different depths run the far field level by level: a
        # single problem run the same way gives the same bits; run by subtrees
        # (the default for one problem) it differs by rounding only
        tb = F.build_tree(dev(zs[b]), Ls[b])
        one = host(F.evaluate(F.plan(tb, 16, 0.5, "mixed", levelwise=True), dev(ms[b])))
        np.testing.assert_array_equal(phi[off[b]:off[b + 1]], one)
        assert e2(host(F.evaluate(F.plan(tb, 16, 0.5, "mixed"), dev(ms[b]))), one) <= 1e-6
        sub = W.subsample(len(zs[b]), 2000, seed=b)
        ref = orc.direct(zs[b], ms[b], sub)
        assert e2(one[sub], ref) <= 1e-6 and einf(one[sub], ref) <= 1e-6


def test_tuned_batch_matches_single_problems(F, orc):
    # the batch autotuner (level offset, P2P split, M2L slots) and its best
    # configuration: every problem equals its own evaluation with the same
    # levels and knobs, and stays within the mixed bar of the direct sum
    from paper_1311_1006_amd.driver import batch_levels, tune_batch
    zs, ms, _ = W.batch(nprob=16, seed=9, nmin=1000, nmax=20000)
    sizes = [len(z) for z in zs]
    off = np.concatenate([[0], np.cumsum(sizes)]).tolist()
    zc, mc = dev(np.concatenate(zs)), dev(np.concatenate(ms))
    best, hist = tune_batch(zc, mc, off, 16, 0.5, "mixed", iterations=16)
    assert len(hist) == 16 and all(sec > 0 for _, sec in hist)
    assert -2 <= best["level_offset"] <= 2
    assert best["levels"] == batch_levels(sizes, best["level_offset"])
    knobs = dict(p2p_split=best["p2p_split"], m2l_batch=best["m2l_batch"])
    tree = F.build_tree(zc, best["levels"], offsets=off)
    phi = host(F.evaluate(F.plan(tree, 16, 0.5, "mixed", graph=True, **knobs), mc))
    # problems of one depth run the far field by subtrees, else level by level
    levelwise = len(set(best["levels"])) > 1
    for b in (0, 5, 15):
        tb = F.build_tree(dev(zs[b]), best["levels"][b])
        one = host(F.evaluate(F.plan(tb, 16, 0.5, "mixed", levelwise=levelwise, **knobs), dev(ms[b])))
        np.testing.assert_array_equal(phi[off[b]:off[b + 1]], one)
        sub = W.subsample(sizes[b], 1000, seed=b)
        ref = orc.direct(zs[b], ms[b], sub)
        assert e2(one[sub], ref) <= 1e-6 and einf(one[sub], ref) <= 1e-6


def test_timestepping_with_tuner(F, orc):
    # a smaller copy of the clustered, dynamically re-tuned workload
    import torch
    from paper_1311_1006_amd.driver import advect, make_tuner
    z, m = W.clustered(100000, seed=0, nclusters=32)
    tu = make_tuner(z.size, cap=0.1, window=2, knob_interval=3)
    errs = {}

    def check(step, zt, phi, prm, sec):
        if step in (0, 7):
            zh = host(zt)
            sub = W.subsample(zh.size, 1000, seed=step)
            ref = orc.direct(zh, m, sub)
            errs[step] = max(e2(host(phi)[sub], ref), einf(host(phi)[sub], ref))

    zf, hist = advect(dev(z), dev(m), 8, 1e-4, p=16, theta=0.5, precision="mixed", tuner=tu, callback=check)
    assert errs[0] <= 1e-6 and errs[7] <= 1e-6
    assert torch.isfinite(zf.real).all() and torch.isfinite(zf.imag).all()
    assert len(hist) == 8 and all(s > 0 for _, s in hist)


def test_choose_order_meets_tolerance_against_direct_sum(F, orc):
    """Measured order selection: the chosen p meets the tolerance against the
    p = 32 FP64 reference, and against the FP64 direct sum (oracle) as well;
    no lower order in the range does; a looser tolerance needs no more."""
    n, L, tol = 40000, 6, 1e-6
    z, m, _ = W.uniform(n, seed=11)
    tree = F.build_tree(dev(z), L)
    md = dev(m)
    p, (e64, emx) = F.choose_order(tree, md, 0.5, tol, p_lo=4, p_hi=24)
    assert 4 < p <= 24 and e64 <= tol and emx <= tol, (p, e64, emx)
    sub = np.arange(0, n, 7)
    ref = orc.direct(z, m, sub)
    for prec in ("fp64", "mixed"):
        out = F.evaluate(F.plan(tree, p, 0.5, prec), md)
        assert e2(host(out)[sub], ref) <= 1.5 * tol, prec
    p_below, _ = F.choose_order(tree, md, 0.5, tol, p_lo=4, p_hi=p - 1)
    assert p_below == -1
    p_loose, _ = F.choose_order(tree, md, 0.5, 1e-3, p_lo=4, p_hi=24)
    assert 4 <= p_loose < p


def test_choose_order_rejects_bad_arguments(F):
    z, m, _ = W.uniform(1000, seed=1)
    tree = F.build_tree(dev(z), 3)
    md = dev(m)
    for args in [(0.5, 1e-6, 0, 10), (0.5, 1e-6, 10, 9), (0.5, 1e-6, 4, 49), (1.0, 1e-6, 4, 10), (0.5, 0.0, 4, 10)]:
        with pytest.raises(F.FmmError):
            F.choose_order(tree, md, *args)


def test_timestepping_with_theta_walk(F, orc):
    """The driver evaluates with the theta and p the tuner hands out (AT3b
    with a theta walk, p from the tolerance by Table 4.1's rule), and every
    such evaluation meets the tolerance against the FP64 direct sum."""
    import torch
    from paper_1311_1006_amd.driver import advect, make_tuner
    z, m = W.clustered(60000, seed=2, nclusters=16)
    tu = make_tuner(z.size, cap=0.1, window=1, knob_interval=5, theta=0.5, theta_interval=1, theta_min=0.40,
                    theta_max=0.60, tol=1e-6)
    seen = []

    def check(step, zt, phi, prm, sec):
        assert prm["p"] == F.p_from_tol(1e-6, prm["theta"])
        if step % 3 == 0:
            zh = host(zt)
            sub = W.subsample(zh.size, 800, seed=step)
            seen.append((prm["theta"], prm["p"], e2(host(phi)[sub], orc.direct(zh, m, sub))))

    zf, hist = advect(dev(z), dev(m), 12, 1e-4, precision="mixed", tuner=tu, callback=check)
    assert all(err <= 1e-6 for _, _, err in seen), seen
    assert len({th for th, _, _ in seen}) >= 2 or len({round(h[0]["theta"], 6) for h in hist}) >= 2
    assert torch.isfinite(zf.real).all() and torch.isfinite(zf.imag).all()
