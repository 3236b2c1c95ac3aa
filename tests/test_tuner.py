"""Behaviour of the AT3b-style autotuner (Sec. 4.2, Algorithm 4) against a
fake clock: the cost model of Sec. 2.3 (P2P ~ N^2/N_f, M2L ~ N_f) with
multiplicative noise.  The tuner's decisions are timing dependent, so these
tests check behaviour, not a reference value (parity unpinned)."""
import numpy as np

import paper_1311_1006_amd as F


def model(L, a=1.0, b=1.0, n=1e6):
    nf = 4.0 ** (L - 1)
    return a * 2e-9 * nf * 60 + b * 1e-11 * n * n / nf


def run(tuner, steps, cost, rng, noise=0.02):
    hist = []
    for i in range(steps):
        p = tuner.next()
        t = cost(i, p) * (1 + noise * rng.random())
        tuner.observe(t)
        hist.append((p["n_levels"], t))
    return hist


def argmin_L(cost_at, lo=3, hi=12):
    return min(range(lo, hi + 1), key=cost_at)


def test_converges_to_the_optimum_and_respects_the_cap():
    rng = np.random.default_rng(0)
    best = argmin_L(lambda L: model(L))
    tu = F.Tuner(n_levels=5, min_levels=3, max_levels=12, p2p_split=2, m2l_batch=8, cap=0.1, window=3)
    hist = run(tu, 600, lambda i, p: model(p["n_levels"]), rng)
    Ls = np.array([h[0] for h in hist])
    # the optimum is where the tuner spends most of its time; it keeps probing
    # the neighbours only as often as the cost cap allows
    vals, counts = np.unique(Ls[-300:], return_counts=True)
    assert vals[np.argmax(counts)] == best
    b, cost, run_s = tu.best()
    assert b["n_levels"] == best
    tail = hist[200:]
    t_opt = model(best)
    extra = sum(max(0.0, t - 1.02 * t_opt) for _, t in tail)
    total = sum(t for _, t in tail)
    # Algorithm 4 keeps the cost of each direction (up, down) below cap * run time
    assert extra <= 2 * 0.1 * total * 1.1


def test_follows_a_drifting_optimum():
    rng = np.random.default_rng(1)

    def cost(i, p):
        b = 1.0 if i < 300 else 16.0       # the near field becomes 16x more expensive
        return model(p["n_levels"], b=b)

    best0 = argmin_L(lambda L: model(L, b=1.0))
    best1 = argmin_L(lambda L: model(L, b=16.0))
    assert best1 == best0 + 1
    tu = F.Tuner(n_levels=best0, min_levels=3, max_levels=12, cap=0.1, window=3)
    hist = run(tu, 900, cost, rng)
    Ls = np.array([h[0] for h in hist])
    for lo, hi, b in ((150, 300, best0), (700, 900, best1)):
        vals, counts = np.unique(Ls[lo:hi], return_counts=True)
        assert vals[np.argmax(counts)] == b


def test_knob_moves_are_accepted_only_when_faster():
    rng = np.random.default_rng(2)
    pref = {1: 1.3, 2: 1.0, 4: 1.2}

    def cost(i, p):
        return model(p["n_levels"]) * pref[p["p2p_split"]] * (1.0 if p["m2l_batch"] == 8 else 1.1)

    tu = F.Tuner(n_levels=8, min_levels=8, max_levels=8, p2p_split=4, m2l_batch=16, cap=0.1, window=3,
                 knob_interval=4)
    hist = run(tu, 400, cost, rng, noise=0.01)
    b, _, _ = tu.best()
    assert b["p2p_split"] == 2 and b["m2l_batch"] == 8


def test_invalid_configuration_is_rejected():
    import pytest
    with pytest.raises(F.FmmError):
        F.Tuner(n_levels=2, min_levels=3, max_levels=12)
    with pytest.raises(F.FmmError):
        F.Tuner(n_levels=5, min_levels=3, max_levels=12, p2p_split=3)
