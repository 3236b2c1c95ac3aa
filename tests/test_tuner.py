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


# ---- theta in the walk (Algorithms 1, 2 and 4)

def theta_model(theta, L=8, centres=((0.55, 1.0, 25.0),)):
    """Run time of the fake clock over theta: the deepest of a few quadratic
    basins (centre, depth factor, curvature), times the N_levels model."""
    f = min(d * (1.0 + c * (theta - t0) ** 2) for t0, d, c in centres)
    return model(L) * f


def run_theta(tuner, steps, cost, rng, noise=0.01):
    hist = []
    for i in range(steps):
        p = tuner.next()
        t = cost(i, p) * (1 + noise * rng.random())
        tuner.observe(t)
        hist.append(p)
    return hist


def tail_mode(hist, key, n):
    vals, counts = np.unique(np.round([h[key] for h in hist[-n:]], 6), return_counts=True)
    return vals[np.argmax(counts)]


def test_theta_walks_converge_to_the_optimum():
    for alg in ("at3b", "at2", "at1"):
        rng = np.random.default_rng(3)
        tu = F.Tuner(n_levels=8, min_levels=8, max_levels=8, p2p_split=2, m2l_batch=8, window=3,
                     algorithm=alg, theta=0.40, theta_interval=2, theta_min=0.30, theta_max=0.70, seed=7)
        hist = run_theta(tu, 1500, lambda i, p: theta_model(p["theta"]), rng)
        assert abs(tail_mode(hist, "theta", 400) - 0.55) <= 0.021, alg
        b, _, _ = tu.best()
        assert abs(b["theta"] - 0.55) <= 0.031, (alg, b)


def test_fibonacci_steps_leave_a_local_minimum():
    """Two basins (the paper's uniform case has a local and a global region):
    started in the shallow one, the directed walk with Fibonacci step cycles
    reaches the deep one."""
    basins = ((0.40, 1.0, 60.0), (0.58, 0.8, 60.0))
    rng = np.random.default_rng(4)
    tu = F.Tuner(n_levels=8, min_levels=8, max_levels=8, p2p_split=2, m2l_batch=8, window=3, algorithm="at2",
                 level_interval=10 ** 6, theta=0.40, theta_interval=2, theta_min=0.30, theta_max=0.70,
                 fib_length=4)
    hist = run_theta(tu, 2000, lambda i, p: theta_model(p["theta"], centres=basins), rng)
    assert abs(tail_mode(hist, "theta", 500) - 0.58) <= 0.021
    thetas = np.array([h["theta"] for h in hist])
    steps = np.unique(np.round(np.abs(np.diff(thetas)) / 0.01)).astype(int)
    assert {1, 2, 3}.issubset(set(steps.tolist()))      # step lengths from the Fibonacci cycle


def test_theta_and_levels_tune_independently():
    rng = np.random.default_rng(5)
    best_L = argmin_L(lambda L: model(L))
    tu = F.Tuner(n_levels=6, min_levels=3, max_levels=12, p2p_split=2, m2l_batch=8, window=3, algorithm="at3b",
                 theta=0.35, theta_interval=3, theta_min=0.30, theta_max=0.70)
    hist = run_theta(tu, 2000, lambda i, p: theta_model(p["theta"], L=p["n_levels"]), rng)
    assert tail_mode(hist, "n_levels", 500) == best_L
    assert abs(tail_mode(hist, "theta", 500) - 0.55) <= 0.021


def test_theta_stays_on_its_grid_and_p_follows_theta():
    rng = np.random.default_rng(6)
    # N_levels moves take precedence when due (Algorithm 1), so they are spaced
    # wider than the theta moves
    tu = F.Tuner(n_levels=8, min_levels=7, max_levels=9, p2p_split=2, m2l_batch=8, window=2, algorithm="at1",
                 level_interval=9, theta=0.5, theta_interval=1, theta_min=0.40, theta_max=0.60,
                 tol=1e-6, seed=11)
    hist = run_theta(tu, 500, lambda i, p: model(p["n_levels"]) * (1 + rng.random()), rng)
    for h in hist:
        assert 0.40 - 1e-12 <= h["theta"] <= 0.60 + 1e-12
        k = (h["theta"] - 0.40) / 0.01
        assert abs(k - round(k)) < 1e-9
        assert h["p"] == F.p_from_tol(1e-6, h["theta"])
    assert len({round(h["theta"], 6) for h in hist}) > 5


def test_random_walk_directions_follow_the_seed():
    def seq(seed):
        rng = np.random.default_rng(0)
        tu = F.Tuner(n_levels=8, min_levels=5, max_levels=11, p2p_split=2, m2l_batch=8, window=1, algorithm="at1",
                     level_interval=2, theta=0.5, theta_interval=3, seed=seed)
        return [(h["n_levels"], round(h["theta"], 6)) for h in
                run_theta(tu, 200, lambda i, p: theta_model(p["theta"], L=p["n_levels"]), rng)]
    assert seq(1) == seq(1)
    assert seq(1) != seq(2)


def test_invalid_theta_configuration_is_rejected():
    import pytest
    base = dict(n_levels=8, min_levels=7, max_levels=9, p2p_split=2, m2l_batch=8)
    for bad in [dict(theta_interval=1, theta=0.8), dict(theta_interval=1, theta_unit=0.0),
                dict(theta_interval=1, theta_min=0.6, theta_max=0.5, theta=0.55),
                dict(theta_interval=1, fib_length=1), dict(algorithm="at2", level_interval=0),
                dict(tol=1.5), dict(theta_interval=-1)]:
        with pytest.raises(F.FmmError):
            F.Tuner(**dict(base, **bad))
