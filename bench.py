"""Benchmark: full FMM evaluation at N = 1e6, mixed precision vs plain FP64.

One step = fmm_build_tree + fmm_plan + fmm_evaluate on device-resident
positions and strengths (the tree is rebuilt every call, as in a
time-stepping code).  Workload: 1,000,000 points uniform in the unit square,
complex N(0,1) strengths (seed 0), theta = 0.5; p is chosen for the 1e-6
error target (fmm_choose_order: the smallest p whose FP64 and mixed results
agree with an FP64 evaluation at p = 32 to half the target, relative 2-norm
over all points); N_levels is chosen by a timing sweep.
The accuracy of both paths is measured against the FP64 direct sum (CPU
oracle) on a 10,000-target subsample.

Prints ONE JSON line (stdout).  Progress goes to stderr.
    python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_VALU = 157.3      # TFLOP/s, MI355X published FP32 vector peak (packed)
PEAK_FP32_NOPACK = 78.6     # TFLOP/s, the same units issuing one FP32 op per lane per cycle
PEAK_FP32_MFMA = 157.3      # TFLOP/s, MI355X published dense FP32 matrix peak
P2P_FLOP_PER_PAIR = 16      # per (target, source) pair: see the near-field kernel's header
M2L_AUTO_SLOTS_MIXED = 4    # M2L pair slots per box chosen automatically for mixed precision
ERR_TARGET = 1e-6           # relative error target of both forms against the FP64 direct sum
PEAK_HBM_GBS = 8000.0       # GB/s, MI355X published HBM3E bandwidth
# tree build: per point and binary split, the 8-byte split coordinate read for
# the median selection plus the 20-byte payload (x, y, index) read and written
# by the partition, and 4 bytes of bookkeeping
TREE_BYTES_PER_POINT_SPLIT = 52


def m2l_flop_per_pair(p):
    # a p x p real matrix times p complex coefficients: 2 p^2 real multiply-adds
    return 4 * p * p


def profile_traffic(name):
    """HBM bytes per launch of a kernel from a committed rocprofv3 counter
    summary (FETCH_SIZE + WRITE_SIZE, scaled by a plain copy of known size),
    or None when a source it names changed after the counters were taken."""
    import hashlib
    try:
        text = open(os.path.join(ROOT, "profiles", name)).read()
    except OSError:
        return None
    fields = {}
    for line in text.splitlines():
        if ":" in line and not line.lstrip().startswith("#"):
            k, v = line.split(":", 1)
            fields[k.strip()] = v.strip()
    try:
        h = hashlib.sha256()
        for src in fields["kernel_sources"].split():
            with open(os.path.join(ROOT, "paper_1311_1006_amd", "csrc", src), "rb") as f:
                h.update(f.read())
        if h.hexdigest() != fields["kernel_sources_sha256"]:
            return None
        return float(fields["traffic_bytes_per_launch"])
    except (KeyError, OSError, ValueError):
        return None


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def _time(fn, reps, torch):
    fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps


def measure_theta(F, W, torch, dev, reps, tol=1e-6, n_levels=9):
    """Static theta sweep (Sec. 4.1): N = 1e6 uniform and line-like points,
    mixed precision, p from tol and theta by Table 4.1's rule, a fixed tree
    (N_levels 9); time of plan + evaluate per theta in [0.35, 0.65]."""
    out = {}
    thetas = [round(0.35 + 0.01 * k, 2) for k in range(31)]
    z_u, m_u, _ = W.uniform(1_000_000, seed=0)
    for name, (z, m) in (("uniform", (z_u, m_u)), ("line", W.line_like(1_000_000, seed=0))):
        zd = torch.from_numpy(z).to(dev)
        md = torch.from_numpy(m).to(dev)
        ob = torch.empty_like(md)
        tree = F.build_tree(zd, n_levels)
        res = {}
        for th in thetas:
            p = F.p_from_tol(tol, th)
            t = _time(lambda: F.evaluate(F.plan(tree, p, th, "mixed"), md, ob), reps, torch)
            res["%.2f" % th] = {"p": p, "ms": t * 1e3}
        best = min(res, key=lambda k: res[k]["ms"])
        out["theta_sweep_" + name] = {"n_levels": n_levels, "tol": tol, "rule": "p = fmm_p_from_tol(tol, theta)",
                                      "ms_by_theta": res, "best_theta": float(best), "best_ms": res[best]["ms"],
                                      "ms_at_0.50": res["0.50"]["ms"]}
        log("theta sweep (%s): best theta %s (p=%d) %.3f ms; theta 0.50 (p=%d) %.3f ms" %
            (name, best, res[best]["p"], res[best]["ms"], res["0.50"]["p"], res["0.50"]["ms"]))
        del tree
    return out


def measure_timestepping(F, W, torch, dev, with_errors, steps=50, dt=1e-4, tune_theta=False):
    """Clustered N = 1e6 (90% in 32 Gaussian clusters, sigma = 1e-3, strengths
    +-1): `steps` explicit Euler steps z += dt conj(phi)/(2 pi i), tree rebuilt
    and the tuner consulted every step (mixed precision, p = 16, theta = 0.5;
    with tune_theta the AT3b walk also moves theta, p following it by Table
    4.1's rule for 1e-6).  Reports per-step device time and, every 10 steps,
    e2 against the FP64 direct sum on a 10,000-target subsample (CPU oracle)."""
    from paper_1311_1006_amd.driver import advect, make_tuner
    z, m = W.clustered(1_000_000, seed=0)
    if tune_theta:
        tu = make_tuner(z.size, cap=0.1, window=3, knob_interval=6, theta=0.5, theta_interval=4,
                        theta_min=0.35, theta_max=0.65, tol=1e-6)
    else:
        tu = make_tuner(z.size, cap=0.1, window=3, knob_interval=6)
    errs = {}

    def check(step, zt, phi, prm, sec):
        if with_errors and step % 10 == 0:
            import oracle
            zh = zt.cpu().numpy()
            sub = W.subsample(zh.size, 10000, seed=step)
            errs[step] = oracle.rel_err2(phi.cpu().numpy()[sub], oracle.direct(zh, m, sub))

    md = torch.from_numpy(m).to(dev)
    zf, hist = advect(torch.from_numpy(z).to(dev), md, steps + 1, dt, p=16, theta=0.5, precision="mixed",
                      tuner=tu, callback=check)
    times = [sec for _, sec in hist]
    best = tu.best()[0]
    key = "timestep_clustered_n1e6" + ("_theta_tuned" if tune_theta else "")
    res = {key: {"steps": steps + 1, "ms_per_step_mean": 1e3 * float(np.mean(times)),
                                       "ms_per_step_median": 1e3 * float(np.median(times)),
                                       "mpoints_s_median": 1e6 / float(np.median(times)) / 1e6,
                                       "tuned": best, "e2_every_10_steps": errs or None}}
    log("time stepping clustered N=1e6%s: median %.3f ms/step, tuned %s, e2 %s" %
        (" (theta walked)" if tune_theta else "", 1e3 * float(np.median(times)), best, errs))
    return res


def measure_clustered_breakdown(F, W, torch, dev, steps=30, dt=1e-4):
    """Where the time of a clustered step goes: the clustered N = 1e6 set
    advanced `steps` Euler steps with the tuner (as in the time-stepping
    form), then the late positions and the start positions evaluated at the
    tuner's best knobs and N_levels best - 1 .. best + 1: tree, plan (list
    build; the call waits for the list totals), evaluate, and the phases of a
    phase-timing plan; the list sizes; the spread of the leaf radii."""
    from paper_1311_1006_amd.driver import advect, make_tuner
    z, m = W.clustered(1_000_000, seed=0)
    zd = torch.from_numpy(z).to(dev)
    md = torch.from_numpy(m).to(dev)
    tu = make_tuner(z.size, cap=0.1, window=3, knob_interval=6)
    zf, hist = advect(zd, md, steps, dt, p=16, theta=0.5, precision="mixed", tuner=tu)
    prm = tu.best()[0]
    knobs = dict(p2p_split=prm["p2p_split"], m2l_batch=prm["m2l_batch"])
    out = torch.empty_like(md)

    def ev(fn):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        r = fn()
        e1.record()
        e1.synchronize()
        return r, e0.elapsed_time(e1) * 1e3

    res = {"steps": steps, "tuned": prm, "step_ms": [round(sec * 1e3, 3) for _, sec in hist]}
    for label, zz in (("late", zf), ("start", zd)):
        for L in (prm["n_levels"] - 1, prm["n_levels"], prm["n_levels"] + 1):
            for _ in range(2):
                F.evaluate(F.plan(F.build_tree(zz, L), 16, 0.5, "mixed", **knobs), md, out)
            # the whole step first, while no other tree or plan is alive (as in
            # the time-stepping loop), then its parts one at a time
            _, t_step = ev(lambda: F.evaluate(F.plan(F.build_tree(zz, L), 16, 0.5, "mixed", **knobs), md, out))
            tr, t_tree = ev(lambda: F.build_tree(zz, L))
            pl, t_plan = ev(lambda: F.plan(tr, 16, 0.5, "mixed", **knobs))
            st = pl.stats()
            _, t_eval = ev(lambda: F.evaluate(pl, md, out))
            pt = F.plan(tr, 16, 0.5, "mixed", timing=True, **knobs)
            for _ in range(2):
                F.evaluate(pt, md, out)
            torch.cuda.synchronize()
            sp = pt.stats()
            geom = tr.download(0)[2]
            r = geom[-(4 ** (L - 1)):, 6]
            rec = {"step_us": t_step, "tree_us": t_tree, "plan_us": t_plan, "evaluate_us": t_eval,
                   "phases_us": {k: sp["t_" + k + "_us"] for k in ("upward", "m2l", "l2l", "p2p", "downward")},
                   "n_p2p_pairs": st["n_p2p_pairs"], "n_m2l_pairs": st["n_m2l_pairs"],
                   "p2p_pairs_per_s": st["n_p2p_pairs"] / (sp["t_p2p_us"] * 1e-6),
                   "leaf_radius_quantiles_50_90_99_max": [float(v) for v in np.quantile(r, [0.5, 0.9, 0.99, 1.0])]}
            res["%s_L%d" % (label, L)] = rec
            log("clustered %s step, N_levels %d: %.0f us = tree %.0f + plan %.0f + evaluate %.0f (P2P %.0f, M2L %.0f), "
                "%.3g P2P pairs, median leaf radius %.2e" % (label, L, t_step, t_tree, t_plan, t_eval, sp["t_p2p_us"],
                                                            sp["t_m2l_us"], st["n_p2p_pairs"], rec["leaf_radius_quantiles_50_90_99_max"][0]))
            del pl, pt, tr
    return {"timestep_clustered_breakdown": res}


def measure_kh_tuners(F, W, torch, dev, steps=300, dt=1e-4, tol=1e-6):
    """Table 5.1's comparison (Sec. 5.1): the vortex sheet (Kelvin-Helmholtz
    start, Gaussian smoother, mixed precision) run from the same start with
    no tuning, AT1, AT2 and AT3b (AT3a balances CPU and GPU work and has no
    counterpart on one GPU), for a small (N = 16,000) and a large (N = 1.5e6)
    problem.  The large run starts one level below the level a short sweep
    finds fastest (the paper starts it one below optimal), the small one at
    that level.  The tuners walk N_levels and theta, p following theta by
    Table 4.1's rule for tol (the untuned run keeps theta = 0.5 and that p);
    AT3b also walks the launch-shape knobs.  Reports the total device time of
    the run, its speedup over the untuned run and the N_levels/theta traces."""
    from paper_1311_1006_amd.driver import advect, default_levels
    out = {}
    p0 = F.p_from_tol(tol, 0.5)
    for name, n, below in (("small_n16000", 16000, 0), ("large_n1p5e6", 1_500_000, 1)):
        z, m, sp = W.kelvin_helmholtz(n, seed=0)
        delta = sp / 2
        zd = torch.from_numpy(z).to(dev)
        md = torch.from_numpy(m).to(dev)
        ob = torch.empty_like(md)
        Ld = default_levels(z.size)
        sweep = {}
        for L in range(max(1, Ld - 1), min(Ld + 1, default_levels(z.size, per_leaf=1)) + 1):
            sweep[L] = _time(lambda: F.evaluate(F.plan(F.build_tree(zd, L), p0, 0.5, "mixed", smooth_delta=delta),
                                                md, ob), 5, torch)
        Lbest = min(sweep, key=sweep.get)
        L0 = max(1, Lbest - below)
        runs = {}
        for scheme in ("none", "at1", "at2", "at3b"):
            tu = None
            if scheme != "none":
                tu = F.Tuner(n_levels=L0, min_levels=max(1, L0 - 3), max_levels=default_levels(z.size, per_leaf=1),
                             p2p_split=4, m2l_batch=4, algorithm=scheme, cap=0.1, window=3, knob_interval=6,
                             level_interval=6, theta=0.5, theta_interval=4, theta_min=0.35, theta_max=0.65,
                             tol=tol, seed=1)
            zf, hist = advect(zd, md, steps, dt, p=p0, theta=0.5, precision="mixed", tuner=tu, n_levels=L0,
                              smooth_delta=delta)
            times = [sec for _, sec in hist]
            runs[scheme] = {"total_ms": 1e3 * float(np.sum(times)), "median_step_ms": 1e3 * float(np.median(times)),
                            "median_step_ms_second_half": 1e3 * float(np.median(times[len(times) // 2:])),
                            "levels": [int(h["n_levels"]) for h, _ in hist],
                            "theta": [round(float(h.get("theta", 0.5)), 2) for h, _ in hist]}
            del zf
        for r in runs.values():
            r["speedup_vs_none"] = runs["none"]["total_ms"] / r["total_ms"]
        out["kh_tuner_comparison_" + name] = {"n": int(z.size), "steps": steps, "tol": tol,
                                              "sweep_ms": {str(k): v * 1e3 for k, v in sweep.items()},
                                              "start_levels": L0, "runs": runs}
        log("KH tuner comparison %s (start N_levels %d): %s" % (name, L0, ", ".join(
            "%s %.1f ms (x%.2f)" % (k, r["total_ms"], r["speedup_vs_none"]) for k, r in runs.items())))
    return out


def measure_kh(F, W, torch, dev, reps, with_errors, steps=20, dt=1e-4):
    """The vortex sheet of Sec. 5.1 (Kelvin-Helmholtz start, about 1.5e6
    vortices, Gaussian smoother with delta = half the grid spacing): Euler
    steps with the tuner (mixed, p = 16); e2 every 10 steps against the
    oracle's smoothed direct sum on 2,000 targets; and the cost of the
    smoother: the first tree evaluated with and without it."""
    from paper_1311_1006_amd.driver import advect, default_levels, make_tuner
    z, m, sp = W.kelvin_helmholtz(1_500_000, seed=0)
    delta = sp / 2
    zd = torch.from_numpy(z).to(dev)
    md = torch.from_numpy(m).to(dev)
    tree = F.build_tree(zd, default_levels(z.size))
    ob = torch.empty_like(md)
    t_s = _time(lambda: F.evaluate(F.plan(tree, 16, 0.5, "mixed", smooth_delta=delta), md, ob), reps, torch)
    t_p = _time(lambda: F.evaluate(F.plan(tree, 16, 0.5, "mixed"), md, ob), reps, torch)
    del tree
    tu = make_tuner(z.size, cap=0.1, window=3, knob_interval=6)
    errs = {}

    def check(step, zt, phi, prm, sec):
        if with_errors and step % 10 == 0:
            import oracle
            zh = zt.cpu().numpy()
            sub = W.subsample(zh.size, 2000, seed=step)
            errs[step] = oracle.rel_err2(phi.cpu().numpy()[sub], oracle.direct_smoothed(zh, m, delta, targets=sub))

    zf, hist = advect(zd, md, steps + 1, dt, p=16, precision="mixed", tuner=tu, callback=check, smooth_delta=delta)
    times = [sec for _, sec in hist]
    res = {"kelvin_helmholtz_n1p5e6": {"n": int(z.size), "delta": delta, "steps": steps + 1,
                                       "ms_per_step_median": 1e3 * float(np.median(times)),
                                       "plan_eval_ms_smoothed": t_s * 1e3, "plan_eval_ms_plain": t_p * 1e3,
                                       "tuned": tu.best()[0], "e2_every_10_steps": errs or None}}
    log("Kelvin-Helmholtz N=%d: median %.3f ms/step; plan+evaluate smoothed %.3f ms, plain %.3f ms; e2 %s" %
        (z.size, 1e3 * float(np.median(times)), t_s * 1e3, t_p * 1e3, errs))
    return res


def measure_forms(F, W, torch, dev, reps, with_errors):
    """(2) 128 problems of uneven size in one graph launch vs 128 sequential
    plain launches (same trees, levels, p, shapes); clustered time stepping
    with the tuner; (3) adjoint / forward time at N = 2e5, p = 16."""
    from paper_1311_1006_amd.driver import batch_levels, default_levels, tune_batch
    out = {}
    zs, ms, kinds = W.batch(nprob=128, seed=0)
    sizes = [len(z) for z in zs]
    Ls = batch_levels(sizes)
    off = [0]
    for z in zs:
        off.append(off[-1] + len(z))
    zc = torch.from_numpy(np.concatenate(zs)).to(dev)
    mc = torch.from_numpy(np.concatenate(ms)).to(dev)
    oc = torch.empty_like(mc)
    for prec in ("mixed", "fp64"):
        tree = F.build_tree(zc, Ls, offsets=off)
        pg = F.plan(tree, 16, 0.5, prec, graph=True)
        tb = _time(lambda: F.evaluate(pg, mc, oc), reps, torch)
        singles = []
        for b in range(len(zs)):
            zb = zc[off[b]:off[b + 1]]
            tr = F.build_tree(zb, Ls[b])
            singles.append((tr, F.plan(tr, 16, 0.5, prec), mc[off[b]:off[b + 1]], oc[off[b]:off[b + 1]]))
        ts = _time(lambda: [F.evaluate(pl, mb, ob) for _, pl, mb, ob in singles], max(2, reps // 4), torch)
        del singles, pg, tree
        # the same batch autotuned (AT3b over a common level offset and the
        # launch-shape knobs), then its best configuration timed like the default
        t0 = time.perf_counter()
        best, hist = tune_batch(zc, mc, off, 16, 0.5, prec, iterations=60, out=oc)
        t_tune = time.perf_counter() - t0
        tt = F.build_tree(zc, best["levels"], offsets=off)
        pt = F.plan(tt, 16, 0.5, prec, p2p_split=best["p2p_split"], m2l_batch=best["m2l_batch"], graph=True)
        tg = _time(lambda: F.evaluate(pt, mc, oc), reps, torch)
        del pt, tt
        out["batch128_" + prec] = {
            "n_total": off[-1], "graph_ms": tb * 1e3, "sequential_ms": ts * 1e3, "speedup": ts / tb,
            "mpoints_s": off[-1] / tb / 1e6,
            "default": {"levels": "about 16 points per leaf", "p2p_split": 0, "m2l_batch": 0},
            "tuned_graph_ms": tg * 1e3, "tuned_mpoints_s": off[-1] / tg / 1e6, "tuned_vs_default": tb / tg,
            "tuned": {"level_offset": best["level_offset"], "p2p_split": best["p2p_split"],
                      "m2l_batch": best["m2l_batch"]},
            "tuning": {"iterations": len(hist), "wall_s": t_tune,
                       "trace": [[h["level_offset"], h["p2p_split"], h["m2l_batch"], round(sec * 1e3, 4)]
                                 for h, sec in hist]}}
        log("batch of 128 (%s): graph %.3f ms (default), %.3f ms (autotuned: level offset %+d, split %d, "
            "batch %d), 128 sequential launches %.3f ms" % (prec, tb * 1e3, tg * 1e3, best["level_offset"],
                                                           best["p2p_split"], best["m2l_batch"], ts * 1e3))
    out.update(measure_timestepping(F, W, torch, dev, with_errors))
    out.update(measure_timestepping(F, W, torch, dev, with_errors, tune_theta=True))
    out.update(measure_theta(F, W, torch, dev, max(3, reps // 4)))
    out.update(measure_kh(F, W, torch, dev, max(3, reps // 4), with_errors))
    out.update(measure_kh_tuners(F, W, torch, dev))
    out.update(measure_clustered_breakdown(F, W, torch, dev))
    # field and its derivative (fmm_evaluate_field) against the plain evaluation
    z, m, _ = W.uniform(1_000_000, seed=0)
    zd = torch.from_numpy(z).to(dev)
    md = torch.from_numpy(m).to(dev)
    tree = F.build_tree(zd, 9)
    for prec in ("mixed", "fp64"):
        pl = F.plan(tree, 13, 0.5, prec)
        phi, dphi = torch.empty_like(md), torch.empty_like(md)
        te = _time(lambda: F.evaluate(pl, md, phi), reps, torch)
        tf = _time(lambda: F.evaluate_field(pl, md, phi, dphi), reps, torch)
        out["field_n1e6_" + prec] = {"p": 13, "n_levels": 9, "evaluate_ms": te * 1e3, "field_ms": tf * 1e3,
                                     "ratio": tf / te}
        log("field N=1e6 (%s, p=13): evaluate %.3f ms, evaluate_field %.3f ms" % (prec, te * 1e3, tf * 1e3))
    # the logarithmic potential (fmm_evaluate_log, real strengths) on the same tree
    q = np.random.default_rng(1).standard_normal(z.size)
    qd = torch.from_numpy(q).to(dev)
    ud = torch.empty_like(qd)
    for prec in ("mixed", "fp64"):
        pl = F.plan(tree, 13, 0.5, prec)
        tl = _time(lambda: F.evaluate_log(pl, qd, ud), reps, torch)
        rec = {"p": 13, "n_levels": 9, "log_ms": tl * 1e3, "mpoints_s": z.size / tl / 1e6}
        if with_errors:
            import oracle
            sub = W.subsample(z.size, 2000, seed=3)
            ref = oracle.direct_log_points(z, q, z[sub])
            rec["e2"] = float(np.linalg.norm(ud.cpu().numpy()[sub] - ref) / np.linalg.norm(ref))
        out["log_n1e6_" + prec] = rec
        log("log kernel N=1e6 (%s, p=13): evaluate_log %.3f ms%s" % (prec, tl * 1e3,
            ", e2 %.2e" % rec["e2"] if "e2" in rec else ""))
    # evaluation points apart from the sources (fmm_evaluate_points, eq. 2.2):
    # the same tree and 1e6 uniform points of their own
    yp = np.random.default_rng(5)
    y = yp.random(z.size) + 1j * yp.random(z.size)
    ydev = torch.from_numpy(y).to(dev)
    for prec in ("mixed", "fp64"):
        pl = F.plan(tree, 13, 0.5, prec)
        py = torch.empty_like(ydev)
        te = _time(lambda: F.evaluate(pl, md, phi), reps, torch)
        tp = _time(lambda: F.evaluate_points(pl, md, ydev, out=py), reps, torch)
        rec = {"p": 13, "n_levels": 9, "n_points": int(y.size), "evaluate_ms": te * 1e3, "points_ms": tp * 1e3,
               "mpoints_s": y.size / tp / 1e6}
        if with_errors:
            import oracle
            sub = W.subsample(y.size, 2000, seed=6)
            ref = oracle.direct_points(z, m, y[sub])
            got = py.cpu().numpy()[sub]
            rec["e2"] = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
            rec["e_inf"] = float(np.abs(got - ref).max() / np.abs(ref).max())
        out["points_n1e6_" + prec] = rec
        log("evaluation points N=1e6 sources, 1e6 points (%s, p=13): evaluate_points %.3f ms (evaluate %.3f ms)%s"
            % (prec, tp * 1e3, te * 1e3, ", e2 %.2e" % rec["e2"] if "e2" in rec else ""))
    del tree, phi, dphi, ydev
    z, m, _ = W.uniform(200000, seed=0)
    zd = torch.from_numpy(z).to(dev)
    md = torch.from_numpy(m).to(dev)
    tree = F.build_tree(zd, default_levels(z.size))
    for prec in ("mixed", "fp64"):
        pl = F.plan(tree, 16, 0.5, prec)
        phi = F.evaluate(pl, md)
        g = 2 * phi
        tf = _time(lambda: F.evaluate(pl, md, phi), reps, torch)
        ta = _time(lambda: F.evaluate_adjoint(pl, md, g), reps, torch)
        out["adjoint_n2e5_" + prec] = {"forward_ms": tf * 1e3, "adjoint_ms": ta * 1e3, "ratio": ta / tf}
        log("adjoint N=2e5 (%s): forward %.3f ms, adjoint %.3f ms, ratio %.2f" % (prec, tf * 1e3, ta * 1e3, ta / tf))
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=1_000_000)
    ap.add_argument("--p", type=int, default=0,
                    help="expansion order; 0 (default): chosen for the error target by fmm_choose_order")
    ap.add_argument("--theta", type=float, default=0.5)
    ap.add_argument("--levels", type=str, default="8,9,10")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle legs")
    ap.add_argument("--no-forms", action="store_true", help="skip the batch and adjoint measurements")
    ap.add_argument("--clustered-breakdown", action="store_true",
                    help="only the per-phase breakdown of the clustered time step (for kernel traces); no JSON")
    ap.add_argument("--pmc-workload", action="store_true",
                    help="for hardware-counter runs: warmup + steps mixed-precision steps at the first "
                         "--levels value, then a 256 MiB device copy (counter calibration); no JSON")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1311_1006_amd as F
    from paper_1311_1006_amd import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    F.lib()
    dev = torch.device("cuda:0")
    n, p, theta = args.n, args.p, args.theta
    z, m, sub = W.uniform(n, seed=0)
    zd = torch.from_numpy(z).to(dev)
    md = torch.from_numpy(m).to(dev)
    out = torch.empty_like(md)
    stream = torch.cuda.current_stream()
    # expansion order per N_levels: fixed (--p), or the smallest p whose FP64
    # and mixed results meet half the error target on that tree
    p_fixed = p
    orders = {}

    def order(L):
        if p_fixed:
            return p_fixed
        if L not in orders:
            t0 = time.perf_counter()
            tr = F.build_tree(zd, L)
            pL, (e64, emx) = F.choose_order(tr, md, theta, ERR_TARGET / 2, p_lo=8, p_hi=24)
            del tr
            if pL < 0:
                raise SystemExit("N_levels=%d: no expansion order in [8, 24] reaches half the error target" % L)
            orders[L] = {"p": pL, "err_fp64": e64, "err_mixed": emx}
            log("N_levels=%d: expansion order p=%d (fp64 %.2e, mixed %.2e against p=32; %.2f s)" %
                (L, pL, e64, emx, time.perf_counter() - t0))
        return orders[L]["p"]

    def step(prec, cfg, timing=False):
        L, split, batch = cfg
        tree = F.build_tree(zd, L)
        pl = F.plan(tree, order(L), theta, prec, p2p_split=split, m2l_batch=batch, timing=timing)
        F.evaluate(pl, md, out)
        return tree, pl

    def time_steps(prec, cfg, k, trials=2):
        """seconds per step: the best of `trials` runs of k steps"""
        for _ in range(2):
            step(prec, cfg)
        best = None
        for _ in range(trials):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(k):
                step(prec, cfg)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / k
            best = dt if best is None else min(best, dt)
        return best

    levels = [int(x) for x in args.levels.split(",") if 4 ** (int(x) - 1) <= n]
    if args.clustered_breakdown:
        measure_clustered_breakdown(F, W, torch, dev)
        return
    if args.pmc_workload:
        for _ in range(args.warmup + args.steps):
            step("mixed", (levels[0], 0, 0))
        torch.cuda.synchronize()
        a = torch.ones(32 << 20, dtype=torch.float64, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        log("pmc workload: %d mixed steps at N_levels=%d, then a copy of %d bytes" %
            (args.warmup + args.steps, levels[0], a.numel() * 8))
        return

    # ---- N_levels, then the P2P split and the M2L batch, by timing sweeps
    best_cfg = {}
    for prec in ("mixed", "fp64"):
        best = None
        for L in levels:
            dt = time_steps(prec, (L, 0, 0), 5)
            log("sweep %s L=%d: %.3f ms" % (prec, L, dt * 1e3))
            if best is None or dt < best[0]:
                best = (dt, (L, 0, 0))
        L = best[1][0]
        # a launch shape replaces the automatic one only when it is at least
        # 1% faster (the spread of this timing between runs)
        for cfg in ((L, 2, 0), (L, 0, 2), (L, 0, 8)):
            dt = time_steps(prec, cfg, 5)
            log("sweep %s L=%d split=%d batch=%d: %.3f ms" % (prec, cfg[0], cfg[1], cfg[2], dt * 1e3))
            if dt < 0.99 * best[0]:
                best = (dt, cfg)
        best_cfg[prec] = best[1]

    # ---- timed region: K steps, mixed precision (the metric), then FP64
    res = {}
    for prec in ("mixed", "fp64"):
        cfg = best_cfg[prec]
        for _ in range(args.warmup):
            step(prec, cfg)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            tree, pl = step(prec, cfg)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        # evaluate-only throughput on the last plan
        for _ in range(3):
            F.evaluate(pl, md, out)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(args.steps):
            F.evaluate(pl, md, out)
        torch.cuda.synchronize()
        dte = (time.perf_counter() - t1) / args.steps
        phi = out.cpu().numpy()
        # per-step device times (events on the stream the step is ordered on;
        # the side streams join it before the end event): median and minimum
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(args.steps)]
        for a, b in evs:
            a.record()
            step(prec, cfg)
            b.record()
        torch.cuda.synchronize()
        per_step = sorted(a.elapsed_time(b) for a, b in evs)
        # the tree build alone, the same way
        for a, b in evs:
            a.record()
            F.build_tree(zd, cfg[0])
            b.record()
        torch.cuda.synchronize()
        per_tree = sorted(a.elapsed_time(b) for a, b in evs)
        # per-phase device times (hipEvents on the evaluation stream) of the same plan shape
        plt = F.plan(tree, order(cfg[0]), theta, prec, p2p_split=cfg[1], m2l_batch=cfg[2], timing=True)
        ph = {}
        for r in range(args.steps + 1):
            F.evaluate(plt, md, out)
            st = plt.stats()
            if r:
                for k in ("t_upward_us", "t_m2l_us", "t_l2l_us", "t_p2p_us", "t_downward_us", "t_total_us"):
                    ph[k] = ph.get(k, 0.0) + st[k] / args.steps
        st = plt.stats()
        res[prec] = dict(L=cfg[0], p=order(cfg[0]), split=cfg[1], batch=cfg[2], t=dt, t_eval=dte, stats=st, phases=ph,
                         p2p_us=ph["t_p2p_us"], m2l_us=ph["t_m2l_us"], phi=phi,
                         step_ms_median=float(np.median(per_step)), step_ms_min=per_step[0],
                         tree_us_median=1e3 * float(np.median(per_tree)), tree_us_min=1e3 * per_tree[0])
        log("%s: L=%d p=%d split=%d batch=%d step %.3f ms (%.1f Mpoints/s), evaluate %.3f ms, phases %s" %
            (prec, cfg[0], order(cfg[0]), cfg[1], cfg[2], dt * 1e3, n / dt / 1e6, dte * 1e3,
             " ".join("%s=%.1f" % (k[2:-3], v) for k, v in ph.items())))

    forms = None if args.no_forms else measure_forms(F, W, torch, dev, args.steps, not args.no_cpu)

    # ---- accuracy vs the FP64 direct sum (CPU oracle) on the subsample
    err = {}
    cpu_baseline = None
    parity = None
    if not args.no_cpu:
        import oracle
        t0 = time.perf_counter()
        ref = oracle.direct(z, m, sub)
        log("direct sum on %d targets: %.1f s" % (sub.size, time.perf_counter() - t0))
        for prec in res:
            err[prec] = oracle.rel_err2(res[prec]["phi"][sub], ref)
            err[prec + "_inf"] = oracle.rel_errinf(res[prec]["phi"][sub], ref)
            log("%s vs direct: e2 %.3e, e_inf %.3e" % (prec, err[prec], err[prec + "_inf"]))
        # CPU oracle (serial FMM O2, its P2P loop OpenMP-parallel) on the full
        # workload; its result is the parity reference of the FP64 path at the
        # same (p, theta, N_levels)
        L = best_cfg["fp64"][0]
        p = order(L)
        t0 = time.perf_counter()
        o2 = oracle.fmm(z, m, p, theta, L)
        tc = time.perf_counter() - t0
        parity = {"n_levels": L, "p": p, "theta": theta,
                  "fp64_e2": oracle.rel_err2(res["fp64"]["phi"], o2),
                  "fp64_einf": oracle.rel_errinf(res["fp64"]["phi"], o2)}
        if res["mixed"]["L"] == L:
            parity["mixed_e2"] = oracle.rel_err2(res["mixed"]["phi"], o2)
            parity["mixed_einf"] = oracle.rel_errinf(res["mixed"]["phi"], o2)
        log("parity against the oracle's serial FMM (all %d points): %s" % (n, parity))
        cpu_baseline = {"value": n / tc / 1e6, "unit": "Mpoints/s", "cores": oracle.threads(),
                        "kind": "oracle",
                        "sample": "one full serial-FMM evaluation (tree, lists, P2M..L2P, P2P) of the "
                                  "same N=1e6 workload at p=%d, theta=%.2f, N_levels=%d; %.1f s" % (p, theta, L, tc)}
        log("cpu oracle FMM: %.2f s" % tc)

    mx, fp = res["mixed"], res["fp64"]
    p_rule = ("fixed by --p" if p_fixed else
              {"rule": "smallest p in [8, 24] whose FP64 and mixed results agree with an FP64 evaluation "
                       "at p=32 to half the error target (relative 2-norm over all points), per N_levels",
               "tol": ERR_TARGET / 2, "per_n_levels": {str(k): v for k, v in orders.items()}})
    st = mx["stats"]
    # roofline of the two evaluation kernels (mixed precision), each from its
    # own average launch duration (hipEvents on the evaluation stream); the
    # one with the longer launch is reported as the dominant kernel
    tflop = P2P_FLOP_PER_PAIR * st["n_p2p_pairs"] / (mx["p2p_us"] * 1e-6) / 1e12
    roof_p2p = {"bound": "alu", "kernel": "k_p2p32 (mixed near field)", "achieved": tflop,
                "peak": PEAK_FP32_VALU, "unit": "TFLOP/s", "frac": tflop / PEAK_FP32_VALU,
                "traffic": profile_traffic("p2p_mixed_uniform_n1e6_L9_pmc.txt"),
                "peak_without_packed_fp32": PEAK_FP32_NOPACK,
                "frac_without_packed_fp32": tflop / PEAK_FP32_NOPACK,
                "avg_us": mx["p2p_us"], "pairs": st["n_p2p_pairs"], "flop_per_pair": P2P_FLOP_PER_PAIR}
    fpp = m2l_flop_per_pair(mx["p"])
    tflop = fpp * st["n_m2l_pairs"] / (mx["m2l_us"] * 1e-6) / 1e12
    slots = mx["batch"] or M2L_AUTO_SLOTS_MIXED   # the counters were taken with the automatic shape
    roof_m2l = {"bound": "mfma", "kernel": "k_m2l<float> (mixed M2L, FP32 MFMA, %d slots per box)" % slots,
                "achieved": tflop, "peak": PEAK_FP32_MFMA, "unit": "TFLOP/s", "frac": tflop / PEAK_FP32_MFMA,
                "traffic": profile_traffic("m2l_mixed_uniform_n1e6_L9_pmc.txt")
                if slots == M2L_AUTO_SLOTS_MIXED else None,
                "avg_us": mx["m2l_us"], "pairs": st["n_m2l_pairs"], "flop_per_pair": fpp}
    # the tree build (every kernel of one build, HBM-bound): algorithmic bytes
    # per build = TREE_BYTES_PER_POINT_SPLIT per point and binary split
    # (2 (N_levels - 1) splits), over the build's median device time
    nsplit = 2 * (mx["L"] - 1)
    tree_bytes = TREE_BYTES_PER_POINT_SPLIT * nsplit * n
    gbs = tree_bytes / (mx["tree_us_median"] * 1e-6) / 1e9
    roof_tree = {"bound": "hbm", "kernel": "tree build (%d binary splits: global split stages + in-LDS stage)" % nsplit,
                 "achieved": gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": gbs / PEAK_HBM_GBS,
                 "traffic": profile_traffic("tree_uniform_n1e6_L9_pmc.txt") if mx["L"] == 9 else None,
                 "avg_us": mx["tree_us_median"], "min_us": mx["tree_us_min"],
                 "bytes_per_build": tree_bytes, "bytes_per_point_split": TREE_BYTES_PER_POINT_SPLIT}
    # the dominant one: the longest device time per step
    cands = {"p2p": roof_p2p, "m2l": roof_m2l, "tree": roof_tree}
    dom = max(cands, key=lambda k: cands[k]["avg_us"])
    roofline = cands[dom]
    other = {k: v for k, v in cands.items() if k != dom}
    line = {
        "metric": "Mpoints/s full FMM eval N=1e6 @rel err<=1e-6: mixed-prec vs plain FP64 GPU",
        "value": n / mx["t"] / 1e6,
        "unit": "Mpoints/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": mx["t"] * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": "uniform unit square N=1e6, complex N(0,1) strengths, seed 0",
                   "n": n, "p": mx["p"], "p_rule": p_rule, "theta": theta, "n_levels": mx["L"], "p2p_split": mx["split"],
                   "m2l_batch": mx["batch"], "precision": "mixed", "step": "build_tree+plan+evaluate"},
        "fp64": {"value": n / fp["t"] / 1e6, "n_levels": fp["L"], "p": fp["p"], "ms_per_step": fp["t"] * 1e3,
                 "step_ms_median": fp["step_ms_median"], "step_ms_min": fp["step_ms_min"],
                 "tree_us_median": fp["tree_us_median"],
                 "eval_only_mpoints_s": n / fp["t_eval"] / 1e6, "e2": err.get("fp64"), "e_inf": err.get("fp64_inf"),
                 "phases_us": fp["phases"]},
        "mixed": {"step_ms_median": mx["step_ms_median"], "step_ms_min": mx["step_ms_min"],
                  "tree_us_median": mx["tree_us_median"],
                  "eval_only_mpoints_s": n / mx["t_eval"] / 1e6, "e2": err.get("mixed"), "e_inf": err.get("mixed_inf"),
                  "phases_us": mx["phases"]},
        "parity_fp64_vs_oracle_e2": parity["fp64_e2"] if parity else None,
        "parity_vs_oracle_fmm": parity,
        "speedup_mixed_vs_fp64": fp["t"] / mx["t"],
        "roofline": roofline,
        "roofline_other": other,
        "cpu_baseline": cpu_baseline,
        "forms": forms,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
