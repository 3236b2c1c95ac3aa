"""Allocation failures: every device allocation of a build / plan /
evaluate sequence is made to fail in turn (fmm_debug_fail_alloc).  The
failing call returns FMM_ENOMEM, writes nothing to its outputs and creates
no handle; the handles made before it stay usable and give the same
results as an undisturbed run; once every handle is destroyed the library
holds as many device blocks as before (fmm_debug_live_blocks)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

FMM_ENOMEM = -2


def _sequence(F, torch, zd, md, prec, outs, made):
    """tree, plan, evaluate, field, graph plan and its evaluation; handles
    go into `made` as they are created (so that a failure leaves the
    earlier ones there); returns the name of each completed step."""
    made["tree"] = F.build_tree(zd, 5)
    made["plan"] = F.plan(made["tree"], 12, 0.5, prec)
    F.evaluate(made["plan"], md, outs["phi"])
    F.evaluate_field(made["plan"], md, outs["phi2"], outs["dphi"])
    made["gplan"] = F.plan(made["tree"], 12, 0.5, prec, graph=True)
    F.evaluate(made["gplan"], md, outs["gphi"])
    torch.cuda.synchronize()


def _outs(torch, md):
    return {k: torch.full_like(md, complex("nan+nanj")) for k in ("phi", "phi2", "dphi", "gphi")}


# which outputs each step writes (the step that fails must leave them NaN)
_STEP_OUTPUTS = {"tree": (), "plan": (), "evaluate": ("phi",), "field": ("phi2", "dphi"), "gplan": (),
                 "gevaluate": ("gphi",)}
_ORDER = ["tree", "plan", "evaluate", "field", "gplan", "gevaluate"]


def _failed_step(made, outs_written):
    if "tree" not in made:
        return "tree"
    if "plan" not in made:
        return "plan"
    if not outs_written["phi"]:
        return "evaluate"
    if not outs_written["phi2"]:
        return "field"
    if "gplan" not in made:
        return "gplan"
    return "gevaluate"


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_every_allocation_failure_is_clean(prec):
    import torch

    import paper_1311_1006_amd as F
    from paper_1311_1006_amd import workloads as W
    z, m, _ = W.uniform(20000, seed=7)
    zd = torch.from_numpy(z).cuda()
    md = torch.from_numpy(m).cuda()
    F.debug_fail_alloc(-1)
    # undisturbed run: reference values, and the schedule and launch tables
    # of this layout cached
    ref = _outs(torch, md)
    made = {}
    _sequence(F, torch, zd, md, prec, ref, made)
    ref = {k: v.cpu().numpy() for k, v in ref.items()}
    assert all(np.isfinite(v).all() for v in ref.values())
    made.clear()
    torch.cuda.synchronize()
    base = F.debug_live_blocks()
    seen = set()
    for k in range(1000):
        outs = _outs(torch, md)
        made = {}
        print("allocation failure at allocation %d (%s)" % (k, prec), flush=True)
        F.debug_fail_alloc(k)
        try:
            _sequence(F, torch, zd, md, prec, outs, made)
            completed = True
        except F.FmmError as e:
            completed = False
            assert e.code == FMM_ENOMEM, (k, e)
            assert "injected" in str(e)
        finally:
            F.debug_fail_alloc(-1)
        torch.cuda.synchronize()
        host = {kk: v.cpu().numpy() for kk, v in outs.items()}
        written = {kk: not np.isnan(v).all() for kk, v in host.items()}
        if completed:
            for kk in ref:
                assert np.array_equal(host[kk], ref[kk]), kk
            made.clear()
            torch.cuda.synchronize()
            assert F.debug_live_blocks() == base
            break
        step = _failed_step(made, written)
        seen.add(step)
        # nothing written by the failing call or the steps after it
        for later in _ORDER[_ORDER.index(step):]:
            for kk in _STEP_OUTPUTS[later]:
                assert np.isnan(host[kk]).all(), (k, step, kk)
        # the handles made before the failure still work and agree with the
        # undisturbed run
        if "plan" in made:
            phi = torch.empty_like(md)
            F.evaluate(made["plan"], md, phi)
            assert np.array_equal(phi.cpu().numpy(), ref["phi"]), (k, step)
        elif "tree" in made:
            pl = F.plan(made["tree"], 12, 0.5, prec)
            phi = F.evaluate(pl, md)
            assert np.array_equal(phi.cpu().numpy(), ref["phi"]), (k, step)
            del pl
        made.clear()
        torch.cuda.synchronize()
        assert F.debug_live_blocks() == base, (k, step)
    else:
        pytest.fail("the sequence never completed")
    # the failures reached the tree build and the plan at least
    assert {"tree", "plan"} <= seen, seen
