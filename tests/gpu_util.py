"""Helpers shared by the GPU tests: device transfer and comparison against
the oracle.  Imported only by tests marked ``gpu``."""
import numpy as np


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.complex128)).to("cuda")


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def e2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def same_tree(orc, F, z, L, offsets=None, prob=0, tree=None):
    """GPU tree of problem `prob` vs the oracle tree of the same points: the
    same boxes (point sets), bit-identical geometry and ranges."""
    if tree is None:
        tree = F.build_tree(dev(z), L)
    perm_g, rng_g, geom_g = tree.download(prob)
    perm_o, rng_o, geom_o = orc.tree(z, L)
    assert np.array_equal(rng_g, rng_o)
    assert np.array_equal(geom_g.view(np.uint64), geom_o.view(np.uint64)), "geometry differs"
    for b in range(rng_o.shape[0]):
        s0, c = rng_o[b]
        assert np.array_equal(np.sort(perm_g[s0:s0 + c]), np.sort(perm_o[s0:s0 + c])), "box %d" % b
    return tree


def einf(a, b):
    """e_inf = max|a - b| / max|b| (the secondary error metric)."""
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def epoint(a, b):
    """Largest error of one value in units of the RMS of the reference:
    max_i |a_i - b_i| / (||b||_2 / sqrt(n)).  Catches a few values that are
    far off while the 2-norm stays small."""
    return float(np.max(np.abs(a - b)) / (np.linalg.norm(b) / np.sqrt(b.size)))
