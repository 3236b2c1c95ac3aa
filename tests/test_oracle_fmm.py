"""Pins of the serial FMM oracle O2: the single expansion operators against
closed forms, the balanced tree and the connectivity lists against their
defining properties (Sec. 2.1-2.2), and the whole FMM against the direct
sum, the error bound of Table 4.1 and the symmetries of the kernel."""
import numpy as np
import pytest

from paper_1311_1006_amd import workloads as W

# ---------------------------------------------------------------- operators


def test_p2m_closed_form_remainder(orc):
    # sum_{k<p} (z_j - c)^k / (z - c)^(k+1) = (1 - rho^p) / (z - z_j), rho = (z_j - c)/(z - c)
    rng = np.random.default_rng(1)
    c = 0.3 + 0.4j
    zs = c + 0.1 * (rng.random(5) - 0.5 + 1j * (rng.random(5) - 0.5))
    ms = rng.standard_normal(5) + 1j * rng.standard_normal(5)
    zt = np.array([1.5 + 0.2j, -0.8 - 0.9j, 0.3 + 2.0j])
    for p in (1, 5, 17):
        a = orc.p2m(c, zs, ms, p)
        got = orc.mpole_eval(c, a, zt)
        ref = np.zeros(3, complex)
        for zj, mj in zip(zs, ms):
            rho = (zj - c) / (zt - c)
            ref += mj * (1 - rho ** p) / (zt - zj)
        assert np.max(np.abs(got - ref)) <= 1e-14 * np.max(np.abs(ref))


def test_l2p_closed_form_remainder(orc):
    # local expansion about c of one far source (written here from the
    # geometric series): b_l = -m / (z_j - c)^(l+1); the truncated series
    # equals m (1 - rho^p) / (z - z_j) with rho = (z - c)/(z_j - c)
    c, zj, mj = 0.1 - 0.2j, 2.0 + 1.5j, 0.7 - 0.3j
    zt = c + np.array([0.05, -0.1j, 0.07 + 0.02j])
    for p in (1, 6, 20):
        b = -mj / (zj - c) ** (np.arange(p) + 1)
        got = orc.l2p(c, b, zt)
        rho = (zt - c) / (zj - c)
        ref = mj * (1 - rho ** p) / (zt - zj)
        assert np.max(np.abs(got - ref)) <= 1e-14 * np.max(np.abs(ref))


def test_m2m_is_exact(orc):
    rng = np.random.default_rng(2)
    cp = 0.5 + 0.5j
    ccs = [0.4 + 0.45j, 0.62 + 0.55j]
    p = 15
    total = np.zeros(p, complex)
    zall, mall = [], []
    for cc in ccs:
        z = cc + 0.05 * (rng.random(7) - 0.5 + 1j * (rng.random(7) - 0.5))
        m = rng.standard_normal(7) + 1j * rng.standard_normal(7)
        total += orc.m2m(cc, cp, orc.p2m(cc, z, m, p))
        zall.append(z)
        mall.append(m)
    direct = orc.p2m(cp, np.concatenate(zall), np.concatenate(mall), p)
    assert np.max(np.abs(total - direct)) <= 1e-14 * np.max(np.abs(direct))


def test_l2l_preserves_the_local_polynomial(orc):
    rng = np.random.default_rng(3)
    p = 18
    b = rng.standard_normal(p) + 1j * rng.standard_normal(p)
    cp, cc = 0.0 + 0.0j, 0.03 - 0.02j
    z = cc + 0.02 * (rng.random(6) - 0.5 + 1j * (rng.random(6) - 0.5))
    ref = orc.l2p(cp, b, z)
    got = orc.l2p(cc, orc.l2l(cp, cc, b), z)
    assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_m2l_converges_to_direct_at_large_p(orc):
    rng = np.random.default_rng(4)
    cs, ct = 0.0 + 0.0j, 1.0 + 0.5j
    zs = cs + 0.2 * (rng.random(9) - 0.5 + 1j * (rng.random(9) - 0.5))
    ms = rng.standard_normal(9) + 1j * rng.standard_normal(9)
    zt = ct + 0.2 * (rng.random(5) - 0.5 + 1j * (rng.random(5) - 0.5))
    ref = np.array([np.sum(ms / (t - zs)) for t in zt])
    errs = []
    for p in (10, 20, 60):
        b = orc.m2l(cs, ct, orc.p2m(cs, zs, ms, p))
        errs.append(np.max(np.abs(orc.l2p(ct, b, zt) - ref)) / np.max(np.abs(ref)))
    assert errs[2] < 1e-13
    assert errs[1] < errs[0]


# --------------------------------------------------------------------- tree


def _check_tree(orc, z, L):
    n = z.size
    perm, rng_, geom = orc.tree(z, L)
    assert np.array_equal(np.sort(perm), np.arange(n))
    zt = z[perm]
    nf = 4 ** (L - 1)
    leaves = rng_[orc.level_base(L - 1):]
    assert set(leaves[:, 1]) <= {n // nf, -(-n // nf)}
    for l in range(L):
        base = orc.level_base(l)
        for b in range(4 ** l):
            s0, cnt = rng_[base + b]
            pts = zt[s0:s0 + cnt]
            g = geom[base + b]
            # tight bounding box, midpoint centre, half-diagonal radius
            assert g[0] == pts.real.min() and g[1] == pts.real.max()
            assert g[2] == pts.imag.min() and g[3] == pts.imag.max()
            assert g[4] == 0.5 * (g[0] + g[1]) and g[5] == 0.5 * (g[2] + g[3])
            dx, dy = g[1] - g[0], g[3] - g[2]
            assert g[6] == 0.5 * np.sqrt(dx * dx + dy * dy)
            if l + 1 < L:
                cb = orc.level_base(l + 1) + 4 * b
                ch = rng_[cb:cb + 4]
                # the four children tile the parent's range in order
                assert ch[0, 0] == s0 and np.all(ch[1:, 0] == ch[:-1, 0] + ch[:-1, 1])
                assert ch[:, 1].sum() == cnt
                _check_median(pts, perm[s0:s0 + cnt], ch[:, 1])
    return perm, rng_, geom


def _key(pts, idx, axis):
    c = pts.real if axis == 0 else pts.imag
    return list(zip(c, idx))


def _check_split(pts, idx, nlow):
    """pts[:nlow] and pts[nlow:] must be separated along the longer side of
    the bounding box of pts, ordering by (coordinate, input index), and
    nlow = floor(n/2)."""
    assert nlow == pts.size // 2
    w = pts.real.max() - pts.real.min()
    h = pts.imag.max() - pts.imag.min()
    axis = 0 if w >= h else 1
    k = _key(pts, idx, axis)
    assert max(k[:nlow]) < min(k[nlow:])


def _check_median(pts, idx, counts):
    h = counts[0] + counts[1]
    _check_split(pts, idx, h)
    _check_split(pts[:h], idx[:h], counts[0])
    _check_split(pts[h:], idx[h:], counts[2])


def test_tree_brute_force_one_point_per_leaf(orc):
    z, _, _ = W.uniform(16, seed=11)
    perm, rng_, geom = _check_tree(orc, z, 3)
    assert np.all(rng_[orc.level_base(2):, 1] == 1)


@pytest.mark.parametrize("n,L", [(1000, 4), (1037, 5), (4096, 6)])
def test_tree_invariants_uniform(orc, n, L):
    z, _, _ = W.uniform(n, seed=n)
    _check_tree(orc, z, L)


def test_tree_with_ties(orc):
    # coincident coordinates: the input index breaks ties
    rng = np.random.default_rng(5)
    z = np.round(rng.random(300) * 4) / 4 + 1j * np.round(rng.random(300) * 4) / 4
    _check_tree(orc, z, 4)


def test_tree_rejects_too_many_levels(orc):
    z, _, _ = W.uniform(15, seed=1)
    with pytest.raises(ValueError):
        orc.tree(z, 3)       # 16 leaves > 15 points


# ---------------------------------------------------------------- lists


def test_theta_criterion_hand_cases(orc):
    # boxes of radius 1 at distance d, theta = 0.5: R + theta r = 1.5 vs theta d
    def g(cx, r):
        return np.array([0, 0, 0, 0, cx, 0.0, r])
    assert orc.well_separated(g(0, 1), g(4, 1), 0.5)          # 1.5 <= 2
    assert orc.well_separated(g(0, 1), g(3, 1), 0.5)          # 1.5 <= 1.5 (equality counts)
    assert not orc.well_separated(g(0, 1), g(2.9, 1), 0.5)
    assert not orc.well_separated(g(0, 1), g(0, 1), 0.5)      # d = 0
    # unequal radii: R = 2, r = 0.5 -> 2.25 <= 0.5 d  <=>  d >= 4.5
    assert orc.well_separated(g(0, 2), g(4.5, 0.5), 0.5)
    assert not orc.well_separated(g(0, 0.5), g(4.4, 2), 0.5)


def _leaf_of(rng_, L, n, orc):
    """level-local box index of every tree position at every level"""
    out = np.zeros((L, n), np.int64)
    for l in range(L):
        base = orc.level_base(l)
        for b in range(4 ** l):
            s0, cnt = rng_[base + b]
            out[l, s0:s0 + cnt] = b
    return out


@pytest.mark.parametrize("kind", ["uniform", "clustered", "line"])
def test_lists_cover_every_pair_exactly_once(orc, kind):
    n, L, theta = 600, 4, 0.5
    if kind == "uniform":
        z, _, _ = W.uniform(n, seed=12)
    elif kind == "line":
        z, _ = W.line_like(n, seed=12)
    else:
        z, _ = W.clustered(n, seed=12, nclusters=4, sigma=0.01)
    perm, rng_, geom = orc.tree(z, L)
    lists = orc.lists(geom, L, theta)
    box = _leaf_of(rng_, L, n, orc)
    cover = np.zeros((n, n), np.int64)
    for l in range(L):
        so, sid, wo, wid = lists[l]
        nb = 4 ** l
        S = np.zeros((nb, nb), bool)
        Wm = np.zeros((nb, nb), bool)
        for b in range(nb):
            S[b, sid[so[b]:so[b + 1]]] = True
            Wm[b, wid[wo[b]:wo[b + 1]]] = True
            assert np.all(np.diff(sid[so[b]:so[b + 1]]) > 0)
            assert np.all(np.diff(wid[wo[b]:wo[b + 1]]) > 0)
            assert S[b, b]
        assert np.array_equal(S, S.T) and np.array_equal(Wm, Wm.T)
        assert not np.any(S & Wm)
        g = geom[orc.level_base(l):orc.level_base(l) + nb]
        for b in range(nb):
            for c in wid[wo[b]:wo[b + 1]]:
                assert orc.well_separated(g[b], g[c], theta)
            for c in sid[so[b]:so[b + 1]]:
                if c != b:
                    assert not orc.well_separated(g[b], g[c], theta)
        cover += Wm[box[l][:, None], box[l][None, :]]
        if l == L - 1:
            cover += S[box[l][:, None], box[l][None, :]]
    assert np.all(cover == 1)


def test_list_sizes_follow_complexity_estimates(orc):
    # (2.6): C_P2P ~ N^2/(2 N_f) pi ((1+theta)/theta)^2 pairs;
    # (2.7): finest-level M2L count ~ (3 N_f / 2) pi ((1+theta)/theta)^2
    n, L, theta = 20000, 6, 0.5
    z, _, _ = W.uniform(n, seed=13)
    perm, rng_, geom = orc.tree(z, L)
    lists = orc.lists(geom, L, theta)
    so, sid, wo, wid = lists[L - 1]
    leaves = rng_[orc.level_base(L - 1):]
    npairs = sum(int(leaves[b, 1]) * int(leaves[sid[so[b]:so[b + 1]], 1].sum()) for b in range(4 ** (L - 1)))
    nf = 4 ** (L - 1)
    fac = np.pi * ((1 + theta) / theta) ** 2
    est_p2p = n * n / (2 * nf) * fac
    est_m2l = 1.5 * nf * fac
    assert 0.5 < npairs / est_p2p < 2.0
    assert 0.5 < wid.size / est_m2l < 2.0


# ------------------------------------------------------------------ FMM


@pytest.mark.parametrize("tol,theta,p", [(1e-6, 0.5, 17), (1e-6, 0.35, 11), (1e-7, 0.4, 16),
                                          (1e-8, 0.65, 39), (1e-8, 0.5, 24)])
def test_fmm_within_table_4_1_tolerance(orc, tol, theta, p):
    z, m, _ = W.uniform(3000, seed=21)
    ref = orc.direct(z, m)
    phi = orc.fmm(z, m, p, theta, 4)
    assert orc.rel_err2(phi, ref) <= tol


def test_fmm_clustered_within_tolerance(orc):
    z, m = W.clustered(4000, seed=22, nclusters=8)
    ref = orc.direct(z, m)
    phi = orc.fmm(z, m, 17, 0.5, 5)
    assert orc.rel_err2(phi, ref) <= 1e-6


def test_fmm_error_decays_geometrically(orc):
    z, m, _ = W.uniform(2000, seed=23)
    ref = orc.direct(z, m)
    e = [orc.rel_err2(orc.fmm(z, m, p, 0.5, 4), ref) for p in (6, 12, 18, 24)]
    assert all(e[i + 1] < 0.2 * e[i] for i in range(3))
    assert e[3] < 1e-9


def test_fmm_parts_and_single_level(orc):
    z, m, _ = W.uniform(500, seed=24)
    phi, near, far = orc.fmm(z, m, 10, 0.5, 3, parts=True)
    np.testing.assert_array_equal(phi, near + far)
    # one level: everything is near field, equal to the direct sum
    phi1 = orc.fmm(z, m, 10, 0.5, 1)
    assert orc.rel_err2(phi1, orc.direct(z, m)) < 1e-14


def test_fmm_operator_is_antisymmetric(orc):
    # with symmetric lists and equal truncation the FMM operator A satisfies
    # A^T = -A, so v^T A u = -u^T A v and sum_i m_i (A m)_i = 0
    z, u, _ = W.uniform(1500, seed=25)
    v = W.uniform(1500, seed=26)[1]
    Au = orc.fmm(z, u, 12, 0.5, 4)
    Av = orc.fmm(z, v, 12, 0.5, 4)
    scale = np.sum(np.abs(v * Au))
    assert abs(np.sum(v * Au) + np.sum(u * Av)) <= 1e-14 * scale
    assert abs(np.sum(u * Au)) <= 1e-14 * np.sum(np.abs(u * Au))


def test_fmm_invariances(orc):
    z, m, _ = W.uniform(2500, seed=27)
    p, theta, L = 17, 0.5, 4
    phi = orc.fmm(z, m, p, theta, L)
    # scaling by a power of two is exact in binary floating point
    np.testing.assert_array_equal(orc.fmm(4.0 * z, m, p, theta, L), phi / 4.0)
    # a permutation of the input permutes the output (distinct coordinates
    # give the same tree and the same summation order)
    pr = np.random.default_rng(1).permutation(z.size)
    np.testing.assert_array_equal(orc.fmm(z[pr], m[pr], p, theta, L), phi[pr])
    ref = orc.direct(z, m)
    tol = 1e-6
    # translation
    assert orc.rel_err2(orc.fmm(z + (0.25 + 0.5j), m, p, theta, L), phi) < 1e-10
    # rotation: phi(e^{ia} z) = e^{-ia} phi(z) (the tree is not rotation equivariant)
    a = 0.7
    rot = orc.fmm(np.exp(1j * a) * z, m, p, theta, L)
    assert orc.rel_err2(rot, np.exp(-1j * a) * ref) < 2 * tol
    # conjugation of positions and strengths conjugates the potential
    cj = orc.fmm(np.conj(z), np.conj(m), p, theta, L)
    assert orc.rel_err2(cj, np.conj(ref)) < 2 * tol
