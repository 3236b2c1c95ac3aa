"""Pins of the direct-sum oracle O1 (eq. 2.1/2.2) and of the direct-sum
gradient O3 against closed forms, invariants and finite differences."""
import os

import numpy as np
import pytest

from paper_1311_1006_amd import workloads as W


def test_roots_of_unity_closed_form(orc):
    # N unit charges at z_k = c + R w^k (w^N = 1): sum_{j!=k} 1/(z_k - z_j)
    # = P''(z_k)/(2 P'(z_k)) for P = prod (z - z_j), which gives (N-1)/(2(z_k - c)).
    for n, c, R in [(7, 0.0, 1.0), (64, 0.3 - 0.2j, 0.01), (501, 2.0 + 1.0j, 3.0)]:
        z = W.roots_of_unity(n, c, R, phase=0.123)
        phi = orc.direct(z, np.ones(n))
        ref = (n - 1) / (2 * (z - c))
        assert orc.rel_errinf(phi, ref) < 1e-13


def test_derivative_roots_of_unity_closed_form(orc):
    # N unit charges at z_k = c + u_k, u_k^N = R^N.  With P = prod (z - z_j) =
    # (z - c)^N - R^N and Q = P/(z - z_k): sum_{j!=k} 1/(z_k - z_j)^2 =
    # (Q'/Q)^2 - Q''/Q at z_k = (P''/(2P'))^2 - P'''/(3P') = (N-1)(5-N)/(12 u^2),
    # so the field's derivative there (self term left out) is (N-1)(N-5)/(12 u^2).
    for n, c, R in [(2, 0.0, 1.0), (7, 0.0, 1.0), (64, 0.3 - 0.2j, 0.01), (301, 2.0 + 1.0j, 3.0)]:
        z = W.roots_of_unity(n, c, R, phase=0.321)
        d = orc.direct_deriv_points(z, np.ones(n), z)
        ref = (n - 1) * (n - 5) / (12 * (z - c) ** 2)
        if n == 5:
            ref = np.zeros(n)
        assert orc.rel_errinf(d, ref) < 1e-12, n


def test_derivative_matches_central_differences_of_the_field(orc):
    rng = np.random.default_rng(3)
    z = rng.random(300) + 1j * rng.random(300)
    m = rng.standard_normal(300) + 1j * rng.standard_normal(300)
    y = 0.2 + 0.6 * (rng.random(40) + 1j * rng.random(40))
    d = orc.direct_deriv_points(z, m, y)

    def err(h):
        fd = (orc.direct_points(z, m, y + h) - orc.direct_points(z, m, y - h)) / (2 * h)
        return np.max(np.abs(fd - d)) / np.max(np.abs(d))
    for h in (1e-6, 1e-6j):       # holomorphic: the same derivative along x and along y
        assert err(h) <= 1e-6
    # the difference converges to it at second order
    assert 80 < err(1e-4) / err(1e-5) < 120


def test_derivative_leaves_out_coincident_sources(orc):
    rng = np.random.default_rng(4)
    z = rng.random(50) + 1j * rng.random(50)
    m = rng.standard_normal(50) + 1j * rng.standard_normal(50)
    a = orc.direct_deriv_points(z, m, z[:1])
    b = orc.direct_deriv_points(z[1:], m[1:], z[:1])
    assert a[0] == b[0]


def test_smoothed_sum_limits(orc):
    """The smoother of Sec. 5.1: with delta far below every distance the
    factor is 1 to the last bit (the plain sum); with every distance far
    below delta, g ~ r^2/delta^2 turns each term into m conj(dz)/delta^2
    (relative deviation ~ r^2/(2 delta^2)); a coincident source adds nothing."""
    rng = np.random.default_rng(8)
    z = rng.random(400) + 1j * rng.random(400)
    m = rng.standard_normal(400) + 1j * rng.standard_normal(400)
    np.testing.assert_array_equal(orc.direct_smoothed(z, m, 1e-30), orc.direct(z, m))
    c = 0.3 + 0.2j + 1e-4 * (rng.random(60) + 1j * rng.random(60))
    mc = m[:60]
    delta = 1.0
    lin = np.array([np.sum(np.delete(mc * np.conj(c[i] - c), i)) / delta ** 2 for i in range(60)])
    assert orc.rel_errinf(orc.direct_smoothed(c, mc, delta), lin) < 1e-7
    zz = np.concatenate([z[:50], z[:1]])
    mm = np.concatenate([m[:50], [5.0 + 0j]])
    a = orc.direct_smoothed(zz, mm, 0.05, targets=[0])
    b = orc.direct_smoothed(z[:50], m[:50], 0.05, targets=[0])
    assert a[0] == b[0]


def test_equispaced_line_harmonic_numbers(orc):
    # z_k = k h, unit strengths: phi_k = (H_k - H_{N-1-k}) / h
    for n, h in [(10, 1.0), (300, 1e-3)]:
        z = np.arange(n) * h + 0j
        phi = orc.direct(z, np.ones(n))
        H = np.concatenate([[0.0], np.cumsum(1.0 / np.arange(1, n + 1))])
        k = np.arange(n)
        ref = (H[k] - H[n - 1 - k]) / h
        assert np.max(np.abs(phi - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_two_points(orc):
    z = np.array([0.1 + 0.2j, -0.3 + 0.5j])
    m = np.array([1.5 - 0.5j, -2.0 + 0.25j])
    phi = orc.direct(z, m)
    np.testing.assert_allclose(phi[0], m[1] / (z[0] - z[1]), rtol=1e-15)
    np.testing.assert_allclose(phi[1], m[0] / (z[1] - z[0]), rtol=1e-15)


def test_antisymmetry_and_linearity(orc):
    z, m, _ = W.uniform(800, seed=3)
    phi = orc.direct(z, m)
    # sum_i m_i phi_i = sum_{i != j} m_i m_j / (z_i - z_j) = 0 (antisymmetric kernel)
    s = np.sum(m * phi)
    assert abs(s) <= 1e-13 * np.sum(np.abs(m * phi))
    m2 = W.uniform(800, seed=4)[1]
    a, b = 0.7 - 1.1j, -0.3 + 0.2j
    lhs = orc.direct(z, a * m + b * m2)
    rhs = a * phi + b * orc.direct(z, m2)
    assert orc.rel_errinf(lhs, rhs) < 1e-13


def test_compensated_agrees(orc):
    z, m, _ = W.uniform(1500, seed=5)
    a = orc.direct(z, m)
    b = orc.direct_compensated(z, m)
    assert orc.rel_err2(a, b) < 1e-14


def test_exclusion_by_position(orc):
    # a duplicated position contributes nothing at its twin (x_j != y_i in 2.2)
    z = np.array([0.0, 1.0, 1.0, 2.0 + 1j])
    m = np.array([1.0, 2.0, 3.0, 4.0])
    phi = orc.direct(z, m)
    assert phi[1] == pytest.approx(m[0] / (z[1] - z[0]) + m[3] / (z[1] - z[3]), rel=1e-15)
    assert phi[2] == pytest.approx(phi[1], rel=1e-15)


def test_points_and_subset_variants(orc):
    z, m, _ = W.uniform(500, seed=6)
    full = orc.direct(z, m)
    t = np.array([0, 17, 499, 250])
    np.testing.assert_array_equal(orc.direct(z, m, t), full[t])
    np.testing.assert_array_equal(orc.direct_points(z, m, z[t]), full[t])


def _loss(orc, z, m):
    return float(np.sum(np.abs(orc.direct(z, m)) ** 2))


def test_grad_direct_vs_central_fd(orc):
    z, m, _ = W.uniform(12, seed=7)
    phi = orc.direct(z, m)
    gm, gz = orc.grad_direct(z, m, 2 * phi)      # L = sum |phi|^2 -> g = 2 phi
    h = 1e-6
    fd_z = np.zeros(12, complex)
    fd_m = np.zeros(12, complex)
    for k in range(12):
        for unit, tgt in [(1.0, "re"), (1j, "im")]:
            e = np.zeros(12, complex)
            e[k] = unit * h
            dz = (_loss(orc, z + e, m) - _loss(orc, z - e, m)) / (2 * h)
            dm = (_loss(orc, z, m + e) - _loss(orc, z, m - e)) / (2 * h)
            if tgt == "re":
                fd_z[k] += dz
                fd_m[k] += dm
            else:
                fd_z[k] += 1j * dz
                fd_m[k] += 1j * dm
    assert np.linalg.norm(gz - fd_z) / np.linalg.norm(fd_z) < 1e-6
    assert np.linalg.norm(gm - fd_m) / np.linalg.norm(fd_m) < 1e-6


def test_grad_direct_identities(orc):
    z, m, _ = W.uniform(400, seed=8)
    phi = orc.direct(z, m)
    Lval = float(np.sum(np.abs(phi) ** 2))
    gm, gz = orc.grad_direct(z, m, 2 * phi)
    scale = np.sum(np.abs(gz * z)) + np.sum(np.abs(gm * m))
    # translation invariance
    assert abs(np.sum(gz)) <= 1e-12 * np.sum(np.abs(gz))
    # z -> (1+e) z scales phi by 1/(1+e): dL/de = -2L
    assert abs(np.sum(np.real(np.conj(gz) * z)) + 2 * Lval) <= 1e-12 * scale
    # m -> (1+e) m: dL/de = 2L
    assert abs(np.sum(np.real(np.conj(gm) * m)) - 2 * Lval) <= 1e-12 * scale
    # rotations of z or m leave |phi| unchanged
    assert abs(np.sum(np.real(np.conj(gz) * 1j * z))) <= 1e-12 * scale
    assert abs(np.sum(np.real(np.conj(gm) * 1j * m))) <= 1e-12 * scale


def test_p_rule_reproduces_table_4_1(orc):
    path = os.path.join(os.path.dirname(__file__), "golden", "table_4_1_p.txt")
    rows = [l.split() for l in open(path) if l.strip() and not l.startswith("#")]
    assert len(rows) == 15
    for tol, theta, p in rows:
        assert orc.p_from_tol(float(tol), float(theta)) == int(p), (tol, theta)


# ---- the logarithmic potential (the paper's second kernel)

def test_log_roots_of_unity_closed_form(orc):
    # N unit charges at z_k = c + u_k, u_k^N = R^N: prod_{j!=k} (z_k - z_j) =
    # P'(z_k) = N u_k^(N-1), so sum_{j!=k} log|z_k - z_j| = log N + (N-1) log R.
    for n, c, R in [(2, 0.0, 1.0), (7, 0.5 + 0.5j, 0.3), (301, 2.0 + 1.0j, 3.0)]:
        z = W.roots_of_unity(n, c, R, phase=0.2)
        u = orc.direct_log_points(z, np.ones(n), z)
        ref = np.log(n) + (n - 1) * np.log(R)
        assert np.max(np.abs(u - ref)) < 1e-11 * max(1.0, abs(ref))


def test_log_two_points_and_exclusion(orc):
    z = np.array([0.1 + 0.2j, 0.7 - 0.3j, 0.1 + 0.2j])      # point 2 coincides with point 0
    q = np.array([1.5, -0.25, 2.0])
    u = orc.direct_log_points(z, q, z)
    d = abs(z[0] - z[1])
    np.testing.assert_allclose(u, [q[1] * np.log(d), (q[0] + q[2]) * np.log(d), q[1] * np.log(d)], rtol=1e-15)


def test_log_scaling_and_translation(orc):
    # scaling every position by s adds (sum_{j != i} q_j) log s; a shift changes nothing
    rng = np.random.default_rng(3)
    z = rng.random(300) + 1j * rng.random(300)
    q = rng.standard_normal(300)
    u = orc.direct_log_points(z, q, z)
    s = 7.5
    us = orc.direct_log_points(s * z, q, s * z)
    np.testing.assert_allclose(us - u, (q.sum() - q) * np.log(s), rtol=1e-12, atol=1e-12)
    ut = orc.direct_log_points(z + (3 - 2j), q, z + (3 - 2j))
    np.testing.assert_allclose(ut, u, rtol=1e-12, atol=1e-12)


def test_log_gradient_is_the_harmonic_field(orc):
    # d/dx log|y - z| = Re 1/(y - z), d/dy log|y - z| = -Im 1/(y - z): central
    # differences of the log oracle against the harmonic oracle (real strengths)
    rng = np.random.default_rng(4)
    z = rng.random(200) + 1j * rng.random(200)
    q = rng.standard_normal(200)
    y = 1.5 + rng.random(20) + 1j * rng.random(20)
    f = orc.direct_points(z, q + 0j, y)
    h = 1e-5
    gx = (orc.direct_log_points(z, q, y + h) - orc.direct_log_points(z, q, y - h)) / (2 * h)
    gy = (orc.direct_log_points(z, q, y + 1j * h) - orc.direct_log_points(z, q, y - 1j * h)) / (2 * h)
    np.testing.assert_allclose(gx, f.real, rtol=1e-7, atol=1e-7)
    np.testing.assert_allclose(gy, -f.imag, rtol=1e-7, atol=1e-7)
