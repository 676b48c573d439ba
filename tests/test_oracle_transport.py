"""Pins of the oracle's helix transport (not self-referential).

The transport uses the tangent-of-half-sum chord and a Maclaurin series of
asin(u)/u.  It is checked against (a) the closed-form circle written with
numpy's arcsin, (b) RK4 integration of the equations of motion in x, (c)
reversibility and composition, (d) the straight line at zero field, and its
Jacobian against central differences.
"""
import numpy as np
import pytest

C_LIGHT = 2.99792458e-3


def closed_form(p, x0, x1, bz):
    y, z, s, t, k = p
    kap = -C_LIGHT * bz * k
    s1 = s + kap * (x1 - x0)
    c0, c1 = np.sqrt(1 - s * s), np.sqrt(1 - s1 * s1)
    y1 = y + (c0 - c1) / kap
    z1 = z + t * (np.arcsin(s1) - np.arcsin(s)) / kap
    return np.array([y1, z1, s1, t, k])


def rk4(p, x0, x1, bz, n=4000):
    y, z, s, t, k = p
    kap = -C_LIGHT * bz * k

    def f(v):
        ss = v[2]
        c = np.sqrt(1 - ss * ss)
        return np.array([ss / c, t / c, kap])

    v = np.array([y, z, s], dtype=np.float64)
    h = (x1 - x0) / n
    for _ in range(n):
        a = f(v); b = f(v + 0.5 * h * a); c = f(v + 0.5 * h * b); d = f(v + h * c)
        v = v + h / 6.0 * (a + 2 * b + 2 * c + d)
    return np.array([v[0], v[1], v[2], t, k])


CASES = [
    # y, z, s, t, k, x0, x1
    (1.0, 5.0, 0.1, 0.3, 1.0, 100.0, 101.025),
    (-3.0, -20.0, -0.5, -0.8, -10.0, 85.0, 86.0253),      # pT = 0.1 GeV
    (0.0, 0.0, 0.3, 1.0, 5.0, 150.0, 140.0),              # inward step
    (2.0, 1.0, 0.7, 0.2, -3.0, 120.0, 129.0),             # gap hop
    (0.5, 100.0, -0.2, -0.5, 0.1, 247.0, 85.0),           # whole chamber inward
]


@pytest.mark.parametrize("case", CASES)
def test_transport_matches_closed_form_circle(orc, case):
    *p, x0, x1 = case
    ok, out, _, _ = orc.transport(p, np.eye(5)[np.triu_indices(5)], x0, x1, bz=0.5)
    assert ok
    ref = closed_form(np.array(p), x0, x1, 0.5)
    np.testing.assert_allclose(out, ref, rtol=0, atol=1e-9 * max(1.0, abs(x1 - x0)))


@pytest.mark.parametrize("case", CASES[:3])
def test_transport_matches_rk4(orc, case):
    *p, x0, x1 = case
    ok, out, _, _ = orc.transport(p, np.zeros(15), x0, x1, bz=0.5)
    assert ok
    np.testing.assert_allclose(out, rk4(np.array(p), x0, x1, 0.5), rtol=0, atol=1e-10)


def test_transport_reversible_and_composes(orc):
    rng = np.random.default_rng(7)
    for _ in range(50):
        p = np.array([rng.normal(0, 5), rng.normal(0, 50), rng.uniform(-0.6, 0.6),
                      rng.uniform(-1, 1), rng.uniform(-10, 10)])
        A = rng.normal(size=(5, 5)); Cm = A @ A.T + np.eye(5)
        cv = Cm[np.triu_indices(5)]
        x0, x1, x2 = 100.0, 100.0 + rng.uniform(-3, 3), 100.0 + rng.uniform(-3, 3)
        ok1, p1, c1, _ = orc.transport(p, cv, x0, x1)
        ok2, p2, c2, _ = orc.transport(p1, c1, x1, x0)
        assert ok1 and ok2
        np.testing.assert_allclose(p2, p, atol=1e-11)
        np.testing.assert_allclose(c2, cv, rtol=1e-9, atol=1e-9)
        ok3, p3, _, _ = orc.transport(p1, c1, x1, x2)
        ok4, p4, _, _ = orc.transport(p, cv, x0, x2)
        assert ok3 and ok4
        np.testing.assert_allclose(p3, p4, atol=1e-10)


def test_transport_zero_field_is_straight_line(orc):
    p = np.array([1.0, 2.0, 0.4, -0.7, 3.0])
    ok, out, _, _ = orc.transport(p, np.zeros(15), 90.0, 97.5, bz=0.0)
    assert ok
    c = np.sqrt(1 - 0.16)
    np.testing.assert_allclose(out, [1.0 + 7.5 * 0.4 / c, 2.0 - 0.7 * 7.5 / c, 0.4, -0.7, 3.0], atol=1e-12)


def test_transport_jacobian_and_covariance(orc):
    rng = np.random.default_rng(3)
    iu = np.triu_indices(5)
    for _ in range(20):
        p = np.array([rng.normal(), rng.normal(), rng.uniform(-0.7, 0.7), rng.uniform(-1, 1),
                      rng.uniform(-8, 8)])
        x0, x1 = 110.0, 110.0 + rng.uniform(-9, 9)
        A = rng.normal(size=(5, 5)); Cm = A @ A.T
        ok, _, cout, F = orc.transport(p, Cm[iu], x0, x1)
        assert ok
        J = np.zeros((5, 5))
        for j in range(5):
            h = 1e-6
            dp = np.zeros(5); dp[j] = h
            _, a, _, _ = orc.transport(p + dp, np.zeros(15), x0, x1)
            _, b, _, _ = orc.transport(p - dp, np.zeros(15), x0, x1)
            J[:, j] = (a - b) / (2 * h)
        np.testing.assert_allclose(F, J, atol=2e-7, rtol=1e-6)
        np.testing.assert_allclose(cout, (F @ Cm @ F.T)[iu], rtol=1e-12, atol=1e-10)


def test_transport_refuses_beyond_sin_max(orc):
    p = np.array([0.0, 0.0, 0.95, 0.0, -10.0])
    kap = -C_LIGHT * 0.5 * -10.0
    x1 = 100.0 + (0.995 - 0.95) / kap
    ok, out, _, _ = orc.transport(p, np.zeros(15), 100.0, x1)
    assert not ok


def test_fp32_transport_close_to_fp64(orc):
    p = [1.0, 5.0, 0.1, 0.3, 1.0]
    ok, a, _, _ = orc.transport(p, np.zeros(15), 100.0, 101.0253, precision=32)
    ok2, b, _, _ = orc.transport(p, np.zeros(15), 100.0, 101.0253, precision=64)
    assert ok and ok2
    np.testing.assert_allclose(a, b, rtol=1e-5, atol=1e-5)
