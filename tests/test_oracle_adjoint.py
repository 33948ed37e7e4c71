"""Pins of the direct-sum gradients (oracle/adjoint.py) to things other than
their own formulas: the C direct sum, central finite differences of the force
sums, translation invariance, a two-body closed form, and finite differences
of a short leapfrog rollout."""
import numpy as np
import pytest

import oracle
from oracle import adjoint as A
from paper_2012_02207_amd import workloads as W


def _L(pos, mass, ga, gp, eps):
    a, pot = A.direct_forces(pos, mass, eps)
    return float((ga * a).sum() + (gp * pot).sum())


def test_direct_forces_match_c_direct_sum():
    pos, _, mass = W.plummer(700, 3)
    for eps in (0.0, 0.01):
        a, pot = A.direct_forces(pos, mass, eps)
        ac, pc = oracle.direct(pos, mass, eps_soft=eps)
        assert np.abs(a - ac).max() <= 1e-12 * np.abs(ac).max()
        assert np.abs(pot - pc).max() <= 1e-12 * np.abs(pc).max()


@pytest.mark.parametrize("eps", [0.0, 0.05])
def test_adjoint_matches_finite_differences(eps):
    rng = np.random.default_rng(5)
    n = 16
    pos = rng.normal(size=(n, 3))
    mass = rng.uniform(0.5, 1.5, n)
    ga = rng.normal(size=(n, 3))
    gp = rng.normal(size=n)
    gx, gm = A.direct_adjoint(pos, mass, ga, gp, eps)
    h = 1e-5
    fx = np.zeros_like(gx)
    for k in range(n):
        for d in range(3):
            e = np.zeros_like(pos)
            e[k, d] = h
            fx[k, d] = (_L(pos + e, mass, ga, gp, eps) - _L(pos - e, mass, ga, gp, eps)) / (2 * h)
    fm = np.zeros(n)
    for k in range(n):
        e = np.zeros(n)
        e[k] = h
        fm[k] = (_L(pos, mass + e, ga, gp, eps) - _L(pos, mass - e, ga, gp, eps)) / (2 * h)
    assert np.abs(gx - fx).max() <= 1e-7 * np.abs(fx).max()
    assert np.abs(gm - fm).max() <= 1e-7 * np.abs(fm).max()


def test_adjoint_translation_invariance():
    """L(a, pot) does not change when every body moves by the same vector."""
    pos, _, mass = W.plummer(300, 9)
    rng = np.random.default_rng(1)
    gx, _ = A.direct_adjoint(pos, mass, rng.normal(size=(300, 3)), rng.normal(size=300), 0.0)
    assert np.abs(gx.sum(axis=0)).max() <= 1e-10 * np.abs(gx).sum()


def test_adjoint_two_body_closed_form():
    """a_1 = m_2 u / |u|^3 with u = x_2 - x_1: dL/dx_2 for L = g . a_1 is
    m_2 (g / r^3 - 3 (u . g) u / r^5), and dL/dm_2 = g . u / r^3."""
    x = np.array([[0.1, -0.3, 0.2], [0.7, 0.4, -0.5]])
    m = np.array([0.3, 1.7])
    g = np.array([[0.2, -1.0, 0.5], [0.0, 0.0, 0.0]])
    gx, gm = A.direct_adjoint(x, m, g, None, 0.0)
    u = x[1] - x[0]
    r = np.linalg.norm(u)
    want = m[1] * (g[0] / r ** 3 - 3 * np.dot(u, g[0]) * u / r ** 5)
    assert np.allclose(gx[1], want, rtol=1e-14, atol=0)
    assert np.allclose(gx[0], -want, rtol=1e-14, atol=0)
    assert np.isclose(gm[1], np.dot(g[0], u) / r ** 3, rtol=1e-14)


def test_rollout_gradient_matches_finite_differences():
    rng = np.random.default_rng(8)
    n, dt, steps = 8, 1e-2, 5
    pos = rng.normal(size=(n, 3))
    vel = 0.3 * rng.normal(size=(n, 3))
    mass = rng.uniform(0.5, 1.5, n) / n
    target = pos + 0.1 * rng.normal(size=(n, 3))
    L, gx, gv, gm = A.rollout_gradient(pos, vel, mass, dt, steps, target, eps_soft=0.01)

    def loss(p, v, m):
        x, _ = A.leapfrog(p, v, m, dt, steps, eps_soft=0.01)
        return float(((x - target) ** 2).sum())
    assert np.isclose(L, loss(pos, vel, mass), rtol=1e-14)
    h = 1e-6
    for k, d in [(0, 0), (3, 2), (7, 1)]:
        e = np.zeros_like(pos)
        e[k, d] = h
        fx = (loss(pos + e, vel, mass) - loss(pos - e, vel, mass)) / (2 * h)
        fv = (loss(pos, vel + e, mass) - loss(pos, vel - e, mass)) / (2 * h)
        assert abs(gx[k, d] - fx) <= 1e-6 * max(1.0, abs(fx))
        assert abs(gv[k, d] - fv) <= 1e-6 * max(1.0, abs(fv))
    for k in (1, 5):
        e = np.zeros(n)
        e[k] = h
        fm = (loss(pos, vel, mass + e) - loss(pos, vel, mass - e)) / (2 * h)
        assert abs(gm[k] - fm) <= 1e-6 * max(1.0, abs(fm))


def test_jerk_matches_time_difference_of_forces():
    """j = da/dt along the motion: central difference of a(x + v t) in t."""
    rng = np.random.default_rng(12)
    n = 40
    pos = rng.normal(size=(n, 3))
    vel = rng.normal(size=(n, 3))
    mass = rng.uniform(0.5, 1.5, n)
    for eps in (0.0, 0.1):
        j = A.direct_jerk(pos, vel, mass, eps)
        h = 1e-5
        ap, _ = A.direct_forces(pos + h * vel, mass, eps)
        am, _ = A.direct_forces(pos - h * vel, mass, eps)
        fd = (ap - am) / (2 * h)
        assert np.abs(j - fd).max() <= 1e-7 * np.abs(fd).max()


def test_jerk_galilean_invariance_and_two_body():
    pos, vel, mass = W.plummer(200, 21)
    j1 = A.direct_jerk(pos, vel, mass)
    j2 = A.direct_jerk(pos, vel + np.array([0.3, -1.0, 2.0]), mass)
    assert np.abs(j1 - j2).max() <= 1e-12 * np.abs(j1).max()
    x = np.array([[0.0, 0.0, 0.0], [1.0, 2.0, -2.0]])
    v = np.array([[0.1, 0.0, 0.0], [0.0, 0.5, 0.0]])
    m = np.array([1.0, 2.0])
    u, w = x[1] - x[0], v[1] - v[0]
    r = np.linalg.norm(u)
    want = m[1] * (w / r ** 3 - 3 * np.dot(u, w) * u / r ** 5)
    assert np.allclose(A.direct_jerk(x, v, m)[0], want, rtol=1e-14, atol=0)
