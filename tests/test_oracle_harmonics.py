"""Pins for the oracle's expansion operators (solid harmonics, P2M, M2M, M2L,
L2L, L2P, swap matrices).  Each test checks the oracle against something it
does not compute itself: the paper's explicit low-order harmonics, the
Laplace equation, the addition theorem, exact invariants, finite differences
or a direct sum."""
import json
import math
import os

import numpy as np
import pytest

import oracle

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def cidx(n, m):
    return n * (n + 1) // 2 + m


def test_low_order_span_matches_paper_list():
    """section 2.2: the order <= 2 harmonics are combinations of the listed
    polynomials (the paper's list is unnormalised)."""
    RNG = np.random.default_rng(33308)
    pts = RNG.normal(size=(40, 3))
    g = GOLD["harmonics_order_le_2"]
    for n, key in ((0, "order0"), (1, "order1"), (2, "order2")):
        ref = np.array([[eval(e, {}, dict(x=x, y=y, z=z)) if e != "1" else 1.0 for e in g[key]]
                        for x, y, z in pts])
        for m in range(n + 1):
            vals = np.array([oracle.regular(2, q)[cidx(n, m)] for q in pts])
            for part in (vals.real, vals.imag):
                if np.abs(part).max() == 0:
                    continue
                coef, *_ = np.linalg.lstsq(ref, part, rcond=None)
                res = np.abs(ref @ coef - part).max() / np.abs(part).max()
                assert res < 1e-13, (n, m, res)
        # and the (2n+1) real functions span the whole listed space
        cols = []
        for m in range(n + 1):
            vals = np.array([oracle.regular(2, q)[cidx(n, m)] for q in pts])
            cols.append(vals.real)
            if m:
                cols.append(vals.imag)
        assert np.linalg.matrix_rank(np.array(cols).T, tol=1e-10) == 2 * n + 1


@pytest.mark.parametrize("n", [2, 5, 9])
def test_regular_harmonics_solve_laplace(n):
    RNG = np.random.default_rng(14044)
    p = n
    x0 = RNG.normal(size=3)
    h = 1e-3
    lap = 0
    for d in range(3):
        e = np.zeros(3)
        e[d] = h
        f = [oracle.regular(p, x0 + k * e)[cidx(n, 0):cidx(n, n) + 1] for k in (-2, -1, 0, 1, 2)]
        lap = lap + (-f[0] + 16 * f[1] - 30 * f[2] + 16 * f[3] - f[4]) / (12 * h * h)
    scale = np.abs(oracle.regular(p, x0)[cidx(n, 0):cidx(n, n) + 1]).max() / np.dot(x0, x0)
    assert np.abs(lap).max() < 1e-6 * scale * n * n


def _full(coef, p):
    """dict (n, m) for all m from the m >= 0 storage"""
    out = {}
    for n in range(p + 1):
        for m in range(-n, n + 1):
            c = coef[cidx(n, abs(m))]
            out[(n, m)] = c if m >= 0 else (-1) ** m * np.conj(c)
    return out


def test_addition_theorem_inverse_distance():
    """1/|x - y| = sum conj(Y_n^m(y)) T_n^m(x): the expansion the multipole
    moments rest on (section 2.2)."""
    RNG = np.random.default_rng(34291)
    p = 30
    for _ in range(5):
        x = RNG.normal(size=3)
        x *= 2.0 / np.linalg.norm(x)
        y = RNG.normal(size=3)
        y *= 0.3 / np.linalg.norm(y)
        Y = _full(oracle.regular(p, y), p)
        T = _full(oracle.irregular(p, x), p)
        s = sum(np.conj(Y[k]) * T[k] for k in Y)
        assert abs(s.imag) < 1e-15
        assert abs(s.real - 1 / np.linalg.norm(x - y)) < 2e-15


def test_pk_of_single_body_is_m_times_a_to_n():
    """P_n (section 2.3 equation) of one body of mass m at distance a is m a^n."""
    RNG = np.random.default_rng(85644)
    p = 20
    for _ in range(5):
        d = RNG.normal(size=3)
        a = RNG.uniform(0.1, 3.0)
        d *= a / np.linalg.norm(d)
        m = RNG.uniform(0.1, 2.0)
        P = oracle.pk(p, oracle.p2m(p, d[None, :], [m], [0, 0, 0]))
        ref = m * a ** np.arange(p + 1)
        np.testing.assert_allclose(P, ref, rtol=5e-14)


def test_pk_rotation_invariant():
    RNG = np.random.default_rng(67217)
    p = 12
    pts = RNG.normal(size=(30, 3)) * 0.5
    ms = RNG.uniform(0.1, 1.0, 30)
    P0 = oracle.pk(p, oracle.p2m(p, pts, ms, [0, 0, 0]))
    for _ in range(3):
        Q, _ = np.linalg.qr(RNG.normal(size=(3, 3)))
        P1 = oracle.pk(p, oracle.p2m(p, pts @ Q.T, ms, [0, 0, 0]))
        np.testing.assert_allclose(P1, P0, rtol=1e-12)


def _order_scaled_diff(A, B, p, scale):
    """max over coefficients of |A - B| relative to scale^n of the order"""
    err = 0.0
    for n in range(p + 1):
        sl = slice(cidx(n, 0), cidx(n, n) + 1)
        err = max(err, np.abs(A[sl] - B[sl]).max() / scale ** n)
    return err


def test_m2m_is_exact():
    """Shifting children's moments (M2M) reproduces the parent's P2M exactly
    up to rounding: no truncation for n <= p."""
    RNG = np.random.default_rng(40094)
    p = 14
    pts = RNG.normal(size=(60, 3)) * 0.4
    ms = RNG.uniform(0.1, 1.0, 60)
    parent = np.array([0.05, -0.02, 0.03])
    direct = oracle.p2m(p, pts, ms, parent)
    tot = np.zeros_like(direct)
    for grp in np.array_split(np.arange(60), 4):
        c = pts[grp].mean(0) + RNG.normal(size=3) * 0.1
        Mc = oracle.p2m(p, pts[grp], ms[grp], c)
        tot += oracle.m2m(p, Mc, c - parent)
    assert _order_scaled_diff(tot, direct, p, 1.5) < 1e-13 * ms.sum()


@pytest.mark.parametrize("p", [3, 6, 10, 12, 20])
def test_rotated_m2l_equals_direct_m2l(p):
    """The rotation-accelerated M2L (section 2.4) equals the O(p^4) operator."""
    RNG = np.random.default_rng(20813)
    pts = RNG.normal(size=(25, 3)) * 0.3
    ms = RNG.uniform(0.1, 1.0, 25)
    M = oracle.p2m(p, pts, ms, [0, 0, 0])
    dirs = [RNG.normal(size=3) for _ in range(4)] + [np.array([0, 0, 1.0]), np.array([0, 0, -1.0]),
                                                     np.array([1.0, 0, 0]), np.array([0, -1.0, 0])]
    for d in dirs:
        R = 2.5 * d / np.linalg.norm(d)
        A = oracle.m2l_direct(p, M, R)
        B = oracle.m2l_rotated(p, M, R)
        # compare in the rotation-invariant norm: the field at distance rho
        # from the sink centre, order by order (L_n^m / sqrt((n-m)!(n+m)!) rho^n)
        rho = 0.5 * 2.5
        err = tot = 0.0
        for n in range(p + 1):
            w = np.array([rho ** n / math.sqrt(math.factorial(n - m) * math.factorial(n + m))
                          for m in range(n + 1)])
            sl = slice(cidx(n, 0), cidx(n, n) + 1)
            err += np.abs((A[sl] - B[sl]) * w).max()
            tot += np.abs(A[sl] * w).max()
        assert err < 1e-14 * tot, (p, d, err / tot)


def test_m2l_l2p_converges_to_direct_sum():
    """Far field of a cluster through M2L + L2P approaches the direct sum
    geometrically in p (truncation error ~ (2 rho / R)^(p+1))."""
    RNG = np.random.default_rng(64312)
    src = RNG.normal(size=(40, 3))
    src *= (0.5 * RNG.uniform(0, 1, 40) ** (1 / 3) / np.linalg.norm(src, axis=1))[:, None]
    ms = RNG.uniform(0.1, 1.0, 40)
    zB = np.array([1.6, 1.2, -1.1])
    X = np.array([0.2, -0.3, 0.25])
    x = zB + X
    d = x - src
    r = np.linalg.norm(d, axis=1)
    phi_ref = -(ms / r).sum()
    acc_ref = -(ms[:, None] * d / r[:, None] ** 3).sum(0)
    errs = []
    for p in (2, 4, 6, 8, 10, 12, 16, 20):
        L = oracle.m2l_rotated(p, oracle.p2m(p, src, ms, [0, 0, 0]), zB)
        phi, acc = oracle.l2p(p, L, X)
        errs.append(max(abs(phi - phi_ref) / abs(phi_ref),
                        np.linalg.norm(acc - acc_ref) / np.linalg.norm(acc_ref)))
    rho = 0.5 + np.linalg.norm(X)
    bound = [3 * (rho / np.linalg.norm(zB)) ** (p + 1) / (1 - rho / np.linalg.norm(zB)) * 10
             for p in (2, 4, 6, 8, 10, 12, 16, 20)]
    assert all(e < b + 1e-14 for e, b in zip(errs, bound)), (errs, bound)
    assert errs[-1] < 1e-8 and errs[0] > 1e6 * errs[-1]


def test_l2l_is_exact_shift():
    RNG = np.random.default_rng(2307)
    p = 10
    src = RNG.normal(size=(30, 3)) * 0.3
    ms = RNG.uniform(0.1, 1.0, 30)
    L = oracle.m2l_rotated(p, oracle.p2m(p, src, ms, [0, 0, 0]), np.array([2.0, -1.0, 1.5]))
    d = np.array([0.1, 0.05, -0.12])
    Lc = oracle.l2l(p, L, d)
    for _ in range(4):
        X = RNG.normal(size=3) * 0.1
        phi0, a0 = oracle.l2p(p, L, d + X)
        phi1, a1 = oracle.l2p(p, Lc, X)
        assert abs(phi1 - phi0) < 1e-15 * abs(phi0) * 4
        assert np.linalg.norm(a1 - a0) < 1e-14 * np.linalg.norm(a0)


def test_l2p_gradient_matches_finite_differences():
    RNG = np.random.default_rng(31585)
    p = 8
    src = RNG.normal(size=(20, 3)) * 0.3
    ms = RNG.uniform(0.1, 1.0, 20)
    L = oracle.m2l_rotated(p, oracle.p2m(p, src, ms, [0, 0, 0]), np.array([-1.5, 2.0, 0.7]))
    X = np.array([0.1, -0.05, 0.08])
    _, acc = oracle.l2p(p, L, X)
    h = 1e-4
    g = np.zeros(3)
    for d in range(3):
        e = np.zeros(3)
        e[d] = h
        f = [oracle.l2p(p, L, X + k * e)[0] for k in (-2, -1, 1, 2)]
        g[d] = (f[0] - 8 * f[1] + 8 * f[2] - f[3]) / (12 * h)
    np.testing.assert_allclose(acc, -g, rtol=1e-9)


def _real_basis(p, x, n):
    c = oracle.regular(p, x)
    v = [c[cidx(n, 0)].real]
    for m in range(1, n + 1):
        v += [c[cidx(n, m)].real, c[cidx(n, m)].imag]
    return np.array(v)


@pytest.mark.parametrize("n", [1, 2, 5, 10, 16, 24, 30])
def test_swap_matrix_maps_harmonics_under_x_z_exchange(n):
    """section 2.4: the swap matrix re-expresses the harmonics after x <-> z."""
    RNG = np.random.default_rng(10697)
    W = oracle.swap_table(n)
    for _ in range(3):
        x = RNG.normal(size=3)
        x /= np.linalg.norm(x)
        u = _real_basis(n, x, n)
        us = _real_basis(n, x[::-1].copy(), n)
        assert np.abs(W @ u - us).max() < 1e-13 * np.abs(W).max() * np.abs(u).max() * (2 * n + 1)


def test_swap_matrices_are_involutions_and_dyadic():
    RNG = np.random.default_rng(82421)
    for n in range(0, 31):
        W = oracle.swap_table(n)
        d = 2 * n + 1
        I = W @ W
        assert np.abs(I - np.eye(d)).max() < 1e-15 * np.abs(W).max() ** 2 * d
        if n <= 24:   # numerators fit 53 bits: entries are exact k / 2^n
            k = W * 2.0 ** n
            assert np.all(k == np.round(k))
            if n in (3, 8, 13, 24):   # exact rational check of W^2 = I
                from fractions import Fraction
                Wf = [[Fraction(float(v)) for v in row] for row in W]
                for i in range(d):
                    for j in range(d):
                        assert sum(Wf[i][t] * Wf[t][j] for t in range(d)) == (i == j)


def test_factorial_table_correctly_rounded():
    RNG = np.random.default_rng(82915)
    f = oracle.factorials()
    for n in range(62):
        assert f[n] == float(math.factorial(n))
