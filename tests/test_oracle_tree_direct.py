"""Pins for the oracle's tree (keys, sort, cells, centres, radii) and its
direct summation, against brute force, closed forms and invariants."""
from fractions import Fraction

import numpy as np
import pytest

import oracle
from paper_2012_02207_amd import workloads as W


def _deinterleave(key):
    q = [0, 0, 0]
    for b in range(21):
        dgt = (int(key) >> (3 * b)) & 7
        q[0] |= ((dgt >> 2) & 1) << b
        q[1] |= ((dgt >> 1) & 1) << b
        q[2] |= (dgt & 1) << b
    return q


def _tree(pos, mass, n_leaf=8):
    o = oracle.Oracle()
    o.run(pos, mass, n_leaf=n_leaf, stage="tree")
    return o


@pytest.mark.parametrize("seed", [1, 2])
def test_keys_contain_their_bodies_and_are_stably_sorted(seed):
    pos, mass = W.uniform_cube(3000, seed)
    pos[::7] = np.round(pos[::7], 2)          # many exact ties on grid lines
    pos[5] = pos[9]                           # exact duplicate
    o = _tree(pos, mass)
    keys, perm = o.get("keys"), o.get("perm")
    lo, L, s = o.get("rootbox")[:3], o.get("rootbox")[3], o.get("rootbox")[4]
    np.testing.assert_array_equal(lo, pos.min(0))
    assert L == (pos.max(0) - pos.min(0)).max()
    assert np.all(np.diff(keys.astype(object)) >= 0)
    assert np.array_equal(np.sort(perm), np.arange(len(perm)))
    same = keys[1:] == keys[:-1]
    assert np.all(perm[1:][same] > perm[:-1][same])      # stable: ties keep input order
    np.testing.assert_array_equal(o.get("sorted_pos"), pos[perm])
    # each body lies in the cube its key names (exact rationals, one-cell slack for rounding)
    for i in range(0, len(keys), 37):
        q = _deinterleave(keys[i])
        x = pos[perm[i]]
        for d in range(3):
            t = (Fraction(float(x[d])) - Fraction(float(lo[d]))) / Fraction(float(L)) * 2 ** 21
            assert q[d] <= t + Fraction(1, 10 ** 9)
            assert t < q[d] + 1 + Fraction(1, 10 ** 9) or q[d] == 2 ** 21 - 1


def test_cells_partition_bodies_breadth_first():
    pos, _, mass = W.plummer(5000, 7)
    n_leaf = 16
    o = _tree(pos, mass, n_leaf)
    keys = o.get("keys").astype(object)
    lev, b, e = o.get("cell_level"), o.get("cell_begin"), o.get("cell_end")
    par, c0, nch = o.get("cell_parent"), o.get("cell_child0"), o.get("cell_nchild")
    nc = len(lev)
    assert (b[0], e[0], lev[0], par[0]) == (0, 5000, 0, -1)
    order = list(zip(lev, b))
    assert order == sorted(order)                          # ids: by level, then key order
    covered = np.zeros(5000, int)
    for c in range(nc):
        pre = {k >> (63 - 3 * int(lev[c])) for k in keys[b[c]:e[c]]} if lev[c] else {0}
        assert len(pre) == 1                               # one key prefix per cell
        cnt = e[c] - b[c]
        if nch[c] == 0:
            covered[b[c]:e[c]] += 1
            assert cnt <= n_leaf or lev[c] == 21
            continue
        assert cnt > n_leaf and lev[c] < 21
        kids = range(c0[c], c0[c] + nch[c])
        assert [b[k] for k in kids][0] == b[c] and e[c0[c] + nch[c] - 1] == e[c]
        for k0, k1 in zip(kids, list(kids)[1:]):
            assert e[k0] == b[k1]
            # siblings differ in the octant digit (maximal runs)
            d0 = (keys[b[k0]] >> (60 - 3 * int(lev[c]))) & 7
            d1 = (keys[b[k1]] >> (60 - 3 * int(lev[c]))) & 7
            assert d0 < d1
        for k in kids:
            assert par[k] == c and lev[k] == lev[c] + 1
    assert np.all(covered == 1)


def test_duplicate_bodies_stop_at_level_21():
    pos = np.zeros((40, 3))
    pos[:, 0] = 0.5
    pos[-1] = [1.0, 1.0, 1.0]
    o = _tree(pos, np.full(40, 1 / 40), n_leaf=4)
    lev, b, e, nch = o.get("cell_level"), o.get("cell_begin"), o.get("cell_end"), o.get("cell_nchild")
    big = [(lev[c], e[c] - b[c]) for c in range(len(lev)) if nch[c] == 0 and e[c] - b[c] > 4]
    assert big == [(21, 39)]


def test_centres_and_radii():
    pos, _, mass = W.plummer(3000, 3)
    mass = mass * np.random.default_rng(0).uniform(0.5, 1.5, 3000)
    o = _tree(pos, mass, 16)
    b, e = o.get("cell_begin"), o.get("cell_end")
    com, rad, M = o.get("cell_com"), o.get("cell_rad"), o.get("cell_mass")
    sp = o.get("sorted_pos")
    sm = mass[o.get("perm")]
    for c in range(0, len(b), 3):
        x = sp[b[c]:e[c]].astype(np.longdouble)
        m = sm[b[c]:e[c]].astype(np.longdouble)
        ref = (m[:, None] * x).sum(0) / m.sum()
        assert np.abs(com[c] - ref).max() <= 1e-15 * max(1.0, np.abs(ref).max())
        assert abs(M[c] - float(m.sum())) <= 1e-15 * float(m.sum())
        d = np.sqrt(((sp[b[c]:e[c]] - com[c]) ** 2).sum(1))
        assert rad[c] >= d.max() * (1 - 1e-15) and np.isclose(rad[c], d.max(), rtol=1e-15)


def test_massless_cell_centre_is_box_centre():
    pos, _ = W.uniform_cube(200, 4)
    mass = np.zeros(200)
    o = _tree(pos, mass, 16)
    com = o.get("cell_com")
    lo, L = o.get("rootbox")[:3], o.get("rootbox")[3]
    np.testing.assert_allclose(com[0], lo + 0.5 * L)


# ---------------------------------------------------------------- direct sum
def test_direct_two_body_closed_form():
    pos = np.array([[0.1, -0.2, 0.3], [1.1, 0.6, -0.3]])
    m = np.array([0.7, 1.9])
    for eps in (0.0, 0.3):
        acc, pot = oracle.direct(pos, m, eps_soft=eps)
        d = pos[1] - pos[0]
        r2 = d @ d + eps * eps
        np.testing.assert_allclose(acc[0], m[1] * d / r2 ** 1.5, rtol=1e-15)
        np.testing.assert_allclose(acc[1], -m[0] * d / r2 ** 1.5, rtol=1e-15)
        np.testing.assert_allclose(pot, [-m[1] / np.sqrt(r2), -m[0] / np.sqrt(r2)], rtol=1e-15)


def test_direct_conserves_momentum_and_angular_momentum():
    pos, _, mass = W.plummer(2000, 11)
    acc, _ = oracle.direct(pos, mass)
    scale = (mass[:, None] * np.abs(acc)).sum()
    assert np.abs((mass[:, None] * acc).sum(0)).max() < 1e-14 * scale
    tq = (mass[:, None] * np.cross(pos, acc)).sum(0)
    assert np.abs(tq).max() < 1e-13 * scale * np.abs(pos).max()


def test_direct_brute_force_long_double():
    rng = np.random.default_rng(5)
    for n in (2, 3, 17, 64):
        pos = rng.normal(size=(n, 3))
        m = rng.uniform(0.1, 1, n)
        acc, pot = oracle.direct(pos, m, compensated=True)
        P = pos.astype(np.longdouble)
        for i in range(n):
            d = P - P[i]
            r = np.sqrt((d * d).sum(1))
            r[i] = 1
            w = m / r ** 3
            w[i] = 0
            ref = (w[:, None] * d).sum(0)
            mag = (np.abs(w[:, None] * d)).sum(0).astype(float)   # rounding of each term
            # ~11 roundings per term (r2, sqrt, divide, four products): bound 11 * 2^-53
            assert np.all(np.abs(acc[i] - ref.astype(float)) <= 1.3e-15 * mag)
            pr = -(np.where(np.arange(n) == i, 0, m / r)).sum()
            assert abs(pot[i] - float(pr)) <= 1.3e-15 * abs(float(pr))


def test_direct_subset_and_coincident_bodies():
    pos, _, mass = W.plummer(500, 12)
    pos[10] = pos[11]
    acc, pot = oracle.direct(pos, mass, compensated=False)
    assert np.all(np.isfinite(acc)) and np.all(np.isfinite(pot))
    sinks = np.array([3, 10, 499])
    a2, p2 = oracle.direct(pos, mass, sinks=sinks, compensated=True)
    np.testing.assert_allclose(a2, acc[sinks], rtol=1e-13)
    np.testing.assert_allclose(p2, pot[sinks], rtol=1e-13)


def test_direct_matches_plummer_field():
    """Shell-averaged radial acceleration of a sampled (truncated) Plummer sphere
    equals the analytic -M(<r)/r^2 within sampling noise."""
    n = 20000
    pos, _, mass = W.plummer(n, 21)
    rng = np.random.default_rng(2)
    sinks = rng.choice(n, 1500, replace=False)
    acc, pot = oracle.direct(pos, mass, sinks=sinks)
    a = W.A_HENON
    r = np.linalg.norm(pos[sinks], axis=1)
    ar = (acc * pos[sinks]).sum(1) / r
    xmax = (100 / 101) ** 1.5
    ana = -(r / (r * r + a * a) ** 1.5) / xmax
    bins = np.quantile(r, [0.1, 0.3, 0.5, 0.7, 0.9])
    for lo, hi in zip(bins[:-1], bins[1:]):
        s = (r >= lo) & (r < hi)
        assert abs(ar[s].mean() / ana[s].mean() - 1) < 0.03
