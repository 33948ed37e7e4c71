"""Pins for the oracle's full force pass: reduction to the direct sum,
coverage of every body pair, the error bound behind the acceptance test,
the paper's accuracy statement, conservation, convergence in p and
determinism."""
import hashlib
import json
import os
import subprocess
import sys

import numpy as np
import pytest

import oracle
from paper_2012_02207_amd import workloads as W

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def relerr(a, ref):
    return np.linalg.norm(a - ref, axis=1) / np.linalg.norm(ref, axis=1)


@pytest.mark.parametrize("n", [1, 2, 5, 33, 64])
def test_single_leaf_fmm_is_direct_sum_bit_for_bit(n):
    """With n_leaf >= N the root is a leaf: the pass is P2P(root, root), the
    plain definition summed in sorted order."""
    rng = np.random.default_rng(n)
    pos = rng.normal(size=(n, 3))
    m = rng.uniform(0.1, 1, n)
    o = oracle.Oracle()
    acc, pot = o.run(pos, m, p=4, err_tol=1e-6, n_leaf=64)
    perm = o.get("perm")
    a2, p2 = oracle.direct(pos[perm], m[perm], compensated=False)
    inv = np.argsort(perm)
    assert np.array_equal(acc, a2[inv]) and np.array_equal(pot, p2[inv])
    if n == 1:
        assert np.all(acc == 0) and pot[0] == 0


def test_single_leaf_scalar_force_is_exact_sum():
    rng = np.random.default_rng(3)
    n = 50
    pos = rng.normal(size=(n, 3))
    m = rng.uniform(0.1, 1, n)
    o = oracle.Oracle()
    o.run(pos, m, n_leaf=64, stage="estimate")
    sp, sm = pos[o.get("perm")], m[o.get("perm")]
    f = o.get("f_part")
    for i in range(n):
        s = 0.0
        for j in range(n):
            if j != i:
                d = sp[j] - sp[i]
                s = s + sm[j] / ((d[0] * d[0] + d[1] * d[1]) + d[2] * d[2])
        assert f[i] == s


def _descendant_bodies(o):
    b, e = o.get("cell_begin"), o.get("cell_end")
    return [np.arange(b[c], e[c]) for c in range(o.ncell)]


@pytest.mark.parametrize("n,n_leaf,mac", [(300, 1, "error"), (300, 4, "geometric"),
                                           (500, 8, "error"), (200, 3, "error")])
def test_every_body_pair_covered_exactly_once(n, n_leaf, mac):
    """Each ordered body pair (i, j), i != j, is handled by exactly one M2L
    or P2P entry (the dual-tree walk, section 2.1)."""
    pos, _, m = W.plummer(n, n + n_leaf)
    o = oracle.Oracle()
    o.run(pos, m, p=5, err_tol=1e-4, n_leaf=n_leaf, mac=mac, theta=0.7, stage="walk")
    bodies = _descendant_bodies(o)
    cover = np.zeros((n, n), np.int32)
    for sink, src in np.vstack([o.get("m2l"), o.get("p2p")]):
        cover[np.ix_(bodies[sink], bodies[src])] += 1
    # the diagonal is reached once, through the leaf's own P2P(A, A) entry
    assert np.all(cover == 1)
    assert len(o.get("m2l")) > 0
    # the estimate walk covers every pair exactly once too
    cover[:] = 0
    for sink, src in np.vstack([o.get("est_far"), o.get("est_near")]):
        cover[np.ix_(bodies[sink], bodies[src])] += 1
    assert np.all(cover == 1)


def test_pk_bounded_by_mass_times_radius_power():
    """P_k <= M r^k (each body contributes m a^k with a <= r): the bound that
    makes E_{A->B} <= 8 max/(rA+rB) theta^p (section 2.3)."""
    pos, _, m = W.plummer(4096, 5)
    o = oracle.Oracle()
    o.run(pos, m, p=10, err_tol=1e-7, n_leaf=32, stage="upward")
    P, M, r = o.get("pk"), o.get("cell_mass"), o.get("cell_rad")
    bound = M[:, None] * r[:, None] ** np.arange(11)
    assert np.all(P <= bound * (1 + 1e-12) + 1e-300)
    np.testing.assert_allclose(P[:, 0], M, rtol=1e-15)


def test_accepted_pairs_satisfy_the_mac():
    pos, _, m = W.plummer(4096, 6)
    p, eps = 6, 1e-6
    o = oracle.Oracle()
    o.run(pos, m, p=p, err_tol=eps, n_leaf=64, stage="walk")
    P, r, com, f = o.get("pk"), o.get("cell_rad"), o.get("cell_com"), o.get("fmin")
    from math import comb
    for B, A in o.get("m2l")[::7]:
        R = np.linalg.norm(com[B] - com[A])
        assert r[A] + r[B] < R
        if r[A] + r[B] == 0:        # two point-like cells: expansion exact, E = 0
            continue
        E = 8 * max(r[A], r[B]) / (r[A] + r[B]) * sum(
            comb(p, k) * P[A, k] * r[B] ** (p - k) for k in range(p + 1)) / R ** p
        assert E / R ** 2 < eps * f[B] * (1 + 1e-12)


def test_scalar_force_estimate_is_close_to_exact():
    pos, _, m = W.plummer(3000, 8)
    o = oracle.Oracle()
    o.run(pos, m, n_leaf=32, stage="estimate")
    sp, sm = pos[o.get("perm")], m[o.get("perm")]
    f = o.get("f_part")
    d = sp[:, None, :] - sp[None, :, :]
    r2 = (d * d).sum(2)
    np.fill_diagonal(r2, np.inf)
    exact = (sm[None, :] / r2).sum(1)
    assert np.all(f > 0)
    rel = np.abs(f / exact - 1)
    # theta = 1 monopole estimate: a "quick but reasonable" approximation (section 2.3)
    assert np.median(rel) < 0.15 and np.abs(np.log(f / exact)).max() < np.log(5.0)
    fmin, b, e = o.get("fmin"), o.get("cell_begin"), o.get("cell_end")
    for c in range(o.ncell):
        assert fmin[c] == f[b[c]:e[c]].min()


def test_median_error_below_tolerance_config_4k():
    """section 4.1: the median relative force error is below epsilon
    (Plummer N = 4096, p = 6, epsilon = 1e-6)."""
    cfg = W.CONFIGS["plummer_4k"]
    pos, _, m = W.plummer(cfg["n"], cfg["seed"])
    o = oracle.Oracle()
    acc, pot = o.run(pos, m, p=cfg["p"], err_tol=cfg["err_tol"], n_leaf=64)
    ad, pd = oracle.direct(pos, m)
    err = relerr(acc, ad)
    assert np.median(err) < cfg["err_tol"]
    assert np.median(np.abs(pot - pd) / np.abs(pd)) < cfg["err_tol"]


def test_median_error_below_tolerance_p10():
    pos, _, m = W.plummer(20000, 77)
    o = oracle.Oracle()
    acc, _ = o.run(pos, m, p=10, err_tol=1e-7, n_leaf=64)
    sinks = np.random.default_rng(1).choice(20000, 2000, replace=False)
    ad, _ = oracle.direct(pos, m, sinks=sinks)
    assert np.median(relerr(acc[sinks], ad)) < 1e-7


def test_error_falls_geometrically_with_p_under_geometric_mac():
    pos, _, m = W.plummer(3000, 9)
    ad, _ = oracle.direct(pos, m)
    med = []
    for p in (2, 4, 6, 8, 10):
        o = oracle.Oracle()
        acc, _ = o.run(pos, m, p=p, n_leaf=16, mac="geometric", theta=0.5)
        med.append(np.median(relerr(acc, ad)))
    assert all(b < a / 4 for a, b in zip(med, med[1:])), med


def test_fmm_conserves_momentum():
    """Mutual acceptance with total-degree truncation makes every approximated
    pair interaction antisymmetric (section 2.3), so sum m_i a_i = 0."""
    pos, _, m = W.plummer(4096, 10)
    m = m * np.random.default_rng(0).uniform(0.2, 2, 4096)
    o = oracle.Oracle()
    acc, _ = o.run(pos, m, p=6, err_tol=1e-5, n_leaf=16)
    scale = (m[:, None] * np.abs(acc)).sum()
    assert np.abs((m[:, None] * acc).sum(0)).max() < 1e-13 * scale


def test_softened_pass_matches_softened_direct():
    pos, _, m = W.plummer(2000, 13)
    o = oracle.Oracle()
    acc, _ = o.run(pos, m, eps_soft=1.0 / 2000, p=8, err_tol=1e-7, n_leaf=32)
    ad, _ = oracle.direct(pos, m, eps_soft=1.0 / 2000)
    assert np.median(relerr(acc, ad)) < 1e-6


def _digest(*arrs):
    h = hashlib.sha256()
    for a in arrs:
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def test_deterministic_and_thread_count_independent():
    """Run-to-run identical results (cf. section 4.4 on reproducibility),
    independent of the number of OpenMP threads."""
    code = (
        "import sys, hashlib, numpy as np; sys.path.insert(0, %r);"
        "import oracle; from paper_2012_02207_amd import workloads as W;"
        "pos,_,m=W.plummer(3000, 14); o=oracle.Oracle();"
        "a,p=o.run(pos,m,p=6,err_tol=1e-6,n_leaf=16);"
        "h=hashlib.sha256(); [h.update(np.ascontiguousarray(x).tobytes()) for x in"
        " (a,p,o.get('m2l'),o.get('p2p'),o.get('f_part'))]; print(h.hexdigest())"
    ) % os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    outs = set()
    for t in ("1", "3", "8"):
        env = dict(os.environ, OMP_NUM_THREADS=t)
        outs.add(subprocess.check_output([sys.executable, "-c", code], env=env).strip())
    assert len(outs) == 1


def test_eval_mask_gives_same_bits():
    pos, _, m = W.plummer(3000, 15)
    o = oracle.Oracle()
    acc, pot = o.run(pos, m, p=6, err_tol=1e-6, n_leaf=32)
    mask = np.zeros(3000, np.uint8)
    mask[::97] = 1
    a2, p2 = o.run(pos, m, p=6, err_tol=1e-6, n_leaf=32, eval_mask=mask)
    sel = mask.astype(bool)
    assert np.array_equal(acc[sel], a2[sel]) and np.array_equal(pot[sel], p2[sel])
