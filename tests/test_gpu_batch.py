"""Batched evaluation of independent systems (fmm_forces_batch) on the GPU.

Each system of a batch must give exactly what it gives alone: the oracle run
on that system by itself fixes its root box, keys, order, cells, multipoles,
estimate and lists bit for bit (cell ids of the forest map to the system's
own breadth-first ids in order), and its forces to the FP64 parity bound
(median <= 1e-12, max <= 1e-9).  Beyond parity, a batch and single-system
calls of the GPU path perform the same arithmetic in the same order, so the
forces of every system agree bit for bit with fmm_forces on it alone, in FP64
and in mixed precision."""
import numpy as np
import pytest

import oracle
from paper_2012_02207_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def fmm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2012_02207_amd import fmm as F
    return F


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def _systems():
    """Uneven systems: a single body, two bodies, a tie-heavy cube, Plummer
    spheres of several sizes (one with a heavy central mass)."""
    out = []
    out.append((np.array([[0.3, -0.2, 0.1]]), np.array([1.0])))
    out.append((np.array([[0.0, 0.0, 0.0], [1.0, 0.5, -0.25]]), np.array([0.5, 0.25])))
    pos, mass = W.uniform_cube(600, 11)
    pos[::4] = np.round(pos[::4], 1)
    out.append((pos, mass))
    for n, seed in ((1500, 21), (257, 22), (3000, 23)):
        pos, _, mass = W.plummer(n, seed)
        out.append((pos, mass))
    pos, _, mass = W.kroupa_with_central(2048, 24)
    out.append((pos, mass))
    return out


def _concat(systems):
    off = np.zeros(len(systems) + 1, dtype=np.int64)
    off[1:] = np.cumsum([len(m) for _, m in systems])
    pos = np.concatenate([p for p, _ in systems])
    mass = np.concatenate([m for _, m in systems])
    return pos, mass, off


def _pairs(a):
    a = np.asarray(a, dtype=np.int64).reshape(-1, 2)
    return a[np.lexsort((a[:, 1], a[:, 0]))]


@pytest.mark.parametrize("p,eps,n_leaf", [(6, 1e-6, 16), (8, 1e-7, 64)])
def test_batch_matches_per_system_oracle(fmm, p, eps, n_leaf):
    systems = _systems()
    pos, mass, off = _concat(systems)
    print(f"[gpu] batch of {len(systems)} systems, N={len(mass)} p={p} eps={eps} n_leaf={n_leaf}",
          flush=True)
    f = fmm.FMM(p=p, err_tol=eps, n_leaf=n_leaf)
    acc, pot = f.forces_batch(_dev(pos), _dev(mass), off)
    acc, pot = acc.cpu().numpy(), pot.cpu().numpy()
    st = f.stats()
    assert st["nsys"] == len(systems)
    keys, perm = f.export("keys"), f.export("perm").astype(np.int64)
    cb, ce = f.export("cell_begin").astype(np.int64), f.export("cell_end").astype(np.int64)
    level, parent = f.export("cell_level"), f.export("cell_parent").astype(np.int64)
    nchild = f.export("cell_nchild")
    cmass, com, rad = f.export("cell_mass"), f.export("cell_com"), f.export("cell_rad")
    mult, pk, fpart, fmin = f.export("mult"), f.export("pk"), f.export("f_part"), f.export("fmin")
    rootbox = f.export("rootbox").reshape(-1, 5)
    lists = {k: f.export(k) for k in ("est_far", "est_near", "m2l", "p2p")}
    sys_of_cell = np.searchsorted(off, cb, side="right") - 1
    assert np.array_equal(sys_of_cell[:len(systems)], np.arange(len(systems)))  # roots first
    for s, (sp, sm) in enumerate(systems):
        b, e = off[s], off[s + 1]
        o = oracle.Oracle()
        oacc, opot = o.run(sp, sm, p=p, err_tol=eps, n_leaf=n_leaf)
        assert np.array_equal(rootbox[s], o.get("rootbox")), s
        assert np.array_equal(keys[b:e], o.get("keys")), s
        assert np.array_equal(perm[b:e] - b, o.get("perm")), s
        cells = np.nonzero(sys_of_cell == s)[0]          # forest ids of this system, in order
        local = np.full(len(cb), -1, dtype=np.int64)
        local[cells] = np.arange(len(cells))
        assert len(cells) == o.ncell, s
        assert np.array_equal(level[cells], o.get("cell_level")), s
        assert np.array_equal(cb[cells] - b, o.get("cell_begin")), s
        assert np.array_equal(ce[cells] - b, o.get("cell_end")), s
        par = parent[cells]
        par = np.where(par >= 0, local[np.maximum(par, 0)], -1)
        assert np.array_equal(par, o.get("cell_parent")), s
        assert np.array_equal(nchild[cells], o.get("cell_nchild")), s
        for name, g in (("cell_mass", cmass[cells]), ("cell_com", com[cells]),
                        ("cell_rad", rad[cells]), ("mult", mult[cells]), ("pk", pk[cells]),
                        ("fmin", fmin[cells]), ("f_part", fpart[b:e])):
            assert np.array_equal(g, o.get(name)), (s, name)
        for k, lst in lists.items():
            lst = np.asarray(lst, dtype=np.int64)
            mine = lst[np.isin(lst[:, 0], cells)]
            assert np.isin(mine[:, 1], cells).all(), (s, k)   # no pair crosses systems
            assert np.array_equal(_pairs(local[mine]), _pairs(o.get(k))), (s, k)
        if e - b > 1:
            rel = np.linalg.norm(acc[b:e] - oacc, axis=1) / np.linalg.norm(oacc, axis=1)
            relp = np.abs(pot[b:e] - opot) / np.abs(opot)
            assert np.median(rel) <= 1e-12 and rel.max() <= 1e-9, (s, np.median(rel), rel.max())
            assert np.median(relp) <= 1e-12 and relp.max() <= 1e-9, s
        else:
            assert np.all(acc[b:e] == 0) and np.all(pot[b:e] == 0)
    assert st["n_m2l"] == len(lists["m2l"])
    f.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batch_equals_single_calls(fmm, precision):
    systems = _systems()
    pos, mass, off = _concat(systems)
    print(f"[gpu] batch vs single calls, precision={precision}", flush=True)
    f = fmm.FMM(p=8, err_tol=1e-7, n_leaf=32, precision=precision, root_levels=2)
    acc, pot = f.forces_batch(_dev(pos), _dev(mass), off)
    acc, pot = acc.cpu().numpy(), pot.cpu().numpy()
    for s, (sp, sm) in enumerate(systems):
        a1, p1 = f.forces(_dev(sp), _dev(sm))
        b, e = off[s], off[s + 1]
        assert np.array_equal(acc[b:e], a1.cpu().numpy()), s
        assert np.array_equal(pot[b:e], p1.cpu().numpy()), s
    f.close()


def test_ensemble_config_batch(fmm):
    """The 256-cluster ensemble workload (sizes 2^U(10,16)), mixed precision,
    p = 8, epsilon = 1e-6: every cluster's median force error against the
    direct sum on sampled sinks stays below epsilon, and FP32 M2L/P2P stays
    within 1e-6 (median) of the FP64 batch."""
    cfg = W.CONFIGS["ensemble_256"]
    clusters = W.ensemble(cfg["count"], cfg["seed"])
    pos = np.concatenate([c[0] for c in clusters])
    mass = np.concatenate([c[2] for c in clusters])
    off = np.zeros(len(clusters) + 1, dtype=np.int64)
    off[1:] = np.cumsum([len(c[2]) for c in clusters])
    print(f"[gpu] ensemble_256: N={len(mass)}", flush=True)
    dpos, dmass = _dev(pos), _dev(mass)
    res = {}
    for precision in ("fp64", "mixed"):
        f = fmm.FMM(p=cfg["p"], err_tol=cfg["err_tol"], n_leaf=64, precision=precision)
        a, _ = f.forces_batch(dpos, dmass, off)
        res[precision] = a.cpu().numpy()
        f.close()
    rng = np.random.default_rng(cfg["seed"] + 5)
    for s in rng.choice(len(clusters), 8, replace=False):
        b, e = off[s], off[s + 1]
        sinks = np.sort(rng.choice(e - b, min(64, e - b), replace=False))
        ad, _ = oracle.direct(pos[b:e], mass[b:e], sinks=sinks)
        for precision, a in res.items():
            err = np.linalg.norm(a[b:e][sinks] - ad, axis=1) / np.linalg.norm(ad, axis=1)
            assert np.median(err) < cfg["err_tol"], (s, precision, np.median(err))
    d = np.linalg.norm(res["mixed"] - res["fp64"], axis=1) / np.linalg.norm(res["fp64"], axis=1)
    assert np.median(d) <= 1e-6 and d.max() <= 1e-3, (np.median(d), d.max())


def test_autotune_picks_a_candidate_and_caches(fmm):
    """The autotuner times the candidate leaf capacities, sets the fastest in
    the context, returns the cached choice for the same workload class, and
    the tuned context still matches the oracle run at that n_leaf."""
    import time
    systems = _systems()
    pos, mass, off = _concat(systems)
    print("[gpu] autotune on the mixed batch", flush=True)
    f = fmm.FMM(p=6, err_tol=1e-6, n_leaf=64)
    nl = f.autotune(_dev(pos), _dev(mass), off)
    assert nl in (16, 24, 32, 48, 64, 96, 128)
    t0 = time.perf_counter()
    assert f.autotune(_dev(pos), _dev(mass), off) == nl
    assert time.perf_counter() - t0 < 0.5
    prm = f.get_params()
    assert prm.n_leaf == nl and prm.m2l_waves == 1 and prm.p2p_groups in (0, 4, 2)
    assert prm.p2p_start in (0, 1)
    acc, _ = f.forces_batch(_dev(pos), _dev(mass), off)
    acc = acc.cpu().numpy()
    s = 5  # the 3000-body Plummer system
    b, e = off[s], off[s + 1]
    o = oracle.Oracle()
    oacc, _ = o.run(systems[s][0], systems[s][1], p=6, err_tol=1e-6, n_leaf=nl)
    rel = np.linalg.norm(acc[b:e] - oacc, axis=1) / np.linalg.norm(oacc, axis=1)
    assert np.median(rel) <= 1e-12 and rel.max() <= 1e-9
    f.close()


def test_autotune_mixed_picks_every_knob(fmm):
    """In mixed precision the autotuner also picks the FP32 M2L's wavefronts
    per sink and the near field's lane groups; the tuned batch stays within
    the mixed bound of the per-system oracle."""
    systems = _systems()
    pos, mass, off = _concat(systems)
    print("[gpu] autotune, mixed precision", flush=True)
    f = fmm.FMM(p=6, err_tol=1e-6, n_leaf=64, precision="mixed", root_levels=2)
    nl = f.autotune(_dev(pos), _dev(mass), off)
    prm = f.get_params()
    assert prm.n_leaf == nl and prm.m2l_waves in (1, 2, 4) and prm.p2p_groups in (0, 4, 2)
    assert prm.p2p_start in (0, 1)
    assert f.params.m2l_waves == prm.m2l_waves and f.params.p2p_start == prm.p2p_start
    acc, _ = f.forces_batch(_dev(pos), _dev(mass), off)
    acc = acc.cpu().numpy()
    s = 5
    b, e = off[s], off[s + 1]
    o = oracle.Oracle()
    oacc, _ = o.run(systems[s][0], systems[s][1], p=6, err_tol=1e-6, n_leaf=nl)
    rel = np.linalg.norm(acc[b:e] - oacc, axis=1) / np.linalg.norm(oacc, axis=1)
    assert np.median(rel) <= 1.5e-7
    f.close()
