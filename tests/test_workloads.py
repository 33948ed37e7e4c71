"""Pins for the seeded input generators against the Plummer model's closed
forms and the values the paper states for Henon units."""
import json
import math
import os

import numpy as np
from scipy import stats

import oracle
from paper_2012_02207_amd import workloads as W

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def test_henon_scale_radius_matches_paper():
    g = GOLD["plummer_scale_radius"]
    assert abs(W.A_HENON / g["a"] - 1) < g["rel_tol"]
    # untruncated Plummer: W = -3 pi G M^2 / (32 a); virial E0 = W / 2
    E0 = -3 * math.pi / (32 * W.A_HENON) / 2
    assert abs(E0 - GOLD["henon_units"]["E0"]) < 1e-15


def test_circular_velocity_at_unit_radius():
    g = GOLD["circular_velocity_at_rvir"]
    a = W.A_HENON
    vc = math.sqrt(1.0 / (1 + a * a) ** 1.5)
    assert abs(vc - g["Vc"]) < g["abs_tol"]
    pos, _, m = W.plummer(100000, 1)
    frac = m[np.linalg.norm(pos, axis=1) < 1].sum()
    # sampled enclosed mass (truncated model) within 4 sigma
    xmax = (100 / 101) ** 1.5
    exp = (1 / (1 + a * a) ** 1.5) / xmax
    assert abs(frac - exp) < 4 * math.sqrt(exp * (1 - exp) / 1e5)


def test_plummer_radii_follow_cumulative_mass_profile():
    pos, vel, m = W.plummer(50000, 2)
    r = np.linalg.norm(pos, axis=1)
    a = W.A_HENON
    xmax = (100 / 101) ** 1.5
    cdf = lambda x: np.clip((x ** 3 / (x * x + a * a) ** 1.5) / xmax, 0, 1)
    # COM shift is O(N^-1/2 a); KS on the radii
    assert stats.kstest(r, cdf).pvalue > 1e-3
    assert r.max() <= 10 * a * 1.01
    assert abs(np.median(r) - a / math.sqrt((0.5 * xmax) ** (-2 / 3) - 1)) < 0.02
    u = pos / r[:, None]
    assert np.abs(u.mean(0)).max() < 0.02                # isotropy
    assert np.abs(m.sum() - 1) < 1e-12
    assert np.abs((m[:, None] * pos).sum(0)).max() < 1e-12


def test_plummer_virial_energies():
    pos, vel, m = W.plummer(4096, 20120220)
    _, pot = oracle.direct(pos, m)
    Wp = 0.5 * (m * pot).sum()
    T = 0.5 * (m * (vel * vel).sum(1)).sum()
    assert abs(Wp + 0.5) < 0.05 and abs(T - 0.25) < 0.03
    assert abs(2 * T / -Wp - 1) < 0.1


def test_kroupa_masses_and_central_particle():
    m = W.kroupa_masses(200000, 3)
    assert m.min() >= 0.08 and m.max() <= 100
    # analytic fraction of stars below the break
    a1, a2, lo, br, hi = 1.3, 2.3, 0.08, 0.5, 100.0
    c1 = (br ** (1 - a1) - lo ** (1 - a1)) / (1 - a1)
    c2 = br ** (a2 - a1) * (hi ** (1 - a2) - br ** (1 - a2)) / (1 - a2)
    f = (m < br).mean()
    assert abs(f - c1 / (c1 + c2)) < 0.005
    pos, vel, mass = W.kroupa_with_central(5000, 4)
    assert mass.shape == (5000,) and abs(mass.sum() - 1) < 1e-12
    assert mass[-1] == 0.01 and np.all(pos[-1] == 0)
    stars = mass[:-1]
    assert 500 < stars.max() / stars.min() < 1250.001


def test_ensemble_sizes():
    s = W.ensemble_sizes(256, 5)
    assert s.min() >= 2 ** 10 and s.max() <= 2 ** 16 and len(s) == 256
    assert np.array_equal(s, W.ensemble_sizes(256, 5))
