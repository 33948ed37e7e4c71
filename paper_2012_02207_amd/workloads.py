"""Seeded synthetic inputs for the force pass (no FMM arithmetic lives here).

The paper's inputs are Plummer spheres in Henon units (G = M = 1,
E0 = -1/4; section 3, "Tests"), scale radius 0.59 (section 3.1.2).  They were
made with an external tool that is not available, so the textbook sampler of
Aarseth, Henon & Wielen (1974) stands in for it:

* radius from the inverted cumulative mass M(<r) = r^3/(r^2+a^2)^(3/2),
  truncated at 10 a by drawing the mass fraction from U(0, (100/101)^(3/2));
* isotropic directions;
* speed q * v_esc with q drawn by rejection from q^2 (1-q^2)^(7/2);
* positions and velocities shifted to the centre-of-mass frame.

Kroupa (2001) masses use the two-segment power law (slope 1.3 below
0.5 Msun, 2.3 above) on [0.08, 100], sampled through the inverse CDF.

All generators use numpy's PCG64 with an explicit seed and return float64
arrays: positions (N, 3), velocities (N, 3), masses (N,).
"""
import numpy as np

A_HENON = 3.0 * np.pi / 16.0          # Plummer scale radius in Henon units
SEED_BASE = 20120220


def _unit_vectors(rng, n):
    cost = rng.uniform(-1.0, 1.0, n)
    phi = rng.uniform(0.0, 2.0 * np.pi, n)
    sint = np.sqrt(1.0 - cost * cost)
    return np.stack([sint * np.cos(phi), sint * np.sin(phi), cost], axis=1)


def plummer(n, seed, a=A_HENON, rmax_over_a=10.0, total_mass=1.0):
    """Equal-mass Plummer sphere: returns (pos, vel, mass)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    xmax = (rmax_over_a ** 2 / (rmax_over_a ** 2 + 1.0)) ** 1.5
    X = rng.uniform(0.0, xmax, n)
    X = np.where(X <= 0.0, np.finfo(float).tiny, X)
    r = a / np.sqrt(X ** (-2.0 / 3.0) - 1.0)
    pos = r[:, None] * _unit_vectors(rng, n)
    q = np.empty(n)
    todo = np.arange(n)
    while todo.size:
        x4 = rng.uniform(0.0, 1.0, todo.size)
        x5 = rng.uniform(0.0, 0.1, todo.size)
        ok = x5 < x4 * x4 * (1.0 - x4 * x4) ** 3.5
        q[todo[ok]] = x4[ok]
        todo = todo[~ok]
    vesc = np.sqrt(2.0) * (r * r + a * a) ** -0.25
    vel = (q * vesc)[:, None] * _unit_vectors(rng, n)
    mass = np.full(n, total_mass / n)
    pos -= (mass[:, None] * pos).sum(0) / mass.sum()
    vel -= (mass[:, None] * vel).sum(0) / mass.sum()
    return pos, vel, mass


def kroupa_masses(n, seed, mlo=0.08, mbreak=0.5, mhi=100.0, a1=1.3, a2=2.3):
    """Kroupa (2001) IMF samples (solar masses), inverse-CDF."""
    rng = np.random.Generator(np.random.PCG64(seed))
    # unnormalised pdf: m^-a1 below the break, mbreak^(a2-a1) m^-a2 above (continuous)
    c1 = (mbreak ** (1 - a1) - mlo ** (1 - a1)) / (1 - a1)
    c2 = mbreak ** (a2 - a1) * (mhi ** (1 - a2) - mbreak ** (1 - a2)) / (1 - a2)
    u = rng.uniform(0.0, 1.0, n) * (c1 + c2)
    lowseg = u < c1
    m = np.empty(n)
    m[lowseg] = (mlo ** (1 - a1) + (1 - a1) * u[lowseg]) ** (1.0 / (1 - a1))
    u2 = (u[~lowseg] - c1) / mbreak ** (a2 - a1)
    m[~lowseg] = (mbreak ** (1 - a2) + (1 - a2) * u2) ** (1.0 / (1 - a2))
    return m


def kroupa_with_central(n, seed, central_fraction=0.01):
    """Plummer positions with Kroupa masses (n-1 stars) plus one central
    particle holding `central_fraction` of the total mass at the origin."""
    pos, vel, _ = plummer(n - 1, seed)
    m = kroupa_masses(n - 1, seed + 7919)
    m *= (1.0 - central_fraction) / m.sum()
    pos = np.vstack([pos, np.zeros((1, 3))])
    vel = np.vstack([vel, np.zeros((1, 3))])
    mass = np.concatenate([m, [central_fraction]])
    return pos, vel, mass


def ensemble_sizes(count, seed, lo_exp=10, hi_exp=16):
    """Cluster sizes round(2^U(lo, hi)), seeded."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.rint(2.0 ** rng.uniform(lo_exp, hi_exp, count)).astype(np.int64)


def ensemble(count, seed):
    """List of independent Plummer clusters (pos, vel, mass) of uneven size."""
    sizes = ensemble_sizes(count, seed)
    return [plummer(int(nc), seed * 1000 + i) for i, nc in enumerate(sizes)]


def uniform_cube(n, seed, scale=1.0):
    """Uniform random positions in a cube and random positive masses (edge cases)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    pos = rng.uniform(-scale, scale, (n, 3))
    mass = rng.uniform(0.5, 1.5, n) / n
    return pos, mass


# The benchmark configurations (seed = SEED_BASE + index)
CONFIGS = {
    "plummer_4k": dict(n=4096, p=6, err_tol=1e-6, seed=SEED_BASE + 0),
    "plummer_1m": dict(n=1 << 20, p=10, err_tol=1e-7, seed=SEED_BASE + 1),
    "kroupa_4m": dict(n=1 << 22, p=12, err_tol=1e-7, seed=SEED_BASE + 2),
    "ensemble_256": dict(count=256, p=8, err_tol=1e-6, seed=SEED_BASE + 3),
    "rollout_256k": dict(n=1 << 18, p=10, err_tol=1e-7, seed=SEED_BASE + 4),
}
