"""Reference gradients of the force pass and of a leapfrog rollout, by direct
summation -- test infrastructure only (plain FP64 numpy, O(N^2)).

The force pass defines, with u_ij = x_j - x_i and s_ij^2 = |u_ij|^2 + eps^2,
    a_i   =  sum_{j != i} m_j u_ij / s_ij^3,
    pot_i = -sum_{j != i} m_j / s_ij
(G = 1, Plummer softening eps; pairs with s = 0 contribute nothing).  For a
scalar L(a, pot) with ga_i = dL/da_i and gp_i = dL/dpot_i, differentiating
these sums term by term gives, with K(u) = I/s^3 - 3 u u^T / s^5 (symmetric,
even in u) and u_ik = x_k - x_i:
    dL/dx_k = sum_{i != k} m_k [K(u_ik) ga_i + gp_i u_ik / s_ik^3]
              - sum_{j != k} m_j K(u_kj) ga_k - gp_k a_k
    dL/dm_k = sum_{i != k} [ga_i . u_ik / s_ik^3 - gp_i / s_ik].
The first line is the source side (body k moves the field every other body
feels), the second the sink side (the tidal tensor at x_k applied to ga_k).

The rollout is kick-drift-kick leapfrog with the direct-sum accelerations; its
gradient is taken in reverse step order, each half kick contributing the
force-pass gradient above with ga = (dt/2) * (the adjoint of the velocity).
"""
import numpy as np


def direct_forces(pos, mass, eps_soft=0.0, block=512):
    """a_i, pot_i by the defining double sum (blocked over sinks)."""
    pos = np.asarray(pos, dtype=np.float64)
    mass = np.asarray(mass, dtype=np.float64)
    n = len(mass)
    acc = np.zeros((n, 3))
    pot = np.zeros(n)
    e2 = float(eps_soft) ** 2
    for b0 in range(0, n, block):
        b1 = min(n, b0 + block)
        u = pos[None, :, :] - pos[b0:b1, None, :]            # x_j - x_i, (blk, n, 3)
        s2 = np.einsum("ijk,ijk->ij", u, u) + e2
        ok = s2 > 0
        ok[np.arange(b1 - b0), np.arange(b0, b1)] = False   # j != i
        inv = np.zeros_like(s2)
        inv[ok] = 1.0 / np.sqrt(s2[ok])
        inv3 = inv ** 3
        acc[b0:b1] = np.einsum("ij,ijk->ik", mass[None, :] * inv3, u)
        pot[b0:b1] = -(inv * mass[None, :]).sum(axis=1)
    return acc, pot


def direct_adjoint(pos, mass, gacc, gpot=None, eps_soft=0.0, block=512):
    """(dL/dpos (n, 3), dL/dmass (n,)) for L with dL/da = gacc, dL/dpot = gpot."""
    pos = np.asarray(pos, dtype=np.float64)
    mass = np.asarray(mass, dtype=np.float64)
    ga = np.asarray(gacc, dtype=np.float64)
    n = len(mass)
    gp = np.zeros(n) if gpot is None else np.asarray(gpot, dtype=np.float64)
    acc, _ = direct_forces(pos, mass, eps_soft, block)
    e2 = float(eps_soft) ** 2
    gx = np.zeros((n, 3))
    gm = np.zeros(n)
    for b0 in range(0, n, block):
        b1 = min(n, b0 + block)
        k = np.arange(b0, b1)
        u = pos[k, None, :] - pos[None, :, :]                # u_ik = x_k - x_i, (blk, n, 3)
        s2 = np.einsum("abc,abc->ab", u, u) + e2
        ok = s2 > 0
        ok[np.arange(b1 - b0), k] = False
        inv = np.zeros_like(s2)
        inv[ok] = 1.0 / np.sqrt(s2[ok])
        inv3 = inv ** 3
        inv5 = inv3 * inv * inv
        # K(u) g = g / s^3 - 3 (u . g) u / s^5
        ug = np.einsum("abc,bc->ab", u, ga)                  # u_ik . ga_i
        src = (inv3[:, :, None] * ga[None, :, :] - 3.0 * (ug * inv5)[:, :, None] * u
               + (gp[None, :] * inv3)[:, :, None] * u).sum(axis=1)
        gx[b0:b1] += mass[k, None] * src
        # sink side: -sum_j m_j K(u_kj) ga_k  (K even in u, so u_ik serves)
        uk = np.einsum("abc,ac->ab", u, ga[k])               # u_kj . ga_k
        tid = (mass[None, :] * inv3)[:, :, None] * ga[k][:, None, :] \
            - 3.0 * (mass[None, :] * uk * inv5)[:, :, None] * u
        gx[b0:b1] -= tid.sum(axis=1)
        gx[b0:b1] -= gp[k, None] * acc[k]
        gm[b0:b1] = (ug * inv3 - gp[None, :] * inv).sum(axis=1)
    return gx, gm


def direct_jerk(pos, vel, mass, eps_soft=0.0, block=512):
    """Time derivative of a_i along the motion (the jerk):
    j_i = sum_{j != i} m_j [w_ij / s^3 - 3 (u_ij . w_ij) u_ij / s^5],
    u_ij = x_j - x_i, w_ij = v_j - v_i, differentiating a_i's defining sum."""
    pos = np.asarray(pos, dtype=np.float64)
    vel = np.asarray(vel, dtype=np.float64)
    mass = np.asarray(mass, dtype=np.float64)
    n = len(mass)
    jerk = np.zeros((n, 3))
    e2 = float(eps_soft) ** 2
    for b0 in range(0, n, block):
        b1 = min(n, b0 + block)
        u = pos[None, :, :] - pos[b0:b1, None, :]
        w = vel[None, :, :] - vel[b0:b1, None, :]
        s2 = np.einsum("abc,abc->ab", u, u) + e2
        ok = s2 > 0
        ok[np.arange(b1 - b0), np.arange(b0, b1)] = False
        inv = np.zeros_like(s2)
        inv[ok] = 1.0 / np.sqrt(s2[ok])
        inv3 = inv ** 3
        inv5 = inv3 * inv * inv
        uw = np.einsum("abc,abc->ab", u, w)
        jerk[b0:b1] = ((mass[None, :] * inv3)[:, :, None] * w
                       - 3.0 * (mass[None, :] * uw * inv5)[:, :, None] * u).sum(axis=1)
    return jerk


def leapfrog(pos, vel, mass, dt, steps, eps_soft=0.0, forces=direct_forces):
    """Kick-drift-kick leapfrog; returns the final positions and velocities."""
    x = np.array(pos, dtype=np.float64)
    v = np.array(vel, dtype=np.float64)
    a, _ = forces(x, mass, eps_soft)
    for _ in range(steps):
        v = v + 0.5 * dt * a
        x = x + dt * v
        a, _ = forces(x, mass, eps_soft)
        v = v + 0.5 * dt * a
    return x, v


def rollout_gradient(pos, vel, mass, dt, steps, target, eps_soft=0.0):
    """L = sum |x_T - target|^2 after `steps` leapfrog steps: returns
    (L, dL/dx_0, dL/dv_0, dL/dm), the gradient taken in reverse step order."""
    x = np.array(pos, dtype=np.float64)
    v = np.array(vel, dtype=np.float64)
    xs = [x.copy()]
    a, _ = direct_forces(x, mass, eps_soft)
    for _ in range(steps):
        v = v + 0.5 * dt * a
        x = x + dt * v
        a, _ = direct_forces(x, mass, eps_soft)
        v = v + 0.5 * dt * a
        xs.append(x.copy())
    d = x - target
    L = float((d * d).sum())
    lx = 2.0 * d
    lv = np.zeros_like(lx)
    lm = np.zeros(len(mass))
    for t in range(steps - 1, -1, -1):
        # v_{t+1} = v_half + (dt/2) a(x_{t+1})
        gx, gm = direct_adjoint(xs[t + 1], mass, 0.5 * dt * lv, None, eps_soft)
        lx = lx + gx
        lm = lm + gm
        # x_{t+1} = x_t + dt v_half
        lv = lv + dt * lx
        # v_half = v_t + (dt/2) a(x_t)
        gx, gm = direct_adjoint(xs[t], mass, 0.5 * dt * lv, None, eps_soft)
        lx = lx + gx
        lm = lm + gm
    return L, lx, lv, lm
