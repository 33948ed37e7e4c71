"""Differentiable force pass and leapfrog rollout on top of the gfx950 FMM.

``FMMForces`` wraps one force evaluation (fmm_forces) as a torch autograd
function; its backward calls the library's hand-written adjoint and returns
dL/dpos and dL/dmass.  When the context still holds that evaluation (no other
evaluation ran on it since) the backward uses fmm_adjoint_last, which reuses
its tree, lists and expansions; otherwise fmm_adjoint, which recomputes them
at the saved positions.  ``leapfrog`` integrates kick-drift-kick steps with it;
with ``checkpoint_every = k`` only every k-th state is kept, and the forces of
a segment (tree, lists, expansions) are recomputed when its gradient is
needed, so the memory of a rollout does not grow with its length beyond the
checkpoints.  Given k contexts, step j of each segment evaluates on context
j mod k, so every step's state is still in place when its gradient is formed.
All arithmetic runs in the library's kernels; this module only orders the
calls.
"""
import torch
from torch.utils.checkpoint import checkpoint

from . import fmm as _fmm


class FMMForces(torch.autograd.Function):
    """acc, pot = FMMForces.apply(pos, mass, solver, eps_soft)"""

    @staticmethod
    def forward(ctx, pos, mass, solver, eps_soft):
        acc, pot = solver.forces(pos.detach().contiguous(), mass.detach().contiguous(), eps_soft=eps_soft)
        # which evaluation of the context this was, saved as a tensor so that a
        # checkpoint's recomputation replaces it along with the positions
        eid = torch.tensor(getattr(solver, "evals", -1), dtype=torch.int64)
        ctx.save_for_backward(pos, mass, acc, eid)
        ctx.solver, ctx.eps_soft = solver, eps_soft
        return acc, pot

    @staticmethod
    def backward(ctx, gacc, gpot):
        pos, mass, acc, eid = ctx.saved_tensors
        if gacc is None:
            gacc = torch.zeros_like(pos)
        gp = None if gpot is None else gpot.contiguous()
        s = ctx.solver
        if int(eid) >= 0 and getattr(s, "evals", None) == int(eid):
            gpos, gmass = s.adjoint_last(acc, gacc.contiguous(), gp)  # the context still holds it
        else:
            gpos, gmass = s.adjoint(pos.detach().contiguous(), mass.detach().contiguous(),
                                    gacc.contiguous(), gp, eps_soft=ctx.eps_soft)
        return gpos, gmass, None, None


def forces(pos, mass, solver, eps_soft=0.0):
    """Differentiable (acc, pot) of one force evaluation."""
    return FMMForces.apply(pos, mass, solver, eps_soft)


def _segment(x, v, a, mass, solvers, dt, nsteps, eps_soft):
    for j in range(nsteps):
        v = v + 0.5 * dt * a
        x = x + dt * v
        a, _ = forces(x, mass, solvers[j % len(solvers)], eps_soft)
        v = v + 0.5 * dt * a
    return x, v, a


def leapfrog(pos, vel, mass, solver, dt, steps, eps_soft=0.0, checkpoint_every=8):
    """Kick-drift-kick leapfrog with FMM forces; returns (x_T, v_T),
    differentiable with respect to pos, vel and mass.  solver is one context
    or a list of them (step j of a segment on solver[j mod len]; with as many
    contexts as steps per segment no adjoint recomputes its forward pass)."""
    solvers = list(solver) if isinstance(solver, (list, tuple)) else [solver]
    a, _ = forces(pos, mass, solvers[-1], eps_soft)
    x, v = pos, vel
    done = 0
    while done < steps:
        k = min(checkpoint_every, steps - done) if checkpoint_every > 0 else steps - done
        if checkpoint_every > 0 and torch.is_grad_enabled():
            x, v, a = checkpoint(_segment, x, v, a, mass, solvers, dt, k, eps_soft, use_reentrant=False)
        else:
            x, v, a = _segment(x, v, a, mass, solvers, dt, k, eps_soft)
        done += k
    return x, v


def leapfrog_frozen(pos, vel, mass, solvers, dt, steps, eps_soft=0.0, record=False):
    """Leapfrog without gradients where force evaluation s uses its own context
    solvers[s] (steps + 1 of them).  record=True builds each context's tree
    and lists (fmm_forces); otherwise every evaluation reuses them
    (fmm_forces_frozen), so the final state is a smooth function of the
    inputs: the form finite differences of a rollout need."""
    with torch.no_grad():
        def F(s, x):
            if record:
                return solvers[s].forces(x.contiguous(), mass, eps_soft=eps_soft)[0]
            return solvers[s].forces_frozen(x.contiguous(), mass, eps_soft=eps_soft)[0]
        x, v = pos, vel
        a = F(0, x)
        for t in range(steps):
            v = v + 0.5 * dt * a
            x = x + dt * v
            a = F(t + 1, x)
            v = v + 0.5 * dt * a
        return x, v


def make_solver(p=10, err_tol=1e-7, n_leaf=64, **kw):
    """An FP64 force context for differentiable use."""
    return _fmm.FMM(p=p, err_tol=err_tol, n_leaf=n_leaf, precision="fp64", **kw)
