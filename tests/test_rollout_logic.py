"""The rollout driver (checkpoint segments, autograd wiring) on the CPU with a
stand-in force solver that evaluates the direct sums of the oracle: the final
state must not depend on the checkpoint spacing, and the autograd gradient
must equal the oracle's reverse-mode rollout gradient."""
import numpy as np
import pytest

from oracle import adjoint as A

torch = pytest.importorskip("torch")


class DirectSolver:
    """forces/adjoint with the signatures of the GPU context, on CPU tensors."""

    def forces(self, pos, mass, eps_soft=0.0):
        a, p = A.direct_forces(pos.numpy(), mass.numpy(), eps_soft)
        return torch.from_numpy(a), torch.from_numpy(p)

    def adjoint(self, pos, mass, gacc, gpot=None, eps_soft=0.0):
        gx, gm = A.direct_adjoint(pos.numpy(), mass.numpy(), gacc.numpy(),
                                  None if gpot is None else gpot.numpy(), eps_soft)
        return torch.from_numpy(gx), torch.from_numpy(gm)


def _case():
    rng = np.random.default_rng(2)
    n = 24
    pos = rng.normal(size=(n, 3))
    vel = 0.2 * rng.normal(size=(n, 3))
    mass = rng.uniform(0.5, 1.5, n) / n
    target = pos + 0.05 * rng.normal(size=(n, 3))
    return pos, vel, mass, target


@pytest.mark.parametrize("every", [0, 1, 3, 8])
def test_checkpoint_spacing_does_not_change_the_state(every):
    from paper_2012_02207_amd import rollout as R
    pos, vel, mass, _ = _case()
    x, v = R.leapfrog(torch.from_numpy(pos), torch.from_numpy(vel), torch.from_numpy(mass),
                      DirectSolver(), 1e-2, 7, checkpoint_every=every)
    xr, vr = A.leapfrog(pos, vel, mass, 1e-2, 7)
    assert np.allclose(x.detach().numpy(), xr, rtol=0, atol=1e-14)
    assert np.allclose(v.detach().numpy(), vr, rtol=0, atol=1e-14)


@pytest.mark.parametrize("every", [2, 5])
def test_autograd_gradient_equals_reverse_mode_reference(every):
    from paper_2012_02207_amd import rollout as R
    pos, vel, mass, target = _case()
    x0, v0, m = (torch.from_numpy(a).requires_grad_(True) for a in (pos, vel, mass))
    xT, _ = R.leapfrog(x0, v0, m, DirectSolver(), 1e-2, 6, checkpoint_every=every)
    loss = ((xT - torch.from_numpy(target)) ** 2).sum()
    loss.backward()
    L, gx, gv, gm = A.rollout_gradient(pos, vel, mass, 1e-2, 6, target)
    assert np.isclose(loss.item(), L, rtol=1e-13)
    for g, r in ((x0.grad, gx), (v0.grad, gv), (m.grad, gm)):
        assert np.allclose(g.numpy(), r, rtol=1e-10, atol=1e-13 * np.abs(r).max())


class ReuseSolver(DirectSolver):
    """DirectSolver with the context's evaluation counter and adjoint_last: the
    adjoint at the positions of its last evaluation (counted when used)."""

    def __init__(self):
        self.evals = 0
        self.reused = self.recomputed = 0
        self._last = None

    def forces(self, pos, mass, eps_soft=0.0):
        self.evals += 1
        self._last = (pos.clone(), mass.clone(), eps_soft)
        return super().forces(pos, mass, eps_soft)

    def adjoint(self, pos, mass, gacc, gpot=None, eps_soft=0.0):
        self.evals += 1  # the GPU adjoint re-evaluates the forward pass
        self.recomputed += 1
        self._last = (pos.clone(), mass.clone(), eps_soft)
        return super().adjoint(pos, mass, gacc, gpot, eps_soft)

    def adjoint_last(self, acc, gacc, gpot=None):
        self.reused += 1
        pos, mass, eps = self._last
        return super().adjoint(pos, mass, gacc, gpot, eps)


@pytest.mark.parametrize("every,nctx", [(3, 4), (3, 1), (2, 3), (0, 2)])
def test_per_step_contexts_reuse_the_forward_state(every, nctx):
    """With one context per step of a checkpoint segment (and one for the
    initial forces) every adjoint reuses its step's evaluation, and the
    gradient is still the reverse-mode reference; with fewer contexts, stale
    ones fall back to the recomputing adjoint and give the same gradient.
    (The last step's forces do not reach x_T, so five steps and the initial
    forces have a backward.)"""
    from paper_2012_02207_amd import rollout as R
    pos, vel, mass, target = _case()
    x0, v0, m = (torch.from_numpy(a).requires_grad_(True) for a in (pos, vel, mass))
    solvers = [ReuseSolver() for _ in range(nctx)]
    xT, _ = R.leapfrog(x0, v0, m, solvers, 1e-2, 6, checkpoint_every=every)
    loss = ((xT - torch.from_numpy(target)) ** 2).sum()
    loss.backward()
    L, gx, gv, gm = A.rollout_gradient(pos, vel, mass, 1e-2, 6, target)
    for g, r in ((x0.grad, gx), (v0.grad, gv), (m.grad, gm)):
        assert np.allclose(g.numpy(), r, rtol=1e-10, atol=1e-13 * np.abs(r).max())
    reused = sum(s.reused for s in solvers)
    recomputed = sum(s.recomputed for s in solvers)
    assert reused + recomputed == 6
    if every and nctx == every + 1:
        assert recomputed == 0
    else:
        assert reused >= 1 and recomputed >= 1
