"""The frozen-tree evaluation replayed as a HIP graph (fmm_forces_frozen_graph)
against the same evaluation launched eagerly (fmm_forces_frozen): bit-identical
on every replay, with positions updated in place between replays, unrelated
GPU work and synchronisations in between, and after a rebuild of the tree."""
import numpy as np
import pytest

from paper_2012_02207_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_graph_replays_match_eager(precision):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2012_02207_amd import fmm
    pos, _, mass = W.plummer(6000, 91)
    print(f"[gpu] graph replay, precision={precision}", flush=True)
    dev = "cuda:0"
    P = torch.from_numpy(pos).to(dev)
    M = torch.from_numpy(mass).to(dev)
    f = fmm.FMM(p=8, err_tol=1e-7, n_leaf=32, precision=precision, root_levels=2)
    other = fmm.FMM(p=6, err_tol=1e-6)
    f.forces(P, M)
    acc = torch.empty((6000, 3), dtype=torch.float64, device=dev)
    pot = torch.empty(6000, dtype=torch.float64, device=dev)
    rng = np.random.default_rng(2)
    for rep in range(4):
        if rep == 2:      # a rebuild drops the graph; the next call captures again
            f.forces(P, M)
        ref_a, ref_p = f.forces_frozen(P.clone(), M)
        f.forces_frozen(P, M, out=(acc, pot), graph=True)
        torch.cuda.synchronize()
        assert torch.equal(acc, ref_a) and torch.equal(pot, ref_p), rep
        other.forces(P[:2000].contiguous(), M[:2000].contiguous())   # unrelated work between replays
        torch.cuda.synchronize()
        P += torch.from_numpy(1e-4 * rng.normal(size=pos.shape)).to(dev)   # in place, same buffer
    f.close()
    other.close()


def test_graph_recaptured_after_set_params():
    """fmm_set_params drops a captured graph: after a switch of precision (or
    of the root split) the graph replay equals the eager frozen evaluation
    under the new parameters, not a replay of the old capture."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2012_02207_amd import fmm
    pos, _, mass = W.plummer(5000, 93)
    print("[gpu] graph after set_params", flush=True)
    dev = "cuda:0"
    P = torch.from_numpy(pos).to(dev)
    M = torch.from_numpy(mass).to(dev)
    f = fmm.FMM(p=8, err_tol=1e-7, n_leaf=32, precision="fp64", root_levels=2)
    f.forces(P, M)
    acc = torch.empty((5000, 3), dtype=torch.float64, device=dev)
    pot = torch.empty(5000, dtype=torch.float64, device=dev)
    f.forces_frozen(P, M, out=(acc, pot), graph=True)
    a64 = acc.clone()
    for kw in ({"precision": "mixed"}, {"root_levels": 0}, {"precision": "fp64"}):
        f.set_params(**kw)
        ref_a, ref_p = f.forces_frozen(P, M)
        f.forces_frozen(P, M, out=(acc, pot), graph=True)
        torch.cuda.synchronize()
        assert torch.equal(acc, ref_a) and torch.equal(pot, ref_p), kw
    assert torch.equal(acc, a64)  # back to FP64: the first capture's result again
    f.close()
