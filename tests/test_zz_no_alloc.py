"""fmm_forces_noalloc (scratch in the library's static device array) against
fmm_forces on the same inputs, through the C ABI: two calls in a row, the
second with fewer bodies, in FP64 and mixed precision.  The two entry points
run the same kernels in the same order, so the outputs must be identical bit
for bit (stricter than the FP64 parity bar of 1e-12)."""
import sys

import numpy as np
import pytest

from paper_2012_02207_amd import fmm, workloads

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    return torch


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_noalloc_matches_fmm_forces(precision):
    torch = _torch()
    dev = torch.device("cuda:0")
    f = fmm.FMM(p=8, err_tol=1e-6, n_leaf=32, precision=precision)
    for n, seed in ((20000, 31), (6000, 32)):
        print(f"noalloc {precision} n={n} seed={seed}", flush=True)
        pos, _, m = workloads.plummer(n, seed)
        tp, tm = torch.from_numpy(pos).to(dev), torch.from_numpy(m).to(dev)
        a0, p0 = f.forces(tp, tm, noalloc=True)
        a1, p1 = f.forces(tp, tm)
        torch.cuda.synchronize()
        a0, p0, a1, p1 = (x.cpu().numpy() for x in (a0, p0, a1, p1))
        assert np.all(np.isfinite(a0)) and np.all(np.isfinite(p0))
        assert np.array_equal(a0, a1), np.abs(a0 - a1).max()
        assert np.array_equal(p0, p1)


def test_noalloc_repeat_after_larger_call_and_limits():
    torch = _torch()
    dev = torch.device("cuda:0")
    f = fmm.FMM(p=6, err_tol=1e-6, n_leaf=64)
    res = []
    for n, seed in ((30000, 41), (3000, 42), (30000, 41)):
        print(f"noalloc fp64 n={n} seed={seed}", flush=True)
        pos, _, m = workloads.plummer(n, seed)
        tp, tm = torch.from_numpy(pos).to(dev), torch.from_numpy(m).to(dev)
        a, p = f.forces(tp, tm, noalloc=True)
        torch.cuda.synchronize()
        res.append((a.cpu().numpy(), p.cpu().numpy()))
    # the scratch keeps the previous call's contents; the result must not depend on them
    assert np.array_equal(res[0][0], res[2][0]) and np.array_equal(res[0][1], res[2][1])
    n = fmm.NOALLOC_MAX_N + 1
    pos, _, m = workloads.plummer(n, 43)
    with pytest.raises(fmm.FmmError) as e:
        f.forces(torch.from_numpy(pos).to(dev), torch.from_numpy(m).to(dev), noalloc=True)
    assert e.value.status == fmm.FMM_EINVAL and "NOALLOC_MAX_N" in str(e.value)
