"""The (epsilon, p) accuracy grid tool on a small sphere: in every cell the
median relative force error against the direct sum stays below epsilon
(section 4.1), and at a fixed epsilon a low order opens more cells than a high
one (the error estimate of a low-order expansion is larger), so its near field
holds at least as many body pairs: the mechanism section 4.1 gives for the
low-order corner of the grid, where accuracy does not grow with p."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def test_small_accuracy_grid():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2012_02207_amd import accuracy_grid as G
    print("[gpu] accuracy grid N=4096", flush=True)
    g = G.run_grid(n=4096, seed=11, eps_list=[1e-3, 1e-6, 1e-9], p_list=[4, 8, 12], repeats=1)
    by = {(c["eps"], c["p"]): c for c in g["cells"]}
    for (e, p), c in by.items():
        assert c["median"] < e, (e, p, c["median"])
    for e in (1e-3, 1e-6, 1e-9):
        assert by[(e, 4)]["n_p2p_pairs"] >= by[(e, 12)]["n_p2p_pairs"]
    md = G.to_markdown(g)
    assert md.count("| 1e-06 |") == 4
