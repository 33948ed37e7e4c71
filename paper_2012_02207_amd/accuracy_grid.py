"""Force-accuracy grid of the GPU FMM over the acceptance tolerance epsilon and
the expansion order p (section 4.1: median and 99.99th-percentile relative
force error heat maps, and the time per force evaluation).

For a seeded Plummer sphere (default N = 10^5, Henon units) every (epsilon, p)
cell runs the GPU force pass and compares it with the GPU direct sum over all
bodies (or with a reference acceleration the caller supplies for a subset of
sinks); the relative force error of body i is |a_i - a_i^direct| / |a_i^direct|.
Prints text heat maps (rows epsilon, columns p: median, 99th and 99.99th
percentiles) plus the evaluation time and the near-field work of each cell,
as Markdown.

    python -m paper_2012_02207_amd.accuracy_grid --n 100000 --out grid.md
"""
import argparse
import json
import sys
import time

import numpy as np


def run_grid(n=100_000, seed=20120225, eps_list=None, p_list=None, precision="fp64", n_leaf=64,
             repeats=3, sinks=None, ref_acc=None):
    """sinks/ref_acc (host arrays): measure the error on these bodies only,
    against the given accelerations, instead of the GPU direct sum."""
    import torch
    from . import fmm, workloads as W
    eps_list = eps_list or [10.0 ** -k for k in range(3, 14)]
    p_list = p_list or list(range(4, 21))
    pos, _, mass = W.plummer(n, seed)
    dev = torch.device("cuda:0")
    dpos = torch.from_numpy(pos).to(dev)
    dmass = torch.from_numpy(mass).to(dev)
    if ref_acc is None:
        sel = torch.arange(n, device=dev)
        ad, _ = fmm.direct(dpos, dmass)
    else:
        sel = torch.from_numpy(np.asarray(sinks, dtype=np.int64)).to(dev)
        ad = torch.from_numpy(np.ascontiguousarray(ref_acc, dtype=np.float64)).to(dev)
    nd = torch.linalg.norm(ad, dim=1)
    cells = []
    for eps in eps_list:
        for p in p_list:
            f = fmm.FMM(p=p, err_tol=eps, n_leaf=n_leaf, precision=precision)
            acc, _ = f.forces(dpos, dmass)          # warm-up (allocations)
            ts = []
            for _ in range(repeats):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                acc, _ = f.forces(dpos, dmass)
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t0)
            st = f.stats()
            rel = (torch.linalg.norm(acc[sel] - ad, dim=1) / nd).cpu().numpy()
            cells.append({"eps": eps, "p": p, "median": float(np.median(rel)),
                          "p99": float(np.percentile(rel, 99)),
                          "p9999": float(np.percentile(rel, 99.99)), "max": float(rel.max()),
                          "ms": 1e3 * float(np.median(ts)), "n_m2l": int(st["n_m2l"]),
                          "n_p2p_pairs": int(st["n_p2p_pairs"])})
            f.close()
            print(f"eps={eps:.0e} p={p:2d} median={cells[-1]['median']:.2e} p99={cells[-1]['p99']:.2e} "
                  f"p99.99={cells[-1]['p9999']:.2e} {cells[-1]['ms']:.2f} ms", file=sys.stderr,
                  flush=True)
    return {"n": n, "seed": seed, "precision": precision, "n_leaf": n_leaf, "cells": cells,
            "eps": eps_list, "p": p_list}


def to_markdown(g):
    eps_list, p_list = g["eps"], g["p"]
    by = {(c["eps"], c["p"]): c for c in g["cells"]}
    out = [f"Plummer N = {g['n']} (seed {g['seed']}), {g['precision']}, n_leaf = {g['n_leaf']}; "
           f"relative force error against the direct sum over all bodies.", ""]

    def table(title, key, fmt):
        out.append(f"**{title}** (rows: epsilon, columns: p)")
        out.append("")
        out.append("| eps \\ p | " + " | ".join(str(p) for p in p_list) + " |")
        out.append("|---|" + "---|" * len(p_list))
        for e in eps_list:
            out.append(f"| {e:.0e} | " + " | ".join(fmt(by[(e, p)][key]) for p in p_list) + " |")
        out.append("")
    table("median relative force error", "median", lambda v: f"{v:.1e}")
    table("99th percentile relative force error", "p99", lambda v: f"{v:.1e}")
    table("99.99th percentile relative force error", "p9999", lambda v: f"{v:.1e}")
    table("GPU time per force evaluation, ms", "ms", lambda v: f"{v:.1f}")
    table("directed near-field body pairs / N^2", "n_p2p_pairs",
          lambda v: f"{v / float(g['n']) ** 2:.2f}")
    return "\n".join(out)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--n", type=int, default=100_000)
    ap.add_argument("--seed", type=int, default=20120225)
    ap.add_argument("--pmin", type=int, default=4)
    ap.add_argument("--pmax", type=int, default=20)
    ap.add_argument("--eps-exp", default="3-13", help="epsilon = 10^-k for k in this range")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--n-leaf", type=int, default=64)
    ap.add_argument("--out", default="")
    ap.add_argument("--json", default="")
    a = ap.parse_args(argv)
    k0, k1 = (int(x) for x in a.eps_exp.split("-"))
    g = run_grid(a.n, a.seed, [10.0 ** -k for k in range(k0, k1 + 1)],
                 list(range(a.pmin, a.pmax + 1)), a.precision, a.n_leaf)
    md = to_markdown(g)
    if a.out:
        with open(a.out, "w") as f:
            f.write(md + "\n")
    else:
        print(md)
    if a.json:
        with open(a.json, "w") as f:
            json.dump(g, f)


if __name__ == "__main__":
    main()
