#!/usr/bin/env python3
"""Benchmark: force evaluations per second of the gfx950 FMM at N = 2^20.

One step = one full force evaluation (fmm_forces: tree build, upward pass,
scalar-force estimate, dual-tree walk, M2L, L2L, L2P + P2P, unpermuted
outputs) on a seeded Plummer sphere already resident in HBM.  Prints ONE JSON
line.  Also reports:
  * the force error (median / 99th percentile of |a - a_direct| / |a_direct|)
    on 4096 seeded sinks against a compensated FP64 direct sum on the GPU;
  * the roofline of the dominant kernel (achieved algorithmic FLOP/s against
    the MI355X peak of its precision), timed with HIP events on the stream the
    library launches on, averaged over the timed steps;
  * the CPU oracle on the same host: one full evaluation of the same
    workload, and the 4096-body configuration with all threads and with one.
The timed calls run back to back; the per-kernel durations (HIP events the
library records around its kernels, read by fmm_stats) come from a second pass
of the same calls, each followed by a stats read.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64 = 78.6e12      # MI355X dense FP64 (vector and matrix), FLOP/s
PEAK_FP32 = 157.3e12     # MI355X FP32 vector, FLOP/s
PEAK_HBM = 8.0e12        # bytes/s


def swap_nnz(n):
    """non-zeros of the order-n swap matrix: Re parts couple when m + m' + n is
    even, Im parts when it is odd"""
    c = sum(1 for a in range(n + 1) for b in range(n + 1) if (a + b + n) % 2 == 0)
    s = sum(1 for a in range(1, n + 1) for b in range(1, n + 1) if (a + b + n) % 2 == 1)
    return c + s


def m2l_flops(p):
    """Algorithmic FLOPs of one directed rotation-based M2L: 4 swap-matrix
    products (2 per non-zero), 4 z-rotations (6 per complex coefficient with
    m >= 1) and the z-translation (2 per multiply-add)."""
    swaps = 4 * 2 * sum(swap_nnz(n) for n in range(p + 1))
    rots = 4 * 6 * sum(n for n in range(p + 1))
    trans = 0
    for n in range(p + 1):
        trans += 2 * (p - n + 1)
        for m in range(1, min(n, p - n) + 1):
            trans += 2 * 2 * (p - n - m + 1)
    return swaps + rots + trans


P2P_FLOPS = 20   # per directed body pair: acc + pot, softened, rsqrt counted once

# HBM bytes per launch of a kernel from rocprofv3 FETCH_SIZE and WRITE_SIZE runs,
# each scaled by what the counter reads for a plain device copy of known size
# (fetch x2.0, write x1.0).  Keyed by (kernel, workload, precision); valid only
# while the kernel's source file has the recorded SHA-1 (else reported as null).
MEASURED_TRAFFIC = {
    ("k_m2l_fp32", "plummer_1m", "mixed"): (1597.0e6, "paper_2012_02207_amd/csrc/m2l_mixed.hip",
                                             "ed1126117fe88dda26a2bd2bc1bd2d18ba1f497b"),
    ("k_leaf_group<true> (mixed P2P)", "plummer_1m", "mixed"): (666.0e6,
                                                                "paper_2012_02207_amd/csrc/local.hip",
                                                                "babcf4bb55be7a5c3c74f1314c40e02ccec38c25"),
}


def measured_traffic(kernel, workload, precision):
    import hashlib
    rec = MEASURED_TRAFFIC.get((kernel, workload, precision))
    if rec is None:
        return None
    nbytes, src, sha = rec
    try:
        with open(os.path.join(ROOT, src), "rb") as f:
            cur = hashlib.sha1(f.read()).hexdigest()
    except OSError:
        return None
    return nbytes if cur == sha else None


SORT_PASSES = 8          # LSD passes of 8 bits over the 63-bit Morton keys
SORT_BYTES = 24          # per body and pass: read key (8) + index (4), write both
GATHER_BYTES = 36 + 64   # per body: read index, position, mass; write SoA x, y, z, m and packed (x, y, z, m)


def hbm_rates(stages, n):
    """Algorithmic HBM rates of the tree stage's bandwidth-bound passes: the
    stable radix sort of the bodies' keys and the gather into sorted order,
    from the library's HIP events around them (averaged over the calls)."""
    out = {}
    for name, per_body in (("body_sort", SORT_PASSES * SORT_BYTES), ("gather", GATHER_BYTES)):
        key = "ms_sort" if name == "body_sort" else "ms_gather"
        ms = float(np.mean([s[key] for s in stages]))
        nbytes = per_body * n
        rate = nbytes / (ms * 1e-3) if ms > 0 else 0.0
        out[name] = {"bytes": nbytes, "bytes_per_body": per_body, "ms": ms, "GB/s": rate / 1e9,
                     "frac": rate / PEAK_HBM}
    out["peak_GB/s"] = PEAK_HBM / 1e9
    return out


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


_ORACLE_C1_SNIPPET = r"""
import json, sys, time
sys.path.insert(0, {root!r})
import oracle
from paper_2012_02207_amd import workloads as W
cfg = W.CONFIGS["plummer_4k"]
pos, _, mass = W.plummer(cfg["n"], cfg["seed"])
o = oracle.Oracle()
o.run(pos, mass, p=cfg["p"], err_tol=cfg["err_tol"], n_leaf=64)
ts = []
for _ in range(3):
    t0 = time.perf_counter()
    o.run(pos, mass, p=cfg["p"], err_tol=cfg["err_tol"], n_leaf=64)
    ts.append(time.perf_counter() - t0)
print(json.dumps({{"median_s": sorted(ts)[1], "threads": oracle.threads()}}))
"""


def _oracle_c1_single_thread():
    """The 4096-body configuration in a child process pinned to one OpenMP
    thread (median of 3 runs)."""
    import subprocess
    env = dict(os.environ, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, "-c", _ORACLE_C1_SNIPPET.format(root=ROOT)], env=env,
                       capture_output=True, text=True, timeout=600)
    if r.returncode != 0:
        return None
    return json.loads(r.stdout.strip().splitlines()[-1])


def cpu_baseline(pos, mass, p, err_tol, n_leaf, workload):
    """The CPU oracle, untuned, on this host: one full force evaluation of the
    benchmark's workload (all stages, every body), plus the 4096-body
    configuration (p = 6, epsilon = 1e-6) timed as the median of 3 runs with
    all threads and with one thread."""
    import oracle
    from paper_2012_02207_amd import workloads as W
    n = len(mass)
    o = oracle.Oracle()
    t0 = time.perf_counter()
    o.run(pos, mass, p=p, err_tol=err_tol, n_leaf=n_leaf)
    t_full = time.perf_counter() - t0
    cfg = W.CONFIGS["plummer_4k"]
    p4, _, m4 = W.plummer(cfg["n"], cfg["seed"])
    o4 = oracle.Oracle()
    o4.run(p4, m4, p=cfg["p"], err_tol=cfg["err_tol"], n_leaf=64)  # first touch
    ts = []
    for _ in range(3):
        t0 = time.perf_counter()
        o4.run(p4, m4, p=cfg["p"], err_tol=cfg["err_tol"], n_leaf=64)
        ts.append(time.perf_counter() - t0)
    single = _oracle_c1_single_thread()
    return {"value": 1.0 / t_full, "unit": "force evals/s", "cores": oracle.threads(), "kind": "oracle",
            "sample": f"one full oracle force evaluation of the {workload} workload (N={n}, p={p}, "
                      f"eps={err_tol:g}, every stage and body): {t_full:.1f} s",
            "host": {"nproc": os.cpu_count(), "cpu_model": _cpu_model(),
                     "omp_threads": oracle.threads()},
            "plummer_4k": {"median_of_3_s": float(np.median(ts)), "threads": oracle.threads(),
                           "single_thread_median_of_3_s": single["median_s"] if single else None}}


def run_ensemble(args):
    """The batched ensemble: 256 Plummer clusters of log-uniform size in
    [2^10, 2^16], p = 8, epsilon = 1e-6.  One step = one force evaluation of
    every cluster.  The value is cluster evaluations/s of the batched mixed
    form (fmm_forces_batch); beside it the batched FP64 form and the
    sequential per-cluster FP64 and mixed forms (one fmm_forces call per
    cluster), each with its median force error against the direct sum on
    sampled sinks."""
    import torch
    from paper_2012_02207_amd import fmm, workloads as W
    cfg = W.CONFIGS["ensemble_256"]
    p, err_tol = cfg["p"], cfg["err_tol"]
    clusters = W.ensemble(cfg["count"], cfg["seed"])
    sizes = np.array([len(c[2]) for c in clusters], dtype=np.int64)
    off = np.zeros(len(clusters) + 1, dtype=np.int64)
    off[1:] = np.cumsum(sizes)
    n = int(off[-1])
    dev = torch.device("cuda:0")
    dpos = torch.from_numpy(np.concatenate([c[0] for c in clusters])).to(dev)
    dmass = torch.from_numpy(np.concatenate([c[2] for c in clusters])).to(dev)
    views = [(dpos[off[i]:off[i + 1]], dmass[off[i]:off[i + 1]]) for i in range(len(clusters))]
    # error sample: 32 clusters x up to 64 sinks each, direct sum on the GPU
    rng = np.random.default_rng(cfg["seed"] + 99)
    picked = np.sort(rng.choice(len(clusters), 32, replace=False))
    ref = []
    for ci in picked:
        m = int(sizes[ci])
        sk = np.sort(rng.choice(m, min(64, m), replace=False)).astype(np.int32)
        ad, _ = fmm.direct(views[ci][0], views[ci][1], sinks=torch.from_numpy(sk).to(dev))
        ref.append((ci, sk, ad))

    def errors(acc):
        e = []
        for ci, sk, ad in ref:
            a = acc[int(off[ci]) + torch.from_numpy(sk).long().to(dev)]
            e.append((torch.linalg.norm(a - ad, dim=1) / torch.linalg.norm(ad, dim=1)).cpu().numpy())
        e = np.concatenate(e)
        return float(np.median(e)), float(np.percentile(e, 99))

    def run(precision, batched):
        f = fmm.FMM(p=p, err_tol=err_tol, n_leaf=args.n_leaf, precision=precision,
                    root_levels=args.root_levels)
        tuned = None
        if batched and not args.no_autotune:  # the batched forms run at the autotuner's choices
            f.autotune(dpos, dmass, off)
            tuned = {"n_leaf": f.params.n_leaf, "m2l_waves": f.params.m2l_waves,
                     "p2p_groups": f.params.p2p_groups, "p2p_start": f.params.p2p_start}
        acc = torch.empty((n, 3), dtype=torch.float64, device=dev)
        pot = torch.empty((n,), dtype=torch.float64, device=dev)
        outs = [(acc[off[i]:off[i + 1]], pot[off[i]:off[i + 1]]) for i in range(len(clusters))]

        def step():
            if batched:
                f.forces_batch(dpos, dmass, off, out=(acc, pot))
            else:
                for (pp, mm), o in zip(views, outs):
                    f.forces(pp, mm, out=o)
        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        st = []
        if batched:  # stage and kernel times from a second pass, a stats read after each call
            for _ in range(args.steps):
                step()
                st.append(f.stats())
        med, p99 = errors(acc)
        f.close()
        return {"ms": 1e3 * dt, "cluster_evals_per_s": len(clusters) / dt, "particle_evals_per_s": n / dt,
                "median_err_vs_direct": med, "p99_err_vs_direct": p99,
                "n_leaf": tuned["n_leaf"] if tuned is not None else args.n_leaf, "tuned": tuned, "stats": st}

    res = {"batched_mixed": run("mixed", True), "batched_fp64": run("fp64", True),
           "sequential_fp64": run("fp64", False), "sequential_mixed": run("mixed", False)}

    def frozen_loop():
        """Steps that keep the batch's tree (fmm_forces_frozen): eager launches
        against the same sequence replayed as one captured HIP graph."""
        f = fmm.FMM(p=p, err_tol=err_tol, n_leaf=res["batched_mixed"]["n_leaf"], precision="mixed",
                    root_levels=args.root_levels)
        if res["batched_mixed"]["tuned"] is not None:
            f.set_params(**res["batched_mixed"]["tuned"])
        acc = torch.empty((n, 3), dtype=torch.float64, device=dev)
        pot = torch.empty((n,), dtype=torch.float64, device=dev)
        f.forces_batch(dpos, dmass, off, out=(acc, pot))
        out = {}
        for graph in (False, True):
            for _ in range(max(1, args.warmup)):
                f.forces_frozen(dpos, dmass, out=(acc, pot), graph=graph)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                f.forces_frozen(dpos, dmass, out=(acc, pot), graph=graph)
            torch.cuda.synchronize()
            out["graph" if graph else "eager"] = {"ms": 1e3 * (time.perf_counter() - t0) / args.steps}
        f.close()
        out["graph_speedup"] = out["eager"]["ms"] / out["graph"]["ms"]
        return out
    frozen = frozen_loop()
    R = res["batched_mixed"]
    st = R["stats"][-1]
    m2l_ms = float(np.mean([s["ms_m2l_kernel"] for s in R["stats"]]))
    p2p_ms = float(np.mean([s["ms_p2p"] for s in R["stats"]]))
    f_m2l = m2l_flops(p) * st["n_m2l_fp32"]
    f_leaf = P2P_FLOPS * st["n_p2p_pairs"]
    if p2p_ms >= m2l_ms:
        dom = {"kernel": "k_leaf_group<true> (mixed P2P)", "flop": f_leaf, "ms": p2p_ms}
    else:
        dom = {"kernel": "k_m2l_fp32", "flop": f_m2l, "ms": m2l_ms}
    achieved = dom["flop"] / (dom["ms"] * 1e-3)
    forms = {k: {kk: vv for kk, vv in v.items() if kk != "stats"} for k, v in res.items()}
    forms["speedup_batched_mixed_over_sequential_fp64"] = res["sequential_fp64"]["ms"] / R["ms"]
    forms["speedup_batched_fp64_over_sequential_fp64"] = (res["sequential_fp64"]["ms"]
                                                          / res["batched_fp64"]["ms"])
    out = {
        "metric": "cluster force evals/sec, 256 Plummer clusters (N log-uniform in [2^10, 2^16]), p=8, "
                  "1e-6; batched mixed vs sequential FP64 GPU",
        "value": R["cluster_evals_per_s"], "unit": "cluster evals/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": R["ms"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"ensemble_256: {len(clusters)} clusters, N={n}, p={p}, eps={err_tol}, "
                               f"n_leaf={R['n_leaf']}, batched mixed", "clusters": len(clusters),
                   "n": n, "p": p, "err_tol": err_tol, "n_leaf": R["n_leaf"],
                   "root_levels": args.root_levels},
        "particle_evals_per_s": R["particle_evals_per_s"],
        "forms": forms,
        "frozen_tree_steps": frozen,
        "stages_ms": {k: round(float(np.mean([s[k] for s in R["stats"]])), 4)
                      for k in ("ms_tree", "ms_upward", "ms_estimate", "ms_walk", "ms_m2l",
                                "ms_local", "ms_p2p", "ms_total")},
        "roofline": {"bound": "alu", "kernel": dom["kernel"], "achieved": achieved / 1e12,
                     "peak": PEAK_FP32 / 1e12, "unit": "TFLOP/s", "frac": achieved / PEAK_FP32,
                     "traffic": None, "flop_per_launch": dom["flop"], "ms_per_launch": dom["ms"]},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = ensemble_cpu_baseline(clusters, p, err_tol, args.n_leaf)
    print(json.dumps(out))


def run_rollout(args):
    """The differentiable rollout: Plummer N = 2^18, 64 kick-drift-kick steps
    (dt = 1e-3), L = sum |x_T - target|^2 with seeded targets x_0 + 0.01 N(0, 1),
    gradients dL/dx_0, dL/dv_0, dL/dm through the FMM adjoint with checkpoints
    every 8 steps (forces of a segment recomputed in the backward pass, on one
    context per step of the segment and one for the initial forces, so that
    each adjoint reuses its step's tree, lists and expansions).  One
    step of the benchmark = one forward rollout plus its full gradient.  The
    gradient is checked against central differences (h = 1e-6) on 32 seeded
    coordinates of x_0, with every force evaluation of the perturbed rollouts
    keeping the tree and lists of the unperturbed one."""
    import torch
    from paper_2012_02207_amd import rollout as R, workloads as W
    cfg = W.CONFIGS["rollout_256k"]
    n, p, err_tol = cfg["n"], cfg["p"], cfg["err_tol"]
    dt, nsteps, every = 1e-3, 64, 8
    pos, vel, mass = W.plummer(n, cfg["seed"])
    rng = np.random.default_rng(cfg["seed"] + 1)
    target = pos + 0.01 * rng.normal(size=pos.shape)
    dev = torch.device("cuda:0")
    P, V, M, T = (torch.from_numpy(a).to(dev) for a in (pos, vel, mass, target))
    ctxs = [R.make_solver(p=p, err_tol=err_tol, n_leaf=args.n_leaf) for _ in range(every + 1)]

    def step():
        x0, v0, m = (a.clone().requires_grad_(True) for a in (P, V, M))
        xT, _ = R.leapfrog(x0, v0, m, ctxs, dt, nsteps, checkpoint_every=every)
        loss = ((xT - T) ** 2).sum()
        loss.backward()
        return loss.item(), x0.grad, v0.grad, m.grad
    def note(msg):
        print(f"[rollout] {msg}", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        step()
        note("warm-up step done")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        L, gx, gv, gm = step()
        note(f"timed step done ({time.perf_counter() - t0:.2f} s)")
    torch.cuda.synchronize()
    t_step = (time.perf_counter() - t0) / args.steps
    with torch.no_grad():
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        xT, _ = R.leapfrog(P, V, M, ctxs[0], dt, nsteps, checkpoint_every=0)
        torch.cuda.synchronize()
        t_fwd = time.perf_counter() - t0
    # the same gradient without checkpoints: one context per force evaluation
    # (a 2^18-body context holds ~0.6 GB of HBM), so that no forward pass is
    # recomputed and every adjoint reuses its evaluation (fmm_adjoint_last)
    solvers = [R.make_solver(p=p, err_tol=err_tol, n_leaf=args.n_leaf) for _ in range(nsteps + 1)]

    def step_nc():
        x0, v0, m = (a.clone().requires_grad_(True) for a in (P, V, M))
        xT, _ = R.leapfrog(x0, v0, m, solvers, dt, nsteps, checkpoint_every=0)
        ((xT - T) ** 2).sum().backward()
        return x0.grad, v0.grad, m.grad
    step_nc()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        gx2, gv2, gm2 = step_nc()
    torch.cuda.synchronize()
    t_nc = (time.perf_counter() - t0) / args.steps
    same_nc = bool(torch.equal(gx, gx2) and torch.equal(gv, gv2) and torch.equal(gm, gm2))
    ws_nc = sum(s_.stats()["workspace_bytes"] for s_ in solvers)
    note(f"without checkpoints: {1e3 * t_nc:.1f} ms per rollout gradient")
    # finite differences with frozen lists
    R.leapfrog_frozen(P, V, M, solvers, dt, nsteps, record=True)
    note("recorded the lists of every force evaluation")

    def loss_frozen(x):
        xT, _ = R.leapfrog_frozen(x, V, M, solvers, dt, nsteps)
        return ((xT - T) ** 2).sum().item()
    gxn = gx.cpu().numpy()
    h, rels = 1e-6, []
    crng = np.random.default_rng(cfg["seed"] + 2)
    for k in crng.choice(n, 32, replace=False):
        d = int(crng.integers(3))
        e = torch.zeros_like(P)
        e[k, d] = h
        fd = (loss_frozen(P + e) - loss_frozen(P - e)) / (2 * h)
        rels.append(abs(fd - gxn[k, d]) / max(abs(fd), 1e-300))
        note(f"finite difference {len(rels)}/32: rel {rels[-1]:.2e}")
    for s_ in solvers + ctxs:
        s_.close()
    rels = np.array(rels)
    out = {
        "metric": "differentiable rollout: forward + gradient of 64 leapfrog steps at N=2^18 "
                  "(p=10, 1e-7), per second",
        "value": 1.0 / t_step, "unit": "rollout gradients/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * t_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"rollout_256k: N={n}, Plummer, {nsteps} KDK steps, dt={dt}, p={p}, "
                               f"eps={err_tol}, checkpoints every {every} steps", "n": n, "p": p,
                   "err_tol": err_tol, "steps": nsteps, "dt": dt, "checkpoint_every": every},
        "forward_rollout_ms": 1e3 * t_fwd,
        "backward_over_forward": (t_step - t_fwd) / t_fwd,
        "force_evals_per_s_forward": (nsteps + 1) / t_fwd,
        "loss": L,
        "grad_norms": {"x0": float(gx.norm()), "v0": float(gv.norm()), "m": float(gm.norm())},
        "finite_difference_check": {"coords": 32, "h": h, "median_rel": float(np.median(rels)),
                                    "max_rel": float(rels.max())},
        "no_checkpoint": {"ms_per_step": 1e3 * t_nc, "rollout_gradients_per_s": 1.0 / t_nc,
                          "contexts": nsteps + 1, "workspace_gb": ws_nc / 1e9,
                          "gradient_equal_to_checkpointed": same_nc},
    }
    print(json.dumps(out))


def ensemble_cpu_baseline(clusters, p, err_tol, n_leaf, count=8, seed=7):
    """The CPU oracle on a sample of whole clusters, scaled to all of them by
    their share of the bodies."""
    import oracle
    rng = np.random.default_rng(seed)
    picked = rng.choice(len(clusters), count, replace=False)
    t = 0.0
    nb = 0
    for ci in picked:
        pos, _, mass = clusters[ci]
        o = oracle.Oracle()
        t0 = time.perf_counter()
        o.run(pos, mass, p=p, err_tol=err_tol, n_leaf=n_leaf)
        t += time.perf_counter() - t0
        nb += len(mass)
    total = sum(len(c[2]) for c in clusters)
    t_all = t * total / nb
    return {"value": len(clusters) / t_all, "unit": "cluster evals/s", "cores": oracle.threads(),
            "kind": "oracle",
            "sample": f"{count} random clusters ({nb} bodies) evaluated in full ({t:.1f} s), scaled by "
                      f"the body share to all {len(clusters)} clusters ({total} bodies): "
                      f"{t_all:.1f} s per ensemble evaluation"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="plummer_1m",
                    choices=["plummer_1m", "plummer_4k", "kroupa_4m", "ensemble_256", "rollout_256k"])
    ap.add_argument("--precisions", default="fp64,mixed",
                    help="comma list; the last one is the reported value")
    ap.add_argument("--root-levels", type=int, default=3)
    ap.add_argument("--n-leaf", type=int, default=64)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true", help="ensemble: keep --n-leaf for batched forms")
    ap.add_argument("--err-sinks", type=int, default=4096)
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only copy a MIB-MiB device buffer 5 times (calibrates byte counters)")
    args = ap.parse_args()
    if args.copy_probe:
        import torch
        a = torch.ones(args.copy_probe << 18, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_per_copy": a.numel() * 4, "copies": 5}))
        return
    args.precisions = [x for x in args.precisions.split(",") if x]
    if args.gpus != 1:
        print(json.dumps({"error": "the force pass runs on one GPU; runs over several GPUs "
                                   "are not supported (use --gpus 1)"}))
        sys.exit(2)

    import torch
    from paper_2012_02207_amd import fmm, workloads as W

    if args.workload == "ensemble_256":
        return run_ensemble(args)
    if args.workload == "rollout_256k":
        return run_rollout(args)
    cfg = W.CONFIGS[args.workload]
    n, p, err_tol = cfg["n"], cfg["p"], cfg["err_tol"]
    if args.workload == "kroupa_4m":
        pos, _, mass = W.kroupa_with_central(n, cfg["seed"])
    else:
        pos, _, mass = W.plummer(n, cfg["seed"])
    dev = torch.device("cuda:0")
    dpos = torch.from_numpy(pos).to(dev)
    dmass = torch.from_numpy(mass).to(dev)
    rng = np.random.default_rng(cfg["seed"] + 99)
    sinks = np.sort(rng.choice(n, min(args.err_sinks, n), replace=False)).astype(np.int32)
    dsinks = torch.from_numpy(sinks).to(dev)
    ad, _ = fmm.direct(dpos, dmass, sinks=dsinks)

    def run(precision):
        f = fmm.FMM(p=p, err_tol=err_tol, n_leaf=args.n_leaf, precision=precision,
                    root_levels=args.root_levels)
        acc = torch.empty((n, 3), dtype=torch.float64, device=dev)
        pot = torch.empty((n,), dtype=torch.float64, device=dev)
        for _ in range(args.warmup):
            f.forces(dpos, dmass, out=(acc, pot))
        torch.cuda.synchronize()
        # timed region: back-to-back calls, nothing read in between
        t0 = time.perf_counter()
        for _ in range(args.steps):
            f.forces(dpos, dmass, out=(acc, pot))
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        # the same calls again, each followed by fmm_stats (a stream sync and
        # read-back of the library's HIP events: stage times and the per-launch
        # durations of the M2L and near-field kernels)
        stage_ms = []
        t1 = time.perf_counter()
        for _ in range(args.steps):
            f.forces(dpos, dmass, out=(acc, pot))
            stage_ms.append(f.stats())
        torch.cuda.synchronize()
        dt_inst = time.perf_counter() - t1
        a = acc[dsinks.long()]
        rel = (torch.linalg.norm(a - ad, dim=1) / torch.linalg.norm(ad, dim=1)).cpu().numpy()
        f.close()
        return {"ms": 1e3 * dt / args.steps, "ms_instrumented": 1e3 * dt_inst / args.steps,
                "stages": stage_ms, "acc": acc, "rel": rel}

    res = {pr: run(pr) for pr in args.precisions}
    main_pr = args.precisions[-1]
    R = res[main_pr]
    st = R["stages"][-1]
    ms_step = R["ms"]
    rel = R["rel"]

    # dominant kernel roofline: algorithmic FLOPs of one launch / its average
    # duration between HIP events recorded around it on the library's stream
    m2l_ms = np.mean([s["ms_m2l_kernel"] for s in R["stages"]])
    m2l_stage_ms = np.mean([s["ms_m2l"] for s in R["stages"]])
    p2p_ms = np.mean([s["ms_p2p"] for s in R["stages"]])
    n_m2l_main = st["n_m2l"] if main_pr == "fp64" else st["n_m2l_fp32"]
    f_m2l = m2l_flops(p) * n_m2l_main
    f_leaf = P2P_FLOPS * st["n_p2p_pairs"]
    peak = PEAK_FP64 if main_pr == "fp64" else PEAK_FP32
    kname = "k_m2l_fp64" if main_pr == "fp64" else "k_m2l_fp32"
    if p2p_ms >= m2l_ms:
        dom = {"kernel": "k_leaf_group<false> (P2P)" if main_pr == "fp64"
                         else "k_leaf_group<true> (mixed P2P)",
               "flop": f_leaf, "ms": p2p_ms}
    else:
        dom = {"kernel": kname, "flop": f_m2l, "ms": m2l_ms}
    achieved = dom["flop"] / (dom["ms"] * 1e-3)
    # the dominant stages are vector-ALU bound (no dense contraction on this path)
    roof = {"bound": "alu", "kernel": dom["kernel"],
            "achieved": achieved / 1e12, "peak": peak / 1e12, "unit": "TFLOP/s",
            "frac": achieved / peak,
            "traffic": measured_traffic(dom["kernel"], args.workload, main_pr),
            "flop_per_launch": dom["flop"], "ms_per_launch": dom["ms"],
            "note": "M2L and the near field run concurrently on two streams, so each kernel's "
                    "event duration includes time shared with the other; concurrent_phase gives "
                    "their combined algorithmic rate over the phase"}
    # the concurrent evaluation phase: main M2L + root-level FP64 M2L + near
    # field, from the fork to the join (events 4 and 5 on the caller's stream)
    phase_ms = m2l_stage_ms
    f_root = m2l_flops(p) * (st["n_m2l"] - n_m2l_main)
    f_phase = f_m2l + f_root + P2P_FLOPS * st["n_p2p_pairs"]
    roof["concurrent_phase"] = {"kernels": f"{kname} + k_leaf_group ({'mixed' if main_pr != 'fp64' else 'fp64'})"
                                           + (" + k_m2l_fp64 (root levels)" if main_pr != "fp64" else ""),
                                "flop": f_phase, "ms": phase_ms,
                                "achieved": f_phase / (phase_ms * 1e-3) / 1e12,
                                "frac": f_phase / (phase_ms * 1e-3) / peak}
    other = {"m2l_main": {"kernel": kname, "pairs": int(n_m2l_main), "ms": m2l_ms,
                          "tflops": f_m2l / (m2l_ms * 1e-3) / 1e12},
             "m2l_stage_ms": m2l_stage_ms,
             "leaf_eval": {"ms": p2p_ms, "tflops": f_leaf / (p2p_ms * 1e-3) / 1e12}}
    forms = {}
    for pr, r in res.items():
        forms[pr] = {"evals_per_s": 1e3 / r["ms"], "ms_per_eval": r["ms"],
                     "ms_per_eval_with_stats_read": r["ms_instrumented"],
                     "median_err_vs_direct": float(np.median(r["rel"])),
                     "p99_err_vs_direct": float(np.percentile(r["rel"], 99))}
    if "fp64" in res and "mixed" in res:
        a64, amx = res["fp64"]["acc"], res["mixed"]["acc"]
        d = (torch.linalg.norm(amx - a64, dim=1) / torch.linalg.norm(a64, dim=1)).cpu().numpy()
        forms["mixed_vs_fp64"] = {"median": float(np.median(d)), "p99": float(np.percentile(d, 99)),
                                  "max": float(d.max())}
        forms["speedup_mixed_over_fp64"] = res["fp64"]["ms"] / res["mixed"]["ms"]

    out = {
        "metric": ("force evals/sec at N=2^20, 1e-7 median rel. force err; mixed vs FP64 GPU"
                   if args.workload == "plummer_1m" else
                   f"force evals/sec at N={n}, {err_tol:g} median rel. force err; {main_pr}"),
        "value": 1e3 / ms_step,
        "unit": "force evals/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if main_pr == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: N={n}, Henon units, p={p}, eps={err_tol}, "
                               f"n_leaf={args.n_leaf}, precision={main_pr}",
                   "n": n, "p": p, "err_tol": err_tol, "n_leaf": args.n_leaf, "precision": main_pr,
                   "root_levels": args.root_levels},
        "direct_interactions_per_s": n * (n - 1) / (ms_step * 1e-3),
        "force_error": {"median": float(np.median(rel)), "p99": float(np.percentile(rel, 99)),
                        "max": float(rel.max()), "sinks": int(len(sinks))},
        "forms": forms,
        "stages_ms": {k: round(float(np.mean([s[k] for s in R["stages"]])), 4)
                      for k in ("ms_tree", "ms_sort", "ms_gather", "ms_upward", "ms_estimate", "ms_walk",
                                "ms_walk_steps", "ms_m2l", "ms_local", "ms_p2p", "ms_total")},
        "counts": {k: int(st[k]) for k in ("ncell", "nleaf", "depth", "n_m2l", "n_p2p_cells",
                                           "n_p2p_pairs", "n_est_far", "n_est_near")},
        "roofline": roof,
        "kernels": other,
        "hbm": hbm_rates(R["stages"], n),
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(pos, mass, p, err_tol, args.n_leaf, args.workload)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
