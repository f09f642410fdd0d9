#!/usr/bin/env python3
"""Throughput of the layered-media Taylor-expansion FMM on one MI355X.

A step is one tefmm_evaluate call: the whole hot path (P2M, M2M, Helmholtz
reduction, M2L of every family on the matrix cores, expansion, L2L, L2P, P2P,
scaling, un-permute) over one charge vector of the workload, with the
particles and the derivative tables already resident in HBM.  Setup (tree,
complex-image fits, tables) is reported separately.

Default workload: N = 1,000,000 particles uniform in the unit cube centred at
(0, 0, -0.6) inside the three-layer medium (interfaces 0 and -1.2, k = 0.8,
1.5, 2.0), one complex charge vector; seeded synthetic data.  Three modes are
timed: the plain FP64 FMM (p = 13, relative error <= 1e-6 at this size), and the mixed
FP32 FMM (complex FP32 M2L and P2P, FP64 tables and accumulation) at p = 7 and at
p = 8, each with a Sigma-table surrogate of its order attached (its validated cells
answer table rows, the rest fall back to the complex images); `value` is the mode
named by --headline (the fastest form within 1e-4: surrogate + mixed FP32 at p = 7;
the surrogate changes the set-up, not the evaluation).

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "target evals/sec at N=1M, rel err≤1e-4: surrogate+FP32 vs plain FP64 FMM"
PEAK = {"fp64": 78.6, "fp32": 157.3}  # TFLOP/s, MI355X published: dense MFMA, and the vector ALUs alike
# algorithmic flops of one P2P pair: distance (3 sub, 3 mul, 2 add), 1/r and r (2),
# k r (1), sin and cos (2), exp(ikr)/r (2), complex multiply-add into the sum (8)
P2P_FLOPS_PER_PAIR = 23
# one charge vector: the pairs of particles in different leaves are evaluated once and
# applied both ways: distance 8, 1/r and r 2, k r 1, sin and cos 2, e^{ikr}/r 2,
# two complex multiply-adds 16
P2P_FLOPS_PER_SYM_PAIR = 31
SHAPES = {"c1": "uniform unit cube centred (0,0,-0.6)", "c2": "uniform unit cube centred (0,0,-0.6)",
          "c4": "uniform unit cube centred (0,0,-0.6)", "c5": "uniform unit cube centred (0,0,-0.6)",
          "c3": "split over three unit cubes centred (0,0,0.6), (0,0,-0.6), (0,0,-1.8), one per layer",
          "ex2": "in the Example-2 domain r = 1/2 - a + a P4(cos theta), a = 0.15, centred (0,0,-0.6)"}


def _sampled_error(workload, phi):
    """Relative 2-norm error on the targets whose oracle values are stored (if any), and the
    largest relative error of one target among them (Err_2 and Err_max of the paper's tests)."""
    import numpy as np
    name = {"c4": "c4s", "c2": "c2s", "c1": "c1", "c3": "c3s", "ex2": "ex2s"}.get(workload)
    path = os.path.join(ROOT, "tests", "golden", f"expected_{name}.txt") if name else None
    if not path or not os.path.exists(path):
        return None, None, 0
    a = np.loadtxt(path)
    idx = a[:, 0].astype(int)
    ref = a[:, 1] + 1j * a[:, 2]
    got = phi[idx]
    return (float(np.linalg.norm(got - ref) / np.linalg.norm(ref)),
            float(np.max(np.abs(got - ref) / np.abs(ref))), len(idx))


def run_mode(xyz, q, p, precision, max_leaf, steps, warmup, workload, surrogate=False, autotune=True):
    import torch
    from paper_1902_05875_amd import api, inputs
    f = api.TEFMM(inputs.MEDIUM_K, inputs.MEDIUM_D, p=p, precision=precision, max_leaf=max_leaf,
                  n_rhs_max=max(64, q.shape[0]))
    sur_info = None
    if surrogate:
        # trained once per medium and layer (untimed, like the rest of the setup), then attached
        t0 = time.perf_counter()
        sur = api.Surrogate(inputs.MEDIUM_K, inputs.MEDIUM_D, 1, p=p)
        sur_info = {"train_wall_s": round(time.perf_counter() - t0, 3), **{k: sur.report[k] for k in (
            "t_data_s", "t_train_s", "final_loss", "max_cell_err", "cells_ok", "cells_total", "n_params")},
            "budget": sur.options["budget"], "n_train": sur.options["n_train"], "epochs": sur.options["epochs"]}
        f.set_surrogate(sur)
    stream = torch.cuda.current_stream()
    xt = torch.from_numpy(xyz).cuda()
    qt = torch.from_numpy(q).cuda()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    f.set_particles(xt)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    tuned = None
    if autotune:
        # depth (occupancy vs far-field work) and M2L tile width, chosen by timing (untimed setup)
        t0 = time.perf_counter()
        tuned = f.autotune()
        torch.cuda.synchronize()
        tuned = {"depth": tuned[0], "m2l_tile": tuned[1], "autotune_s": round(time.perf_counter() - t0, 3)}
    out = torch.empty_like(qt)
    for _ in range(warmup):
        f.evaluate(qt, out=out)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    f.reset_timers()  # phase times below average over exactly the timed evaluations
    ev0.record(stream)
    for _ in range(steps):
        f.evaluate(qt, out=out)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / steps
    # per-phase kernel times: library HIP events on the evaluate stream, recorded inside
    # every timed evaluation and averaged over them
    st = f.stats()
    assert st["timed_evaluations"] == min(steps, 64)
    phases = {k: st[k] for k in ("t_p2m_ms", "t_m2m_ms", "t_m2l_ms", "t_l2l_ms", "t_l2p_ms", "t_p2p_ms", "t_total_ms")}
    phi = out[0].cpu().numpy() if out.dim() == 2 else out.cpu().numpy()
    err, err_max, nchk = _sampled_error(workload, phi)
    n_eval = q.shape[0] * q.shape[1] if q.ndim == 2 else xyz.shape[0]
    res = {
        "p": p, "precision": precision, "ms_per_step": ms, "setup_s": setup_s,
        "evals_per_s": n_eval / (ms / 1e3),
        # set-up (tree, image fits, tables) spread over 1, 10, 100 evaluations of one geometry, as an
        # iterative solver applies the operator; the autotuner's trial runs are not included
        "amortised_evals_per_s": {str(m): n_eval * m / (setup_s + m * ms / 1e3) for m in (1, 10, 100)},
        "phases_ms": {k[2:-3]: round(v, 4) for k, v in phases.items()},
        "m2l_flops": st["m2l_flops"], "m2l_launches": st["m2l_launches"], "depth": st["depth"][0],
        "p2p_flops": _p2p_flops(st, precision, q), "p2p_sym": _p2p_sym(precision, q),
        "n_groups": sum(1 for d in st["depth"] if d),
        "images": st["n_images"], "p2p_pairs": st["p2p_pairs"], "p2p_pairs_same_leaf": st["p2p_pairs_same_leaf"],
        "p2p_poly_err": st["p2p_poly_err"],
        "rel_err_sampled": err, "err_max_sampled": err_max, "n_checked": nchk, "t_setup_tables_ms": st["t_setup_tables_ms"],
        "sigma_keys": st["sigma_keys"], "surrogate_keys": st["surrogate_keys"], "surrogate": sur_info,
        "cross_pairs": st["cross_pairs"], "autotune": tuned, "workload": workload,
        "mean_leaf_occupancy": round(xyz.shape[0] / max(1, st["occupied_leaves"]), 2),
        "max_leaf_count": st["max_leaf_count"], "sigma_direct_pairs": st["sigma_direct_pairs"],
    }
    f.close()
    del xt, qt, out
    torch.cuda.empty_cache()
    return res


def _p2p_sym(precision, q):
    """Whether the near field ran the kernel that evaluates each cross-leaf pair once
    (the default with one charge vector, in both precisions)."""
    return q.ndim == 1 or q.shape[0] == 1


def _p2p_flops(st, precision, q):
    """Algorithmic near-field flops of one evaluation (per charge vector: pairs times flops)."""
    pairs, same = st["p2p_pairs"], st["p2p_pairs_same_leaf"]
    if _p2p_sym(precision, q):
        return P2P_FLOPS_PER_SYM_PAIR * (pairs - same) // 2 + P2P_FLOPS_PER_PAIR * same
    return P2P_FLOPS_PER_PAIR * pairs * (1 if q.ndim == 1 else q.shape[0])


def _traffic(kernel, prec, src, workload):
    """HBM bytes per launch of `kernel` from the committed counter summary (FETCH_SIZE and
    WRITE_SIZE runs, each scaled by the same counter on a copy of known size), if the
    kernel's source is unchanged since the counters were taken; else None."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{prec}_{workload}.md")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and line.startswith("- "):
            k, v = line[2:].split(":", 1)
            vals[k.strip()] = v.strip()
    sha = hashlib.sha256(open(os.path.join(ROOT, "paper_1902_05875_amd", "csrc", src), "rb").read()).hexdigest()
    if vals.get("source_sha256") != sha:
        return None
    return float(vals["hbm_bytes_per_launch"])


def roofline(head):
    """Roofline of the dominant kernel (the larger of the P2P and M2L phases) and of the other."""
    prec = "fp32" if head["precision"] == "fp32" else "fp64"
    ph = head["phases_ms"]
    n_launch = max(1, head["n_groups"])
    if head.get("p2p_sym"):
        same = head["p2p_pairs_same_leaf"]
        what = (f"k_p2p_sym<{'float' if prec == 'fp32' else 'double'}> + k_p2p_sym_gather (vector ALU), {n_launch} launch(es)/step, avg "
                f"{ph['p2p'] / n_launch:.3f} ms; {P2P_FLOPS_PER_SYM_PAIR} flop x {(head['p2p_pairs'] - same) // 2} "
                f"cross-leaf pairs (each once) + {P2P_FLOPS_PER_PAIR} flop x {same} same-leaf ordered pairs"
                + (" (FP32 pair value from quadratics in r^2)" if head.get("p2p_poly_err") else ""))
    else:
        what = (f"k_p2p<{'float' if prec == 'fp32' else 'double'}> (vector ALU), {n_launch} launch(es)/step, "
                f"avg {ph['p2p'] / n_launch:.3f} ms; {P2P_FLOPS_PER_PAIR} flop per pair x {head['p2p_pairs']} pairs")
    p2p = {"bound": "alu", "achieved": head["p2p_flops"] / (ph["p2p"] / 1e3) / 1e12 if ph["p2p"] > 0 else 0.0,
           "peak": PEAK[prec], "unit": "TFLOP/s", "kernel": what}
    m2l = {"bound": "mfma", "achieved": head["m2l_flops"] / (ph["m2l"] / 1e3) / 1e12 if ph["m2l"] > 0 else 0.0,
           "peak": PEAK[prec], "unit": "TFLOP/s",
           "kernel": f"k_m2l ({prec.upper()} MFMA 16x16x4), {head['m2l_launches']} launch(es)/step, "
                     f"avg {ph['m2l'] / max(1, head['m2l_launches']):.3f} ms; 8 (p+1)^4 flop per box pair"}
    wl = head["workload"]
    tp = _traffic("k_p2p_sym" if head.get("p2p_sym") else "k_p2p", prec, "fmm_kernels.hip", wl)
    tm = _traffic("k_m2l", prec, "fmm_m2l.hip", wl)
    p2p["traffic"] = tp
    m2l["traffic"] = tm
    for r in (p2p, m2l):
        r["achieved"] = round(r["achieved"], 3)
        r["frac"] = round(r["achieved"] / r["peak"], 4)
    return (p2p, m2l) if ph["p2p"] >= ph["m2l"] else (m2l, p2p)


def _cpu_sample(workload, n, procs):
    """The bounded oracle sample: a random eighth of the sources (at least 2000) and one
    target among them per worker (seeded: every worker rebuilds the same sample)."""
    import numpy as np
    from paper_1902_05875_amd import inputs
    xyz, q = inputs.workload(workload, n=n)
    if q.ndim == 2:
        q = q[:, 0]
    N = xyz.shape[0]
    n_sub = max(2000, N // 8)
    rng = np.random.default_rng(77)
    src = np.sort(rng.choice(N, size=n_sub, replace=False))
    targets = rng.choice(src, size=procs, replace=False)
    return xyz[src], q[src], [int(np.searchsorted(src, t)) for t in targets], N, n_sub


def cpu_baseline(workload, n):
    """The oracle (direct sum with Sommerfeld quadrature), unchanged, on the host cores: each
    worker process (a child of its own, one BLAS thread) evaluates one target against a random
    eighth of the sources and times its own computation; the per-target time is scaled to all
    N sources.  The workers are plain subprocesses, all waited for."""
    import subprocess
    import numpy as np
    procs = max(1, min(16, os.cpu_count() or 1))
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    cmd = [sys.executable, os.path.abspath(__file__), "--workload", workload, "--cpu-procs", str(procs)]
    if n:
        cmd += ["--n", str(n)]
    t0 = time.perf_counter()
    workers = [subprocess.Popen(cmd + ["--cpu-worker", str(k)], env=env, stdout=subprocess.PIPE, text=True)
               for k in range(procs)]
    outs = [json.loads(w.communicate()[0].strip().splitlines()[-1]) for w in workers]
    wall = time.perf_counter() - t0
    if any(w.returncode != 0 for w in workers):
        raise RuntimeError("cpu baseline worker failed")
    secs = [o["secs"] for o in outs]
    N, n_sub = outs[0]["N"], outs[0]["n_sub"]
    per_target = float(np.mean(secs)) * (N / n_sub)  # one core, one target, all N sources
    return {"value": procs / per_target, "unit": "evals/s", "cores": procs, "kind": "oracle",
            "sample": f"{procs} worker processes x 1 target each against {n_sub} of the {N} sources "
                      f"(free + reaction direct sum, one BLAS thread each); mean compute "
                      f"{np.mean(secs):.1f} s per worker, scaled by N/{n_sub}; wall {wall:.1f} s"}


def _cpu_worker(workload, n, procs, k):
    """One oracle target of the bounded sample (no GPU use); prints its compute time."""
    import numpy as np
    from oracle import direct
    from oracle.medium import Medium
    from paper_1902_05875_amd import inputs
    xyz, q, tg, N, n_sub = _cpu_sample(workload, n, procs)
    t0 = time.perf_counter()
    direct.potential(Medium(inputs.MEDIUM_K, inputs.MEDIUM_D), xyz, q, np.array([tg[k]]))
    print(json.dumps({"secs": time.perf_counter() - t0, "N": N, "n_sub": n_sub}))


def _c5g_error(outs):
    """Err_2 and Err_max against the oracle's stored values of the 16 geometries (16 targets
    each; tests/golden/expected_c5g.txt), or None without them."""
    import numpy as np
    path = os.path.join(ROOT, "tests", "golden", "expected_c5g.txt")
    if not os.path.exists(path):
        return None
    a = np.loadtxt(path)
    got, ref = [], []
    for g, o in enumerate(outs):
        rows = a[a[:, 0] == g]
        got.append(o.cpu().numpy()[rows[:, 1].astype(int)])
        ref.append(rows[:, 2] + 1j * rows[:, 3])
    got, ref = np.concatenate(got), np.concatenate(ref)
    return {"err_2": float(np.linalg.norm(got - ref) / np.linalg.norm(ref)),
            "err_max": float(np.max(np.abs(got - ref) / np.abs(ref))), "targets": int(ref.size)}


def run_batch(steps, warmup, p):
    """C5: (i) one geometry of 500,000 particles with 32 charge vectors; (ii) 16 geometries of
    10k-300k particles evaluated together through tefmm_evaluate_batch (one HIP graph) and
    through tefmm_evaluate_batch_queue (the near fields in one persistent launch), against the
    same 16 evaluated one after another, each path's result checked against the oracle's
    stored values.  Mixed FP32, autotuned per geometry."""
    import numpy as np
    import torch
    from paper_1902_05875_amd import api, inputs
    res = {}
    xyz, q = inputs.workload("c5")
    qm = np.ascontiguousarray(q.T)
    r = run_mode(xyz, qm, p, "fp32", 64, steps, warmup, "c5", surrogate=False, autotune=True)
    res["multi_rhs"] = {"n": xyz.shape[0], "n_rhs": qm.shape[0], "ms_per_step": r["ms_per_step"],
                        "evals_per_s": r["evals_per_s"], "depth": r["depth"], "autotune": r["autotune"]}
    geoms = inputs.c5_geometries()
    hs, qs, outs = [], [], []
    t0 = time.perf_counter()
    for xyz_g, q_g in geoms:
        f = api.TEFMM(inputs.MEDIUM_K, inputs.MEDIUM_D, p=p, precision="fp32")
        f.set_particles(xyz_g)
        f.autotune()
        hs.append(f)
        qs.append(torch.from_numpy(q_g).cuda())
        outs.append(torch.empty_like(qs[-1]))
    torch.cuda.synchronize()
    setup = time.perf_counter() - t0
    ntot = sum(x.shape[0] for x, _ in geoms)
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for _ in range(warmup):
        api.evaluate_batch(hs, qs, outs)
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(steps):
        api.evaluate_batch(hs, qs, outs)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms_b = ev0.elapsed_time(ev1) / steps
    err_b = _c5g_error(outs)
    # the near fields of all 16 geometries in one persistent launch (work queue), far
    # fields on per-geometry streams beside it
    for _ in range(warmup):
        api.evaluate_batch(hs, qs, outs, queue=True)
    api.batch_check(hs[0])
    ev0.record(stream)
    for _ in range(steps):
        api.evaluate_batch(hs, qs, outs, queue=True)
    ev1.record(stream)
    torch.cuda.synchronize()
    api.batch_check(hs[0])
    ms_q = ev0.elapsed_time(ev1) / steps
    err_q = _c5g_error(outs)
    for f, qg, og in zip(hs, qs, outs):
        f.evaluate(qg, out=og)
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(steps):
        for f, qg, og in zip(hs, qs, outs):
            f.evaluate(qg, out=og)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms_s = ev0.elapsed_time(ev1) / steps
    res["geometries"] = {"count": len(geoms), "n_total": ntot, "sizes": [int(x.shape[0]) for x, _ in geoms],
                         "ms_per_step_batched": ms_b, "ms_per_step_queue": ms_q, "ms_per_step_one_by_one": ms_s,
                         "evals_per_s_batched": ntot / (ms_b / 1e3), "evals_per_s_queue": ntot / (ms_q / 1e3),
                         "err_vs_oracle_batched": err_b, "err_vs_oracle_queue": err_q, "setup_s": round(setup, 3)}
    for f in hs:
        f.close()
    return res


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c4",
                    help="c4: N=1M mid-layer cube (default); c2: N=200k; c3: N=1M over three layers; "
                         "ex2: N=1M in the Example-2 domain; c5: the batched workload (its own JSON line)")
    ap.add_argument("--n", type=int, default=None, help="override N (same recipe)")
    ap.add_argument("--p64", type=int, default=13, help="Taylor order of the plain FP64 mode")
    ap.add_argument("--p32", type=int, default=7,
                    help="Taylor order of the mixed FP32 mode (the smallest meeting 1e-4 at N = 1M: "
                         "relative 2-norm error 3.7e-5 over all targets against FP64 p = 13)")
    ap.add_argument("--max-leaf", type=int, default=64)
    ap.add_argument("--n-rhs", type=int, default=1)
    ap.add_argument("--headline", choices=["fp32", "fp64"], default="fp32")
    ap.add_argument("--modes", default="fp64,fp32,fp32_p8",
                    help="comma-separated: fp64 (order --p64), fp32 (order --p32), fp32_pN (mixed at order N)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-surrogate", action="store_true", help="FP32 mode without the Sigma-table surrogate")
    ap.add_argument("--no-autotune", action="store_true", help="keep the occupancy-based depth and tile width")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="first run one device copy of this many MiB (calibrates HBM counters under a profiler)")
    ap.add_argument("--cpu-worker", type=int, default=None, help=argparse.SUPPRESS)
    ap.add_argument("--cpu-procs", type=int, default=1, help=argparse.SUPPRESS)
    args = ap.parse_args()
    if args.cpu_worker is not None:
        _cpu_worker(args.workload, args.n, args.cpu_procs, args.cpu_worker)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU decomposition "
              f"is a design, not a build", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    from paper_1902_05875_amd import inputs
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.calib_copy_mib > 0:
        src = torch.ones(args.calib_copy_mib * (1 << 18), dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.workload == "c5":
        b = run_batch(args.steps, args.warmup, args.p32)
        ms = b["multi_rhs"]["ms_per_step"] + b["geometries"]["ms_per_step_batched"]
        evals = b["multi_rhs"]["n"] * b["multi_rhs"]["n_rhs"] + b["geometries"]["n_total"]
        print(json.dumps({
            "metric": "target evals/sec, batched: 500k particles x 32 charge vectors + 16 geometries (10k-300k)",
            "value": evals / (ms / 1e3), "unit": "evals/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
            "config": {"workload": "c5: 500,000 uniform in the mid-layer cube with 32 complex charge vectors, plus "
                                   "16 geometries log-uniform in [1e4, 3e5] (cubes and Example-2 domains), 3 layers",
                       "p": args.p32, "precision": "fp32", "parallelism": "single GPU"},
            "batch": b}))
        return
    xyz, q = inputs.workload(args.workload, n=args.n, n_rhs=args.n_rhs)
    qm = q.reshape(1, -1) if q.ndim == 1 else np.ascontiguousarray(q.T)
    N = xyz.shape[0]
    modes = {}
    for m in args.modes.split(","):
        # "fp32_p8": the mixed mode at another order (the surrogate configuration's p = 8)
        prec, _, po = m.partition("_p")
        p = int(po) if po else (args.p64 if prec == "fp64" else args.p32)
        print(f"[bench] mode {m} p={p} N={N} n_rhs={qm.shape[0]}", file=sys.stderr, flush=True)
        modes[m] = run_mode(xyz, qm, p, prec, args.max_leaf, args.steps, args.warmup, args.workload,
                            surrogate=(prec == "fp32" and not args.no_surrogate and args.workload != "c3"),
                            autotune=not args.no_autotune)
        print(f"[bench] {m}: {modes[m]['ms_per_step']:.2f} ms/step, err {modes[m]['rel_err_sampled']}",
              file=sys.stderr, flush=True)
    head = modes[args.headline] if args.headline in modes else next(iter(modes.values()))
    roof, roof_other = roofline(head)
    cpu = None
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        cpu = cpu_baseline(args.workload, args.n)
    line = {
        "metric": METRIC, "value": head["evals_per_s"] * 1.0, "unit": "evals/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": head["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64" if head["precision"] == "fp32" else "f64", "data": "synthetic",
        "config": {"workload": f"{args.workload}: N={N} {SHAPES.get(args.workload, '')}, 3 layers "
                               f"(d=0,-1.2; k=0.8,1.5,2.0), {qm.shape[0]} complex charge vector(s)",
                   "p": head["p"], "precision": head["precision"],
                   "mean_leaf_occupancy": head["mean_leaf_occupancy"], "max_leaf_count": head["max_leaf_count"],
                   "depth": head["depth"], "m2l_tile": (head["autotune"] or {}).get("m2l_tile"),
                   "parallelism": "single GPU"},
        "roofline": roof, "roofline_other": roof_other, "cpu_baseline": cpu,
        "headline_form": (f"mixed FP32 p={head['p']}" + (f", {head['surrogate_keys']} surrogate rows"
                                                           if head.get("surrogate_keys") else ", no surrogate rows")),
        "modes": modes,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
