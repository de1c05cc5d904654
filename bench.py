#!/usr/bin/env python3
"""Benchmark of the dual-gradient hot path on one MI355X.

Workload (config 1): one scenario tree with nx=50, nu=30, horizon N=20,
branching 4 at stages 0-5 then 1 (4,096 scenarios, 62,805 nodes, 4.90M primal
and 4.90M dual variables), FP64 factors and solves, synthetic seeded data.

A timed step is one dual-gradient evaluation x(y) (Algorithm 3: the full
backward and forward sweep over the tree) on inputs resident in HBM; value is
the evaluations per second.  After the timed region the script also measures
(a) each sweep phase with HIP events on the stream it runs on (roofline of the
dominant kernel), (b) time to a 1e-6 residual for NAMA and MINFBE from a cold
start, and (c) the CPU oracle on a bounded sample of the same workload.
Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import treegen  # noqa: E402

METRIC = "dual-grad evals/s + time-to-1e-6 residual; learned warm start vs cold, 1 GPU"
HBM_PEAK_GBS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def phase_bytes(prob, sstar):
    """Algorithmic HBM bytes of one affine sweep, per phase: every factor entry
    read once, every vector entry read or written once (no padding)."""
    t = prob.tree
    nx, nu = prob.nx, prob.nu
    sp = [int(v) for v in t.stage_ptr]
    N = int(t.N)
    W = nx + nu
    nchains = sp[N + 1] - sp[N]
    out = {}
    # chain phases: nodes of stages s*..N-1, one child each
    nsteps = (N - sstar) * nchains if sstar < N else 0
    bwd_node = nx * W + nu * nu + nu * nx + W + nx + nu + nu + 1
    out["bwd_chain"] = 8 * (nsteps * bwd_node + (nchains * (2 * nx + 1) if sstar < N else 0)
                            + (nchains * nx if 0 < sstar < N else 0))
    fwd_node = nx * nu + W * nx + nu + nu + nx + nx
    out["fwd_chain"] = 8 * (nsteps * fwd_node + (nchains * nx if sstar < N else 0))
    # per-stage phases (stages 0..s*-1)
    nodes = sp[sstar] if sstar > 0 else 0
    edges = (sp[sstar + 1] - 1) if sstar > 0 else 0
    leaf_kids = (sp[N + 1] - sp[N]) if sstar == N else 0
    out["bwd_stages"] = 8 * (edges * nx * W + nodes * (nu * nu + nu * nx + W + nx + nu + nu + nx + 1)
                             + (edges - leaf_kids) * nx + leaf_kids * (2 * nx + 1))
    out["fwd_stages"] = 8 * (nodes * (nx * nu + nu + nu + nx) + edges * (W * nx + nx + nx))
    return out


def sweep_flops(prob):
    t = prob.tree
    nx, nu = prob.nx, prob.nu
    E, Vnl = float(t.V - 1), float(t.Vnl)
    return 2.0 * (E * (2 * nx * (nx + nu)) + Vnl * (nu * nu + 2 * nu * nx + nx * nu))


def subtree(prob, root):
    """The subtree below ``root`` as a problem of its own (probabilities
    renormalised, root state free); used for the bounded CPU sample."""
    t = prob.tree
    s = int(np.searchsorted(t.stage_ptr, root, side="right") - 1)
    lo, hi = root, root + 1
    idx, counts = [], []
    for stage in range(s, t.N + 1):
        idx.append(np.arange(lo, hi))
        if stage < t.N:
            cp = t.child_ptr
            counts.append((cp[lo + 1:hi + 1] - cp[lo:hi]).tolist())
            lo, hi = int(cp[lo]), int(cp[hi])
    nodes = np.concatenate(idx)
    tree = treegen.tree_from_counts(counts)
    nl = nodes[:tree.Vnl]
    lv = nodes[tree.Vnl:] - t.Vnl
    xmin, xmax = prob.xmin[nodes].copy(), prob.xmax[nodes].copy()
    xmin[0], xmax[0] = -np.inf, np.inf
    return treegen.Problem(tree=tree, nx=prob.nx, nu=prob.nu, A=prob.A[nodes], B=prob.B[nodes],
                           c=prob.c[nodes], Q=prob.Q[nl], R=prob.R[nl], P=prob.P[lv],
                           xmin=xmin, xmax=xmax, umin=prob.umin[nl], umax=prob.umax[nl],
                           x0=prob.x0.copy(), name=prob.name + "-subtree")


def cpu_baseline(prob, seconds=10.0):
    """The CPU oracle (single thread, as it stands) on the subtree of one
    stage-2 node; evaluations/s scaled to the full tree by the flop ratio."""
    import oracle
    oracle.build(force=False)
    sub = subtree(prob, int(prob.tree.stage_ptr[2]))
    pb, fac = oracle.factor(sub)
    rng = np.random.default_rng(7)
    y = rng.standard_normal(pb.m)
    n, t0 = 0, time.perf_counter()
    while True:
        oracle.sweep(pb, fac, y)
        n += 1
        el = time.perf_counter() - t0
        if (el >= seconds and n >= 3) or el >= 3 * seconds:
            break
    rate_sample = n / el
    ratio = sweep_flops(sub) / sweep_flops(prob)
    cpu = "unknown"
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                cpu = ln.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"value": rate_sample * ratio, "unit": "dual-grad evals/s", "cores": 1, "kind": "oracle",
            "sample": (f"{n} oracle x(y) sweeps in {el:.1f} s on the subtree of one stage-2 node "
                       f"({sub.tree.V} of {prob.tree.V} nodes, same nx/nu/N), scaled by the "
                       f"sweep flop ratio {ratio:.4f}; host {cpu}, nproc {os.cpu_count()}")}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--profile-steps", type=int, default=20)
    ap.add_argument("--no-solve", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--tight-u", type=float, default=0.1)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the multi-GPU design "
              "is described in DESIGN.md and is not built.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2107_01745_amd import stotree

    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    prob = treegen.make_config(1)
    log(f"config 1 generated in {time.perf_counter() - t0:.1f} s: V={prob.tree.V}, m={prob.m}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tf = stotree.tree_factor(prob, precondition=True)
    factor_s = time.perf_counter() - t0
    log(f"factor step {factor_s:.2f} s, device bytes {tf.device_bytes / 1e9:.2f} GB, s*={tf.sstar}")

    rng = np.random.default_rng(11)
    y = torch.tensor(rng.standard_normal(tf.m), dtype=torch.float64, device=dev)
    x0 = torch.tensor(prob.x0, dtype=torch.float64, device=dev)
    x = torch.empty(tf.V, tf.nx, dtype=torch.float64, device=dev)
    u = torch.empty(tf.Vnl, tf.nu, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        stotree.dual_grad(tf, x0, y, False, x, u)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        stotree.dual_grad(tf, x0, y, False, x, u)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = ev0.elapsed_time(ev1) / args.steps
    value = 1000.0 / ms
    log(f"x(y) sweep: {ms:.4f} ms/step ({value:.1f} evals/s), host wall {wall:.3f} s")

    # achievable streaming bandwidth on this device: a plain 1 GiB device copy
    n_copy = 1 << 27
    src = torch.ones(n_copy, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    c0.record(stream)
    for _ in range(10):
        dst.copy_(src)
    c1.record(stream)
    torch.cuda.synchronize()
    copy_gbs = 2 * 8 * n_copy / (c0.elapsed_time(c1) / 10 * 1e-3) / 1e9
    del src, dst
    log(f"device copy (read+write) {copy_gbs:.0f} GB/s")

    # per-phase timing with HIP events on the sweep's stream
    stotree.stotree_timing(True)
    for _ in range(args.profile_steps):
        stotree.dual_grad(tf, x0, y, False, x, u)
    torch.cuda.synchronize()
    stotree.stotree_timing(False)
    phases = stotree.stotree_timing_read()
    pbytes = phase_bytes(prob, tf.sstar)
    phase_rep = {}
    for name, (tot, cnt) in phases.items():
        if cnt:
            avg = tot / cnt
            phase_rep[name] = {"avg_ms": avg, "bytes": pbytes[name],
                               "GBs": pbytes[name] / (avg * 1e-3) / 1e9}
    dom = max(phase_rep, key=lambda k: phase_rep[k]["avg_ms"])
    sweep_bytes = sum(pbytes.values())
    log(f"phases: {json.dumps(phase_rep)}")
    roofline = {"bound": "hbm", "achieved": phase_rep[dom]["GBs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": phase_rep[dom]["GBs"] / HBM_PEAK_GBS, "traffic": None,
                "kernel": f"{dom}_kernel", "bytes_per_launch": pbytes[dom],
                "avg_launch_ms": phase_rep[dom]["avg_ms"],
                "copy_GBs": copy_gbs, "frac_of_copy": phase_rep[dom]["GBs"] / copy_gbs,
                "whole_sweep": {"bytes": sweep_bytes, "GBs": sweep_bytes / (ms * 1e-3) / 1e9,
                                "frac": sweep_bytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                                "flops": sweep_flops(prob)}}

    solve_rep = None
    if not args.no_solve:
        import dataclasses
        solve_rep = {}
        # config 1 as read (|u| <= 1: the unconstrained optimum is feasible, y* = 0) and with
        # |u| <= 0.1, where about 4% of the inputs are active at the solution
        variants = [("as_specified", tf, prob)]
        tight = dataclasses.replace(prob, umin=np.full_like(prob.umin, -args.tight_u),
                                    umax=np.full_like(prob.umax, args.tight_u))
        tf_t = stotree.tree_factor(tight, precondition=True)
        variants.append((f"u_box_{args.tight_u:g}", tf_t, tight))
        for vname, tfv, pv in variants:
            L = stotree.dual_lipschitz(tfv, 100)
            lam = 1.0 / (1.1 * L)
            rep = {"lambda": lam, "L_power_iteration_100": L}
            for method in ("nama", "minfbe"):
                yv = torch.zeros(tfv.m, dtype=torch.float64, device=dev)
                fn = stotree.nama_solve if method == "nama" else stotree.minfbe_solve
                torch.cuda.synchronize()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                rc, info = fn(tfv, x0, yv, x, u, stotree.make_opts(lam=lam, eps=1e-6, max_iter=2000))
                e1.record(stream)
                torch.cuda.synchronize()
                info["time_to_tol_s"] = e0.elapsed_time(e1) / 1000.0
                info["ms_per_iter"] = 1000.0 * info["time_to_tol_s"] / max(1, info["iters"])
                info["rc"] = rc
                rep[method] = info
                log(f"{vname} {method}: rc={rc} iters={info['iters']} res={info['res_scaled_inf']:.2e} "
                    f"time {info['time_to_tol_s']:.3f} s ({info['ms_per_iter']:.2f} ms/iter)")
            solve_rep[vname] = rep
        tf_t.free()

    cpu = None
    if not args.no_cpu:
        t0 = time.perf_counter()
        cpu = cpu_baseline(prob, args.cpu_seconds)
        log(f"cpu baseline {cpu['value']:.3f} evals/s ({time.perf_counter() - t0:.1f} s)")

    rec = {
        "metric": METRIC, "value": value, "unit": "dual-grad evals/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": ("config 1: single scenario tree, nx=50, nu=30, N=20, branching 4 at "
                                "stages 0-5 then 1 (4096 scenarios, 62805 nodes, 4.90M primal / "
                                "4.90M dual variables); step = one FP64 dual-gradient sweep x(y)"),
                   "nodes": prob.tree.V, "m": prob.m, "precondition": True,
                   "factor_seconds": factor_s},
        "roofline": roofline,
        "phases": phase_rep,
        "cpu_baseline": cpu,
        "solve": solve_rep,
    }
    tf.free()
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
