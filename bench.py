"""Throughput of the per-cell stiff chemistry integration on one MI355X.

One step = one chemistry step of every cell of the workload (all cells
integrated over dt from the same seeded synthetic input batch, resident in
HBM). Prints one JSON line. The metric is cells integrated per second per
chemistry step on the 54-species FP64 workload; the roofline object refers
to the integration kernel, whose algorithmic flops per launch are counted
from the mechanism's structure and each cell's accepted/rejected step counts.
"""
import argparse
import json
import os
import sys
import tempfile
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "cells integrated/s per chemistry step (54-sp FP64), binned persistent vs plain"
FP64_VECTOR_PEAK = 78.6e12        # 256 CU x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz
HBM_PEAK = 8.0e12


def flops_per_launch(work, n, n_acc, n_rej):
    """Algorithmic flops of one chemistry step: per step start an RHS and the
    analytical Jacobian; per attempted step two more RHS, forming M, the LU,
    four triangular solves and the stage vector arithmetic."""
    f_lu = n * (n - 1) / 2 + (n - 1) * n * (2 * n - 1) / 3
    f_sol = 2 * n * n - n
    f_att = 2 * work["flops_rhs"] + (n + 1) + f_lu + 4 * f_sol + 35 * n
    f_start = work["flops_rhs"] + work["flops_jac"]
    starts = float(n_acc.sum())
    att = float((n_acc + n_rej).sum())
    return starts * f_start + att * f_att


def time_schedule(S, chem, torch, x, dt, steps, warmup, **opts):
    S.set_opts(chem.default_opts(**opts))
    out = torch.empty_like(x)
    for _ in range(warmup):
        r = S.integrate(x, dt, h_io=False, out=out)
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    t0 = time.perf_counter()
    for k in range(steps):
        ev[k][0].record(st)
        r = S.integrate(x, dt, h_io=False, out=out)
        ev[k][1].record(st)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = [a.elapsed_time(b) for a, b in ev]
    return r, wall, ms


def cpu_baseline(path, phi, dt, n_sample, seed):
    from oracle import oracle as O
    from paper_2112_05834_amd import synth
    idx = synth.sample_indices(phi.shape[0], n_sample, seed)
    cores = os.cpu_count() or 1
    M = O.Mech(path)
    t0 = time.perf_counter()
    out, h, na, nr, st = M.integrate(phi[idx], dt, n_threads=cores)
    wall = time.perf_counter() - t0
    return {"value": len(idx) / wall, "unit": "cells/s", "cores": cores, "kind": "oracle",
            "sample": "%d seeded uniformly sampled cells of the same workload (seed %d), "
                      "all host threads, %.1f s wall" % (len(idx), seed, wall)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="spray54_262144")
    ap.add_argument("--cpu-sample", type=int, default=384)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--schedules", default="plain,persistent")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="first run one plain device copy of MIB MiB (reference kernel for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only; --gpus %d is not supported "
              "(cells are independent: a multi-GPU run would give each GPU its own share of the cells)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2112_05834_amd import chem, synth

    d = tempfile.mkdtemp(prefix="chem_bench_")
    wl, mech, path, phi = synth.workload_inputs(args.workload, d)
    M = chem.Mechanism(path)
    S = chem.Solver(M, chem.default_opts(), device=0)
    x = torch.from_numpy(phi).to("cuda:0")
    if args.copy_calibration > 0:
        nb = args.copy_calibration << 20
        src = torch.ones(nb // 8, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print("bench: copy calibration, %d bytes read and %d bytes written" % (nb, nb), file=sys.stderr, flush=True)
        del src, dst
    n_cells = phi.shape[0]
    n = mech.n_species + 1
    work = M.work()
    print("bench: workload %s, %d cells, n=%d, dt=%g" % (args.workload, n_cells, n, wl.dt),
          file=sys.stderr, flush=True)

    results = {}
    for sched in args.schedules.split(","):
        code = {"plain": chem.PLAIN, "persistent": chem.PERSISTENT,
                "binned": chem.PERSISTENT_BINNED}[sched]
        r, wall, ms = time_schedule(S, chem, torch, x, wl.dt, args.steps, args.warmup, schedule=code)
        na = r.n_acc.cpu().numpy().astype(np.int64)
        nr = r.n_rej.cpu().numpy().astype(np.int64)
        st = r.status.cpu().numpy()
        results[sched] = dict(wall=wall, ms=ms, na=na, nr=nr, status=st,
                              cells_per_s=n_cells * args.steps / wall)
        print("bench: %s %.1f ms/step (events %s), %.3e cells/s, failed cells %d" %
              (sched, 1e3 * wall / args.steps, ["%.1f" % m for m in ms], n_cells * args.steps / wall,
               int((st != 0).sum())), file=sys.stderr, flush=True)

    head = "binned" if "binned" in results else ("persistent" if "persistent" in results else "plain")
    if "plain" in results and results["plain"]["cells_per_s"] > results[head]["cells_per_s"] and head != "binned":
        head = "plain"
    R = results[head]
    plain = results.get("plain", R)
    flops = flops_per_launch(work, n, plain["na"], plain["nr"])
    kern_s = float(np.mean(plain["ms"])) / 1e3
    achieved = flops / kern_s
    line = {
        "metric": METRIC,
        "value": R["cells_per_s"],
        "unit": "cells/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * R["wall"] / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "cells": n_cells, "species": mech.n_species,
                   "reactions": mech.n_reactions, "pressure_Pa": wl.pressure, "dt_s": wl.dt,
                   "schedule": head, "rtol": 1e-6, "atol": 1e-10},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": FP64_VECTOR_PEAK / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / FP64_VECTOR_PEAK, "traffic": None,
                     "kernel": "k_integrate (plain, one launch per chemistry step)",
                     "flops_per_launch": flops, "kernel_ms": kern_s * 1e3},
        "schedules": {k: {"cells_per_s": v["cells_per_s"], "ms_per_step": 1e3 * v["wall"] / args.steps}
                      for k, v in results.items()},
        "substeps": {"mean": float((plain["na"] + plain["nr"]).mean()),
                     "p50": float(np.percentile(plain["na"] + plain["nr"], 50)),
                     "p99": float(np.percentile(plain["na"] + plain["nr"], 99)),
                     "max": int((plain["na"] + plain["nr"]).max())},
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(path, phi, wl.dt, args.cpu_sample, 7)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
