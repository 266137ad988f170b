"""Throughput of the per-cell stiff chemistry integration on one MI355X.

One step = one chemistry step of every cell of the workload: all cells
integrated over dt from the same seeded synthetic batch, resident in HBM.
The headline schedule is the persistent kernel with its work queue ordered
by the learned cost model (features, MLP inference and binning are inside
the timed step; training on logged samples of other seeds is not). Plain
(one launch, static cell-to-wave mapping), persistent in index order, and
persistent with bins of the true cost are timed beside it.

Prints one JSON line. The roofline object describes the headline's
integration kernel: algorithmic FP64 flops counted from the mechanism's
structure and every cell's accepted/rejected step counts, over the kernel's
own duration measured with HIP events recorded around its launches on the
stream it runs on.
"""
import argparse
import hashlib
import json
import os
import re
import sys
import tempfile
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "cells integrated/s per chemistry step (54-sp FP64), binned persistent vs plain"
FP64_VECTOR_PEAK = 78.6e12        # 256 CU x 4 SIMD x 16 lanes x 2 flop (FMA) x 2.4 GHz
HBM_PEAK = 8.0e12
TRAIN_SEEDS = {"spray54_262144": list(range(1040, 1048)),
               "spray54_heavytail_1048576": list(range(1040, 1042)),
               "tiny9_1024": [1010, 1011]}


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


def bytes_per_launch_wide(n, n_acc, n_rej, cells):
    """Algorithmic HBM bytes of one launch of the workgroup-per-cell kernel
    (J and M of each cell live in HBM): per attempted step, forming M (read
    J, write M), one read and one write of M by the LU and four solves each
    reading the factors, 64 n^2 bytes; per step start, writing J and the
    chain rule's read and write, 24 n^2 bytes; per cell, phi in and out."""
    att = float((n_acc + n_rej).sum())
    starts = float(n_acc.sum())
    return 64.0 * n * n * att + 24.0 * n * n * starts + 2.0 * 8 * (n + 1) * cells


def _sources_current(text, sources):
    """True if the summary names a sha256 prefix for every kernel source and
    each matches the file as it is now."""
    for src in sources:
        m = re.search(re.escape(src) + r" sha256 prefix ([0-9a-f]+)", text)
        full = os.path.join(ROOT, "paper_2112_05834_amd", "csrc", src)
        if not m or not hashlib.sha256(open(full, "rb").read()).hexdigest().startswith(m.group(1)):
            return False
    return True


# sources the wave-per-cell integration kernel is compiled from
WAVE_KERNEL_SOURCES = ("integrator.hip", "device_common.hpp")


def measured_traffic():
    """HBM bytes per launch from the committed counter summary, if it was
    taken on the current kernel sources (else None)."""
    path = os.path.join(ROOT, "profiles", "k_integrate_spray54_262144_hbm_counters.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    t = re.search(r"total ([0-9.]+) MB\.", text)
    if not t or not _sources_current(text, WAVE_KERNEL_SOURCES):
        return None
    return float(t.group(1)) * 1e6


def measured_wide_traffic():
    """HBM bytes per launch of the workgroup kernel on the first 16384 cells of
    the 160-species workload (persistent schedule), from the committed counter
    summary, if it was taken on the current sources (else None)."""
    path = os.path.join(ROOT, "profiles", "k_integrate_wide_large160_16384_hbm_counters.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    t = re.search(r"total ([0-9.]+) TB\.", text)
    if not t or not _sources_current(text, ("integrator_wide.hip", "device_common.hpp")):
        return None
    return float(t.group(1)) * 1e12


def measured_fp64_ops():
    """Executed FP64 operations per launch (all lanes) from the committed FP64
    instruction-counter summary, if it was taken on the current kernel sources
    (else None)."""
    path = os.path.join(ROOT, "profiles", "k_integrate_spray54_262144_fp64_counters.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    t = re.search(r"executed FP64 operations: ([0-9.e+]+) per launch", text)
    if not t or not _sources_current(text, WAVE_KERNEL_SOURCES):
        return None
    return float(t.group(1))


# integration tolerances of every solver the benchmark configures
TOL = {"rtol": 1e-6, "atol": 1e-10}


def time_schedule(S, chem, torch, x, dt, steps, warmup, chain, zonal=False, **opts):
    """(last result, wall s, per-step event ms, per-launch kernel ms). zonal:
    one step with zonal reference mapping (chem_integrate_zonal) per step."""
    S.set_opts(chem.default_opts(**TOL, **opts))
    out = torch.empty_like(x)

    def one():
        if zonal:
            return S.integrate_zonal(x, dt, h_io=False, out=out)[0]
        if chain > 1:
            return S.integrate_steps(x, dt, chain, h_io=False, out=out)
        return S.integrate(x, dt, h_io=False, out=out)

    for _ in range(warmup):
        r = one()
    torch.cuda.synchronize()
    S.kernel_timing(True)
    st = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        ev[k][0].record(st)
        r = one()
        ev[k][1].record(st)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kms = S.kernel_times()
    S.kernel_timing(False)
    ms = [a.elapsed_time(b) for a, b in ev]
    return r, wall, ms, kms


def train_model(S, chem, torch, synth, wl, mech, seeds, log, n_cells):
    """Log (features, ln substeps) of every cell of other seeds' states in
    one persistent step each, then train the predictor on all of them."""
    t0 = time.perf_counter()
    feats, targ = [], []
    S.set_opts(chem.default_opts(schedule=chem.PERSISTENT, **TOL))
    for sd in seeds:
        phi = synth.generate_states(mech, wl.n_cells, wl.pressure, wl.recipe, sd)[:n_cells]
        x = torch.from_numpy(phi.copy()).to("cuda:0")
        S.log_enable(x.shape[0])
        S.integrate(x, wl.dt, h_io=False)
        f, t = S.log_fetch(x.shape[0])
        feats.append(f.clone())
        targ.append(t.clone())
        del x
        log("logged training seed %d" % sd)
    S.log_enable(0)
    F = torch.cat(feats).contiguous()
    T = torch.cat(targ).contiguous()
    t1 = time.perf_counter()
    S.model_train(F, T, chem.default_train_opts())
    torch.cuda.synchronize()
    loss, _ = S.model_grad(F, T)
    t2 = time.perf_counter()
    return {"samples": int(F.shape[0]), "seeds": seeds, "log_s": t1 - t0, "train_s": t2 - t1,
            "mse_ln_substeps": float(loss.cpu()[0]), "target_var": float(T.var().cpu())}


def cpu_baseline(path, phi, dt, budget_s, seed):
    """The oracle on a seeded uniform sample of the workload's cells, in
    chunks, until about budget_s of wall time has passed."""
    import numpy as np

    from oracle import oracle as O
    idx = np.random.Generator(np.random.PCG64(seed)).permutation(phi.shape[0])[:65536]
    cores = min(16, os.cpu_count() or 1)     # a one-GPU share of the host
    M = O.Mech(path)
    done, chunk = 0, 4 * cores
    t0 = time.perf_counter()
    while done < len(idx) and time.perf_counter() - t0 < budget_s:
        sel = idx[done:done + chunk]
        M.integrate(phi[sel], dt, n_threads=cores, **TOL)
        done += len(sel)
    wall = time.perf_counter() - t0
    # the same oracle on one thread, on the next cells of the sample, for a
    # quarter of the budget
    one, t1 = 0, time.perf_counter()
    while done + one < len(idx) and time.perf_counter() - t1 < budget_s / 4:
        sel = idx[done + one:done + one + 8]
        M.integrate(phi[sel], dt, n_threads=1, **TOL)
        one += len(sel)
    wall1 = time.perf_counter() - t1
    return {"value": done / wall, "unit": "cells/s", "cores": cores, "kind": "oracle",
            "sample": "%d cells drawn uniformly at random (seed %d) from the workload, in chunks of %d until "
                      "%.0f s had passed; %d host threads, %.1f s wall" % (done, seed, chunk, budget_s, cores, wall),
            "value_1_thread": one / wall1 if one else None,
            "sample_1_thread": "the next %d cells of the same sample on one thread, %.1f s wall" % (one, wall1)}


def fig2(args, S, chem, torch, synth, wl, mech, phi, log):
    """Analogue of the paper's Fig. 2 (Methodology, the Analytical Jacobian
    paragraph: mean time of one cell's chemistry problem against the absolute
    tolerance, with a finite-difference Jacobian and generic linear algebra
    against the analytical Jacobian and LAPACK). On the GPU: time per cell of
    the whole integration (kernel time over the cells of a seeded sample)
    with the analytical against the forward-difference Jacobian, for atol
    1e-8 .. 1e-12 at the chosen rtol; and the library's per-wave LU with one
    solve against rocSOLVER's batched getrf + getrs on the same integrator
    matrices M = I/(gamma h) - J of real cell states."""
    import numpy as np
    n_cells = min(args.fig2_cells, phi.shape[0])
    idx = synth.sample_indices(phi.shape[0], n_cells, 17)
    x = torch.from_numpy(np.ascontiguousarray(phi[idx])).to("cuda:0")
    sweep = []
    for atol in (1e-8, 1e-9, 1e-10, 1e-11, 1e-12):
        row = {"atol": atol, "rtol": args.rtol}
        for jac, code in (("analytical", chem.JAC_ANALYTICAL), ("fd", chem.JAC_FD)):
            S.set_opts(chem.default_opts(schedule=chem.PERSISTENT, rtol=args.rtol, atol=atol, jacobian=code))
            S.integrate(x, wl.dt, h_io=False)
            torch.cuda.synchronize()
            S.kernel_timing(True)
            r = S.integrate(x, wl.dt, h_io=False)
            kms = float(np.mean(S.kernel_times()))
            S.kernel_timing(False)
            sub = (r.n_acc + r.n_rej).double().mean().item()
            row[jac] = {"kernel_ms": kms, "us_per_cell": 1e3 * kms / n_cells, "mean_substeps": sub,
                        "failed_cells": int((r.status != 0).sum().item())}
        row["fd_over_analytical"] = row["fd"]["kernel_ms"] / row["analytical"]["kernel_ms"]
        log("fig2 atol %g: analytical %.3f us/cell, fd %.3f us/cell (x%.1f), substeps %.1f / %.1f" %
            (atol, row["analytical"]["us_per_cell"], row["fd"]["us_per_cell"], row["fd_over_analytical"],
             row["analytical"]["mean_substeps"], row["fd"]["mean_substeps"]))
        sweep.append(row)
    # linear algebra: the same batch of integrator matrices through both LUs
    n = mech.n_species + 1
    nb = min(args.fig2_lu_batch, phi.shape[0])
    idx = synth.sample_indices(phi.shape[0], nb, 19)
    y = torch.from_numpy(np.ascontiguousarray(phi[idx])).to("cuda:0")
    _, J = S.eval_rhs_jac(y)
    h = 1e-7
    M0 = torch.eye(n, dtype=torch.float64, device="cuda:0")[None] / (0.5 * h) - J
    Mt0 = M0.transpose(1, 2).contiguous()        # column-major for the library
    b0 = torch.ones((nb, n), dtype=torch.float64, device="cuda:0")
    st = torch.cuda.current_stream()

    def timed(fn, reps=3):
        best = 1e30
        for _ in range(reps):
            a, bb = fn()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(st)
            out = fn.call(a, bb)
            e1.record(st)
            torch.cuda.synchronize()
            best = min(best, e0.elapsed_time(e1))
        return best, out

    class Ours:
        def __call__(self):
            return M0.clone(), b0.clone()

        def call(self, a, bb):
            return S.lu_batch(a, bb)

    class Lib:
        def __call__(self):
            return Mt0.clone(), b0.clone()

        def call(self, a, bb):
            return chem.lu_batch_rocsolver(a, bb)

    t_ours, (A1, p1, i1, x1) = timed(Ours())
    t_lib, (A2, p2, i2, x2) = timed(Lib())
    same_piv = bool(torch.equal(p1 + 1, p2))
    dx = float(((x1 - x2).abs().max() / x1.abs().max()).item())
    lu = {"n": n, "batch": nb, "h_s": h, "wave_lu_ms": t_ours, "rocsolver_ms": t_lib,
          "wave_lu_us_per_matrix": 1e3 * t_ours / nb, "rocsolver_us_per_matrix": 1e3 * t_lib / nb,
          "rocsolver_over_wave_lu": t_lib / t_ours, "identical_pivots": same_piv, "max_rel_solution_diff": dx,
          "what": "LU with partial pivoting and one solve per matrix, matrices read and written in HBM"}
    log("fig2 LU n=%d batch %d: wave LU %.3f ms, rocSOLVER getrf+getrs %.3f ms (x%.1f), pivots identical %s" %
        (n, nb, t_ours, t_lib, t_lib / t_ours, same_piv))
    return {"metric": "Fig. 2 analogue: time per cell vs atol (analytical vs finite-difference Jacobian) and "
                      "per-wave LU vs rocSOLVER batched getrf/getrs",
            "workload": args.workload, "cells": n_cells, "sweep": sweep, "lu": lu}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="spray54_262144")
    ap.add_argument("--chain", type=int, default=1, help="chemistry steps per graph launch (chained in a HIP graph)")
    ap.add_argument("--cells", type=int, default=0,
                    help="use only the first CELLS cells of the workload (profiling runs)")
    ap.add_argument("--train-cells", type=int, default=0, metavar="N",
                    help="log the cost model's training samples on the first N cells of each training seed "
                         "(default: as many cells as the workload)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--rtol", type=float, default=1e-6, help="relative tolerance (default: the Spray A setting)")
    ap.add_argument("--atol", type=float, default=1e-10, help="absolute tolerance")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--order", default="generated", choices=("generated", "t-ascending", "t-descending"),
                    help="cell order: as generated, or sorted by temperature (a mesh-like order that puts the "
                         "stiff hot cells together)")
    ap.add_argument("--schedules", default="plain,persistent,binned,truebins",
                    help="comma list of plain, persistent, binned, truebins, zonal")
    ap.add_argument("--zone", default="1e-6,1.0", metavar="Z_MAX,T_TOL[,DZ]",
                    help="zonal schedule: cells with Z <= Z_MAX within T_TOL kelvin of their Z band's reference "
                         "are mapped (bands of width DZ; default one band)")
    ap.add_argument("--autotune", type=int, default=0, metavar="CELLS",
                    help="pick launch shape and queue chunk by timing a seeded sample of this many cells first")
    ap.add_argument("--fig2", action="store_true",
                    help="instead of the throughput line, print the Fig. 2 analogue (time per cell against atol "
                         "with analytical and finite-difference Jacobians; per-wave LU against rocSOLVER)")
    ap.add_argument("--fig2-cells", type=int, default=32768, help="cells of the --fig2 atol sweep")
    ap.add_argument("--fig2-lu-batch", type=int, default=65536, help="matrices of the --fig2 LU comparison")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="first run one plain device copy of MIB MiB (reference kernel for HBM byte counters)")
    args = ap.parse_args()
    TOL.update(rtol=args.rtol, atol=args.atol)
    if args.gpus != 1:
        print("bench.py: runs on one GPU only; --gpus %d is not supported "
              "(cells are independent: a multi-GPU run would give each GPU its own share of the cells)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2112_05834_amd import chem, synth

    def log(msg):
        print("bench: " + msg, file=sys.stderr, flush=True)

    d = tempfile.mkdtemp(prefix="chem_bench_")
    wl, mech, path, phi = synth.workload_inputs(args.workload, d, args.cells if args.cells > 0 else None)
    if args.order != "generated":
        phi = np.ascontiguousarray(phi[np.argsort(phi[:, 0] if args.order == "t-ascending" else -phi[:, 0],
                                                  kind="stable")])
    M = chem.Mechanism(path)
    S = chem.Solver(M, chem.default_opts(**TOL), device=0)
    x = torch.from_numpy(phi).to("cuda:0")
    if args.copy_calibration > 0:
        nb = args.copy_calibration << 20
        src = torch.ones(nb // 8, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log("copy calibration, %d bytes read and %d bytes written" % (nb, nb))
        del src, dst
    if args.fig2:
        print(json.dumps(fig2(args, S, chem, torch, synth, wl, mech, phi, log)), flush=True)
        return
    n_cells = phi.shape[0]
    n = mech.n_species + 1
    work = M.work()
    log("workload %s, %d cells, n=%d, dt=%g, chain %d" % (args.workload, n_cells, n, wl.dt, args.chain))
    scheds = args.schedules.split(",")

    training = None
    if "binned" in scheds or "truebins" in scheds:
        training = train_model(S, chem, torch, synth, wl, mech, TRAIN_SEEDS.get(args.workload, [1040, 1041]), log,
                               args.train_cells if args.train_cells > 0 else n_cells)
        log("model trained on %d samples: log %.1f s, train %.1f s, mse %.3f (target variance %.3f)" %
            (training["samples"], training["log_s"], training["train_s"], training["mse_ln_substeps"],
             training["target_var"]))

    tuned = None
    if args.autotune > 0:
        idx = synth.sample_indices(n_cells, args.autotune, 11)
        sample = torch.from_numpy(np.ascontiguousarray(phi[idx])).to("cuda:0")
        tuned = {}
        for sched in ("persistent",):
            S.set_opts(chem.default_opts(schedule=chem.PERSISTENT, **TOL))
            S.autotune(sample, wl.dt)
            o = S.opts
            tuned = {"waves_per_block": o.waves_per_block, "queue_chunk": o.queue_chunk,
                     "cells_per_wave": o.cells_per_wave, "sample_cells": len(idx)}
        log("autotuned on %d cells: %s" % (len(idx), tuned))

    # plain gets its own best launch shape (waves per block, cells per wave),
    # picked by the autotuner on a seeded sample, so that the schedules are
    # compared at their best shapes rather than at a shape chosen for another
    plain_shape = None
    if "plain" in scheds:
        idx = synth.sample_indices(n_cells, min(16384, n_cells), 13)
        sample = torch.from_numpy(np.ascontiguousarray(phi[idx])).to("cuda:0")
        S.set_opts(chem.default_opts(schedule=chem.PLAIN, **TOL))
        S.autotune(sample, wl.dt)
        o = S.opts
        plain_shape = {"waves_per_block": o.waves_per_block, "cells_per_wave": o.cells_per_wave,
                       "tuned_on_cells": len(idx)}
        log("plain launch shape autotuned on %d cells: %s" % (len(idx), plain_shape))
        del sample

    codes = {"plain": chem.PLAIN, "persistent": chem.PERSISTENT, "binned": chem.PERSISTENT_BINNED,
             "truebins": chem.PERSISTENT_BINNED, "zonal": chem.PERSISTENT}
    if "zonal" in scheds:
        if args.chain > 1:
            raise SystemExit("the zonal schedule runs one chemistry step per call (--chain 1)")
        zv = [float(v) for v in args.zone.split(",")]
        z_max, t_tol = zv[0], zv[1]
        dz = zv[2] if len(zv) > 2 else 0.0
        S.zone_config(*synth.bilger_streams(mech), z_max, t_tol, dz=dz)
    results = {}
    true_cost = None
    for sched in scheds:
        if sched == "truebins":
            ref = results.get("plain") or results.get("persistent") or results.get("binned")
            if ref is None or args.chain > 1:
                continue
            true_cost = torch.from_numpy(np.log(np.maximum(ref["na"] + ref["nr"], 1)).astype(np.float32)).to(
                "cuda:0")
            S.set_cost_override(true_cost)
        extra = {}
        if sched == "plain" and plain_shape:
            extra = {"waves_per_block": plain_shape["waves_per_block"],
                     "cells_per_wave": plain_shape["cells_per_wave"]}
        if tuned and sched != "plain":
            extra = {"waves_per_block": tuned["waves_per_block"], "queue_chunk": tuned["queue_chunk"],
                     "cells_per_wave": tuned["cells_per_wave"]}
        r, wall, ms, kms = time_schedule(S, chem, torch, x, wl.dt, args.steps, args.warmup, args.chain,
                                         zonal=sched == "zonal", schedule=codes[sched], **extra)
        used = S.last_binning_used() if codes[sched] == chem.PERSISTENT_BINNED else None
        if sched == "truebins":
            S.set_cost_override(None)
        na = r.n_acc.cpu().numpy().astype(np.int64)
        nr = r.n_rej.cpu().numpy().astype(np.int64)
        stt = r.status.cpu().numpy()
        cells = n_cells * args.steps * args.chain
        results[sched] = dict(wall=wall, ms=ms, kms=kms, na=na, nr=nr, status=stt, used=used,
                              cells_per_s=cells / wall)
        if "zonal" in scheds and sched in ("zonal", "persistent"):
            results[sched]["T"] = r.phi[:, 0].cpu().numpy()
        if sched == "zonal":
            mapped = S.integrate_zonal(x, wl.dt, h_io=False)[1].cpu().numpy() > 0
            results[sched]["mapped"] = mapped
            log("zonal: %.1f%% of the cells mapped (Z <= %g, |T - T_ref| <= %g K, band width %g)" %
                (100 * mapped.mean(), z_max, t_tol, dz))
        log("%s %.1f ms/step (events %s), kernel ms %s, %.4e cells/s, failed cells %d, binning used %s" %
            (sched, 1e3 * wall / (args.steps * args.chain), ["%.1f" % m for m in ms],
             ["%.1f" % m for m in kms[:4]], cells / wall, int((stt != 0).sum()), used))

    head = "binned" if "binned" in results else ("persistent" if "persistent" in results else scheds[0])
    R = results[head]
    ref = results.get("plain", R)
    flops = flops_per_launch(work, n, R["na"], R["nr"])
    wide = n > 64
    if args.chain > 1:
        kern_s = achieved = None
    else:
        kern_s = float(np.mean(R["kms"])) / 1e3 if len(R["kms"]) else float(np.mean(R["ms"])) / 1e3
        achieved = flops / kern_s
    traffic = measured_traffic()
    executed = measured_fp64_ops()
    if (args.workload != "spray54_262144" or args.chain > 1 or args.cells > 0 or args.order != "generated" or
            (args.rtol, args.atol) != (1e-6, 1e-10)):
        traffic = None
        executed = None
    steps_total = args.steps * args.chain
    line = {
        "metric": METRIC,
        "value": R["cells_per_s"],
        "unit": "cells/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * R["wall"] / steps_total,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "cells": n_cells, "species": mech.n_species,
                   "reactions": mech.n_reactions, "pressure_Pa": wl.pressure, "dt_s": wl.dt,
                   "schedule": head, "chained_steps_per_graph": args.chain, "rtol": args.rtol, "atol": args.atol,
                   "cell_order": args.order},
        "roofline": {"bound": "alu", "achieved": None if achieved is None else achieved / 1e12,
                     "peak": FP64_VECTOR_PEAK / 1e12, "unit": "TFLOP/s",
                     "frac": None if achieved is None else achieved / FP64_VECTOR_PEAK,
                     "traffic": traffic,
                     "kernel": "k_integrate<%d,...> (%s schedule)" % (n, head),
                     "flops_per_launch": flops, "kernel_ms": None if kern_s is None else kern_s * 1e3,
                     # FP64 operations the kernel executes (instruction counters, all lanes), beside
                     # the algorithmic flops that `achieved` counts
                     "executed": None if executed is None or kern_s is None else executed / kern_s / 1e12,
                     "executed_frac": None if executed is None or kern_s is None else
                     executed / kern_s / FP64_VECTOR_PEAK},
        "schedules": {k: {"cells_per_s": v["cells_per_s"], "ms_per_step": 1e3 * v["wall"] / steps_total,
                          "kernel_ms": float(np.mean(v["kms"])) if len(v["kms"]) else None,
                          "binning_used": v["used"]}
                      for k, v in results.items()},
        "substeps": {"mean": float((ref["na"] + ref["nr"]).mean()),
                     "p50": float(np.percentile(ref["na"] + ref["nr"], 50)),
                     "p99": float(np.percentile(ref["na"] + ref["nr"], 99)),
                     "max": int((ref["na"] + ref["nr"]).max())},
    }
    if wide:
        # J and M live in HBM: the bandwidth roof applies, FP64 is secondary
        hb = bytes_per_launch_wide(n, R["na"], R["nr"], n_cells)
        fp64 = line["roofline"]
        line["roofline"] = {"bound": "hbm", "achieved": None if kern_s is None else hb / kern_s / 1e9,
                            "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                            "frac": None if kern_s is None else hb / kern_s / HBM_PEAK,
                            # measured bytes exist for one configuration: these cells, this schedule
                            "traffic": measured_wide_traffic() if (
                                args.workload == "large160_524288" and n_cells == 16384 and args.chain == 1 and
                                head == "persistent" and (args.rtol, args.atol) == (1e-6, 1e-10)) else None,
                            "kernel": "k_integrate_wide (%s schedule)" % head, "bytes_per_launch": hb,
                            "kernel_ms": fp64["kernel_ms"],
                            "fp64": {"achieved": fp64["achieved"], "peak": fp64["peak"], "unit": "TFLOP/s",
                                     "frac": fp64["frac"], "flops_per_launch": flops}}
    if "plain" in results and head != "plain":
        line["speedup_vs_plain"] = R["cells_per_s"] / results["plain"]["cells_per_s"]
    if plain_shape is not None:
        line["plain_shape"] = plain_shape
    if "zonal" in results:
        Zr = results["zonal"]
        zl = {"z_max": z_max, "t_tol_K": t_tol, "band_width": dz, "mapped_frac": float(Zr["mapped"].mean())}
        if "persistent" in results:
            P = results["persistent"]
            zl["speedup_vs_persistent"] = Zr["cells_per_s"] / P["cells_per_s"]
            m = Zr["mapped"]
            # what mapping changes against integrating every cell
            zl["max_abs_dT_mapped_K"] = float(np.abs(Zr["T"][m] - P["T"][m]).max()) if m.any() else 0.0
        line["zonal"] = zl
    if training is not None:
        line["training"] = training
    if tuned is not None:
        line["autotuned"] = tuned
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(path, phi, wl.dt, args.cpu_seconds, 7)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
