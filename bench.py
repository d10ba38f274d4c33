#!/usr/bin/env python3
"""Throughput benchmark of the matrix-free FIT hot path on one MI355X.

Workload: the 128^3-cell graded layered device (6 layers, eps_r in [2, 12],
loss tangents 0.001-0.02, PEC strips, one 50-Ohm lumped port; seed 2) at its
seeded frequency 10.624 GHz.  One step = one frequency point solved to a true
relative residual <= 1e-8 (complex128, symmetric M_eps^-1/2 scaling, COCG =
the paper's CG in its complex-symmetric form) followed by the port-voltage
readout.  The grid is created and the source uploaded before the timed
region.

Reported: freq-points solved per second (the value), the dominant kernel's
achieved algorithmic HBM bandwidth against the 8 TB/s peak (HIP events
around every launch during the timed region), the plain operator's GB/s, and
the CPU oracle on a bounded sample of the same workload.  Prints one JSON
line.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "freq-points solved/sec at 1e-8 rel. residual; matvec GB/s vs HBM peak"
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_pcocg_step1_c128.json")
# tile table for the bench grid, written by `bench.py --autotune --save-tune`
TUNE_FILE = os.path.join(ROOT, "paper_1705_08849_amd", "tune_gfx950.json")
KERNEL_SOURCES = ["paper_1705_08849_amd/csrc/stencil.h", "paper_1705_08849_amd/csrc/krylov.h",
                  "paper_1705_08849_amd/csrc/fit_internal.h", "paper_1705_08849_amd/csrc/reduce.h"]


def kernel_source_hash():
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(tile, path=None):
    """HBM bytes per launch of the dominant kernel from the committed
    rocprofv3 counter summary, if it was taken on the current kernel source
    and with the tile this run uses."""
    try:
        with open(path or TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_hash") != kernel_source_hash():
        return None
    if tile is not None and t.get("tile") is not None and list(t["tile"]) != list(tile):
        return None
    return t.get("bytes_per_launch")


def bench_tile(fit, g, dev, omega, args):
    """The tile the bench's grid runs with: the committed tile table's entry
    for its node dimensions (so that repeated runs and the counter passes use
    the same tile), or a fresh autotune with --autotune or when the table has
    no entry; --no-autotune keeps the library's default shape."""
    if args.no_autotune:
        return None
    nx, ny, nz = dev.nodes
    if not args.autotune and os.path.exists(TUNE_FILE):
        with open(TUNE_FILE) as f:
            table = json.load(f)
        for e in table.get("entries", []):
            if (e["nx"], e["ny"], e["nz"], e["dtype"]) == (nx, ny, nz, fit.C128):
                fit.tune_load(TUNE_FILE)
                return (e["tx"], e["ty"], e["zc"])
    # tuned on the solver's own iteration (fused COCG step + update kernel)
    tile, _ = g.autotune_solver(omega, iters=1000)
    if args.save_tune:
        fit.tune_save(TUNE_FILE)
    return tile


def counter_sample(args):
    """Short program for the HBM-counter passes: the bench's grid and tile,
    40 COCG iterations, then a plain float64 negation of one complex128
    vector (a copy-shaped kernel of exactly known traffic) that calibrates
    the counters."""
    import numpy as np
    import torch

    from paper_1705_08849_amd import devices as D
    from paper_1705_08849_amd import fit

    dev = D.plain_device_128(2)
    omega = 2 * np.pi * D.log_uniform_frequency(2)
    g = fit.Grid(dev)
    tile = bench_tile(fit, g, dev, omega, args)
    src = torch.from_numpy(D.port_source(dev, 0)).to("cuda:0")
    g.solve(omega, src, tol=1e-8, solver="cocg", max_iters=40, raise_on_error=False)
    xr = torch.randn(dev.n_edges * 2, dtype=torch.float64, device="cuda:0")
    yr = torch.empty_like(xr)
    for _ in range(3):
        torch.neg(xr, out=yr)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_each_way": xr.numel() * 8, "tile": tile}), flush=True)


def _counter_rows(path):
    import csv
    with open(path) as f:
        return list(csv.DictReader(f))


def _counter_run_info(log_path):
    """The JSON line that a `--counters` run prints: the calibration copy's
    bytes each way and the tile the run used."""
    with open(log_path) as f:
        for line in f:
            if line.startswith("{") and "copy_bytes_each_way" in line:
                return json.loads(line)
    raise SystemExit(f"{log_path}: no line from a --counters run")


def ingest_counters(fetch_csv, write_csv, fetch_log, write_log, commands, out_path=None):
    """Turn the two rocprofv3 counter CSVs of `--counters` into the per-launch
    HBM traffic of the fused COCG step-1 kernel, each counter scaled by what
    it reads for the copy-shaped calibration kernel.  Both runs must have
    used the same tile; it is recorded with the result."""
    info_f, info_w = _counter_run_info(fetch_log), _counter_run_info(write_log)
    if info_f != info_w:
        raise SystemExit(f"the two counter runs differ: {info_f} vs {info_w}")
    copy_bytes = int(info_f["copy_bytes_each_way"])
    def per_kernel(rows, counter):
        acc = {}
        for r in rows:
            if r.get("Counter_Name") != counter:
                continue
            name = r["Kernel_Name"]
            acc.setdefault(name, []).append(float(r["Counter_Value"]))
        return acc

    def pick(acc, *keys):
        hits = [v for k, v in acc.items() if all(s in k for s in keys)]
        if not hits:
            raise SystemExit(f"no dispatch of a kernel matching {keys}")
        vals = [x for h in hits for x in h]
        # a solver kernel launched after convergence returns at once; those
        # dispatches move no vector data and are left out
        top = max(vals)
        vals = [x for x in vals if x > 0.05 * top]
        return sum(vals) / len(vals), len(vals)

    out = {"kernel": "pcocg_step1_c128", "kernel_source_hash": kernel_source_hash(),
           "tile": info_f.get("tile"), "commands": commands}
    for counter, path, key in (("FETCH_SIZE", fetch_csv, "fetch"), ("WRITE_SIZE", write_csv, "write")):
        acc = per_kernel(_counter_rows(path), counter)
        kib, n = pick(acc, "stencil_kernel<double", "OpCocgPX")
        cal_kib, _ = pick(acc, "neg")
        scale = (copy_bytes / 1024.0) / cal_kib
        out[f"{key}_kib_raw"] = kib
        out[f"{key}_dispatches"] = n
        out[f"{key}_calibration_kib"] = cal_kib
        out[f"{key}_scale"] = scale
        out[f"{key}_bytes_per_launch"] = kib * 1024.0 * scale
    out["bytes_per_launch"] = out["fetch_bytes_per_launch"] + out["write_bytes_per_launch"]
    with open(out_path or TRAFFIC_FILE, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out, indent=1))


def sweep_row(fit, D, np, torch, with_cpu):
    """The batched sweep (fit_sweep) against the same systems solved one
    fit_solve at a time, on the smallest sweep-family grid."""
    sd = D.sweep_devices(seeds=[40], shapes=[(64, 64, 32)])[0]
    g = fit.Grid(sd)
    oms = D.log_spaced_omegas(16, 5e9, 40e9)
    # an iteration on this grid takes ~20 us: 400-iteration timings keep the
    # tile and batch choices from changing run to run.  Each side runs with
    # its own tuned block shape: the solver tuner's for one system at a time,
    # the sweep tuner's (chosen on batched launches) for the sweep.
    tile, _ = g.autotune_solver(float(oms[8]), iters=400)
    batch, _ = g.autotune_sweep(oms, iters=200)
    sweep_tile = g.tile("c128_batched")
    src = torch.from_numpy(D.port_source(sd, 0)).to("cuda:0")
    fit.sweep([g], oms[:2], [src[None, :]], tol=1e-8)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st, _, infos = fit.sweep([g], oms, [src[None, :]], tol=1e-8, precision="fp64")
    torch.cuda.synchronize()
    tb = time.perf_counter() - t0
    t0 = time.perf_counter()
    for om in oms:
        g.solve(float(om), src, tol=1e-8, solver="cocg", raise_on_error=False)
    torch.cuda.synchronize()
    ts = time.perf_counter() - t0
    iters = [i["iterations"] for i in infos]
    row = {"workload": "64x64x32-cell sweep-family device (seed 40), 16 log-spaced frequencies "
                       "5-40 GHz, one port excitation, COCG fp64 to 1e-8",
           "status": fit.STATUS_NAMES[st], "points": 16, "tile_sequential": list(tile),
           "tile_batched": list(sweep_tile), "systems_per_batch": batch,
           "batched_points_per_s": round(16 / tb, 3),
           "sequential_points_per_s": round(16 / ts, 3), "speedup": round(ts / tb, 3),
           "iterations": [min(iters), max(iters)]}
    if with_cpu:
        import multiprocessing as mp
        workers = max(1, min(16, os.cpu_count() or 1, len(oms)))
        t0 = time.perf_counter()
        with mp.get_context("spawn").Pool(workers) as pool:
            per = pool.map(_sweep_cpu_point, [(float(om), it) for om, it in zip(oms, iters)])
        wall = time.perf_counter() - t0
        # every worker ran one frequency's sample concurrently (memory
        # bandwidth shared as in a full run); each sample is extrapolated to
        # its GPU iteration count and the points are spread over the workers
        est = sum(per) / workers
        row["cpu_baseline"] = {"value": round(len(oms) / est, 5), "unit": "freq-points/s",
                               "cores": workers, "kind": "oracle",
                               "sample": f"{len(oms)} frequencies on a pool of {workers} single-thread "
                                         "workers, each: assembly + 20 COCG iterations, extrapolated "
                                         "with that point's GPU iteration count; points spread over "
                                         f"the workers (sample wall {wall:.1f} s)"}
    return row


def baseline_row(fit, D, np, torch):
    """The batched sweep against the plain method of the comparison: every
    one of 64 log-spaced frequencies (1-40 GHz) on the smallest sweep-family
    grid, port 1 excitation, to a true relative residual of 1e-8, solved by
    complex128 BiCGStab one fit_solve at a time (capped at 60k iterations)
    and by fit_sweep (COCG, complex128 and the mixed form).  The speedup is
    quoted on the frequencies the plain BiCGStab reaches 1e-8 at, re-solved
    there by the sweep, so both sides are timed at the same accuracy on the
    same systems.  Not part of the default run (about four minutes)."""
    dev = D.sweep_devices()[0]
    g = fit.Grid(dev)
    oms = D.log_spaced_omegas(64)
    src = torch.from_numpy(D.port_source(dev, 0)).to("cuda:0")
    # each side with its own tuned block shape: the solver tuner's for one
    # system at a time, the sweep tuner's (a tile-table key of its own) for
    # the batched launches
    tile, _ = g.autotune_solver(float(oms[32]), iters=400)
    batch, _ = g.autotune_sweep(oms[:16], iters=200)
    sweep_tile = g.tile("c128_batched")
    fit.sweep([g], oms[:2], [src[None, :]], tol=1e-8)  # warm-up
    torch.cuda.synchronize()

    def run_sweep(om_list, prec):
        t0 = time.perf_counter()
        _, _, infos = fit.sweep([g], om_list, [src[None, :]], tol=1e-8, max_iters=60000, precision=prec)
        torch.cuda.synchronize()
        ok = sum(1 for i in infos if i["status"] == 0 and i["true_relres"] <= 1e-8)
        return time.perf_counter() - t0, ok

    full = {p: run_sweep(oms, p) for p in ("fp64", "mixed")}
    conv, t_conv, t_all = [], 0.0, 0.0
    for k, om in enumerate(oms):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, info = g.solve(float(om), src, tol=1e-8, solver="bicgstab", max_iters=60000,
                          raise_on_error=False)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        t_all += dt
        if info["status_name"] == "FIT_OK" and info["true_relres"] <= 1e-8:
            conv.append(k)
            t_conv += dt
        if k % 16 == 15:
            print(f"bench.py: plain BiCGStab {k + 1}/64 frequencies, {len(conv)} at 1e-8",
                  file=sys.stderr, flush=True)
    row = {"workload": "64x64x32-cell sweep-family device (seed 40), 64 log-spaced frequencies "
                       "1-40 GHz, port 1, true relative residual 1e-8",
           "systems_per_batch": batch, "tile_sweep": list(sweep_tile), "tile_single": list(tile),
           "plain_bicgstab_c128": {"wall_s": round(t_all, 2), "converged": len(conv), "of": 64},
           "sweep_cocg_c128": {"wall_s": round(full["fp64"][0], 2), "converged": full["fp64"][1], "of": 64},
           "sweep_cocg_mixed": {"wall_s": round(full["mixed"][0], 2), "converged": full["mixed"][1], "of": 64}}
    if conv:
        sub = oms[conv]
        s64, ok64 = run_sweep(sub, "fp64")
        smx, okmx = run_sweep(sub, "mixed")
        row["matched"] = {"frequencies_GHz": [round(o / 2 / np.pi / 1e9, 2) for o in sub],
                          "plain_bicgstab_s": round(t_conv, 2),
                          "sweep_cocg_c128_s": round(s64, 2), "sweep_cocg_c128_converged": ok64,
                          "sweep_cocg_mixed_s": round(smx, 2), "sweep_cocg_mixed_converged": okmx,
                          "speedup_c128": round(t_conv / s64, 2), "speedup_mixed": round(t_conv / smx, 2)}
    return row


def _progress(msg):
    print(f"bench.py: {msg}", file=sys.stderr, flush=True)


def solvers_row(fit, D, np, torch, big=False):
    """Every method of the solver comparison on the 64x64x48-cell graded
    layered device (4 layers, 3 PEC strips, one port, seed 12) -- or, with
    big, on the 128^3-cell bench device (tile from the committed table) --
    at 1, 10 and 40 GHz to a true relative residual of 1e-8, capped at 60k
    iterations (GMRES(30) at 20k on the big device): COCG with each
    diagonal, COCR, TFQMR, CGS, BiCGStab and GMRES(30).  Not part of the
    default run (several minutes; about ten with big)."""
    if big:
        dev = D.plain_device_128(2)
        if os.path.exists(TUNE_FILE):
            fit.tune_load(TUNE_FILE)
    else:
        dev = D.layered_device(64, 64, 48, n_layers=4, n_strips=3, n_ports=1, seed=12)
    g = fit.Grid(dev)
    src = torch.from_numpy(D.port_source(dev, 0)).to("cuda:0")
    runs = [("cocg", "auto"), ("cocg", "mass"), ("cocg", "paper"), ("cocg", "jacobi"), ("cocr", "auto"),
            ("tfqmr", "auto"), ("cgs", "auto"), ("bicgstab", "auto"), ("gmres", "auto")]
    if big:
        runs.remove(("cocg", "mass"))  # the same iterates as auto, through the stored-diagonal path
    out = []
    for f in (1e9, 10e9, 40e9):
        for solver, diag in runs:
            cap = 20000 if (big and solver == "gmres") else 60000
            _, info = g.solve(2 * np.pi * f, src, tol=1e-8, solver=solver, diag=diag, max_iters=cap,
                              raise_on_error=False)
            out.append({"f_GHz": f / 1e9, "solver": solver, "diag": diag, "status": info["status_name"],
                        "iterations": info["iterations"], "true_relres": info["true_relres"],
                        "time_s": round(info["time_ms"] / 1e3, 2)})
            _progress(f"solvers {f / 1e9:.0f} GHz {solver}/{diag}: {info['status_name']} "
                      f"{info['iterations']} it, relres {info['true_relres']:.1e}")
    name = ("128x128x128-cell graded layered device (seed 2, 6 layers, 4 PEC strips, one port)" if big
            else "64x64x48-cell graded layered device (seed 12, 4 layers, 3 PEC strips, one port)")
    return {"workload": name + ", 1/10/40 GHz, true relative residual 1e-8, cap 60k iterations"
                        + (" (GMRES(30) 20k)" if big else ""),
            "runs": out}


def learned_row(fit, D, np, torch):
    """The learned form on the 192x192x96-cell family: the c = 16 U-Net
    trained for 1,500 Adam steps on 8 solver pairs per (device, frequency)
    from 8 seeded 64x64x32-cell family devices at 2, 10 and 30 GHz, then
    FGMRES(30) with it (falling back to COCG on stagnation) against COCG and
    GMRES(30) (cap 3,000) on the held-out devices 9000-9002 to 1e-8, and the
    residual of FGMRES + U-Net and GMRES(30) after 300 steps.  Not part of
    the default run (about ten minutes)."""
    if os.path.exists(TUNE_FILE):
        fit.tune_load(TUNE_FILE)
    freqs = [2e9, 10e9, 30e9]
    tg = [fit.Grid(D.learned_family_device(1000 + s, (64, 64, 32))) for s in range(8)]
    t0 = time.perf_counter()
    pre = fit.Precond.train(tg, [2 * np.pi * f for f in freqs], base_channels=16, steps=1500, batch=4,
                            crop=32, seed=3, pairs_per_system=8, lr=1e-3)
    torch.cuda.synchronize()
    h = fit.Precond.train_history()
    train = {"seconds": round(time.perf_counter() - t0, 1), "loss_first10": float(h[:10].mean()),
             "loss_last50": float(h[-50:].mean())}
    _progress(f"learned: trained in {train['seconds']} s, loss {train['loss_first10']:.3f} -> "
              f"{train['loss_last50']:.3f}")
    del tg
    torch.cuda.empty_cache()
    out = []
    for seed in (9000, 9001, 9002):
        dev = D.learned_family_device(seed)
        g = fit.Grid(dev)
        src = torch.from_numpy(D.port_source(dev, 0)).to("cuda:0")
        for f in freqs:
            om = 2 * np.pi * f
            row = {"seed": seed, "f_GHz": f / 1e9}
            for name, kw, cap in (("cocg", dict(solver="cocg"), 100000),
                                  ("fgmres_unet", dict(solver="fgmres", precond=pre), 100000),
                                  ("gmres30", dict(solver="gmres"), 3000)):
                x, i = g.solve(om, src, tol=1e-8, max_iters=cap, raise_on_error=False, **kw)
                row[name] = {"status": i["status_name"], "iterations": i["iterations"],
                             "fell_back": i["fell_back"], "time_s": round(i["time_ms"] / 1e3, 2),
                             "true_relres": i["true_relres"]}
                del x
            x, i = g.solve(om, src, tol=1e-8, max_iters=300, raise_on_error=False, solver="fgmres",
                           precond=pre)
            x2, i2 = g.solve(om, src, tol=1e-8, max_iters=300, raise_on_error=False, solver="gmres")
            row["after_300"] = {"fgmres_unet": i["true_relres"], "gmres30": i2["true_relres"]}
            del x, x2
            out.append(row)
            _progress(f"learned seed {seed} {f / 1e9:.0f} GHz: cocg {row['cocg']['iterations']} it, "
                      f"fgmres+unet {row['fgmres_unet']['iterations']} it (fell back "
                      f"{row['fgmres_unet']['fell_back']})")
        del g, src
        torch.cuda.empty_cache()
    return {"workload": "c=16 U-Net trained on solver pairs from 8 64x64x32 family devices; held-out "
                        "192x192x96 family devices 9000-9002 at 2/10/30 GHz, true relative residual 1e-8",
            "training": train, "runs": out}


def precision_row(fit, D, np, torch):
    """The precision form on the 256x256x128 interconnect at 1, 10 and 40 GHz:
    COCG in complex128 and the mixed form (complex64 inner iterations,
    complex128 refinement), each capped at 100k iterations, with the mixed
    result's forward error and port-voltage difference against the complex128
    one.  Not part of the default run (about six minutes)."""
    dev = D.interconnect_256(3)
    if os.path.exists(TUNE_FILE):
        fit.tune_load(TUNE_FILE)
    g = fit.Grid(dev)
    src = torch.from_numpy(D.port_source(dev, 0)).to("cuda:0")
    out = []
    for f in (1e9, 10e9, 40e9):
        om = 2 * np.pi * f
        x64, i64 = g.solve(om, src, tol=1e-8, solver="cocg", max_iters=100000, raise_on_error=False)
        u64 = complex(g.port_voltages(x64)[0][0])
        _progress(f"precision {f / 1e9:.0f} GHz complex128: {i64['status_name']} {i64['iterations']} it")
        xm, im = g.solve(om, src, tol=1e-8, solver="cocg", precision="mixed", max_iters=100000,
                         raise_on_error=False)
        um = complex(g.port_voltages(xm)[0][0])
        fe = (torch.linalg.vector_norm(xm - x64) / torch.linalg.vector_norm(x64)).item()
        _progress(f"precision {f / 1e9:.0f} GHz mixed: {im['status_name']} {im['iterations']} it")
        out.append({"f_GHz": f / 1e9,
                    "c128": {"status": i64["status_name"], "iterations": i64["iterations"],
                             "true_relres": i64["true_relres"], "time_s": round(i64["time_ms"] / 1e3, 2)},
                    "mixed": {"status": im["status_name"], "iterations": im["iterations"],
                              "refinements": im["refinements"], "fell_back": im["fell_back"],
                              "true_relres": im["true_relres"], "time_s": round(im["time_ms"] / 1e3, 2)},
                    "forward_error_mixed_vs_c128": fe,
                    "port_voltage_rel_diff": abs(um - u64) / abs(u64) if u64 != 0 else None})
        del x64, xm
        torch.cuda.empty_cache()
    return {"workload": "256x256x128-cell graded interconnect (seed 3), one port, 1/10/40 GHz, true "
                        "relative residual 1e-8, cap 100k iterations", "runs": out}


def family_row(fit, D, np, torch):
    """The sweep over the six uneven sweep-family devices (64x64x32 to
    192x192x96 cells, sigma strips, 4 ports), sampled: 8 of the 64
    log-spaced frequencies over 1-40 GHz, port 1 excitation, complex128, cap
    50k iterations, one fit_sweep per device after its shape tuning.  Not
    part of the default run (about six minutes)."""
    oms = D.log_spaced_omegas(64)[list(range(0, 64, 9))]
    out = []
    for dev in D.sweep_devices():
        g = fit.Grid(dev)
        batch, _ = g.autotune_sweep(oms, iters=100)
        src = torch.from_numpy(D.port_source(dev, 0)).to("cuda:0")
        t0 = time.perf_counter()
        _, _, infos = fit.sweep([g], oms, [src[None, :]], tol=1e-8, max_iters=50000, precision="fp64")
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        ok = [k for k, i in enumerate(infos) if i["status"] == 0 and i["true_relres"] <= 1e-8]
        its = [i["iterations"] for i in infos]
        out.append({"device": dev.name, "cells": [dev.ncx, dev.ncy, dev.ncz], "unknowns": dev.n_edges,
                    "systems_per_batch": batch, "tile": list(g.tile("c128_batched")), "points": len(oms),
                    "converged": len(ok), "wall_s": round(dt, 1), "iterations": [min(its), max(its)],
                    "missed": [[round(oms[k] / 2 / np.pi / 1e9, 2), f"{infos[k]['true_relres']:.1e}"]
                               for k in range(len(oms)) if k not in ok]})
        _progress(f"family {dev.name}: {len(ok)}/{len(oms)} in {dt:.1f} s")
        del g, src
        torch.cuda.empty_cache()
    return {"workload": "six sweep-family devices, 8 of 64 log-spaced frequencies 1-40 GHz, port 1, "
                        "complex128 COCG, true relative residual 1e-8, cap 50k iterations", "devices": out}


def family_full_row(fit, D, np, torch):
    """The sweep at full size on the two smallest sweep-family devices
    (64x64x32 and 96x96x48 cells): all 64 log-spaced frequencies over
    1-40 GHz times all 4 port excitations (256 systems each), complex128,
    cap 50k iterations, in fit_sweep calls of 8 frequencies.  Not part of the
    default run (about five minutes)."""
    oms = D.log_spaced_omegas(64)
    out = []
    for dev in D.sweep_devices()[:2]:
        g = fit.Grid(dev)
        srcs = torch.stack([torch.from_numpy(D.port_source(dev, p)) for p in range(4)]).to("cuda:0")
        batch, _ = g.autotune_sweep(oms[:16], iters=100)
        ok, total, wall, its, missed = 0, 0, 0.0, [], []
        for c in range(0, 64, 8):
            o = oms[c:c + 8]
            t0 = time.perf_counter()
            _, _, infos = fit.sweep([g], o, [srcs], tol=1e-8, max_iters=50000, precision="fp64")
            torch.cuda.synchronize()
            wall += time.perf_counter() - t0
            for k in range(len(o)):
                for r in range(4):
                    i = infos[k * 4 + r]
                    total += 1
                    its.append(i["iterations"])
                    if i["status"] == 0 and i["true_relres"] <= 1e-8:
                        ok += 1
                    else:
                        missed.append([round(o[k] / 2 / np.pi / 1e9, 2), r, f"{i['true_relres']:.1e}"])
            _progress(f"family_full {dev.name}: {c + len(o)}/64 frequencies, {ok}/{total} at 1e-8")
        out.append({"device": dev.name, "cells": [dev.ncx, dev.ncy, dev.ncz], "unknowns": dev.n_edges,
                    "systems": total, "converged": ok, "systems_per_batch": batch,
                    "tile": list(g.tile("c128_batched")), "wall_s": round(wall, 1),
                    "systems_per_s": round(ok / wall, 3), "iterations": [min(its), max(its)],
                    "missed": missed})
        del g, srcs
        torch.cuda.empty_cache()
    return {"workload": "64 log-spaced frequencies 1-40 GHz x 4 port excitations on the 64x64x32 and "
                        "96x96x48 sweep-family devices, complex128 COCG, true relative residual 1e-8",
            "devices": out}


def _sweep_cpu_point(arg):
    """One sweep point of the oracle in a pool worker (one thread):
    assembly and scaling, 20 COCG iterations, extrapolated to `iters`."""
    om, iters = arg
    from threadpoolctl import threadpool_limits
    import scipy.sparse as sp

    from oracle import fit_oracle as O
    from paper_1705_08849_amd import devices as D
    sd = D.sweep_devices(seeds=[40], shapes=[(64, 64, 32)])[0]
    with threadpool_limits(1):
        t0 = time.perf_counter()
        a = O.system_matrix(sd, om)
        s = O.sym_scaling(sd, om)
        as_ = (sp.diags(s) @ a @ sp.diags(s)).tocsr()
        b = s * O.rhs(sd, om, D.port_source(sd, 0))
        t1 = time.perf_counter()
        O.cocg(as_, b, tol=1e-30, maxiter=20)
        t2 = time.perf_counter()
    return (t1 - t0) + (t2 - t1) / 20 * iters


def precond_row(fit, D, np, torch, with_cpu):
    """The learned preconditioner: one application on the 192x192x96-cell
    family device against the BF16 MFMA peak, and one training step."""
    fd = D.learned_family_device(9000)
    g = fit.Grid(fd)
    c = 16
    pre = fit.Precond.create(base_channels=c, seed=1)
    v = torch.randn(fd.n_edges, dtype=torch.complex128, device="cuda:0")
    om = 2 * np.pi * 1e10
    pre.apply(g, om, v)
    torch.cuda.synchronize()
    n = 5
    t0 = time.perf_counter()
    for _ in range(n):
        pre.apply(g, om, v)
    torch.cuda.synchronize()
    ta = (time.perf_counter() - t0) / n
    X, Y, Z = [(k + 1 + 3) // 4 * 4 for k in (fd.ncx, fd.ncy, fd.ncz)]
    v1 = X * Y * Z
    # (K, N, rows) of the 15 GEMMs of one forward pass
    lay = [(27 * 16, c, v1), (27 * c, c, v1), (8 * c, 2 * c, v1 / 8), (27 * 2 * c, 2 * c, v1 / 8),
           (27 * 2 * c, 2 * c, v1 / 8), (8 * 2 * c, 4 * c, v1 / 64), (27 * 4 * c, 4 * c, v1 / 64),
           (27 * 4 * c, 4 * c, v1 / 64), (4 * c, 16 * c, v1 / 64), (27 * 4 * c, 2 * c, v1 / 8),
           (27 * 2 * c, 2 * c, v1 / 8), (2 * c, 8 * c, v1 / 8), (27 * 2 * c, c, v1),
           (27 * c, c, v1), (c, 6, v1)]
    flops = sum(2.0 * k * nn * m for k, nn, m in lay)
    sd = D.layered_device(48, 48, 32, n_layers=4, n_strips=3, n_ports=1, seed=4)
    gt = fit.Grid(sd)
    fit.Precond.train([gt], [2 * np.pi * 5e9], base_channels=c, steps=2, batch=4, crop=32, seed=3)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fit.Precond.train([gt], [2 * np.pi * 5e9], base_channels=c, steps=20, batch=4, crop=32, seed=3)
    torch.cuda.synchronize()
    tt = (time.perf_counter() - t0) / 20
    row = {"workload": "3-level U-Net (c=16) preconditioner application on the 192x192x96-cell "
                       "family device (seed 9000); training steps of 4 crops of 32^3 nodes",
           "apply_ms": round(ta * 1e3, 3),
           "roofline": {"bound": "mfma", "achieved": round(flops / ta / 1e12, 2), "peak": 2500.0,
                        "unit": "TFLOP/s", "frac": round(flops / ta / 1e12 / 2500.0, 4),
                        "traffic": None},
           "train_step_ms": round(tt * 1e3, 3)}
    if with_cpu:
        from oracle import fit_oracle as O
        from oracle import unet_oracle as U
        small = D.layered_device(47, 47, 23, n_layers=3, n_strips=2, n_ports=1, seed=6)
        free = O.free_edges(small)
        p = U.init_params(c, seed=1)
        vv = np.where(free, 1.0 + 0.0j, 0.0)
        t0 = time.perf_counter()
        U.apply(small, om, p, vv, free, c=c, bf16=False)
        tc = time.perf_counter() - t0
        scale = v1 / (48 * 48 * 24)
        row["cpu_baseline"] = {"value": round(1.0 / (tc * scale), 5), "unit": "applications/s",
                               "cores": int(__import__("torch").get_num_threads()), "kind": "oracle",
                               "sample": "one oracle application (plain PyTorch CPU fp64) on a "
                                         "48x48x24-node device, scaled by voxel count"}
    return row


def interconnect_row(fit, D, np, torch, mean_us):
    """The 256x256x128-cell interconnect (25.6M unknowns, 835 MB per complex128
    operator application, beyond the 256 MB last-level cache): the plain
    operator's bandwidth and the copy bandwidth on vectors of its size, one
    COCG complex128 solve at 10 GHz, and the fused COCG step's HIP-event
    time per launch during that solve."""
    dev = D.interconnect_256(3)
    nx, ny, nz = dev.nodes
    n_nodes, n_cells = nx * ny * nz, dev.ncx * dev.ncy * dev.ncz
    om = 2 * np.pi * 10e9
    g = fit.Grid(dev)
    if os.path.exists(TUNE_FILE):
        fit.tune_load(TUNE_FILE)  # the committed table's tile for this grid, if it has one
    xv = torch.randn(dev.n_edges, dtype=torch.complex128, device="cuda:0")
    yv = torch.empty_like(xv)
    mv_us = mean_us(lambda: g.matvec(om, xv, yv, scaling="none"))
    mv_bytes = n_nodes * 6 * 16 + n_cells
    cp_us = mean_us(lambda: yv.copy_(xv))
    copy_gbs = 2 * xv.numel() * 16 / cp_us / 1e3
    x32 = xv.to(torch.complex64)
    y32 = torch.empty_like(x32)
    mv32_us = mean_us(lambda: g.matvec(om, x32, y32, scaling="none"))
    mv32_bytes = n_nodes * 6 * 8 + n_cells
    del xv, yv, x32, y32
    src = torch.from_numpy(D.port_source(dev, 0)).to("cuda:0")
    torch.cuda.synchronize()
    fit.profile_start()
    t0 = time.perf_counter()
    x, info = g.solve(om, src, tol=1e-8, solver="cocg", raise_on_error=False)
    torch.cuda.synchronize()
    ts = time.perf_counter() - t0
    stats = fit.profile_stop()
    launches, total_ms = stats.get("pcocg_step1_c128", (0, 0.0))
    step_us = total_ms * 1e3 / launches if launches else None
    step_bytes = n_nodes * 3 * 16 * 6 + n_cells
    row = {"workload": "256x256x128-cell graded interconnect (seed 3, 8 layers, 12 PEC strips, one "
                       "50-Ohm port), 10 GHz, COCG complex128 to 1e-8, symmetric scaling",
           "unknowns": dev.n_edges,
           "status": info["status_name"], "iterations": info["iterations"],
           "true_relres": info["true_relres"], "solve_s": round(ts, 2),
           "points_per_s": round((1.0 if info["status_name"] == "FIT_OK" else 0.0) / ts, 5),
           "matvec": {"kernel": "matvec A(omega) c128", "us": round(mv_us, 2),
                      "achieved": round(mv_bytes / mv_us / 1e3, 1), "unit": "GB/s",
                      "frac": round(mv_bytes / mv_us / 1e3 / HBM_PEAK_GBS, 4), "alg_bytes": mv_bytes,
                      "copy_gbs": round(copy_gbs, 1),
                      "frac_of_copy": round(mv_bytes / mv_us / 1e3 / copy_gbs, 4),
                      "timing": "mean of 20 back-to-back launches, HIP events"},
           "matvec_c64": {"us": round(mv32_us, 2), "achieved": round(mv32_bytes / mv32_us / 1e3, 1),
                          "unit": "GB/s", "frac": round(mv32_bytes / mv32_us / 1e3 / HBM_PEAK_GBS, 4),
                          "alg_bytes": mv32_bytes}}
    if step_us:
        row["pcocg_step1_c128"] = {"avg_launch_us": round(step_us, 2), "launches": launches,
                                   "alg_bytes_per_launch": step_bytes,
                                   "achieved": round(step_bytes / step_us / 1e3, 1), "unit": "GB/s",
                                   "frac": round(step_bytes / step_us / 1e3 / HBM_PEAK_GBS, 4)}
    del x, src, g
    torch.cuda.empty_cache()
    return row


def mean_us(fn, reps=20):
    """Mean launch time over `reps` back-to-back launches between two HIP
    events on torch's current stream, which the launches use (events around
    each launch would add the event overhead)."""
    import torch
    for _ in range(3):
        fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) * 1000 / reps


def cpu_baseline(dev, omega, src, gpu_iters):
    """The FP64 oracle as it stands, one thread: assemble and scale the
    system, time 30 COCG iterations (about 10 s of CPU work in all),
    extrapolate one solve with the GPU's iteration count."""
    import numpy as np
    import scipy.sparse as sp
    from threadpoolctl import threadpool_limits

    from oracle import fit_oracle as O

    with threadpool_limits(1):
        t0 = time.perf_counter()
        a = O.system_matrix(dev, omega)
        s = O.sym_scaling(dev, omega)
        as_ = (sp.diags(s) @ a @ sp.diags(s)).tocsr()
        b = s * O.rhs(dev, omega, src)
        t1 = time.perf_counter()
        n_it = 30
        O.cocg(as_, b, tol=1e-30, maxiter=n_it)
        t2 = time.perf_counter()
    t_setup, t_iter = t1 - t0, (t2 - t1) / n_it
    per_point = t_setup + gpu_iters * t_iter
    return {
        "value": 1.0 / per_point,
        "unit": "freq-points/s",
        "cores": 1,
        "kind": "oracle",
        "sample": (f"oracle assembly+scaling of the 128^3 system ({t_setup:.1f} s) and "
                   f"{n_it} COCG iterations ({t_iter:.3f} s each) on 1 host thread; one point "
                   f"extrapolated with the GPU's {gpu_iters} iterations"),
        "host_cpus": os.cpu_count(),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--solver", default="cocg")
    ap.add_argument("--precision", default="fp64")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="run with the library's default tile shape")
    ap.add_argument("--autotune", action="store_true",
                    help="autotune the bench grid instead of reading the committed tile table")
    ap.add_argument("--save-tune", action="store_true",
                    help="with --autotune: write the tile table to the committed file")
    ap.add_argument("--tune-interconnect", action="store_true",
                    help="tune the 256x256x128 interconnect grid's tile on the COCG iteration and "
                         "add it to the committed tile table")
    ap.add_argument("--no-rows", action="store_true",
                    help="skip the secondary rows (256x256x128 interconnect, batched sweep, learned "
                         "preconditioner): only the bench grid runs")
    ap.add_argument("--row", choices=["sweep", "precond", "interconnect", "baseline", "solvers",
                                      "solvers128", "precision", "family", "family_full", "learned"],
                    help="run only this secondary row and print it as one JSON line")
    ap.add_argument("--counters", action="store_true",
                    help="run only the short sample profiled by the HBM-counter passes")
    ap.add_argument("--ingest", nargs=4, metavar=("FETCH_CSV", "WRITE_CSV", "FETCH_LOG", "WRITE_LOG"),
                    help="write the measured per-launch traffic from two counter CSVs and the "
                         "stdout of the two --counters runs")
    args = ap.parse_args()
    if args.ingest:
        cmds = ["rocprofv3 --pmc FETCH_SIZE -f csv -- python3 bench.py --counters",
                "rocprofv3 --pmc WRITE_SIZE -f csv -- python3 bench.py --counters"]
        ingest_counters(*args.ingest, cmds)
        return
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); "
              "frequency points shard across GPUs with no exchange, but nothing here "
              "launches on more than one device.", file=sys.stderr)
        sys.exit(2)
    if args.counters:
        counter_sample(args)
        return
    if args.tune_interconnect:
        import numpy as np

        import torch

        from paper_1705_08849_amd import devices as D
        from paper_1705_08849_amd import fit
        torch.cuda.init()
        if os.path.exists(TUNE_FILE):
            fit.tune_load(TUNE_FILE)
        g = fit.Grid(D.interconnect_256(3))
        tile, us = g.autotune_solver(2 * np.pi * 10e9, iters=400)
        fit.tune_save(TUNE_FILE)
        print(json.dumps({"interconnect_tile": tile, "us_per_iteration": us}), flush=True)
        return
    if args.row:
        import numpy as np
        import torch

        from paper_1705_08849_amd import devices as D
        from paper_1705_08849_amd import fit

        torch.cuda.init()
        if args.row == "interconnect":
            row = interconnect_row(fit, D, np, torch, mean_us)
        elif args.row == "baseline":
            row = baseline_row(fit, D, np, torch)
        elif args.row in ("solvers", "solvers128"):
            row = solvers_row(fit, D, np, torch, big=args.row == "solvers128")
        elif args.row == "learned":
            row = learned_row(fit, D, np, torch)
        elif args.row == "precision":
            row = precision_row(fit, D, np, torch)
        elif args.row == "family":
            row = family_row(fit, D, np, torch)
        elif args.row == "family_full":
            row = family_full_row(fit, D, np, torch)
        else:
            fn = {"sweep": sweep_row, "precond": precond_row}[args.row]
            row = fn(fit, D, np, torch, not args.no_cpu_baseline)
        print(json.dumps({"row": args.row, **row}), flush=True)
        return

    import numpy as np
    import torch

    from paper_1705_08849_amd import devices as D
    from paper_1705_08849_amd import fit

    dev = D.plain_device_128(2)
    freq = D.log_uniform_frequency(2)
    omega = 2 * np.pi * freq
    src_np = D.port_source(dev, 0)
    nx, ny, nz = dev.nodes
    n_nodes, n_cells = nx * ny * nz, dev.ncx * dev.ncy * dev.ncz

    torch.cuda.init()
    t0 = time.perf_counter()
    g = fit.Grid(dev)
    torch.cuda.synchronize()
    t_create = time.perf_counter() - t0
    src = torch.from_numpy(src_np).to("cuda:0")
    x = torch.empty_like(src)
    tile = bench_tile(fit, g, dev, omega, args)

    # plain operator bandwidth (the metric's second part)
    xv = torch.randn(dev.n_edges, dtype=torch.complex128, device="cuda:0")
    yv = torch.empty_like(xv)
    mv_us = mean_us(lambda: g.matvec(omega, xv, yv, scaling="none"))
    mv_bytes = n_nodes * 6 * 16 + n_cells
    # this device's copy bandwidth on vectors of the same size, as a
    # second reference besides the 8 TB/s peak (two 103 MB vectors fit the
    # 256 MB last-level cache: the HBM figures come from the interconnect row)
    cp_us = mean_us(lambda: yv.copy_(xv))
    copy_gbs = 2 * xv.numel() * 16 / cp_us / 1e3
    del xv, yv

    def step():
        xs, info = g.solve(omega, src, tol=1e-8, solver=args.solver, precision=args.precision,
                           x=x, raise_on_error=False)
        u = g.port_voltages(xs, noalloc=True)  # no allocation inside the timed region
        return info, u

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    fit.profile_start()
    t0 = time.perf_counter()
    infos = [step() for _ in range(args.steps)]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    stats = fit.profile_stop()
    elapsed = t1 - t0
    ok = [i for i, _ in infos if i["status_name"] == "FIT_OK" and i["true_relres"] <= 1e-8]
    value = len(ok) / elapsed

    kname = "pcocg_step1_c128" if args.solver == "cocg" and args.precision == "fp64" else None
    if kname is None or kname not in stats:
        kname = max(stats, key=lambda k: stats[k][1]) if stats else None
    roof = None
    if kname:
        launches, total_ms = stats[kname]
        avg_s = total_ms / 1e3 / launches
        # fused step-1 kernel: reads r, p_old and x, writes p_new, q and x
        # (6 complex 3-vectors per node) plus the 1-byte cell ids
        vec = 16 if kname.endswith("c128") else 8
        passes = {"pcocg_step1": 6, "cocg_step1": 4, "bicgstab_step1": 6, "bicgstab_step2": 4,
                  "gmres_matvec": 3, "residual": 3, "matvec": 2}
        base = kname.rsplit("_", 1)[0]
        alg = n_nodes * 3 * vec * passes.get(base, 2) + n_cells
        achieved = alg / avg_s / 1e9
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": measured_traffic(tile), "kernel": kname,
                "avg_launch_us": round(avg_s * 1e6, 2), "alg_bytes_per_launch": alg,
                "launches": launches, "frac_of_copy": round(achieved / copy_gbs, 4)}
    share = {k: round(v[1] / 1e3 / elapsed, 3) for k, v in sorted(stats.items())}
    iters = int(np.mean([i["iterations"] for i, _ in infos])) if infos else 0
    out = {
        "metric": METRIC,
        "value": round(value, 6),
        "unit": "freq-points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1000 * elapsed / max(1, args.steps), 1),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c128" if args.precision == "fp64" else "c64+c128",
        "data": "synthetic",
        "config": {
            "workload": (f"128x128x128-cell graded layered device (seed 2), one 50-Ohm port, "
                         f"f={freq / 1e9:.3f} GHz, {args.solver.upper()} {args.precision} to "
                         f"1e-8 true relative residual, symmetric scaling"),
            "cells": [dev.ncx, dev.ncy, dev.ncz],
            "unknowns": dev.n_edges,
            "solver": args.solver,
            "precision": args.precision,
            "tile": tile,
            "points_converged": len(ok),
            "iterations_per_point": iters,
            "true_relres": [i["true_relres"] for i, _ in infos],
            "grid_create_s": round(t_create, 4),
            "value_incl_grid_create": round(len(ok) / (elapsed + t_create), 6),
        },
        "matvec": {"kernel": "matvec A(omega) c128", "us": round(mv_us, 2),
                   "achieved": round(mv_bytes / mv_us / 1e3, 1), "unit": "GB/s",
                   "frac": round(mv_bytes / mv_us / 1e3 / HBM_PEAK_GBS, 4),
                   "alg_bytes": mv_bytes, "timing": "mean of 20 back-to-back launches, HIP events",
                   "copy_gbs": round(copy_gbs, 1),
                   "frac_of_copy": round(mv_bytes / mv_us / 1e3 / copy_gbs, 4)},
        "roofline": roof,
        "kernel_time_share": share,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(dev, omega, src_np, iters)
    # the plain operator's bandwidth on the largest single-GPU grid (its
    # working set exceeds the last-level cache), with the fused COCG step and
    # one solve there; --no-rows keeps only the bench grid (profiled runs)
    del g, x
    torch.cuda.empty_cache()
    if not args.no_rows:
        ic = interconnect_row(fit, D, np, torch, mean_us)
        out["matvec_128"] = out["matvec"]
        out["matvec"] = dict(ic["matvec"], grid="256x256x128 cells (835 MB per application)")
        out["rows"] = {"interconnect": ic,
                       "sweep": sweep_row(fit, D, np, torch, not args.no_cpu_baseline),
                       "precond": precond_row(fit, D, np, torch, not args.no_cpu_baseline)}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
