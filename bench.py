#!/usr/bin/env python3
"""Benchmark of the PIC hot path on one MI355X: particle pushes per second.

One step is the full leap-frog cycle (fused gather + Boris push + deposit per
tile, Yee updates of b and e, periodic counting-sort repacks).  The headline
workload (the default) is the thermal pair plasma: 64^3 cells, 64 pairs per
cell (33.5 M particles), theta = 0.1, dt = 0.5, n_x = 10.  --workload selects
one of the other families instead: counter-streaming beams 256x256x4, the
double Harris sheet 512x256x4, the ensemble of 256 boxes in one launch, or
the small 16^3 thermal box (8 pairs/cell), which is launch-bound.
All inputs are synthetic and seeded; they stand in for the paper's thermal,
beam and current-sheet test problems.

Prints ONE JSON line.  Besides the headline value it carries:
  roofline      the push kernel's algorithmic HBM bytes per launch divided by
                its average launch time (HIP events on the library's stream
                around each launch, over the timed steps), against 8 TB/s;
                traffic is the counter-measured HBM bytes per launch
                (FETCH_SIZE + WRITE_SIZE, scaled by a plain copy) when the
                committed counter summary matches the current kernel source;
  cpu_baseline  the FP64 CPU oracle timed on a bounded sample of the thermal
                workload on this host (thermal workload only);
  fp64_form     the same workload in the FP64 GPU form, and the speedup.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "particle pushes/s (gather+push+deposit) at 1 GPU; % HBM roofline vs FP64 form"
HBM_PEAK_GBS = 8000.0
# algorithmic bytes per cell of one FP32 push launch: e and b read (24),
# b^{t+dt/2} of the tile's cells written (12), current flushed (24)
PUSH_CELL_BYTES = 60.0
PMC_FILE = os.path.join(ROOT, "profiles", "push_kernel_{}_pmc.txt")
KERNEL_SRC = os.path.join(ROOT, "paper_1308_5892_amd", "csrc", "pic_kernels.hip")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_sha():
    return hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()[:16]


def pmc_traffic(workload):
    """Counter-based HBM bytes per push launch from the committed summary, or
    None when it is missing or was taken on another version of the kernel."""
    path = PMC_FILE.format(workload)
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel_source_sha256_16") != kernel_sha():
        return None
    try:
        return float(kv["fetch_bytes_per_launch"]) + float(kv["write_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def harris_parameters(w):
    """Relativistic Harris equilibrium (App. C) for the sheet workload: current
    sheet half-thickness L in cells and b0 = omega_ce in code units, from the
    electron temperature, the electron drift Gamma_e U_e / c, chi and the mass
    ratio; d_e = n_x cells at the peak density."""
    r = math.sqrt(4.0 * w["chi"] * w["theta_e"])              # omega_ce / omega'_pe
    gamma = math.sqrt(1.0 + w["gu_e"] ** 2)
    L_de = 2.0 * w["theta_e"] / (r * w["gu_e"]) * math.sqrt(gamma)
    return {"L": L_de * w["n_x"], "b0": r / math.sqrt(gamma) / w["n_x"],
            "theta_i": (2.0 * w["chi"] - 1.0) * w["theta_e"] / w["mass_ratio"],
            "gu_i": (2.0 * w["chi"] - 1.0) * w["gu_e"]}


# box classes of the ensemble breakdown, by pairs per cell per species
ENSEMBLE_CLASSES = (("ppc 4-15", 4, 16), ("ppc 16-63", 16, 64), ("ppc 64-256", 64, 257))


def workload(name, tile, ppc_range=None):
    """Boxes, species, dt, loads (pic_load_desc list) and Harris fields of one
    workload family, with every box on the given tile shape.  For the ensemble,
    ppc_range = (lo, hi) keeps only the boxes with lo <= ppc < hi."""
    from paper_1308_5892_amd import pic as P
    import pic_inputs as W
    pair = [(-1.0, 1.0), (1.0, 1.0)]
    harris = []
    if name in ("thermal64", "thermal16"):
        w = W.THERMAL64 if name == "thermal64" else W.THERMAL16
        cells = w["dims"][0] * w["dims"][1] * w["dims"][2]
        npairs = w["ppc"] * cells
        boxes = [{"n": w["dims"], "n_x": w["n_x"], "rho0": 2.0 * w["ppc"], "max_particles": [npairs, npairs],
                  "tile": tile}]
        species, dt = pair, w["dt"]
        loads = [P.load_desc(0, 0, 1, (w["theta"], 0.0, 1), (w["theta"], 0.0, 1), w["ppc"], seed=w["seed"])]
    elif name == "beams":
        w = W.FILAMENT
        cells = w["dims"][0] * w["dims"][1] * w["dims"][2]
        npairs = 2 * w["ppc_per_beam"] * cells
        boxes = [{"n": w["dims"], "n_x": w["n_x"], "rho0": w["rho0"], "max_particles": [npairs, npairs],
                  "tile": tile}]
        species, dt = pair, w["dt"]
        gb = math.sqrt(w["gamma"] ** 2 - 1.0)
        loads = [P.load_desc(0, 0, 1, (w["theta"], sg * gb, 0), (w["theta"], sg * gb, 0), w["ppc_per_beam"],
                             seed=w["seed"], stream=k) for k, sg in ((0, 1.0), (1, -1.0))]
    elif name == "harris":
        w = W.HARRIS
        hp = harris_parameters(w)
        nx, ny, nz = w["dims"]
        cells = nx * ny * nz
        L, hw = hp["L"], nx / 4.0
        n_sheet = round(w["ppc"] * (cells / nx) * 2 * L * math.tanh(hw / L))
        npairs = 2 * n_sheet + round(w["background"] * w["ppc"] * cells)
        boxes = [{"n": w["dims"], "n_x": w["n_x"], "rho0": w["rho0"], "max_particles": [npairs + 64] * 2,
                  "tile": tile}]
        species, dt = [(-1.0, 1.0), (1.0, w["mass_ratio"])], w["dt"]
        harris = [(0, 0, 1, hp["b0"], L, [nx / 4.0, 3.0 * nx / 4.0])]
        loads = [P.load_desc(0, 0, 1, (w["theta_e"], -sg * w["gu_e"], 2), (hp["theta_i"], sg * hp["gu_i"], 2),
                             w["ppc"], seed=w["seed"], stream=k, profile=1, profile_axis=0, centre=c, thickness=L,
                             half_width=hw)
                 for k, (c, sg) in enumerate(((nx / 4.0, 1.0), (3.0 * nx / 4.0, -1.0)))]
        loads.append(P.load_desc(0, 0, 1, (w["theta_e"], 0.0, 2), (hp["theta_i"], 0.0, 2),
                                 w["background"] * w["ppc"], seed=w["seed"], stream=2))
    elif name == "ensemble":
        spec = W.ENSEMBLE
        blist = W.ensemble_boxes(spec)
        if ppc_range is not None:
            blist = [bx for bx in blist if ppc_range[0] <= bx["ppc"] < ppc_range[1]]
        boxes = []
        for bx in blist:
            n = bx["dims"][0] * bx["dims"][1] * bx["dims"][2] * bx["ppc"]
            boxes.append({"n": bx["dims"], "n_x": spec["n_x"], "rho0": 2.0 * bx["ppc"], "max_particles": [n, n],
                          "tile": tile})
        species, dt = pair, spec["dt"]
        loads = [P.load_desc(i, 0, 1, (bx["theta"], 0.0, 1), (bx["theta"], 0.0, 1), bx["ppc"], seed=bx["seed"])
                 for i, bx in enumerate(blist)]
    else:
        raise SystemExit(f"unknown workload {name}")
    return {"boxes": boxes, "species": species, "dt": dt, "loads": loads, "harris": harris,
            "thetas": [bx["theta"] for bx in blist] if name == "ensemble" else None}


def make_sim(wl, fp64, sort_interval):
    """Build and load a workload; returns (sim, particles, cells)."""
    from paper_1308_5892_amd import pic as P
    sim = P.Simulation(wl["boxes"], wl["species"], wl["dt"], fp64=fp64, sort_interval=sort_interval,
                       filter_current=wl.get("filter", False))
    for h in wl["harris"]:
        sim.harris_field(*h)
    for d in wl["loads"]:
        P.pic_load_maxwell_juttner(sim.ctx, d)
    sim.step(0)  # bin the loaded pairs and integrate u back by dt/2
    npart = sum(int(sim.diag(i)["count"].sum()) for i in range(len(sim.boxes)))
    ncell = sum(b["n"][0] * b["n"][1] * b["n"][2] for b in wl["boxes"])
    return sim, npart, ncell


WORKLOAD_TEXT = {
    "thermal64": "thermal pair plasma 64^3, 64 pairs/cell, theta=0.1, dt=0.5, n_x=10",
    "thermal16": "thermal pair plasma 16^3, 8 pairs/cell, theta=0.1, dt=0.5, n_x=10 (launch-bound; not a roofline case)",
    "beams": "counter-streaming pair beams 256x256x4, gamma=3 along +-x, 32 pairs/cell/beam, theta=0.01, n_x=20",
    "harris": "double Harris sheet 512x256x4, m_i/m_e=25, theta_e=1, 64 pairs/cell at peak, background 0.1, n_x=15",
    "ensemble": "ensemble of 256 periodic thermal boxes, edges 8..32, 4..256 pairs/cell, theta 0.05..1, n_x=10",
}


def time_form(wl, fp64, steps, warmup, sort_interval, made=None):
    """Load a workload (or take the loaded `made` = make_sim(...)), run
    `warmup` untimed steps, then time `steps` steps; the push launches are
    timed by the library's events (mode 2: no events around the other
    launches, which would add to the step time)."""
    import torch
    from paper_1308_5892_amd import pic as P
    sim, npart, cells = made if made is not None else make_sim(wl, fp64, sort_interval)
    torch.cuda.synchronize()
    if warmup:
        sim.step(warmup)
    torch.cuda.synchronize()
    P.pic_set_timing(sim.ctx, 2)      # events around the push launches only
    t0 = time.perf_counter()
    sim.step(steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    tm = P.pic_get_timing(sim.ctx)
    ds = [sim.diag(i) for i in range(len(sim.boxes))]
    d = {"flags": 0, "count": 0, "gauss_max": 0.0, "n_overflow": 0}
    for x in ds:
        d["flags"] |= x["flags"]
        d["count"] += int(x["count"].sum())
        d["n_overflow"] += int(x["n_overflow"].sum())
        d["gauss_max"] = max(d["gauss_max"], x["gauss_max"])
    sim.close()
    return {"seconds": t1 - t0, "npart": npart, "cells": cells, "timing": tm, "diag": d}


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, all_steps=3):
    """The FP64 oracle on this host's cores, on the workload's own shape (its
    cells, density and temperature), built -O3 -march=native with OpenMP:
    loaded and integrated back by dt/2 with all threads, then one full step on
    one thread and `all_steps` full steps on all threads (OMP_NUM_THREADS, else
    every core), each timed."""
    from oracle import oracle as O
    L = O.lib_native()
    nthreads = L.orc_threads(0)
    dims = tuple(w["dims"])
    npairs = w["ppc"] * dims[0] * dims[1] * dims[2]
    sp = {"theta": w["theta"], "gb": 0.0, "axis": 1}
    x, ua, ub = O.load_pairs(dims, w["seed"], 0, npairs, sp, sp, lib_=L)
    st = O.State(dims, w["dt"], w["n_x"], 2.0 * w["ppc"], [(-1.0, 1.0), (1.0, 1.0)], L=L)
    st.add_particles(0, x, ua)
    st.add_particles(1, x, ub)
    del x, ua, ub
    st.backward_half()
    L.orc_threads(1)
    t0 = time.perf_counter()
    st.step(1)
    t1 = time.perf_counter() - t0
    L.orc_threads(nthreads)
    t0 = time.perf_counter()
    st.step(all_steps)
    tn = time.perf_counter() - t0
    one = 2 * npairs / t1
    return {"value": 2 * npairs * all_steps / tn, "unit": "pushes/s", "cores": nthreads, "kind": "oracle",
            "single_thread": one, "host": {"nproc": os.cpu_count(), "cpu_model": cpu_model()},
            "build": "gcc -O3 -march=native -fopenmp (per-thread current, added in thread order)",
            "sample": f"{dims[0]}x{dims[1]}x{dims[2]} cells at {w['ppc']} pairs/cell, theta={w['theta']} "
                      f"(the workload itself): {all_steps} full steps on {nthreads} threads "
                      f"({2 * npairs * all_steps} pushes, {tn:.1f} s) and 1 step on one thread ({t1:.1f} s)"}


def copy_calibration(nbytes):
    """A plain device copy of known size, for scaling the FETCH_SIZE/WRITE_SIZE
    counters of a --pmc run."""
    import torch
    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    log(f"copy calibration: 3 copies of {nbytes} bytes")


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", default="thermal64", choices=sorted(WORKLOAD_TEXT),
                    help="thermal64 (the headline line) or one of the other workload families")
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--tile", type=int, nargs=3, default=(4, 4, 4))
    ap.add_argument("--sort-interval", type=int, default=200)
    ap.add_argument("--fp64-steps", type=int, default=40)
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 GPU form")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--filter-current", action="store_true",
                    help="smooth the current with the 27-point filter before it enters e")
    ap.add_argument("--autotune", action="store_true",
                    help="pick tile shapes and sort interval with pic_autotune before timing")
    ap.add_argument("--no-workloads", action="store_true",
                    help="thermal64: skip timing the beam, Harris and ensemble workloads")
    ap.add_argument("--no-breakdown", action="store_true",
                    help="ensemble: skip timing each box class (by pairs per cell) in its own launch")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="also run a plain copy of BYTES bytes (counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): this build has no multi-GPU path; "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import pic_inputs as W
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    wl = args.workload
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)

    spec = workload(wl, tuple(args.tile))
    spec["filter"] = args.filter_current
    sort_interval, tune = args.sort_interval, None
    if args.autotune:
        from paper_1308_5892_amd import pic as P
        boxes, sort_interval, tune = P.autotune(spec["boxes"], spec["species"], spec["dt"], spec["loads"], steps=10,
                                                sort_interval=args.sort_interval)
        spec["boxes"] = boxes
        shapes = sorted({tuple(b["tile"]) for b in boxes})
        tune.update({"tiles": [list(t) for t in shapes], "sort_interval": sort_interval})
        log(f"autotune: {tune}")
    # The FP32 workload is loaded first, then the FP64 form is measured, then
    # the FP32 warm-up and timed steps follow at once: a GPU that starts
    # pushing from idle runs the push 10-20 % slower over its first ~30 steps
    # (its clock settling; the same after any pause of a second), and the
    # FP64 steps take it past that.
    made32 = make_sim(spec, False, sort_interval)
    fp64 = None
    if not args.no_fp64:
        log(f"FP64 form: {args.fp64_steps} timed steps")
        r64 = time_form(spec, True, args.fp64_steps, 5, sort_interval)
    log(f"FP32 form: {WORKLOAD_TEXT[wl]}, {args.warmup} warmup + {args.steps} timed steps")
    r32 = time_form(spec, False, args.steps, args.warmup, sort_interval, made=made32)
    npart, cells = r32["npart"], r32["cells"]
    value = npart * args.steps / r32["seconds"]
    tm = r32["timing"]
    push_avg_s = tm["push_ms"] / max(1, tm["push_launches"]) / 1e3
    # algorithmic bytes of one push launch: particle state read + written (28 B
    # each way: packed cell, 3 offsets, 3 momenta; the library stores the cell
    # of a binned particle as a one-byte tile-local code, so it moves 25 B each
    # way); per cell e and b read (6 x 4 B), b^{t+dt/2} written (3 x 4 B) and
    # the current flushed (3 x 8 B)
    push_bytes = 56.0 * npart + PUSH_CELL_BYTES * cells
    achieved = push_bytes / push_avg_s / 1e9
    traffic = pmc_traffic(wl)
    step_bytes = 56.0 * npart + 144.0 * cells
    log(f"FP32: {value / 1e9:.2f} G pushes/s, push kernel {push_avg_s * 1e3:.3f} ms "
        f"({achieved:.0f} GB/s)")

    if not args.no_fp64:
        v64 = r64["npart"] * args.fp64_steps / r64["seconds"]
        t64 = r64["timing"]
        p64 = t64["push_ms"] / max(1, t64["push_launches"]) / 1e3
        # this build's FP64 state is 49 B (one-byte tile-local cell, 3 FP64
        # offsets, 3 FP64 u), read and written; the plain FP64 form's count is
        # 48 B (six FP64 values) each way; both with 6 x 8 B fields read,
        # 3 x 8 B of b written and 3 x 8 B current flushed per cell
        b64 = 98.0 * npart + 96.0 * cells
        b64_plain = 96.0 * npart + 96.0 * cells
        fp64 = {"value": v64, "unit": "pushes/s", "steps": args.fp64_steps,
                "push_kernel_ms": p64 * 1e3, "roofline_frac": b64 / p64 / 1e9 / HBM_PEAK_GBS,
                "roofline_frac_96B": b64_plain / p64 / 1e9 / HBM_PEAK_GBS,
                "speedup_fp32_over_fp64": value / v64}
        log(f"FP64: {v64 / 1e9:.2f} G pushes/s, speedup {value / v64:.2f}x")

    cpu = None
    if not args.no_cpu and wl == "thermal64":
        log("CPU oracle baseline (bounded sample)")
        cpu = cpu_baseline(W.THERMAL64)
        log(f"CPU: {cpu['value'] / 1e6:.2f} M pushes/s")

    workloads = None
    if wl == "thermal64" and not args.no_workloads:
        # the other workload families under the same clock: same tiles, sort
        # interval, warm-up and timed steps as the headline
        workloads = []
        for name in ("beams", "harris", "ensemble"):
            sub = workload(name, tuple(args.tile))
            log(f"workload {name}: {WORKLOAD_TEXT[name]}")
            rw = time_form(sub, False, args.steps, args.warmup, sort_interval)
            tw = rw["timing"]
            pw = tw["push_ms"] / max(1, tw["push_launches"]) / 1e3
            bw = 56.0 * rw["npart"] + PUSH_CELL_BYTES * rw["cells"]
            workloads.append({"workload": WORKLOAD_TEXT[name], "particles": rw["npart"], "cells": rw["cells"],
                              "pushes_per_s": rw["npart"] * args.steps / rw["seconds"],
                              "ms_per_step": rw["seconds"] / args.steps * 1e3,
                              "push_kernel_ms": pw * 1e3, "roofline_frac": bw / pw / 1e9 / HBM_PEAK_GBS,
                              "flags": rw["diag"]["flags"], "overflow": rw["diag"]["n_overflow"]})
            log(f"  {workloads[-1]['pushes_per_s'] / 1e9:.2f} G pushes/s, push {pw * 1e3:.3f} ms, "
                f"roofline {workloads[-1]['roofline_frac']:.3f}")

    classes = None
    if wl == "ensemble" and not args.no_breakdown:
        # per-class throughput: each class of boxes in its own launch, same
        # tiles and sort interval, half the timed steps
        classes = []
        for label, lo, hi in ENSEMBLE_CLASSES:
            sub = workload(wl, tuple(args.tile), (lo, hi))
            if tune is not None:
                sub["boxes"] = [dict(b, tile=tuple(tune["tiles"][0])) for b in sub["boxes"]]
            rc = time_form(sub, False, max(1, args.steps // 2), args.warmup, sort_interval)
            pc = rc["timing"]["push_ms"] / max(1, rc["timing"]["push_launches"]) / 1e3
            bc = 56.0 * rc["npart"] + PUSH_CELL_BYTES * rc["cells"]
            classes.append({"class": label, "boxes": len(sub["boxes"]), "particles": rc["npart"],
                            "cells": rc["cells"], "mean_theta": sum(sub["thetas"]) / len(sub["thetas"]),
                            "pushes_per_s": rc["npart"] * max(1, args.steps // 2) / rc["seconds"],
                            "push_kernel_ms": pc * 1e3, "roofline_frac": bc / pc / 1e9 / HBM_PEAK_GBS,
                            "flags": rc["diag"]["flags"]})
            log(f"class {label}: {len(sub['boxes'])} boxes, {rc['npart']} particles, "
                f"{classes[-1]['pushes_per_s'] / 1e9:.2f} G pushes/s, roofline {classes[-1]['roofline_frac']:.3f}")

    d = r32["diag"]
    out = {
        "metric": METRIC, "value": value, "unit": "pushes/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": r32["seconds"] / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": WORKLOAD_TEXT[wl], "boxes": 256 if wl == "ensemble" else 1,
                   "cells": cells, "particles": npart,
                   "tile": list(args.tile) if tune is None else tune["tiles"],
                   "sort_interval": sort_interval, "autotune": tune, "filter_current": args.filter_current, "current": "int64 fixed point, 2^-31"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic,
                     "kernel": "push_kernel<float> (gather+push+deposit)",
                     "bytes_per_launch": push_bytes, "avg_launch_ms": push_avg_s * 1e3,
                     "whole_step_frac": value * step_bytes / npart / 1e9 / HBM_PEAK_GBS},
        "cpu_baseline": cpu,
        "fp64_form": fp64,
        "classes": classes,
        "workloads": workloads,
        "check": {"flags": d["flags"], "particles": d["count"], "gauss_max": d["gauss_max"],
                  "overflow": d["n_overflow"]},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
