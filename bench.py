"""Benchmark: Dufort-Frankel cell-updates/s on one MI355X.

Workload: 65,536 identical-grid walls (1001 nodes, 30 cm), per-wall material
scales log-uniform over a decade, random outdoor sinusoids, dt = 1 s (the
batched identical-grid configuration).  A step is one DF time step of the
whole batch (outdoor air, coefficients, moisture and heat updates, surface
fluxes and their compensated integrals).  Inputs are resident in HBM before
the timed region; the start-up step runs in the warm-up.

Prints one JSON line (value = FP64 cell-updates/s; the FP32 run of the same
batch is reported under "fp32").  Further keys measure the other batches in
the same run ("workloads": the uneven layered batch and the building batch,
each with its roofline), the DF step against the Euler-implicit comparator at
the setting of the paper's Table 3 ("table3"), the surface-flux surrogate
("surrogate": an ensemble of three networks trained on 65,536 walls x 156
windows of DF histories, about 10 M samples, its fallback threshold
calibrated on 2,048 other walls, error and speed-up measured on 4,096 more),
and the CPU oracle on samples of every batch ("cpu_baseline").
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

N_WALLS = 65536
NX = 1001
DT = 1.0
# Algorithmic floating-point operations per cell-update of the DF step (one
# node, both fields): face coefficients at the face state 21, node
# coefficients 17, moisture update 9, heat update 22 -- 69 operations, of
# which 2 exponentials and 4 divisions, each counted as one operation (FMA as
# two).  The per-wall outdoor air and flux work adds < 1 % at 1001 nodes.
FLOPS_PER_CELL = 69
# The same count under the Table 1 material law (streaming kernel): face law
# 73 (face state 4, saturation pressure 5, phi and its log 2, isotherm 36,
# delta_v 8, k_M 11, scaling 7), node law 51 (saturation pressure 5, phi
# and its log 2, isotherm 36, capacities 8), updates 31.
FLOPS_PER_CELL_TABLE1 = 155
# Minimum HBM bytes per cell-update of a streaming step: read T, P at n-1 and
# n, write T, P at n+1 (8 B each in FP64, 4 B in FP32).
BYTES_PER_CELL = {"f64": 48, "f32": 24}
PEAK = {"f64": 78.6, "f32": 157.3}       # TFLOP/s, MI355X vector
HBM_PEAK = 8000.0                         # GB/s


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5000)
    ap.add_argument("--warmup", type=int, default=1000)
    ap.add_argument("--schedule", default="resident", choices=["auto", "stream", "resident"])
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--walls", type=int, default=N_WALLS)
    ap.add_argument("--workload", default="identical",
                    choices=["identical", "layered", "building", "implicit", "table1"],
                    help="identical: the 65,536 x 1001 batch (the default and the headline); "
                         "layered: 100,000 uneven 1-3 layer walls (FP32, dt = 1 s); "
                         "building: 4,096 rooms x 6 walls coupled to the room-air balance; "
                         "implicit: the identical batch through the Euler-implicit and "
                         "Crank-Nicolson comparators against DF; table1: the identical "
                         "grid under the Table 1 material law")
    ap.add_argument("--rooms", type=int, default=4096)
    ap.add_argument("--radiation", action="store_true",
                    help="building workload with the radiative surface sources")
    ap.add_argument("--link-group", type=int, default=1,
                    help="building workload: rooms linked by airflow in chains of this many")
    ap.add_argument("--shape", default=None,
                    help="resident launch shape THREADSxNODES (e.g. 256x4); default: the library's")
    ap.add_argument("--dt", type=float, default=None)
    ap.add_argument("--cpu-walls", type=int, default=1024)
    ap.add_argument("--cpu-steps", type=int, default=10000)
    ap.add_argument("--precision", default="both", choices=["both", "fp64", "fp32"])
    ap.add_argument("--no-surrogate", action="store_true")
    ap.add_argument("--surrogate-epochs", type=int, default=60)
    ap.add_argument("--no-workloads", action="store_true",
                    help="skip the layered and building legs of the default line")
    ap.add_argument("--no-table3", action="store_true",
                    help="skip the DF vs Euler-implicit leg at the paper's Table 3 setting")
    ap.add_argument("--copy-calibration", type=int, default=0,
                    help="MiB copied by a plain device copy before the run (counter calibration)")
    return ap.parse_args()


SHAPE = (0, 0)


def run_gpu(dfhm, walls, cfg, prec, schedule, steps, warmup, rooms=None):
    import torch
    sched = {"auto": dfhm.SCHED_AUTO, "stream": dfhm.SCHED_STREAM,
             "resident": dfhm.SCHED_RESIDENT}[schedule]
    s = dfhm.Solver(walls, cfg, rooms=rooms, precision=prec, schedule=sched,
                    threads=SHAPE[0], npt=SHAPE[1])
    if schedule == "auto":
        s.autotune(probe_steps=50)
    s.step(warmup)
    s.sync()
    info = s.info()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    s.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    s.sync()
    ms = e0.elapsed_time(e1)
    now, integ = s.fluxes()
    finite = bool(np.all(np.isfinite(integ)))
    s.close()
    return ms, info, finite


COUNTERS = os.path.join(ROOT, "profiles", "counters_k_df_resident_65536x1001.md")
KERNEL_SOURCES = ("df_resident.hpp", "df_kernels.hpp", "dfhm_device.hpp")


def _counter_block():
    """Key/value lines of the last fenced block of the committed counter
    summary, or None when the kernel sources have changed since the counters
    were taken (their digest is recorded with them)."""
    import hashlib
    try:
        text = open(COUNTERS).read().split("```")
        block = text[-2] if len(text) >= 3 else ""        # the last fenced block
        kv = dict((k.strip(), v.strip()) for k, v in
                  (ln.split(":", 1) for ln in block.splitlines() if ":" in ln))
        h = hashlib.sha256()
        for f in KERNEL_SOURCES:
            h.update(open(os.path.join(ROOT, "paper_1703_10119_amd", "csrc", f), "rb").read())
        return kv if kv.get("kernel_sources_sha256") == h.hexdigest() else None
    except (OSError, ValueError):
        return None


def resident_traffic(dtype):
    """HBM bytes per 1000-step launch of the resident kernel on the 65,536 x
    1001 batch from the committed FETCH_SIZE / WRITE_SIZE counters (scaled by
    a plain copy's readings in the same profiled run), or None."""
    kv = _counter_block()
    try:
        gib = float(kv["copy.bytes"]) / 1024.0
        fetch = float(kv[f"{dtype}.fetch_kib"]) * gib / float(kv["copy.fetch_kib"])
        write = float(kv[f"{dtype}.write_kib"]) * gib / float(kv["copy.write_kib"])
        return round((fetch + write) * 1024.0)
    except (TypeError, KeyError, ValueError):
        return None


def counted_flops(dtype):
    """Floating-point operations per cell-update the hardware executed, from
    the committed counters (VALU FMA x 2 + MUL + ADD + transcendental, 64
    lanes per wave instruction), or None."""
    kv = _counter_block()
    try:
        return float(kv[f"{dtype}.valu_flops_per_cell"])
    except (TypeError, KeyError, ValueError):
        return None


def roofline(dtype, cells, steps, ms, info, law=0):
    if law == 1:                # Table 1 law: VALU-bound on either schedule
        launches = math.ceil(steps / info["chunk_steps"]) if info["schedule"] == 2 else steps
        per_launch_s = ms / 1e3 / launches
        ach = FLOPS_PER_CELL_TABLE1 * cells * steps / launches / per_launch_s / 1e12
        return {"bound": "alu", "achieved": round(ach, 3), "peak": PEAK[dtype], "unit": "TFLOP/s",
                "frac": round(ach / PEAK[dtype], 4), "traffic": None,
                "kernel": "k_df_resident" if info["schedule"] == 2 else "k_df_stream",
                "launch_ms": round(per_launch_s * 1e3, 4)}
    if info["schedule"] == 2:   # resident: VALU-bound, one launch per chunk
        launches = math.ceil(steps / info["chunk_steps"])
        per_launch_s = ms / 1e3 / launches
        flops = FLOPS_PER_CELL * cells * steps / launches
        ach = flops / per_launch_s / 1e12
        chunk_full = steps % info["chunk_steps"] == 0 and info["chunk_steps"] == 1000
        main_batch = cells == 65536 * NX
        out = {"bound": "alu", "achieved": round(ach, 3), "peak": PEAK[dtype],
               "unit": "TFLOP/s", "frac": round(ach / PEAK[dtype], 4),
               "traffic": resident_traffic(dtype) if chunk_full and main_batch else None,
               "kernel": "k_df_resident", "launch_ms": round(per_launch_s * 1e3, 3),
               "flops_per_cell": FLOPS_PER_CELL}
        if main_batch:
            out["traffic_source"] = (
                "rocprofv3 FETCH_SIZE / WRITE_SIZE of a 1000-step launch, "
                "profiles/counters_k_df_resident_65536x1001.md" if out["traffic"] is not None else
                "null: no 1000-step launch timed, or the committed counters are of other kernel sources")
            hw = counted_flops(dtype)
            if hw is not None:
                # what the VALU executed (each exponential and division expands
                # into its polynomial and Newton steps), beside the algorithmic count
                out["hw_flops_per_cell"] = hw
                out["hw_achieved"] = round(hw * cells * steps / launches / per_launch_s / 1e12, 3)
                out["hw_frac"] = round(out["hw_achieved"] / PEAK[dtype], 4)
        return out
    per_launch_s = ms / 1e3 / steps
    ach = BYTES_PER_CELL[dtype] * cells / per_launch_s / 1e9
    return {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK, "unit": "GB/s",
            "frac": round(ach / HBM_PEAK, 4), "traffic": None, "kernel": "k_df_stream",
            "launch_ms": round(per_launch_s * 1e3, 4)}


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(walls_fn, cfg, n_walls, steps):
    """The FP64 oracle on the host threads (at most 16, the machine's CPU share)
    over a bounded sample of the batch, plus a single-thread figure."""
    import oracle
    oracle.build()
    walls = walls_fn(n_walls)
    threads = max(1, min(16, len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity")
                         else (os.cpu_count() or 1)))
    sim = oracle.RefSim(walls, cfg)
    sim.step(1, threads=threads)          # start-up step outside the timing
    t = time.perf_counter()
    sim.step(steps, threads=threads)
    dt = time.perf_counter() - t
    cells = int(np.sum(walls["nx"])) * steps
    one = oracle.RefSim(walls_fn(16), cfg)
    one.step(1, threads=1)
    t1 = time.perf_counter()
    one.step(steps // 5, threads=1)
    dt1 = time.perf_counter() - t1
    cells1 = 16 * NX * (steps // 5)
    return {"value": cells / dt, "unit": "cell-updates/s", "cores": threads, "kind": "oracle",
            "single_thread_value": cells1 / dt1, "cpu_model": cpu_model(),
            "host_cpus": os.cpu_count(),
            "sample": f"{n_walls} walls x {NX} nodes x {steps} steps of the same batch "
                      f"(FP64 C oracle, OpenMP over walls), {dt:.1f} s; single thread: 16 walls x "
                      f"{steps // 5} steps, {dt1:.1f} s"}


def leg_batch(dfhm, wl, kind, steps, warmup, precisions=("fp32", "fp64"), dt=None,
              schedule="resident", n_walls=None, n_rooms=4096, radiation=False, link_group=1):
    """Cell-updates/s of one of the other batches (resident schedule by
    default), each precision with its roofline.  kind: "layered" (the uneven
    batch of 100,000 walls), "building" (4,096 rooms x 6 walls with the
    room-air balance) or "table1" (the identical grid under the Table 1 law)."""
    rooms = None
    law = 0
    if kind == "table1":
        dt = dt or 1.0
        law = 1
        walls = wl.table1_batch(n_walls or N_WALLS, seed=707, nx=NX)
        name = (f"identical-grid batch under the Table 1 material law: {len(walls['nx'])} walls x "
                f"{NX} nodes (30 cm), scales within 1.5x of the paper's material, dt = {dt:g} s")
    elif kind == "layered":
        dt = dt or 1.0
        walls = wl.layered_batch(n_walls or 100000, seed=303, dt=dt)
        name = (f"uneven batch: {len(walls['nx'])} walls, 1-3 layers of 1-20 cm, lognormal Nx "
                f"(median 300, 51-2001) capped at dt/dx <= 3333 s/m (the nonlinear stability "
                f"limit: 22 % of the walls), dt = {dt:g} s")
    else:
        dt = dt or 10.0
        walls, rooms = wl.building_batch(n_rooms, seed=404, dt=dt, radiation=radiation,
                                         link_group=link_group)
        name = (f"building batch: {n_rooms} rooms x 6 layered walls (Nx 101-801, capped at dt/dx "
                f"<= 3333 s/m: mean Nx {np.mean(walls['nx']):.0f}), room-air balance every step, "
                f"dt = {dt:g} s"
                + (", long-wave exchange among each room's surfaces and incident radiation"
                   if radiation else "")
                + (f", rooms linked in chains of {link_group} (0.3 h^-1 airflow)"
                   if link_group > 1 else ""))
    cfg = wl.default_config(dt=dt, law=law)
    cells = int(wl.total_nodes(walls))
    out = {"workload": name, "walls": len(walls["nx"]), "cells": cells, "dt_s": dt,
           "rooms": 0 if rooms is None else len(rooms["volume"]), "steps": steps}
    for key, prec, dtype in (("fp32", dfhm.FP32, "f32"), ("fp64", dfhm.FP64, "f64")):
        if key not in precisions:
            continue
        ms, info, fin = run_gpu(dfhm, walls, cfg, prec, schedule, steps, warmup, rooms)
        out[key] = {"value": cells * steps / (ms / 1e3), "ms_per_step": ms / steps,
                    "roofline": roofline(dtype, cells, steps, ms, info, law), "finite": fin,
                    "schedule": ["", "stream", "resident"][info["schedule"]],
                    "block_threads": info["block_threads"],
                    "nodes_per_thread": info["nodes_per_thread"]}
    return out


def leg_table3(dfhm, wl, torch, n_walls=N_WALLS, df_steps=1000, imp_steps=40):
    """The setting of the paper's Table 3: the 10 cm wall of the Table 1
    material on 101 nodes at dt* = 1e-3 (3.6 s), DF against Euler implicit
    with the fixed-point tolerance eta = 1e-2 dt* (Sec. 4, Sec. 5.2 and
    Algorithm 1), FP64, cost per step at equal dt on a batch of such walls."""
    walls = wl.paper_wall_batch(n_walls)
    dt, eta = 3.6, 1e-5
    cfg = wl.default_config(dt=dt, law=1)
    cells = n_walls * 101
    ms, info, fin = run_gpu(dfhm, walls, cfg, dfhm.FP64, "resident", df_steps, 10)
    df_ms = ms / df_steps
    stream = torch.cuda.current_stream()
    ic = dfhm.Implicit(walls, dt=dt, theta=1.0, eta=eta, max_iters=200, law=1)
    ic.step(2)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    ic.step(imp_steps)
    e1.record(stream)
    torch.cuda.synchronize()
    imp_ms = e0.elapsed_time(e1) / imp_steps
    it = ic.iterations()
    ic.close()
    return {"workload": f"{n_walls} walls of the paper's Sec. 4 / Table 3 case: 10 cm of the Table 1 "
                        f"material, 101 nodes, outdoor T 293.15 +- 10 K and RH 0.5 +- 0.2 (random "
                        f"phases), dt = 3.6 s (dt* = 1e-3)",
            "eta": eta, "df_ms_per_step": df_ms, "df_cell_updates_per_s": cells / (df_ms / 1e3),
            "df_finite": fin, "euler_implicit_ms_per_step": imp_ms,
            "euler_implicit_sub_iterations": it, "df_cost_fraction": df_ms / imp_ms,
            "paper": ("Table 3 (MATLAB, one Intel i7 core; context only): DF 150 s, Euler implicit "
                      "530 s with 3 sub-iterations per step: DF at 28 %")}


def cpu_by_config(wl, threads):
    """The FP64 oracle on bounded samples of the other batches (host threads:
    `threads`; the single wall on one thread), and the FP64 network oracle's
    forward pass."""
    import oracle
    from oracle import mlp_ref
    oracle.build()
    res = {}
    w = wl.single_wall()
    sim = oracle.RefSim(w, wl.default_config(dt=1.0))
    t = time.perf_counter()
    sim.step(86400, threads=1)
    dt = time.perf_counter() - t
    res["single_wall"] = {"value": 101 * 86400 / dt, "unit": "cell-updates/s", "cores": 1,
                          "sample": f"the whole run: 1 wall x 101 nodes x 86,400 steps, {dt:.2f} s"}
    walls = wl.layered_batch(100000, seed=303, dt=1.0)
    idx = np.argsort(walls["nx"], kind="stable")[np.linspace(0, 99999, 1000).astype(int)]
    sub = wl.subset(walls, idx)
    sim = oracle.RefSim(sub, wl.default_config(dt=1.0))
    sim.step(1, threads=threads)
    t = time.perf_counter()
    sim.step(1000, threads=threads)
    dt = time.perf_counter() - t
    res["layered"] = {"value": wl.total_nodes(sub) * 1000 / dt, "unit": "cell-updates/s",
                      "cores": threads, "sample": f"1,000 walls stratified by Nx x 1,000 steps, "
                                                  f"{dt:.2f} s"}
    for step_s in (60.0, 10.0):
        bw, br = wl.building_batch(4096, seed=404, dt=step_s)
        nr = 64
        bw = {k: np.ascontiguousarray(v[:6 * nr]) for k, v in bw.items()}
        br = {k: (np.ascontiguousarray(v[:nr]) if hasattr(v, "__len__") else v) for k, v in br.items()}
        n = int(round(86400 / step_s))
        sim = oracle.RefSim(bw, wl.default_config(dt=step_s), br)
        sim.step(1, threads=threads)
        t = time.perf_counter()
        sim.step(n, threads=threads)
        dt = time.perf_counter() - t
        res[f"building_dt{step_s:g}"] = {
            "value": wl.total_nodes(bw) * n / dt, "unit": "cell-updates/s", "cores": threads,
            "room_steps_per_s": nr * n / dt,
            "sample": f"{nr} rooms x 6 walls ({wl.total_nodes(bw)} cells) x 1 day at dt = {step_s:g} s "
                      f"({n} steps), {dt:.2f} s"}
    rng = np.random.default_rng(0)
    dims = (584, 512, 4, 8)
    theta = mlp_ref.init(584, 512, 4, seed=1, n_out=8)
    x = rng.normal(0, 1, (4096, 584))
    t = time.perf_counter()
    mlp_ref.forward(theta, x, dims)
    dt = time.perf_counter() - t
    res["surrogate_forward"] = {"value": 4096 / dt, "unit": "samples/s", "cores": threads,
                                "sample": f"FP64 network oracle (numpy), forward pass of 4,096 samples, "
                                          f"{dt:.2f} s"}
    return res


def other_workload(a, torch, dfhm, wl):
    """One of the other batches on its own line (--workload)."""
    precs = ("fp32", "fp64") if a.precision == "both" else (a.precision,)
    leg = leg_batch(dfhm, wl, a.workload, a.steps, a.warmup, precs, a.dt, a.schedule,
                    None if a.walls == N_WALLS else a.walls, a.rooms, a.radiation, a.link_group)
    out = {"metric": "DF cell-updates/s", "unit": "cell-updates/s", "n_gpus": 1,
           "steps": a.steps, "warmup": a.warmup, "higher_is_better": True, "data": "synthetic",
           "config": {k: leg[k] for k in ("workload", "walls", "cells", "dt_s", "rooms")}}
    out.update({k: leg[k] for k in precs})
    print(json.dumps(out), flush=True)


def implicit_workload(a, torch, dfhm, wl):
    """DF against the implicit comparators (fixed-point sub-iterations,
    eta = 1e-10) on the identical-grid batch at the same dt: cost per step."""
    walls = wl.uniform_batch(a.walls, seed=202, nx=NX)
    cfg = wl.default_config(dt=DT)
    cells = a.walls * NX
    out = {"metric": "DF vs implicit comparator, cell-updates/s at equal dt", "unit": "cell-updates/s",
           "n_gpus": 1, "data": "synthetic", "higher_is_better": True,
           "config": {"workload": "identical-grid batch: 65,536 walls x 1001 nodes (30 cm), dt = 1 s",
                      "walls": a.walls, "nx": NX, "dt_s": DT}}
    ms, info, fin = run_gpu(dfhm, walls, cfg, dfhm.FP64, a.schedule, a.steps, a.warmup)
    out["df_fp64"] = {"value": cells * a.steps / (ms / 1e3), "ms_per_step": ms / a.steps,
                      "steps": a.steps}
    steps = max(1, min(a.steps, 50))
    stream = torch.cuda.current_stream()
    for name, theta in (("euler_implicit", 1.0), ("crank_nicolson", 0.5)):
        ic = dfhm.Implicit(walls, dt=DT, theta=theta, eta=1e-10, max_iters=200)
        ic.step(2)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        ic.step(steps)
        e1.record(stream)
        torch.cuda.synchronize()
        ims = e0.elapsed_time(e1)
        it = ic.iterations()
        # algorithmic HBM bytes per node and sub-iteration: the two forward
        # sweeps read 4 + 5 values and write 2 + 2, the two back
        # substitutions read 3 + 4 and write 1 + 2 (8 B each): 200 B
        gbs = 200.0 * cells * it / (ims / 1e3 / steps) / 1e9
        out[name] = {"value": cells * steps / (ims / 1e3), "ms_per_step": ims / steps, "steps": steps,
                     "mean_sub_iterations": it,
                     "df_cost_fraction": (ms / a.steps) / (ims / steps),
                     "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK,
                                  "unit": "GB/s", "frac": round(gbs / HBM_PEAK, 4), "traffic": None,
                                  "kernel": "k_imp_step"}}
        ic.close()
    print(json.dumps(out), flush=True)


def main():
    a = parse()
    global SHAPE
    if a.shape:
        SHAPE = tuple(int(v) for v in a.shape.lower().split("x"))
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {a.gpus}); the batch shards by "
              "walls with no per-step communication, see the design notes", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1703_10119_amd import dfhm, workloads as wl
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if a.copy_calibration:
        n = a.copy_calibration * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if a.workload == "implicit":
        implicit_workload(a, torch, dfhm, wl)
        return
    if a.workload != "identical":
        other_workload(a, torch, dfhm, wl)
        return
    cfg = wl.default_config(dt=DT)
    walls = wl.uniform_batch(a.walls, seed=202, nx=NX)
    cells = a.walls * NX
    if a.precision == "fp32":
        ms32, info32, fin32 = run_gpu(dfhm, walls, cfg, dfhm.FP32, a.schedule, a.steps, a.warmup)
        print(json.dumps({"fp32_value": cells * a.steps / (ms32 / 1e3),
                          "roofline": roofline("f32", cells, a.steps, ms32, info32)}), flush=True)
        return
    ms64, info64, fin64 = run_gpu(dfhm, walls, cfg, dfhm.FP64, a.schedule, a.steps, a.warmup)
    value = cells * a.steps / (ms64 / 1e3)
    out = {
        "metric": "DF cell-updates/s (fp64 vs fp32 batched) + surrogate speedup at <=1% flux err",
        "value": value, "unit": "cell-updates/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": ms64 / a.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "identical-grid batch: 65,536 walls x 1001 nodes, 30 cm thick (the "
                               "batch names no thickness; 30 cm keeps dt/dx at 3333 s/m, within the "
                               "nonlinear scheme's stability limit), dt = 1 s, material scales "
                               "log-uniform over a decade, random outdoor sinusoids",
                   "walls": a.walls, "nx": NX, "dt_s": DT,
                   "schedule": ["", "stream", "resident"][info64["schedule"]],
                   "block_threads": info64["block_threads"],
                   "nodes_per_thread": info64["nodes_per_thread"],
                   "chunk_steps": info64["chunk_steps"]},
        "roofline": roofline("f64", cells, a.steps, ms64, info64),
        "finite": fin64,
    }
    if not a.no_fp32 and a.precision == "both":
        ms32, info32, fin32 = run_gpu(dfhm, walls, cfg, dfhm.FP32, a.schedule, a.steps, a.warmup)
        out["fp32"] = {"value": cells * a.steps / (ms32 / 1e3), "ms_per_step": ms32 / a.steps,
                       "dtype": "f32", "roofline": roofline("f32", cells, a.steps, ms32, info32),
                       "finite": fin32}
    if not a.no_workloads:
        out["workloads"] = {
            "layered": leg_batch(dfhm, wl, "layered", 1000, 100),
            "building": leg_batch(dfhm, wl, "building", 1000, 100, dt=10.0),
        }
    if not a.no_table3:
        out["table3"] = leg_table3(dfhm, wl, torch)
    if not a.no_surrogate:
        from paper_1703_10119_amd import surrogate as S
        # progress of the study's phases and training (stderr; the result
        # line alone goes to stdout)
        r = S.study(epochs=a.surrogate_epochs,
                    log=lambda *m: print(*m, file=sys.stderr, flush=True))
        kb = S.kernel_bench()
        out["surrogate"] = {
            "roofline": {"bound": "mfma", "achieved": round(kb["infer_tflops"], 2),
                         "peak": 2500.0, "unit": "TFLOP/s",
                         "frac": round(kb["infer_tflops"] / 2500.0, 4), "traffic": None,
                         "kernel": ("k_mlp_infer_fused + k_decode (dfhm_mlp_infer: forward pass "
                                    "and flux decode, batch 65,536; FLOPs = 2 per weight per sample)"),
                         "infer_ms": round(kb["infer_s"] * 1e3, 4),
                         "layered_forward_tflops": round(kb["forward_tflops"], 2),
                         "layered_forward_ms": round(kb["forward_s"] * 1e3, 4),
                         "train_step_tflops": round(kb["train_tflops"], 2)},
            "speedup": r["speedup"],
            "speedup_definition": ("executed: DF time of all held-out walls from their initial state "
                                   "to the end of each query window, over the time of the networks "
                                   "plus the DF re-run, from the initial state, of just the walls "
                                   "whose error estimate exceeds tau; both include solver set-up "
                                   "and flux read-back; summed over the query windows"),
            "speedup_network_only": r["speedup_network_only"],
            "err_target": "p99 <= 1% of the per-wall RMS flux, after fallback",
            "err_p99": r["err_p99"], "err_max": r["err_max"],
            "fallback_err_max": r["fallback_err_max"],
            "fallback_fraction": r["fallback_fraction"], "tau": r["tau"],
            "raw_err_p50": r["raw_err_p50"], "raw_err_p99": r["raw_err_p99"],
            "raw_frac_above_target": r["raw_frac_above_target"],
            "fp32_df_err_p99": r["fp32_df_err_p99"], "fp32_df_err_max": r["fp32_df_err_max"],
            "query_windows": [{k: (round(v, 5) if isinstance(v, float) else v) for k, v in w.items()}
                              for w in r["serve_windows"]],
            "test_walls": r["n_test"], "test_samples": r["samples"], "mlp_seconds": r["mlp_seconds"],
            "df_seconds": r["df_seconds"], "surrogate_seconds": r["surrogate_seconds"],
            "inference_tflops_end_to_end": r["mlp_tflops"], "train_tflops_end_to_end": r["train_tflops"],
            "ensemble": r["n_nets"],
            "train": {"walls": r["n_train"], "samples_per_epoch": r["n_train"] * S.N_WINDOWS,
                      "epochs": r["epochs"], "batch": r["batch"], "lr": r["lr"],
                      "seconds": r["train_seconds"], "data_seconds": r["data_seconds"]},
            "dtype": "bf16 (FP32 accumulate, FP32 master weights)"}
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(
            lambda n: wl.uniform_batch(N_WALLS, seed=202, nx=NX) if n == N_WALLS
            else wl.subset(wl.uniform_batch(N_WALLS, seed=202, nx=NX), np.arange(n)),
            cfg, a.cpu_walls, a.cpu_steps)
        out["cpu_baseline"]["by_config"] = cpu_by_config(wl, out["cpu_baseline"]["cores"])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
