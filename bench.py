#!/usr/bin/env python3
"""Throughput of the Active Flux step on one MI355X: DOF-updates/s, FP32-bulk vs FP64.

Workload: the isentropic vortex (strength 5, centre (5,5), background (1,1,1,1), gamma 1.4)
on a periodic 4096 x 4096 grid of [0,10]^2, Algorithm 1 with the correction term, CFL 0.3,
time step computed on the device before every step.  A step is one pass of the whole hot path
(point values at the intermediate and new time levels, Simpson fluxes, conservative update,
time-step reduction).  One DOF-update is one DOF site (cell average, corner, x- or y-edge
midpoint; a 4-vector) advanced one full step: 4 N^2 sites per step on a periodic grid.

Inputs are generated on the host and copied to HBM before the timed region.  The timed region
runs `--steps` steps with HIP events around every kernel on the library's stream (the events
give both the step time and the average duration of the dominant kernel for the roofline).

Prints one JSON line.  Only N=1 is supported: the run uses one GPU.
"""
from __future__ import annotations

import argparse
import hashlib
import re
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "DOF-updates/s per step, FP32-bulk vs FP64 on 1 GPU at stated L1 error"
PEAK_FP32 = 157.3  # TFLOP/s, MI355X vector FP32 (published)
PEAK_FP64 = 78.6   # TFLOP/s, MI355X vector FP64 (published)

# ------------------------------------------------------------------------------------------
# Algorithmic FLOPs of the point kernel per cell and step (add, sub, mul, div, sqrt, acos,
# asin = 1; FMA = 2), counted operation by operation from the exact-moment formulation that
# each path evaluates, for the generic subsonic DOF (one arc piece per arc set):
#   EG2 set-up, foot point and outputs                                    82
#   corner (full circle + two half circles + one quadrant arc set; the
#           half-circle moments 46 + 48 formed once per evaluation)      1443
#   x-edge (full circle + one half circle)                                575
#   y-edge                                                                580
#   per DOF: derivatives 16, correction 74, assembly 31, Simpson-in-time
#            fluxes 54 + sums (K 32, X/Y 16), wave speed 4               213 / 197 / 197
#   per cell: inverse Simpson 197, centre value 25, Simpson average 72,
#             monomials 120 + aspect 24, constants 2                       440
# (the EG2 figures include the set-up; the moments are those of the circle of radius c' tau,
# from scaled arc end points).  Algorithm 1 evaluates EG2 three times per DOF, the averaged
# linearisation twice (plus 32 for the mean of the adjacent averages).
# ------------------------------------------------------------------------------------------
EG2_K = {"fp32": 1443, "fp64": 1443}
EG2_X, EG2_Y = 575, 580
PER_DOF = 213 + 197 + 197
PER_CELL = 440
PEAK_NONPACKED = 78.6  # TFLOP/s: 256 CU x 4 SIMD x 16 lanes x 2 (FMA) x 2.4 GHz


def flops_per_cell(mode: int, prec: str) -> float:
    """Algorithmic FLOPs of the point kernel per cell-step (3 DOFs per cell)."""
    rounds = 3 if mode == 0 else 2
    extra = 0 if mode == 0 else 32
    return rounds * (EG2_K[prec] + EG2_X + EG2_Y) + PER_DOF + PER_CELL + extra


def source_hash() -> str:
    """Hash of the device code of the single-grid kernels: the device headers and the kernel
    part of af_lib.hip (before its host-runtime section).  Host-side changes leave it alone."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2508_06273_amd", "csrc")
    for f in ("af_device.hpp", "af_kernels.hpp", "af_step.hpp", "af_lib.hip"):
        with open(os.path.join(csrc, f), "r") as fh:
            text = fh.read()
        if f == "af_lib.hip":
            text = text.split("// Host runtime")[0]
        # comments and layout do not change the code
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]


def traffic_record(kernel: str, workload: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it was taken
    on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    r = rec.get(f"{kernel}|{workload}")
    if not r or r.get("source_sha") != source_hash():
        return None
    return r


def _counter_means(db: str, counter: str):
    """Mean value of one rocprofv3 counter per kernel name (rocpd SQLite output)."""
    import sqlite3
    con = sqlite3.connect(db)
    cur = con.cursor()
    cols = [d[0] for d in cur.execute("select * from counters_collection limit 1").description]
    acc = {}
    for row in cur.execute("select * from counters_collection"):
        d = dict(zip(cols, row))
        if d["counter_name"] == counter:
            acc.setdefault(d["kernel_name"], []).append(float(d["value"]))
    con.close()
    return acc


def record_traffic(fetch_db: str, write_db: str, copy_mib: int, n: int):
    """Write profiles/traffic.json from two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE, in
    KiB per dispatch) of `bench.py --calibrate-copy MIB`: each counter is scaled by what it
    reads for the elementwise copy kernel, which reads and writes exactly MIB MiB."""
    fetch = _counter_means(fetch_db, "FETCH_SIZE")
    write = _counter_means(write_db, "WRITE_SIZE")
    nb_kib = copy_mib * 1024.0
    cf = max(v for k, vals in fetch.items() if "elementwise" in k for v in vals)
    cw = max(v for k, vals in write.items() if "elementwise" in k for v in vals)
    sf, sw = nb_kib / cf, nb_kib / cw
    out = {"_calibration": {"copy_kib": nb_kib, "fetch_kib_read": cf, "write_kib_read": cw,
                            "fetch_scale": sf, "write_scale": sw}}
    for prec in ("f32", "f64"):
        for kname in ("k_points", "k_update"):
            kf = [v for k, vals in fetch.items() if f"{kname}_{prec}" in k or
                  (kname == "k_update" and "k_update" in k) for v in vals]
            kw = [v for k, vals in write.items() if f"{kname}_{prec}" in k or
                  (kname == "k_update" and "k_update" in k) for v in vals]
            if not kf or not kw:
                continue
            f_kib, w_kib = sum(kf) / len(kf), sum(kw) / len(kw)
            b = (f_kib * sf + w_kib * sw) * 1024.0
            out[f"{kname}|vortex{n}_fp{prec[1:]}"] = {
                "bytes_per_launch": round(b), "fetch_kib_raw": f_kib, "write_kib_raw": w_kib,
                "source_sha": source_hash()}
    path = os.path.join(ROOT, "profiles", "traffic.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)
    print(json.dumps(out, indent=1, sort_keys=True))


def run_gpu(st, prec, steps, warmup, stream):
    from paper_2508_06273_amd import af
    import torch
    s = af.Solver.for_state(st, precision=prec)
    s.set_stream(stream)
    s.run(1e9, 0.3, warmup)
    s.set_option(af.AF_OPT_TIMING, 1)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    w0 = time.perf_counter()
    t, n = s.run(1e9, 0.3, steps)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    ms = e0.elapsed_time(e1)
    kp, ku, nt = s.timing()
    out = s.get_state()
    dofs = s.dof_count()
    s.close()
    assert n == steps and nt == steps, (n, nt)
    return dict(ms_total=ms, wall_s=wall, ms_points=kp / nt, ms_update=ku / nt, t=out["t"],
                dofs=dofs, state=out)


def run_batched(prec, steps, warmup, stream, n_gl=2, step_kernel=None):
    """The batched workload (256 periodic grids, N ~ U{64..512}, own dt per grid): DOF-updates/s
    of one graph-captured launch sequence per step for all grids, on the schedule the
    autotuner picks during the warm-up run.  With `step_kernel` (AF_STEP_SPLIT or
    AF_STEP_PERSISTENT) the autotuner is off and that step kernel runs on the default tile
    order and update size; with the persistent kernel `ms_points` is the whole step."""
    from paper_2508_06273_amd import af, inputs as I
    import torch
    states = run_batched.states
    if states is None:
        states = run_batched.states = I.batched_states(n_gl=n_gl)
    b = af.BatchSolver.for_states(states, precision=prec)
    b.set_stream(stream)
    if step_kernel is None:
        b.set_option(af.AF_OPT_AUTOTUNE, 1)  # the warm-up run picks the schedule
    else:
        b.set_option(af.AF_OPT_STEP_KERNEL, step_kernel)
    b.run(1e9, 0.3, warmup)
    schedule = {"tile_order": ["xcd", "linear", "grids"][b.get_option(af.AF_OPT_TILE_ORDER)],
                "update_threads": b.get_option(af.AF_OPT_UPDATE_THREADS),
                "step_kernel": ["split", "persistent"][b.get_option(af.AF_OPT_STEP_KERNEL)]}
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    t, n = b.run(1e9, 0.3, steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    assert n == steps
    # per-kernel times from a few eager steps with events
    b.set_option(af.AF_OPT_TIMING, 1)
    b.run(1e9, 0.3, 16)
    kp, ku, nt = b.timing()
    dofs = b.dof_count()
    b.close()
    return dict(value=dofs * steps / (ms * 1e-3), ms_per_step=ms / steps,
                ms_points=kp / nt, ms_update=ku / nt, dofs=dofs, schedule=schedule,
                cells=sum(st.grid.nx * st.grid.ny for st in states), grids=len(states))


run_batched.states = None


def accuracy_ladder(sizes, t_end, stream):
    """Vortex convergence ladder: L1/Linf per conserved variable against the exact translated
    vortex at t_end, FP64 and FP32-bulk, with the observed order between successive sizes."""
    from paper_2508_06273_amd import af, inputs as I
    out = {"t_end": t_end, "cfl": 0.3, "variables": "rho, rho u, rho v, E", "sizes": {}}
    prev = None
    for n in sizes:
        print(f"[bench] ladder {n}^2", file=sys.stderr, flush=True)
        st = I.shu_vortex(n, n_gl=3)
        ex = I.cell_average(I.shu_vortex_field(t_end), st.grid, n_gl=3)
        rec = {}
        for prec, name in ((af.AF_PREC_FP64, "fp64"), (af.AF_PREC_FP32, "fp32")):
            s = af.Solver.for_state(st, precision=prec)
            s.set_stream(stream)
            t, steps = s.run(t_end, 0.3)
            avg = s.get_state()["avg"]
            s.close()
            l1, linf = I.norms(avg, ex, st.grid)
            # the window [2.5, 7.5]^2, away from the seams where the vortex's Gaussian tail is
            # not periodic
            w = slice(n // 4, 3 * n // 4)
            l1w = np.abs(avg[:, w, w] - ex[:, w, w]).reshape(4, -1).sum(axis=1) * \
                st.grid.dx * st.grid.dy
            rec[name] = {"steps": steps, "L1": [float(v) for v in l1],
                         "Linf": [float(v) for v in linf],
                         "L1_window": [float(v) for v in l1w]}
        if prev is not None:
            r = math.log(n / prev[0])
            rec["order_fp64"] = [float(math.log(a / b) / r)
                                 for a, b in zip(prev[1]["fp64"]["L1"], rec["fp64"]["L1"])]
            rec["order_fp64_window"] = [
                float(math.log(a / b) / r)
                for a, b in zip(prev[1]["fp64"]["L1_window"], rec["fp64"]["L1_window"])]
        out["sizes"][str(n)] = rec
        prev = (n, rec)
        del st, ex
    return out


def extra_workloads(stream):
    """Throughput of the two limiter workloads (averaged linearisation, positivity limiter on):
    the 2048^2 radial outflow (outflow boundaries, flux limiting of the averages on: all 500
    steps of the configuration, 10 warm-up + 490 timed) and the 8192^2 shear layer (10 warm-up
    + 100 timed steps), the latter also with Algorithm 2 and the shock-indicator blend; then
    the shock-reflection problem."""
    from paper_2508_06273_amd import af, inputs as I
    import torch
    out = {}
    for name, make, warm, steps in (("radial_outflow_2048", lambda: I.radial_state(2048, n_gl=2),
                                     10, 490),
                                    ("shear_layer_8192", lambda: I.shear_state(8192), 10, 100)):
        print(f"[bench] {name}", file=sys.stderr, flush=True)
        st = make()
        rec = {}
        legs = [(af.AF_PREC_FP32, "fp32", False), (af.AF_PREC_FP64, "fp64", False)]
        if name.startswith("shear"):
            # the same run with Algorithm 2 and the shock-indicator blend of Sec. 3.4 on
            legs += [(af.AF_PREC_FP32, "fp32_indicators", True),
                     (af.AF_PREC_FP64, "fp64_indicators", True)]
        for prec, pname, ind in legs:
            s = af.Solver.for_state(st, precision=prec, linearisation=af.AF_LIN_AVG, limiter=True,
                                    transonic=ind, shock_limiter=ind,
                                    flux_limiter=name.startswith("radial"))
            s.set_stream(stream)
            s.run(1e9, 0.3, warm)
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            t, n = s.run(1e9, 0.3, steps)
            e1.record(stream)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1)
            assert n == steps
            cnt = s.counters()
            rec[pname] = {"value": s.dof_count() * steps / (ms * 1e-3), "ms_per_step": ms / steps,
                          "t": t, "eg1_fallbacks": int(cnt[0]), "lf_fallbacks": int(cnt[1]),
                          "centre_fallbacks": int(cnt[2]), "transonic_flags": int(cnt[5]),
                          "flux_limited_faces": int(cnt[6])}
            s.close()
        rec["speedup_fp32_vs_fp64"] = rec["fp32"]["value"] / rec["fp64"]["value"]
        rec["steps"] = steps
        out[name] = rec
        del st
    out.update(shock_reflection(stream))
    return out


def pcie_inclusive(n, stream, steps=(1, 40)):
    """Whole-job rate when the state is handed over in host memory, as the C ABI's
    af_set_state / af_get_state do: copy the 4096^2 vortex in (host to device, pageable numpy
    arrays), run K steps, copy the state out, all timed on the host clock; also the two copies
    alone.  This is a reported figure beside the benchmark, never its value."""
    from paper_2508_06273_amd import af, inputs as I
    import torch
    st = I.shu_vortex(n, n_gl=3)
    out = {"workload": f"isentropic vortex {n}x{n}, Algorithm 1, CFL 0.3; state FP64 in host "
                       "memory (pageable) before and after", "state_bytes": int(
                           sum(getattr(st, k).nbytes for k in ("avg", "K", "X", "Y")))}
    for prec, name in ((af.AF_PREC_FP32, "fp32"), (af.AF_PREC_FP64, "fp64")):
        s = af.Solver.for_state(st, precision=prec)
        s.set_stream(stream)
        s.run(1e9, 0.3, 2)  # warm-up (graph capture, first launches)
        rec = {}
        t0 = time.perf_counter()
        s.set_state(st.avg, st.K, st.X, st.Y, st.t)
        t1 = time.perf_counter()
        s.get_state()
        t2 = time.perf_counter()
        rec["set_state_ms"] = (t1 - t0) * 1e3
        rec["get_state_ms"] = (t2 - t1) * 1e3
        for k in steps:
            t0 = time.perf_counter()
            s.set_state(st.avg, st.K, st.X, st.Y, st.t)
            s.run(1e9, 0.3, k)
            s.get_state()
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            rec[f"steps_{k}"] = {"ms": dt * 1e3, "dof_updates_per_s": s.dof_count() * k / dt}
        s.close()
        out[name] = rec
    return out


def _region_mean(avg, grid, box):
    """Mean primitive state of the cells whose centres lie in box = (x0, x1, y0, y1)."""
    xc, yc = grid.cell_centres()
    m = (xc > box[0]) & (xc < box[1]) & (yc > box[2]) & (yc < box[3])
    Q = avg[:, m]
    rho = Q[0]
    u, v = Q[1] / rho, Q[2] / rho
    p = 0.4 * (Q[3] - 0.5 * rho * (u * u + v * v))
    return [float(rho.mean()), float(u.mean()), float(v.mean()), float(p.mean())]


def shock_reflection(stream):
    """The shock-reflection problem of Sec. 4.3 (inflow left and top, wall below, outflow
    right) run to t = 6 without limiter, FP64 and FP32 bulk, averaged linearisation: wall time,
    steps, and the mean states upstream of the incident shock, between the shocks and between
    the reflected shock and the wall (boxes 0.1 away from the shocks)."""
    from paper_2508_06273_amd import af, inputs as I
    import torch
    boxes = {"upstream": (0.2, 0.9, 0.05, 0.3), "between_shocks": (1.8, 2.6, 0.75, 0.95),
             "reflected": (3.0, 3.9, 0.05, 0.3)}
    out = {}
    for nx, ny in ((120, 30), (240, 60)):
        print(f"[bench] shock reflection {nx}x{ny}", file=sys.stderr, flush=True)
        st = I.shock_reflection_state(nx, ny)
        rec = {}
        for prec, pname in ((af.AF_PREC_FP32, "fp32"), (af.AF_PREC_FP64, "fp64")):
            s = af.Solver.for_state(st, precision=prec, linearisation=af.AF_LIN_AVG)
            s.set_stream(stream)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            t, n = s.run(6.0, 0.3)
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            o = s.get_state()
            s.close()
            rec[pname] = {"seconds_to_t6": el, "steps": n, "ms_per_step": 1e3 * el / n,
                          "regions": {k: _region_mean(o["avg"], st.grid, b)
                                      for k, b in boxes.items()}}
        out[f"shock_reflection_{nx}x{ny}"] = rec
    return out


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(seconds: float, n_cpu: int):
    """The FP64 oracle on the host: as many OpenMP threads as the process may use (its CPU
    affinity), bounded by OMP_NUM_THREADS when the environment sets it (the host's share of
    cores for this GPU)."""
    import oracle
    from paper_2508_06273_amd import inputs as I
    avail = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    threads = avail
    if os.environ.get("OMP_NUM_THREADS", "").isdigit():
        threads = min(threads, int(os.environ["OMP_NUM_THREADS"]))
    threads = max(1, threads)
    st = I.shu_vortex(n_cpu, n_gl=3)
    oracle.run(st, 1e9, 0.3, max_steps=1, nthreads=threads)  # warm-up step
    steps = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        e, n, _ = oracle.run(st, 1e9, 0.3, max_steps=1, nthreads=threads)
        assert e == 0
        steps += 1
    el = time.perf_counter() - t0
    dofs = 4 * n_cpu * n_cpu
    return {"value": dofs * steps / el, "unit": "DOF-updates/s", "cores": threads,
            "kind": "oracle", "nproc": os.cpu_count(), "affinity_cpus": avail,
            "omp_num_threads_env": os.environ.get("OMP_NUM_THREADS"), "cpu_model": _cpu_model(),
            "sample": f"isentropic vortex {n_cpu}x{n_cpu} (same per-DOF work as the GPU "
                      f"workload), Algorithm 1, CFL 0.3, {steps} steps after 1 warm-up step, "
                      f"{el:.1f} s"}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--n", type=int, default=4096, help="cells per side")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--cpu-n", type=int, default=512)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the batched-grids leg (256 uneven grids)")
    ap.add_argument("--batched-steps", type=int, default=32,
                    help="timed steps of the batched leg (a multiple of 16: whole graphs)")
    ap.add_argument("--batched-only", action="store_true",
                    help="profiling aid: run only the batched leg, printed as JSON instead of "
                         "the benchmark line")
    ap.add_argument("--step-kernel", choices=("auto", "split", "persistent"), default="auto",
                    help="step kernel of the batched leg: chosen by the autotuner (auto), or "
                         "fixed on the default schedule")
    ap.add_argument("--prec", choices=("both", "fp32", "fp64"), default="both",
                    help="profiling aid: run one precision only (no JSON line)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="profiling aid: also run a plain device copy of MIB MiB (the "
                         "reference kernel for the HBM byte counters)")
    ap.add_argument("--record-traffic", nargs=2, metavar=("FETCH_DB", "WRITE_DB"),
                    help="profiling aid: write profiles/traffic.json from two rocprofv3 --pmc "
                         "result databases of a --calibrate-copy run, then exit")
    ap.add_argument("--ladder", action="store_true",
                    help="accuracy aid: vortex convergence ladder (256^2, 1024^2, 4096^2 to "
                         "t = 0.1), printed as JSON instead of the benchmark line")
    ap.add_argument("--pcie", action="store_true",
                    help="whole-job rate with the state copied in from and out to host memory "
                         "(1 and 40 steps of the vortex), printed as JSON instead of the "
                         "benchmark line")
    ap.add_argument("--extra", action="store_true",
                    help="throughput of the limiter workloads (2048^2 radial outflow, 8192^2 "
                         "shear layer), printed as JSON instead of the benchmark line")
    args = ap.parse_args()
    if args.record_traffic:
        record_traffic(args.record_traffic[0], args.record_traffic[1],
                       args.calibrate_copy or 1024, args.n)
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: this library runs the Active Flux step on one GPU only; "
              f"--gpus {args.gpus} (WORLD_SIZE={world}) is not supported.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2508_06273_amd import af, inputs as I
    af.load()
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()

    if args.calibrate_copy:
        nb = args.calibrate_copy << 20
        src = torch.ones(nb // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.add(src, 1.0, out=dst)  # one elementwise kernel: reads nb bytes, writes nb
        torch.cuda.synchronize()
        print(f"[bench] copy calibration: 3 elementwise copies of {nb} bytes", file=sys.stderr,
              flush=True)
        del src, dst

    if args.extra:
        print(json.dumps(extra_workloads(stream)), flush=True)
        return
    if args.pcie:
        print(json.dumps(pcie_inclusive(args.n, stream)), flush=True)
        return
    if args.ladder:
        print(json.dumps(accuracy_ladder([256, 1024, 4096], 0.1, stream)), flush=True)
        return
    step_kernel = {"auto": None, "split": af.AF_STEP_SPLIT,
                   "persistent": af.AF_STEP_PERSISTENT}[args.step_kernel]
    if args.batched_only:
        out = {}
        for prec, name in ((af.AF_PREC_FP32, "fp32"), (af.AF_PREC_FP64, "fp64")):
            print(f"[bench] batched workload, {name}", file=sys.stderr, flush=True)
            r = run_batched(prec, args.batched_steps, 32, stream, step_kernel=step_kernel)
            out[name] = {k: r[k] for k in ("value", "ms_per_step", "ms_points", "ms_update",
                                           "schedule")}
        print(json.dumps({"batched": out, "steps": args.batched_steps}), flush=True)
        return

    n = args.n
    print(f"[bench] generating the {n}x{n} vortex", file=sys.stderr, flush=True)
    st = I.shu_vortex(n, n_gl=3)
    res = {}
    precs = [(af.AF_PREC_FP32, "fp32"), (af.AF_PREC_FP64, "fp64")]
    if args.prec != "both":
        precs = [p for p in precs if p[1] == args.prec]
    for prec, name in precs:
        print(f"[bench] {name}: {args.warmup} warm-up + {args.steps} timed steps",
              file=sys.stderr, flush=True)
        res[name] = run_gpu(st, prec, args.steps, args.warmup, stream)
    if args.prec != "both":
        for name, r in res.items():
            print(f"[bench] {name}: {r['ms_total'] / args.steps:.3f} ms/step, k_points "
                  f"{r['ms_points']:.3f} ms, k_update {r['ms_update']:.3f} ms", file=sys.stderr)
        return
    cells = n * n
    out = {}
    for name, r in res.items():
        r["value"] = r["dofs"] * args.steps / (r["ms_total"] * 1e-3)
        r["ms_per_step"] = r["ms_total"] / args.steps

    # accuracy: L1 per conserved variable against the exact (translated) vortex averages,
    # and between the two precisions after the same steps
    print("[bench] accuracy", file=sys.stderr, flush=True)
    grid = st.grid
    exact = I.cell_average(I.shu_vortex_field(res["fp64"]["t"]), grid, n_gl=3)
    acc = {}
    for name in ("fp32", "fp64"):
        l1, linf = I.norms(res[name]["state"]["avg"], exact, grid)
        acc[f"L1_vs_exact_{name}"] = [float(x) for x in l1]
    l1d, linfd = I.norms(res["fp32"]["state"]["avg"], res["fp64"]["state"]["avg"], grid)
    acc["L1_fp32_vs_fp64"] = [float(x) for x in l1d]
    acc["Linf_fp32_vs_fp64"] = [float(x) for x in linfd]
    acc["t"] = res["fp64"]["t"]
    acc["variables"] = "rho, rho u, rho v, E"

    def roofline(name, peak):
        r = res[name]
        fpc = flops_per_cell(0, name)
        achieved = fpc * cells / (r["ms_points"] * 1e-3) / 1e12
        rec = traffic_record("k_points", f"vortex{n}_{name}")
        traffic = None if rec is None else rec["bytes_per_launch"]
        return {"bound": "alu", "achieved": round(achieved, 3), "peak": peak,
                "unit": "TFLOP/s", "frac": round(achieved / peak, 4), "traffic": traffic,
                "kernel": "k_points", "kernel_ms": round(r["ms_points"], 4),
                "flops_per_cell": fpc,
                "frac_of_nonpacked_issue_peak": round(achieved / PEAK_NONPACKED, 4)}

    line = {
        "metric": METRIC,
        "value": res["fp32"]["value"],
        "unit": "DOF-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": res["fp32"]["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"isentropic vortex {n}x{n} periodic on [0,10]^2, "
                               "Algorithm 1 with correction, CFL 0.3",
                   "cells": cells, "dof_sites": res["fp32"]["dofs"],
                   "precision": "fp32-bulk (FP64 averages, fluxes, tests, dt)"},
        "fp64": {"value": res["fp64"]["value"], "ms_per_step": res["fp64"]["ms_per_step"],
                 "speedup_fp32_vs_fp64": res["fp32"]["value"] / res["fp64"]["value"]},
        "accuracy": acc,
        "roofline": roofline("fp32", PEAK_FP32),
        "roofline_fp64": roofline("fp64", PEAK_FP64),
        "kernel_ms": {name: {"k_points": r["ms_points"], "k_update": r["ms_update"]}
                      for name, r in res.items()},
        "source_sha": source_hash(),
    }
    if not args.no_batched:
        print("[bench] batched workload: 256 grids", file=sys.stderr, flush=True)
        bres = {name: run_batched(prec, args.batched_steps, 32, stream, step_kernel=step_kernel)
                for prec, name in ((af.AF_PREC_FP32, "fp32"), (af.AF_PREC_FP64, "fp64"))}
        line["batched"] = {
            "workload": "256 periodic grids N x N on [0,1]^2, N ~ U{64..512} (seeded), random "
                        "Fourier data, Algorithm 1 with correction, CFL 0.3, own dt per grid",
            "grids": bres["fp32"]["grids"], "cells": bres["fp32"]["cells"],
            "dof_sites": bres["fp32"]["dofs"], "steps": args.batched_steps,
            "fp32": {k: bres["fp32"][k] for k in ("value", "ms_per_step", "ms_points",
                                                   "ms_update", "schedule")},
            "fp64": {k: bres["fp64"][k] for k in ("value", "ms_per_step", "ms_points",
                                                   "ms_update", "schedule")},
            "speedup_fp32_vs_fp64": bres["fp32"]["value"] / bres["fp64"]["value"],
            "unit": "DOF-updates/s"}
    if not args.no_cpu_baseline:
        print("[bench] CPU oracle baseline", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(args.cpu_seconds, args.cpu_n)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
