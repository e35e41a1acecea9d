#!/usr/bin/env python3
"""Benchmark of the SME time step on one MI355X.

A step is one full SME time step (face fluxes, non-conservative fluctuations,
friction, CFL reduction) over every cell of the workload.  Default workload:
the 1024 x 1024 periodic structured grid at level 2 (7 FP64 fields, 16-Gaussian
bathymetry, 0.5 m hump), 200 steps.  Inputs are resident in HBM before the timed
region; the timed region is K steps queued as HIP-graph replays, bracketed by
device synchronisation, timed with HIP events on the library's stream.

Prints one JSON line with the throughput (cell-updates/s), the roofline of the
step kernel (algorithmic bytes per launch / average launch time against the
8 TB/s HBM peak) and the CPU oracle timed on a bounded sample of the same grid.
"""
import argparse
import glob
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# the headline metric: cell-updates/s of the structured step (with its HBM
# roofline fraction) and, in the same line, the closure's speedup over level 8
METRIC = "SME cell-updates/s (FP64, % HBM peak); closure vs level-8 speedup at equal L1 error"
FP64_PEAK_TFS = 78.6  # MI355X FP64 vector peak

# Algorithmic bytes per cell-update of the step kernel: read every field of
# Q^n and the bathymetry once, write every field of Q^{n+1} once.
def bytes_per_cell(kind, level):
    nf = level + 2 if kind == "1d" else 2 * level + 3
    b = nf * 8 * 2 + 8
    if kind == "tri":
        # + 3 int32 neighbour ids, 3 scaled normals n |e| (2 FP64 each), 1/|V|
        b += 3 * 4 + 3 * 2 * 8 + 8
    return b


def bytes_per_cell_o2(kind, level):
    """Second-order step.  Structured grids up to level 6, two launches that
    compute the limited slopes themselves: stage 1 (state and b in, Q1 out),
    stage 2 (Q1, b and Q^n in, the new state out).  1D grids and higher
    levels, four launches: two reconstructions (the state and b in, the
    slopes of the nf + 1 reconstruction variables per axis out), stage 1
    (state, b and slopes in, Q1 out) and stage 2 (Q1, b, slopes and Q^n in,
    the new state out)."""
    nf = level + 2 if kind == "1d" else 2 * level + 3
    if kind == "2d" and level <= 6:
        return 8 * ((nf + 1) + nf + (nf + 1) + 2 * nf)
    axes = 1 if kind == "1d" else 2
    slopes = axes * (nf + 1)
    recon = (nf + 1) + slopes
    stage1 = (nf + 1) + slopes + nf
    stage2 = (nf + 1) + slopes + 2 * nf
    return 8 * (2 * recon + stage1 + stage2)


def lift_bytes_per_cell(kind, level, nz):
    """3D lifting of a 1D or structured state: the state and b in, z, u, v,
    w, p at nz sigma levels out."""
    nf = level + 2 if kind == "1d" else 2 * level + 3
    return 8 * (nf + 1) + 8 * 5 * nz


WORKLOADS = {
    "struct_2d_1024_l2": dict(gen="struct_2d", args={}, kernel="k_step_2d", name="struct_2d_1024x1024_level2_periodic"),
    "tri_4m_l3": dict(gen="tri_2d", args={}, kernel="k_step_tri", name="tri_delaunay_4M_level3_walls"),
    # 1000 cells: sme_run keeps the state in one workgroup's LDS and takes up to 2048 steps per launch
    "dam_break_1d": dict(gen="dam_break_1d", args={}, kernel="k_run_1d_lds", name="dam_break_1d_1000_level1",
                         timing="HIP events around the K timed steps, / K (the steps run inside one multi-step "
                                "launch of up to 2048 steps)"),
    "struct_2d_4096_l2": dict(gen="struct_2d", args=dict(n=4096), kernel="k_step_2d",
                              name="struct_2d_4096x4096_level2_periodic"),
    # the closure's level-8 reference size: FP64-arithmetic heavy (roofline also against the FP64 peak)
    "struct_2d_2048_l8": dict(gen="struct_2d", args=dict(n=2048, level=8), kernel="k_step_2d",
                              name="struct_2d_2048x2048_level8_periodic"),
    "batch_512": dict(gen="batch", args={}, kernel="k_batch_step",
                      name="batch_512_grids_side64-512_levels1-4_walls"),
    "closure_2048": dict(gen="closure", args={}, kernel="k_closure_rates_mfma",
                         name="closure_level1_vs_level8_2048x2048_periodic"),
    # the non-hydrostatic VAM channel: a step is the predictor, the corrector's solve (assembly,
    # block cyclic reduction level by level, back substitution, pressure update), its Newton step on
    # the residual (on the stored factors) and the correction
    "vam_1d": dict(gen="vam", args=dict(n=1 << 20, L=1000.0), kernel="k_vam_cr_reduce",
                   name="vam_1d_channel_1048576_cells_bore_over_hump"),
    # the default grid with the friction step by backward Euler (cell-local solve)
    "struct_2d_1024_l2_implicit": dict(gen="struct_2d", args=dict(params=dict(implicit_friction=1)),
                                       kernel="k_step_2d",
                                       name="struct_2d_1024x1024_level2_periodic_implicit_friction"),
    # the default grid with the second-order scheme: a step is two launches
    "struct_2d_1024_l2_o2": dict(gen="struct_2d", args=dict(params=dict(order=2)), kernel="k_stage2_band",
                                 name="struct_2d_1024x1024_level2_periodic_second_order",
                                 timing="HIP events on the step stream around the K timed steps, / K (a launch "
                                        "here is one step: k_stage2_band stage 1 and stage 2)"),
    # 3D lifting of a level-2 1024^2 state to 32 sigma levels
    "lift_1024_l2": dict(gen="lift", args=dict(n=1024, level=2, nz=32), kernel="k_lift",
                         name="lift_3d_1024x1024_level2_32_sigma_levels"),
}


def vam_bytes_per_cell(nx):
    """Algorithmic bytes per cell of one VAM step (FP64 words x 8):
    - predictor: 5 fields + b in, 5 out;
    - assembly: 5 fields + b in, 52 block entries per pair of cells out;
    - first solve, per reduction level of n equations: A, B, C, d of every
      equation in, the factors E, F, g, B^-1 of the even ones (52 each) and
      the next level (52 per odd one) out; the top equation: B, d in, its
      factors and unknowns out;
    - residual at the pressure found: 5 fields + b + p in, d out (2 per cell);
    - second solve on the stored factors, per level: d in, B^-1 of the even
      equations and A, C of the odd ones in, g of the even ones and d of the
      next level out; the top: B^-1, d in, unknowns out;
    - back substitution of each solve, per level: E, F, g of the even
      equations and the unknowns of the level above in, the unknowns out;
    - pressure updates: x in, p out (p also in the second time);
    - correction: 5 fields, p, b in, 4 fields out.
    The last levels (a few dozen equations) are counted like the others,
    though they stay in LDS."""
    nb = (nx + 1) // 2
    sizes = [nb]
    while sizes[-1] > 1:
        sizes.append(sizes[-1] // 2)
    full, rhs, back = 20 + 52 + 4, 20 + 4, 0
    for n in sizes[:-1]:
        ne, nd = (n + 1) // 2, n // 2
        full += 52 * n + 52 * ne + 52 * nd
        rhs += 4 * n + 16 * ne + 32 * nd + 4 * ne + 4 * nd
        back += 36 * ne + 4 * nd + 4 * n
    predict = 11 * 8 * nx
    assemble = (6 + 26) * 8 * nx
    residual = (8 + 2) * 8 * nx
    scatter = (4 + 6) * 8 * nx
    correct = (8 + 4) * 8 * nx
    solves = 8 * (full + rhs + 2 * back)
    return (predict + assemble + residual + scatter + correct + solves) / nx


def warm_clocks(torch, chunk, seconds):
    """Run chunk() (GPU work; it starts again from the workload's initial
    state where the state evolves) until `seconds` have passed.  The GPU's
    clocks ramp up over the first tens of milliseconds of sustained load, so a
    short timed region that starts on an idle GPU measures the ramp: the
    1024^2 level-2 step takes 36-39 us per step after 20 warmup steps and
    31 us after a second of load.  Returns the seconds spent."""
    t0 = time.perf_counter()
    while True:
        chunk()
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        if el >= seconds:
            return el


# Library sources each workload's launches are built from, besides every
# header and k_misc.hip (slots, reductions), which all of them include or run.
# A change to any other source leaves its committed counter figures valid.
_STEP = ("sme_lib.cpp",)
WORKLOAD_SOURCES = {
    "struct_2d_1024_l2": ("k_step_2d.hip",) + _STEP,
    "struct_2d_4096_l2": ("k_step_2d.hip",) + _STEP,
    "struct_2d_2048_l8": ("k_step_2d.hip",) + _STEP,
    "struct_2d_1024_l2_implicit": ("k_step_2d.hip",) + _STEP,
    "tri_4m_l3": ("k_step_tri.hip", "sme_mesh.cpp") + _STEP,
    "dam_break_1d": ("k_step_1d.hip",) + _STEP,
    "batch_512": ("k_batch.hip", "sme_batch.cpp"),
    "closure_2048": ("k_closure.hip", "k_mlp.hip", "sme_closure.cpp", "k_step_2d.hip", "k_step_1d.hip") + _STEP,
    "vam_1d": ("k_vam.hip", "sme_vam.cpp"),
    "struct_2d_1024_l2_o2": ("k_step2.hip",) + _STEP,
    "lift_1024_l2": ("k_lift.hip", "k_step_2d.hip") + _STEP,
}


def source_hash(workload=None):
    """Hash of the library sources a workload runs (every source for None or
    an unknown workload)."""
    csrc = os.path.join(ROOT, "paper_2601_04826_amd", "csrc")
    files = sorted(glob.glob(os.path.join(csrc, "*")))
    own = WORKLOAD_SOURCES.get(workload)
    if own is not None:
        files = [f for f in files
                 if f.endswith(".h") or os.path.basename(f) in own or os.path.basename(f) == "k_misc.hip"]
    h = hashlib.sha256()
    for f in files:
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(workload, launches_bytes):
    """HBM traffic per launch from committed rocprofv3 counter runs, if they
    were taken on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("source_hash") != source_hash(workload):
        return None
    return d.get("bytes_per_launch")


def load_flops(workload):
    """Executed FP64 flops per launch of the workload's kernel, from committed
    rocprofv3 counter runs (SQ_INSTS_VALU_FLOPS_FP64) taken on the current
    kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", f"flops_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("source_hash") != source_hash(workload):
        return None
    return d.get("fp64_flops_per_launch")


def copy_rate(torch, stream, nbytes, reps=20):
    """GB/s of a plain device copy moving nbytes in total (half read, half
    written), timed with HIP events on the same stream: the bandwidth that a
    kernel streaming the same bytes can practically reach at this size (the
    256 MB last-level cache holds part of a small working set)."""
    n = max(1, nbytes // 16)
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    with torch.cuda.stream(stream):
        for _ in range(3):
            dst.copy_(src)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            dst.copy_(src)
        e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    return 2 * n * 8 / (ms * 1e-3) / 1e9


def cpu_baseline(problem, seconds=15.0):
    """The oracle, as is, on a bounded number of steps of the same grid."""
    from oracle import sme as orc

    o = orc.from_problem(problem)
    q = problem["q"]
    steps = 0
    t0 = time.perf_counter()
    while True:
        q, _ = o.step(q)
        steps += 1
        el = time.perf_counter() - t0
        if el >= seconds or steps >= problem["steps"]:
            break
    return dict(value=problem["ncells"] * steps / el, unit="cell-updates/s", cores=orc.max_threads(),
                kind="oracle", sample=f"first {steps} steps of the same {problem['ncells']}-cell grid "
                f"({el:.1f} s, OpenMP threads={orc.max_threads()})")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--warmup-seconds", type=float, default=1.0,
                    help="load the GPU for this long before the warmup steps (its clocks ramp up under load)")
    ap.add_argument("--workload", default="struct_2d_1024_l2", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-tune", action="store_true", help="batch: skip the tile autotuner")
    ap.add_argument("--closure-seeds", type=int, default=64, help="closure: level-8 training runs")
    ap.add_argument("--closure-steps", type=int, default=1000, help="closure: steps per training run")
    ap.add_argument("--closure-epochs", type=int, default=15)
    ap.add_argument("--closure-ref-steps", type=int, default=200, help="closure: level-8 steps fixing the end time")
    ap.add_argument("--no-closure", action="store_true", help="default workload: skip the closure comparison")
    ap.add_argument("--closure-precision", default="fp16", choices=["fp16", "fp32"],
                    help="closure: network evaluation whose throughput is the headline value")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (read + write), 5 times: "
                         "calibrates the HBM byte counters against a kernel of known traffic")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU decomposition "
              "is designed but not implemented", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2601_04826_amd import sme, workloads

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    if args.copy_probe:
        n = args.copy_probe * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": n * 8, "copy_probe_bytes_written": n * 8, "launches": 5}))
        return
    wl = WORKLOADS[args.workload]
    if wl["gen"] == "batch":
        return bench_batch(args, wl, torch, sme, workloads)
    if wl["gen"] == "closure":
        return bench_closure(args, wl, torch, sme, workloads)
    if wl["gen"] == "vam":
        return bench_vam(args, wl, torch, sme, workloads)
    if wl["gen"] == "lift":
        return bench_lift(args, wl, torch, sme, workloads)
    t0 = time.perf_counter()
    problem = getattr(workloads, wl["gen"])(**wl["args"])
    print(f"[bench] workload {wl['name']}: {problem['ncells']} cells, level {problem['level']} "
          f"(generated in {time.perf_counter() - t0:.1f} s)", file=sys.stderr, flush=True)

    stream = torch.cuda.Stream()
    solver = sme.Solver(problem, stream=stream.cuda_stream)
    q0 = torch.from_numpy(problem["q"]).cuda()  # initial state from device memory
    torch.cuda.synchronize()
    def chunk():
        solver.set_state(q0)
        solver.run(200, sync=True)

    warm_s = warm_clocks(torch, chunk, args.warmup_seconds)
    solver.set_state(q0)
    torch.cuda.synchronize()
    solver.run(args.warmup, sync=True)
    torch.cuda.synchronize()

    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    ev0.record(stream)
    solver.run(args.steps, sync=False)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    ms = ev0.elapsed_time(ev1)
    # average duration of one step-kernel launch: HIP events recorded on the
    # library's stream right before and after single-step launches
    launches = max(10, min(args.steps, 50))
    pairs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(launches)]
    for e0, e1 in pairs:
        e0.record(stream)
        solver.step(0.0)
        e1.record(stream)
    torch.cuda.synchronize()
    per_launch_ms = sorted(e0.elapsed_time(e1) for e0, e1 in pairs)[launches // 2]
    t_sim, nsteps = solver.time()
    solver.close()
    print(f"[bench] {args.steps} steps in {ms:.3f} ms (events), {wall * 1e3:.3f} ms wall; "
          f"simulated t = {t_sim:.6g} s over {nsteps} steps", file=sys.stderr, flush=True)
    order = problem["params"].get("order", 1)
    bpc = (bytes_per_cell_o2 if order == 2 else bytes_per_cell)(problem["kind"], problem["level"])
    copy_gbs = copy_rate(torch, stream, bpc * problem["ncells"])

    ncells = problem["ncells"]
    value = ncells * args.steps / (ms * 1e-3)
    per_launch_s = ms * 1e-3 / args.steps  # one step (one kernel, or the four of the second order) per step
    alg_bytes = bpc * ncells
    achieved = alg_bytes / per_launch_s / 1e9
    traffic = load_traffic(args.workload, alg_bytes)
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "warmup_seconds": round(warm_s, 3),
        "ms_per_step": ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": wl["name"], "cells": ncells, "level": problem["level"],
                   "fields": problem["q"].shape[0], "cfl": problem["params"]["cfl"], "order": order,
                   "implicit_friction": int(problem["params"].get("implicit_friction", 0))},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": wl["kernel"], "alg_bytes_per_launch": alg_bytes,
                     "avg_launch_us": per_launch_s * 1e6,
                     "launch_timing": wl.get("timing", "HIP events on the step stream around the K timed steps, / K"),
                     "single_launch_us": per_launch_ms * 1e3,
                     "copy_gbs_same_bytes": copy_gbs, "frac_of_copy": achieved / copy_gbs},
        "cpu_baseline": None,
    }
    flops = load_flops(args.workload)
    if flops:
        tf = flops / per_launch_s / 1e12
        out["roofline"]["fp64"] = {"achieved": tf, "peak": FP64_PEAK_TFS, "unit": "TFLOP/s",
                                   "frac": tf / FP64_PEAK_TFS, "flops_per_launch": flops,
                                   "source": "executed FP64 flops per launch from rocprofv3 counters"}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(problem, args.cpu_seconds)
    if args.workload == "struct_2d_1024_l2" and not args.no_closure:
        # the second half of the headline metric: level 1 + closure against
        # level 8 at the same simulated time (2048^2 periodic grid)
        cmp_, mlp = closure_comparison(args, torch, sme, workloads,
                                       lambda m: print(m, file=sys.stderr, flush=True))
        mlp.close()
        out["closure"] = cmp_
    print(json.dumps(out), flush=True)


def _project_level(q8, p8, lev):
    """(h, moments 0..lev of each direction) of a level-8 2D state."""
    n8 = p8["level"] + 1
    return np.ascontiguousarray(np.concatenate([q8[:1], q8[1:2 + lev], q8[1 + n8:2 + n8 + lev]]))


def _state_hhu(torch, solver):
    """Fields 0 and 1 (h and h u, at the same place at every level) of the
    current state, kept in device memory."""
    full = torch.empty((solver.nf, solver.ncells), dtype=torch.float64, device="cuda")
    solver.get_state(full)
    torch.cuda.synchronize()
    return full[:2].clone()


def _rel_l1(q, ref):
    """E_x = sum_i |x_i - x_i^ref| / sum_i |x_i^ref| for x = h, h u (equal cells), on the device."""
    return [float((q[f] - ref[f]).abs().sum() / ref[f].abs().sum()) for f in (0, 1)]


def closure_comparison(args, torch, sme, workloads, log):
    """Learned closure against the plain hierarchy on a 2048^2 periodic 2D grid.

    Trains the network on level-8 1D runs the solver generates (library
    kernels: sample extraction, sme_closure_train), runs plain level 8 for
    args.closure_ref_steps steps to fix the end time T, then level 1 + closure
    through the fallback policy (ClosureSolver: chunks with device
    checkpoints, level 8 from the lifted state if the features leave the
    training box), plain level 1, and plain levels 2, 3, ... until one reaches
    the closure's error.  Returns a dict of wall times (synchronised, same T),
    speedups and relative L1 errors of (h, hu) against level 8."""
    from paper_2601_04826_amd import closure

    st = torch.cuda.Stream()
    t0 = time.perf_counter()
    # trained at the evaluation grid spacing (2048 cells on [0, 10] m): the
    # features hold neighbour differences, which scale with the spacing
    feat, targ = closure.generate(range(1000, 1000 + args.closure_seeds), n=2048, steps=args.closure_steps,
                                  every=5, cells_per_snapshot=256, stream=st)
    t1 = time.perf_counter()
    mlp, sc, hist = closure.fit(feat, targ, epochs=args.closure_epochs, batch=4096, lr=3e-3, lr_end=1e-4,
                                stream=st)
    t2 = time.perf_counter()
    log(f"[bench] closure data: {feat.shape[0]} samples from {args.closure_seeds} level-8 runs in {t1 - t0:.1f} s; "
        f"training {args.closure_epochs} epochs in {t2 - t1:.1f} s (loss {hist[0]:.4f} -> {hist[-1]:.4f})")
    p8 = workloads.smooth_2d(n=2048, level=8, seed=2000)
    cells = p8["ncells"]

    def wall(fn):
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - w0) * 1e3

    # level 8 reference: a fixed number of steps fixes the end time T
    s8 = sme.Solver(p8, stream=st.cuda_stream)
    q8_init = torch.from_numpy(p8["q"]).cuda()  # initial states from device memory
    torch.cuda.synchronize()
    s8.set_state(q8_init)
    s8.run(3)
    s8.set_state(q8_init)
    ms8 = wall(lambda: s8.run(args.closure_ref_steps))
    T, n8 = s8.time()
    ref = _state_hhu(torch, s8)
    s8.close()
    del q8_init
    q8_dev = torch.from_numpy(p8["q"]).cuda()
    torch.cuda.synchronize()
    res = {}
    # level 1 + closure through the fallback policy (the projection of the
    # level-8 initial state is taken on the device)
    cs = closure.ClosureSolver(p8, mlp, chunk=50, stream=st.cuda_stream, precision=args.closure_precision)
    cs.set_state(q8_dev)
    cs.run_to(T / 50, lifted=False)  # warm-up (graphs, kernels)
    cs.set_state(q8_dev)
    ms = wall(lambda: cs.run_to(T, lifted=False))
    q1 = _state_hhu(torch, cs.final_solver())
    err = _rel_l1(q1, ref)
    res["closure"] = dict(ms=ms, steps=cs.steps, t=cs.t, err_h=err[0], err_hu=err[1],
                          fell_back_at=cs.fell_back_at, out_of_range_cell_steps=cs.s1.out_of_range(),
                          precision=args.closure_precision)
    cs.close()

    def plain(lev):
        pN = dict(p8, level=lev, q=None)
        qN = torch.from_numpy(_project_level(p8["q"], p8, lev)).cuda()
        sN = sme.Solver(pN, stream=st.cuda_stream)
        sN.set_state(qN)
        sN.run(3)
        sN.set_state(qN)
        msN = wall(lambda: sN.run(100 * args.closure_ref_steps, t_end=T))
        tN, nN = sN.time()
        e = _rel_l1(_state_hhu(torch, sN), ref)
        sN.close()
        return dict(level=lev, ms=msN, steps=nN, t=tN, err_h=e[0], err_hu=e[1])

    res["plain_level1"] = plain(1)
    c, pl = res["closure"], res["plain_level1"]
    ce = c["err_h"] + c["err_hu"]
    equal = None
    for lev in range(2, 8):
        r = plain(lev)
        log(f"[bench] plain level {lev}: {r['ms']:.1f} ms, err_h {r['err_h']:.3e}, err_hu {r['err_hu']:.3e}")
        if r["err_h"] + r["err_hu"] <= ce:
            equal = dict(r, speedup_closure_over_it=r["ms"] / c["ms"])
            break
    out = {
        "grid": "2048x2048 periodic smooth 2D, level-8 reference", "t_end": T, "cells": cells,
        "training": f"{args.closure_seeds} level-8 1D runs x {args.closure_steps} steps, {feat.shape[0]} samples, "
                    f"{args.closure_epochs} epochs",
        "level8": dict(ms=ms8, steps=n8, cell_updates_per_s=cells * n8 / (ms8 * 1e-3)),
        "closure": c, "plain_level1": pl,
        "speedup_vs_level8": ms8 / c["ms"],
        "error_ratio_over_plain_level1": ce / (pl["err_h"] + pl["err_hu"]),
        "within_error_budget": ce <= 2.0 * (pl["err_h"] + pl["err_hu"]),
        "smallest_plain_level_at_closure_error": equal,
        "timing": "wall clock between device synchronisations, same simulated end time",
    }
    return out, mlp


def bench_closure(args, wl, torch, sme, workloads):
    """The closure workload: the comparison above, with the closure's
    throughput as the headline value."""
    cmp_, mlp = closure_comparison(args, torch, sme, workloads,
                                   lambda m: print(m, file=sys.stderr, flush=True))
    c = cmp_["closure"]
    cells = cmp_["cells"]
    value = cells * c["steps"] / (c["ms"] * 1e-3)
    # network work per cell and step: two directions x (9x64 + 64x64 + 64x2) multiply-adds
    flops = 2 * 2 * (9 * 64 + 64 * 64 + 64 * 2) * cells * c["steps"]
    fp16 = args.closure_precision == "fp16"
    peak = 2500.0 if fp16 else 157.3
    achieved = flops / (c["ms"] * 1e-3) / 1e12
    out = {
        "metric": "SME cell-updates/s, level 1 + learned closure (FP64 state, " +
                  ("FP16-operand matrix-core" if fp16 else "FP32") + " network)", "value": value,
        "unit": "cell-updates/s", "n_gpus": 1, "steps": c["steps"], "warmup": 3,
        "ms_per_step": c["ms"] / c["steps"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64+f16mfma" if fp16 else "f64+f32", "data": "synthetic",
        "config": {"workload": wl["name"], "cells": cells, "t_end": cmp_["t_end"]},
        "roofline": {"bound": "mfma" if fp16 else "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak, "traffic": None,
                     "kernel": "k_closure_rates_mfma + k_step_2d<1,closure>" if fp16 else
                               "k_closure_rates_valu + k_step_2d<1,closure>",
                     "alg_bytes_per_launch": bytes_per_cell("2d", 1) * cells,
                     "avg_launch_us": c["ms"] * 1e3 / max(1, c["steps"]),
                     "note": "network flops over the whole level-1 + closure step time"},
        "closure": cmp_,
        "cpu_baseline": None,
    }
    mlp.close()
    print(json.dumps(out), flush=True)


def bench_batch(args, wl, torch, sme, workloads):
    """The ensemble: every grid advances one step per launch (its own CFL step)."""
    t0 = time.perf_counter()
    probs = workloads.batch()
    cells = sum(p["ncells"] for p in probs)
    print(f"[bench] workload {wl['name']}: {len(probs)} grids, {cells} cells "
          f"(generated in {time.perf_counter() - t0:.1f} s)", file=sys.stderr, flush=True)
    stream = torch.cuda.Stream()
    bt = sme.Batch(probs, stream=stream.cuda_stream)
    cache = os.environ.get("SME_TUNE_CACHE")
    if not args.no_tune:
        bt.autotune(cache)
    print("[bench] band rows per level: " + ", ".join(f"L{l}={bt.rows(l)}" for l in range(5)), file=sys.stderr,
          flush=True)
    for i, p in enumerate(probs):
        bt.set_state(i, p["q"])
    torch.cuda.synchronize()
    # at most a few hundred extra steps of the ensemble (about 2 ms each)
    warm_s = warm_clocks(torch, lambda: bt.run(6), args.warmup_seconds)
    bt.run(args.warmup)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    bt.run(args.steps)  # synchronises at the end (error check), after ev1 is queued below
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    bt.close()
    value = cells * args.steps / (ms * 1e-3)
    alg = sum(bytes_per_cell(p["kind"], p["level"]) * p["ncells"] for p in probs)
    per_launch_s = ms * 1e-3 / args.steps
    out = {
        "metric": "SME cell-updates/s (FP64)", "value": value, "unit": "cell-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "warmup_seconds": round(warm_s, 3), "ms_per_step": ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": wl["name"], "grids": len(probs), "cells": cells,
                   "levels": sorted({p["level"] for p in probs})},
        "roofline": {"bound": "hbm", "achieved": alg / per_launch_s / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": alg / per_launch_s / 1e9 / HBM_PEAK_GBS, "traffic": load_traffic(args.workload, alg),
                     "kernel": wl["kernel"], "alg_bytes_per_launch": alg, "avg_launch_us": per_launch_s * 1e6,
                     "launch_timing": "HIP events on the step stream around the K timed steps, / K"},
        "cpu_baseline": None,
    }
    if not args.no_cpu_baseline:
        # the oracle on a bounded sample: whole grids of the ensemble, first step each
        from oracle import sme as orc

        done, t0 = 0, time.perf_counter()
        for p in probs:
            orc.from_problem(p).step(p["q"])
            done += p["ncells"]
            if time.perf_counter() - t0 > args.cpu_seconds:
                break
        el = time.perf_counter() - t0
        out["cpu_baseline"] = dict(value=done / el, unit="cell-updates/s", cores=orc.max_threads(), kind="oracle",
                                   sample=f"one step of the first {done} cells of the ensemble ({el:.1f} s)")
    print(json.dumps(out), flush=True)


def bench_lift(args, wl, torch, sme, workloads):
    """3D lifting (interpolate_3d) of a structured level-N state to nz sigma
    levels: K launches, each writing z, u, v, w, p of every cell and level."""
    a = wl["args"]
    p = workloads.struct_2d(n=a["n"], level=a["level"])
    nz, ncells = a["nz"], p["ncells"]
    zeta = np.linspace(0.0, 1.0, nz)
    print(f"[bench] workload {wl['name']}: {ncells} cells, {nz} sigma levels", file=sys.stderr, flush=True)
    stream = torch.cuda.Stream()
    s = sme.Solver(p, stream=stream.cuda_stream)
    s.set_state(torch.from_numpy(p["q"]).cuda())
    s.run(20)  # a state with flow: every moment and gradient generic
    out = torch.empty((5, nz, ncells), dtype=torch.float64, device="cuda")
    def chunk():
        for _ in range(10):
            s.interpolate_3d_into(zeta, out)

    warm_s = warm_clocks(torch, chunk, args.warmup_seconds)
    for _ in range(args.warmup):
        s.interpolate_3d_into(zeta, out)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(args.steps):
        s.interpolate_3d_into(zeta, out)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    Q = s.get_state()
    s.close()
    per_launch_s = ms * 1e-3 / args.steps
    alg = lift_bytes_per_cell("2d", p["level"], nz) * ncells
    copy_gbs = copy_rate(torch, stream, alg)
    out_ = {
        "metric": "lifted cells/s (FP64, z u v w p at every sigma level)", "value": ncells * args.steps / (ms * 1e-3),
        "unit": "cells/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "warmup_seconds": round(warm_s, 3),
        "ms_per_step": ms / args.steps, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": wl["name"], "cells": ncells, "level": p["level"], "sigma_levels": nz},
        "roofline": {"bound": "hbm", "achieved": alg / per_launch_s / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": alg / per_launch_s / 1e9 / HBM_PEAK_GBS, "traffic": load_traffic(args.workload, alg),
                     "kernel": wl["kernel"], "alg_bytes_per_launch": alg, "avg_launch_us": per_launch_s * 1e6,
                     "launch_timing": "HIP events on the solver's stream around the K timed launches, / K",
                     "copy_gbs_same_bytes": copy_gbs, "frac_of_copy": alg / per_launch_s / 1e9 / copy_gbs},
        "cpu_baseline": None,
    }
    if not args.no_cpu_baseline:
        from oracle import lift as olift
        from oracle import sme as orc

        m = orc.mesh_of(p)
        done, t0 = 0, time.perf_counter()
        while done < ncells:
            cells = np.arange(done, min(ncells, done + 65536))
            olift.interpolate_3d(p["level"], m, Q, p["b"], zeta, g=p["params"]["g"], spacing=olift.spacing_of(p),
                                 cells=cells)
            done += cells.size
            if time.perf_counter() - t0 >= args.cpu_seconds:
                break
        el = time.perf_counter() - t0
        out_["cpu_baseline"] = dict(value=done / el, unit="cells/s", cores=1, kind="oracle",
                                    sample=f"the first {done} cells of the same state ({el:.1f} s, numpy)")
    print(json.dumps(out_), flush=True)


def bench_vam(args, wl, torch, sme, workloads):
    """The non-hydrostatic VAM channel: K predictor-corrector steps."""
    p = workloads.vam_1d(**wl["args"])
    nx = p["nx"]
    print(f"[bench] workload {wl['name']}: {nx} cells", file=sys.stderr, flush=True)
    stream = torch.cuda.Stream()
    v = sme.Vam(p, stream=stream.cuda_stream)
    q0 = torch.from_numpy(p["q"]).cuda()
    torch.cuda.synchronize()

    def chunk():
        v.set_state(q0)
        v.run(20)

    warm_s = warm_clocks(torch, chunk, args.warmup_seconds)
    v.set_state(q0)
    v.run(args.warmup)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    t_sim, n_done = v.run(args.steps)  # synchronises at the end (error check), after ev1 is queued below
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    v.close()
    per_step_s = ms * 1e-3 / args.steps
    alg = int(round(vam_bytes_per_cell(nx) * nx))
    copy_gbs = copy_rate(torch, stream, min(alg, 4 << 30))
    out = {
        "metric": "VAM cell-updates/s (FP64, predictor + corrector)", "value": nx * args.steps / (ms * 1e-3),
        "unit": "cell-updates/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "warmup_seconds": round(warm_s, 3), "ms_per_step": ms / args.steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": wl["name"], "cells": nx, "levels_of_reduction": max(0, ((nx + 1) // 2 - 1).bit_length())},
        "roofline": {"bound": "hbm", "achieved": alg / per_step_s / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": alg / per_step_s / 1e9 / HBM_PEAK_GBS, "traffic": load_traffic(args.workload, alg),
                     "kernel": "one VAM step (k_vam_predict; k_vam_assemble, k_vam_cr_reduce per level, k_vam_cr_tail, "
                               "k_vam_cr_back per level, k_vam_scatter; k_vam_residual, k_vam_cr_rhs per level, "
                               "k_vam_cr_tail, k_vam_cr_back per level, k_vam_scatter; k_vam_correct)",
                     "alg_bytes_per_launch": alg, "avg_launch_us": per_step_s * 1e6,
                     "launch_timing": "HIP events on the step stream around the K timed steps, / K (a launch here "
                                      "is one step's kernel sequence)",
                     "copy_gbs_same_bytes": copy_gbs, "frac_of_copy": alg / per_step_s / 1e9 / copy_gbs},
        "cpu_baseline": None,
    }
    if not args.no_cpu_baseline:
        from oracle import vam as ovam

        o = ovam.Vam1D(nx, p["x0"], p["x1"], b=p["b"], g=p["params"]["g"], cfl=p["params"]["cfl"],
                       quad_points=p["params"]["quad_points"])
        q = p["q"]
        steps, t0 = 0, time.perf_counter()
        while True:
            q, _, _ = o.step(q)
            steps += 1
            el = time.perf_counter() - t0
            if el >= args.cpu_seconds or steps >= args.steps:
                break
        out["cpu_baseline"] = dict(value=nx * steps / el, unit="cell-updates/s", cores=1, kind="oracle",
                                   sample=f"first {steps} steps of the same {nx}-cell channel ({el:.1f} s, numpy "
                                          "and a sparse direct solve, one thread)")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
