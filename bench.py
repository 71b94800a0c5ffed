#!/usr/bin/env python3
"""Benchmark of the Voronoi hot path on one MI355X.

The workload is the clustered 2,097,152-particle periodic box (side 100, FP32 positions, half
uniform background and half in 200 NFW-like halos).  `value` is the metric's own rate,
neighbours + volume + density: one step is the Morton sort and the clipping (vt_build, facets
kept), the neighbour CSR and volumes (vt_cells) and the densities (vt_density), timed over K steps
with the inputs resident in HBM.  The whole per-particle path (adding density gradients, the exact
256^3 grid deposit and the volume adjoint) is timed separately (`whole_step`), with per-stage HIP
event times.

Also printed on the same JSON line: the roofline of the dominant kernel (the clipping kernel;
VALU-bound, algorithmic flops from the cost model 6 P V + 60 V per cell, P = particles inside the
security radius, V = final vertices) with counter figures from the committed rocprofv3 summary,
the backward rate of the 262k differentiation workload, the forward rates of the 4096 and 16.7M
workloads, the precision variants, the batched and decomposed forms, and the brute-force FP64
oracle timed on a bounded sample of the same workload on the host cores.
"""
import argparse
import ctypes
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Voronoi cells/sec (neighbours+volume+density) at 2M clustered pts; bwd cells/s"
# vector peaks from unit counts: 256 CU x 4 SIMD x 16 lanes x 2 flop (FMA) x 2.4 GHz = 78.6 TFLOP/s in FP64;
# FP32 counts two packed operations per lane (157.3 TFLOP/s)
PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="clustered2m", choices=["clustered2m", "uniform4096", "lattice16m",
                                                                  "diff262k"])
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=8192)
    ap.add_argument("--no-variants", action="store_true", help="skip the mixed/fp64 forward comparison")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched 64-item form")
    ap.add_argument("--no-decomposed", action="store_true", help="skip the AUTOBORDER decomposed form")
    ap.add_argument("--no-tune", action="store_true", help="library default launch options instead of the autotuner's")
    ap.add_argument("--fwd-only", action="store_true", help="time only vt_build + vt_cells + vt_density")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the backward (262k) and other-workload (4096, 16.7M) forms")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 256 MiB device copy (traffic calibration for rocprofv3 counters)")
    return ap.parse_args()


COPY_BYTES = 256 << 20
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_clip_clustered2m_traffic.md")
CLIP_SOURCES = ["paper_1601_06429_amd/csrc/clip.hip", "paper_1601_06429_amd/csrc/poly.h",
                "paper_1601_06429_amd/csrc/vt_internal.h"]


def copy_calibration():
    """A plain device copy of COPY_BYTES, five times: rocprofv3 FETCH_SIZE / WRITE_SIZE read
    on it give the factor between the counters and true HBM bytes."""
    import torch

    x = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(5):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": COPY_BYTES, "launches": 5}))


def clip_sources_sha1():
    import hashlib

    h = hashlib.sha1()
    for f in CLIP_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per launch of the fast clip kernel, from the committed counter summary;
    None when the kernel sources changed since the counters were taken."""
    try:
        with open(TRAFFIC_FILE) as fh:
            kv = dict(line.strip("- \n").split(": ", 1) for line in fh if line.startswith("- ") and ": " in line)
    except OSError:
        return None
    if kv.get("source_sha1") != clip_sources_sha1():
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


COUNTERS_FILE = os.path.join(ROOT, "profiles", "k_clip_k_grid_clustered2m_counters.md")
GRID_SOURCES = ["paper_1601_06429_amd/csrc/grid.hip", "paper_1601_06429_amd/csrc/rebuild.h",
                "paper_1601_06429_amd/csrc/poly.h", "paper_1601_06429_amd/csrc/vt_internal.h"]


def sources_sha1(files):
    import hashlib

    h = hashlib.sha1()
    for f in files:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def _summary(path):
    try:
        with open(path) as fh:
            return dict(line.strip("- \n").split(": ", 1) for line in fh if line.startswith("- ") and ": " in line)
    except OSError:
        return {}


def clip_counters():
    """Per-launch counter figures of the fast clip kernel from the committed rocprofv3 summary,
    while the kernel's sources are the ones they were taken from; else None."""
    kv = _summary(COUNTERS_FILE)
    if kv.get("clip_source_sha1") != sources_sha1(CLIP_SOURCES):
        return None
    try:
        return {"fp64_wave_flops": float(kv["clip_fp64_wave_flops"]), "valu_busy": float(kv["clip_valu_busy"]),
                "valu_lane_util": float(kv["clip_valu_lane_util"])}
    except (KeyError, ValueError):
        return None


SORT_FILE = os.path.join(ROOT, "profiles", "sort_clustered2m_traffic.md")
SORT_SOURCES = ["paper_1601_06429_amd/csrc/sort.hip", "paper_1601_06429_amd/csrc/vt_internal.h"]


def sort_traffic():
    """HBM bytes of one build's sort pass from the committed counter summary, while the sort's
    sources are the ones they were taken from; else None."""
    kv = _summary(SORT_FILE)
    if kv.get("sort_source_sha1") != sources_sha1(SORT_SOURCES):
        return None
    try:
        return float(kv["sort_hbm_bytes_per_build"])
    except (KeyError, ValueError):
        return None


def grid_counters():
    """The same for the grid deposit kernel: VALU issue and lane use against the VALU issue
    peak (one wavefront instruction per SIMD every 4 cycles)."""
    kv = _summary(COUNTERS_FILE)
    if kv.get("grid_source_sha1") != sources_sha1(GRID_SOURCES):
        return None
    try:
        busy = float(kv["grid_valu_busy"])
        return {"achieved": busy, "peak": 1.0, "unit": "fraction of VALU issue cycles", "frac": busy,
                "valu_lane_utilisation": float(kv["grid_valu_lane_util"]),
                "traffic": float(kv["grid_hbm_bytes_per_launch"]) if "grid_hbm_bytes_per_launch" in kv else None}
    except (KeyError, ValueError):
        return None


def batched_forms(torch, vt, reps=5):
    """64 uneven ghost-buffered sub-volumes in one build: eager vs HIP-graph replay, FP64 vs mixed."""
    from paper_1601_06429_amd import workloads as wl

    items = wl.batched64()
    worlds = [(it.owned, it.ghosts, it.buffered_lo, it.buffered_hi) for it in items]
    pos, desc, gid = vt.pack_worlds(worlds)
    t = torch.from_numpy(pos).cuda()
    g_id = torch.from_numpy(gid).cuda()
    n_owned = sum(d["n_owned"] for d in desc)
    res = {"workload": "batched-64-items-fp32", "items": len(desc), "n_owned": n_owned,
           "n_ghost": sum(d["n_ghost"] for d in desc), "step": "build+cells+density"}
    # launch options tuned on a representative subset (the first 8 items)
    sub_pos, sub_desc, sub_gid = vt.pack_worlds(worlds[:8])
    tuned = {}
    for name, p in (("fp64", vt.PREC_FP64), ("mixed", vt.PREC_MIXED)):
        tuned[name], _ = vt.autotune.tune(vt.Context, torch.from_numpy(sub_pos).cuda(), sub_desc,
                                          global_id=torch.from_numpy(sub_gid).cuda(), precision=p, reps=1)
    keep = {}
    for name, p in (("fp64", vt.PREC_FP64), ("mixed", vt.PREC_MIXED)):
        opts = tuned[name]
        ctx = vt.Context().vt_build(t, desc, global_id=g_id, precision=p, **opts)
        code, nnz, retried, inc = ctx.vt_query()
        vol = torch.empty(n_owned, dtype=torch.float64, device="cuda")
        off = torch.empty(n_owned + 1, dtype=torch.int64, device="cuda")
        ids = torch.empty(int(nnz * 1.05) + 4096, dtype=torch.int32, device="cuda")
        st = torch.empty(n_owned, dtype=torch.uint8, device="cuda")
        rho = torch.empty(n_owned, dtype=torch.float64, device="cuda")

        def step():
            ctx.vt_build(t, desc, global_id=g_id, precision=p, **opts)
            ctx.vt_cells_into(vol, off, ids, st)
            ctx.vt_density(None, out=rho)

        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            step()
            torch.cuda.synchronize()
            ta = time.perf_counter()
            for _ in range(reps):
                step()
            torch.cuda.synchronize()
            tb = time.perf_counter()
        torch.cuda.current_stream().wait_stream(side)
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            step()
        graph.replay()
        torch.cuda.synchronize()
        tc = time.perf_counter()
        for _ in range(reps):
            graph.replay()
        torch.cuda.synchronize()
        td = time.perf_counter()
        code = ctx.vt_query()[0]
        res[name] = {"eager_cells_per_s": n_owned * reps / (tb - ta), "graph_cells_per_s": n_owned * reps / (td - tc),
                     "graph_ms": (td - tc) * 1e3 / reps, "status": vt.STATUS_NAMES.get(code), "tuned": opts,
                     "retried": retried, "incomplete": inc}
        keep[name] = (vol.cpu().numpy(), off.cpu().numpy(), ids[: int(off[-1])].cpu().numpy())
        del graph, ctx
    v64, o64, i64 = keep["fp64"]
    vm, om, im = keep["mixed"]
    res["mixed_vs_fp64"] = {"max_rel_volume_diff": float(np.max(np.abs(vm - v64) / v64)),
                            "neighbours_identical": bool(np.array_equal(o64, om) and np.array_equal(i64, im))}
    return res


def decomposed_form(torch, vt, w, nt=(4, 4, 4), border_factor=1.5, reps=3, opts=None):
    """The workload as nt tasks with AUTOBORDER buffers (section 2), in the library
    (vt_decomposed_build): thicknesses, all tasks packed and built as one batch, incomplete cells
    built again with wider buffers, results stitched in particle order.  An untimed run checks the
    result against the whole-box cells; the timed runs repeat the whole call plus vt_cells."""
    pos = torch.from_numpy(w.pos).cuda()
    n = w.n
    opts = dict(opts or {})
    res = vt.decomposed_build(pos, w.box_lo, w.box_hi, nt, border_factor=border_factor, **opts)
    whole = vt.Context().vt_build(pos, vt.whole_box(n, w.box_lo, w.box_hi)).vt_cells()
    same_nbrs = bool(np.array_equal(res["nbr_off"], whole.nbr_off.cpu().numpy()) and
                     np.array_equal(res["nbr_ids"], whole.nbr_ids.cpu().numpy()))
    wv = whole.volume.cpu().numpy()
    max_rel = float(np.max(np.abs(res["volume"] - wv) / wv))
    del whole
    ctx = res["ctx"]
    nnz = int(res["nbr_off"][-1])
    vol = torch.empty(n, dtype=torch.float64, device="cuda")
    off = torch.empty(n + 1, dtype=torch.int64, device="cuda")
    ids = torch.empty(nnz, dtype=torch.int32, device="cuda")

    def run():
        ctx.vt_decomposed_build(pos, w.box_lo, w.box_hi, nt, border_factor=border_factor, **opts)
        ctx.vt_cells_into(vol, off, ids)

    run()
    torch.cuda.synchronize()
    ta = time.perf_counter()
    for _ in range(reps):
        run()
    torch.cuda.synchronize()
    tb = time.perf_counter()
    ms = (tb - ta) * 1e3 / reps
    s = float(np.cbrt(np.prod(w.box_len) / n))
    grow = res["thick"] / (border_factor * s)
    return {"workload": w.name, "tasks": list(nt), "border_factor": border_factor, "launch_options": opts or "defaults",
            "ms": ms,
            "cells_per_s": n / (ms * 1e-3),
            "step": "vt_decomposed_build (thicknesses, packing, builds of every pass, stitching) + vt_cells",
            "faces_widened": float(np.mean(grow > 1.0 + 1e-12)), "max_widening": float(grow.max()),
            "passes": res["passes"], "equals_whole_box": {"neighbours_identical": same_nbrs,
                                                          "max_rel_volume_diff": max_rel}}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def _target(torch, x, lam, phi, amp, mean):
    import math

    s = torch.ones(x.shape[0], dtype=x.dtype, device=x.device)
    for a in range(3):
        s = s * torch.sin(2.0 * math.pi * x[:, a] / float(lam[a]) + float(phi[a]))
    return mean * (1.0 + amp * s)


def backward_form(torch, vt, reps=10):
    """The differentiation workload: 262,144 clustered particles in the periodic unit cube, loss
    sum_i (log rho_i - log rho_t(x_i))^2 against a smooth sinusoidal target.  Timed: the backward
    pass of that loss, i.e. dL/dV (elementwise), the adjoint kernel vt_backward and the explicit
    target term, with the forward build (facets kept) done once before; cells/s = N / time."""
    from paper_1601_06429_amd import workloads as wl

    w = wl.diff262k()
    n = w.n
    lam, phi, amp = w.extra["target_lambda"], w.extra["target_phase"], w.extra["target_amplitude"]
    mean = float(w.mass.sum())
    x = torch.from_numpy(w.pos.astype(np.float64)).cuda()
    ctx = vt.Context().vt_build(x, vt.whole_box(n, 0.0, 1.0), want_faces=True)
    vol = ctx.vt_cells().volume
    xr = x.clone().requires_grad_(True)
    rt = _target(torch, xr, lam, phi, amp, mean)
    dx = torch.empty((n, 3), dtype=torch.float64, device="cuda")

    def bwd():
        r = torch.log(1.0 / vol) - torch.log(rt.detach())
        dldv = (-2.0 * r / vol).contiguous()
        ctx.vt_backward(dldv, out=dx)
        # the explicit dependence of rho_t on x_i
        gt, = torch.autograd.grad(rt, xr, grad_outputs=-2.0 * r / rt.detach(), retain_graph=True)
        dx.add_(gt)

    bwd()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        bwd()
    e1.record()
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    e0.record()
    for _ in range(reps):
        ctx.vt_backward(torch.ones(n, dtype=torch.float64, device="cuda"), out=dx)
    e1.record()
    e1.synchronize()
    ms_k = e0.elapsed_time(e1) / reps
    code = ctx.vt_query()[0]
    return {"workload": w.name, "n_cells": n, "ms": ms, "cells_per_s": n / (ms * 1e-3), "adjoint_kernel_ms": ms_k,
            "status": vt.STATUS_NAMES.get(code),
            "step": "dL/dV + vt_backward + target term (backward of the density-matching loss)"}


def other_configs(torch, vt, reps=5):
    """Forward rate (build + cells + density) of the other workloads: the 4096-particle FP64
    box (launch-bound at this size) and the 16.7M lattice+halos set in both precisions."""
    from paper_1601_06429_amd import workloads as wl

    res = {}
    for name, w, precs in (("uniform4096", wl.uniform4096(), (vt.PREC_FP64,)),
                           ("lattice16m", wl.lattice_halos16m(), (vt.PREC_FP64, vt.PREC_MIXED))):
        pos = torch.from_numpy(w.pos).cuda()
        items = vt.whole_box(w.n, w.box_lo, w.box_hi)
        for p in precs:
            ctx = vt.Context().vt_build(pos, items, precision=p)
            nnz = ctx.vt_query()[1]
            vol = torch.empty(w.n, dtype=torch.float64, device="cuda")
            off = torch.empty(w.n + 1, dtype=torch.int64, device="cuda")
            ids = torch.empty(int(nnz * 1.05) + 1024, dtype=torch.int32, device="cuda")
            rho = torch.empty(w.n, dtype=torch.float64, device="cuda")
            for _ in range(2):
                ctx.vt_build(pos, items, precision=p)
            torch.cuda.synchronize()
            ta = time.perf_counter()
            for _ in range(reps):
                ctx.vt_build(pos, items, precision=p)
                ctx.vt_cells_into(vol, off, ids)
                ctx.vt_density(None, out=rho)
            torch.cuda.synchronize()
            tb = time.perf_counter()
            code = ctx.vt_query()[0]
            res["%s_%s" % (name, "fp64" if p == vt.PREC_FP64 else "mixed")] = {
                "workload": w.name, "n_cells": w.n, "fwd_cells_per_s": w.n * reps / (tb - ta),
                "ms": (tb - ta) * 1e3 / reps, "status": vt.STATUS_NAMES.get(code)}
            del ctx, vol, off, ids, rho
        del pos
        torch.cuda.empty_cache()
    return res


def load_workload(name):
    from paper_1601_06429_amd import workloads as wl

    if name == "clustered2m":
        return wl.clustered2m()
    if name == "uniform4096":
        return wl.uniform4096()
    if name == "lattice16m":
        return wl.lattice_halos16m()
    return wl.diff262k()


def main():
    args = parse()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU: the library has no multi-GPU path; got --gpus %d" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_1601_06429_amd as vt

    vt.lib()
    dev = torch.device("cuda:0")
    w = load_workload(args.workload)
    grid_dims = w.grid or (128, 128, 128)
    prec = vt.PREC_MIXED if args.precision == "mixed" else vt.PREC_FP64
    pos = torch.from_numpy(w.pos).to(dev)
    mass = torch.from_numpy(w.mass).to(dev)
    items = vt.whole_box(w.n, w.box_lo, w.box_hi, True)
    N = w.n

    # launch options from the library's autotuner (untimed; results do not depend on them)
    tuned = {} if args.no_tune else vt.autotune.tune(vt.Context, pos, items, precision=prec, reps=1)[0]
    ctx = vt.Context()
    ctx.vt_build(pos, items, precision=prec, want_faces=True, timing=True, **tuned)
    code, nnz, retried, incomplete = ctx.vt_query()
    if code != 0:
        raise SystemExit("build failed: %s" % vt.STATUS_NAMES.get(code))
    vol = torch.empty(N, dtype=torch.float64, device=dev)
    off = torch.empty(N + 1, dtype=torch.int64, device=dev)
    ids = torch.empty(int(nnz * 1.05) + 1024, dtype=torch.int32, device=dev)
    st = torch.empty(N, dtype=torch.uint8, device=dev)
    rho = torch.empty(N, dtype=torch.float64, device=dev)
    grad = torch.empty((N, 3), dtype=torch.float64, device=dev)
    grid = torch.empty(grid_dims, dtype=torch.float64, device=dev)
    dx = torch.empty((N, 3), dtype=torch.float64, device=dev)
    # adjoint input: dL/dV of a density-matching loss against the mean density (fixed, outside the timed region)
    ctx.vt_cells_into(vol, off, ids, st)
    ctx.vt_density(mass, out=rho)
    torch.cuda.synchronize()
    rho_mean = float(mass.sum()) / float(np.prod(w.box_len))
    dLdV = (-2.0 * (torch.log(rho) - np.log(rho_mean)) / vol).contiguous()

    ev = [torch.cuda.Event(enable_timing=True) for _ in range(7)]
    stage_ms = np.zeros(6)
    build_ms = np.zeros(3)

    def step(record):
        if record:
            ev[0].record()
        ctx.vt_build(pos, items, precision=prec, want_faces=True, timing=record, **tuned)
        if record:
            ev[1].record()
        ctx.vt_cells_into(vol, off, ids, st)
        if record:
            ev[2].record()
        ctx.vt_density(mass, out=rho)
        if record:
            ev[3].record()
        if not args.fwd_only:
            ctx.vt_gradient(rho, out=grad)
            if record:
                ev[4].record()
            ctx.vt_grid_deposit(rho, grid_dims, out=grid)
            if record:
                ev[5].record()
            ctx.vt_backward(dLdV, out=dx)
            if record:
                ev[6].record()

    def fwd_step():
        ctx.vt_build(pos, items, precision=prec, want_faces=True, **tuned)
        ctx.vt_cells_into(vol, off, ids, st)
        ctx.vt_density(mass, out=rho)

    # the metric's own rate: neighbours + volume + density (build, CSR, densities), K timed steps
    for _ in range(args.warmup):
        fwd_step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        fwd_step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps

    # the whole per-particle path (adds gradients, the grid deposit and the adjoint), K timed steps
    whole_ms = None
    if not args.fwd_only:
        for _ in range(max(1, args.warmup // 2)):
            step(False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            step(False)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        whole_ms = (t1 - t0) * 1e3 / args.steps

    # stage breakdown (separate, event-recorded steps)
    nrec = 3
    for _ in range(nrec):
        step(True)
        torch.cuda.synchronize()
        n_ev = 4 if args.fwd_only else 7
        for k in range(n_ev - 1):
            stage_ms[k] += ev[k].elapsed_time(ev[k + 1]) / nrec
        bm = ctx.vt_timings()
        build_ms += np.asarray(bm) / nrec
    code, nnz, retried, incomplete = ctx.vt_query()
    if code != 0:
        raise SystemExit("timed run reported: %s" % vt.STATUS_NAMES.get(code))

    # cost model of the fast clipping kernel over the cells it computed (retried cells excluded)
    nv, npl, ntest = ctx.vt_stats()
    ctx.vt_cells_into(vol, off, ids, st)
    fast = (st & 2) == 0
    nv = nv.to(torch.float64)
    npl = npl.to(torch.float64)
    alg_flops = float(((6.0 * npl * nv + 60.0 * nv) * fast).sum())
    clip_ms = build_ms[1]
    achieved = alg_flops / (clip_ms * 1e-3) / 1e12
    dtype = "f64" if prec == vt.PREC_FP64 else "f32"
    counters = clip_counters() if prec == vt.PREC_FP64 else None
    bench_vol, bench_off = vol.cpu().numpy(), off.cpu().numpy()
    bench_ids, bench_rho = ids[: int(bench_off[-1])].cpu().numpy(), rho.cpu().numpy()
    bench_grad = None if args.fwd_only else grad.cpu().numpy()
    # the deposit conserves mass: the voxel averages times the voxel volume sum to the total mass
    grid_mass_err = None if args.fwd_only else float(
        abs(float(grid.sum()) * float(np.prod(w.box_len)) / float(np.prod(grid_dims)) - float(w.mass.sum())) /
        float(w.mass.sum()))

    out = {
        "metric": METRIC,
        "value": N / (ms_per_step * 1e-3),
        "unit": "cells/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic",
        "config": {"workload": w.name, "n_cells": N, "box": float(w.box_len[0]), "positions": str(w.pos.dtype),
                   "precision": args.precision,
                   "step": "build (sort + clip, facets kept) + neighbour CSR and volumes + densities",
                   "launch_options": tuned or "defaults"},
        "whole_step": None if whole_ms is None else {
            "ms": whole_ms, "cells_per_s": N / (whole_ms * 1e-3), "grid": list(grid_dims),
            "step": "build + cells + density + gradient + grid deposit + adjoint"},
        "stage_ms": {"build": stage_ms[0], "cells": stage_ms[1], "density": stage_ms[2],
                     "gradient": stage_ms[3], "grid": stage_ms[4], "backward": stage_ms[5],
                     "sort": build_ms[0], "clip": build_ms[1], "clip_large": build_ms[2]},
        "nnz": nnz,
        "retried_cells": retried,
        "grid_mass_rel_err": grid_mass_err,
        "roofline": {"kernel": "k_clip fast (cells up to 64 vertices)", "bound": "alu", "achieved": achieved,
                     "peak": PEAK_TFLOPS[dtype], "unit": "TFLOP/s", "frac": achieved / PEAK_TFLOPS[dtype],
                     "traffic": measured_traffic() if prec == vt.PREC_FP64 else None,
                     "alg_flops_per_launch": alg_flops, "launch_ms": clip_ms,
                     "issued_fp64_lane_flops_per_alg_flop": (counters["fp64_wave_flops"] * 64.0 / alg_flops)
                     if counters else None,
                     "valu_busy": counters["valu_busy"] if counters else None,
                     "valu_lane_utilisation": counters["valu_lane_util"] if counters else None,
                     "mean_planes": float(npl.mean()), "mean_vertices": float(nv.mean()),
                     "mean_tested": float(ntest.to(torch.float64).mean())},
    }
    # the sort pass against HBM: the algorithmic bytes of a counting sort, about 40 B per particle
    # (positions read, keys written and read, the permutation and the sorted arrays written), over
    # its event-timed duration; `traffic` the bytes the counters measured for the radix sort used
    sort_alg = 40.0 * N
    st_b = sort_traffic() if w.name.startswith("clustered") else None
    out["sort_roofline"] = {"kernel": "sort pass (keys, six 8-bit radix passes, sorted gather, level table, owned list)",
                            "bound": "hbm", "achieved": sort_alg / (build_ms[0] * 1e-3) / 1e9, "peak": 8000.0,
                            "unit": "GB/s", "frac": sort_alg / (build_ms[0] * 1e-3) / 1e9 / 8000.0,
                            "alg_bytes_per_build": sort_alg, "launch_ms": build_ms[0], "traffic": st_b,
                            "traffic_GB_per_s": st_b / (build_ms[0] * 1e-3) / 1e9 if st_b else None}
    gc = grid_counters()
    if gc and not args.fwd_only:
        out["grid_roofline"] = dict(gc, kernel="k_grid_fused (256^3 deposit)", bound="alu",
                                    launch_ms=stage_ms[4])

    if not args.fwd_only:
        # the cheaper grid variant: nearest-particle sampling at the same grid
        samp = {}
        for sub in (1, 2):
            gs = ctx.vt_grid_sample(rho, grid_dims, sub=sub)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(3):
                ctx.vt_grid_sample(rho, grid_dims, sub=sub, out=gs)
            e1.record()
            e1.synchronize()
            ms_s = e0.elapsed_time(e1) / 3
            samp["sub%d" % sub] = {"ms": ms_s, "points_per_s": float(np.prod(grid_dims)) * sub ** 3 / (ms_s * 1e-3),
                                   "mean_abs_diff_vs_exact_over_mean": float((gs - grid).abs().mean() / grid.mean())}
        out["grid_sample"] = dict(samp, grid=list(grid_dims), exact_deposit_ms=stage_ms[4])

        # grid tensors of the deposit (tidal tensor; the Hessian takes the same passes)
        tt = ctx.vt_grid_tensor(grid, vt.TENSOR_TIDAL)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(3):
            ctx.vt_grid_tensor(grid, vt.TENSOR_TIDAL, out=tt)
        e1.record()
        e1.synchronize()
        ms_t = e0.elapsed_time(e1) / 3
        npts = float(np.prod(grid_dims))
        # algorithmic bytes per grid point: the field read once (8) and six components written (48);
        # the implementation moves 600 per point (real->complex 24, forward FFT 3 x 32, per
        # component pair the multiply 32, the inverse FFT 3 x 32 and the unpack 32)
        abytes = npts * (8 + 6 * 8)
        ibytes = npts * (24 + 3 * 32 + 3 * (32 + 3 * 32 + 32))
        out["grid_tensor"] = {"ms": ms_t, "grid": list(grid_dims), "points_per_s": npts / (ms_t * 1e-3),
                              "algorithmic_GB_per_s": abytes / (ms_t * 1e-3) / 1e9,
                              "implementation_GB_per_s": ibytes / (ms_t * 1e-3) / 1e9}
        del tt

        # the full structure output (vertices and faces as loops): one library call with the
        # output arrays in place (count pass, scans, totals read back, write pass)
        so = ctx.vt_structure()
        sizes = (ctypes.c_int64 * 3)()
        nv_, nf_, nl_ = so.verts.shape[0], so.face_nbr.numel(), so.loop_vert.numel()

        def structure_call():
            rc = vt.lib().vt_structure(ctx._ctx, vt._ptr(so.vert_off), vt._ptr(so.verts), nv_, vt._ptr(so.face_off),
                                       vt._ptr(so.face_nbr), nf_, vt._ptr(so.loop_off), vt._ptr(so.loop_vert), nl_,
                                       sizes, vt._stream())
            assert rc == vt.VT_OK, rc

        structure_call()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(3):
            structure_call()
        e1.record()
        e1.synchronize()
        ms_st = e0.elapsed_time(e1) / 3
        nbytes = 16 * (N + 1) + 24 * nv_ + 4 * nf_ + 8 * (nf_ + 1) + 4 * nl_
        out["structure"] = {"ms": ms_st, "cells_per_s": N / (ms_st * 1e-3), "bytes_per_particle": nbytes / N,
                            "written_GB_per_s": nbytes / (ms_st * 1e-3) / 1e9,
                            "vertices_per_cell": nv_ / N, "faces_per_cell": nf_ / N}
        del so

    if not args.no_variants:
        # forward-only comparison of the two precisions at the same accuracy bar
        var = {}
        for name, p in (("fp64", vt.PREC_FP64), ("mixed", vt.PREC_MIXED)):
            opts = {} if args.no_tune else vt.autotune.tune(vt.Context, pos, items, precision=p, reps=1)[0]
            c2 = vt.Context()
            for _ in range(2):
                c2.vt_build(pos, items, precision=p, want_faces=False, **opts)
            torch.cuda.synchronize()
            ta = time.perf_counter()
            reps = 5
            for _ in range(reps):
                c2.vt_build(pos, items, precision=p, want_faces=False, **opts)
                c2.vt_cells_into(vol, off, ids, st)
                c2.vt_density(mass, out=rho)
            torch.cuda.synchronize()
            tb = time.perf_counter()
            code2 = c2.vt_query()[0]
            # the fast clip kernel of this precision against its own vector peak: the same cells, so
            # the same algorithmic flops as the benchmarked build (its cost model above)
            kms = 0.0
            for _ in range(3):
                c2.vt_build(pos, items, precision=p, want_faces=False, timing=True, **opts)
                kms += c2.vt_timings()[1] / 3
            dt = "f64" if p == vt.PREC_FP64 else "f32"
            var[name] = {"fwd_cells_per_s": N * reps / (tb - ta), "status": vt.STATUS_NAMES.get(code2),
                         "launch_options": opts or "defaults",
                         "clip_roofline": {"kernel": "k_clip fast", "bound": "alu", "launch_ms": kms,
                                           "achieved": alg_flops / (kms * 1e-3) / 1e12, "peak": PEAK_TFLOPS[dt],
                                           "unit": "TFLOP/s",
                                           "frac": alg_flops / (kms * 1e-3) / 1e12 / PEAK_TFLOPS[dt]}}
            del c2
        out["precision_variants"] = var

    if not args.no_batched and not args.fwd_only:
        del ctx
        torch.cuda.empty_cache()
        out["batched"] = batched_forms(torch, vt)

    if not args.no_decomposed and not args.fwd_only and w.name.startswith("clustered"):
        torch.cuda.empty_cache()
        out["decomposed"] = decomposed_form(torch, vt, w)

    if not args.no_extra:
        torch.cuda.empty_cache()
        out["backward"] = backward_form(torch, vt)
        out["other_configs"] = other_configs(torch, vt)

    if not args.no_cpu_baseline:
        import oracle

        # the machine's CPU share is 16 cores whatever the host shows; the oracle runs its OpenMP loop
        # over that many threads, and once more on one thread (a smaller sample)
        nthr = min(len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1), 16)
        rng = np.random.default_rng(12345)
        sample = np.sort(rng.choice(N, min(args.cpu_sample, N), replace=False))
        p64 = w.pos.astype(np.float64)
        oracle.cells(p64, w.box_lo, w.box_hi, query=sample[:16], nthreads=nthr)  # warm (page-in)
        ta = time.perf_counter()
        ref = oracle.cells(p64, w.box_lo, w.box_hi, query=sample, nthreads=nthr)
        dens = oracle.density(w.mass[sample], ref.volume)
        tb = time.perf_counter()
        one = sample[: max(16, len(sample) // 32)]
        tc = time.perf_counter()
        oracle.cells(p64, w.box_lo, w.box_hi, query=one, nthreads=1)
        td = time.perf_counter()
        out["cpu_baseline"] = {"value": len(sample) / (tb - ta), "unit": "cells/s", "cores": nthr, "kind": "oracle",
                               "sample": "%d seeded cells of the same workload (neighbours+volume+density, "
                                         "brute force over all %d particles per cell), %.1f s wall" %
                                         (len(sample), N, tb - ta),
                               "one_thread": {"value": len(one) / (td - tc), "cells": int(len(one))},
                               "cpu_model": cpu_model(), "host_cpus": os.cpu_count()}
        # parity of the benchmarked configuration on the same sample
        same = all(np.array_equal(bench_ids[bench_off[i]:bench_off[i + 1]], ref.neighbours(q))
                   for q, i in enumerate(sample))
        rel = np.abs(bench_vol[sample] - ref.volume) / ref.volume
        drel = np.abs(bench_rho[sample] - dens) / dens
        out["parity_on_sample"] = {"neighbours_bit_exact": bool(same), "max_rel_volume_err": float(rel.max()),
                                   "p99_rel_volume_err": float(np.percentile(rel, 99)),
                                   "max_rel_density_err": float(drel.max()),
                                   "p99_rel_density_err": float(np.percentile(drel, 99))}
        if bench_grad is not None:
            # density gradients of the sample's first 256 cells: the oracle's densities of those
            # cells and of all their neighbours (the others from its local-world cells), its
            # least-squares formula; error scaled by max(|grad|, rho / V^(1/3))
            ng = min(256, len(sample))
            grows = sample[:ng]
            nb = np.unique(np.concatenate([ref.neighbours(q) for q in range(ng)]))
            need = np.setdiff1d(nb, sample)
            refn = oracle.local_cells(p64, w.box_lo, w.box_hi, need, workers=nthr)
            rho_ref = np.full(N, np.nan)
            rho_ref[sample] = w.mass[sample] / ref.volume
            rho_ref[need] = w.mass[need] / refn.volume
            goff = np.zeros(ng + 1, np.int64)
            goff[1:] = np.cumsum([ref.nnb[q] for q in range(ng)])
            gids = np.concatenate([ref.neighbours(q) for q in range(ng)])
            gref = oracle.gradient(p64, w.box_lo, w.box_hi, True, goff, gids, rho_ref, rows=grows)
            scale = np.maximum(np.linalg.norm(gref, axis=1), rho_ref[grows] / np.cbrt(ref.volume[:ng]))
            gerr = np.linalg.norm(bench_grad[grows] - gref, axis=1) / scale
            out["parity_on_sample"]["gradient_cells"] = int(ng)
            out["parity_on_sample"]["max_scaled_gradient_err"] = float(gerr.max())
    print(json.dumps(out))


if __name__ == "__main__":
    main()
