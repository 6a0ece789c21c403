#!/usr/bin/env python3
"""BC-apply benchmark on one MI355X.

Headline workload: cubed sphere C384, halo 3, 64 levels x 4 fields (h, tracer
scalars; u, v vector with component rotation across faces), FP64,
point-major storage; BC = face-edge 4-point Lagrange interpolation along the
neighbour's grid line (weights built in FP64 on the GPU) + zero corners.
Inputs are seeded synthetic spherical-harmonic fields + N(0, 1e-3) noise.

One step = one apply of the whole BC (corner zero rows, interpolation rows,
component rotation) to one field.  The K timed steps run as one HIP graph of
K applies cycling over `--copies` independent fields, so the touched data
(about 115 MB per apply) is not served from the 256 MB Infinity Cache.

The other workloads run after the headline and are reported under "extras":
C48 single-field latency, the C384 workload in FP32 and on the plane-major
layout (autotuned), a device copy of the headline's bytes, the C384 plan
trimmed to a radius-1 cross consumer's footprint and that consumer (unfused
and fused with the BC), wide quadrature rows (C384 and C90 (h, u, v)),
block-edge averaging on an Np = 385 grid, the HPCG-shaped 256^3 BC +
27-point operator (BC only, unfused, fused), 64 batched grids of uneven
sizes in FP32 (persistent launch vs 64 plain launches, autotuned), and the
C768 forward / adjoint in FP64 and FP32.  The CPU oracle is timed on the
host and every GPU result is checked against it in the same run.
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import re
import subprocess
import sys
import tempfile
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash():
    """Hash of the sources the apply kernels and their tables are built from,
    with comments and whitespace left out (an edited comment keeps committed
    counters valid; any change to the code voids them)."""
    h = hashlib.sha256()
    for f in ("kernels.hip", "plan.cpp", "hbc_internal.hpp"):
        with open(os.path.join(ROOT, "paper_2605_14780_amd", "csrc", f)) as fh:
            src = fh.read()
        src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
        src = re.sub(r"//[^\n]*", " ", src)
        h.update(" ".join(src.split()).encode())
    return h.hexdigest()[:16]


def traffic_from_profile(name, kernel):
    """HBM bytes per launch of `kernel` from committed counter runs, if they were taken on that
    kernel (the launch shape the autotuner chose in this run) and on the current kernel source."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path))
    except Exception:
        return None
    if rec.get("kernel_source_hash") != kernel_source_hash():
        return None
    return rec.get("kernels", {}).get(kernel, {}).get("hbm_bytes_per_launch")


class Timer:
    """Device events on the current stream around `fn` (which launches `calls` calls)."""

    def __init__(self, torch):
        self.torch = torch

    def __call__(self, fn, calls, warm=1):
        torch = self.torch
        for _ in range(warm):
            fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) * 1e3 / calls  # microseconds per call


def torch_graph(torch, fn):
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        fn()
    return g


# ---------------------------------------------------------------------------------------------
# cpu_baseline leg: the CPU oracle timed on the host, and every GPU result checked against it
# ---------------------------------------------------------------------------------------------
def cpu_baseline_and_checks(ctx, budget_s):
    import numpy as np
    import torch

    import paper_2605_14780_amd as hb
    from oracle import VectorSub, apply as o_apply, assemble, vjp as o_vjp
    from oracle import cubed_sphere as ocs
    from oracle import hpcg as ohpcg
    from tests.helpers import lagrange_tolerance, normwise_error, oracle_weights_program

    out = {}
    # headline: the library's own FP64 weights (arithmetic + position bound, and
    # the plain arithmetic bound for reference), then the program carrying the
    # oracle's own weights in the headline's launch shape (plain bound)
    N, h, vec, full = ctx["c2_N"], ctx["c2_h"], ctx["c2_vec"], ctx["c2_full"]
    og = ocs.grid(N, h)
    op = assemble(og, ocs.subs(N, h, "lagrange", vector=True))
    ref = o_apply(op, full, vec)
    G, Dc = og.ghost_cells, og.data_cells
    got = ctx["c2_got"]
    tol = lagrange_tolerance(N, h, full, ref, vec)
    tol0 = lagrange_tolerance(N, h, full, ref, vec, ds=0.0)
    diff = np.abs(got[G] - ref[G])
    grid_o, prog_o = oracle_weights_program(hb, N, h, True)
    plan_o = hb.Plan(prog_o, inner=full.shape[1], vec=vec, dtype=hb.F64)
    plan_o.tune = ctx["c2_tune"]
    x = torch.from_numpy(full).cuda()
    hb.apply(plan_o, x)
    got_o = x.cpu().numpy()
    del x
    out["c384_f64"] = {
        "normwise_rel_err": normwise_error(got[G], ref[G], full[Dc]),
        "max_err_over_tolerance": float((diff / np.maximum(tol, 1e-300)).max()),
        "tolerance": "1e-13 max(|ref|, sum|w x|) + 4 ulp(N) sum|dw/ds||x|",
        "max_err_over_plain_bound": float((diff / np.maximum(tol0, 1e-300)).max()),
        "oracle_weights_program_max_err_over_plain_bound":
            float((np.abs(got_o[G] - ref[G]) / np.maximum(tol0, 1e-300)).max()),
        "data_cells_untouched": bool(np.array_equal(got[Dc], full[Dc])),
        "all_ghosts_written": bool(np.isfinite(got[G]).all()),
    }
    del got_o, tol0
    if "c2_got32" in ctx:
        g32 = ctx["c2_got32"]
        ref32in = o_apply(op, full.astype(np.float32).astype(np.float64), vec)
        out["c384_f32"] = {
            "normwise_err_vs_fp64_oracle": normwise_error(g32[G], ref[G], full[Dc]),
            "normwise_err_vs_oracle_on_fp32_input": normwise_error(g32[G], ref32in[G], full[Dc]),
            "rms_err_vs_fp64_oracle_rel": float(np.sqrt(np.mean((g32[G] - ref[G]) ** 2)) / np.abs(full[Dc]).max()),
        }
    del ref
    # C48
    if "c1" in ctx:
        N1, h1, f1, res = ctx["c1"]
        og1 = ocs.grid(N1, h1)
        for mode, got1 in res.items():
            op1 = assemble(og1, ocs.subs(N1, h1, mode))
            r1 = o_apply(op1, f1)
            G1 = og1.ghost_cells
            if mode == "sync":
                out[f"c48_{mode}_bit_exact"] = bool(np.array_equal(got1[G1], r1[G1]))
            else:
                t1 = lagrange_tolerance(N1, h1, f1, r1, None)
                out[f"c48_{mode}_max_err_over_tolerance"] = float(
                    (np.abs(got1[G1] - r1[G1]) / np.maximum(t1, 1e-300)).max())
    # HPCG-shaped
    if "c3" in ctx:
        x, ghosted_got, y_fused, y_unfused = ctx["c3"]
        blocks = ohpcg.ghosted_blocks(x, 2)
        want = np.concatenate([b.reshape(-1) for b in blocks])
        out["hpcg_ghosts_bit_exact"] = bool(np.array_equal(ghosted_got, want))
        yref = np.concatenate([ohpcg.stencil27(b).reshape(-1) for b in blocks])
        bound = np.concatenate([ohpcg.abs_row_sum(b).reshape(-1) for b in blocks])
        for name, y in (("fused", y_fused), ("unfused", y_unfused)):
            out[f"hpcg_{name}_max_err_over_bound"] = float((np.abs(y - yref) / (64 * 2.0 ** -53 * bound)).max())
    # 64-grid FP32 batch: sampled ghost rows of three grids against the FP64
    # oracle on the FP64 fields the FP32 inputs were rounded from
    if "c4" in ctx:
        rng = np.random.default_rng(8)
        worst = worst_in = 0.0
        sq, cnt = 0.0, 0
        for k, N4, h4, L4, out32, x64 in ctx["c4"]:
            W4 = N4 + 2 * h4
            scale = float(x64.abs().max())
            picked = 0
            while picked < 300:
                f = int(rng.integers(6))
                j, i = (int(v) for v in rng.integers(-h4, N4 + h4, size=2))
                if (0 <= j < N4 and 0 <= i < N4) or ocs.is_corner(j, i, N4):
                    continue
                ents = ocs.lagrange_entries(f, j, i, N4)
                src = [(g * W4 + (jj + h4)) * W4 + (ii + h4) for (g, jj, ii), _ in ents]
                w = np.array([wv for _, wv in ents])
                X = x64[torch.tensor(src, device=x64.device)].cpu().numpy()
                ref4 = w @ X
                ref4in = w @ X.astype(np.float32).astype(np.float64)
                got4 = out32[(f * W4 + (j + h4)) * W4 + (i + h4)].cpu().numpy().astype(np.float64)
                e = np.abs(got4 - ref4) / scale
                worst = max(worst, float(e.max()))
                worst_in = max(worst_in, float((np.abs(got4 - ref4in) / scale).max()))
                sq += float((e ** 2).sum())
                cnt += e.size
                picked += 1
        out["batch_64_grids_f32"] = {
            "grids_checked": [k for k, *_ in ctx["c4"]], "rows_per_grid": 300,
            "normwise_err_vs_fp64_oracle": worst, "normwise_err_vs_oracle_on_fp32_input": worst_in,
            "rms_err_vs_fp64_oracle_rel": float(np.sqrt(sq / max(cnt, 1)))}
    # C768 forward (FP64 and FP32) and adjoint (FP64 and FP32) against the oracle
    if "c5" in ctx:
        c5 = ctx["c5"]
        N5, h5, f5, bvals = c5["N"], c5["h"], c5["x"], c5["b"]
        og5 = ocs.grid(N5, h5)
        subs = ocs.subs(N5, h5, "lagrange")
        k = 0
        for box in c768_b_boxes(N5, h5):
            n = int(np.prod([b - a for a, b in box]))
            subs.append(VectorSub(box, bvals[k:k + n]))
            k += n
        op5 = assemble(og5, subs)
        r5 = o_apply(op5, f5)
        G5, D5 = og5.ghost_cells, og5.data_cells
        out["c768_f64_forward_normwise_err"] = normwise_error(c5["fwd_f64"][G5], r5[G5], f5[D5])
        r5in = o_apply(op5, f5.astype(np.float32).astype(np.float64))
        out["c768_f32_forward"] = {
            "normwise_err_vs_fp64_oracle": normwise_error(c5["fwd_f32"][G5], r5[G5], f5[D5]),
            "normwise_err_vs_oracle_on_fp32_input": normwise_error(c5["fwd_f32"][G5], r5in[G5], f5[D5]),
            "rms_err_vs_fp64_oracle_rel": float(np.sqrt(np.mean((c5["fwd_f32"][G5] - r5[G5]) ** 2)) /
                                                np.abs(f5[D5]).max())}
        del r5, r5in
        for name in ("f64", "f32"):
            ybar, aty = c5[f"adj_{name}"]
            vref = o_vjp(op5, ybar)
            scale = np.abs(ybar).max(axis=0)
            out[f"c768_{name}_adjoint_normwise_err_vs_fp64_oracle"] = float(
                (np.abs(aty - vref).max(axis=0) / np.where(scale > 0, scale, 1.0)).max())
    return out


# The oracle timed on the host: runs in a child process of bench.py started
# before the parent touches the GPU (a fresh interpreter with no GPU handles);
# it waits on stdin for the path of the headline field, then times full C384
# applies single-threaded and split over a pool of worker processes, and
# prints one JSON line.
_CL = {}


def _cpu_leg_work(cols):
    import numpy as np
    from oracle import apply as o_apply
    nlw = len(cols) // 4
    out = o_apply(_CL["op"], _CL["full"][:, cols], (2 * nlw, nlw, nlw))
    return float(np.abs(out[_CL["G"][:8]]).sum())


def cpu_leg_child(budget_s):
    import multiprocessing as mp
    import numpy as np
    from oracle import apply as o_apply, assemble
    from oracle import cubed_sphere as ocs
    N, h, nf, nl = 384, 3, 4, 64
    path = sys.stdin.readline().strip()
    if not path:
        return
    full = np.load(path, mmap_mode="r")
    og = ocs.grid(N, h)
    op = assemble(og, ocs.subs(N, h, "lagrange", vector=True))
    vec = (2 * nl, nl, nl)
    ghost_values = len(og.ghost_cells) * nf * nl
    res = {"ghost_values_per_apply": ghost_values}
    # (i) one thread: whole applies (A @ X over all 256 slots, rotation, scatter)
    reps, t0 = 0, time.perf_counter()
    while True:
        o_apply(op, full, vec)
        reps += 1
        if time.perf_counter() - t0 >= budget_s / 2:
            break
    dt = time.perf_counter() - t0
    res["single"] = {"applies": reps, "seconds": dt, "cells_per_s": ghost_values * reps / dt}
    # (ii) every core of this process's share: the 64 levels split over worker
    # processes (each takes its levels of all four fields, so (u, v) stay paired)
    naff = len(os.sched_getaffinity(0))
    nw = max(1, min(naff, 16, nl))
    lv = np.array_split(np.arange(nl), nw)
    chunks = [[f * nl + int(l) for f in range(nf) for l in ls] for ls in lv]
    _CL.update(op=op, full=full, G=og.ghost_cells)
    ctx = mp.get_context("fork")
    with ctx.Pool(nw) as pool:
        pool.map(_cpu_leg_work, chunks)  # warm
        reps, t0 = 0, time.perf_counter()
        while True:
            pool.map(_cpu_leg_work, chunks)
            reps += 1
            if time.perf_counter() - t0 >= budget_s / 2:
                break
        dt = time.perf_counter() - t0
    res["all_cores"] = {"workers": nw, "affinity_cpus": naff, "applies": reps, "seconds": dt,
                        "cells_per_s": ghost_values * reps / dt}
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    res["cpu_model"] = model
    print(json.dumps(res), flush=True)


def c768_b_boxes(N, h):
    """Ghost boxes of every face (4 strips, then 4 corners), index (face, j, i)."""
    out = []
    for f in range(6):
        fb = (f, f + 1)
        out += [[fb, (0, N), (-h, 0)], [fb, (0, N), (N, N + h)], [fb, (-h, 0), (0, N)], [fb, (N, N + h), (0, N)]]
    for f in range(6):
        fb = (f, f + 1)
        out += [[fb, a, b] for a in ((-h, 0), (N, N + h)) for b in ((-h, 0), (N, N + h))]
    return out


# ---------------------------------------------------------------------------------------------
def headline(ctx, args, hb, torch, tm):
    import numpy as np
    from tests.helpers import cs_full_field

    N, h, nf, nl = 384, 3, 4, 64
    I = nf * nl
    vec = (2 * nl, nl, nl)
    t0 = time.perf_counter()
    grid, prog = hb.cs_program(N, h, hb.CS_LAGRANGE, vector=True)
    plan = hb.Plan(prog, inner=I, vec=vec, dtype=hb.F64)
    st = plan.stats()
    full = cs_full_field(N, h, nf, nl, seed=2, noise=1e-3)
    src = torch.from_numpy(full).cuda()
    fields = [src.clone() for _ in range(args.copies)]
    torch.cuda.synchronize()
    log(f"C384 setup {time.perf_counter() - t0:.1f}s: {st['segments']} segments, {st['tiles']} tiles, "
        f"tune {plan.tune}")
    hb.apply(plan, fields[0])
    torch.cuda.synchronize()
    ctx.update(c2_N=N, c2_h=h, c2_vec=vec, c2_full=full, c2_got=fields[0].cpu().numpy())
    fields[0].copy_(src)
    del src

    # the default launch shape, then the autotuned one (specialise once, run many)
    g0 = hb.ApplyGraph(plan, fields, args.steps)
    default_us = tm(g0.launch, args.steps)
    default_tune = plan.tune
    del g0
    tune_ms = plan.autotune(fields, os.path.join(tempfile.gettempdir(), "hbc_plan_tune.jsonl"))
    ctx["c2_tune"] = plan.tune
    # timed region: 7 launches of one graph of R applies cycling over the
    # copies, R >= K and >= 2 ms of work; the median launch gives the time per
    # apply
    R = max(args.steps, int(math.ceil(2.0 / max(tune_ms, 1e-4))))
    graph = hb.ApplyGraph(plan, fields, R)
    for k in range(args.warmup):
        hb.apply(plan, fields[k % len(fields)])
    graph.launch()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    launches = []
    w0 = time.perf_counter()
    for _ in range(7):
        e0.record()
        graph.launch()
        e1.record()
        e1.synchronize()
        launches.append(e0.elapsed_time(e1))
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    ms_step = sorted(launches)[3] / R
    res = {"plan": plan, "stats": st, "ms_step": ms_step, "wall": wall,
           "protocol": {"applies_per_launch": R, "launches": 7, "ms_per_launch": launches,
                        "median_ms_per_launch": sorted(launches)[3]},
           "tuning": {"default_tune": default_tune, "default_us_per_apply": default_us, "tuned": plan.tune,
                      "tuned_ms_in_autotune": tune_ms},
           "kernels": plan.kernels()}
    # warm (cache-resident) and eager numbers for context
    g1 = hb.ApplyGraph(plan, [fields[0]], args.steps)
    res["warm_us"] = tm(g1.launch, args.steps)

    def eager():
        for k in range(args.steps):
            hb.apply(plan, fields[k % len(fields)])

    res["eager_us"] = tm(eager, args.steps, warm=0)
    del g1, graph
    # FP32 storage / accumulation on the same workload
    plan32 = hb.Plan(prog, inner=I, vec=vec, dtype=hb.F32)
    src32 = torch.from_numpy(full.astype(np.float32)).cuda()
    f32 = [src32.clone() for _ in range(args.copies)]
    hb.apply(plan32, f32[0])
    torch.cuda.synchronize()
    ctx["c2_got32"] = f32[0].cpu().numpy().astype(np.float64)
    g32 = hb.ApplyGraph(plan32, f32, args.steps)
    us32_default = tm(g32.launch, args.steps)
    del g32
    plan32.autotune(f32, os.path.join(tempfile.gettempdir(), "hbc_plan_tune.jsonl"))  # as the FP64 plan
    g32 = hb.ApplyGraph(plan32, f32, args.steps)
    us32 = tm(g32.launch, args.steps)
    st32 = plan32.stats()
    res["f32"] = {"us_per_apply": us32, "ghost_cells_per_s": st32["ghost_values"] / us32 * 1e6,
                  "hbm_frac": st32["alg_bytes"] / us32 / 1e3 / HBM_PEAK_GBS,
                  "f64_over_f32_time": (ms_step * 1e3) / us32,
                  "default_shape_us_per_apply": us32_default, "tune": plan32.tune}
    del g32, f32, src32, fields
    torch.cuda.empty_cache()
    return res


def extra_c384_plane_major(ctx, hb, torch, tm):
    """The headline operator on the plane-major layout (value l of every cell contiguous)."""
    N, h, nf, nl = 384, 3, 4, 64
    I = nf * nl
    vec = (2 * nl, nl, nl)
    grid, prog = hb.cs_program(N, h, hb.CS_LAGRANGE, vector=True)
    plan = hb.Plan(prog, inner=I, vec=vec, dtype=hb.F64, order=hb.PLANE_MAJOR)
    st = plan.stats()
    src = torch.from_numpy(ctx["c2_full"]).cuda().t().contiguous().reshape(-1)
    fields = [src.clone() for _ in range(3)]
    del src
    g = hb.ApplyGraph(plan, fields, 90)
    us_default = tm(g.launch, 90)
    del g
    plan.autotune(fields, os.path.join(tempfile.gettempdir(), "hbc_plan_tune.jsonl"))
    g = hb.ApplyGraph(plan, fields, 90)
    us = tm(g.launch, 90)
    del g, fields
    # the same operator on the point-major layout is the headline's (oracle-checked) result
    x = torch.from_numpy(ctx["c2_full"]).cuda().t().contiguous()
    hb.apply(plan, x.reshape(-1))
    got = x.t().contiguous()
    del x
    ref = torch.from_numpy(ctx["c2_got"]).cuda()
    finite = torch.isfinite(ref).all(dim=1)
    scale = float(ref[finite].abs().max())
    out = {"us_per_apply": us, "default_shape_us_per_apply": us_default, "tune": plan.tune,
           "ghost_cells_per_s": st["ghost_values"] / us * 1e6,
           "hbm_frac": st["alg_bytes"] / us / 1e3 / HBM_PEAK_GBS, "copies": 3,
           "bit_identical_to_point_major": bool(torch.equal(got, ref)),
           "max_diff_vs_point_major_over_max_value": float((got[finite] - ref[finite]).abs().max()) / scale}
    del got, ref, finite
    torch.cuda.empty_cache()
    return out


def default_and_tuned(hb, plan, fields, reps, tm, op=None):
    """Microseconds per call of `reps` applies over `fields` in one graph, at the
    plan's default launch shape and after the plan autotuner."""
    kw = {} if op is None else {"op": op}
    g = hb.ApplyGraph(plan, fields, reps, **kw)
    us0 = tm(g.launch, reps)
    del g
    plan.autotune(fields, os.path.join(tempfile.gettempdir(), "hbc_plan_tune.jsonl"))
    g = hb.ApplyGraph(plan, fields, reps, **kw)
    us1 = tm(g.launch, reps)
    del g
    return us0, us1


def extra_edge_average(ctx, hb, torch, tm):
    """Vertex-centred C384 (385 points per side), h 3, 256 values per point, FP64:
    rotated ghost copies plus block-edge averaging of the co-located boundary
    points (data rows, staged through scratch) vs the ghost copies alone."""
    import synthinputs
    Np, h, I = 385, 3, 256
    W = Np + 2 * h
    data = synthinputs.cs_sh_field_torch(Np, 4, 64, seed=6)  # point values at cell-centre angles of Np
    full = torch.zeros((6, W, W, I), dtype=torch.float64, device="cuda")
    full[:, h:h + Np, h:h + Np, :] = data
    full = full.reshape(-1)
    del data
    out = {}
    for name, avg in (("ghosts_only", False), ("ghosts_and_edge_average", True)):
        g = hb.Grid.cubed_sphere(Np, h)
        p = hb.Program(g)
        p.cs_add(Np, h, hb.CS_SYNC)
        if avg:
            p.cs_add_edge_average(Np)
        plan = hb.Plan(p, inner=I, dtype=hb.F64)
        st = plan.stats()
        fields = [full.clone() for _ in range(3)]
        us0, us = default_and_tuned(hb, plan, fields, 60, tm)
        out[name] = {"us_per_apply": us, "default_shape_us_per_apply": us0, "rows_data": st["rows_data"],
                     "rows_covered": st["rows_covered"], "alg_bytes": st["alg_bytes"],
                     "hbm_frac": st["alg_bytes"] / us / 1e3 / HBM_PEAK_GBS}
        del fields
        torch.cuda.empty_cache()
    out["data_rows_extra_us"] = out["ghosts_and_edge_average"]["us_per_apply"] - out["ghosts_only"]["us_per_apply"]
    return out


def extra_footprint(ctx, hb, torch, tm):
    """The headline operator with a consumer footprint declared: a radius-1
    cross stencil reads one ghost layer of the three (Sec. IV-C removes the
    other rows), against the full halo."""
    N, h, nf, nl = 384, 3, 4, 64
    I = nf * nl
    vec = (2 * nl, nl, nl)
    offs = [(0, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)]
    grid, prog = hb.cs_program(N, h, hb.CS_LAGRANGE, vector=True)
    prog.set_consumer(offs)
    plan = hb.Plan(prog, inner=I, vec=vec, dtype=hb.F64)
    st = plan.stats()
    src = torch.from_numpy(ctx["c2_full"]).cuda()
    fields = [src.clone() for _ in range(9)]
    del src
    us0, us = default_and_tuned(hb, plan, fields, 90, tm)
    del fields
    # the kept rows equal the headline's (oracle-checked) rows bit for bit;
    # dead rows stay untouched (NaN in the input)
    x = torch.from_numpy(ctx["c2_full"]).cuda()
    ghost = torch.isnan(x).any(dim=1)
    hb.apply(plan, x)
    ref = torch.from_numpy(ctx["c2_got"]).cuda()
    kept = ghost & ~torch.isnan(x).any(dim=1)
    same = int(kept.sum()) == st["rows_covered"] and torch.equal(x[kept], ref[kept])
    del x, ref, ghost, kept
    out = {"consumer": "cross radius 1", "rows_covered": st["rows_covered"], "rows_dead": st["rows_dead"],
           "us_per_apply": us, "default_shape_us_per_apply": us0, "alg_bytes": st["alg_bytes"],
           "hbm_frac": st["alg_bytes"] / us / 1e3 / HBM_PEAK_GBS,
           "kept_rows_equal_full_halo_rows_bitwise": bool(same)}
    torch.cuda.empty_cache()
    return out


def extra_consumer(ctx, hb, torch, tm):
    """The C384 fields (I = 256, FP64) read by a radius-1 cross stencil after
    the BC (Sec. IV-C): the BC compiled for the stencil's footprint, then the
    stencil reading the stored ghosts (unfused), against the stencil fused
    with the BC (boundary cells' rows composed with the BC rows, x only
    read)."""
    N, h, nf, nl = 384, 3, 4, 64
    I = nf * nl
    vec = (2 * nl, nl, nl)
    cross = [(0, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)]
    wts = [-4.0, 1.0, 1.0, 1.0, 1.0]
    grid, prog = hb.cs_program(N, h, hb.CS_LAGRANGE, vector=True)
    prog.set_consumer(cross)
    plan = hb.Plan(prog, inner=I, vec=vec, dtype=hb.F64)
    cons = hb.Consumer(plan, cross, wts)
    src = torch.from_numpy(ctx["c2_full"]).cuda()
    C = 3
    xs = [src.clone() for _ in range(C)]
    del src
    ndata = 6 * N * N
    ys = [torch.empty(ndata * I, dtype=torch.float64, device="cuda") for _ in range(C)]
    R = 12

    def apply_only():
        for r in range(R):
            hb.apply(plan, xs[r % C])

    def stencil_only():
        for r in range(R):
            cons.apply(xs[r % C], ys[r % C], fused=False)

    def unfused():
        for r in range(R):
            hb.apply(plan, xs[r % C])
            cons.apply(xs[r % C], ys[r % C], fused=False)

    def fused():
        for r in range(R):
            cons.apply(xs[r % C], ys[r % C], fused=True)

    alg = 2.0 * ndata * I * 8  # x data read once, y written once
    out = {"consumer": "cross radius 1, weights (-4, 1, 1, 1, 1)", "boundary_rows": cons.stats()["boundary_rows"],
           "alg_bytes_stencil": alg}
    for name, fn in (("bc_apply_footprint", apply_only), ("stencil_on_stored_ghosts", stencil_only),
                     ("unfused_apply_then_stencil", unfused), ("fused", fused)):
        g = torch_graph(torch, fn)
        us = tm(g.replay, R)
        del g
        out[name] = {"us": us, "hbm_frac": (alg if name != "bc_apply_footprint" else plan.stats()["alg_bytes"]) /
                     us / 1e3 / HBM_PEAK_GBS}
    out["fused_speedup_vs_unfused"] = out["unfused_apply_then_stencil"]["us"] / out["fused"]["us"]
    del xs, ys
    torch.cuda.empty_cache()
    return out


def extra_wide_rows(ctx, hb, torch, tm):
    """Wide interpolation rows (Gauss average over each ghost cell of cubic
    tensor-product reconstructions, 16..25 entries per row, CSR): the
    headline's C384 fields (I = 256, FP64, 9 cold copies) and the paper's
    6 x 90 x 90 shallow-water grid with (h, u, v) per cell."""
    import numpy as np
    out = {}
    N, h, nf, nl = 384, 3, 4, 64
    I = nf * nl
    vec = (2 * nl, nl, nl)
    g = hb.Grid.cubed_sphere(N, h)
    p = hb.Program(g)
    p.cs_add_quadrature(N, h, 2, vector=True)
    plan = hb.Plan(p, inner=I, vec=vec, dtype=hb.F64)
    st = plan.stats()
    src = torch.from_numpy(ctx["c2_full"]).cuda()
    fields = [src.clone() for _ in range(9)]
    del src
    gr = hb.ApplyGraph(plan, fields, 90)
    us = tm(gr.launch, 90)
    out["c384_i256_f64"] = {"us_per_apply": us, "nnz_per_row": st["nnz"] / st["rows_csr"],
                            "ghost_cells_per_s": st["ghost_values"] / us * 1e6, "alg_bytes": st["alg_bytes"],
                            "hbm_frac": st["alg_bytes"] / us / 1e3 / HBM_PEAK_GBS}
    del gr, fields
    torch.cuda.empty_cache()
    N, h, L = 90, 3, 1
    from tests.helpers import cs_full_field
    g = hb.Grid.cubed_sphere(N, h)
    p = hb.Program(g)
    p.cs_add_quadrature(N, h, 2, vector=True)
    plan = hb.Plan(p, inner=3, vec=(1, 1, 1), dtype=hb.F64)
    st = plan.stats()
    full = torch.from_numpy(cs_full_field(N, h, 3, L, seed=9)).cuda()
    gr = hb.ApplyGraph(plan, [full], 2000)
    us = tm(gr.launch, 2000)
    out["c90_hUV_f64"] = {"us_per_apply": us, "ghost_cells_per_s": st["ghost_values"] / us * 1e6,
                          "nnz_per_row": st["nnz"] / st["rows_csr"], "alg_bytes": st["alg_bytes"],
                          "rows_narrow": st["rows_narrow"]}
    return out


def extra_copy_ceiling(ctx, hb, torch, tm):
    """A plain device-to-device copy (the runtime's copy kernel) that reads and
    writes the headline apply's algorithmic bytes (half read, half written),
    cycling 9 buffers in one graph like the headline: what a straight copy of
    the same byte count reaches on this GPU at this size."""
    alg = ctx["c2_alg_bytes"]
    n = int(alg / 2 / 8)
    bufs = [torch.randn(2 * n, dtype=torch.float64, device="cuda") for _ in range(9)]
    R = 90

    def copies():
        for r in range(R):
            b = bufs[r % len(bufs)]
            b[n:].copy_(b[:n])

    g = torch_graph(torch, copies)
    us = tm(g.replay, R)
    del g, bufs
    torch.cuda.empty_cache()
    return {"bytes_per_copy": 2 * n * 8, "us_per_copy": us, "GBs": 2 * n * 8 / us / 1e3,
            "hbm_frac": 2 * n * 8 / us / 1e3 / HBM_PEAK_GBS,
            "apply_over_copy_rate": (ctx["c2_apply_GBs"] / (2 * n * 8 / us / 1e3))}


def extra_c48(ctx, hb, torch, tm):
    from tests.helpers import cs_full_field
    N, h = 48, 3
    full = cs_full_field(N, h, 1, 1, seed=1)
    out, got = {}, {}
    for mode, m in (("lagrange", hb.CS_LAGRANGE), ("sync", hb.CS_SYNC)):
        grid, prog = hb.cs_program(N, h, m)
        plan = hb.Plan(prog, inner=1)
        t = torch.from_numpy(full.copy()).cuda()
        hb.apply(plan, t)
        torch.cuda.synchronize()
        got[mode] = t.cpu().numpy()
        g = hb.ApplyGraph(plan, [t], 2000)
        us = tm(g.launch, 2000)
        out[mode] = {"us_per_apply": us, "ghost_cells_per_s": plan.stats()["ghost_values"] / us * 1e6}
    ctx["c1"] = (N, h, full, got)
    return out


def extra_hpcg(ctx, hb, torch, tm):
    import numpy as np
    import synthinputs
    nb, n = 2, 128
    x = synthinputs.uniform((nb * n,) * 3, seed=3)
    grid = hb.Grid.cartesian([nb] * 3, [n] * 3, 1)
    prog = hb.Program(grid)
    prog.cart_add_halo([nb] * 3, [n] * 3, 1)
    plan = hb.Plan(prog, inner=1)
    st = plan.stats()
    W = n + 2
    full = np.full((nb ** 3, W, W, W), np.nan)
    for bz in range(nb):
        for by in range(nb):
            for bx in range(nb):
                full[(bz * nb + by) * nb + bx, 1:-1, 1:-1, 1:-1] = x[bz * n:(bz + 1) * n, by * n:(by + 1) * n,
                                                                    bx * n:(bx + 1) * n]
    full = full.reshape(-1)
    src = torch.from_numpy(full).cuda()
    C = 3
    xs = [src.clone() for _ in range(C)]
    ys = [torch.empty(nb ** 3 * n ** 3, dtype=torch.float64, device="cuda") for _ in range(C)]
    hb.fused_stencil27(plan, xs[0], ys[0])
    torch.cuda.synchronize()
    ghosted = xs[0].cpu().numpy()
    y_fused = ys[0].cpu().numpy()
    xs[0].copy_(src)
    hb.apply(plan, xs[0])
    hb.stencil27(plan, xs[0], ys[0])
    torch.cuda.synchronize()
    y_unfused = ys[0].cpu().numpy()
    ctx["c3"] = (x, ghosted, y_fused, y_unfused)
    R = 60

    def bc_only():
        for r in range(R):
            hb.apply(plan, xs[r % C])

    def unfused():
        for r in range(R):
            hb.apply(plan, xs[r % C])
            hb.stencil27(plan, xs[r % C], ys[r % C])

    def fused():
        for r in range(R):
            hb.fused_stencil27(plan, xs[r % C], ys[r % C])

    def fused_no_ghost_store():
        for r in range(R):
            hb.fused_stencil27(plan, xs[r % C], ys[r % C], write_ghosts=False)

    out = {}
    data_b = nb ** 3 * n ** 3 * 8
    ghost_b = st["rows_covered"] * 8
    alg = {"bc_only": st["alg_bytes"],
           "unfused": st["alg_bytes"] + (len(full) * 8 + data_b),
           "fused": 2 * data_b + ghost_b,
           "fused_no_ghost_store": 2 * data_b}
    for name, fn in (("bc_only", bc_only), ("unfused", unfused), ("fused", fused),
                     ("fused_no_ghost_store", fused_no_ghost_store)):
        g = torch_graph(torch, fn)
        us = tm(g.replay, R)
        out[name] = {"us": us, "alg_bytes": alg[name], "hbm_frac": alg[name] / us / 1e3 / HBM_PEAK_GBS}
    out["fused_speedup_vs_unfused"] = out["unfused"]["us"] / out["fused"]["us"]
    out["fused_no_ghost_store_speedup_vs_unfused"] = out["unfused"]["us"] / out["fused_no_ghost_store"]["us"]
    out["ghost_cells_per_s_bc_only"] = st["ghost_values"] / out["bc_only"]["us"] * 1e6
    return out


def extra_batch(ctx, hb, torch, tm):
    import synthinputs
    draws = synthinputs.batch_draw()
    plans, plain, batched = [], [], []
    t0 = time.perf_counter()
    for k, (N, h, L) in enumerate(draws):
        grid, prog = hb.cs_program(N, h, hb.CS_LAGRANGE)
        plan = hb.Plan(prog, inner=L, dtype=hb.F32)
        W = N + 2 * h
        full = torch.full((6, W, W, L), float("nan"), dtype=torch.float32, device="cuda")
        full[:, h:h + N, h:h + N, :] = synthinputs.cs_sh_field_torch(N, 1, L, seed=4000 + k, dtype=torch.float32)
        full = full.reshape(-1)
        plans.append(plan)
        plain.append(full)
        batched.append(full.clone())
    torch.cuda.synchronize()
    log(f"batch setup {time.perf_counter() - t0:.1f}s")
    ghost_values = sum(p.stats()["ghost_values"] for p in plans)
    alg = sum(p.stats()["alg_bytes"] for p in plans)

    def plain_all():
        for p, f in zip(plans, plain):
            hb.apply(p, f)

    gp = torch_graph(torch, plain_all)
    us_plain = tm(gp.replay, 1)
    batch = hb.Batch(plans)
    batch.bind(batched)
    s = torch.cuda.current_stream()
    batch.graph_capture(s.cuda_stream)
    us_default = tm(lambda: batch.graph_launch(s.cuda_stream), 1)
    tuned_ms = batch.autotune(os.path.join(tempfile.gettempdir(), "hbc_autotune_cache.jsonl"))
    batch.graph_capture(s.cuda_stream)
    us_tuned = tm(lambda: batch.graph_launch(s.cuda_stream), 1)
    # bit identity of batched vs plain (both applied once more from the same inputs)
    for p, b in zip(plain, batched):
        b.copy_(p)
    gp.replay()
    batch.graph_launch(s.cuda_stream)
    torch.cuda.synchronize()
    same = all(torch.equal(p, b) for p, b in zip(plain, batched))
    # three grids' FP32 results and the FP64 fields their inputs were rounded
    # from, for the error against the FP64 oracle (cpu_baseline leg)
    sizes = [N for N, _, _ in draws]
    ctx["c4"] = []
    for k in sorted({int(min(range(len(draws)), key=lambda q: sizes[q])),
                     int(max(range(len(draws)), key=lambda q: sizes[q])), 17}):
        N, h, L = draws[k]
        W = N + 2 * h
        x64 = torch.zeros((6, W, W, L), dtype=torch.float64, device="cuda")
        x64[:, h:h + N, h:h + N, :] = synthinputs.cs_sh_field_torch(N, 1, L, seed=4000 + k)
        ctx["c4"].append((k, N, h, L, batched[k].view(-1, L), x64.view(-1, L)))
    out = {"grids": len(plans), "ghost_values": ghost_values, "alg_bytes": alg,
           "plain_64_launches_us": us_plain, "batched_default_us": us_default, "batched_tuned_us": us_tuned,
           "tune": batch.tune, "autotune_ms": tuned_ms,
           "speedup_batched_vs_plain": us_plain / us_tuned,
           "ghost_cells_per_s": ghost_values / us_tuned * 1e6,
           "hbm_frac": alg / us_tuned / 1e3 / HBM_PEAK_GBS,
           "bit_identical_to_plain": bool(same),
           "resident_bytes": sum(f.numel() * 4 for f in plain) * 2}
    del gp, batch, plain, batched
    torch.cuda.empty_cache()
    return out


def extra_adjoint(ctx, hb, torch, tm):
    import numpy as np
    import synthinputs
    N, h, L = 768, 3, 32
    rng = np.random.default_rng(5)
    boxes = c768_b_boxes(N, h)
    nrows = sum(int(np.prod([b - a for a, b in box])) for box in boxes)
    bvals = rng.normal(0.0, 1.0, size=(nrows, L))
    W = N + 2 * h
    data = synthinputs.cs_sh_field_torch(N, 1, L, seed=5)
    out = {}
    for name, dt, tdt in (("f64", hb.F64, torch.float64), ("f32", hb.F32, torch.float32)):
        grid, prog = hb.cs_program(N, h, hb.CS_LAGRANGE)
        k = 0
        for box in boxes:
            n = int(np.prod([b - a for a, b in box]))
            prog.add_vector(box, bvals[k:k + n], ninner=L)
            k += n
        plan = hb.Plan(prog, inner=L, dtype=dt)
        st = plan.stats()
        full = torch.zeros((6, W, W, L), dtype=tdt, device="cuda")
        full[:, h:h + N, h:h + N, :] = data.to(tdt)
        full = full.reshape(-1)
        C = 3
        xs = [full.clone() for _ in range(C)]
        c5 = ctx.setdefault("c5", {"N": N, "h": h, "b": bvals})
        if name == "f64":
            c5["x"] = full.view(-1, L).cpu().numpy()
        hb.apply(plan, xs[0])
        torch.cuda.synchronize()
        c5[f"fwd_{name}"] = xs[0].view(-1, L).cpu().numpy().astype(np.float64)
        xs[0].copy_(full)
        gf = hb.ApplyGraph(plan, xs, 60)
        us_f = tm(gf.launch, 60)
        gen = torch.Generator(device="cuda")
        gen.manual_seed(7)
        ys = [torch.randn(full.numel(), dtype=tdt, device="cuda", generator=gen) for _ in range(C)]
        ga = hb.ApplyGraph(plan, ys, 60, op=hb.OP_ADJOINT)
        us_a = tm(ga.launch, 60)
        # dot-product test <A x, y> = <x, A^T y>, accumulated in FP64
        x = full.clone()
        z = torch.zeros_like(full)
        Ax = x.clone()
        hb.apply(plan, Ax)
        hb.apply(plan, z)
        y = torch.randn(full.numel(), dtype=tdt, device="cuda", generator=gen)
        Aty = y.clone()
        hb.apply_adjoint(plan, Aty)
        torch.cuda.synchronize()
        lhs = float(((Ax.double() - z.double()) * y.double()).sum())
        rhs = float((x.double() * Aty.double()).sum())
        c5[f"adj_{name}"] = (y.view(-1, L).cpu().numpy().astype(np.float64),
                             Aty.view(-1, L).cpu().numpy().astype(np.float64))
        out[name] = {"forward_us": us_f, "adjoint_us": us_a, "adjoint_over_forward": us_a / us_f,
                     "forward_hbm_frac": st["alg_bytes"] / us_f / 1e3 / HBM_PEAK_GBS,
                     "adjoint_hbm_frac": st["alg_bytes_adjoint"] / us_a / 1e3 / HBM_PEAK_GBS,
                     "ghost_cells_per_s_forward": st["ghost_values"] / us_f * 1e6,
                     "dot_product_rel": abs(lhs - rhs) / max(abs(lhs), abs(rhs))}
        del gf, ga, xs, ys
        torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--copies", type=int, default=9, help="independent fields cycled for cold-cache timing")
    ap.add_argument("--cpu-budget", type=float, default=10.0, help="seconds of oracle work for cpu_baseline")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--extras", default="all",
                    help="comma-separated subset of: copy_ceiling, c384_plane_major, c384_cross_footprint, c384_cross_consumer, wide_rows, edge_average_np385, "
                         "c48_latency, hpcg_256cube, "
                         "batched_64_grids_f32, c768_adjoint")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain device copy of 256 MiB, 20 times (counter calibration)")
    ap.add_argument("--cpu-leg", action="store_true", help=argparse.SUPPRESS)  # the child of the cpu_baseline leg
    args = ap.parse_args()
    if args.cpu_leg:
        cpu_leg_child(args.cpu_budget)
        return
    if args.calibrate_copy:
        import torch
        a = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(20):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"calibration": "copy", "bytes_read": a.numel() * 8, "bytes_written": b.numel() * 8}))
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the library runs on one GPU; applies sharded over several GPUs are not implemented"}))
        sys.exit(2)

    # the cpu_baseline leg's child process, started before anything touches
    # the GPU; it waits for the headline field, then times the oracle
    cpu_child = subprocess.Popen([sys.executable, os.path.abspath(__file__), "--cpu-leg", "--cpu-budget",
                                  str(args.cpu_budget)], stdin=subprocess.PIPE, stdout=subprocess.PIPE, text=True)

    import torch

    import paper_2605_14780_amd as hb

    torch.cuda.set_device(0)
    # graph capture needs a stream other than the legacy default one
    stream = torch.cuda.Stream()
    torch.cuda.set_stream(stream)
    tm = Timer(torch)
    ctx = {}
    res = headline(ctx, args, hb, torch, tm)
    st = res["stats"]
    log("headline done")
    ctx["c2_alg_bytes"] = st["alg_bytes"]
    ctx["c2_apply_GBs"] = st["alg_bytes"] / (res["ms_step"] / 1e3) / 1e9
    extras = {"c384_warm_cache_us_per_apply": res["warm_us"], "c384_eager_us_per_apply": res["eager_us"],
              "c384_f32": res["f32"], "c384_launch_shape": res["tuning"]}
    if not args.no_extras:
        table = (("copy_ceiling", extra_copy_ceiling),
                 ("c384_plane_major", extra_c384_plane_major), ("c384_cross_footprint", extra_footprint),
                 ("c384_cross_consumer", extra_consumer),
                 ("wide_rows", extra_wide_rows),
                 ("edge_average_np385", extra_edge_average),
                 ("c48_latency", extra_c48),
                 ("hpcg_256cube", extra_hpcg), ("batched_64_grids_f32", extra_batch),
                 ("c768_adjoint", extra_adjoint))
        want = {n for n, _ in table} if args.extras == "all" else set(args.extras.split(","))
        unknown = want - {n for n, _ in table}
        if unknown:
            raise SystemExit(f"unknown extras: {sorted(unknown)}")
        for name, fn in table:
            if name not in want:
                continue
            t0 = time.perf_counter()
            extras[name] = fn(ctx, hb, torch, tm)
            log(f"{name} done in {time.perf_counter() - t0:.1f}s")
        if "batched_64_grids_f32" in extras:
            f64_ns = res["ms_step"] * 1e6 / st["ghost_values"]
            b32 = extras["batched_64_grids_f32"]
            extras["ns_per_ghost_value_plain_f64_over_batched_f32"] = f64_ns / (b32["batched_tuned_us"] * 1e3 /
                                                                                b32["ghost_values"])

    log("cpu_baseline leg: oracle timing (child process) and checks")
    import numpy as np
    fpath = os.path.join(tempfile.gettempdir(), f"hbc_c384_field_{os.getpid()}.npy")
    np.save(fpath, ctx["c2_full"])
    try:
        out_child, _ = cpu_child.communicate(fpath + "\n", timeout=60 + 20 * args.cpu_budget)
    finally:
        os.remove(fpath)
    timing = json.loads(out_child.strip().splitlines()[-1])
    chk = cpu_baseline_and_checks(ctx, args.cpu_budget)
    ms_step = res["ms_step"]
    value = st["ghost_values"] / (ms_step / 1e3)
    achieved = st["alg_bytes"] / (ms_step / 1e3) / 1e9
    kern = [k.split("(")[0].replace("void ", "", 1) for k in res["kernels"]]
    allc, one = timing["all_cores"], timing["single"]
    out = {
        "metric": "BC-apply ghost cells/s + % HBM peak; batched FP32 & adjoint vs plain FP64",
        "value": value,
        "unit": "ghost cells/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded spherical-harmonic fields + N(0,1e-3) noise)",
        "config": {"workload": "cubed-sphere C384, halo 3, 64 levels x 4 fields (h, tracer, u, v), "
                               "Lagrange face-edge interpolation + component rotation + zero corners, "
                               "point-major FP64, cache-rotated over independent fields", "N": 384, "halo": 3,
                   "inner": 256, "ghost_values_per_apply": st["ghost_values"], "copies": args.copies},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic_from_profile("apply_c384_f64_pmc.json", kern[0]) if len(kern) == 1 else None,
                     "alg_bytes_per_launch": st["alg_bytes"], "kernel": kern[0],
                     **({"kernels": kern} if len(kern) > 1 else {})},
        "cpu_baseline": {"value": allc["cells_per_s"], "unit": "ghost cells/s", "cores": allc["workers"],
                         "kind": "oracle",
                         "sample": f"{allc['applies']} full applies of the C384 operator (scipy CSR A @ X + "
                                   f"rotation + scatter; the 64 levels split over {allc['workers']} worker "
                                   f"processes), assembly excluded",
                         "cpu_model": timing["cpu_model"], "affinity_cpus": allc["affinity_cpus"],
                         "single_thread": {"value": one["cells_per_s"], "applies": one["applies"],
                                           "seconds": one["seconds"]},
                         "gpu_over_cpu_all_cores": value / allc["cells_per_s"],
                         "gpu_over_cpu_single_thread": value / one["cells_per_s"]},
        "timing_protocol": res["protocol"],
        "checks_vs_oracle": chk,
        "wall_s_timed": res["wall"],
        "extras": extras,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
