"""Benchmark: GDoF/s of the sum-factorised Q_p Laplace action, p = 1..8, FP64.

Workload: 64^3 = 262,144 axis-aligned box cells with edge lengths U[0.5, 1.5],
kappa U[0.5, 2] per Gauss point ((p+1)^3 points), DOF vectors N(0, 1), FP64
storage and arithmetic.  One step is one Laplace action of every degree
p = 1..8 over the whole mesh (8 launches).  value = sum over p of the global
Q_p DOF count (64p+1)^3 divided by the summed time; the per-degree rates,
local-DOF rates, roofline fractions and the mixed-precision comparison are
reported beside it.  Inputs are resident in HBM before timing; several input
copies are rotated so that every launch streams more than the 256 MB
last-level cache.  Kernel durations come from HIP events recorded on the
stream the kernels run on; each degree's time is the median over the timed
steps (side legs: the median over their repetitions).  The library is told that every cell is a box
(sf_set_geometry) and each degree's kernel variant is autotuned first.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]
"""
import argparse
import json
import math
import os
import sys
import tempfile
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

NCELL1 = 64
PEAK_HBM_GBS = 8000.0
PEAK_FP64_TFLOPS = 78.6


def action_bytes_per_cell(p, io_bytes=8):
    """Algorithmic HBM bytes per cell of the action: u, y and kappa (n^3 each,
    n = p+1) plus the 8 FP64 vertices."""
    n = p + 1
    return 3 * io_bytes * n ** 3 + 192


def action_flops_per_cell(p):
    """Algorithmic flops per cell of the sum-factorised Laplace action on a box
    (the measurement model of the hot-path scope): 16 one-axis contractions of
    2 n^4 (forward B/D to values and gradients, their transposes back) plus
    about 5 n^3 for the pointwise stage.  The kernels reach the same sum with
    fewer operations (collocated derivative, even-odd tables)."""
    n = p + 1
    return 32 * n ** 4 + 5 * n ** 3


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--degrees", default="1,2,3,4,5,6,7,8")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=16.0)
    ap.add_argument("--mixed-degrees", default="1,2,3,4,5,6,7,8", help="degrees of the mixed-precision leg ('' = off)")
    ap.add_argument("--tune", choices=("cached", "run", "off"), default="cached",
                    help="kernel variants: 'cached' loads the autotuner's recorded choices for this GPU "
                         "(paper_1711_02473_amd/tuning/gfx950.json) and tunes what it lacks; 'run' autotunes "
                         "every degree now; 'off' keeps the library defaults")
    ap.add_argument("--no-tune", dest="tune", action="store_const", const="off", help="same as --tune off")
    ap.add_argument("--save-tuning", default="", help="write the tuning choices used to this JSON file")
    ap.add_argument("--legs", default="mass,collocated,trilinear,vq,svk,global,vec,matrix,batch",
                    help="side measurements beside the headline: mass (Q_p mass action, 64^3), collocated "
                         "(Laplace action with the GLL rule, B = I, 64^3), trilinear (Laplace action on general "
                         "trilinear cells, per-point geometry, 64^3 cells), vq (vector Q_p Laplace action, 64^3, and "
                         "its block-diagonal element matrices), svk (Saint Venant-Kirchhoff "
                         "linearised residual on vector Q_p, 64^3 cells), global (the "
                         "assembled C0 Q_p Laplace action on global vectors, 64^3), vec (NCF/NCE "
                         "actions, 48^3), matrix (Q_p Laplace element matrices), batch (2048-mesh batched "
                         "launch); '' = none")
    ap.add_argument("--calib-copy", action="store_true",
                    help="end with one 1 GiB device copy, the reference for HBM byte counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: measures one GPU only (the action is cell-local, so more GPUs would each "
              "take a share of the cells); --gpus %d is not supported" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1711_02473_amd as sf
    from paper_1711_02473_amd import synth

    sf.load()
    ctx = sf.Context(0)
    degrees = [int(x) for x in args.degrees.split(",")]
    ncells = NCELL1 ** 3
    V = torch.from_numpy(synth.box_mesh(NCELL1, NCELL1, NCELL1, 2)).cuda()
    stream = torch.cuda.current_stream()

    # inputs per degree, rotated copies to defeat the last-level cache
    bufs = {}
    for p in degrees:
        n3 = (p + 1) ** 3
        per_set = 3 * 8 * n3 * ncells
        nsets = max(1, min(6, math.ceil(768e6 / per_set)))
        bufs[p] = [(kap, u, torch.empty_like(u)) for kap, u in synth.device_action_inputs(ncells, n3, 2, p, nsets)]
    ops = {p: sf.make_op("Q", p, "LAPLACE") for p in degrees}
    # every cell is an axis-aligned box: the library may use its box-cell kernels
    sf.sf_set_geometry(ctx, "box")
    tuned = {}
    if args.tune != "off":
        cache = os.path.join(ROOT, "paper_1711_02473_amd", "tuning", "gfx950.json")
        if args.tune == "cached" and os.path.exists(cache):
            sf.sf_load_tuning(ctx, cache)
            with open(cache) as f:
                tuned = json.load(f)
        with tempfile.TemporaryDirectory() as td:
            path = os.path.join(td, "tune.json")
            for op, keys in tuning_classes(sf, degrees, [int(x) for x in args.mixed_degrees.split(",") if x],
                                           [x for x in args.legs.split(",") if x]):
                if args.tune == "run" or any(k not in tuned for k in keys):
                    sf.sf_autotune(ctx, op, ncells, path)
            if os.path.exists(path):
                with open(path) as f:
                    tuned.update(json.load(f))
                sf.sf_load_tuning(ctx, path)
        if args.save_tuning:
            with open(args.save_tuning, "w") as f:
                json.dump(tuned, f, indent=1, sort_keys=True)
    torch.cuda.synchronize()

    def step(timers=None, it=0):
        for p in degrees:
            kap, u, y = bufs[p][it % len(bufs[p])]
            if timers is not None:
                timers[p][0].record(stream)
            sf.assemble_action(ctx, ops[p], ncells, V, kap, u, y, stream)
            if timers is not None:
                timers[p][1].record(stream)

    for it in range(args.warmup):
        step(None, it)
    torch.cuda.synchronize()
    assert sf.sf_check_errors(ctx) == 0

    ev = {p: [] for p in degrees}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for it in range(args.steps):
        timers = {p: (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for p in degrees}
        step(timers, it)
        for p in degrees:
            ev[p].append(timers[p])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = {p: float(np.median([a.elapsed_time(b) for a, b in ev[p]])) for p in degrees}
    ms_mean = {p: float(np.mean([a.elapsed_time(b) for a, b in ev[p]])) for p in degrees}

    glob = {p: (NCELL1 * p + 1) ** 3 for p in degrees}
    loc = {p: ncells * (p + 1) ** 3 for p in degrees}
    t_step = sum(ms.values()) / 1e3
    value = sum(glob.values()) / t_step / 1e9
    per_p = {}
    for p in degrees:
        t = ms[p] / 1e3
        gbs = action_bytes_per_cell(p) * ncells / t / 1e9
        tfl = action_flops_per_cell(p) * ncells / t / 1e12
        per_p[str(p)] = {"ms": round(ms[p], 4), "ms_mean": round(ms_mean[p], 4),
                         "gdofs_global": round(glob[p] / t / 1e9, 3),
                         "gdofs_local": round(loc[p] / t / 1e9, 3), "hbm_gbs": round(gbs, 1),
                         "hbm_frac": round(gbs / PEAK_HBM_GBS, 4), "fp64_tflops": round(tfl, 2),
                         "fp64_frac": round(tfl / PEAK_FP64_TFLOPS, 4),
                         "roof_frac": round(max(gbs / PEAK_HBM_GBS, tfl / PEAK_FP64_TFLOPS), 4)}
    dom = max(degrees, key=lambda p: ms[p])
    variant = int(tuned.get("gfx950|fam0|p%d|form1|nq%d|prec0|io0|standalone" % (dom, dom + 1), 0))
    roofline = roofline_of(dom, ms[dom], ncells, variant)

    mixed = None
    if args.mixed_degrees:
        mixed = mixed_leg(sf, ctx, V, bufs, ncells, [int(x) for x in args.mixed_degrees.split(",")], ms, glob,
                          args.steps, stream)

    legs = [x for x in args.legs.split(",") if x]
    copy_gbs = measured_copy_gbs()
    side = {}
    if "mass" in legs:
        side["mass_action"] = mass_leg(sf, ctx, V, bufs, ncells, degrees, glob, args.steps, stream)
    if "collocated" in legs:
        side["collocated_gll_laplace"] = mass_leg(sf, ctx, V, bufs, ncells, degrees, glob, args.steps, stream,
                                                  family="QGLL", form="LAPLACE")
    if "trilinear" in legs:
        side["trilinear_laplace"] = trilinear_leg(sf, V.shape[0], degrees, bufs, args.steps, stream)
    if "vq" in legs:
        side["vector_q"] = vq_leg(sf, ctx, V, degrees, args.steps, stream)
    if "svk" in legs:
        side["svk_hyperelastic"] = svk_leg(sf, ctx, V, degrees, args.steps, stream)
    if "global" in legs:
        side["global_action"] = global_leg(sf, ctx, V, bufs, degrees, glob, args.steps, stream)
    if "vec" in legs:
        side["vec_action"] = vec_leg(sf, ctx, args.steps, stream)
    if "matrix" in legs:
        side["element_matrix"] = matrix_leg(sf, ctx, V, degrees, stream)
    if "batch" in legs:
        side["batched"] = batch_leg(sf, ctx, stream)

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(degrees, bufs, V, glob, ncells, args.cpu_seconds, mixed)

    out = {
        "metric": "GDoF/s of Q_p Laplace action p=1..8; mixed-prec vs FP64 at <=1e-6 rel err",
        "value": round(value, 3), "unit": "GDoF/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(sum(ms.values()), 4), "wall_ms_per_step": round(wall / args.steps * 1e3, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (seeded box mesh, kappa U[0.5,2], u N(0,1))",
        "config": {"workload": "Q_p Laplace action, p=%s, 64^3 box cells, (p+1)^3 GL points, FP64"
                   % ",".join(map(str, degrees)), "ncells": ncells, "degrees": degrees},
        "roofline": roofline, "cpu_baseline": cpu, "per_p": per_p, "mixed_precision": mixed,
        "tuned_variants": {k.split("|", 1)[1]: v for k, v in tuned.items()},
        "measured_copy_gbs": round(copy_gbs, 1), "frac_vs_measured_copy": round(roofline["hbm_gbs"] / copy_gbs, 4),
        "legs": side,
    }
    if mixed:
        for row in mixed.values():
            row.pop("_sample_fp64", None)
            for r in row.values():
                if isinstance(r, dict):
                    r.pop("_sample", None)
    if args.calib_copy:
        a = torch.empty(1 << 27, dtype=torch.float64, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)  # reads and writes exactly 1 GiB
        torch.cuda.synchronize()
        out["calib_copy_bytes"] = 1 << 30
    print(json.dumps(out))
    ctx.close()


def tune_key(op, what):
    return "gfx950|fam%d|p%d|form%d|nq%d|prec%d|io%d|%s" % (op.family, op.degree, op.form, op.degree + 1,
                                                          op.precision, op.io_dtype, what)


def tuning_classes(sf, degrees, mixed_degrees, legs):
    """Every op class the run times whose kernel choice the autotuner makes, with the
    choice keys it records: the headline (stand-alone box kernel, batched tiles of
    actions and element matrices), the mass and collocated legs, the FP32 rows of the
    mixed-precision leg, the batched BF16 / BF16x3 tiles and the H(div) / H(curl)
    actions."""
    out = []
    for p in degrees:
        op = sf.make_op("Q", p, "LAPLACE")
        out.append((op, [tune_key(op, w) for w in ("standalone", "batch", "batch_matrix")]))
        if "mass" in legs:
            op = sf.make_op("Q", p, "MASS")
            out.append((op, [tune_key(op, "standalone")]))
        if "collocated" in legs:
            op = sf.make_op("QGLL", p, "LAPLACE")
            out.append((op, [tune_key(op, "standalone")]))
    for p in mixed_degrees:
        for io in ("f64", "f32"):
            op = sf.make_op("Q", p, "LAPLACE", precision="fp32", io=io)
            out.append((op, [tune_key(op, "standalone")]))
    if "batch" in legs:
        for p in range(2, 9):
            for prec in ("bf16", "bf16x3"):
                op = sf.make_op("Q", p, "LAPLACE", precision=prec)
                out.append((op, [tune_key(op, "batch")]))
    if "vec" in legs:
        for fam, form in (("NCF", "HDIV"), ("NCE", "HCURL")):
            for io in ("f64", "f32"):
                for k in range(1, 7):
                    op = sf.make_op(fam, k, form, io=io)
                    out.append((op, [tune_key(op, "standalone")]))
    return out


def roofline_of(p, ms, ncells, variant):
    """Roofline line of the degree-p Laplace launch: the fraction
    max(bytes / 8 TB/s, flops / 78.6 TFLOP/s) / t of the algorithmic bytes and
    flops per launch (the larger term names the bound: "hbm", or "alu" for the
    FP64 vector FMAs), both fractions beside it; t = the median launch time."""
    t = ms / 1e3
    nbytes = action_bytes_per_cell(p) * ncells
    nflops = action_flops_per_cell(p) * ncells
    gbs, tfl = nbytes / t / 1e9, nflops / t / 1e12
    hbm_frac, alu_frac = gbs / PEAK_HBM_GBS, tfl / PEAK_FP64_TFLOPS
    name = {3: "action_q_kernel", 6: "action_q_cell2_kernel"}.get(variant, "action_q_fast_kernel")
    kernel = "%s Q_%d Laplace FP64 (variant %d)" % (name, p, variant)
    common = {"traffic": recorded_traffic(p, variant), "kernel": kernel, "time_ms": round(ms, 4),
              "bytes_per_launch": nbytes, "flops_per_launch": nflops,
              "hbm_gbs": round(gbs, 1), "hbm_frac": round(hbm_frac, 4),
              "fp64_tflops": round(tfl, 2), "alu_frac": round(alu_frac, 4)}
    if alu_frac > hbm_frac:
        line = {"bound": "alu", "achieved": round(tfl, 2), "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                "frac": round(alu_frac, 4)}
    else:
        line = {"bound": "hbm", "achieved": round(gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": round(hbm_frac, 4)}
    line.update(common)
    return line


def source_digest():
    """SHA-256 over the sources of the headline kernels (the box-cell action, the
    general action that low degrees select, and the device building blocks they
    include): identifies the kernels a recorded counter profile was taken from;
    any change to them makes the record stale."""
    import hashlib

    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1711_02473_amd", "csrc")
    files = [os.path.join(csrc, f) for f in ("action_q_fast.hip", "action_box_body.inc", "action_q.hip",
                                             "action_q_body.inc", "sf_device.hpp")]
    for f in files:
        h.update(os.path.relpath(f, ROOT).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def recorded_traffic(p, variant):
    """HBM bytes per launch of the degree-p action kernel from the committed
    rocprofv3 counter record (FETCH_SIZE and WRITE_SIZE, each scaled by what
    the counter reads for a copy of known size), or None when there is no
    record for this degree, kernel variant and these sources."""
    path = os.path.join(ROOT, "profiles", "action_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    k = rec.get("kernels", {}).get(str(p))
    if rec.get("source_sha256") != source_digest() or not k or k.get("variant") != variant:
        return None
    return k.get("traffic_bytes")


def timed(fn, reps, stream):
    """Median milliseconds of fn() over reps launches, each bracketed by HIP events on `stream`."""
    import torch

    ts = []
    for it in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        fn(it)
        b.record(stream)
        ts.append((a, b))
    torch.cuda.synchronize()
    return float(np.median([a.elapsed_time(b) for a, b in ts]))


def measured_copy_gbs():
    """Device-to-device copy of 1 GiB (read + write = 2 GiB of traffic): the
    practical HBM rate next to the 8 TB/s specification."""
    import torch

    a = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    ms = timed(lambda it: b.copy_(a), 5, torch.cuda.current_stream())
    del a, b
    return 2.0 * (1 << 30) / (ms / 1e3) / 1e9


def mass_leg(sf, ctx, V, bufs, ncells, degrees, glob, reps, stream, family="Q", form="MASS"):
    """Q_p mass action (kappa per Gauss point) on the same 64^3 box mesh, FP64;
    HBM-bound at every p: bytes = 24 n^3 + 192 per cell.  With family QGLL and form
    LAPLACE: the collocated GLL Laplace action (B = I, six derivative contractions),
    same bytes."""
    import torch

    out = {}
    for p in degrees:
        op = sf.make_op(family, p, form)
        sets = bufs[p]
        y = torch.empty_like(sets[0][1])
        sf.assemble_action(ctx, op, ncells, V, sets[0][0], sets[0][1], y, stream)
        ms = timed(lambda it: sf.assemble_action(ctx, op, ncells, V, sets[it % len(sets)][0], sets[it % len(sets)][1],
                                                 y, stream), reps, stream)
        gbs = action_bytes_per_cell(p) * ncells / (ms / 1e3) / 1e9
        out[str(p)] = {"ms": round(ms, 4), "gdofs_global": round(glob[p] / (ms / 1e3) / 1e9, 3),
                       "hbm_gbs": round(gbs, 1), "hbm_frac": round(gbs / PEAK_HBM_GBS, 4)}
    assert sf.sf_check_errors(ctx) == 0
    return out


def trilinear_leg(sf, ncells, degrees, bufs, reps, stream):
    """Q_p Laplace action on general trilinear hexahedra (every vertex of a unit-ish
    cube moved by up to 0.15; a separate context with geometry SF_GEOM_TRILINEAR), the
    geometric factor computed at every Gauss point; same kappa and u as the headline.
    Bytes as the headline (24 n^3 + 192 per cell)."""
    import torch

    from paper_1711_02473_amd import synth

    c = sf.Context(0)
    sf.sf_set_geometry(c, "trilinear")
    Vt = torch.from_numpy(synth.trilinear_cells(ncells, 7)).cuda()
    out = {}
    for p in degrees:
        op = sf.make_op("Q", p, "LAPLACE")
        sets = bufs[p]
        y = torch.empty_like(sets[0][1])
        sf.assemble_action(c, op, ncells, Vt, sets[0][0], sets[0][1], y, stream)
        ms = timed(lambda it: sf.assemble_action(c, op, ncells, Vt, sets[it % len(sets)][0], sets[it % len(sets)][1],
                                                 y, stream), reps, stream)
        gbs = action_bytes_per_cell(p) * ncells / (ms / 1e3) / 1e9
        out[str(p)] = {"ms": round(ms, 4), "gdofs_local": round(ncells * (p + 1) ** 3 / (ms / 1e3) / 1e9, 3),
                       "hbm_gbs": round(gbs, 1), "hbm_frac": round(gbs / PEAK_HBM_GBS, 4)}
        del y
    assert sf.sf_check_errors(c) == 0
    c.close()
    return out


def vq_leg(sf, ctx, V, degrees, reps, stream):
    """Vector Q_p element (3 (p+1)^3 DOFs per cell): the vector Laplace action on the 64^3 box
    mesh (kappa per point U[0.5, 2], u N(0, 1), drawn on the GPU; algorithmic bytes per cell
    8 (6 n^3 + n^3) + 192), and its block-diagonal element matrices on the first cells (p = 1..4,
    at least 4096 cells and 400 MB of output; bytes written 8 (3 n^3)^2 per cell, of which the
    off-diagonal two thirds are the cleared buffer)."""
    import torch

    from paper_1711_02473_amd import synth

    ncells = V.shape[0]
    act, mat = {}, {}
    for p in degrees:
        n3 = (p + 1) ** 3
        op = sf.make_op("VQ", p, "LAPLACE")
        # input copies rotated so that every launch streams more than the last-level cache
        nrot = max(1, min(4, math.ceil(768e6 / (ncells * (8 * 7 * n3 + 192)))))
        sets = [(synth.device_kappa(ncells, n3, 3 + 10 * r, p), synth.device_displacements(ncells, 3 * n3, 3 + 10 * r, p)[1])
                for r in range(nrot)]
        y = torch.empty_like(sets[0][1])
        sf.assemble_action(ctx, op, ncells, V, sets[0][0], sets[0][1], y, stream)
        ms = timed(lambda it: sf.assemble_action(ctx, op, ncells, V, sets[it % nrot][0], sets[it % nrot][1], y, stream),
                   reps, stream)
        gbs = ncells * (8 * 7 * n3 + 192) / (ms / 1e3) / 1e9
        act[str(p)] = {"ms": round(ms, 4), "gdofs_local": round(ncells * 3 * n3 / (ms / 1e3) / 1e9, 3),
                       "hbm_gbs": round(gbs, 1), "hbm_frac": round(gbs / PEAK_HBM_GBS, 4)}
        del sets, y
        if p <= 4:
            # at least 4096 cells and 400 MB of matrices, so that the writes leave the last-level cache
            nm = int(min(ncells, max(4096, math.ceil(400e6 / (8 * (3 * n3) ** 2)))))
            A = torch.empty((nm, 3 * n3, 3 * n3), dtype=torch.float64, device="cuda")
            kap = synth.device_kappa(nm, n3, 3, p)
            sf.assemble_element_matrix(ctx, op, nm, V[:nm], kap, A, stream)
            ms = timed(lambda it: sf.assemble_element_matrix(ctx, op, nm, V[:nm], kap, A, stream), reps, stream)
            gbs = nm * 8 * (3 * n3) ** 2 / (ms / 1e3) / 1e9
            mat[str(p)] = {"ms": round(ms, 4), "cells": nm, "hbm_gbs": round(gbs, 1),
                           "hbm_frac": round(gbs / PEAK_HBM_GBS, 4)}
            del A, kap
    assert sf.sf_check_errors(ctx) == 0
    return {"laplace_action": act, "laplace_element_matrix": mat}


def svk_leg(sf, ctx, V, degrees, reps, stream, lam=1.3, mu=0.8):
    """Saint Venant-Kirchhoff hyperelastic operator on the vector Q_p element (3 (p+1)^3 DOFs
    per cell), 64^3 box cells: the linearised residual at u0 applied to du (SF_SVK), u0 =
    0.01 N(0,1), du N(0,1), drawn on the GPU.  Algorithmic bytes per cell: u0, du and y,
    3 n^3 FP64 each, plus 192 B of vertices.  Inputs are rotated between two copies when
    one set would fit the 256 MB last-level cache."""
    import torch

    from paper_1711_02473_amd import synth

    ncells = V.shape[0]
    out = {}
    for p in degrees:
        n3 = (p + 1) ** 3
        op = sf.make_op("Q", p, "SVK", alpha=lam, beta=mu)
        sets = [synth.device_displacements(ncells, 3 * n3, 1, p)]
        if ncells * 3 * n3 * 8 * 3 < (1 << 30):
            sets.append(synth.device_displacements(ncells, 3 * n3, 2, p))
        y = torch.empty_like(sets[0][1])
        sf.assemble_action(ctx, op, ncells, V, sets[0][0], sets[0][1], y, stream)
        ms = timed(lambda it: sf.assemble_action(ctx, op, ncells, V, sets[it % len(sets)][0], sets[it % len(sets)][1],
                                                 y, stream), reps, stream)
        nbytes = ncells * (3 * 3 * n3 * 8 + 192)
        gbs = nbytes / (ms / 1e3) / 1e9
        out[str(p)] = {"ms": round(ms, 4), "gdofs_local": round(ncells * 3 * n3 / (ms / 1e3) / 1e9, 3),
                       "gdofs_global": round(3 * (64 * p + 1) ** 3 / (ms / 1e3) / 1e9, 3),
                       "hbm_gbs": round(gbs, 1), "hbm_frac": round(gbs / PEAK_HBM_GBS, 4)}
        del sets, y
        if True:
            # element matrices of the linearised residual (left-hand-side assembly) on the first
            # cells: at least 4096 cells and 400 MB of output, at most 4 GiB of output;
            # algorithmic work per cell: 9 blocks x 2 (4 n^7 + 18 n^6 + 9 n^5) flops
            n = p + 1
            cb = 8 * (3 * n3) ** 2
            nm = int(min(ncells, (4 << 30) // cb, max(4096, math.ceil(400e6 / cb))))
            u0 = synth.device_displacements(nm, 3 * n3, 1, p)[0]
            A = torch.empty((nm, 3 * n3, 3 * n3), dtype=torch.float64, device="cuda")
            sf.assemble_element_matrix(ctx, op, nm, V[:nm], u0, A, stream)
            ms = timed(lambda it: sf.assemble_element_matrix(ctx, op, nm, V[:nm], u0, A, stream), reps, stream)
            gbs = nm * 8 * (3 * n3) ** 2 / (ms / 1e3) / 1e9
            fl = nm * 18 * (4 * n ** 7 + 18 * n ** 6 + 9 * n ** 5)
            out["matrix_%d" % p] = {"ms": round(ms, 4), "cells": nm, "hbm_gbs": round(gbs, 1),
                                    "hbm_frac": round(gbs / PEAK_HBM_GBS, 4),
                                    "fp64_tflops": round(fl / (ms / 1e3) / 1e12, 2)}
            del A, u0
    assert sf.sf_check_errors(ctx) == 0
    return out


def global_leg(sf, ctx, V, bufs, degrees, glob, reps, stream, n1=NCELL1):
    """The assembled C0 Q_p Laplace action on global vectors ((64p+1)^3 DOFs): each cell
    gathers its local DOFs, applies the box-cell action and adds its result with FP64
    atomics.  Algorithmic bytes: the global u and y once each (8 B per global DOF each;
    the clearing of y not counted), kappa (8 n^3 per cell) and the vertices."""
    import torch

    out = {}
    ncells = n1 ** 3
    for p in degrees:
        op = sf.make_op("Q", p, "LAPLACE")
        ng = glob[p]
        bts = 16 * ng + (8 * (p + 1) ** 3 + 192) * ncells
        # (vertices, kappa, u) copies rotated so that every launch streams more than the
        # last-level cache (the vertex array alone is 50 MB)
        nrot = max(2, min(6, math.ceil(768e6 / bts)))
        g = torch.Generator(device="cuda")
        g.manual_seed(171102473 * 1000 + 230 + p)
        ug = torch.randn((nrot, ng), generator=g, device="cuda", dtype=torch.float64)
        sets = [(V if r == 0 else V.clone(), bufs[p][r % len(bufs[p])][0], ug[r]) for r in range(nrot)]
        y = torch.empty((ng,), device="cuda", dtype=torch.float64)
        sf.assemble_action_global_q(ctx, op, n1, n1, n1, V, sets[0][1], ug[0], y, stream)
        ms = timed(lambda it: sf.assemble_action_global_q(ctx, op, n1, n1, n1, sets[it % nrot][0], sets[it % nrot][1],
                                                          sets[it % nrot][2], y, stream), reps, stream)
        out[str(p)] = {"ms": round(ms, 4), "gdofs_global": round(ng / (ms / 1e3) / 1e9, 3),
                       "hbm_gbs": round(bts / (ms / 1e3) / 1e9, 1), "hbm_frac": round(bts / (ms / 1e3) / 1e9 / PEAK_HBM_GBS, 4)}
        del ug, y, sets
    assert sf.sf_check_errors(ctx) == 0
    return out


def vec_leg(sf, ctx, reps, stream, n1=48):
    """H(div) NCF_k (alpha mass + beta div-div) and H(curl) NCE_k (alpha mass +
    beta curl-curl) actions, k = 1..6, alpha = beta = 1, kappa = 1, on n1^3 box
    cells with FP64 and FP32 storage.  Bytes per cell: u + y + 192 (vertices)."""
    import torch

    from paper_1711_02473_amd import synth

    ncells = n1 ** 3
    V = torch.from_numpy(synth.box_mesh(n1, n1, n1, 4)).cuda()
    g = torch.Generator(device="cuda")
    g.manual_seed(synth.SEED * 100 + 40)
    out = {}
    for fam, form in (("NCF", "HDIV"), ("NCE", "HCURL")):
        for io, tdt, isz in (("f64", torch.float64, 8), ("f32", torch.float32, 4)):
            for k in range(1, 7):
                op = sf.make_op(fam, k, form, io=io)
                nd, _ = sf.sf_element_dims(op)
                u = torch.randn((2, ncells, nd), generator=g, device="cuda", dtype=torch.float64).to(tdt)
                y = torch.empty((ncells, nd), device="cuda", dtype=tdt)
                sf.assemble_action(ctx, op, ncells, V, None, u[0], y, stream)
                ms = timed(lambda it: sf.assemble_action(ctx, op, ncells, V, None, u[it % 2], y, stream), reps, stream)
                gbs = (2 * nd * isz + 192) * ncells / (ms / 1e3) / 1e9
                out["%s%d_%s" % (fam, k, io)] = {"ms": round(ms, 4), "gdofs_local": round(ncells * nd / (ms / 1e3) / 1e9, 3),
                                                 "hbm_gbs": round(gbs, 1), "hbm_frac": round(gbs / PEAK_HBM_GBS, 4)}
                del u, y
    assert sf.sf_check_errors(ctx) == 0
    return out


def matrix_leg(sf, ctx, V, degrees, stream, budget_bytes=4 << 30):
    """Q_p Laplace element matrices (kappa per Gauss point), FP64, on the first
    cells of the 64^3 mesh: as many cells as fit in a 4 GiB output.  Bound by
    the HBM writes of the matrices: bytes = 8 n^6 + 8 n^3 + 192 per cell."""
    import torch

    from paper_1711_02473_amd import synth

    out = {}
    for p in degrees:
        n3 = (p + 1) ** 3
        nc = matrix_leg_cells(p, V.shape[0], budget_bytes)
        kap = synth.device_kappa(nc, n3, 2, p)
        # output buffers rotated so that the written matrices leave the last-level cache
        nrot = max(1, min(3, math.ceil(600e6 / (8 * n3 * n3 * nc))))
        As = [torch.empty((nc, n3, n3), device="cuda", dtype=torch.float64) for _ in range(nrot)]
        op = sf.make_op("Q", p, "LAPLACE")
        sf.assemble_element_matrix(ctx, op, nc, V, kap, As[0], stream)
        ms = timed(lambda it: sf.assemble_element_matrix(ctx, op, nc, V, kap, As[it % nrot], stream), 10, stream)
        bts = (8 * n3 * n3 + 8 * n3 + 192) * nc
        out[str(p)] = {"cells": nc, "ms": round(ms, 4), "cells_per_s": round(nc / (ms / 1e3), 1),
                       "hbm_gbs": round(bts / (ms / 1e3) / 1e9, 1),
                       "hbm_frac": round(bts / (ms / 1e3) / 1e9 / PEAK_HBM_GBS, 4)}
        # the final contraction on MFMA (BF16 single term, BF16 x3 split), FP32 accumulation,
        # FP64 output; error against the FP64 matrices of the same cells
        sf.assemble_element_matrix(ctx, op, nc, V, kap, As[0], stream)
        Am = torch.empty_like(As[0])
        errs = {}
        for prec in ("bf16", "bf16x3"):
            sf.assemble_element_matrix(ctx, sf.make_op("Q", p, "LAPLACE", precision=prec), nc, V, kap, Am, stream)
            errs[prec] = float(torch.linalg.vector_norm(Am - As[0]) / torch.linalg.vector_norm(As[0]))
        del Am
        for prec in ("bf16", "bf16x3"):
            opm = sf.make_op("Q", p, "LAPLACE", precision=prec)
            err = errs[prec]
            msm = timed(lambda it: sf.assemble_element_matrix(ctx, opm, nc, V, kap, As[it % nrot], stream), 10,
                        stream)
            out[str(p)][prec] = {"ms": round(msm, 4), "hbm_frac": round(bts / (msm / 1e3) / 1e9 / PEAK_HBM_GBS, 4),
                                 "speedup_vs_fp64": round(ms / msm, 3), "rel_l2_vs_fp64_gpu": float("%.3e" % err)}
        del kap, As
    assert sf.sf_check_errors(ctx) == 0
    return out


def matrix_leg_cells(p, ncells, budget_bytes=4 << 30):
    """Cells of the element-matrix leg: the first ones of the mesh, as many as fit."""
    n3 = (p + 1) ** 3
    return int(min(ncells, budget_bytes // (8 * n3 * n3)))


def batch_leg(sf, ctx, stream, nmeshes=2048, arena_bytes=2 << 30):
    """The batched workload: 2048 box meshes of n_m^3 cells (n_m uniform in
    4..16) and degree p_m (uniform in 2..8), Laplace action with kappa per Gauss
    point in one persistent launch replayed from a hipGraph, FP64 and with
    BF16 / BF16 x3 contractions (error against the FP64 batch), then the same
    meshes' element matrices together with the actions in one launch (FP64, and
    BF16 with the matrices' final contraction on MFMA), matrices written into a
    per-degree arena of 2 GiB cycled per job."""
    import torch

    from paper_1711_02473_amd import synth

    wl = synth.batched_workload(nmeshes)
    verts = [synth.batch_mesh(m, n) for m, (n, p) in enumerate(wl)]
    ncell = [n ** 3 for n, p in wl]
    off = np.concatenate([[0], np.cumsum(ncell)])
    V = torch.from_numpy(np.concatenate(verts)).cuda()
    del verts
    degs = sorted(set(p for n, p in wl))
    # per degree: one slab of kappa, u, y holding that degree's meshes back to back
    slabs, slab_off = synth.batched_device_inputs(wl)
    kap, u, y, yb = {}, {}, {}, {}
    for p in degs:
        kap[p], u[p] = slabs[p]
        y[p] = torch.empty_like(u[p])
        yb[p] = torch.empty_like(u[p])
    arena = {p: torch.empty(arena_bytes // 8, device="cuda", dtype=torch.float64) for p in degs}
    esz = 8

    def jobs(precision, ybuf, matrices=False, actions=True):
        js = []
        for m, (n, p) in enumerate(wl):
            n3 = (p + 1) ** 3
            vp = V.data_ptr() + int(off[m]) * 24 * esz
            kp = kap[p].data_ptr() + slab_off[m] * n3 * esz
            if actions:
                js.append(sf.make_job(sf.make_op("Q", p, "LAPLACE", precision=precision), ncell[m], vp, kp,
                                      u[p].data_ptr() + slab_off[m] * n3 * esz,
                                      ybuf[p].data_ptr() + slab_off[m] * n3 * esz))
            if matrices:
                js.append(sf.make_job(sf.make_op("Q", p, "LAPLACE", precision=precision), ncell[m], vp, kp,
                                      A=arena[p], A_arena_cells=max(1, arena_bytes // (esz * n3 * n3))))
        return js

    loc = sum(ncell[m] * (p + 1) ** 3 for m, (n, p) in enumerate(wl))
    act_bytes = sum(ncell[m] * (24 * (p + 1) ** 3 + 192) for m, (n, p) in enumerate(wl))
    mat_bytes = sum(ncell[m] * (8 * (p + 1) ** 6 + 8 * (p + 1) ** 3 + 192) for m, (n, p) in enumerate(wl))
    out = {"meshes": nmeshes, "cells": int(off[-1]), "local_dofs": int(loc)}
    for prec, yy in (("fp64", y), ("bf16", yb), ("bf16x3", yb)):
        b = sf.Batch(ctx, jobs(prec, yy))
        b.launch(stream)
        ms = timed(lambda it: b.launch(stream), 5, stream)
        row = {"ms": round(ms, 4), "gdofs_local": round(loc / (ms / 1e3) / 1e9, 3),
               "hbm_gbs": round(act_bytes / (ms / 1e3) / 1e9, 1), "tiles_workgroups": list(b.info())}
        if prec != "fp64":
            num = sum(float(torch.linalg.vector_norm(yb[p] - y[p]) ** 2) for p in degs)
            den = sum(float(torch.linalg.vector_norm(y[p]) ** 2) for p in degs)
            row["rel_l2_vs_fp64_gpu"] = float("%.3e" % (num / den) ** 0.5)
        out["action_" + prec] = row
        b.close()
    for prec, yy in (("fp64", y), ("bf16", yb)):
        b = sf.Batch(ctx, jobs(prec, yy, matrices=True, actions=True))
        b.launch(stream)
        ms = timed(lambda it: b.launch(stream), 3, stream)
        out["action_and_matrix_" + prec] = {
            "ms": round(ms, 3), "hbm_gbs": round((act_bytes + mat_bytes) / (ms / 1e3) / 1e9, 1),
            "hbm_frac": round((act_bytes + mat_bytes) / (ms / 1e3) / 1e9 / PEAK_HBM_GBS, 4),
            "matrix_bytes": int(mat_bytes), "tiles_workgroups": list(b.info())}
        b.close()
    assert sf.sf_check_errors(ctx) == 0
    del kap, u, y, yb, arena
    return out


def mixed_leg(sf, ctx, V, bufs, ncells, degrees, ms64, glob, reps, stream):
    """Laplace action with lower-precision contractions (FP32 on the vector
    ALUs; BF16 / FP16 single term and BF16 x3 split on MFMA: the dense
    Kronecker kernels, one n^3 x n^3 product per component at p <= 3 and plane x
    axis-0 products at p = 4..8, BF16 x3 at p = 8 on the sum-factorised MFMA
    kernel), geometry and pointwise factors in FP64, against the FP64 GPU path on
    the same inputs: rate, algorithmic HBM GB/s (u, y, kappa at the row's storage
    width plus the vertices), speed-up and relative L2 difference.  Rows without a suffix keep FP64
    storage; rows "_f32io" also store kappa, u and y in FP32 (the inputs are
    rounded once, outside the timed region, and the error is measured against
    the FP64 result of the unrounded inputs, so it includes that rounding).
    "best_le_1e-6" names, per degree, the fastest row within 1e-6.  The outputs of
    every row on MIXED_SAMPLE cells are kept (key "_sample") for the CPU-baseline
    leg, which adds each row's error against the oracle on those cells."""
    import torch

    modes = [("fp32", "f64"), ("bf16", "f64"), ("fp16", "f64"), ("bf16x3", "f64"), ("fp32", "f32"),
             ("bf16x3", "f32")]
    out = {}
    for p in degrees:
        if p not in bufs:
            continue
        kap, u, y = bufs[p][0]
        ref = torch.empty_like(y)
        sf.assemble_action(ctx, sf.make_op("Q", p, "LAPLACE"), ncells, V, kap, u, ref, stream)
        row = {}
        for mode, io in modes:
            op = sf.make_op("Q", p, "LAPLACE", precision=mode, io=io)
            if io == "f32":
                sets = [(k2.float(), u2.float()) for k2, u2, _ in bufs[p]]
                ym = torch.empty(y.shape, dtype=torch.float32, device=y.device)
            else:
                sets = [(k2, u2) for k2, u2, _ in bufs[p]]
                ym = torch.empty_like(y)
            sf.assemble_action(ctx, op, ncells, V, sets[0][0], sets[0][1], ym, stream)
            torch.cuda.synchronize()
            ts = []
            for it in range(reps):
                k2, u2 = sets[it % len(sets)]
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record(stream)
                sf.assemble_action(ctx, op, ncells, V, k2, u2, ym, stream)
                b.record(stream)
                ts.append((a, b))
            torch.cuda.synchronize()
            sf.assemble_action(ctx, op, ncells, V, sets[0][0], sets[0][1], ym, stream)
            err = float(torch.linalg.vector_norm(ym.double() - ref) / torch.linalg.vector_norm(ref))
            t = float(np.median([a.elapsed_time(b) for a, b in ts]))
            key = mode if io == "f64" else mode + "_f32io"
            gbs = action_bytes_per_cell(p, 8 if io == "f64" else 4) * ncells / (t / 1e3) / 1e9
            row[key] = {"ms": round(t, 4), "gdofs_global": round(glob[p] / (t / 1e3) / 1e9, 3),
                        "hbm_gbs": round(gbs, 1), "hbm_frac": round(gbs / PEAK_HBM_GBS, 4),
                        "speedup_vs_fp64": round(ms64[p] / t, 3), "rel_l2_vs_fp64_gpu": float("%.3e" % err),
                        "_sample": ym[sample_idx(ncells)].double().cpu().numpy()}
            del sets, ym
        ok = {k: v for k, v in row.items() if v["rel_l2_vs_fp64_gpu"] <= 1e-6}
        row["_sample_fp64"] = ref[sample_idx(ncells)].cpu().numpy()
        if ok:
            best = max(ok, key=lambda k: ok[k]["speedup_vs_fp64"])
            row["best_le_1e-6"] = {"mode": best, "speedup_vs_fp64": ok[best]["speedup_vs_fp64"]}
        out[str(p)] = row
    return out


MIXED_SAMPLE = 24


def sample_idx(ncells, n=MIXED_SAMPLE):
    """Evenly spaced cells, first and last included (the mixed-precision sample)."""
    import torch
    return torch.from_numpy(np.linspace(0, ncells - 1, n).astype(np.int64)).cuda()


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(degrees, bufs, V, glob, ncells, budget, mixed=None):
    """The FP64 oracle (direct quadrature) on a bounded, evenly spaced sample of
    the same cells, on all host threads and on one thread; its rate is
    extrapolated to the whole mesh.  The sampled GPU outputs are compared with
    it on the way, the FP64 path and every mixed-precision row (whose outputs
    on MIXED_SAMPLE cells the mixed leg kept)."""
    import oracle
    import torch

    Vh = V.cpu().numpy()
    per = budget / len(degrees)
    t_total = 0.0
    errs = {}
    samples = {}
    for p in degrees:
        kap, u, y = bufs[p][0]
        n = 8
        while True:
            idx = (np.arange(n) * (ncells // n)).astype(np.int64)
            it = torch.from_numpy(idx).cuda()
            uh, kh, yh = u[it].cpu().numpy(), kap[it].cpu().numpy(), y[it].cpu().numpy()
            t0 = time.perf_counter()
            ref = oracle.action("Q", p, "LAPLACE", Vh[idx], uh, kappa=kh)
            dt = time.perf_counter() - t0
            if dt * 4 > per or n >= ncells // 4:
                break
            n *= 4
        t_total += dt * ncells / n
        errs[str(p)] = float(np.linalg.norm(yh - ref) / np.linalg.norm(ref))
        samples[str(p)] = n
    cores = oracle.num_threads()
    value = sum(glob[p] for p in degrees) / t_total / 1e9
    # one thread, on a sixteenth of each degree's sample (at least 8 cells)
    t1 = 0.0
    samples1 = {}
    oracle.set_num_threads(1)
    try:
        for p in degrees:
            kap, u, _ = bufs[p][0]
            n = max(8, samples[str(p)] // 16)
            idx = (np.arange(n) * (ncells // n)).astype(np.int64)
            it = torch.from_numpy(idx).cuda()
            uh, kh = u[it].cpu().numpy(), kap[it].cpu().numpy()
            t0 = time.perf_counter()
            oracle.action("Q", p, "LAPLACE", Vh[idx], uh, kappa=kh)
            t1 += (time.perf_counter() - t0) * ncells / n
            samples1[str(p)] = n
    finally:
        oracle.set_num_threads(cores)
    out = {"value": round(value, 6), "unit": "GDoF/s", "cores": cores, "kind": "oracle",
           "sample": "evenly spaced cells per degree %s of %d, extrapolated to the full mesh" % (samples, ncells),
           "cpu_model": cpu_model(),
           "value_1thread": round(sum(glob[p] for p in degrees) / t1 / 1e9, 7),
           "sample_1thread": "evenly spaced cells per degree %s, extrapolated" % samples1,
           "sample_rel_err_vs_gpu": errs}
    if mixed:
        # each mixed-precision row's error against the oracle on the kept sample cells
        idx = sample_idx(ncells).cpu().numpy()
        for p, row in mixed.items():
            pp = int(p)
            kap, u, _ = bufs[pp][0]
            it = torch.from_numpy(idx).cuda()
            ref = oracle.action("Q", pp, "LAPLACE", Vh[idx], u[it].cpu().numpy(), kappa=kap[it].cpu().numpy())
            nr = np.linalg.norm(ref)
            for key, r in row.items():
                if isinstance(r, dict) and "_sample" in r:
                    r["rel_l2_vs_oracle_sampled"] = float("%.3e" % (np.linalg.norm(r["_sample"] - ref) / nr))
            if "_sample_fp64" in row:
                row["fp64_rel_l2_vs_oracle_sampled"] = float("%.3e" % (np.linalg.norm(row["_sample_fp64"] - ref) / nr))
    return out


if __name__ == "__main__":
    main()
