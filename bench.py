#!/usr/bin/env python3
"""Throughput of the P-SPIR system-matrix hot path on one MI355X.

One step = one pass of the whole path over one synthetic input:
  build_psf_sysmat (count + fill phases: CSR of A^T, every voxel of the image;
  the 3D image is built in ranges of the library's voxel order, each range's
  CSR overwriting the last), project_fwd (y = A x on the fly) and project_adj
  (A^T y on the fly).
Prints ONE JSON line.  ``value`` is system-matrix elements (CSR non-zeros)
produced per second of the build; the same line carries the forward+adjoint
projection rate in LORs/s, a roofline object for the dominant kernel (timed
with HIP events around its launches, on the stream it runs on), the error of
each precision form against the FP64 oracle on sampled voxels, and the FP64
oracle timed on the host cores.

Workloads (all inputs seeded and synthetic, resident in HBM before timing):
  cyl3d_full   3D scanner of 32 blocks x 12 x 12 crystals (2 x 2 x 15 mm),
               4 block rings, faces at 130 mm; the whole 128 x 128 x 96 image
               (1 mm voxels); analytic 61x61x4x4x5x5 table; all non-zeros kept.
  cyl3d_sub16  the same scanner, the central 16 x 16 x 16 voxels only.
  ring2d_64    2D ring of 16 blocks x 8 crystals, faces at 65 mm; 64 x 64 image;
               61 x 4 x 5 table; CSR threshold 1e-6.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

T_START = time.perf_counter()
WALL_BUDGET_S = 520.0        # extras after the timed steps run only while the whole run stays under this

HBM_PEAK_GBS = 8000.0        # MI355X HBM3E
FP32_MATRIX_TFLOPS = 157.3   # MI355X dense FP32 matrix cores
BF16_MATRIX_TFLOPS = 2500.0  # MI355X dense BF16 matrix cores
PREC_NAMES = ["fp32", "bf16", "bf16x2"]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=None)
    ap.add_argument("--workload", default="cyl3d_full", choices=["cyl3d_full", "cyl3d_sub16", "ring2d_64"])
    ap.add_argument("--precision", type=int, default=0, help="0 FP32 plain, 1 BF16, 2 BF16 hi/lo")
    ap.add_argument("--slab", type=int, default=16384, help="voxels per build range of the full 3D image")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra-rows", action="store_true",
                    help="skip the rows timed after the steps (table gradient, list mode, precision forms), e.g. "
                         "under a profiler, so that its kernel mix is the timed step's")
    ap.add_argument("--copy-probe", action="store_true",
                    help="first copy 1 GiB on the device (a kernel of known traffic, to scale PMC byte counters)")
    return ap.parse_args()


def log(msg):
    print(f"[bench] {time.perf_counter() - T_START:7.1f} s  {msg}", file=sys.stderr, flush=True)


def kernel_source_digest():
    """SHA-256 of the 3D kernel sources: a traffic figure is reported only for the sources it was measured on."""
    h = hashlib.sha256()
    for f in ("cyl3d.hip", "common.hpp"):
        with open(os.path.join(ROOT, "paper_1607_06170_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(kernel_file):
    """HBM bytes per launch from a committed rocprofv3 --pmc summary (FETCH_SIZE, WRITE_SIZE scaled by a
    copy kernel of known size), or None when the kernel sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", kernel_file)
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if kv.get("source_sha256") != kernel_source_digest():
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def workload(name):
    from paper_1607_06170_amd import synth
    if name == "cyl3d_full":
        cfg = dict(synth.CFG_3D)
        desc = ("3D: 32 blocks x 12x12 LYSO crystals (2x2x15 mm), 4 block rings (48 crystal rings), faces at "
                "130 mm; the whole 128x128x96 image of 1 mm voxels (1,572,864 voxels); analytic 61x61x4x4x5x5 "
                "table; all non-zeros kept; matrix built in ranges of the voxel order, each range's CSR "
                "overwriting the last")
        return cfg, dict(workload=desc, mode3d=True, full=True, batch=1, steps=2, warmup=1)
    if name == "cyl3d_sub16":
        cfg = dict(synth.CFG_3D, nx=16, ny=16, nz=16)
        desc = ("3D: the same scanner; the central 16x16x16 voxels (1 mm) of the 128x128x96 image; analytic "
                "61x61x4x4x5x5 table; all non-zeros kept")
        return cfg, dict(workload=desc, mode3d=True, full=False, batch=1, steps=3, warmup=1)
    cfg = dict(synth.CFG_2D)
    desc = ("2D ring: 16 blocks x 8 LYSO crystals (2 mm, 15 mm deep), faces at 65 mm; 64x64 image of 1 mm "
            "voxels; 61 x 4 x 5 table; threshold 1e-6")
    return cfg, dict(workload=desc, mode3d=False, full=False, batch=1, steps=20, warmup=3)


def phantom(cfg, meta):
    from paper_1607_06170_amd import synth
    if meta["mode3d"]:
        full = dict(cfg, nx=128, ny=128, nz=96)
        img = synth.phantom_blobs(full, seed=2).reshape(96, 128, 128)
        if not meta["full"]:
            img = img[40:56, 56:72, 56:72]   # the central 16^3 voxels
        return np.ascontiguousarray(img.reshape(1, -1))
    return synth.phantom_uniform(cfg, seed=1, batch=meta["batch"])


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "bench.py runs on one GPU only (--gpus 1): sharding voxels across GPUs, "
                                   "with one all-reduce of the sinogram, is not implemented"}))
        sys.exit(2)
    import torch
    from paper_1607_06170_amd import Scanner

    cfg, meta = workload(args.workload)
    steps = args.steps if args.steps is not None else meta["steps"]
    warmup = args.warmup if args.warmup is not None else meta["warmup"]
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    if args.copy_probe:
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)   # 1 GiB read, 1 GiB written per copy
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    sc = Scanner(cfg, mode3d=meta["mode3d"])
    tab = sc.build_table(cfg["n_rows"], cfg["n_sub"], cfg["step_deg"])
    x_np = phantom(cfg, meta)
    x = torch.tensor(x_np, dtype=torch.float32, device=dev)
    thr = cfg["threshold"]
    prec = args.precision
    ones = torch.ones(1, sc.n_voxels, device=dev)
    lors = int((sc.project_fwd(tab, ones) > 0).sum().item())   # bins with sensitivity > 0
    del ones
    torch.cuda.synchronize()
    full = meta["full"]
    slabs = [(v, min(v + args.slab, sc.n_voxels)) for v in range(0, sc.n_voxels, args.slab)] if full \
        else [(0, sc.n_voxels)]

    ev = lambda: torch.cuda.Event(enable_timing=True)
    rec = dict(build=[], fwd=[], adj=[], nnz=0, tiles=0, vtiles=0)

    def step(record):
        e0, e1, e2, e3 = ev(), ev(), ev(), ev()
        e0.record()
        # tile counters of each call (each build phase): copied on the device, in stream order, read after
        # the step; a fill phase that copies the rows its count phase staged contracts nothing
        h_build = [] if meta["mode3d"] and record else None
        nnz = 0
        for vb, ve in slabs:
            rp, col, val = sc.build_psf_sysmat(tab, threshold=thr, vox_begin=vb, vox_end=ve, precision=prec,
                                               counters=h_build, class_order=full)
            nnz += int(col.numel())
            del rp, col, val
        e1.record()
        y = sc.project_fwd(tab, x, precision=prec)
        e2.record()
        h_fwd = sc.header_counters() if meta["mode3d"] and record else None
        xb = sc.project_adj(tab, y, precision=prec)
        e3.record()
        if record:
            torch.cuda.synchronize()
            h_adj = sc.header_counters() if meta["mode3d"] else None
            t_build, v_build = (sum(c) for c in zip(*[sc.read_counters(h) for h in h_build])) if h_build \
                else (0, 0)
            t_fwd, v_fwd = sc.read_counters(h_fwd)
            t_adj, v_adj = sc.read_counters(h_adj)
            rec["build"].append(e0.elapsed_time(e1))
            rec["fwd"].append(e1.elapsed_time(e2))
            rec["adj"].append(e2.elapsed_time(e3))
            rec["nnz"] += nnz
            rec["tiles"] += t_build + t_fwd + t_adj
            rec["vtiles"] += v_build + v_fwd + v_adj
        return y, xb

    log(f"workload {args.workload}: {sc.n_voxels} voxels, {sc.n_bins} bins, {len(slabs)} build ranges; "
        f"warmup {warmup}, steps {steps}")
    for i in range(warmup):
        step(False)
        torch.cuda.synchronize()
        log(f"warmup step {i + 1} done")
    torch.cuda.synchronize()
    sc.profile_start()
    t0 = time.perf_counter()
    last = [None, None]
    for i in range(steps):
        last[:] = step(True)
        log(f"step {i + 1}: build {rec['build'][-1]:.1f} ms, fwd {rec['fwd'][-1]:.1f} ms, adj {rec['adj'][-1]:.1f} ms")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    prof = sc.profile_stop()
    k_ms, k_launches = prof["contraction"]
    g_ms, g_launches = prof["geometry"]

    build_s = sum(rec["build"]) / 1e3
    proj_s = (sum(rec["fwd"]) + sum(rec["adj"])) / 1e3
    nnz = rec["nnz"] // steps
    out = {
        "metric": "PSF sysmat elements/s; fwd+adjoint projection LORs/s at stated rel-err vs FP64",
        "value": rec["nnz"] / build_s,
        "unit": "elements/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": 1e3 * wall / steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if prec == 0 else PREC_NAMES[prec],
        "data": "synthetic (seeded blob phantom, analytic response table)",
        "config": {"workload": meta["workload"], "voxels": sc.n_voxels, "bins": sc.n_bins,
                   "batch": meta["batch"], "nnz": nnz, "lors": lors, "build_ranges": len(slabs)},
        "fwd_adj_lors_per_s": lors * meta["batch"] * steps / proj_s,
        "build_ms": float(np.mean(rec["build"])), "fwd_ms": float(np.mean(rec["fwd"])),
        "adj_ms": float(np.mean(rec["adj"])),
    }
    avg_ms = k_ms / max(k_launches, 1)
    if meta["mode3d"]:
        K = cfg["n_sub"] ** 2
        flops_tile = 2 * (K * K * 25 + 25 * K * 25)   # X = W V, then T = U^T X (unpadded): 32 800 for P = 4
        tiles_per_launch = rec["tiles"] / max(k_launches, 1)
        vtiles_per_launch = rec["vtiles"] / max(k_launches, 1)
        executed = tiles_per_launch * flops_tile / (avg_ms * 1e-3) / 1e12
        amortised = vtiles_per_launch * flops_tile / (avg_ms * 1e-3) / 1e12
        peak = [FP32_MATRIX_TFLOPS, BF16_MATRIX_TFLOPS, BF16_MATRIX_TFLOPS][prec]
        traffic = measured_traffic(f"k_cyl3d_mma.{args.workload}.{PREC_NAMES[prec]}.pmc.txt")
        out["roofline"] = {
            "bound": "mfma", "achieved": executed, "peak": peak, "unit": "TFLOP/s", "frac": executed / peak,
            "traffic": traffic,
            "kernel": "k_cyl3d_mma (tile contraction T = U^T (W V) on matrix cores, "
                      + ["FP32", "BF16", "BF16 hi/lo"][prec] + ", and its emission; all modes)",
            "avg_launch_ms": avg_ms, "launches": k_launches, "flops_per_tile": flops_tile,
            "tiles_contracted_per_launch": tiles_per_launch,
            "note": "achieved counts the tiles the kernel contracts; each also serves the other voxels of its "
                    "symmetry class (below), whose work a voxel-by-voxel method would repeat",
            "voxel_tiles_per_launch": vtiles_per_launch,
            "symmetry_amortised_tflops": amortised}
        if traffic is not None:
            # what bounds the kernel instead: its emission (FP32 atomics into the build's
            # accumulators and the sinogram, gathers in the adjoint), measured as HBM bytes
            hbm = traffic / (avg_ms * 1e-3) / 1e9
            out["roofline"]["hbm_traffic_gbps"] = hbm
            out["roofline"]["hbm_traffic_frac"] = hbm / HBM_PEAK_GBS
        out["geometry_kernel"] = {"kernel": "k_cyl3d_geom (FP64 homogenization weights and response rows)",
                                  "total_ms_per_step": g_ms / steps, "launches": g_launches,
                                  "contraction_total_ms_per_step": k_ms / steps}
    else:
        # the per-voxel sweep kernel; algorithmic HBM bytes = the CSR it writes
        algo = nnz * 8 + (sc.n_voxels + 1) * 8
        gbs = algo / 2 / (avg_ms * 1e-3) / 1e9   # count + fill launches per build
        out["roofline"] = {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": gbs / HBM_PEAK_GBS, "traffic": None,
                           "kernel": "k_voxel2d (per-voxel sweep, all modes)", "avg_launch_ms": avg_ms,
                           "launches": k_launches}
    skipped = []
    if meta["mode3d"] and not args.no_extra_rows:
        per_step = (time.perf_counter() - t0) / max(steps, 1)
        out.update(extra_rows_3d(sc, tab, x, last[0], last[1], cfg, prec, per_step, skipped))
    del last
    vox, loc = _sample_voxels(cfg, meta)
    gpu = None
    if not args.no_cpu_baseline:
        gpu = gpu_samples(sc, tab, cfg, meta, vox)    # the sampled voxels' rows, all forms
    if meta["mode3d"]:
        sc._ws = None   # release the workspace before the 16^3 grid's handle takes its own
        torch.cuda.empty_cache()
        s16 = None
        if not args.no_extra_rows or gpu is not None:
            from paper_1607_06170_amd import Scanner as _S
            c16, m16 = workload("cyl3d_sub16")
            s16 = _S(c16, mode3d=True)
        if not args.no_extra_rows:
            out["forms"] = forms_rows(s16, skipped)
            out["table_grad"] = table_grad_row(s16, skipped)
            out["top_n"] = top_n_rows(skipped)
            out["mc_tables"] = mc_table_rows(skipped)
        if gpu is not None and loc is not None:
            gpu.update(gpu_projections_16(s16, loc))
        del s16
    if not args.no_cpu_baseline:
        log("timing the FP64 oracle on the host cores")
        out["cpu_baseline"], out["rel_err_vs_fp64"] = cpu_baseline(cfg, meta, sc, lors, vox, loc, gpu)
    if skipped:
        out["skipped_rows"] = skipped
    log("done")
    print(json.dumps(out))


def _left():
    return WALL_BUDGET_S - (time.perf_counter() - T_START)


def extra_rows_3d(sc, tab, x, y, xt, cfg, prec, per_step_s, skipped):
    """One list-mode OSEM subset update of 1e6 events (9e5 drawn from the
    forward projection of the phantom, 1e5 uniform over the LORs, seeded) on
    the same workload, timed once after the timed steps, while the whole run
    stays within its wall-clock budget."""
    import torch
    ev = lambda: torch.cuda.Event(enable_timing=True)
    res = {}
    if _left() > 2.0 * per_step_s:
        # events: bins drawn on the device from the expected counts, then crystal pairs
        g = torch.Generator(device="cuda").manual_seed(300)
        w = y[0].double().clamp_min(0)
        cdf = torch.cumsum(w, 0)
        n_true, n_rand = 900_000, 100_000
        trues = torch.searchsorted(cdf, torch.rand(n_true, generator=g, device="cuda", dtype=torch.float64) * cdf[-1])
        lors = torch.nonzero(w > 0).reshape(-1)
        rnd = lors[torch.randint(0, lors.numel(), (n_rand,), generator=g, device="cuda")]
        bins = torch.cat([trues.clamp_max(w.numel() - 1), rnd])
        bins = bins[torch.randperm(bins.numel(), generator=g, device="cuda")]
        del cdf, trues, lors, rnd
        Nc = cfg["n_blocks"] * cfg["n_ct"]
        NR = cfg["n_cz"] * cfg["n_brings"]
        tb, rr = bins // (NR * NR), bins % (NR * NR)
        starts = torch.tensor([i * Nc - i * (i + 1) // 2 for i in range(Nc)], device="cuda", dtype=torch.int64)
        gi = torch.searchsorted(starts, tb, right=True) - 1
        gj = tb - starts[gi] + gi + 1
        events = torch.stack([(rr // NR) * Nc + gi, (rr % NR) * Nc + gj], 1).to(torch.int32).contiguous()
        sens = sc.sensitivity(tab, precision=prec)
        x0 = torch.ones_like(x[0])
        randoms = 0.1 * float(w.mean())
        del w
        e0, e1 = ev(), ev()
        e0.record()
        sc.lm_osem_update(tab, events, x0, sens, 10, randoms, precision=prec)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        res["listmode"] = {"events": int(events.shape[0]), "ms": ms, "events_per_s": events.shape[0] / (ms * 1e-3),
                           "what": "one LM-OSEM subset update (M = 10) of the whole image: forward rows of the "
                                   "events and their back projection"}
        log(f"list-mode subset update: {events.shape[0]} events in {ms:.1f} ms")
    else:
        skipped.append("listmode (wall-clock budget)")
    return res


def table_grad_row(s16, skipped):
    """The adjoint with the table gradient, x = A^T y and d <y, A x> / d table,
    on the central 16^3 voxels (their own image grid, one image of the
    phantom, y its forward projection): timed once after a warm-up call."""
    import torch
    if _left() < 30.0:
        skipped.append("table_grad (wall-clock budget)")
        return None
    c16, m16 = workload("cyl3d_sub16")
    t16 = s16.build_table(c16["n_rows"], c16["n_sub"], c16["step_deg"])
    x = torch.tensor(phantom(c16, m16), dtype=torch.float32, device="cuda")
    y = s16.project_fwd(t16, x)
    s16.project_adj(t16, y, xt=x, want_table_grad=True)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    s16.project_adj(t16, y, xt=x, want_table_grad=True)
    e1.record()
    torch.cuda.synchronize()
    e0b, e1b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0b.record()
    s16.project_adj(t16, y)
    e1b.record()
    torch.cuda.synchronize()
    ms, ms_adj = e0.elapsed_time(e1), e0b.elapsed_time(e1b)
    log(f"adjoint with table gradient (16^3): {ms:.1f} ms (adjoint alone {ms_adj:.1f} ms)")
    return {"ms": ms, "adjoint_alone_ms": ms_adj, "table_entries": int(t16.data.numel()),
            "what": "x = A^T y and d<y, A x>/d table, one image, the central 16^3 voxels on their own grid"}


def mc_table_rows(skipped):
    """The response tables by photon-transport Monte Carlo (Sec 2.1.1, Eq.1;
    psf_build_table_mc), timed once each after a warm-up: the 2D table (61
    rows x 4 sub-positions, 1e6 photons per cell) and the 3D table (61 x 61
    rows x 4 x 4 sub-positions, 1e4 photons per cell), first interaction
    only and with Compton scatter."""
    import torch
    if _left() < 30.0:
        skipped.append("mc_tables (wall-clock budget)")
        return None
    from paper_1607_06170_amd import Scanner
    from paper_1607_06170_amd import synth
    res = {}
    for name, cfg, mode3d, n in (("2d", synth.CFG_2D, False, 1_000_000), ("3d", synth.CFG_3D, True, 10_000)):
        sc = Scanner(cfg, mode3d=mode3d)
        cells = 61 * 61 * 16 if mode3d else 61 * 4
        for scatter in (False, True):
            sc.build_table_mc(61, 4, 1.0, photons=1000, seed=2, scatter=scatter)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            sc.build_table_mc(61, 4, 1.0, photons=n, seed=3, scatter=scatter)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1)
            res[f"{name}_{'scatter' if scatter else 'first_interaction'}"] = {
                "ms": ms, "cells": cells, "photons_per_cell": n, "photons_per_s": cells * n / (ms * 1e-3)}
        del sc
    log("MC tables: " + ", ".join(f"{k} {v['ms']:.0f} ms" for k, v in res.items()))
    return res


def top_n_rows(skipped):
    """Sec 3.3 / Table 3 on the 2D ring (config 1: 64 x 64 voxels, 128
    crystals, threshold 1e-6): for N = 3, 5, 7 and untruncated, the matrix's
    non-zeros, its build time, and the forward projection of the uniform
    phantom against the untruncated one (largest entry error relative to the
    largest entry, and relative 2-norm)."""
    import torch
    if _left() < 20.0:
        skipped.append("top_n (wall-clock budget)")
        return None
    from paper_1607_06170_amd import Scanner
    from paper_1607_06170_amd import synth
    cfg = dict(synth.CFG_2D)
    sc = Scanner(cfg)
    t = sc.build_table(cfg["n_rows"], cfg["n_sub"], cfg["step_deg"])
    x = torch.tensor(synth.phantom_uniform(cfg, seed=1), dtype=torch.float32, device="cuda")
    rows = {}
    y_full = None
    for n in (0, 7, 5, 3):
        sc.build_psf_sysmat(t, threshold=cfg["threshold"], top_n=n)   # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rp, col, val = sc.build_psf_sysmat(t, threshold=cfg["threshold"], top_n=n)
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0)
        y = sc.project_fwd(t, x, top_n=n)[0].double()
        if n == 0:
            y_full = y
        d = y - y_full
        rows["untruncated" if n == 0 else f"N={n}"] = {
            "nnz": int(rp[-1].item()), "build_ms": ms,
            "fwd_max_err_of_max": float(d.abs().max() / y_full.abs().max()),
            "fwd_rel_2norm": float(d.norm() / y_full.norm())}
    log("top-N on the 2D ring: " + ", ".join(f"{k} nnz {v['nnz']}" for k, v in rows.items()))
    return {"workload": "2D ring, 64x64 voxels, 128 crystals, threshold 1e-6; forward of the uniform phantom",
            "rows": rows}


def forms_rows(sc, skipped):
    """The three precision forms of the tile contraction on the central
    16 x 16 x 16 voxels: one step each (matrix build, forward of the phantom,
    adjoint of the sinogram), timed after a warm-up step of every form; their
    errors against the FP64 oracle are in rel_err_vs_fp64."""
    import torch
    if _left() < 30.0:
        skipped.append("forms (wall-clock budget)")
        return None
    c16, m16 = workload("cyl3d_sub16")
    tab = sc.build_table(c16["n_rows"], c16["n_sub"], c16["step_deg"])
    x = torch.tensor(phantom(c16, m16), dtype=torch.float32, device="cuda")
    ev = lambda: torch.cuda.Event(enable_timing=True)
    res = {"workload": "the central 16x16x16 voxels of the 128x128x96 image, one call each"}
    for p in range(len(PREC_NAMES)):  # a warm-up step of every form first
        rp, col, val = sc.build_psf_sysmat(tab, threshold=0.0, precision=p)
        sc.project_adj(tab, sc.project_fwd(tab, x, precision=p), precision=p)
        del rp, col, val
    torch.cuda.synchronize()
    for p, name in enumerate(PREC_NAMES):
        for _ in range(1):
            e = [ev() for _ in range(4)]
            e[0].record()
            rp, col, val = sc.build_psf_sysmat(tab, threshold=0.0, precision=p)
            e[1].record()
            y = sc.project_fwd(tab, x, precision=p)
            e[2].record()
            sc.project_adj(tab, y, precision=p)
            e[3].record()
            torch.cuda.synchronize()
        res[name] = {"build_ms": e[0].elapsed_time(e[1]), "fwd_ms": e[1].elapsed_time(e[2]),
                     "adj_ms": e[2].elapsed_time(e[3]), "nnz": int(col.numel())}
        log(f"{name} on 16^3: build {res[name]['build_ms']:.1f} ms, fwd {res[name]['fwd_ms']:.1f} ms, "
            f"adj {res[name]['adj_ms']:.1f} ms")
        del rp, col, val, y
    return res


def _sample_voxels(cfg, meta):
    """Voxels the oracle computes: 24 spread over the image (seeded) and, for the
    3D scanner, 24 of its central 16^3 voxels (full-image indices): about 10 s
    of the oracle on 16 host cores."""
    rng = np.random.default_rng(7)
    nx, ny, nz = cfg["nx"], cfg["ny"], cfg.get("nz", 1)
    if not meta["mode3d"]:
        return np.arange(nx * ny), None
    if meta["full"]:
        spread = rng.choice(nx * ny * nz, 24, replace=False)
        loc = rng.choice(16 ** 3, 24, replace=False)
        li, lj, lk = loc % 16, (loc // 16) % 16, loc // 256
        central = ((lk + 40) * ny + lj + 56) * nx + li + 56
        return np.concatenate([spread, central]).astype(np.int64), loc
    loc = rng.choice(16 ** 3, 24, replace=False)
    return loc.astype(np.int64), None


def gpu_samples(sc, tab, cfg, meta, vox):
    """The GPU path's matrix rows of the sampled voxels (each built alone), in
    every precision form, copied to the host."""
    res = {}
    for p, name in enumerate(PREC_NAMES):
        if meta["mode3d"]:
            rows = []
            for v in vox:
                rp, col, val = sc.build_psf_sysmat(tab, threshold=0.0, vox_begin=int(v), vox_end=int(v) + 1,
                                                   precision=p)
                rows.append((col.cpu().numpy().astype(np.int64), val.cpu().numpy().astype(np.float64)))
            res[name] = {"rows": rows}
        else:
            rp, col, val = sc.build_psf_sysmat(tab, threshold=0.0, precision=p)
            res[name] = {"csr": (rp.cpu().numpy(), col.cpu().numpy().astype(np.int64),
                                 val.cpu().numpy().astype(np.float64))}
    return res


def _sparse_phantom_16(loc):
    c16, m16 = workload("cyl3d_sub16")
    ph = phantom(c16, m16)[0]
    xs = np.zeros(16 ** 3, np.float32)
    xs[loc] = ph[loc]
    return xs


def gpu_projections_16(s16, loc):
    """On the central 16^3 grid: the forward projection of an image non-zero on
    the sampled central voxels only, and the adjoint of a seeded uniform
    sinogram at those voxels, in every precision form (host copies)."""
    import torch
    c16, _ = workload("cyl3d_sub16")
    t16 = s16.build_table(c16["n_rows"], c16["n_sub"], c16["step_deg"])
    xs_d = torch.tensor(_sparse_phantom_16(loc), device="cuda")[None]
    ysyn = np.random.default_rng(8).random(s16.n_bins, dtype=np.float32)
    ysyn_d = torch.tensor(ysyn, device="cuda")[None]
    res = {"proj": {}}
    for p, name in enumerate(PREC_NAMES):
        y = s16.project_fwd(t16, xs_d, precision=p)[0]
        nzb = torch.nonzero(y).reshape(-1)
        xb = s16.project_adj(t16, ysyn_d, precision=p)[0][torch.tensor(loc, device="cuda")]
        res["proj"][name] = (nzb.cpu().numpy(), y[nzb].double().cpu().numpy(), xb.double().cpu().numpy())
    res["ysyn"] = ysyn
    return res


def cpu_baseline(cfg, meta, sc, lors, vox, loc, gpu):
    """The FP64 oracle, as it stands, on the host cores, on a sample of the
    workload's voxels (their full matrix columns); and, on the same voxels, the
    error of each precision form of the GPU path against it:
      - matrix rows of the sampled voxels (pattern and values);
      - 3D: on the central 16^3 voxels (their own image grid), the forward
        projection of an image that is non-zero on the sampled central voxels
        only (every bin) and the adjoint of a seeded uniform sinogram at those
        voxels."""
    from oracle import oracle as O
    nthreads = int(os.environ.get("OMP_NUM_THREADS") or (os.cpu_count() or 1))
    if meta["mode3d"]:
        nr, P = cfg["n_rows"], cfg["n_sub"]
        rt, rz = np.meshgrid(np.arange(nr), np.arange(nr), indexing="ij")
        t0 = time.perf_counter()
        otab = O.TableRef(O.table3_rows(cfg, rt.ravel(), rz.ravel(), P, cfg["step_deg"], nthreads), nr, P,
                          cfg["step_deg"])
        t_tab = time.perf_counter() - t0
        log(f"oracle table: {t_tab:.1f} s")
        t0 = time.perf_counter()
        cols, flags = O.columns_3d(cfg, otab, vox, cap=1 << 21, nthreads=nthreads)
        t1 = time.perf_counter()
        nnz = sum(len(b) for b, _ in cols)
        t2 = time.perf_counter()
        cols1, _ = O.columns_3d(cfg, otab, vox[:1], cap=1 << 21, nthreads=1)
        t3 = time.perf_counter()
        nnz1, single_n = len(cols1[0][0]), 1
        what = ("24 voxels spread over the image and 24 of its central 16^3" if meta["full"]
                else "24 voxels of the workload")
    else:
        t_tab = 0.0
        t0 = time.perf_counter()
        otab = O.table_2d(cfg)
        cols, flags = O.columns_2d(cfg, otab, vox, nthreads=nthreads)
        t1 = time.perf_counter()
        nnz = int(((cols > 0) & (cols >= cfg["threshold"])).sum())
        t2 = time.perf_counter()
        c1, _ = O.columns_2d(cfg, otab, vox[:64], nthreads=1)
        t3 = time.perf_counter()
        nnz1, single_n = int(((c1 > 0) & (c1 >= cfg["threshold"])).sum()), 64
        what = "every voxel of the workload"
    t_all = (t1 - t0) * sc.n_voxels / len(vox)    # every voxel's column, extrapolated by voxel count
    base = {"value": nnz / (t1 - t0), "unit": "elements/s", "cores": nthreads, "kind": "oracle",
            "sample": f"{what}: FP64 matrix columns (oracle table of {t_tab:.1f} s not counted)",
            "seconds": t1 - t0,
            "extrapolated_to_workload": {
                "what": "every voxel's column at the sample's per-voxel cost (forward and adjoint projections "
                        "and a list-mode update need them all; their products are not counted)",
                "build_s": t_all, "fwd_adj_lors_per_s": lors / t_all, "listmode_events_per_s": 1e6 / t_all},
            "single_thread": {"value": nnz1 / (t3 - t2), "unit": "elements/s", "voxels": single_n,
                              "seconds": t3 - t2}}
    errs = None
    if gpu is not None:
        errs = rel_errors(meta, vox, loc, cols, flags, gpu, O)
    return base, errs


def rel_errors(meta, vox, loc, cols, flags, gpu, O):
    """Each precision form against the FP64 oracle on the sampled voxels."""
    res = {}
    if not meta["mode3d"]:
        for name in PREC_NAMES:
            rp, col, val = gpu[name]["csr"]
            worst = 0.0
            for v in range(len(rp) - 1):
                g, gv = col[rp[v]:rp[v + 1]], val[rp[v]:rp[v + 1]]
                ov = cols[v, g]
                ok = ov > 0
                if ok.any():
                    worst = max(worst, float(np.max(np.abs(gv[ok] - ov[ok]) / ov[ok])))
            res[name] = {"matrix_max_rel": worst}
        return res
    for name in PREC_NAMES:
        worst, worst_big, same, n = 0.0, 0.0, True, 0
        tie_n, tie_common, tie_worst = 0, 1.0, 0.0
        for k, (g, gv) in enumerate(gpu[name]["rows"]):
            ob, ov = cols[k]
            if flags[k] & O.F_TIES:
                # a decision within a hair of a boundary: compare the common entries
                _, ia, ib = np.intersect1d(g, ob, assume_unique=True, return_indices=True)
                tie_n += 1
                tie_common = min(tie_common, len(ia) / max(len(np.union1d(g, ob)), 1))
                if len(ia):
                    tie_worst = max(tie_worst, float(np.max(np.abs(gv[ia] - ov[ib]) / ov[ib])))
                continue
            n += 1
            if not np.array_equal(g, ob):
                same = False
                continue
            rel = np.abs(gv - ov) / ov
            worst = max(worst, float(np.max(rel)))
            big = ov >= 1e-9 * ov.max()
            worst_big = max(worst_big, float(np.max(rel[big])))
        res[name] = {"matrix_rows": {
            "voxels": n, "same_pattern": same, "max_rel": worst, "max_rel_above_1e-9_of_row_max": worst_big,
            "note": "the largest relative errors sit on elements 1e-12 or more below their row's largest, whose "
                    "homogenization weights are sets of about 1e-14 of the sphere (the empty-set threshold), "
                    "where the FP64 closed form and the oracle's quadrature differ relatively",
            "voxels_with_flagged_ties": {"n": tie_n, "min_common_fraction": tie_common,
                                         "max_rel_on_common": tie_worst}}}
    if loc is None or "proj" not in gpu:
        return res
    central = cols[len(vox) - len(loc):]
    xs = _sparse_phantom_16(loc).astype(np.float64)
    yo = {}
    for (b, v), xv in zip(central, xs[loc]):
        for bb, vv in zip(b.tolist(), v.tolist()):
            yo[bb] = yo.get(bb, 0.0) + vv * xv
    bins = np.array(sorted(yo), dtype=np.int64)
    yref = np.array([yo[b] for b in bins])
    ysyn = gpu["ysyn"].astype(np.float64)
    xref = np.array([float(np.dot(v, ysyn[b])) for b, v in central])
    for name in PREC_NAMES:
        nzb, yv, xb = gpu["proj"][name]
        ymap = dict(zip(nzb.tolist(), yv.tolist()))
        yg = np.array([ymap.get(int(b), 0.0) for b in bins])
        outside = float(sum(abs(v) for b, v in ymap.items() if b not in yo))
        d = yg - yref
        res[name]["fwd_sparse_image_16cube"] = {
            "bins": int(len(bins)), "max_rel_entry": float(np.max(np.abs(d) / yref)),
            "max_rel_entry_above_1e-3_of_max": float(np.max((np.abs(d) / yref)[yref > 1e-3 * yref.max()])),
            "max_abs_over_max": float(np.abs(d).max() / yref.max()),
            "rel_l2": float(np.linalg.norm(d) / np.linalg.norm(yref)), "mass_outside_oracle_bins": outside}
        res[name]["adj_sampled_voxels_16cube"] = {"voxels": int(len(loc)),
                                                  "max_rel": float(np.max(np.abs(xb - xref) / np.abs(xref)))}
        log(f"{name} vs FP64: rows {res[name]['matrix_rows']['max_rel']:.2e}, fwd entry "
            f"{res[name]['fwd_sparse_image_16cube']['max_rel_entry']:.2e}, adj "
            f"{res[name]['adj_sampled_voxels_16cube']['max_rel']:.2e}")
    return res


if __name__ == "__main__":
    main()
