#!/usr/bin/env python3
"""Throughput of the P-SPIR system-matrix hot path on one MI355X.

One step = one pass of the whole path over one synthetic input:
  build_psf_sysmat (count + fill phases: CSR of A^T over the voxel range),
  project_fwd (y = A x on the fly) and project_adj (A^T y on the fly).
Prints ONE JSON line.  ``value`` is system-matrix elements (CSR non-zeros)
produced per second of the build; the same line carries the forward+adjoint
projection rate in LORs/s, a roofline object for the dominant kernel (timed
with HIP events around its launches, on the stream it runs on) and the FP64
oracle timed on the host cores.

Workloads (all inputs seeded and synthetic, resident in HBM before timing):
  cyl3d_sub16  3D scanner of 32 blocks x 12 x 12 crystals (2 x 2 x 15 mm),
               4 block rings, faces at 130 mm; the central 16 x 16 x 16 voxels
               (1 mm) of its 128 x 128 x 96 image; analytic 61x61x4x4x5x5 table.
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

HBM_PEAK_GBS = 8000.0        # MI355X HBM3E
FP32_VALU_TFLOPS = 157.3     # MI355X vector FP32
FP64_VALU_TFLOPS = 78.6      # MI355X vector FP64
FP32_MATRIX_TFLOPS = 157.3   # MI355X dense FP32 matrix cores
BF16_MATRIX_TFLOPS = 2500.0  # MI355X dense BF16 matrix cores


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=None)
    ap.add_argument("--workload", default="cyl3d_sub16", choices=["cyl3d_sub16", "ring2d_64"])
    ap.add_argument("--precision", type=int, default=0, help="0 FP32 plain, 1 BF16, 2 BF16 hi/lo")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra-rows", action="store_true",
                    help="skip the rows timed after the steps (table gradient, list mode, BF16 forms), e.g. under a "
                         "profiler, so that its kernel mix is the timed step's")
    ap.add_argument("--copy-probe", action="store_true",
                    help="first copy 1 GiB on the device (a kernel of known traffic, to scale PMC byte counters)")
    return ap.parse_args()


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
    if name == "cyl3d_sub16":
        cfg = dict(synth.CFG_3D, nx=16, ny=16, nz=16)
        desc = ("3D: 32 blocks x 12x12 LYSO crystals (2x2x15 mm), 4 block rings (48 crystal rings), faces at "
                "130 mm; central 16x16x16 voxels (1 mm) of the 128x128x96 image; analytic 61x61x4x4x5x5 table; "
                "all non-zeros kept")
        return cfg, dict(workload=desc, mode3d=True, batch=1, steps=3, warmup=1)
    cfg = dict(synth.CFG_2D)
    desc = ("2D ring: 16 blocks x 8 LYSO crystals (2 mm, 15 mm deep), faces at 65 mm; 64x64 image of 1 mm "
            "voxels; 61 x 4 x 5 table; threshold 1e-6")
    return cfg, dict(workload=desc, mode3d=False, batch=1, steps=20, warmup=3)


def phantom(cfg, meta):
    from paper_1607_06170_amd import synth
    if meta["mode3d"]:
        full = dict(cfg, nx=128, ny=128, nz=96)
        img = synth.phantom_blobs(full, seed=2).reshape(96, 128, 128)
        sub = img[40:56, 56:72, 56:72]   # the central 16^3 voxels
        return np.ascontiguousarray(sub.reshape(1, -1))
    return synth.phantom_uniform(cfg, seed=1, batch=meta["batch"])


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; the multi-GPU layout (voxel sharding plus "
                                   "one all-reduce of the sinogram) is described in the design notes, not built"}))
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
    torch.cuda.synchronize()

    ev = lambda: torch.cuda.Event(enable_timing=True)
    rec = dict(build=[], fwd=[], adj=[], nnz=0, tiles=0, vtiles=0)
    last = {}   # the last timed step's outputs

    def step(record):
        e0, e1, e2, e3 = ev(), ev(), ev(), ev()
        e0.record()
        # tile counters of each call (each build phase): copied on the device, in stream order, read after
        # the step; a fill phase that copies the rows its count phase staged contracts nothing
        h_build = [] if meta["mode3d"] and record else None
        rp, col, val = sc.build_psf_sysmat(tab, threshold=thr, precision=prec, counters=h_build)
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
            rec["nnz"] += int(col.numel())
            rec["tiles"] += t_build + t_fwd + t_adj
            rec["vtiles"] += v_build + v_fwd + v_adj
            last.update(rp=rp, col=col, val=val, y=y, xb=xb)
        return xb

    def log(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    log(f"workload {args.workload}: {sc.n_voxels} voxels, {sc.n_bins} bins; warmup {warmup}, steps {steps}")
    for i in range(warmup):
        step(False)
        torch.cuda.synchronize()
        log(f"warmup step {i + 1} done")
    torch.cuda.synchronize()
    sc.profile_start()
    t0 = time.perf_counter()
    xb_last = [None]
    for i in range(steps):
        xb_last[0] = step(True)
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
        "dtype": ["f32", "bf16", "bf16x2"][prec] + " tiles, f64 geometry and weights",
        "data": "synthetic (seeded phantom, analytic response table)",
        "config": {"workload": meta["workload"], "voxels": sc.n_voxels, "bins": sc.n_bins,
                   "batch": meta["batch"], "nnz": nnz, "lors": lors},
        "fwd_adj_lors_per_s": lors * meta["batch"] * steps / proj_s,
        "build_ms": float(np.mean(rec["build"])), "fwd_ms": float(np.mean(rec["fwd"])),
        "adj_ms": float(np.mean(rec["adj"])),
        "rel_err_vs_fp64": "<= 1e-5 per element, FP32 form (tests/test_gpu_2d.py, tests/test_gpu_3d.py)",
    }
    avg_ms = k_ms / max(k_launches, 1)
    if meta["mode3d"]:
        K = cfg["n_sub"] ** 2
        flops_tile = 2 * (K * K * 25 + 25 * K * 25)   # X = W V, then T = U^T X (unpadded): 32 800 for P = 4
        # algorithmic units: (voxel, tile) pairs -- the tiles a voxel-by-voxel method contracts; a contracted
        # tile serves every voxel of its z-column class that sees both its rings
        vtiles_per_launch = rec["vtiles"] / max(k_launches, 1)
        tiles_per_launch = rec["tiles"] / max(k_launches, 1)
        achieved = vtiles_per_launch * flops_tile / (avg_ms * 1e-3) / 1e12
        executed = tiles_per_launch * flops_tile / (avg_ms * 1e-3) / 1e12
        peak = [FP32_MATRIX_TFLOPS, BF16_MATRIX_TFLOPS, BF16_MATRIX_TFLOPS][prec]
        traffic = measured_traffic(f"k_cyl3d_mma.{args.workload}.{['fp32', 'bf16', 'bf16x2'][prec]}.pmc.txt")
        out["roofline"] = {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                           "frac": achieved / peak, "traffic": traffic,
                           "kernel": "k_cyl3d_mma (tile contraction T = U^T (W V) on matrix cores, "
                                     + ["FP32", "BF16", "BF16 hi/lo"][prec] + ", and its emission; all modes)",
                           "avg_launch_ms": avg_ms, "launches": k_launches,
                           "voxel_tiles_per_launch": vtiles_per_launch, "flops_per_voxel_tile": flops_tile,
                           "tiles_contracted_per_launch": tiles_per_launch,
                           "executed_tflops": executed, "executed_frac": executed / peak}
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
    if meta["mode3d"] and not args.no_extra_rows:
        out.update(extra_rows_3d(sc, tab, x, xb_last[0], cfg, prec, log))
        if prec == 0:
            out["forms"] = forms_rows(sc, tab, x, last, thr, log)
    if not args.no_cpu_baseline:
        log("timing the FP64 oracle on the host cores")
        out["cpu_baseline"] = cpu_baseline(cfg, meta, x_np, thr)
    print(json.dumps(out))


def extra_rows_3d(sc, tab, x, xt, cfg, prec, log):
    """The hot path's other two rows on the same workload, each timed once
    after a warm-up call (outside the timed steps above):
      - the adjoint with the table gradient d <y, A xt> / d table;
      - one list-mode OSEM subset update of 1e6 events (9e5 drawn from the
        forward projection of the phantom, 1e5 uniform over the LORs, seeded)."""
    import torch
    ev = lambda: torch.cuda.Event(enable_timing=True)
    res = {}
    y = sc.project_fwd(tab, x, precision=prec)
    for _ in range(2):
        e0, e1 = ev(), ev()
        e0.record()
        sc.project_adj(tab, y, xt=xt, want_table_grad=True, precision=prec)
        e1.record()
        torch.cuda.synchronize()
    res["table_grad"] = {"ms": e0.elapsed_time(e1), "table_entries": int(tab.data.numel()),
                         "what": "x = A^T y and d<y, A xt>/d table, one image"}
    log(f"adjoint with table gradient: {res['table_grad']['ms']:.1f} ms")
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
    for _ in range(2):
        e0, e1 = ev(), ev()
        e0.record()
        sc.lm_osem_update(tab, events, x0, sens, 10, randoms, precision=prec)
        e1.record()
        torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    res["listmode"] = {"events": int(events.shape[0]), "ms": ms, "events_per_s": events.shape[0] / (ms * 1e-3),
                       "what": "one LM-OSEM subset update (M = 10), forward rows of the events and their back projection"}
    log(f"list-mode subset update: {events.shape[0]} events in {ms:.1f} ms")
    return res


def forms_rows(sc, tab, x, ref, thr, log):
    """The BF16 forms of the tile contraction beside the FP32 form, on the same
    workload and GPU: one step each (matrix build, forward of the phantom,
    adjoint of the FP32 form's sinogram), timed after a warm-up step, and the
    results against the FP32 form's (max over elements of |d| / |ref| for the
    matrix when both have the same pattern; max |d| / max |ref| and the
    relative 2-norm for the projections)."""
    import torch
    ev = lambda: torch.cuda.Event(enable_timing=True)
    res = {}

    def rel(a, b):
        a, b = a.double(), b.double()
        d = a - b
        return {"max_rel_to_max": float(d.abs().max() / b.abs().max()),
                "rel_l2": float(d.norm() / b.norm())}

    for p, name in ((1, "bf16"), (2, "bf16x2")):
        for _ in range(2):
            e = [ev() for _ in range(4)]
            e[0].record()
            rp, col, val = sc.build_psf_sysmat(tab, threshold=thr, precision=p)
            e[1].record()
            y = sc.project_fwd(tab, x, precision=p)
            e[2].record()
            xb = sc.project_adj(tab, ref["y"], precision=p)
            e[3].record()
            torch.cuda.synchronize()
        r = {"build_ms": e[0].elapsed_time(e[1]), "fwd_ms": e[1].elapsed_time(e[2]),
             "adj_ms": e[2].elapsed_time(e[3]), "nnz": int(col.numel()),
             "same_pattern": bool(torch.equal(rp, ref["rp"]) and torch.equal(col, ref["col"]))}
        if r["same_pattern"]:
            v32 = ref["val"].double()
            r["matrix_max_rel_err"] = float(((val.double() - v32).abs() / v32.abs()).max())
        r["fwd_vs_fp32"] = rel(y, ref["y"])
        r["adj_vs_fp32"] = rel(xb, ref["xb"])
        res[name] = r
        log(f"{name}: build {r['build_ms']:.1f} ms, fwd {r['fwd_ms']:.1f} ms, adj {r['adj_ms']:.1f} ms; "
            f"matrix max rel err {r.get('matrix_max_rel_err', float('nan')):.2e}, "
            f"fwd {r['fwd_vs_fp32']['max_rel_to_max']:.2e}, adj {r['adj_vs_fp32']['max_rel_to_max']:.2e} vs FP32")
        del rp, col, val, y, xb
    return res


def cpu_baseline(cfg, meta, x_np, thr):
    """The FP64 oracle, as it stands, on the host cores."""
    from oracle import oracle as O
    nthreads = min(16, os.cpu_count() or 1)
    if meta["mode3d"]:
        nr, P = cfg["n_rows"], cfg["n_sub"]
        rt, rz = np.meshgrid(np.arange(nr), np.arange(nr), indexing="ij")
        t0 = time.perf_counter()
        tab = O.TableRef(O.table3_rows(cfg, rt.ravel(), rz.ravel(), P, cfg["step_deg"], nthreads), nr, P,
                         cfg["step_deg"])
        t_tab = time.perf_counter() - t0
        print(f"[bench] oracle table: {t_tab:.1f} s", file=sys.stderr, flush=True)
        vox = np.linspace(0, 16 ** 3 - 1, 2 * nthreads).astype(np.int64)
        t0 = time.perf_counter()
        cols, _ = O.columns_3d(cfg, tab, vox, cap=1 << 21, nthreads=nthreads)
        t1 = time.perf_counter()
        nnz = sum(len(b) for b, _ in cols)
        # one thread, two of the same voxels
        v1 = vox[[len(vox) // 3, 2 * len(vox) // 3]]
        t2 = time.perf_counter()
        cols1, _ = O.columns_3d(cfg, tab, v1, cap=1 << 21, nthreads=1)
        t3 = time.perf_counter()
        nnz1 = sum(len(b) for b, _ in cols1)
        return {"value": nnz / (t1 - t0), "unit": "elements/s", "cores": nthreads, "kind": "oracle",
                "sample": f"{len(vox)} voxels spread over the 16^3 sub-volume: FP64 sparse columns "
                          f"(table build of {t_tab:.1f} s not counted)", "seconds": t1 - t0,
                "single_thread": {"value": nnz1 / (t3 - t2), "unit": "elements/s", "voxels": len(v1),
                                  "seconds": t3 - t2}}
    t0 = time.perf_counter()
    tab = O.table_2d(cfg)
    cols, _ = O.columns_2d(cfg, tab, np.arange(cfg["nx"] * cfg["ny"]), nthreads=nthreads)
    rp, col, val = O.csr_from_columns(cols, thr)
    t1 = time.perf_counter()
    return {"value": len(col) / (t1 - t0), "unit": "elements/s", "cores": nthreads, "kind": "oracle",
            "sample": "full workload: every voxel's FP64 column and the CSR", "seconds": t1 - t0}


if __name__ == "__main__":
    main()
