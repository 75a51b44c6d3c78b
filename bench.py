#!/usr/bin/env python3
"""Throughput of weighted-quadrature row assembly on one MI355X.

A step is one pass of the whole assembly for one coefficient field: wq_assemble_rows
(interior rows by line-blocked sum factorization, cut rows with DWQ boxes) followed by
cut_assemble (element Gauss remainders, then octree cut cells), forming the mass and the
stiffness matrix on the fixed CSR pattern.  The rules handle (Gauss rule, WQ/DWQ rules,
classification, pattern, octree) is built once before the timed region, and kappa is
resident in device memory.

Prints one JSON line.  Default workload: 48^3 elements, p=4, domain {x+y+z < 1.6},
kappa = exp of a seeded Gaussian random field.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "assembled nnz/s at p=4, 48³ cut cube: FP64 vs FP32 path at ≤2e-6 rel err"
PEAK = {"hbm_GBps": 8000.0, "fp64_TFLOPs": 78.6, "fp32_TFLOPs": 157.3}


KAPPA_TEXT = {"rf": "exp(seeded Gaussian random field, 8 modes/axis, sigma 0.5)",
              "sin3": "1+0.5 sin(2 pi x) sin(2 pi y) sin(2 pi z)", "one": "1"}


def domain_text(ls):
    import workloads as W
    if ls.kind == W.LS_PLANE:
        return f"{ls.n[0]:g}x+{ls.n[1]:g}y+{ls.n[2]:g}z<{ls.r0:g}"
    if ls.kind == W.LS_BALL:
        return f"|x-({ls.c[0]:g},{ls.c[1]:g},{ls.c[2]:g})|<{ls.r0:g}"
    if ls.kind == W.LS_TORUS:
        return f"torus about z through ({ls.c[0]:g},{ls.c[1]:g},{ls.c[2]:g}), R={ls.r0:g}, r={ls.r1:g}"
    return "unit cube (uncut)"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="plane48_p4")
    ap.add_argument("--dtype", default="f32", choices=["f32", "f64"])
    ap.add_argument("--skip-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-rows", type=int, default=128, help="rows in the oracle's timed sample")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 256 MiB device copy (calibrates the HBM byte counters)")
    ap.add_argument("--paper-sweep", action="store_true",
                    help="the paper's accuracy and timing experiment instead of the benchmark: L2 projection of "
                         "sin(2xz)cos(3yz) on [-1,1]^3 below the inclined plane, schemes Ref / Hybrid / DWQ, one JSON "
                         "line per (h, p)")
    ap.add_argument("--tensor", choices=["fit", "octree"], default=None,
                    help="only the stiffness with the map's coefficient tensor (wq_assemble_tensor) on the workload, "
                         "cut elements by the fitted rule or the octree; one JSON line")
    ap.add_argument("--sweep-h", default="4,8,16,32,64")
    ap.add_argument("--sweep-p", default="2,3,4,5,6")
    return ap.parse_args()


def copy_probe():
    """A plain device-to-device copy of 256 MiB, three times: the reference for scaling the
    FETCH_SIZE / WRITE_SIZE counters of the assembly kernels."""
    import torch
    n = 64 * 1024 * 1024
    x = torch.ones(n, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": 4 * n, "copies": 3}))


# HBM bytes per launch from rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE (KiB per dispatch, the
# median over a run), scaled by what the same counters read for `bench.py --copy-probe` (a
# 256 MiB copy reads FETCH_SIZE = 128 MiB, WRITE_SIZE = 256 MiB: fetch x 2.0, write x 1.0).  A
# group of kernels sums its members.  Valid only for the kernel sources they were taken on:
# the SHA-1 over the members' source digests is checked, else traffic is null.
TRAFFIC = {
    # (kernels, workload, dtype): (sha1 over the kernels' source digests, fetch KiB, write KiB)
    (("k_cut_remainder",), "plane48_p4", "f32"): ("05a0d4aa6f6e58b4b3a3c5f552922a5bf6bb28b0", 159177.4, 115167.4),
    (("k_cut_remainder",), "plane48_p4", "f64"): ("05a0d4aa6f6e58b4b3a3c5f552922a5bf6bb28b0", 251025.1, 228916.3),
    (("k_rows_block", "k_rows_box", "k_rows_zero"), "plane48_p4", "f32"): ("01574deff6b788284331e48f2376cdd61c267fc6", 57726.9, 458689.5),
    (("k_cut_moments", "k_cut_local", "k_cut_gather"), "plane48_p4", "f32"): ("747ff50a7cad0b53651a12e61d4bbe0fe61289c4", 759447.2, 775283.6),
}


def kernel_digest(name):
    import hashlib
    import re
    for f in ("cut.hip", "rows.hip", "adjoint.hip"):
        src = open(os.path.join(ROOT, "paper_2211_06427_amd", "csrc", f)).read()
        m = re.search(r"\n(template <[^\n]*>\n__global__[^\n]*\n)?" + name + r"\(", src)
        if m:
            start = src.rfind("\n// ", 0, m.start())
            end = src.find("\n}\n", m.end())
            return hashlib.sha1(src[start:end].encode()).hexdigest()
    return None


def group_digest(kernels):
    import hashlib
    parts = [kernel_digest(k) for k in kernels]
    if any(p is None for p in parts):
        return None
    return hashlib.sha1("".join(parts).encode()).hexdigest()


def measured_traffic(kernels, workload, dtype):
    rec = TRAFFIC.get((tuple(kernels), workload, dtype))
    if rec is None or group_digest(kernels) != rec[0]:
        return None
    return (rec[1] * 2.0 + rec[2] * 1.0) * 1024


def timed(fn, n, torch):
    """Mean duration (ms) of fn over n calls, HIP events on the current stream."""
    s = torch.cuda.Event(enable_timing=True)
    e = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    s.record()
    for _ in range(n):
        fn()
    e.record()
    torch.cuda.synchronize()
    return s.elapsed_time(e) / n


# rows whose FP64 maximum is below 2^-100 (26 bits above FP32's smallest normal) lie where
# FP32 underflows (thin slivers of a cut support); they are counted, not compared
FP32_ROW_FLOOR = 2.0 ** -100


def row_scaled_err(a, b, row_ptr, torch):
    """(max over rows of max|a-b| / max|b| for rows with max|b| >= FP32_ROW_FLOOR, number of
    rows below that floor, Frobenius relative error over all entries); b is the reference."""
    rows = torch.repeat_interleave(torch.arange(len(row_ptr) - 1, device=a.device), torch.diff(row_ptr))
    d = torch.zeros(len(row_ptr) - 1, dtype=torch.float64, device=a.device)
    m = torch.zeros_like(d)
    diff = a.double() - b.double()
    d.scatter_reduce_(0, rows, diff.abs(), "amax")
    m.scatter_reduce_(0, rows, b.double().abs(), "amax")
    ok = m >= FP32_ROW_FLOOR
    e = float((d[ok] / m[ok]).max()) if bool(ok.any()) else 0.0
    return {"row_scaled": e, "rows_below_fp32_range": int((~ok).sum()),
            "frobenius": float(diff.norm() / b.double().norm())}


def _oracle_rows_timed(args):
    """Worker: builds the oracle's Problem (untimed), then times its share of the sampled rows."""
    name, rows = args
    import numpy as np
    from threadpoolctl import threadpool_limits

    import workloads as W
    from oracle.assemble import Problem, kappa_numpy
    wl = W.workload(name)
    P = Problem(wl)
    rp = P.row_ptr()
    kap = kappa_numpy(wl)
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        P.assemble_rows(np.asarray(rows, dtype=np.int64), kap)
        dt = time.perf_counter() - t0
    return int(sum(rp[r + 1] - rp[r] for r in rows)), dt


def cpu_baseline(wl, nrows):
    """The oracle (unchanged) on a seeded sample of rows: one process per host core (at most 16),
    each single-threaded on an equal share of the rows; nnz/s over both matrices = sampled
    entries / the slowest worker's time.  The single-core rate of the same sample is kept beside it."""
    import multiprocessing as mp

    import workloads as W
    from oracle.assemble import Problem
    n_active = Problem(wl).dom.n_active
    rows = [int(r) for r in W.sample_indices(7, n_active, nrows)]
    cores = max(1, min(16, os.cpu_count() or 1, len(rows)))
    shares = [rows[k::cores] for k in range(cores)]
    saved = {v: os.environ.get(v) for v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")}
    for v in saved:
        os.environ[v] = "1"
    try:
        with mp.get_context("spawn").Pool(cores) as pool:
            res = pool.map(_oracle_rows_timed, [(wl.name, s) for s in shares])
    finally:
        for v, old in saved.items():
            if old is None:
                os.environ.pop(v, None)
            else:
                os.environ[v] = old
    nnz = sum(r[0] for r in res)
    wall = max(r[1] for r in res)
    serial = sum(r[1] for r in res)
    return {"value": 2 * nnz / wall, "unit": "nnz/s", "cores": cores, "kind": "oracle",
            "single_core_value": 2 * nnz / serial,
            "sample": f"{len(rows)} seeded rows of {n_active} (all row classes), {nnz} entries per matrix, "
                      f"mass+stiffness; {cores} single-threaded processes on equal shares, slowest {wall:.1f} s "
                      f"(one core: {serial:.1f} s); rule setup excluded"}


def paper_sweep(args):
    """Section 3.1 / 3.2: mass matrix of the cut cube [-1,1]^3 (kappa = 1, FP64), L2 projection of
    f = sin(2xz) cos(3yz) with extended B-splines (PCG to a relative residual of 1e-14), relative
    L2 error, for the three schemes: Ref (element-by-element Gauss), Hybrid Gauss and DWQ, plus
    DWQ with the fitted cut-element rule.  Times are HIP-event means over repeated calls; the Ref load vector is the row sums of
    its mass matrix with kappa = f."""
    import torch

    import workloads as W
    from paper_2211_06427_amd import Rules
    from paper_2211_06427_amd._lib import WQ_CUT_OCTREE, WQ_CUT_REMAINDER, WQ_MASS
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    f64 = torch.float64
    for p in [int(v) for v in args.sweep_p.split(",")]:
        for h in [int(v) for v in args.sweep_h.split(",")]:
            wl = W.paper_plane(h, p)
            rec = {"h": h, "p": p}
            nrep = 5 if h <= 32 else 2
            ref_rules = None
            for scheme, hyb in (("dwq", False), ("hybrid", True), ("dwq_fit", False)):
                wls = W.with_cut_rule(wl, "fit") if scheme == "dwq_fit" else wl
                t0 = time.perf_counter()
                R = Rules.from_workload(wls, hybrid_gauss=hyb)
                torch.cuda.synchronize()
                build_ms = (time.perf_counter() - t0) * 1e3
                one = torch.ones(R.n_kappa, dtype=f64, device=dev)
                f = W.target_f(R.kappa_xyz())
                vm = torch.empty(R.nnz, dtype=f64, device=dev)
                one32, vm32 = one.float(), torch.empty(R.nnz, dtype=torch.float32, device=dev)

                def mass(o=one, v=vm):
                    R.assemble_rows(o, v, None, which=WQ_MASS)
                    R.cut_assemble(o, v, None, which=WQ_MASS)

                mass()
                r = {"build_rules_ms": build_ms, "n_active": R.n_active, "nnz": R.nnz,
                     "rows_ms": timed(lambda: R.assemble_rows(one, vm, None, which=WQ_MASS), nrep, torch),
                     "remainder_ms": timed(lambda: R.cut_assemble(one, vm, None, which=WQ_MASS | WQ_CUT_REMAINDER),
                                           nrep, torch),
                     "octree_ms": timed(lambda: R.cut_assemble(one, vm, None, which=WQ_MASS | WQ_CUT_OCTREE),
                                        nrep, torch),
                     "mass_ms": timed(mass, nrep, torch),
                     "mass_f32_ms": timed(lambda: mass(one32, vm32), nrep, torch)}
                mass()
                t0 = time.perf_counter()
                b = R.load_vector(f)
                torch.cuda.synchronize()
                r["load_vector_ms"] = (time.perf_counter() - t0) * 1e3
                t0 = time.perf_counter()
                ext = R.extension()
                r["extension_ms"] = (time.perf_counter() - t0) * 1e3
                t0 = time.perf_counter()
                u, it, rel = R.project(ext, vm, b, tol=1e-14, max_iter=100000)
                r["solve_ms"] = (time.perf_counter() - t0) * 1e3
                fg = W.target_f(R.gauss_coords())
                e2, n2 = R.l2_error(u, fg, f)
                r.update({"cg_iterations": it, "cg_relres": rel, "rel_l2_error": math.sqrt(e2 / n2),
                          "n_inner": ext.n_inner, "n_outer": ext.n_outer})
                rec[scheme] = r
                print(f"# h={h} p={p} {scheme}: err {r['rel_l2_error']:.3e} mass {r['mass_ms']:.3f} ms "
                      f"cg {it}", file=sys.stderr, flush=True)
                if scheme == "dwq":
                    ref_rules, ref_ext, ref_f, ref_fg = R, ext, f, fg
                else:
                    del R
                del ext
            # Ref: conventional element-by-element Gauss on the same pattern, slots and octree
            R = ref_rules
            one = torch.ones(R.n_kappa, dtype=f64, device=dev)
            og = torch.ones(R.n_gauss_elems * (p + 1) ** 3, dtype=f64, device=dev)
            ms = timed(lambda: R.gauss_assemble(og, one, which=WQ_MASS), max(2, nrep // 2), torch)
            ms32 = timed(lambda: R.gauss_assemble(og.float(), one.float(), which=WQ_MASS), max(2, nrep // 2), torch)
            M, _ = R.gauss_assemble(og, one, which=WQ_MASS)
            Mf, _ = R.gauss_assemble(ref_fg, ref_f, which=WQ_MASS)
            rp = R.row_ptr()
            rows = torch.repeat_interleave(torch.arange(R.n_active, device=dev), torch.diff(rp))
            b = torch.zeros(R.n_active, dtype=f64, device=dev).index_add_(0, rows, Mf)
            u, it, rel = R.project(ref_ext, M, b, tol=1e-14, max_iter=100000)
            e2, n2 = R.l2_error(u, ref_fg, ref_f)
            rec["ref"] = {"mass_ms": ms, "mass_f32_ms": ms32, "cg_iterations": it, "cg_relres": rel,
                          "rel_l2_error": math.sqrt(e2 / n2)}
            # the same Gauss integrals formed row by row with sum factorization, no atomics
            Rg = Rules.from_workload(wl, gauss_rows=True)
            og_, vg = torch.ones(Rg.n_kappa, dtype=f64, device=dev), torch.empty(Rg.nnz, dtype=f64, device=dev)

            def mass_g(o=og_, v=vg):
                Rg.assemble_rows(o, v, None, which=WQ_MASS)
                Rg.cut_assemble(o, v, None, which=WQ_MASS)

            mass_g()
            o32, v32 = og_.float(), torch.empty(Rg.nnz, dtype=torch.float32, device=dev)
            rec["gauss_rows"] = {"mass_ms": timed(mass_g, nrep, torch),
                                 "mass_f32_ms": timed(lambda: mass_g(o32, v32), nrep, torch)}
            del Rg, og_, vg, o32, v32
            print(f"# h={h} p={p} ref: err {rec['ref']['rel_l2_error']:.3e} mass {ms:.3f} ms", file=sys.stderr,
                  flush=True)
            del R, ref_rules, ref_ext, M, Mf
            print(json.dumps(rec), flush=True)


def tensor_only(args):
    """K steps of wq_assemble_tensor (the map's coefficient tensor at the slots, resident in
    HBM) after W warm-ups; prints nnz/s and the mean step time."""
    import torch

    import workloads as W
    from paper_2211_06427_amd import Rules
    wl = W.with_cut_rule(W.workload(args.workload), args.tensor)
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    R = Rules.from_workload(wl, tensor=True)
    dt = torch.float32 if args.dtype == "f32" else torch.float64
    Cm = W.tensor_components(W.map_tensor(R.kappa_xyz())).to(dt).contiguous()
    vk = torch.empty(R.nnz, dtype=dt, device=dev)
    for _ in range(args.warmup):
        R.assemble_tensor(Cm, vk)
    ms = timed(lambda: R.assemble_tensor(Cm, vk), args.steps, torch)
    print(json.dumps({"metric": "tensor stiffness nnz/s", "value": R.nnz / (ms * 1e-3), "unit": "nnz/s",
                      "ms_per_step": ms, "steps": args.steps, "warmup": args.warmup, "dtype": args.dtype,
                      "config": {"workload": wl.name, "cut_rule": args.tensor, "field": "map pull-back tensor",
                                 "nnz": R.nnz, "n_kappa": R.n_kappa}}), flush=True)


def main():
    args = parse()
    if args.copy_probe:
        copy_probe()
        return
    if args.tensor:
        tensor_only(args)
        return
    if args.paper_sweep:
        paper_sweep(args)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the library assembles on a "
              f"single device.", file=sys.stderr)
        sys.exit(2)
    import torch

    import workloads as W
    from paper_2211_06427_amd import Rules
    from paper_2211_06427_amd._lib import WQ_CUT_OCTREE, WQ_CUT_REMAINDER
    wl = W.workload(args.workload)
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)

    t0 = time.perf_counter()
    R = Rules.from_workload(wl)
    torch.cuda.synchronize()
    build_cold_ms = (time.perf_counter() - t0) * 1e3
    t0 = time.perf_counter()
    R2 = Rules.from_workload(wl)
    torch.cuda.synchronize()
    build_ms = (time.perf_counter() - t0) * 1e3
    del R2

    k64 = W.kappa_at(wl, R.kappa_xyz())
    kap = {"f64": k64, "f32": k64.float()}
    dt = {"f64": torch.float64, "f32": torch.float32}
    main_dt = args.dtype
    vals = {k: (torch.empty(R.nnz, dtype=dt[k], device=dev), torch.empty(R.nnz, dtype=dt[k], device=dev))
            for k in ("f64", "f32")}

    def step(k):
        vm, vk = vals[k]
        R.assemble_rows(kap[k], vm, vk)
        R.cut_assemble(kap[k], vm, vk)

    # --- the timed region: K steps of the main dtype ---------------------------------
    # A step is rows + remainder + octree (the two cut parts are issued as two calls so
    # that HIP events on the launch stream bracket each kernel group inside the timed
    # region; together they are exactly one cut_assemble).
    PARTS = ("rows", "remainder", "octree")
    for _ in range(args.warmup):
        step(main_dt)
    stream = torch.cuda.current_stream(dev)
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(args.steps)]
    vm_main, vk_main = vals[main_dt]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        ev[i][0].record(stream)
        R.assemble_rows(kap[main_dt], vm_main, vk_main)
        ev[i][1].record(stream)
        R.cut_assemble(kap[main_dt], vm_main, vk_main, parts=WQ_CUT_REMAINDER)
        ev[i][2].record(stream)
        R.cut_assemble(kap[main_dt], vm_main, vk_main, parts=WQ_CUT_OCTREE)
        ev[i][3].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = wall * 1e3 / args.steps
    n_mat = 2
    value = n_mat * R.nnz / (wall / args.steps)
    timed_ms = {name: sum(e[j].elapsed_time(e[j + 1]) for e in ev) / args.steps for j, name in enumerate(PARTS)}
    per_step = sorted(e[0].elapsed_time(e[3]) for e in ev)
    step_stats = {"median": per_step[len(per_step) // 2], "min": per_step[0], "max": per_step[-1]}

    # --- breakdown (outside the timed region) ----------------------------------------
    nrep = max(3, min(args.steps, 10))
    parts = {}
    kg = None
    if wl.octree_levels <= 3:
        kg64 = W.kappa_at(wl, R.gauss_coords())
        kg = {"f64": kg64, "f32": kg64.float()}
    for k in ("f64", "f32"):
        vm, vk = vals[k]
        step(k)
        parts[k] = {
            "step_ms": timed(lambda: step(k), nrep, torch),
            "rows_ms": timed(lambda: R.assemble_rows(kap[k], vm, vk), nrep, torch),
            "remainder_ms": timed(lambda: R.cut_assemble(kap[k], vm, vk, parts=WQ_CUT_REMAINDER), nrep, torch),
            "octree_ms": timed(lambda: R.cut_assemble(kap[k], vm, vk, parts=WQ_CUT_OCTREE), nrep, torch),
        }
        g = torch.ones(R.nnz, dtype=dt[k], device=dev)
        parts[k]["adjoint_ms"] = timed(lambda: R.adjoint(g, g), nrep, torch)
        # conventional element-by-element Gauss assembly of the same matrices (octrees of depth
        # <= 3 only)
        if kg is not None:
            parts[k]["gauss_ms"] = timed(lambda: R.gauss_assemble(kg[k], kap[k]), max(2, nrep // 3), torch)
    step("f64")
    step("f32")
    torch.cuda.synchronize()
    rp = R.row_ptr()
    err32 = {"mass": row_scaled_err(vals["f32"][0], vals["f64"][0], rp, torch),
             "stiff": row_scaled_err(vals["f32"][1], vals["f64"][1], rp, torch)}
    # BF16x3 experiment: interior rows' direction-1 contraction on matrix cores with split
    # bf16 operands (the rest as FP32); rows pass time and error of the whole matrices
    vb = (torch.empty(R.nnz, device=dev), torch.empty(R.nnz, device=dev))

    def step_bf3():
        R.assemble_rows(kap["f32"], vb[0], vb[1], bf16x3=True)
        R.cut_assemble(kap["f32"], vb[0], vb[1])

    step_bf3()
    bf3 = {"rows_ms": timed(lambda: R.assemble_rows(kap["f32"], vb[0], vb[1], bf16x3=True), nrep, torch),
           "step_ms": timed(step_bf3, nrep, torch)}
    step_bf3()
    torch.cuda.synchronize()
    bf3["rel_err_vs_fp64"] = {"mass": row_scaled_err(vb[0], vals["f64"][0], rp, torch),
                              "stiff": row_scaled_err(vb[1], vals["f64"][1], rp, torch)}
    del vb
    # the three schemes the paper compares: conventional Gauss (Ref), Hybrid Gauss (interior
    # rows by WQ, the regular support of cut rows by element Gauss) and DWQ (this path)
    Rh = Rules.from_workload(wl, hybrid_gauss=True)
    schemes = {k: {"ref_gauss_ms": parts[k].get("gauss_ms"), "dwq_ms": parts[k]["step_ms"]} for k in parts}
    for k in ("f64", "f32"):
        vm, vk = vals[k]

        def step_h():
            Rh.assemble_rows(kap[k], vm, vk)
            Rh.cut_assemble(kap[k], vm, vk)

        step_h()
        schemes[k]["hybrid_gauss_ms"] = timed(step_h, nrep, torch)
    del Rh
    # the conventional Gauss matrices formed row by row with sum factorization and no atomics
    # (no weighted quadrature): the same-engineering comparison for the gain of WQ / DWQ
    Rg = Rules.from_workload(wl, gauss_rows=True)
    kg_slots = W.kappa_at(wl, Rg.kappa_xyz())
    for k in ("f64", "f32"):
        vm, vk = vals[k]
        kr = kg_slots.to(dt[k])

        def step_g():
            Rg.assemble_rows(kr, vm, vk)
            Rg.cut_assemble(kr, vm, vk)

        step_g()
        schemes[k]["gauss_rows_ms"] = timed(step_g, nrep, torch)
    del Rg, kg_slots
    # DWQ with the fitted cut-element rule ((2p+1)^3 points per cut element instead of the octree)
    Rf = Rules.from_workload(W.with_cut_rule(wl, "fit"))
    kf_slots = W.kappa_at(wl, Rf.kappa_xyz())
    for k in ("f64", "f32"):
        vm, vk = vals[k]
        kr = kf_slots.to(dt[k])

        def step_f():
            Rf.assemble_rows(kr, vm, vk)
            Rf.cut_assemble(kr, vm, vk)

        step_f()
        schemes[k]["dwq_fit_ms"] = timed(step_f, nrep, torch)
    schemes["fit_kappa_slots"] = {"octree": R.n_kappa, "fit": Rf.n_kappa}
    del Rf, kf_slots
    # the same step through wq_assemble (rows, remainder and the cut elements' element work on
    # three streams, then the gather): bitwise the values of the timed step
    fused = {}
    for k in ("f64", "f32"):
        vm, vk = vals[k]
        R.assemble_fused(kap[k], vm, vk)
        fused[k] = timed(lambda: R.assemble_fused(kap[k], vm, vk), nrep, torch)
    schemes["fused_step_ms"] = fused
    # stiffness with the coefficient tensor of a geometry map (wq_assemble_tensor), beside the
    # scalar stiffness of the same rules; cut elements by the octree and by the fitted rule
    if wl.degree <= 4:
        tens = {}
        for rule in ("octree", "fit"):
            Rt = Rules.from_workload(W.with_cut_rule(wl, rule), tensor=True)
            Cm = W.tensor_components(W.map_tensor(Rt.kappa_xyz()))
            ks = W.kappa_at(wl, Rt.kappa_xyz())
            vt = {}
            for k in ("f64", "f32"):
                Ck = Cm.to(dt[k]).contiguous()
                vk_t = torch.empty(Rt.nnz, dtype=dt[k], device=dev)
                Rt.assemble_tensor(Ck, vk_t)
                vt[k] = vk_t.clone()
                kk = ks.to(dt[k])

                def step_s():
                    Rt.assemble_rows(kk, None, vk_t, which=2)
                    Rt.cut_assemble(kk, None, vk_t, which=2)

                tens.setdefault(rule, {})[k + "_ms"] = timed(lambda: Rt.assemble_tensor(Ck, vk_t), 3, torch)
                tens[rule][k + "_scalar_stiff_ms"] = timed(step_s, 3, torch)
                del vk_t, Ck, kk
            tens[rule]["fp32_rel_err_vs_fp64"] = row_scaled_err(vt["f32"], vt["f64"], Rt.row_ptr(), torch)
            del Rt, Cm, ks, vt
        schemes["tensor_stiffness"] = tens

    # --- rooflines (durations from the timed region) -----------------------------------
    esz = 8 if main_dt == "f64" else 4
    peak = PEAK["fp64_TFLOPs"] if main_dt == "f64" else PEAK["fp32_TFLOPs"]
    P1, NK = wl.degree + 1, 2 * wl.degree + 1
    # rows pass (k_rows_interior + k_rows_cut): every value written once + the kappa grid read once
    rows_bytes = R.nnz * n_mat * esz + R.n_grid * esz
    # a plain coalesced store kernel writing the same byte count: the write rate this GPU
    # reaches in practice, beside the published peak
    probe = torch.empty(n_mat * R.nnz, dtype=dt[main_dt], device=dev)
    probe.fill_(1.0)
    probe_ms = timed(lambda: probe.fill_(0.5), 10, torch)
    write_probe = probe.numel() * probe.element_size() / (probe_ms * 1e-3) / 1e9
    del probe
    rows_kernels = "k_rows_block" if (main_dt == "f32" and wl.degree <= 4) else "k_rows_interior"
    roofs = {"rows": {"bound": "hbm", "kernel": f"{rows_kernels} + k_rows_box + k_rows_zero (wq_assemble_rows)",
                      "achieved": rows_bytes / (timed_ms["rows"] * 1e-3) / 1e9, "peak": PEAK["hbm_GBps"],
                      "unit": "GB/s", "traffic": measured_traffic(("k_rows_block", "k_rows_box", "k_rows_zero"), wl.name,
                                                                  main_dt),
                      "write_probe_GBps": write_probe}}
    roofs["rows"]["frac_of_write_probe"] = roofs["rows"]["achieved"] / write_probe
    # remainder (k_cut_remainder, one launch): per (cut row, remainder element) pair the three
    # sum-factorized stages of mass + stiffness, 2 P1^4 + 3 P1^4 + 3 P1^4 FMA
    rem_flop = 2 * R.n_rem_pairs * 8 * P1 ** 4
    roofs["remainder"] = {"bound": "alu", "kernel": "k_cut_remainder (cut_assemble, remainder part)",
                          "achieved": rem_flop / (timed_ms["remainder"] * 1e-3) / 1e12, "peak": peak,
                          "unit": "TFLOP/s", "traffic": measured_traffic(("k_cut_remainder",), wl.name, main_dt)}
    # cut elements in moment form (k_cut_moments + k_cut_local + k_cut_gather), M + K: moments
    # with direction 3 per leaf P1^3 NK, direction 2 per column P1^2 NK^2, direction 1 per
    # x-group NK^3 P1; then per element and a3: 2 NK^3 P1 + 3 NK^2 P1^3 + 3 NK P1^5
    oct_fma = (R.n_cells * P1 ** 3 * NK + R.n_oct_columns * P1 ** 2 * NK ** 2 + R.n_oct_xgroups * NK ** 3 * P1
               + R.n_cut_elems * P1 * (2 * NK ** 3 * P1 + 3 * NK ** 2 * P1 ** 3 + 3 * NK * P1 ** 5))
    roofs["octree"] = {"bound": "alu", "kernel": "k_cut_moments + k_cut_local + k_cut_gather (cut_assemble, octree part)",
                       "achieved": 2 * oct_fma / (timed_ms["octree"] * 1e-3) / 1e12, "peak": peak, "unit": "TFLOP/s",
                       "traffic": measured_traffic(("k_cut_moments", "k_cut_local", "k_cut_gather"), wl.name, main_dt)}
    for v in roofs.values():
        v["frac"] = v["achieved"] / v["peak"]
    # flop per HBM byte of the counted traffic (where it was measured)
    for name, fl in (("remainder", rem_flop), ("octree", 2 * oct_fma)):
        if roofs[name]["traffic"]:
            roofs[name]["intensity_flop_per_byte"] = fl / roofs[name]["traffic"]
            # fraction of the HBM roof the counted traffic reaches, beside the flop fraction
            roofs[name]["hbm_frac_of_traffic"] = (roofs[name]["traffic"] / (timed_ms[name] * 1e-3) / 1e9 /
                                                  PEAK["hbm_GBps"])
    # neither roof is near for the remainder: its counters (profiles/) show LDS latency
    roofs["remainder"]["limiter"] = "LDS latency between the contraction stages (SQ_WAIT_INST_LDS 34% of wave cycles)"
    # the longest single kernel of a step (rocprofv3 summary in profiles/) is k_cut_remainder
    dominant = "remainder"
    roof = roofs[dominant]

    out = {
        "metric": METRIC, "value": value, "unit": "nnz/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": main_dt, "data": "synthetic",
        "config": {"workload": wl.name, "nel": list(wl.nel), "degree": wl.degree, "domain": domain_text(wl.levelset),
                   "kappa": KAPPA_TEXT[wl.kappa], "matrices": "mass+stiffness",
                   "octree_levels": wl.octree_levels, "n_active": R.n_active, "nnz_per_matrix": R.nnz,
                   "parallelism": "single GPU"},
        "roofline": roof,
        "roofline_rows": roofs["rows"],
        "roofline_octree": roofs["octree"],
        "attainable_fp32_tflops_without_packed_math": 78.6,
        "timed_pass_ms": timed_ms,
        "step_ms_events": step_stats,
        "breakdown_ms": parts,
        "fp32_over_fp64": parts["f64"]["step_ms"] / parts["f32"]["step_ms"],
        "fp32_rows_over_fp64_rows": parts["f64"]["rows_ms"] / parts["f32"]["rows_ms"],
        "adjoint_over_forward": {k: parts[k]["adjoint_ms"] / parts[k]["step_ms"] for k in parts},
        "speedup_vs_gauss_assembly": ({k: parts[k]["gauss_ms"] / parts[k]["step_ms"] for k in parts}
                                      if kg is not None else None),
        "speedup_vs_gauss_rows": {k: schemes[k]["gauss_rows_ms"] / parts[k]["step_ms"] for k in parts},
        "fp32_rel_err_vs_fp64": err32,
        "bf16x3_experiment": bf3,
        "schemes_ms": schemes,
        "build_rules_ms": {"cold": build_cold_ms, "warm": build_ms},
    }
    if not args.skip_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl, args.cpu_rows)
        out["gpu_over_cpu"] = value / out["cpu_baseline"]["value"]
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
