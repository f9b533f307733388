#!/usr/bin/env python3
"""Benchmark: one IPC Newton iteration on one MI355X.

A step is one full pass of the hot path: per-stencil energy / gradient /
projected Hessian, atomic-free BSR assembly, block-Jacobi PCG to 1e-8, and the
feasibility line search.  Every step starts from the same positions (copied on
the device), so every step does the same work.  Workloads:

* ``block40`` (default): 40x40x40-cell block, 384,000 stable Neo-Hookean tets,
  68,921 free vertices, 200k point-triangle + 200k edge-edge barrier stencils
  against a fixed collider, float64;
* ``cloth``: the heterogeneous scene, 300,000 tets + four 250x250 cloth sheets
  (500,000 StVK membrane triangles, 748,000 hinges) + 1M PT/EE/PE/PP contacts
  (40/40/15/5 %), float64;
* ``block80``: 80x80x52-cell block, 1,996,800 tets + 750k PT + 750k EE, run in
  float64 or (``--precision mixed``) in the precision form.

Prints ONE JSON line.  `value` is stencils processed per second of Newton
iteration (Mstencils/s); `ms_per_step` is the Newton-iteration time.  After the
timed steps a profiled pass times every kernel class with HIP events on the
library's stream (the `roofline` object), the contact index is rebuilt a few
times (`contact_index_ms`; `full_ms` = Newton iteration + one rebuild), and the
CPU oracle runs Newton steps (or, on the large workloads, evaluation + assembly)
on a seeded sample of the workload's stencils: the median of five runs on the
host's threads and one run on a single thread (`cpu_baseline`).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

METRIC = "Newton-iter ms (eval+BSR assembly+PCG) at 384k tets; Mstencils/s; HBM % peak"
HBM_PEAK_GBS = 8000.0
FP64_VECTOR_TFLOPS = 78.6

# Algorithmic work per unit:
SNH_FLOPS_PER_TET = 4.0e3        # closed-form F-space eigensystem: 3x3 SVD, 9 rank-one modes, J_F map
# Contacts: distance, barrier and u-space Hessian plus the structured projection
# of the free Hessian over m vertex slots (m = free vertices, or 3 / 2 / 1 for
# all-free PT, EE / PE / PP): PT and EE in the stencil's plane frame (2m x 2m
# eigenproblem: 6x6 Jacobi for m = 3, 4x4 for m = 2, closed form for m = 1), PE
# in the edge frame (2m x 2m + m x m), PP in closed form; calibrated on the
# measured FP64 VALU operations of the kernels
CONTACT_FLOPS = {(0, 3): 1.6e4, (0, 2): 5.5e3, (0, 1): 2.5e3, (1, 3): 1.6e4, (1, 2): 5.5e3, (1, 1): 2.5e3,
                 (2, 2): 5.0e3, (2, 1): 2.5e3, (3, 1): 1.0e3}
MEMBRANE_FLOPS = 6.0e3           # 6x6 F-space Jacobi eigenproblem and the J_F map
HINGE_FLOPS = 3.0e4              # 9x9 Helmert-reduced Jacobi eigenproblem


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def algorithmic(prob, g, view, projected=True, mixed=False):
    """Per-launch algorithmic bytes / flops of each kernel class: what the
    method must move or compute, with staging and re-reads counted against the
    kernel.  The flop models count the eigen-projections; with projected=False
    (exact Hessians, no projection) the evaluation kernels are left
    unmodelled.  mixed: the precision form (float32 BSR values and Krylov
    vectors; float64 positions, gradient, solution and block inverses)."""
    import numpy as np
    n = g.n
    nt = g.nt
    ct = prob["ctype"]
    nnzb = view.nnzb_static + view.nnzb_dynamic + view.nnzb_body
    ci = np.asarray(prob["cidx"]).reshape(-1, 4)
    c_flops = 0.0
    if len(ct):
        nv = np.array([4, 4, 3, 2])[np.asarray(ct)]
        k = ((ci >= 0) & (ci < n)).sum(axis=1)
        m = np.where(k == nv, nv - 1, k)
        for (t, mm), f in CONTACT_FLOPS.items():
            c_flops += f * int(((ct == t) & (m == mm)).sum())
    vb = 36.0 if mixed else 72.0   # bytes of one stored 3x3 block
    vv = 12.0 if mixed else 24.0   # bytes of one vertex of a Krylov vector
    cl_flops = MEMBRANE_FLOPS * len(prob.get("tri_idx", [])) + HINGE_FLOPS * len(prob.get("hinge_idx", []))
    model = {
        "cloth_eval": ("alu", cl_flops, "TFLOP/s"),
        # FP64 ALU bound
        "snh_eval": ("alu", SNH_FLOPS_PER_TET * nt, "TFLOP/s"),
        "contact_eval": ("alu", c_flops, "TFLOP/s"),
        # HBM bound.  Assembly: every stored upper block written once and the
        # gradient written once; reading staged contributions is overhead
        "assemble": ("hbm", vb * nnzb + 24.0 * n, "GB/s"),
        "block_inverse": ("hbm", 2 * 72.0 * n, "GB/s"),
        # values + column index once per stored block, row pointers, u read, w written
        "pcg_spmv": ("hbm", (vb + 4.0) * nnzb + 8.0 * (n + 1) + 2 * vv * n, "GB/s"),
        # p, s, w, u, r (Krylov, vv each), x (24) and M^-1 (72) read; p, s, r, u and x written
        "pcg_update": ("hbm", n * (5 * vv + 24.0 + 72.0 + 4 * vv + 24.0), "GB/s"),
        "inertia": ("hbm", n * (24.0 * 2 + 8.0 + 72.0 + 24.0), "GB/s"),
    }
    if not projected:
        for k in ("cloth_eval", "snh_eval", "contact_eval"):
            del model[k]
    return model


def staged_bytes(prob, g, view, mixed=False):
    """Bytes the staged assembly moves: every staged block contribution written
    by the evaluation kernels and read by the segmented sums, every staged
    gradient row likewise, plus the stored blocks and gradient written."""
    import numpy as np
    n = g.n
    vb = 36.0 if mixed else 72.0

    def contributions(idx):  # (upper blocks, gradient rows) one stencil class contributes
        if len(idx) == 0:
            return 0, 0
        k = ((np.asarray(idx) >= 0) & (np.asarray(idx) < n)).sum(axis=1)
        return int((k * (k + 1) // 2).sum()), int(k.sum())

    nb, ng = n if not prob.get("static") else 0, n  # inertia: diagonal block (dynamic form), gradient row
    for key in ("tet_idx", "tri_idx", "hinge_idx", "cidx"):
        b, r = contributions(prob.get(key, []))
        nb, ng = nb + b, ng + r
    nnzb = view.nnzb_static + view.nnzb_dynamic
    return 2 * (vb * nb + 24.0 * ng) + vb * nnzb + 24.0 * n


KERNEL_SOURCES = {"pcg_spmv": "pcg.hip", "pcg_update": "pcg.hip", "assemble": "assembly.hip",
                  "snh_eval": "elastic.hip", "contact_eval": "contact.hip", "cloth_eval": "cloth.hip"}


def measured_traffic(kernel, workload, precision):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (FETCH_SIZE + WRITE_SIZE scaled by a plain copy of known size), or
    None when there is none or the kernel's source changed since it was taken."""
    import hashlib
    here = os.path.dirname(os.path.abspath(__file__))
    path = os.path.join(here, "profiles", f"traffic_{kernel}_{workload}_{precision}.json")
    src = KERNEL_SOURCES.get(kernel)
    if not src or not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    with open(os.path.join(here, "paper_2605_23088_amd", "csrc", src), "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()
    return rec["bytes_per_launch"] if rec.get("source_sha256") == sha else None


# kernel class -> the device kernel's name in rocprofv3 output
KERNEL_NAMES = {"pcg_spmv": "spmv_chunk_kernel", "pcg_update": "pcg_update_kernel"}


def _pmc_rows(d):
    """(kernel name, counter value) per dispatch from a rocprofv3 --pmc CSV directory."""
    import csv
    import glob
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise FileNotFoundError(f"no counter_collection.csv under {d}")
    rows = []
    for fn in files:
        with open(fn, newline="") as f:
            for r in csv.DictReader(f):
                rows.append((r["Kernel_Name"], float(r["Counter_Value"])))
    return rows


def _pmc_sum_per_dispatch(d, prefix):
    vals = [v for name, v in _pmc_rows(d) if prefix + "<" in name or name.endswith(prefix)]
    if not vals:
        raise ValueError(f"no dispatch of {prefix} in {d}")
    # launches that exit at once after convergence carry almost no traffic
    keep = [v for v in vals if v >= 0.1 * max(vals)]
    return sum(keep) / len(keep), len(keep), len(vals)


def traffic_record(spec, dirs, commands):
    """Writes profiles/traffic_<kernel>_<workload>_<precision>.json from four
    rocprofv3 --pmc runs: FETCH_SIZE and WRITE_SIZE of the workload, then of the
    plain copy of --copy-calibration-mb (the factors that turn KiB into bytes)."""
    import hashlib
    kernel, workload, precision = spec.split(":")
    prefix = KERNEL_NAMES[kernel]
    fetch, nf, tf = _pmc_sum_per_dispatch(dirs[0], prefix)
    write, nw, tw = _pmc_sum_per_dispatch(dirs[1], prefix)
    cf = max(v for name, v in _pmc_rows(dirs[2]) if "copyBuffer" in name)
    cw = max(v for name, v in _pmc_rows(dirs[3]) if "copyBuffer" in name)
    cal_bytes = None
    for c in commands:
        if "--copy-calibration-mb" in c:
            cal_bytes = int(c.split("--copy-calibration-mb")[1].split()[0]) << 20
    ff, wf = cal_bytes / 1024.0 / cf, cal_bytes / 1024.0 / cw
    here = os.path.dirname(os.path.abspath(__file__))
    with open(os.path.join(here, "paper_2605_23088_amd", "csrc", KERNEL_SOURCES[kernel]), "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()
    rec = {"kernel": kernel, "workload": workload, "precision": precision, "device_kernel": prefix,
           "fetch_kib_per_launch": fetch, "write_kib_per_launch": write,
           "copy_calibration": {"bytes": cal_bytes, "fetch_kib": cf, "write_kib": cw, "fetch_factor": ff,
                                "write_factor": wf},
           "bytes_per_launch": 1024.0 * (ff * fetch + wf * write),
           "launches_averaged": min(nf, nw), "launches_traced": max(tf, tw),
           "note": "launches that exit at once after convergence (counters under 10 % of the largest) are excluded",
           "commands": list(commands), "source_sha256": sha}
    out = os.path.join(here, "profiles", f"traffic_{kernel}_{workload}_{precision}.json")
    with open(out, "w") as f:
        json.dump(rec, f, indent=1)
        f.write("\n")
    print(json.dumps({"written": out, "bytes_per_launch": rec["bytes_per_launch"]}))


VALU_F64 = ("SQ_INSTS_VALU_ADD_F64", "SQ_INSTS_VALU_MUL_F64", "SQ_INSTS_VALU_FMA_F64", "SQ_INSTS_VALU_TRANS_F64")


def valu_record(workload, pmc_dir, command):
    """Writes profiles/valu_<workload>.json from one rocprofv3 --pmc run of the
    four FP64 VALU instruction counters: per kernel, the FP64 operations per
    dispatch, 64 lanes x (ADD + MUL + TRANS + 2 FMA) wave instructions (an
    upper bound: inactive lanes count), and the kernel's registers, scratch
    and LDS from the same records."""
    import csv
    import glob
    files = glob.glob(os.path.join(pmc_dir, "**", "*counter_collection.csv"), recursive=True)
    per = {}
    for fn in files:
        with open(fn, newline="") as f:
            for r in csv.DictReader(f):
                name = r["Kernel_Name"]
                short = name.replace("void ", "").replace("yasps::(anonymous namespace)::", "").replace("yasps::", "")
                short = short[:short.index("(")] if "(" in short else short
                k = per.setdefault(short, {"dispatches": set(), "counts": {c: 0.0 for c in VALU_F64},
                                           "vgpr": int(r["VGPR_Count"]), "agpr": int(r["Accum_VGPR_Count"]),
                                           "scratch_bytes": int(r["Scratch_Size"]),
                                           "lds_bytes": int(r["LDS_Block_Size"]), "grid": int(r["Grid_Size"])})
                k["dispatches"].add(r["Dispatch_Id"])
                if r["Counter_Name"] in k["counts"]:
                    k["counts"][r["Counter_Name"]] += float(r["Counter_Value"])
    out = {}
    for name, k in per.items():
        nd = len(k["dispatches"])
        c = {n: v / nd for n, v in k["counts"].items()}
        flops = 64.0 * (c["SQ_INSTS_VALU_ADD_F64"] + c["SQ_INSTS_VALU_MUL_F64"] + c["SQ_INSTS_VALU_TRANS_F64"] +
                        2.0 * c["SQ_INSTS_VALU_FMA_F64"])
        if flops == 0.0:
            continue
        out[name] = {"dispatches": nd, "fp64_ops_per_dispatch": flops, "wave_instructions_per_dispatch": c,
                     "vgpr": k["vgpr"], "agpr": k["agpr"], "scratch_bytes": k["scratch_bytes"],
                     "lds_bytes": k["lds_bytes"], "grid": k["grid"]}
    here = os.path.dirname(os.path.abspath(__file__))
    path = os.path.join(here, "profiles", f"valu_{workload}.json")
    with open(path, "w") as f:
        json.dump({"workload": workload, "command": command, "kernels": out}, f, indent=1)
        f.write("\n")
    print(json.dumps({"written": path, "kernels": len(out)}))


def n_stencils(prob):
    return (prob["tet_idx"].shape[0] + prob["ctype"].shape[0] + len(prob.get("tri_idx", [])) +
            len(prob.get("hinge_idx", [])))


def subsample(prob, frac, seed=1):
    """Every stencil class thinned to a seeded fraction (same vertices)."""
    import numpy as np
    rng = np.random.default_rng(seed)
    q = dict(prob)

    def pick(n):
        return np.sort(rng.choice(n, max(1, int(n * frac)), replace=False))

    k = pick(prob["tet_idx"].shape[0])
    q["tet_idx"], q["dm_inv"], q["vol"] = prob["tet_idx"][k], prob["dm_inv"][k], prob["vol"][k]
    for key in ("mu_t", "lam_t", "theta"):  # per-tet parameters
        if key in prob:
            q[key] = prob[key][k]
    k = pick(prob["ctype"].shape[0])
    q["ctype"], q["cidx"] = prob["ctype"][k], prob["cidx"][k]
    if len(prob.get("tri_idx", [])):
        k = pick(len(prob["tri_idx"]))
        q["tri_idx"], q["tri_dm_inv"], q["tri_area"] = prob["tri_idx"][k], prob["tri_dm_inv"][k], prob["tri_area"][k]
        k = pick(len(prob["hinge_idx"]))
        q["hinge_idx"], q["hinge_rest"] = prob["hinge_idx"][k], prob["hinge_rest"][k]
    return q


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline(prob, frac=1.0, solve=True, runs=5):
    """The oracle on a seeded fraction of the workload's stencils (host cores):
    one Newton step (eval + assembly + PCG to 1e-8 + line search), or with
    solve=False only the evaluation and assembly.  Median of `runs` runs on
    torch's thread count, then one run on a single thread."""
    import numpy as np
    import torch
    from oracle import assemble as oasm
    from oracle import newton as onewton
    q = prob if frac >= 1.0 else subsample(prob, frac)
    t0 = time.perf_counter()
    o = oasm.Oracle(q)
    t1 = time.perf_counter()
    ns = n_stencils(q)
    log(f"[bench] oracle set up in {t1 - t0:.1f} s; {'Newton step' if solve else 'eval + assembly'} on {ns} stencils")

    def once():
        t = time.perf_counter()
        if solve:
            _, info = onewton.newton_step(o, q["x0"], rtol=1e-8)
        else:
            o.assemble(o.eval(q["x0"]))
            info = {}
        return time.perf_counter() - t, info

    threads = torch.get_num_threads()
    ts, info = [], {}
    for _ in range(runs):
        dt, info = once()
        ts.append(dt)
    torch.set_num_threads(1)
    try:
        t_single, _ = once()
    finally:
        torch.set_num_threads(threads)
    med = float(np.median(ts))
    log(f"[bench] oracle median {med:.2f} s over {runs} runs ({threads} threads), {t_single:.2f} s on 1 thread")
    what = (f"one Newton step (eval + assembly + PCG to 1e-8 + line search, {info['cg_iters']} PCG iterations)"
            if solve else "evaluation + assembly only (the PCG takes thousands of iterations here)")
    part = "the full workload" if frac >= 1.0 else f"a seeded {frac:g} fraction of every stencil class"
    return {"value": ns / med / 1e6, "unit": "Mstencils/s", "cores": threads, "kind": "oracle",
            "sample": f"{part} ({ns} stencils): {what}; median of {runs} runs {med:.2f} s "
                      f"(runs {', '.join(f'{t:.2f}' for t in ts)} s), pattern set-up {t1 - t0:.2f} s excluded",
            "single_thread": {"value": ns / t_single / 1e6, "unit": "Mstencils/s", "seconds": t_single},
            "cpu_model": cpu_model(), "host_logical_cpus": os.cpu_count()}


def kernel_table(stats, model, steps, cg_work, workload, precision):
    """Per-kernel-class launches, average device time and roofline position
    from the profiler's statistics over `steps` profiled steps that ran
    `cg_work` PCG iterations in all; the roofline entry is the class with the
    largest time that has a work model."""
    kernels = {}
    for name, st in stats.items():
        if not st["launches"]:
            continue
        avg_ms = st["total_ms"] / st["launches"]
        if name in ("pcg_spmv", "pcg_update") and cg_work > 0:
            avg_ms = st["total_ms"] / cg_work
        k = {"launches_per_step": st["launches"] / steps, "avg_ms": avg_ms, "ms_per_step": st["total_ms"] / steps}
        if name in model:
            bound, work, unit = model[name]
            rate = work / (avg_ms * 1e-3)
            if bound == "hbm":
                k.update(bound="hbm", achieved=rate / 1e9, peak=HBM_PEAK_GBS, unit="GB/s",
                         frac=rate / 1e9 / HBM_PEAK_GBS, algorithmic_bytes=work)
            else:
                k.update(bound="alu", achieved=rate / 1e12, peak=FP64_VECTOR_TFLOPS, unit="TFLOP/s",
                         frac=rate / 1e12 / FP64_VECTOR_TFLOPS, algorithmic_flops=work)
        kernels[name] = k
    dom = max((n for n in kernels if "bound" in kernels[n]), key=lambda n: kernels[n]["ms_per_step"])
    d = kernels[dom]
    roofline = {"kernel": dom, "bound": d["bound"], "achieved": d["achieved"], "peak": d["peak"],
                "unit": d["unit"], "frac": d["frac"], "traffic": measured_traffic(dom, workload, precision)}
    return kernels, roofline


def bench_static(args):
    """Differentiation form on the 48x48x29-cell static block (400,896 tets,
    bottom rim fixed, per-tet Young's moduli, 300k PT stencils): the forward
    equilibrium solve from x0 (Newton to max|g| <= 1e-9 of the weight scale)
    and the backward pass (adjoint PCG on the exact Hessian + per-tet mixed
    partials), each timed end to end after one untimed warm-up pair; then one
    profiled backward pass for the per-kernel table."""
    import numpy as np
    import torch

    from paper_2605_23088_amd import synth
    from paper_2605_23088_amd.adjoint import StaticEquilibrium

    log("[bench] generating the static workload")
    prob = synth.c5_static()
    s = StaticEquilibrium(prob, gtol=1e-9, verbose=True)
    theta = torch.as_tensor(prob["theta"], dtype=torch.float64, device="cuda")
    x0 = torch.as_tensor(prob["x0"], dtype=torch.float64, device="cuda").contiguous()
    xt = torch.as_tensor(prob["x_tgt"], dtype=torch.float64, device="cuda")
    s.set_theta(theta)
    fw, bw, iters, cg = [], [], [], []
    for k in range(1 + max(1, args.steps)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        xs = s.solve(x0)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        g, lam = s.adjoint(xs, theta, 2.0 * (xs - xt))
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        log(f"[bench] static pass {k}: forward {t1 - t0:.3f} s in {s.newton_iters} Newton steps "
            f"({s.cg_iters} PCG iterations), backward {t2 - t1:.3f} s ({s.adjoint_info['iters']} PCG iterations)")
        if k > 0:
            fw.append(t1 - t0)
            bw.append(t2 - t1)
            iters.append(s.newton_iters)
            cg.append(s.cg_iters)
    n_it = float(np.mean(iters))
    ms_iter = 1e3 * float(np.mean(fw)) / n_it

    kernels, roofline = {}, None
    if args.profiled_steps > 0:
        s.lib.profile(True)
        s.adjoint(xs, theta, 2.0 * (xs - xt))
        stats = s.lib.profile_stats()
        s.lib.profile(False)
        kernels, roofline = kernel_table(stats, algorithmic(prob, s.lib, s.lib.view(), projected=False), 1,
                                         float(s.adjoint_info["iters"]), "static", "fp64")

    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] CPU oracle baseline")
        cpu = cpu_baseline(prob, 0.125, False)

    stencils = n_stencils(prob)
    line = {
        "metric": METRIC,
        "value": stencils / (ms_iter / 1000.0) / 1e6,
        "unit": "Mstencils/s",
        "n_gpus": 1,
        "steps": len(fw),
        "warmup": 1,
        "ms_per_step": ms_iter,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"static 48x48x29-cell block, {len(prob['tet_idx'])} tets with per-tet moduli, "
                               f"{len(prob['ctype'])} PT stencils, bottom rim fixed; equilibrium to max|g| <= "
                               "1e-9 m g_max, then the adjoint of L = |x* - x_tgt|^2",
                   "tets": len(prob["tet_idx"]), "contacts": len(prob["ctype"]),
                   "free_vertices": int(prob["n_free"])},
        "forward_s": float(np.mean(fw)),
        "newton_iters": n_it,
        "newton_iter_ms": ms_iter,
        "forward_pcg_iters": float(np.mean(cg)),
        "backward_ms": 1e3 * float(np.mean(bw)),
        "backward_pcg_iters": int(s.adjoint_info["iters"]),
        "roofline": roofline,
        "kernels": kernels,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


def frames_cpu_baseline(runs=3):
    """The oracle's time stepping on a small drop scene (3x3x2 cells), timed
    per frame: the oracle as it stands (brute-force pair search in Python),
    median over the first frames with contact."""
    import numpy as np
    from oracle import collision as ocol
    from oracle import timestep as ots
    from paper_2605_23088_amd import synth
    p = synth.drop_scene()
    S = ocol.Surface(p["surf_points"], p["surf_edges"], p["surf_tris"], p["n_free"], p["surf_len2"])
    st = ots.Stepper(p, S)
    x, v = p["x0"], p["v0"]
    ts = []
    for _ in range(runs):
        t0 = time.perf_counter()
        x, v, info = st.frame(x, v)
        ts.append(time.perf_counter() - t0)
    med = float(np.median(ts))
    import torch
    return {"value": 1.0 / med, "unit": "frames/s", "cores": torch.get_num_threads(), "kind": "oracle",
            "sample": f"the 3x3x2-cell drop scene ({len(p['tet_idx'])} tets): median of {runs} frames "
                      f"({', '.join(f'{t:.2f}' for t in ts)} s)"}


def bench_frames(args):
    """Time stepping with contact: a free Kuhn block (rest shape, falling at
    1 m/s) landing on a fixed, rotated ground grid; every frame runs Newton
    iterations with a proximity search per iterate and per line-search trial,
    the CCD step bound, and the stop rule max|p|/h < 1e-2 m/s.  Timed: K
    frames after W warm-up frames (the block is already in contact when the
    timed frames start)."""
    import numpy as np
    import torch

    from paper_2605_23088_amd import synth
    from paper_2605_23088_amd.yasps import Yasps

    c = args.cells
    nz = max(2, c // 2)
    log(f"[bench] generating the drop scene {c}x{c}x{nz}")
    a = 1.0 / c
    p = synth.drop_scene(nx=c, ny=c, nz=nz, a=a, gap=0.2 * a, ground_cells=int(1.25 * c), ground_size=1.5,
                         kappa=1e4, dhat=(0.4 * a) ** 2)
    g = Yasps(p, contacts=False)
    g.set_surface(p["surf_points"], p["surf_edges"], p["surf_tris"], p["surf_len2"], p["cell"])
    x = torch.as_tensor(p["x0"], dtype=torch.float64, device="cuda").contiguous()
    v = torch.as_tensor(p["v0"], dtype=torch.float64, device="cuda").contiguous()
    for k in range(args.warmup):
        info = g.frame(x, v)
        log(f"[bench] warm-up frame {k}: {info['newton_iters']} Newton, {info['cg_iters']} PCG, "
            f"{info['n_contacts_max']} contacts")
    torch.cuda.synchronize()
    infos = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        infos.append(g.frame(x, v))
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / args.steps
    log(f"[bench] {args.steps} frames: {ms:.2f} ms per frame")
    mean = lambda k: float(np.mean([i[k] for i in infos]))
    cpu = None if args.no_cpu_baseline else frames_cpu_baseline()
    line = {
        "metric": "time-stepping frames/s (IPC frame: proximity search + Newton + CCD line search)",
        "value": 1e3 / ms,
        "unit": "frames/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{c}x{c}x{nz}-cell Kuhn block ({len(p['tet_idx'])} tets) dropped on a "
                               f"{int(1.25 * c)}^2-cell rotated ground; h = {p['h']}, dhat = {p['dhat']:.3g}, "
                               f"kappa = {p['kappa']:.3g}",
                   "tets": len(p["tet_idx"]), "free_vertices": int(p["n_free"]),
                   "surface_points": len(p["surf_points"]), "surface_edges": len(p["surf_edges"]),
                   "surface_triangles": len(p["surf_tris"])},
        "newton_iters_per_frame": mean("newton_iters"),
        "pcg_iters_per_frame": mean("cg_iters"),
        "ls_trials_per_frame": mean("ls_trials"),
        "contacts_max": int(max(i["n_contacts_max"] for i in infos)),
        "phases_ms_per_frame": {k: mean("ms_" + k) for k in ("detect", "newton", "ccd", "linesearch")},
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--profiled-steps", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-index-timing", dest="index_timing", action="store_false",
                    help="skip timing the contact index rebuild (device and host builds)")
    ap.add_argument("--cells", type=int, default=40, help="block size of the block40 workload")
    ap.add_argument("--workload", choices=["block40", "cloth", "block80", "static", "frames"], default="block40")
    ap.add_argument("--precision", choices=["fp64", "mixed"], default="fp64")
    ap.add_argument("--permute", action="store_true",
                    help="relabel the free vertices by a seeded random permutation (block and cloth workloads)")
    ap.add_argument("--copy-calibration-mb", type=int, default=0,
                    help="only run 5 device-to-device copies of this many MiB (the reference kernel that scales "
                         "rocprofv3 FETCH_SIZE / WRITE_SIZE counters to bytes) and exit")
    ap.add_argument("--traffic-record", metavar="KERNEL:WORKLOAD:PRECISION",
                    help="summarise four rocprofv3 --pmc runs (--pmc-dirs) into the profiles/ traffic record and "
                         "exit (no GPU use)")
    ap.add_argument("--pmc-dirs", nargs="+", metavar="DIR",
                    help="counter directories: FETCH, WRITE, COPY_FETCH, COPY_WRITE (--traffic-record) or one "
                         "(--valu-record)")
    ap.add_argument("--pmc-commands", nargs="+", help="the rocprofv3 commands, recorded with the summary")
    ap.add_argument("--valu-record", metavar="WORKLOAD",
                    help="summarise one rocprofv3 --pmc run of the FP64 VALU counters (--pmc-dirs DIR, "
                         "--pmc-commands CMD) into profiles/valu_<workload>.json and exit (no GPU use)")
    args = ap.parse_args()
    if args.valu_record:
        return valu_record(args.valu_record, args.pmc_dirs[0], args.pmc_commands[0])
    if args.traffic_record:
        return traffic_record(args.traffic_record, args.pmc_dirs, args.pmc_commands)
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (the path is not sharded "
              "across GPUs)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    if args.copy_calibration_mb:
        nbytes = args.copy_calibration_mb << 20
        src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": nbytes, "copies": 5}), flush=True)
        return

    from paper_2605_23088_amd import synth
    from paper_2605_23088_amd.yasps import FP64, KERNEL_CLASSES, MIXED, Yasps

    if args.workload == "static":
        return bench_static(args)
    if args.workload == "frames":
        return bench_frames(args)

    log(f"[bench] generating workload {args.workload}")
    cpu_frac, cpu_solve = 0.25, True
    if args.workload == "cloth":
        prob = synth.c3_cloth()
        cpu_frac, cpu_solve = 1.0 / 32, False
        desc = ("heterogeneous scene: 50x50x20-cell tet block + four 250x250 cloth sheets (StVK membranes, "
                "dihedral hinges), 1M PT/EE/PE/PP contacts 40/40/15/5 %")
    elif args.workload == "block80":
        prob = synth.c4_block()
        cpu_frac, cpu_solve = 1.0 / 32, False
        desc = "80x80x52-cell Kuhn block + 750k PT + 750k EE collider stencils"
    elif args.cells == 40:
        prob = synth.c2_block()
        desc = "40x40x40-cell Kuhn block"
    else:
        c = args.cells
        prob = synth.block_problem(c, c, c, 1.0 / c, 200_000 * c ** 3 // 64000, 200_000 * c ** 3 // 64000,
                                   synth.SEEDS["C2"], name=f"C2-{c}")
        desc = f"{c}x{c}x{c}-cell Kuhn block"
    if args.permute:  # seeded random relabelling of the free vertices (no favourable locality)
        prob, _ = synth.permute_vertices(prob)
        desc += " (free vertex ids randomly permuted)"
    nt, nc = prob["tet_idx"].shape[0], prob["ctype"].shape[0]
    nf, nh = len(prob.get("tri_idx", [])), len(prob.get("hinge_idx", []))
    log(f"[bench] {nt} tets, {nf} triangles, {nh} hinges, {prob['n_free']} free vertices, {nc} contacts; "
        "creating context")
    g = Yasps(prob, precision=MIXED if args.precision == "mixed" else FP64)
    x0 = torch.as_tensor(prob["x0"], dtype=torch.float64, device="cuda").contiguous()
    x = x0.clone()
    for i in range(args.warmup):
        x.copy_(x0)
        info = g.newton_step(x)
        log(f"[bench] warmup {i}: cg {info['cg_iters']} alpha {info['alpha']:.4g}")
    torch.cuda.synchronize()
    infos = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        x.copy_(x0)
        infos.append(g.newton_step(x))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1000.0 / args.steps
    log(f"[bench] timed {args.steps} steps: {ms:.3f} ms/step")
    phases = {k: float(np.mean([i[f"ms_{k}"] for i in infos])) for k in ("eval", "assemble", "pcg", "linesearch")}

    # profiled pass: per-kernel-class device time with HIP events on the library stream
    kernels, roofline = {}, None
    view = g.view()
    if args.profiled_steps > 0:
        g.profile(True)
        pinfos = []
        for _ in range(args.profiled_steps):
            x.copy_(x0)
            pinfos.append(g.newton_step(x))
        stats = g.profile_stats()
        g.profile(False)
        # PCG launches that do work: one SpMV and one update per iteration (the
        # last polling batch also issues launches that exit at once)
        cg_work = args.profiled_steps * float(np.mean([i["cg_iters"] for i in pinfos]))
        # counter records are per workload: the block workload at another size has none
        traffic_key = args.workload if args.workload != "block40" or args.cells == 40 else f"block{args.cells}cube"
        if args.permute:
            traffic_key += "_permuted"  # counters are taken per vertex order
        mixed = args.precision == "mixed"
        kernels, roofline = kernel_table(stats, algorithmic(prob, g, view, mixed=mixed), args.profiled_steps,
                                         cg_work, traffic_key, args.precision)
        if "assemble" in kernels:  # the staged design's bytes against the method's minimum
            a = kernels["assemble"]
            a["staged_bytes"] = staged_bytes(prob, g, view, mixed)
            a["staged_to_min_ratio"] = a["staged_bytes"] / a["algorithmic_bytes"]

    # rebuild of the contact index (yasps_set_contacts), outside the timed step:
    # the device build of this context against a host-build context
    index_ms = {}
    if args.index_timing:
        from paper_2605_23088_amd.yasps import INDEX_HOST
        gh = Yasps(prob, precision=MIXED if args.precision == "mixed" else FP64, index_build=INDEX_HOST)
        ct = torch.as_tensor(np.asarray(prob["ctype"], np.int32), device="cuda")
        ci = torch.as_tensor(np.ascontiguousarray(np.asarray(prob["cidx"], np.int32).T), device="cuda")
        for name, ctx in (("device", g), ("host", gh)):
            ts = []
            for _ in range(3):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                ctx.set_contacts_device(ct, ci)  # contact arrays already on the device
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t0)
            index_ms[name] = 1e3 * min(ts)
        gh.close()
        log(f"[bench] contact index rebuild: device {index_ms['device']:.2f} ms, host {index_ms['host']:.2f} ms")

    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] CPU oracle baseline")
        cpu = cpu_baseline(prob, cpu_frac, cpu_solve)

    stencils = n_stencils(prob)
    types = np.bincount(prob["ctype"], minlength=4)
    line = {
        "metric": METRIC,
        "value": stencils / (ms / 1000.0) / 1e6,
        "unit": "Mstencils/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"{desc}: {nt} tets, {nf} membrane triangles, {nh} hinges, "
                               f"{prob['n_free']} free vertices, {types[0]} PT + {types[1]} EE + {types[2]} PE + "
                               f"{types[3]} PP contact stencils; {args.precision.upper()} Newton step, PCG rtol 1e-8",
                   "tets": nt, "triangles": nf, "hinges": nh, "contacts": nc, "free_vertices": int(prob["n_free"]),
                   "nnzb_static": view.nnzb_static, "nnzb_dynamic": view.nnzb_dynamic},
        "newton_iter_ms": ms,
        # the Newton iteration plus a rebuild of the contact index (yasps_set_contacts)
        "full_ms": ms + index_ms["device"] if index_ms else None,
        "phases_ms": phases,
        "pcg_iters": int(np.mean([i["cg_iters"] for i in infos])),
        "line_search_trials": int(np.mean([i["ls_trials"] for i in infos])),
        "roofline": roofline,
        "kernels": kernels,
        "contact_index_ms": index_ms or None,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
