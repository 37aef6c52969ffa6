#!/usr/bin/env python3
"""Benchmark: sign(H_w(mu)) b solves per second on one MI355X.

Headline workload (the configuration the metric is quoted on): 16^4 lattice
(N = 786432), disordered links U = exp(i eps H) with eps = 0.5 stored FP32,
m_w = -1.5, mu = 0.2, the 12 spin-colour point sources of site 0, a shared LR
deflation basis of 40 critical eigenpairs (Eq. 20-22), Krylov size up to 500,
tol 1e-8.  The deflation data is computed once before the timed region (the
paper's initialisation phase, reusable for every source of the operator) and
reported as init_ms.  One step = one lockstep solve of the 12 sources
(osa_apply with max_batch 12): stencil, LR projection, Arnoldi with
Gram-Schmidt, convergence checks with the small sign, assembly.  The "plain"
figure is the same 12 solved one at a time by the single-source FP64 path on
the same context; both must give bitwise equal results.  Inputs are resident
in GPU memory before the timed region starts.

Kernel classes are timed with HIP events on the launching stream on one
launch in PROF_EVERY (all launches are counted); the roofline object reports
the dominant class.  cpu_baseline times the oracle's Eq. 22 (numpy/scipy) on
one source at a fixed Krylov size on the host cores, beside the GPU at the
same fixed size.

Other workloads: --workload dis8 (8^4, eigensolver inside every step),
haar4, haar12 (mixed precision), uneven64, fig1.

Prints one JSON line (see the fields at the end of each workload function).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PROF_EVERY = 16   # event-bracket one launch in 16 of each kernel class in the timed steps
CHECK_EVERY = 25  # convergence checks every 25 Arnoldi steps (fewer far from convergence)
HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, vendor figure
FP64_PEAK_TFLOPS = 78.6   # MI355X FP64, vector and matrix cores (dense)
PROFILES = os.path.join(ROOT, "profiles")

# kernel classes of osa_profile: the kernels behind each, the bound, and the
# rocprofv3 counter summary (FETCH_SIZE / WRITE_SIZE) of the class, if any
CLASS_INFO = {
    "cgs_dot": ("k_dot_partial + k_dot2_partial + k_dot4_partial", "hbm"),
    "cgs_update": ("k_update_* + k_dcgs_* + k_blk_update", "hbm"),
    "stencil": ("k_wilson_h", "hbm"),
    "small_inverse": ("k_gj_*", "alu"),
    "small_gemm": ("k_zgemm_mfma", "mfma"),
}


def measured_traffic(cls, workload):
    """HBM bytes per launch of a kernel class from the committed rocprofv3
    FETCH_SIZE/WRITE_SIZE summary profiles/<cls>_<workload>_hbm_traffic.json
    (scaled by the copy-kernel factors it records).  None when there is no
    summary, or once the kernel source region it records has changed."""
    import hashlib
    path = os.path.join(PROFILES, f"{cls}_{workload}_hbm_traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f)
        for reg in rec["kernel_regions"]:
            with open(os.path.join(ROOT, reg["file"])) as f:
                src = f.read()
            a, b = src.index(reg["from"]), src.index(reg["to"])
            if hashlib.sha256(src[a:b].encode()).hexdigest() != reg["sha256"]:
                return None
    except (OSError, ValueError, KeyError):
        return None
    return rec.get("hbm_bytes_per_launch")


def class_table(profs, steps):
    """Per kernel class, summed over the given osa_profile dicts: launches
    (all), event-timed launches, average duration, estimated total per step,
    algorithmic GB/s and TFLOP/s over the event-timed launches."""
    agg = {}
    for p in profs:
        for k, v in p.items():
            if k == "counters":
                continue
            a = agg.setdefault(k, dict(ms=0.0, bytes=0.0, flops=0.0, launches=0, calls=0))
            for f in ("ms", "bytes", "flops", "launches", "calls"):
                a[f] += v[f]
    out = {}
    for k, a in agg.items():
        if not a["launches"]:
            continue
        avg = a["ms"] / a["launches"]
        out[k] = {"launches_per_step": a["calls"] / steps, "avg_us": avg * 1e3,
                  "ms_per_step": avg * a["calls"] / steps,
                  "GB/s": a["bytes"] / (a["ms"] * 1e-3) / 1e9 if a["ms"] else 0.0,
                  "TFLOP/s": a["flops"] / (a["ms"] * 1e-3) / 1e12 if a["ms"] else 0.0,
                  "bytes_per_launch": a["bytes"] / a["launches"],
                  "flops_per_launch": a["flops"] / a["launches"],
                  "event_timed": a["launches"], "calls": a["calls"]}
    return out


def roofline(table, workload):
    """The roofline object for the dominant class (largest estimated time)."""
    cands = {k: v for k, v in table.items() if k in CLASS_INFO}
    dom = max(cands, key=lambda k: cands[k]["ms_per_step"])
    d = cands[dom]
    kernels, bound = CLASS_INFO[dom]
    if bound == "hbm":
        ach, peak, unit = d["GB/s"], HBM_PEAK_GBS, "GB/s"
    else:
        ach, peak, unit = d["TFLOP/s"], FP64_PEAK_TFLOPS, "TFLOP/s"
    return {"bound": bound, "kernel_class": dom, "kernel": kernels, "achieved": ach,
            "peak": peak, "unit": unit, "frac": ach / peak,
            "traffic": measured_traffic(dom, workload) if bound == "hbm" else None,
            "algorithmic_bytes_per_launch": d["bytes_per_launch"],
            "algorithmic_flops_per_launch": d["flops_per_launch"],
            "avg_launch_us": d["avg_us"], "launches_per_step": d["launches_per_step"],
            "event_timed_launches": d["event_timed"],
            "share_of_step_kernel_time": d["ms_per_step"] / sum(v["ms_per_step"]
                                                                for v in table.values())}


class roctx_range:
    """A named ROCTx range (rocprofv3 --marker-trace records it) around a block;
    a no-op where the ROCTx library is not found."""
    _lib = None

    def __init__(self, name):
        self.name = name.encode()
        if roctx_range._lib is None:
            import ctypes
            roctx_range._lib = False
            for so in ("librocprofiler-sdk-roctx.so.1", "libroctx64.so.4"):
                try:
                    lib = ctypes.CDLL(so)
                    lib.roctxRangePushA.argtypes = [ctypes.c_char_p]
                    roctx_range._lib = lib
                    break
                except OSError:
                    continue

    def __enter__(self):
        if roctx_range._lib:
            roctx_range._lib.roctxRangePushA(self.name)
        return self

    def __exit__(self, *exc):
        if roctx_range._lib:
            roctx_range._lib.roctxRangePop()
        return False


def summarize_trace(trace_dir, out_md):
    """Per-kernel statistics of the dispatches inside the 'timed_steps' ROCTx range
    of a rocprofv3 --kernel-trace --marker-trace run of this benchmark."""
    import csv
    import glob
    import re
    kt = glob.glob(os.path.join(trace_dir, "**", "*kernel_trace.csv"), recursive=True)
    mk = glob.glob(os.path.join(trace_dir, "**", "*marker_api_trace.csv"), recursive=True)
    t0 = t1 = None
    with open(mk[0]) as f:
        for r in csv.DictReader(f):
            if r.get("Function", "").find("timed_steps") >= 0 or \
                    r.get("Operation", "").find("timed_steps") >= 0 or \
                    any("timed_steps" in str(v) for v in r.values()):
                t0, t1 = int(r["Start_Timestamp"]), int(r["End_Timestamp"])
    stats = {}
    with open(kt[0]) as f:
        for r in csv.DictReader(f):
            a, b = int(r["Start_Timestamp"]), int(r["End_Timestamp"])
            if t0 is None or a < t0 or b > t1:
                continue
            name = re.sub(r"\(.*", "", r["Kernel_Name"]).replace("void ", "").replace("osa::", "")
            name = name.replace("HIP_vector_type<double, 2u>", "cd").replace(
                "HIP_vector_type<float, 2u>", "cf")
            st = stats.setdefault(name, [0, 0])
            st[0] += 1
            st[1] += b - a
    tot = sum(v[1] for v in stats.values())
    rows = sorted(stats.items(), key=lambda kv: -kv[1][1])
    lines = ["| kernel | calls | total ms | avg us | % |", "|---|---:|---:|---:|---:|"]
    for name, (n, ns) in rows:
        lines.append(f"| {name} | {n} | {ns / 1e6:.1f} | {ns / n / 1e3:.2f} | "
                     f"{100.0 * ns / tot:.2f} |")
    classes = {}
    for cls, pat in CLASS_KERNELS.items():
        rx = re.compile(pat)
        n = sum(v[0] for k, v in stats.items() if rx.search(k))
        ns = sum(v[1] for k, v in stats.items() if rx.search(k))
        if n:
            classes[cls] = {"dispatches": n, "avg_us": ns / n / 1e3, "total_ms": ns / 1e6}
    with open(out_md, "w") as f:
        f.write("\n".join(lines) + "\n")
    print(json.dumps({"range_ns": [t0, t1], "kernels": len(stats), "classes": classes}, indent=1))


def host_info():
    """nproc, the CPU model and the BLAS thread count of this host."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    blas = None
    try:
        import threadpoolctl
        blas = max([i.get("num_threads", 1) for i in threadpoolctl.threadpool_info()] + [1])
    except Exception:
        pass
    nproc = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    return {"nproc": nproc, "cpu_model": model, "blas_threads": blas}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--eig-prec", choices=["fp64", "fp32"], default="fp64")
    ap.add_argument("--orth", type=int, choices=[0, 1, 2], default=2,
                    help="Arnoldi orthogonalisation of the solves (osa_opts.orth): 0 delayed "
                         "one-step CGS2, 1 plain CGS2, 2 two-step blocks")
    ap.add_argument("--eig-ncv", type=int, default=0,
                    help="eigensolver active block (0: the library default)")
    ap.add_argument("--workload", choices=["dis16", "dis8", "haar4", "uneven64", "fig1", "haar12"],
                    default="dis16",
                    help="dis16 (headline): 16^4, 12 point sources in one lockstep batch; "
                         "dis8: 8^4 with the eigensolver inside every step; "
                         "uneven64: 64 independent instances (6^4/8^4/10^4), solved "
                         "concurrently; "
                         "fig1: the error-vs-Krylov-size study of the results section; "
                         "haar12: 12^4 with FP32 links, FP32 vs FP64 eigensearch")
    ap.add_argument("--counters-sample", action="store_true",
                    help="dis16 kernel-counter sample: one 12-source lockstep solve at the "
                         "headline's Krylov size (fixed k = 225, m = 40 placeholder deflation "
                         "data, no eigensolver), every launch event-timed; prints the class "
                         "table (for rocprofv3 --pmc runs)")
    ap.add_argument("--summarize-counters", nargs=5,
                    metavar=("FETCH_DIR", "WRITE_DIR", "COPY_FETCH_DIR", "COPY_WRITE_DIR",
                             "SAMPLE_JSON"),
                    help="reduce rocprofv3 --pmc outputs of --counters-sample and "
                         "--copy-calibration to profiles/<class>_dis16_hbm_traffic.json")
    ap.add_argument("--with-block", action="store_true",
                    help="dis16: also time the block Krylov variant on the 12 sources")
    ap.add_argument("--summarize-trace", nargs=2, metavar=("TRACE_DIR", "OUT_MD"),
                    help="per-kernel statistics of the timed steps from a rocprofv3 "
                         "--kernel-trace --marker-trace run of this benchmark")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (HBM counter calibration)")
    ap.add_argument("--solve-only", action="store_true",
                    help="only the solves of one instance (eigenpairs computed untimed first)")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched-vs-plain record")
    ap.add_argument("--deflation", choices=["lr", "schur"], default="lr",
                    help="deflation scheme: LR (Eq. 20-22, the default) or Schur (Eq. 13-19)")
    ap.add_argument("--batched-only", action="store_true",
                    help="only the 12-source lockstep batch (eigenpairs computed untimed first)")
    return ap.parse_args()


def copy_calibration():
    """A plain device copy of known size: 1 GiB read + 1 GiB written per launch."""
    import torch
    n = (1 << 30) // 16
    a = torch.ones(n, dtype=torch.complex128, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": n * 16, "copy_bytes_written": n * 16, "launches": 5}))


COUNTER_K = 225   # the headline's Krylov size (k_used of every source)

# kernels behind each profiled class (rocprofv3 kernel names), and the source
# regions whose hash dates a counter summary
CLASS_KERNELS = {
    "cgs_dot": r"k_dot_partial|k_dot2_partial|k_dot4_partial",
    "cgs_update": r"k_update_direct|k_update_split|k_update_finish|k_dcgs_update|k_dcgs_split|"
                  r"k_dcgs_finish|k_blk_update",
    "stencil": r"k_wilson_h",
}
CLASS_REGIONS = {
    "cgs_dot": [("paper_0710_0341_amd/csrc/blas.hip", "static TsPlan dot_plan(",
                 "// ---------------------------------------------------------------- reduce"),
                ("paper_0710_0341_amd/csrc/blas.hip", "// Dots of ncols columns of B with the four vectors",
                 "// Columns o0 .. o0+NO-1")],
    "cgs_update": [("paper_0710_0341_amd/csrc/blas.hip",
                    "// ---------------------------------------------------------------- update",
                    "// ------------------------------------------- shared basis, several vectors"),
                   ("paper_0710_0341_amd/csrc/blas.hip",
                    "// ------------------------------------------------ delayed reorthogonalisation",
                    "// ------------------------------------------- two-step block Arnoldi"),
                   ("paper_0710_0341_amd/csrc/blas.hip", "// Columns o0 .. o0+NO-1",
                    "// Per-problem workspace of the two-step form")],
    "stencil": [("paper_0710_0341_amd/csrc/stencil.hip",
                 "// ------------------------------------------------------------------ stencil",
                 "void launch_wilson_h_contig(")],
}


def counters_sample(args):
    """One 12-source lockstep solve with the headline's shapes, for counter runs."""
    import torch

    import lattice_inputs as LI
    import paper_0710_0341_amd as osa
    w = LI.WORKLOADS[3]
    dims = w["dims"]
    links_np = LI.round_links_fp32(LI.make_links(dims, "disordered", eps=w["eps"], cfg=3, inst=0))
    links = torch.from_numpy(links_np.astype(np.complex64)).to("cuda:0")
    B = torch.from_numpy(point_sources(dims)).to("cuda:0")
    n = B.shape[1]
    r, l, lam = LI.placeholder_deflation(n, w["n_defl"], cfg=3, inst=0)
    k = COUNTER_K
    ctx = osa.Context(links, dims, w["mu"], w["m_w"], k_max=k, check_every=-1,
                      max_batch=B.shape[0], orth=args.orth)
    ctx.set_deflation(torch.from_numpy(np.ascontiguousarray(r.T)).to("cuda:0"),
                      torch.from_numpy(np.ascontiguousarray(l.T)).to("cuda:0"), lam)
    ctx.profile(True, every=1)
    ctx.apply(B, tol=1.0)
    torch.cuda.synchronize()
    table = class_table([ctx.profile_read()], 1)
    ctx.close()
    print(json.dumps({"counters_sample": "dis16_12pt", "k": k, "orth": args.orth, "classes": table}))


def summarize_counters(args):
    """HBM traffic per launch of each class from rocprofv3 --pmc FETCH_SIZE and
    WRITE_SIZE runs of --counters-sample, scaled by the same counters' readings
    for the plain 1 GiB copy of --copy-calibration (bytes per KiB reading)."""
    import csv
    import glob
    import hashlib
    import re
    fetch_dir, write_dir, cf_dir, cw_dir, sample_json = args.summarize_counters

    def rows(d, counter):
        out = []
        for fn in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            with open(fn) as f:
                for r in csv.DictReader(f):
                    if r.get("Counter_Name") == counter:
                        out.append((r["Kernel_Name"], float(r["Counter_Value"]), r["Dispatch_Id"]))
        return out

    def per_dispatch(rs):
        acc = {}
        for name, v, did in rs:   # a counter can come in several rows per dispatch
            key = (did, name)
            acc[key] = acc.get(key, 0.0) + v
        return acc

    cf = per_dispatch(rows(cf_dir, "FETCH_SIZE"))
    cw = per_dispatch(rows(cw_dir, "WRITE_SIZE"))
    copy_f = [v for (d, n), v in cf.items() if "copy" in n.lower()]
    copy_w = [v for (d, n), v in cw.items() if "copy" in n.lower()]
    gib = float(1 << 30)
    fetch_factor = gib / float(np.median(copy_f))    # bytes per unit of FETCH_SIZE
    write_factor = gib / float(np.median(copy_w))
    fetch = per_dispatch(rows(fetch_dir, "FETCH_SIZE"))
    write = per_dispatch(rows(write_dir, "WRITE_SIZE"))
    with open(sample_json) as f:
        sample = json.loads(f.read().strip().splitlines()[-1])
    out = {}
    for cls, pat in CLASS_KERNELS.items():
        rx = re.compile(pat)
        fs = [v for (d, n), v in fetch.items() if rx.search(n)]
        ws = [v for (d, n), v in write.items() if rx.search(n)]
        if not fs or not ws:
            continue
        hbm = (np.sum(fs) * fetch_factor + np.sum(ws) * write_factor) / len(fs)
        alg = sample["classes"][cls]["bytes_per_launch"]
        regions = []
        for fn, a, b in CLASS_REGIONS[cls]:
            with open(os.path.join(ROOT, fn)) as f:
                src = f.read()
            i, j = src.index(a), src.index(b)
            regions.append({"file": fn, "from": a, "to": b,
                            "sha256": hashlib.sha256(src[i:j].encode()).hexdigest()})
        rec = {"kernel_class": cls, "kernels": pat, "workload": "dis16_12pt counters sample "
               f"(12 sources, fixed k = {COUNTER_K}, m = 40)",
               "dispatches": len(fs), "fetch_factor": fetch_factor, "write_factor": write_factor,
               "hbm_bytes_per_launch": float(hbm), "algorithmic_bytes_per_launch": alg,
               "measured_over_algorithmic": float(hbm / alg), "kernel_regions": regions}
        with open(os.path.join(PROFILES, f"{cls}_dis16_hbm_traffic.json"), "w") as f:
            json.dump(rec, f, indent=1)
        out[cls] = rec
    print(json.dumps({k: {"hbm_MB": v["hbm_bytes_per_launch"] / 1e6,
                          "alg_MB": v["algorithmic_bytes_per_launch"] / 1e6,
                          "ratio": v["measured_over_algorithmic"], "dispatches": v["dispatches"]}
                      for k, v in out.items()}, indent=1))


def workload(name):
    import lattice_inputs as LI
    if name == "dis8":
        w = LI.WORKLOADS[1]
        return dict(name="dis8_eps0.6_mw-1.5", dims=w["dims"], kind="disordered", eps=w["eps"],
                    m_w=w["m_w"], mus=list(w["mu"]), ms=list(w["n_defl"]), k_max=w["k_max"],
                    tol=w["tol"], cfg=1)
    w = LI.WORKLOADS[0]
    return dict(name="haar4_mu0.3_mw-1.5", dims=w["dims"], kind="haar", eps=0.0, m_w=w["m_w"],
                mus=[w["mu"]], ms=[w["n_defl"]], k_max=w["k_max"], tol=w["tol"], cfg=0)


def point_sources(dims, site=0):
    """The 12 spin-colour unit sources at one site (boundary layout)."""
    n = 12 * int(np.prod(dims))
    B = np.zeros((12, n), dtype=np.complex128)
    for sc in range(12):
        B[sc, 12 * site + sc] = 1.0
    return B


def batched_vs_plain(osa, ctx, dims, tol, m, reps=1):
    """12 point sources: one at a time (max_batch 1) vs one lockstep batch."""
    import torch
    B = torch.from_numpy(point_sources(dims)).to("cuda:0")
    k_max, eig_prec, ncv = ctx._opts.k_max, ctx._opts.eig_prec, ctx._opts.eig_ncv
    defl, orth = ctx._opts.deflation, ctx._opts.orth
    out = {}
    ys = {}
    for name, mb in (("plain", 1), ("batched", 12)):
        ctx.set_opts(k_max=k_max, check_every=50, max_batch=mb, eig_prec=eig_prec, eig_ncv=ncv,
                     deflation=defl, orth=orth)
        ctx.set_active_deflation(m)
        ctx.apply(B, tol=tol)            # warm-up (workspace growth)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            y, infos, st = ctx.apply(B, tol=tol)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        ys[name] = y
        out[name] = {"solves_per_s": 12.0 / dt, "ms": dt * 1e3, "status": int(st),
                     "k_used": [i["k_used"] for i in infos],
                     "max_resid_est": max(i["resid_est"] for i in infos)}
    ctx.set_opts(k_max=k_max, check_every=50, eig_prec=eig_prec, eig_ncv=ncv, deflation=defl,
                 orth=orth)
    out["speedup"] = out["batched"]["solves_per_s"] / out["plain"]["solves_per_s"]
    out["bitwise_equal"] = bool(torch.equal(ys["plain"], ys["batched"]))
    out["sources"] = "12 spin-colour point sources at site 0"
    out["mu"], out["n_defl"], out["tol"] = ctx.mu, m, tol
    return out


def uneven_batch(args):
    """64 independent instances with lattices from {6^4, 8^4, 10^4}, random mu,
    m_w, eps and 8-32 deflated pairs, one Gaussian source each.  Deflation runs
    on 8 host threads (one stream per instance), then one osa_batch_apply solves
    all 64 concurrently; the same 64 solved one after another give the
    sequential reference (results must agree bitwise)."""
    import threading
    import torch

    import lattice_inputs as LI
    import paper_0710_0341_amd as osa
    w = LI.WORKLOADS[4]
    params = LI.uneven_batch_params(64)
    ctxs, srcs = [], []
    for p in params:
        links = LI.make_links(p["dims"], "disordered", eps=p["eps"], cfg=4, inst=p["inst"])
        b = LI.gaussian_source(p["dims"], cfg=4, inst=p["inst"])
        ctxs.append(osa.Context(torch.from_numpy(links).to("cuda:0"), p["dims"], p["mu"], p["m_w"],
                                k_max=w["k_max"], check_every=50, orth=args.orth,
                                stream=torch.cuda.Stream()))
        srcs.append(torch.from_numpy(b).to("cuda:0"))
    torch.cuda.synchronize()
    eig_ms = [0.0] * len(ctxs)
    defl_err = [0] * len(ctxs)
    defl_msg = [""] * len(ctxs)
    nxt = [0]
    lock = threading.Lock()

    def deflate_worker():
        while True:
            with lock:
                i = nxt[0]
                nxt[0] += 1
            if i >= len(ctxs):
                return
            t0 = time.perf_counter()
            try:
                ctxs[i].deflate(params[i]["n_defl"])
            except osa.OsaError as e:      # the instance is then solved without deflation
                defl_err[i] = e.status
                defl_msg[i] = str(e)
            eig_ms[i] = (time.perf_counter() - t0) * 1e3
            print(f"deflated instance {i} {params[i]['dims']} m={params[i]['n_defl']}: "
                  f"{eig_ms[i]:.0f} ms status {defl_err[i]}", file=sys.stderr, flush=True)

    t0 = time.perf_counter()
    th = [threading.Thread(target=deflate_worker) for _ in range(8)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    t_defl = time.perf_counter() - t0
    print("batch warm-up", file=sys.stderr, flush=True)
    for _ in range(2):   # workspace growth, dot autotuning, then recording of segment graphs
        osa.batch_apply(ctxs, srcs, tol=w["tol"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ys, infos, st = osa.batch_apply(ctxs, srcs, tol=w["tol"])
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    print("sequential reference", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    seq = [c.apply(b, tol=w["tol"])[0] for c, b in zip(ctxs, srcs)]
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t0
    lat = np.array([i["t_solve_ms"] for i in infos])
    out = {
        "metric": "uneven batch: instances/s and per-instance latency", "unit": "instances/s",
        "value": len(ctxs) / t_batch, "n_gpus": 1, "higher_is_better": True, "data": "synthetic",
        "dtype": "c128",
        "config": {"workload": "uneven64", "instances": len(ctxs), "lattices": "6^4/8^4/10^4",
                   "k_max": w["k_max"], "tol": w["tol"], "concurrent_instances": 8},
        "batch_ms": t_batch * 1e3, "sequential_ms": t_seq * 1e3,
        "speedup_vs_sequential": t_seq / t_batch,
        "bitwise_equal": all(bool(torch.equal(a, b)) for a, b in zip(ys, seq)),
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                       "max": float(lat.max())},
        "statuses": sorted(set(int(i["status"]) for i in infos)),
        "graphs": {"recorded": int(sum(c.graph_stats()[0] for c in ctxs)),
                   "launches": int(sum(c.graph_stats()[1] for c in ctxs))},
        "k_used": {"min": int(min(i["k_used"] for i in infos)),
                   "max": int(max(i["k_used"] for i in infos))},
        "deflation": {"wall_ms": t_defl * 1e3, "host_threads": 8,
                      "per_instance_ms_p50": float(np.percentile(eig_ms, 50)),
                      "per_instance_ms_p99": float(np.percentile(eig_ms, 99)),
                      "failed": [{"inst": i, "status": e, "message": defl_msg[i],
                                  "dims": params[i]["dims"],
                                  "n_defl": params[i]["n_defl"], "m_w": params[i]["m_w"],
                                  "mu": params[i]["mu"]} for i, e in enumerate(defl_err) if e]},
    }
    print(json.dumps(out), flush=True)
    for c in ctxs:
        c.close()


CPU_SAMPLE_K = 30   # Krylov size of the oracle's timed sample at 16^4 (~10-30 s of host work)


def cpu_baseline_fixed_k(dims, links_np, mu, m_w, m, b, k, links_dev, cfg):
    """The oracle's Eq. 22 (CGS2 Arnoldi with the oblique re-projection, Newton
    small sign, assembly) on one source at the fixed Krylov size k, with an
    m-pair deflation of the workload's shape (placeholder vectors from the
    seeded generator: the timing does not depend on their values), on the host
    cores.  The GPU runs the same fixed-k sample on the same inputs beside it.
    The sparse H is assembled before timing."""
    import torch

    import lattice_inputs as LI
    import oracle as O
    import paper_0710_0341_amd as osa
    n = b.shape[0]
    h = O.hermitian_wilson_sparse(links_np, dims, mu, m_w)
    r, l, lam = LI.placeholder_deflation(n, m, cfg=cfg, inst=0)
    defl = O.Deflation(r, l, lam)
    t0 = time.perf_counter()
    y_cpu, _ = O.lr_arnoldi_sign(lambda x: h @ x, b, defl, k=k)
    t_cpu = time.perf_counter() - t0
    ctx = osa.Context(links_dev, dims, mu, m_w, k_max=k, check_every=-1)
    ctx.set_deflation(torch.from_numpy(np.ascontiguousarray(r.T)).to("cuda:0"),
                      torch.from_numpy(np.ascontiguousarray(l.T)).to("cuda:0"), lam)
    bd = torch.from_numpy(b).to("cuda:0")
    ctx.apply(bd, tol=1.0)                     # workspace growth
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    y_gpu, _, _ = ctx.apply(bd, tol=1.0)
    torch.cuda.synchronize()
    t_gpu = time.perf_counter() - t0
    diff = float(np.linalg.norm(y_gpu.cpu().numpy() - y_cpu) / np.linalg.norm(y_cpu))
    ctx.close()
    hi = host_info()
    lat = "x".join(str(d) for d in dims)
    return {"value": 1.0 / t_cpu, "unit": f"solves/s at fixed k={k} (one source)",
            "cores": hi["blas_threads"] or hi["nproc"], "kind": "oracle",
            "sample": f"oracle Eq. 22 on one source at {lat}, k={k} fixed, m={m} placeholder "
                      f"deflation, {t_cpu:.1f} s; sparse matvec single-threaded, dense BLAS on "
                      f"{hi['blas_threads']} threads",
            "host": hi, "seconds": t_cpu,
            "gpu_same_sample": {"seconds": t_gpu, "solves_per_s": 1.0 / t_gpu,
                                "rel_diff_vs_oracle": diff}}


def headline16(args):
    """The headline: 12 point sources at 16^4 (FP32-stored links) in one lockstep
    batch, against the same 12 one at a time (the plain single-source FP64 GPU
    path), with the deflation data (m = 40, FP64 Krylov-Schur on the FP32-rounded
    links) computed once before the timed region."""
    import torch

    import lattice_inputs as LI
    import paper_0710_0341_amd as osa
    w = LI.WORKLOADS[3]
    dims, tol = w["dims"], w["tol"]
    links_np = LI.round_links_fp32(LI.make_links(dims, "disordered", eps=w["eps"], cfg=3, inst=0))
    links = torch.from_numpy(links_np.astype(np.complex64)).to("cuda:0")   # stored FP32
    B_np = point_sources(dims)
    B = torch.from_numpy(B_np).to("cuda:0")
    nsrc = B.shape[0]
    ctx = osa.Context(links, dims, w["mu"], w["m_w"], k_max=w["k_max"], check_every=CHECK_EVERY,
                      max_batch=nsrc, orth=args.orth)
    torch.cuda.synchronize()
    print("dis16: deflation (40 pairs)", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    dinfo = ctx.deflate(w["n_defl"])
    torch.cuda.synchronize()
    init_ms = (time.perf_counter() - t0) * 1e3
    _, _, lam = ctx.get_deflation(left=False)
    print(f"dis16: deflation {init_ms / 1e3:.1f} s; warm-up", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        ctx.apply(B, tol=tol)
    torch.cuda.synchronize()
    ctx.profile(True, every=PROF_EVERY)
    with roctx_range("timed_steps"):
        t0 = time.perf_counter()
        for i in range(args.steps):
            Y, infos, st = ctx.apply(B, tol=tol)
            print(f"dis16: step {i + 1}/{args.steps}", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
    table = class_table([ctx.profile_read()], args.steps)
    ctx.profile(False)
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    value = nsrc * args.steps / (t1 - t0)
    # the plain single-source path on the same context and sources
    print("dis16: the 12 sources one at a time", file=sys.stderr, flush=True)
    ctx.set_opts(k_max=w["k_max"], check_every=CHECK_EVERY, max_batch=1, orth=args.orth)
    ctx.profile(True, every=PROF_EVERY)
    t0 = time.perf_counter()
    Yp, infp, stp = ctx.apply(B, tol=tol)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    table_plain = class_table([ctx.profile_read()], 1)
    ctx.profile(False)
    bitwise = bool(torch.equal(Y, Yp))
    block = None
    if args.with_block:
        # the block Krylov variant (one Krylov space for the 12 sources; not the paper's
        # method), second of two runs, against the lockstep result
        print("dis16: block Krylov variant", file=sys.stderr, flush=True)
        ctx.set_opts(k_max=w["k_max"], check_every=CHECK_EVERY, max_batch=nsrc, orth=args.orth)
        ctx.apply_block(B, tol=tol, check=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        Yb, infb, stb = ctx.apply_block(B, tol=tol, check=False)
        torch.cuda.synchronize()
        tb = time.perf_counter() - t0
        block = {"solves_per_s": nsrc / tb, "ms": tb * 1e3, "status": int(stb),
                 "dimension": infb[0]["k_used"],
                 "max_resid_est": max(i["resid_est"] for i in infb),
                 "max_rel_diff_vs_lockstep": max(
                     float(torch.linalg.vector_norm(Yb[i] - Y[i]) / torch.linalg.vector_norm(Y[i]))
                     for i in range(nsrc))}
    # accuracy: the same 12 against a tighter solve (tol 1e-12, change rule, k <= 800)
    print("dis16: reference solve at tol 1e-12", file=sys.stderr, flush=True)
    ctx.set_opts(k_max=800, check_every=50, max_batch=nsrc, stop_rule=1)
    Yr, infr, str_ = ctx.apply(B, tol=1e-12)
    torch.cuda.synchronize()
    errs = [float(torch.linalg.vector_norm(Y[i] - Yr[i]) / torch.linalg.vector_norm(Yr[i]))
            for i in range(nsrc)]
    out = {
        "metric": "sign(H_w(\u03bc))\u00b7b solves/sec + HBM GB/s at 1e-8 rel err, batched vs plain",
        "value": value, "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "c128", "data": "synthetic",
        "config": {"workload": "dis16_12pt", "lattice": list(dims), "N": 12 * int(np.prod(dims)),
                   "links": "disordered eps=0.5, stored FP32", "m_w": w["m_w"], "mu": w["mu"],
                   "sources": "12 spin-colour point sources at site 0, one lockstep batch",
                   "n_defl": w["n_defl"], "deflation": "LR (Eq. 20-22), computed once",
                   "k_max": w["k_max"], "tol": tol,
                   "check_every": CHECK_EVERY,
                   "orth": ["delayed one-step CGS2", "plain CGS2", "two-step blocks"][args.orth],
                   "stop_rule": "geometric tail of the checkpoint changes (x2)",
                   "parallelism": "single GPU"},
        "roofline": roofline(table, "dis16"),
        "plain": {"solves_per_s": nsrc / t_plain, "ms": t_plain * 1e3, "status": int(stp),
                  "kernels": table_plain},
        "batched_vs_plain": value / (nsrc / t_plain),
        "bitwise_equal_batched_vs_plain": bitwise,
        "accuracy": {"max_rel_err_vs_tight_solve": max(errs),
                     "tight_solve": {"tol": 1e-12, "k_used": [i["k_used"] for i in infr],
                                     "max_resid_est": max(i["resid_est"] for i in infr),
                                     "status": int(str_)}},
        "init_ms": init_ms,
        "block_krylov_variant": block,
        "whole_path_solves_per_s": nsrc / (init_ms * 1e-3 + ms_per_step * 1e-3),
        "kernels": table,
        "profiling": f"HIP events on one launch in {PROF_EVERY} of each class, on the launching "
                     "stream, inside the timed region; per-step class time = average x launches",
        "solve": {"status": int(st), "k_used": [i["k_used"] for i in infos],
                  "max_resid_est": max(i["resid_est"] for i in infos),
                  "newton_iters": [i["newton_iters"] for i in infos]},
        "deflation": {"eig_matvecs": dinfo["eig_matvecs"], "restarts": dinfo["eig_restarts"],
                      "max_eig_resid": dinfo["max_eig_resid"],
                      "min_abs_re_lambda": dinfo["min_abs_re_lambda"],
                      "count_abs_re_below_0.05": int(np.sum(np.abs(lam.real) < 0.05)),
                      "eigensearch": "FP64 Krylov-Schur on H^2, Rayleigh-Ritz on H"},
    }
    ctx.close()
    if not args.no_cpu_baseline:
        print("dis16: oracle sample on the host", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline_fixed_k(dims, links_np, w["mu"], w["m_w"], w["n_defl"],
                                                   B_np[0], CPU_SAMPLE_K, links, cfg=3)
    print(json.dumps(out), flush=True)


FIG1_LATTICES = [((4, 4, 4, 4), [0, 5, 10, 15, 25]), ((6, 6, 6, 6), [0, 12, 24, 36, 48])]
FIG1_KS = list(range(25, 801, 25))


def mixed12(args):
    """12^4 Haar links stored FP32 (rounded once: that array is the instance),
    m_w = -1.8, mu = 0.3, m = 30, Gaussian source.  The critical pairs from an
    FP32 Krylov-Schur search refined in FP64 and from an all-FP64 search; one
    solve with each (k <= 2000, tol 1e-8), their difference, and the Krylov
    size this operator needs."""
    import torch

    import lattice_inputs as LI
    import paper_0710_0341_amd as osa
    w = LI.WORKLOADS[2]
    dims = w["dims"]
    links = torch.from_numpy(LI.make_links(dims, "haar", cfg=2, inst=0)
                             .astype(np.complex64)).to("cuda:0")
    b = torch.from_numpy(LI.gaussian_source(dims, cfg=2, inst=0)).to("cuda:0")
    kmax = 2000
    out = {"workload": "haar12_fp32links", "lattice": list(dims), "m_w": w["m_w"], "mu": w["mu"],
           "n_defl": w["n_defl"], "tol": w["tol"], "k_max": kmax,
           "deflation": args.deflation}
    scheme = osa.SCHUR if args.deflation == "schur" else osa.LR
    ys = {}
    for name, prec in (("fp32_search", osa.FP32), ("fp64_search", osa.FP64)):
        ctx = osa.Context(links, dims, w["mu"], w["m_w"], k_max=kmax, check_every=50,
                          eig_prec=prec, deflation=scheme)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        dinfo = ctx.deflate(w["n_defl"])
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        y, infos, st = ctx.apply(b, tol=w["tol"], check=False)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        ys[name] = y
        out[name] = {"eig_s": round(t1 - t0, 2), "eig_matvecs": dinfo["eig_matvecs"],
                     "min_abs_re_lambda": dinfo["min_abs_re_lambda"],
                     "max_eig_resid": dinfo["max_eig_resid"], "solve_s": round(t2 - t1, 3),
                     "k_used": infos[0]["k_used"], "resid_est": infos[0]["resid_est"],
                     "status": int(st)}
        print(f"haar12 {name}: eig {t1 - t0:.1f} s, k_used {infos[0]['k_used']}, "
              f"est {infos[0]['resid_est']:.1e}, solve {t2 - t1:.2f} s", file=sys.stderr,
              flush=True)
        ctx.close()
    d = torch.linalg.vector_norm(ys["fp32_search"] - ys["fp64_search"]).item()
    out["rel_diff_fp32_vs_fp64_search"] = d / torch.linalg.vector_norm(ys["fp64_search"]).item()
    print(json.dumps(out))


def fig1_study(args):
    """The convergence study of the results section (Fig. 1): relative error of
    the LR-deflated approximation (Eq. 22) against the Krylov size k, for several
    deflation sizes m, at mu = 0.3 with the source x = (1, ..., 1) on 4^4 and 6^4
    lattices.  Synthetic links (m_w = -1.5) stand in for the paper's gauge
    configurations: Haar-random links, and disordered links (eps = 0.6) whose
    spectrum has fewer eigenvalues near the imaginary axis.  Each point is one fixed-k solve (no convergence check); the
    reference y is the converged solve with the largest m at tol 1e-12.  The m
    values cover the paper's m ~ 0.008 N at 4^4; at 6^4 the eigensolver's limit
    of 48 pairs reaches 0.003 N."""
    import torch

    import lattice_inputs as LI
    import paper_0710_0341_amd as osa
    mu, m_w, eps_target = 0.3, -1.5, 1e-8
    scheme = osa.SCHUR if args.deflation == "schur" else osa.LR
    out = {}
    t_all = time.perf_counter()
    for (dims, ms), (kind, leps) in [(a, b) for b in (("haar", 0.0), ("disordered", 0.6))
                                     for a in FIG1_LATTICES]:
        N = 12 * int(np.prod(dims))
        tag = kind + "_" + "x".join(str(d) for d in dims)
        links = torch.from_numpy(LI.make_links(dims, kind, eps=leps, cfg=5, inst=0)).to("cuda:0")
        x = torch.from_numpy(LI.ones_source(dims)).to("cuda:0")
        ctx = osa.Context(links, dims, mu, m_w, k_max=1500, check_every=25, deflation=scheme)
        dinfo = ctx.deflate(max(ms))
        yref, info, st = ctx.apply(x, tol=1e-12, check=False)
        print(f"fig1 {tag}: m={max(ms)} eigensearch {dinfo['t_init_ms'] / 1e3:.1f} s, reference "
              f"k={info[0]['k_used']} est={info[0]['resid_est']:.1e} status={st}",
              file=sys.stderr, flush=True)
        nref = torch.linalg.vector_norm(yref).item()
        curves = {}
        for m in ms:
            ctx.set_active_deflation(m)
            errs = []
            for k in FIG1_KS:
                ctx.set_opts(k_max=k, check_every=-1, deflation=scheme)
                y, inf, st = ctx.apply(x, tol=1e-12, check=False)
                err = torch.linalg.vector_norm(y - yref).item() / nref if st >= 0 else float("nan")
                errs.append(err)
            curves[m] = errs
            hit = [k for k, e in zip(FIG1_KS, errs) if e <= eps_target]
            print(f"fig1 {tag}: m={m} ({m / N:.4f} N) eps(k={FIG1_KS[-1]})={errs[-1]:.1e} "
                  f"k(1e-8)={hit[0] if hit else None}", file=sys.stderr, flush=True)
            ctx.set_opts(k_max=1500, check_every=25, deflation=scheme)
        ctx.close()
        out[tag] = {"N": N, "m": ms, "k": FIG1_KS,
                    "eps": {str(m): [float("%.3e" % e) for e in curves[m]] for m in ms},
                    "k_at_1e-8": {str(m): next((k for k, e in zip(FIG1_KS, curves[m])
                                                if e <= eps_target), None) for m in ms},
                    "reference": {"m": max(ms), "k": info[0]["k_used"],
                                  "resid_est": info[0]["resid_est"]}}
    print(json.dumps({"study": "fig1_eps_vs_k", "deflation": args.deflation, "mu": mu,
                      "m_w": m_w, "links": "synthetic",
                      "source": "ones", "eps_target": eps_target,
                      "seconds": round(time.perf_counter() - t_all, 1), "lattices": out}))


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              f"(the sign(H) path shards by source and instance; this benchmark covers one GPU)", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration()
        return
    if args.summarize_counters:
        summarize_counters(args)
        return
    if args.summarize_trace:
        summarize_trace(*args.summarize_trace)
        return
    if args.counters_sample:
        counters_sample(args)
        return
    if args.workload == "uneven64":
        uneven_batch(args)
        return
    if args.workload == "dis16":
        headline16(args)
        return
    if args.workload == "fig1":
        fig1_study(args)
        return
    if args.workload == "haar12":
        mixed12(args)
        return
    import torch

    import lattice_inputs as LI
    import paper_0710_0341_amd as osa

    wl = workload(args.workload)
    dims = wl["dims"]
    dev = torch.device("cuda:0")
    links_np = LI.make_links(dims, wl["kind"], eps=wl["eps"], cfg=wl["cfg"], inst=0)
    b_np = LI.gaussian_source(dims, cfg=wl["cfg"], inst=0)
    links = torch.from_numpy(links_np).to(dev)
    b = torch.from_numpy(b_np).to(dev)
    eig_prec = osa.FP32 if args.eig_prec == "fp32" else osa.FP64
    scheme = osa.SCHUR if args.deflation == "schur" else osa.LR
    ctxs = [osa.Context(links, dims, mu, wl["m_w"], k_max=wl["k_max"], check_every=50,
                        eig_prec=eig_prec, eig_ncv=args.eig_ncv, deflation=scheme, orth=args.orth)
            for mu in wl["mus"]]
    mmax = max(wl["ms"])
    records = []

    def step(record):
        for ctx in ctxs:
            ctx.set_links(links)
            dinfo = ctx.deflate(mmax)
            for m in wl["ms"]:
                ctx.set_active_deflation(m)
                y, infos, st = ctx.apply(b, tol=wl["tol"])
                if record:
                    rec = dict(infos[0])
                    rec.update(mu=ctx.mu, m=m, status=int(st), eig_ms=dinfo["t_init_ms"])
                    records.append(rec)

    if args.batched_only:
        ctx = ctxs[-1]
        ctx.deflate(mmax)
        rec = batched_vs_plain(osa, ctx, dims, 1e-8, mmax)
        print(json.dumps({"batched_only": True, **rec}), flush=True)
        return
    if args.solve_only:
        ctx = ctxs[-1]
        ctx.deflate(mmax)
        ctx.set_active_deflation(mmax)
        ctx.apply(b, tol=wl["tol"])
        rec = {"solve_only": True, "mu": ctx.mu, "m": mmax}
        for orth in (0, 1, 2):
            ctx.set_opts(k_max=wl["k_max"], check_every=50, orth=orth, deflation=scheme)
            ctx.set_active_deflation(mmax)
            torch.cuda.synchronize()
            ctx.profile(True)
            t0 = time.perf_counter()
            for _ in range(args.steps):
                _, infos, _ = ctx.apply(b, tol=wl["tol"])
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / args.steps
            prof = ctx.profile_read()
            ctx.profile(False)
            rec[f"orth{orth}"] = {"ms_per_solve": dt * 1e3, "k_used": infos[0]["k_used"],
                                  "newton_iters": infos[0]["newton_iters"],
                                  "classes": {k: (round(v["ms"] / args.steps, 2), v["launches"] // args.steps)
                                              for k, v in prof.items() if k != "counters"},
                                  "counters": prof["counters"]}
        print(json.dumps(rec))
        return
    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    for ctx in ctxs:
        ctx.profile(True, every=PROF_EVERY)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = [ctx.profile_read() for ctx in ctxs]
    for ctx in ctxs:
        ctx.profile(False)

    n_solves = len(wl["mus"]) * len(wl["ms"])
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    value = n_solves * args.steps / (t1 - t0)
    counters = {}
    for p in prof:
        for k, v in p.pop("counters").items():
            counters[k] = counters.get(k, 0) + v // args.steps
    table = class_table(prof, args.steps)
    k_used = [r["k_used"] for r in records]
    init_ms = float(np.mean([r["eig_ms"] for r in records])) if records else 0.0
    solve_ms = float(np.mean([r["t_solve_ms"] for r in records])) if records else 0.0
    out = {
        "metric": "sign(H_w(mu)) b solves/sec + HBM GB/s at 1e-8 rel err, batched vs plain",
        "value": value,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c128" if args.eig_prec == "fp64" else "c128 (eigensearch c64)",
        "data": "synthetic",
        "config": {"workload": wl["name"], "lattice": list(dims), "N": 12 * int(np.prod(dims)),
                   "mu": wl["mus"], "n_defl": wl["ms"], "k_max": wl["k_max"], "tol": wl["tol"],
                   "sources_per_step": n_solves, "deflation": args.deflation,
                   "parallelism": "single GPU"},
        "roofline": roofline(table, "dis8"),
        "kernels": table,
        "profiling": f"HIP events on one launch in {PROF_EVERY} of each class, on the launching "
                     "stream, inside the timed region; class totals = average x launches",
        "counters_per_step": counters,
        "solve": {"k_used": k_used, "max_resid_est": max(r["resid_est"] for r in records),
                  "statuses": [r["status"] for r in records], "init_ms_per_instance": init_ms,
                  "solve_ms_mean": solve_ms,
                  "apply_only_solves_per_s": 1e3 / solve_ms if solve_ms else None,
                  "eig_matvecs": [r["eig_matvecs"] for r in records[:: len(wl["ms"])]],
                  "min_abs_re_lambda": [r["min_abs_re_lambda"] for r in records]},
    }
    if not args.no_batched:
        # the metric's 1e-8 (point sources need k > 600 for the workload's 1e-10)
        out["batched"] = batched_vs_plain(osa, ctxs[-1], dims, 1e-8, mmax)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_fixed_k(dims, links_np, wl["mus"][-1], wl["m_w"],
                                                   mmax, b_np, 120, links, cfg=wl["cfg"])
    print(json.dumps(out), flush=True)
    for ctx in ctxs:
        ctx.close()


if __name__ == "__main__":
    main()
