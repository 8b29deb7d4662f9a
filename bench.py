#!/usr/bin/env python3
"""AIRG benchmark on one MI355X: setup + solve to 1e-10 relative residual.

Workload (default): DG-P1 upwind advection on a 512 x 512 jittered
triangulation, 1,572,864 unknowns, 7,860,224 nonzeros, theta = 1.1 rad,
sigma in {1e-4, 1} on a seeded 16 x 16 block checkerboard (seeded synthetic
input, resident in device memory before timing starts).

A step is one pass of the whole hot path: the full AIRG setup (CF splitting,
extraction, GMRES polynomials, restrictor, prolongator, Galerkin products,
finalisation) followed by the solve to ||b - A x|| <= 1e-10 ||b||.  The
headline form is FP64 flexible GMRES right-preconditioned by an FP32 V-cycle;
plain FP64 AIRG (Richardson, FP64 V-cycle) is timed on the same GPU for the
comparison.  value = seconds per step (lower is better).

Also reported: the roofline of the finest-operator SpMV kernel (event-timed
inside the timed steps) against the 8 TB/s HBM3E peak, and the CPU oracle's
time on the same workload (setup + Richardson, one host core).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "AIRG solve time to 1e-10 rel resid + setup s, FP32-precond/batched vs FP64"


WORKLOADS = ("dg_square_512", "p0_cube_128", "batch48")


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=3)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--workload", default="dg_square_512", choices=WORKLOADS)
    p.add_argument("--size", type=int, default=None, help="override the side of the square/cube workload")
    p.add_argument("--truncate", type=int, default=None, help="truncate_n (p0_cube default 65536)")
    p.add_argument("--rtol", type=float, default=1e-10)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-fp64", action="store_true", help="skip the FP64 comparison form")
    p.add_argument("--sweep-poly", action="store_true",
                   help="only sweep polynomial order x sparsity order (setup + FP32-FGMRES solve per pair)")
    p.add_argument("--opt", action="append", default=[], metavar="KEY=VALUE",
                   help="extra AIRG option for every form and the oracle (e.g. strong_threshold=0.0)")
    p.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                   help="only run a plain device copy of MIB MiB (x5), the reference for HBM byte counters")
    p.add_argument("--record-traffic", nargs=4, metavar=("FETCH_CSV", "WRITE_CSV", "COPY_FETCH_CSV", "COPY_WRITE_CSV"),
                   help="only write the workload's measured HBM traffic per top-SpMV launch into "
                        "profiles/traffic.json from rocprofv3 --pmc counter_collection CSVs")
    return p.parse_args()


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
TOP_KERNEL = "k_spmv_stream<double, double, 0, 1>"
TOP_SPMM = "k_spmm_stream<4, double, double, 0, 1>"


def top_kernel(workload):
    """The roofline kernel: the outer iteration's product with the finest operator(s)."""
    return TOP_SPMM if workload == "batch48" else TOP_KERNEL


def kernel_digest(workload="dg_square_512"):
    """Digest of the source text that defines the timed roofline kernel: the stream SpMV (or, for the
    batch, the persistent stream SpMM and its grid), its constants, the XCD tile order and the choice of
    the finest operator's ordering.  Stored counter readings count only while it is unchanged."""
    import hashlib
    import re
    csr = open(os.path.join(ROOT, "paper_2408_08262_amd", "csrc", "csr.hip")).read()
    com = open(os.path.join(ROOT, "paper_2408_08262_amd", "csrc", "common.hpp")).read()
    if workload == "batch48":
        i = csr.index("__global__ void __launch_bounds__(kStreamRows) k_spmm_stream(")
        j = csr.index("static unsigned persistent_grid(")
        parts = [csr[i:csr.index("\n}\n", i)], csr[j:csr.index("\n}\n", j)]]
    else:
        i = csr.index("__global__ void __launch_bounds__(kStreamRows) k_spmv_stream(")
        parts = [csr[i:csr.index("\n}\n", i)]]
    parts += re.findall(r"constexpr int\w* kStream\w+ = [^;]+;", csr)
    k = com.index("constexpr int kXcds")
    parts.append(com[k:com.index("\n}\n", com.index("xcd_grid", k))])
    if workload != "batch48":
        # which ordering of the finest operator the Arnoldi product runs on (the traffic depends on it)
        sol = open(os.path.join(ROOT, "paper_2408_08262_amd", "csrc", "solve.hip")).read()
        parts.append(sol[sol.index("CsrView top_view("):sol.index("\n", sol.index("CsrView top_view("))])
    return hashlib.sha256("\n".join(parts).encode()).hexdigest()[:16]


def stored_traffic(workload):
    try:
        rec = json.load(open(TRAFFIC_FILE)).get(workload)
    except (OSError, ValueError):
        return None
    if not rec or rec.get("digest") != kernel_digest(workload):
        return None
    return rec["bytes_per_launch"]


def record_traffic(workload, files):
    """Counters are read per dispatch in KiB; each is scaled by the factor that makes the plain copy's
    reading equal the bytes it moves."""
    import csv
    import statistics

    def med(path, name_part):
        vals = [float(r["Counter_Value"]) for r in csv.DictReader(open(path)) if name_part in r["Kernel_Name"]]
        if not vals:
            raise SystemExit("no %s dispatch in %s" % (name_part, path))
        return statistics.median(vals), len(vals)

    kern = top_kernel(workload)
    fetch, nf = med(files[0], kern)
    write, nw = med(files[1], kern)
    cfetch, _ = med(files[2], "vectorized_elementwise_kernel")
    cwrite, _ = med(files[3], "vectorized_elementwise_kernel")
    copy_kib = 1024.0 * 1024.0              # the 1024 MiB calibration copy reads and writes 1 GiB
    fs, ws = copy_kib / cfetch, copy_kib / cwrite
    total = (fetch * fs + write * ws) * 1024.0
    try:
        data = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        data = {}
    data[workload] = {"kernel": kern, "digest": kernel_digest(workload), "dispatches": [nf, nw],
                      "fetch_kib_per_launch": round(fetch, 1), "write_kib_per_launch": round(write, 1),
                      "fetch_scale": round(fs, 4), "write_scale": round(ws, 4),
                      "bytes_per_launch": int(round(total))}
    with open(TRAFFIC_FILE, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
        f.write("\n")
    print(json.dumps({workload: data[workload]}))
    return 0


def roofline_from_timing(airg, workload):
    launches, tbytes, tsec = airg.airg_kernel_timing_read()
    airg.airg_kernel_timing(False)
    if launches == 0:
        return None
    avg = tsec / launches
    bpl = tbytes / launches
    ach = bpl / avg / 1e9
    what = (" (finest operators Y = A X on 4 rhs, the batched FGMRES Arnoldi product)" if workload == "batch48"
            else " (finest-operator y = A x, the FGMRES Arnoldi product)")
    return {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": stored_traffic(workload),
            "kernel": top_kernel(workload) + what,
            "launches": launches, "bytes_per_launch": int(bpl), "avg_launch_us": round(avg * 1e6, 2)}


def parse_opts(items):
    out = {}
    for it in items:
        k, v = it.split("=", 1)
        out[k] = float(v) if any(c in v for c in ".eE") or v in ("inf", "-inf") else int(v)
    return out


def sweep_poly(a, airg, torch):
    """Polynomial order (1..6) against sparsity order (1..3) on one workload: the time of the
    coefficient and assembly phase over all levels, the whole setup, and the solve."""
    from workloads import dg_square
    N = a.size or 512
    P = dg_square(N)
    A = airg.to_device(P.rowptr, P.col, P.val)
    b = torch.as_tensor(P.b, device="cuda")
    rows = []
    for order in range(1, 7):
        for sp in (1, 2, 3):
            if sp > order:
                continue
            opts = airg.default_opts(seed=P.seed, outer=airg.OUTER_FGMRES, precond_precision=32,
                                     poly_order=order, poly_sparsity_order=sp, **parse_opts(a.opt))
            best = None
            for _ in range(2):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                h = airg.airg_setup(*A, opts)
                x, info = airg.airg_solve(h, b, rtol=a.rtol, max_it=300, allow_not_converged=True)
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                st = airg.airg_get_stats(h)
                rec = {"order": order, "sparsity": sp, "iterations": info["iterations"],
                       "converged": info["converged"],
                       "poly_s": round(st["phase_seconds"]["poly"], 4), "setup_s": round(st["setup_seconds"], 4),
                       "solve_s": round(info["seconds"], 4), "step_s": round(t1 - t0, 4),
                       "storage_complexity": round(st["storage_complexity"], 3),
                       "vcycle_bytes_fp32": st["vcycle_bytes_fp32"]}
                del h
                if best is None or rec["step_s"] < best["step_s"]:
                    best = rec
            rows.append(best)
            print(json.dumps(best), flush=True)
    print(json.dumps({"sweep_poly": "dg_square_%d" % N, "rows": rows}), flush=True)
    return 0


def single(a, airg, torch):
    """One problem: setup + solve per step."""
    from workloads import dg_square, p0_cube
    if a.workload == "dg_square_512":
        N = a.size or 512
        P = dg_square(N)
        desc = ("dg_square_%d: DG-P1 upwind advection, %dx%d jittered triangulation, n=%d, nnz=%d, theta=1.1, "
                "sigma {1e-4,1} 16x16 block checkerboard" % (N, N, N, P.n, P.nnz))
        trunc = a.truncate or 0
    else:
        N = a.size or 128
        P = p0_cube(N)
        trunc = a.truncate if a.truncate is not None else 65536
        desc = ("p0_cube_%d: P0 upwind advection, %d^3 cubes x 6 Kuhn tetrahedra, n=%d, nnz=%d, "
                "Omega=(0.5,0.3,0.81)/|.|, sigma=1e-4, truncate_n=%d" % (N, N, P.n, P.nnz, trunc))
    A = airg.to_device(P.rowptr, P.col, P.val)
    b = torch.as_tensor(P.b, device="cuda")
    torch.cuda.synchronize()

    def step(opts):
        h = airg.airg_setup(*A, opts)
        x, info = airg.airg_solve(h, b, rtol=a.rtol, max_it=300)
        st = airg.airg_get_stats(h)
        del h
        return info, st

    extra_opts = parse_opts(a.opt)
    extra_opts.setdefault("use_graph", 1)      # both forms replay a captured V-cycle graph
    opts32 = airg.default_opts(seed=P.seed, outer=airg.OUTER_FGMRES, precond_precision=32, truncate_n=trunc,
                               **extra_opts)
    opts64 = airg.default_opts(seed=P.seed, outer=airg.OUTER_RICHARDSON, precond_precision=64, truncate_n=trunc,
                               **extra_opts)
    for _ in range(a.warmup):
        step(opts32)
    torch.cuda.synchronize()
    airg.airg_kernel_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    runs = [step(opts32) for _ in range(a.steps)]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    roof = roofline_from_timing(airg, a.workload)
    sec = (t1 - t0) / a.steps
    info32, st32 = runs[-1]
    fp64 = None
    if not a.no_fp64:
        step(opts64)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        r64 = [step(opts64) for _ in range(a.steps)]
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        i64, s64 = r64[-1]
        fp64 = {"seconds_per_step": round((t3 - t2) / a.steps, 4), "setup_s": round(s64["setup_seconds"], 4),
                "solve_s": round(i64["seconds"], 4), "iterations": i64["iterations"],
                "rel_residual": i64["rel_residual"], "levels": s64["levels"], "form": "Richardson, FP64 V-cycle"}
    # numeric re-setup (kept splittings and patterns) for an operator with the same pattern and
    # values perturbed by U(0.9, 1.1), then the solve: timed after the timed region, own handle
    import numpy as np
    h = airg.airg_setup(*A, opts32)
    newval = torch.as_tensor(P.val * np.random.default_rng(77).uniform(0.9, 1.1, P.val.shape), device="cuda")
    airg.airg_resetup(h, newval)
    torch.cuda.synchronize()
    r0 = time.perf_counter()
    for _ in range(a.steps):
        airg.airg_resetup(h, newval)
        xr, ir = airg.airg_solve(h, b, rtol=a.rtol, max_it=300)
    torch.cuda.synchronize()
    r1 = time.perf_counter()
    resetup = {"seconds_per_step": round((r1 - r0) / a.steps, 4),
               "resetup_s": round(airg.airg_get_stats(h)["resetup_seconds"], 4),
               "solve_s": round(ir["seconds"], 4), "iterations": ir["iterations"],
               "rel_residual": ir["rel_residual"],
               "form": "numeric re-setup (kept CF splittings and patterns) + FGMRES/FP32, values x U(0.9, 1.1)"}
    del h
    cpu = None
    if not a.no_cpu_baseline:
        import oracle as O
        c0 = time.perf_counter()
        oracle_opts = {k: v for k, v in extra_opts.items() if k != "use_graph"}
        H = O.Hierarchy((P.rowptr, P.col, P.val), O.default_params(seed=P.seed, truncate_n=trunc, **oracle_opts))
        c1 = time.perf_counter()
        _, its, rr = H.richardson(P.b, a.rtol, 300)
        c2 = time.perf_counter()
        cpu = {"value": round(c2 - c0, 3), "unit": "s", "cores": 1, "kind": "oracle",
               "sample": "whole workload: oracle setup (%.2f s) + FP64 Richardson to %.0e (%.2f s, %d its), "
                         "single thread" % (c1 - c0, a.rtol, c2 - c1, its)}
    extra = {"setup_s": round(st32["setup_seconds"], 4), "solve_s": round(info32["seconds"], 4),
             "iterations": info32["iterations"], "rel_residual": info32["rel_residual"], "levels": st32["levels"],
             "complexity": {"grid": round(st32["grid_complexity"], 3),
                            "operator": round(st32["operator_complexity"], 3),
                            "storage": round(st32["storage_complexity"], 3)},
             "phase_seconds": {k: round(v, 4) for k, v in st32["phase_seconds"].items()},
             "vcycle_bytes_fp32": st32["vcycle_bytes_fp32"], "fp64_comparison": fp64, "resetup": resetup}
    cfg = {"workload": desc, "form": "FGMRES(30) FP64 outer + FP32 AIRG V-cycle", "rtol": a.rtol,
           "parallelism": "single GPU"}
    cfg["options"] = extra_opts
    return sec, cfg, "f64 (f32 V-cycle)", roof, cpu, extra


def batched(a, airg, torch):
    """48 independent DG-P1 problems x 4 rhs: batched FP32 form vs sequential FP64."""
    from workloads import batch as batch_problems, concat
    probs = batch_problems()
    rp, ci, val, b, offs, seeds = concat(probs)
    A = airg.to_device(rp, ci, val)
    B = torch.as_tensor(b, device="cuda")
    optsb = airg.default_opts(outer=airg.OUTER_FGMRES, precond_precision=32, use_graph=1, autotune=1)
    opts64 = airg.default_opts(outer=airg.OUTER_RICHARDSON, precond_precision=64)

    def step(opts):
        h = airg.airg_setup(*A, opts, seg_offsets=offs, seg_seeds=seeds)
        x, info = airg.airg_solve(h, B, rtol=a.rtol, max_it=300)
        st = airg.airg_get_stats(h)
        del h
        return info, st

    for _ in range(a.warmup):
        step(optsb)
    torch.cuda.synchronize()
    airg.airg_kernel_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    runs = [step(optsb) for _ in range(a.steps)]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    roof = roofline_from_timing(airg, a.workload)
    sec = (t1 - t0) / a.steps
    infob, stb = runs[-1]
    fp64 = None
    if not a.no_fp64:
        step(opts64)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        r64 = [step(opts64) for _ in range(a.steps)]
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        i64, s64 = r64[-1]
        fp64 = {"seconds_per_step": round((t3 - t2) / a.steps, 4), "setup_s": round(s64["setup_seconds"], 4),
                "solve_s": round(i64["seconds"], 4), "iterations": i64["iterations"],
                "rel_residual": i64["rel_residual"],
                "form": "48 segments solved one after another, 4 rhs one after another, FP64 Richardson"}
    n = int(offs[-1])
    desc = ("batch48: 48 DG-P1 upwind problems, sides U{64..384}, theta ~ U(0, 2 pi), sigma=1e-3, 4 rhs each; "
            "n=%d, nnz=%d" % (n, int(rp[-1])))
    extra = {"setup_s": round(stb["setup_seconds"], 4), "solve_s": round(infob["seconds"], 4),
             "iterations": infob["iterations"], "rel_residual": infob["rel_residual"], "levels": stb["levels"],
             "complexity": {"grid": round(stb["grid_complexity"], 3),
                            "operator": round(stb["operator_complexity"], 3),
                            "storage": round(stb["storage_complexity"], 3)},
             "phase_seconds": {kk: round(v, 4) for kk, v in stb["phase_seconds"].items()},
             "vcycle_bytes_fp32": stb["vcycle_bytes_fp32"], "fp64_comparison": fp64}
    cfg = {"workload": desc, "form": "batched FGMRES(30) FP64 per (segment, rhs) + batched FP32 V-cycle, "
                                     "one SpMM launch per stage, HIP graph, autotuned kernels",
           "rtol": a.rtol, "parallelism": "single GPU"}
    return sec, cfg, "f64 (f32 V-cycle)", roof, None, extra


def copy_calibration(mib, torch):
    """y = 1.0 * x over mib MiB of float32, once untimed and five times timed: each launch reads and
    writes mib MiB."""
    n = mib * (1 << 20) // 4
    x = torch.rand(n, device="cuda")
    y = torch.empty_like(x)
    torch.mul(x, 1.0, out=y)          # loads the kernel's code object
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record()
    for _ in range(5):
        torch.mul(x, 1.0, out=y)
    ev[1].record()
    torch.cuda.synchronize()
    sec = ev[0].elapsed_time(ev[1]) / 5e3
    print(json.dumps({"copy_calibration": {"bytes_read": n * 4, "bytes_written": n * 4, "launches": 5,
                                           "avg_launch_us": round(sec * 1e6, 2),
                                           "GBps": round(2 * n * 4 / sec / 1e9, 1)}}), flush=True)
    return 0


def main():
    a = parse()
    if a.record_traffic:
        return record_traffic(a.workload, a.record_traffic)
    if a.gpus != 1:
        print("bench.py: this build runs on one GPU only (no sharding, no collectives); "
              "--gpus %d is not supported" % a.gpus, file=sys.stderr)
        return 2
    import torch
    if a.copy_calibration:
        return copy_calibration(a.copy_calibration, torch)
    from paper_2408_08262_amd import airg
    if a.sweep_poly:
        return sweep_poly(a, airg, torch)
    if a.workload == "batch48":
        sec, cfg, dtype, roof, cpu, extra = batched(a, airg, torch)
    else:
        sec, cfg, dtype, roof, cpu, extra = single(a, airg, torch)
    out = {"metric": METRIC, "value": round(sec, 4), "unit": "s", "n_gpus": 1, "steps": a.steps,
           "warmup": a.warmup, "ms_per_step": round(sec * 1e3, 2), "higher_is_better": False, "scaling": "weak",
           "vs_baseline": None, "dtype": dtype, "data": "synthetic", "config": cfg}
    out.update(extra)
    out["roofline"] = roof
    out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
