#!/usr/bin/env python3
"""AIRG benchmark on one MI355X: setup + solve to 1e-10 relative residual.

Headline workload: DG-P1 upwind advection on a 512 x 512 jittered
triangulation, 1,572,864 unknowns, 7,860,224 nonzeros, theta = 1.1 rad,
sigma in {1e-4, 1} on a seeded 16 x 16 block checkerboard, hierarchy truncated
at 98,304 unknowns with 6 iterations of the order-12 coarse polynomial (seeded
synthetic input, resident in device memory before timing starts).

A step is one pass of the whole hot path: the full AIRG setup (CF splitting,
extraction, GMRES polynomials, restrictor, prolongator, Galerkin products,
finalisation) followed by the solve to ||b - A x|| <= 1e-10 ||b||.  The
headline form is FP64 flexible GMRES right-preconditioned by an FP32 V-cycle;
on the same GPU and hierarchy options the line also times plain FP64 AIRG
(undamped Richardson, FP64 V-cycle) and FGMRES around an FP64 V-cycle (which
separates the precision from the outer solver).  value = seconds per step
(lower is better).

Also reported for every form: the error against the exact sweep solution and
against the oracle's own solution, the residual recomputed by the oracle, work
units and grind time; the roofline of the finest-operator SpMV (event-timed
inside the timed steps) against the 8 TB/s HBM3E peak; the solve's and the
setup's algorithmic bytes over their times; two sub-records on workloads whose
operators do not fit the 256 MB Infinity Cache (the 128^3 tetrahedral P0
problem, and the 48-problem batch in its batched FP32 form against sequential
FP64 solves); and the CPU oracle's time on the same workload on all host cores
and on one.
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


WORKLOADS = ("dg_square_512", "p0_cube_128", "batch48", "p0_square_64", "adjoint_256")
# hierarchy options of the timed forms per workload (truncation of the hierarchy and the
# coarse polynomial's iterations; the sweep that chose them is in the design notes)
TRUNCATE = {"dg_square_512": (98304, 6), "p0_cube_128": (65536, 3), "batch48": (0, 3),
            "p0_square_64": (0, 3), "adjoint_256": (0, 3)}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=3)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--workload", default="dg_square_512", choices=WORKLOADS)
    p.add_argument("--size", type=int, default=None, help="override the side of the square/cube workload")
    p.add_argument("--truncate", type=int, default=None, help="truncate_n (default per workload)")
    p.add_argument("--coarse-iters", type=int, default=None, help="coarse polynomial iterations")
    p.add_argument("--rtol", type=float, default=1e-10)
    p.add_argument("--sub-steps", type=int, default=3, help="timed steps of each sub-record")
    p.add_argument("--quick", action="store_true", help="headline only: no sub-records, no oracle legs")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-fp64", action="store_true", help="skip the FP64 comparison forms")
    p.add_argument("--levels", action="store_true",
                   help="only print per-level setup (by phase) and V-cycle times of the workload")
    p.add_argument("--ladder", action="store_true",
                   help="only run the work-growth ladder: dg_square at 64^2..512^2 and p0_cube at 32^3..128^3, "
                        "untruncated, both timed forms")
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
                                     poly_order=order, poly_sparsity_order=sp, time_phases=1, **parse_opts(a.opt))
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


def truncation(a):
    t, c = TRUNCATE[a.workload]
    return (a.truncate if a.truncate is not None else t), (a.coarse_iters if a.coarse_iters is not None else c)


def make_problem(name, size=None):
    from workloads import dg_square, p0_cube, p0_square
    if name == "dg_square_512":
        N = size or 512
        P = dg_square(N)
        desc = ("dg_square_%d: DG-P1 upwind advection, %dx%d jittered triangulation, n=%d, nnz=%d, theta=1.1, "
                "sigma {1e-4,1} 16x16 block checkerboard" % (N, N, N, P.n, P.nnz))
        bs = 3
    elif name == "p0_cube_128":
        N = size or 128
        P = p0_cube(N)
        desc = ("p0_cube_%d: P0 upwind advection, %d^3 cubes x 6 Kuhn tetrahedra, n=%d, nnz=%d, "
                "Omega=(0.5,0.3,0.81)/|.|, sigma=1e-4" % (N, N, P.n, P.nnz))
        bs = 1
    else:
        N = size or 64
        P = p0_square(N)
        desc = ("p0_square_%d: P0 upwind advection, %dx%d squares x 2 triangles, n=%d, nnz=%d, theta=0.3, "
                "sigma=1e-3" % (N, N, N, P.n, P.nnz))
        bs = 1
    return P, desc, bs


def forms(airg):
    return {
        "fp32_fgmres": (dict(outer=airg.OUTER_FGMRES, precond_precision=32),
                        "FGMRES(30) FP64 outer + FP32 AIRG V-cycle"),
        "fp64_richardson": (dict(outer=airg.OUTER_RICHARDSON, precond_precision=64),
                            "undamped Richardson + FP64 AIRG V-cycle (plain AIRG)"),
        "fp64_fgmres": (dict(outer=airg.OUTER_FGMRES, precond_precision=64),
                        "FGMRES(30) FP64 outer + FP64 AIRG V-cycle"),
    }


def time_form(airg, torch, A, b, opts, steps, warmup, rtol, workload=None, seg=None, allow_not_converged=False):
    """warmup untimed and `steps` timed passes of setup + solve on fresh handles; the
    finest-operator product is event-timed over the timed passes when workload is given."""
    segkw = {} if seg is None else {"seg_offsets": seg[0], "seg_seeds": seg[1]}

    def step():
        h = airg.airg_setup(*A, opts, **segkw)
        x, info = airg.airg_solve(h, b, rtol=rtol, max_it=300, allow_not_converged=allow_not_converged)
        st = airg.airg_get_stats(h)
        del h
        return x, info, st

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    if workload:
        airg.airg_kernel_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    last = None
    for _ in range(steps):
        last = None
        last = step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    roof = roofline_from_timing(airg, workload) if workload else None
    x, info, st = last
    return {"sec": (t1 - t0) / steps, "x": x, "info": info, "st": st, "roof": roof}


def cycle_bytes(st, vb, k=1):
    """Algorithmic bytes of one V-cycle with vb-byte values and k right-hand sides."""
    return st["vcycle_index_bytes"] + vb * st["vcycle_nnz"] + vb * k * st["vcycle_vec_entries"]


def top_bytes(st, n, k=1):
    """Algorithmic bytes of one FP64 product with the top operator(s) on k right-hand sides."""
    return st["top_nnz"] * 12 + 4 * (n + 1) + 8 * k * 2 * n


def outer_bytes(form, its, n, restart=30):
    """Vector traffic of the outer iterations around the cycles and top products: the casts and
    permutations into and out of the cycle, FGMRES's classical Gram-Schmidt twice in three passes
    over the basis (the products; the first update fused with the second products; the second update
    fused with the norm: 3 (j + 1) basis reads, w read three times and written twice) and the
    normalisation (w read and written), or Richardson's update and norm."""
    if form == "fp64_richardson":
        return its * (24 + 8 + 40) * n
    cast = 32 if form == "fp32_fgmres" else 40
    tot = 0
    for i in range(its):
        j = i % restart
        nv = 3 * (j + 1) + 7 if j + 1 <= 32 else 4 * (j + 1) + 9
        tot += nv * 8 * n + cast * n
    return tot


def form_record(form, label, r, n, top_us=None, k=1):
    """k: right-hand sides solved together (the batched form's vectors are n x k)."""
    info, st = r["info"], r["st"]
    its = max(1, info["iterations"])
    wu_cycle = st["vcycle_nnz"] / st["top_nnz"]
    wus = info["iterations"] * (wu_cycle + 1.0)
    vb = cycle_bytes(st, 4 if form == "fp32_fgmres" else 8, k)
    solve_bytes = info["iterations"] * (vb + top_bytes(st, n, k)) + outer_bytes(form, info["iterations"], n * k)
    solve_gbs = solve_bytes / info["seconds"] / 1e9 if info["seconds"] > 0 else 0.0
    setup_gbs = st["setup_bytes"] / st["setup_seconds"] / 1e9 if st["setup_seconds"] > 0 else 0.0
    rec = {"form": label, "seconds_per_step": round(r["sec"], 4), "setup_s": round(st["setup_seconds"], 4),
           "solve_s": round(info["seconds"], 4), "iterations": info["iterations"],
           "rel_residual": info["rel_residual"], "levels": st["levels"],
           "wu_per_cycle": round(wu_cycle, 3), "wus": round(wus, 1),
           "grind_ns_per_unknown_per_cycle": round(info["seconds"] / n / its * 1e9, 4),
           "cycles": {"eager": st["cycles_eager"], "graph_replays": st["cycles_graph"]},
           "solve_roofline": {"bound": "hbm", "achieved": round(solve_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                              "frac": round(solve_gbs / HBM_PEAK_GBS, 4), "bytes": int(solve_bytes),
                              "what": "iterations x (V-cycle + top-product algorithmic bytes) + outer vector "
                                      "traffic, over the solve time"},
           "setup_roofline": {"bound": "hbm", "achieved": round(setup_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                              "frac": round(setup_gbs / HBM_PEAK_GBS, 4), "bytes": int(st["setup_bytes"]),
                              "what": "bytes the setup steps must move (each reading its inputs and writing its "
                                      "outputs once), over the setup time"}}
    if top_us:
        rec["wu_ratio"] = round(info["seconds"] / (wus * top_us * 1e-6), 3) if wus > 0 else None
    return rec


def accuracy(P, x, xs, xo=None, A=None):
    """Errors of a device solution against the exact sweep and the oracle's solution, and its
    residual recomputed by the oracle's product (FP64)."""
    import numpy as np
    import oracle as O
    A = A or (P.rowptr, P.col, P.val)
    b = P.b
    out = {"rel_residual_oracle": float(np.linalg.norm(b - O.spmv(A, x)) / np.linalg.norm(b)),
           "err_vs_sweep": float(np.linalg.norm(x - xs) / np.linalg.norm(xs))}
    if xo is not None:
        out["err_vs_oracle"] = float(np.linalg.norm(x - xo) / np.linalg.norm(xo))
    return out


def oracle_baseline(P, params, rtol):
    """The oracle on the headline workload: setup + FP64 Richardson, on every host core the process
    may use and on one."""
    import oracle as O
    want = int(os.environ.get("OMP_NUM_THREADS") or os.cpu_count() or 1)
    res = {}
    for thr in (want, 1):
        O.set_threads(thr)
        used = O.get_threads()
        c0 = time.perf_counter()
        H = O.Hierarchy((P.rowptr, P.col, P.val), params)
        c1 = time.perf_counter()
        x, its, rr = H.richardson(P.b, rtol, 300)
        c2 = time.perf_counter()
        res[thr] = {"cores": used, "setup_s": c1 - c0, "solve_s": c2 - c1, "its": its, "x": x}
        del H
        if want == 1:
            res[1] = res[thr]
            break
    O.set_threads(want)
    return res[want], res[1]


def single(a, airg, torch):
    """The headline workload: three forms of setup + solve, accuracy, work units, rooflines and the
    oracle baseline."""
    import numpy as np
    P, desc, bs = make_problem(a.workload, a.size)
    trunc, citers = truncation(a)
    desc += ", truncate_n=%d, coarse_iters=%d" % (trunc, citers)
    A = airg.to_device(P.rowptr, P.col, P.val)
    b = torch.as_tensor(P.b, device="cuda")
    torch.cuda.synchronize()
    extra_opts = parse_opts(a.opt)
    # a single hierarchy's cycle replayed from a captured graph is no faster than launched kernel by
    # kernel (the small levels are bound by the kernels' own dispatch, not by host launches), and the
    # capture after 16 cycles costs the Richardson form 0.2 ms: the single-hierarchy forms run eager;
    # the batched form keeps its captured graph
    extra_opts.setdefault("use_graph", 0)
    base = dict(seed=P.seed, truncate_n=trunc, coarse_iters=citers, **extra_opts)
    F = forms(airg)
    names = ["fp32_fgmres"] + ([] if a.no_fp64 else ["fp64_richardson", "fp64_fgmres"])
    runs = {}
    for k in names:
        kw, _ = F[k]
        log("timing %s: %s" % (a.workload, k))
        runs[k] = time_form(airg, torch, A, b, airg.default_opts(**base, **kw), a.steps if k == "fp32_fgmres" else
                            max(1, min(a.steps, 10)), a.warmup if k == "fp32_fgmres" else 1, a.rtol,
                            workload=a.workload if k == "fp32_fgmres" else None)
    roof = runs["fp32_fgmres"]["roof"]
    top_us = roof["avg_launch_us"] if roof else None
    recs = {k: form_record(k, F[k][1], runs[k], P.n, top_us) for k in names}
    # numeric re-setup (kept splittings and patterns) for an operator with the same pattern and
    # values perturbed by U(0.9, 1.1), then the solve: timed after the timed region, own handle
    h = airg.airg_setup(*A, airg.default_opts(**base, **F["fp32_fgmres"][0]))
    newval = torch.as_tensor(P.val * np.random.default_rng(77).uniform(0.9, 1.1, P.val.shape), device="cuda")
    airg.airg_resetup(h, newval)
    torch.cuda.synchronize()
    r0 = time.perf_counter()
    nre = max(1, min(a.steps, 10))
    for _ in range(nre):
        airg.airg_resetup(h, newval)
        xr, ir = airg.airg_solve(h, b, rtol=a.rtol, max_it=300)
    torch.cuda.synchronize()
    r1 = time.perf_counter()
    resetup = {"seconds_per_step": round((r1 - r0) / nre, 4),
               "resetup_s": round(airg.airg_get_stats(h)["resetup_seconds"], 4),
               "solve_s": round(ir["seconds"], 4), "iterations": ir["iterations"],
               "rel_residual": ir["rel_residual"],
               "form": "numeric re-setup (kept CF splittings and patterns) + FGMRES/FP32, values x U(0.9, 1.1)"}
    del h, xr, newval
    # the setup phases' device times come from one more setup with the phase events on (the timed
    # steps run without them: they cost the setup about 3%)
    ph_opts = dict(base, **F["fp32_fgmres"][0])
    ph_opts["time_phases"] = 1
    h = airg.airg_setup(*A, airg.default_opts(**ph_opts))
    phase_st = airg.airg_get_stats(h)
    del h
    cpu = None
    if not a.quick:
        import oracle as O
        from oracle.sweep import sweep_solve
        xs = sweep_solve(P.rowptr, P.col, P.val, P.b, bs)
        xo = None
        if not a.no_cpu_baseline:
            log("oracle baseline")
            oracle_opts = {k: v for k, v in extra_opts.items() if k != "use_graph"}
            params = O.default_params(seed=P.seed, truncate_n=trunc, coarse_iters=citers, **oracle_opts)
            allc, one = oracle_baseline(P, params, a.rtol)
            xo = allc["x"]
            cpu = {"value": round(allc["setup_s"] + allc["solve_s"], 3), "unit": "s", "cores": allc["cores"],
                   "kind": "oracle",
                   "sample": "whole workload: oracle setup (%.2f s) + FP64 Richardson to %.0e (%.2f s, %d its) on "
                             "%d threads" % (allc["setup_s"], a.rtol, allc["solve_s"], allc["its"], allc["cores"]),
                   "single_core": {"value": round(one["setup_s"] + one["solve_s"], 3), "cores": 1,
                                   "setup_s": round(one["setup_s"], 3), "solve_s": round(one["solve_s"], 3)}}
            oerr = {"oracle_rel_residual": float(np.linalg.norm(P.b - O.spmv((P.rowptr, P.col, P.val), xo)) /
                                                 np.linalg.norm(P.b)),
                    "oracle_err_vs_sweep": float(np.linalg.norm(xo - xs) / np.linalg.norm(xs))}
            cpu["accuracy"] = oerr
        for k in names:
            recs[k]["accuracy"] = accuracy(P, runs[k]["x"].cpu().numpy(), xs, xo)
    head = recs["fp32_fgmres"]
    st = runs["fp32_fgmres"]["st"]
    extra = dict(head)
    del extra["form"]
    extra["complexity"] = {"grid": round(st["grid_complexity"], 3), "operator": round(st["operator_complexity"], 3),
                           "storage": round(st["storage_complexity"], 3)}
    extra["phase_seconds"] = {k: round(v, 4) for k, v in phase_st["phase_seconds"].items()}
    extra["phase_seconds_from"] = "one setup with time_phases=1 after the timed steps, which run without the events"
    extra["vcycle_bytes_fp32"] = st["vcycle_bytes_fp32"]
    extra["comparison"] = {k: recs[k] for k in names if k != "fp32_fgmres"}
    extra["resetup"] = resetup
    cfg = {"workload": desc, "form": F["fp32_fgmres"][1], "rtol": a.rtol, "parallelism": "single GPU",
           "options": extra_opts}
    del runs, A, b
    return a.steps, cfg, "f64 (f32 V-cycle)", roof, cpu, extra


def hbm_subrecord(a, airg, torch):
    """The 128^3 tetrahedral P0 problem (operator 703.5 MB in FP64, beyond the Infinity Cache):
    FP32-preconditioned FGMRES against plain FP64 AIRG, truncated hierarchy."""
    import numpy as np
    P, desc, bs = make_problem("p0_cube_128")
    trunc, citers = TRUNCATE["p0_cube_128"]
    desc += ", truncate_n=%d, coarse_iters=%d" % (trunc, citers)
    A = airg.to_device(P.rowptr, P.col, P.val)
    b = torch.as_tensor(P.b, device="cuda")
    F = forms(airg)
    out = {"workload": desc}
    xs = None
    if not a.quick:
        from oracle.sweep import sweep_solve
        xs = sweep_solve(P.rowptr, P.col, P.val, P.b, bs)
    for k in ("fp32_fgmres", "fp64_richardson"):
        log("timing p0_cube_128: %s" % k)
        r = time_form(airg, torch, A, b, airg.default_opts(seed=P.seed, truncate_n=trunc, coarse_iters=citers,
                                                           use_graph=0, **F[k][0]),
                      a.sub_steps, 1, a.rtol, workload="p0_cube_128" if k == "fp32_fgmres" else None)
        top_us = out["roofline"]["avg_launch_us"] if "roofline" in out else (r["roof"] or {}).get("avg_launch_us")
        rec = form_record(k, F[k][1], r, P.n, top_us)
        if xs is not None:
            rec["accuracy"] = accuracy(P, r["x"].cpu().numpy(), xs)
        if r["roof"]:
            out["roofline"] = r["roof"]
        out[k] = rec
        del r
    out["steps"] = a.sub_steps
    out["value"] = out["fp32_fgmres"]["seconds_per_step"]
    out["fp64_over_fp32"] = round(out["fp64_richardson"]["seconds_per_step"] / out["value"], 3)
    del A, b
    torch.cuda.empty_cache()
    return out


def batched_subrecord(a, airg, torch):
    """48 independent DG-P1 problems x 4 rhs: the batched FP32 form (one SpMM launch per stage,
    captured graph, autotuned kernels) against the 48 problems solved one after another in plain FP64
    AIRG."""
    import numpy as np
    from workloads import batch as batch_problems, concat
    probs = batch_problems()
    rp, ci, val, bb, offs, seeds = concat(probs)
    A = airg.to_device(rp, ci, val)
    B = torch.as_tensor(bb, device="cuda")
    n = int(offs[-1])
    out = {"workload": "batch48: 48 DG-P1 upwind problems, sides U{64..384}, theta ~ U(0, 2 pi), sigma=1e-3, "
                       "4 rhs each; n=%d, nnz=%d" % (n, int(rp[-1]))}
    log("timing batch48: batched FP32")
    rb = time_form(airg, torch, A, B, airg.default_opts(outer=airg.OUTER_FGMRES, precond_precision=32, use_graph=1,
                                                        autotune=1),
                   a.sub_steps, 1, a.rtol, workload="batch48", seg=(offs, seeds))
    out["roofline"] = rb["roof"]
    recb = form_record("fp32_fgmres", "batched FGMRES(30) FP64 per (segment, rhs) + batched FP32 V-cycle, one "
                                      "SpMM launch per stage, HIP graph, autotuned kernels", rb, n,
                       rb["roof"]["avg_launch_us"] if rb["roof"] else None, k=bb.shape[1])
    log("timing batch48: sequential FP64")
    r64 = time_form(airg, torch, A, B, airg.default_opts(outer=airg.OUTER_RICHARDSON, precond_precision=64),
                    1, 1, a.rtol, seg=(offs, seeds))
    rec64 = form_record("fp64_richardson", "48 segments solved one after another, 4 rhs one after another, "
                                           "plain FP64 AIRG (Richardson)", r64, n)
    # each (segment, rhs) pair iterates to its own count, of which only the largest is reported:
    # no byte count for this form's solve
    rec64["solve_roofline"] = None
    if not a.quick:
        import oracle as O
        from oracle.sweep import sweep_solve
        Xb, X64 = rb["x"].cpu().numpy(), r64["x"].cpu().numpy()
        worst = {"fp32": [0.0, 0.0], "fp64": [0.0, 0.0]}
        for p, Pp in enumerate(probs):
            Ap = (Pp.rowptr, Pp.col, Pp.val)
            xs = sweep_solve(Pp.rowptr, Pp.col, Pp.val, Pp.b, 3)
            for key, X in (("fp32", Xb), ("fp64", X64)):
                Xp = X[offs[p]:offs[p + 1]]
                for c in range(Pp.b.shape[1]):
                    r = np.linalg.norm(Pp.b[:, c] - O.spmv(Ap, Xp[:, c])) / np.linalg.norm(Pp.b[:, c])
                    e = np.linalg.norm(Xp[:, c] - xs[:, c]) / np.linalg.norm(xs[:, c])
                    worst[key][0] = max(worst[key][0], float(r))
                    worst[key][1] = max(worst[key][1], float(e))
        recb["accuracy"] = {"max_rel_residual_oracle": worst["fp32"][0], "max_err_vs_sweep": worst["fp32"][1],
                            "pairs": len(probs) * bb.shape[1]}
        rec64["accuracy"] = {"max_rel_residual_oracle": worst["fp64"][0], "max_err_vs_sweep": worst["fp64"][1],
                             "pairs": len(probs) * bb.shape[1]}
    out["batched_fp32"] = recb
    out["sequential_fp64"] = rec64
    out["steps"] = a.sub_steps
    out["value"] = recb["seconds_per_step"]
    out["fp64_over_batched"] = round(rec64["seconds_per_step"] / recb["seconds_per_step"], 3)
    del A, B, rb, r64
    torch.cuda.empty_cache()
    return out


def level_cycle_bytes(lv, ups, citers, k):
    """Algorithmic bytes (FP32, FP64) of a level's own work in one cycle on k right-hand sides: the
    restriction [Z I], the prolongation [W; I] and ups x ([A_ff A_fc] residual + Ainv update); on the
    coarsest level Ainv once and (A residual + Ainv update) citers - 1 times."""
    def spmv(rows, cols, nz, reads_y, vb):
        return nz * (vb + 4) + 4 * (rows + 1) + vb * k * (cols + rows + (rows if reads_y else 0))
    out = []
    for vb in (4, 8):
        n, nf, nc = lv["n"], lv["n_f"], lv["n_c"]
        if lv["coarsest"]:
            b = spmv(n, n, lv["nnz_ainv"], False, vb) + (citers - 1) * (spmv(n, n, lv["nnz_a"], True, vb) +
                                                                         spmv(n, n, lv["nnz_ainv"], True, vb))
        else:
            b = spmv(nc, n, lv["nnz_z"] + nc, False, vb) + spmv(n, nc, lv["nnz_w"] + nc, False, vb)
            b += ups * (spmv(nf, n, lv["nnz_aff"] + lv["nnz_afc"], True, vb) + spmv(nf, nf, lv["nnz_ainv"], True, vb))
        out.append(int(b))
    return out


def levels_report_batch(a, airg, torch):
    """Per-level setup time by phase (all segments together) and per-level batched FP32 cycle time."""
    from workloads import batch as batch_problems, concat
    probs = batch_problems()
    rp, ci, val, bb, offs, seeds = concat(probs)
    A = airg.to_device(rp, ci, val)
    B = torch.as_tensor(bb, device="cuda")
    opts = airg.default_opts(outer=airg.OUTER_FGMRES, precond_precision=32, use_graph=1, autotune=1, time_phases=1)
    for _ in range(2):
        h = airg.airg_setup(*A, opts, seg_offsets=offs, seg_seeds=seeds)
        del h
    h = airg.airg_setup(*A, opts, seg_offsets=offs, seg_seeds=seeds)
    airg.airg_solve(h, B, rtol=a.rtol, max_it=300)
    st = airg.airg_get_stats(h)
    t32 = airg.airg_batch_vcycle_profile(h, nrhs=bb.shape[1], reps=20)
    rows = []
    for l in range(st["levels"]):
        lv, n, nnz, segs, b32 = None, 0, 0, 0, 0
        for p in range(len(probs)):
            try:
                x = airg.airg_get_level(h, l, segment=p, with_cf=False)
            except airg.AirgError:
                continue
            lv = x
            n += x["n"]
            nnz += x["nnz_a"]
            segs += 1
            b32 += level_cycle_bytes(x, opts.up_smooths, opts.coarse_iters, bb.shape[1])[0]
        rows.append({"level": l, "n": n, "nnz_a": nnz, "segments": segs, "coarsest": False,
                     "setup_ms": {k: round(v * 1e3, 4) for k, v in lv["setup_seconds"].items()},
                     "setup_bytes": lv["setup_bytes"], "vcycle_us_fp32": round(t32[l] * 1e6, 2),
                     "vcycle_us_fp64": 0.0, "vcycle_bytes_fp32": b32, "vcycle_bytes_fp64": 0})
    print(json.dumps({"levels_report": "batch48: 48 DG-P1 upwind problems x 4 rhs, batched FP32 cycle, "
                                       "n=%d, nnz=%d" % (int(offs[-1]), int(rp[-1])),
                      "setup_s": st["setup_seconds"], "phase_seconds": st["phase_seconds"], "rows": rows}),
          flush=True)
    return 0


def levels_report(a, airg, torch):
    """Per-level setup time by phase and per-level V-cycle time (FP32 and FP64) of one workload."""
    if a.workload == "batch48":
        return levels_report_batch(a, airg, torch)
    P, desc, bs = make_problem(a.workload, a.size)
    trunc, citers = truncation(a)
    A = airg.to_device(P.rowptr, P.col, P.val)
    opts = airg.default_opts(seed=P.seed, truncate_n=trunc, coarse_iters=citers, outer=airg.OUTER_FGMRES,
                             precond_precision=32, use_graph=1, time_phases=1)
    for _ in range(2):
        h = airg.airg_setup(*A, opts)
        del h
    h = airg.airg_setup(*A, opts)
    st = airg.airg_get_stats(h)
    t32 = airg.airg_vcycle_profile(h, precision=32, reps=20)
    t64 = airg.airg_vcycle_profile(h, precision=64, reps=20)
    rows = []
    for l in range(st["levels"]):
        lv = airg.airg_get_level(h, l, with_cf=False)
        b32, b64 = level_cycle_bytes(lv, opts.up_smooths, citers, 1)
        rows.append({"level": l, "n": lv["n"], "nnz_a": lv["nnz_a"], "coarsest": lv["coarsest"],
                     "setup_ms": {k: round(v * 1e3, 4) for k, v in lv["setup_seconds"].items()},
                     "setup_bytes": lv["setup_bytes"],
                     "vcycle_us_fp32": round(t32[l] * 1e6, 2), "vcycle_us_fp64": round(t64[l] * 1e6, 2),
                     "vcycle_bytes_fp32": b32, "vcycle_bytes_fp64": b64})
    # the levels' cycle bytes add up to the hierarchy's
    assert sum(r["vcycle_bytes_fp64"] for r in rows) == st["vcycle_bytes_fp64"]
    print(json.dumps({"levels_report": desc + ", truncate_n=%d, coarse_iters=%d" % (trunc, citers),
                      "setup_s": st["setup_seconds"], "phase_seconds": st["phase_seconds"], "rows": rows}),
          flush=True)
    return 0


def ladder(a, airg, torch):
    """Iterations, work units and grind time of both timed forms as the problem grows (flat
    iterations and WUs = work linear in n), untruncated hierarchies with the default options."""
    F = forms(airg)
    for name, sizes in (("dg_square_512", (64, 128, 256, 512)), ("p0_cube_128", (32, 64, 128))):
        for N in sizes:
            P, desc, bs = make_problem(name, N)
            A = airg.to_device(P.rowptr, P.col, P.val)
            b = torch.as_tensor(P.b, device="cuda")
            row = {"ladder": desc, "n": P.n, "nnz": P.nnz}
            for k in ("fp32_fgmres", "fp64_richardson"):
                # undamped Richardson may diverge (a level polynomial with an outlier eigenvalue): recorded
                r = time_form(airg, torch, A, b, airg.default_opts(seed=P.seed, use_graph=0, **F[k][0]),
                              a.sub_steps, 1, a.rtol, allow_not_converged=True)
                rec = form_record(k, F[k][1], r, P.n)
                row[k] = {kk: rec[kk] for kk in ("seconds_per_step", "setup_s", "solve_s", "iterations", "levels",
                                                 "wu_per_cycle", "wus", "grind_ns_per_unknown_per_cycle")}
                row[k]["converged"] = bool(r["info"]["converged"])
                row[k]["complexity"] = [round(r["st"]["grid_complexity"], 3), round(r["st"]["operator_complexity"], 3)]
                del r
            print(json.dumps(row), flush=True)
            del A, b, P
            torch.cuda.empty_cache()
    return 0


def small_workload(a, airg, torch):
    """C1 (p0_square_64, plain untruncated FP64 AIRG) or C5 (adjoint_256: forward solve and the
    adjoint A^T solve with the gradients) timed per step."""
    import numpy as np
    if a.workload == "p0_square_64":
        P, desc, bs = make_problem("p0_square_64", a.size)
        A = airg.to_device(P.rowptr, P.col, P.val)
        b = torch.as_tensor(P.b, device="cuda")
        r = time_form(airg, torch, A, b, airg.default_opts(seed=P.seed, outer=airg.OUTER_RICHARDSON,
                                                           precond_precision=64, use_graph=0),
                      a.steps, a.warmup, a.rtol)
        rec = form_record("fp64_richardson", "undamped Richardson + FP64 AIRG V-cycle (plain AIRG)", r, P.n)
        if not a.quick:
            from oracle.sweep import sweep_solve
            rec["accuracy"] = accuracy(P, r["x"].cpu().numpy(), sweep_solve(P.rowptr, P.col, P.val, P.b, 1))
        cfg = {"workload": desc, "form": rec.pop("form"), "rtol": a.rtol, "parallelism": "single GPU"}
        return r["sec"], cfg, "f64", None, None, rec
    # adjoint_256: loss = sum of u^2 over the detector patch; one step = forward setup + solve, the
    # adjoint hierarchy and A^T solve, and both gradients
    from paper_2408_08262_amd import adjoint as adj
    from workloads import adjoint as adjoint_problem
    N = a.size or 256
    P = adjoint_problem(N)
    m = P.meta
    prob = adj.DiffProblem(P.rowptr, P.col, m["val_adv"], m["mass"], opts=airg.default_opts(seed=P.seed))
    s = torch.as_tensor(m["src"], device="cuda")
    sg = torch.as_tensor(m["sigma"], device="cuda")
    mask = torch.as_tensor(m["patch_mask"], device="cuda")

    def step():
        si = s.clone().requires_grad_(True)
        gi = sg.clone().requires_grad_(True)
        u = adj.solve(si, gi, prob)
        (u[mask] ** 2).sum().backward()
        return u, si.grad, gi.grad

    for _ in range(a.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        u, gs, gsig = step()
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / a.steps
    rec = {"seconds_per_step": round(sec, 4)}
    if not a.quick:
        import scipy.sparse as sp
        from oracle.sweep import sweep_solve
        nc = m["mass"].shape[0]
        K = np.repeat(np.arange(nc), 9)
        rr = K * 3 + np.tile(np.repeat(np.arange(3), 3), nc)
        cc = K * 3 + np.tile(np.arange(3), nc * 3)
        Mb = sp.csr_matrix((m["mass"].ravel(), (rr, cc)), shape=(P.n, P.n))
        us = sweep_solve(P.rowptr, P.col, P.val, Mb @ m["src"], 3)
        lam = sweep_solve(P.rowptr, P.col, P.val, np.where(m["patch_mask"], 2.0 * us, 0.0), 3, transpose=True)
        want_s = Mb.T @ lam
        want_sig = -np.einsum("ka,kab,kb->k", lam.reshape(-1, 3), m["mass"], us.reshape(-1, 3))
        rec["accuracy"] = {
            "u_err_vs_sweep": float(np.linalg.norm(u.detach().cpu().numpy() - us) / np.linalg.norm(us)),
            "grad_source_err_vs_sweeps": float(np.linalg.norm(gs.cpu().numpy() - want_s) / np.linalg.norm(want_s)),
            "grad_sigma_err_vs_sweeps": float(np.linalg.norm(gsig.cpu().numpy() - want_sig) /
                                              np.linalg.norm(want_sig))}
    desc = ("adjoint_256: DG-P1 upwind advection, %dx%d jittered triangulation, n=%d, nnz=%d, theta=1.1, "
            "sigma_K = exp(N(ln 1e-2, 1)), loss = sum of u^2 over a 32x32-square detector patch" % (N, N, P.n, P.nnz))
    cfg = {"workload": desc, "form": "forward AIRG setup + FP64 Richardson solve, A^T hierarchy + adjoint solve, "
                                     "gradients wrt source and sigma", "rtol": 1e-10, "parallelism": "single GPU"}
    return sec, cfg, "f64", None, None, rec


def main():
    a = parse()
    if a.record_traffic:
        return record_traffic(a.workload, a.record_traffic)
    if a.gpus != 1:
        print("bench.py: the library runs on one GPU only (no sharding, no collectives); "
              "--gpus %d is not supported" % a.gpus, file=sys.stderr)
        return 2
    import torch
    if a.copy_calibration:
        return copy_calibration(a.copy_calibration, torch)
    from paper_2408_08262_amd import airg
    if a.sweep_poly:
        return sweep_poly(a, airg, torch)
    if a.levels:
        return levels_report(a, airg, torch)
    if a.ladder:
        return ladder(a, airg, torch)
    sub = {}
    if a.workload == "batch48":
        rec = batched_subrecord(a, airg, torch)
        sec = rec["value"]
        cfg = {"workload": rec.pop("workload"), "form": rec["batched_fp32"]["form"], "rtol": a.rtol,
               "parallelism": "single GPU"}
        roof, cpu, extra, dtype = rec.pop("roofline"), None, rec, "f64 (f32 V-cycle)"
        steps = a.sub_steps
    elif a.workload in ("p0_square_64", "adjoint_256"):
        sec, cfg, dtype, roof, cpu, extra = small_workload(a, airg, torch)
        steps = a.steps
    else:
        steps, cfg, dtype, roof, cpu, extra = single(a, airg, torch)
        sec = extra["seconds_per_step"]
        if a.workload == "dg_square_512" and not a.quick and a.size is None:
            sub["hbm"] = hbm_subrecord(a, airg, torch)
            sub["batched"] = batched_subrecord(a, airg, torch)
    out = {"metric": METRIC, "value": round(sec, 4), "unit": "s", "n_gpus": 1, "steps": steps,
           "warmup": a.warmup, "ms_per_step": round(sec * 1e3, 2), "higher_is_better": False, "scaling": "weak",
           "vs_baseline": None, "dtype": dtype, "data": "synthetic", "config": cfg}
    out.update(extra)
    out.update(sub)
    out["roofline"] = roof
    out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
