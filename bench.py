"""Benchmark: hPLMM set-up + FGMRES solve to a 1e-8 relative residual on the
64^3 headline workload, one MI355X.

A step is one pass of the whole hot path on one load case: the numeric
set-up on the device (grain and contact-grid factorisations, basis, Galerkin
coarse operator and its factor) followed by the preconditioned FGMRES solve
from x0 = 0.  Inputs (matrix, load, partition, plans) are resident in HBM
before the timed region.

Prints one JSON line (see the repository's design notes for the fields).
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

METRIC = "GMRES time-to-1e-8 residual (setup+solve) & SpMV/apply HBM GB/s, 64^3 case"
HBM_PEAK_GBS = 8000.0           # MI355X HBM3E
FP64_MFMA_TFLOPS = 78.6         # MI355X dense FP64 matrix peak
FP32_MFMA_TFLOPS = 157.3
CPU_SAMPLE_N = 32               # voxels per side of the oracle's sample of the workload
KERNEL_NAMES = {
    "tile_gemm": "tile_gemm_kernel<double>",
    "gemv_smoother": "gemv_kernel (grain + contact smoother)",
    "gemv_coarse": "gemv_kernel (coarse solve)",
    "gemv_basis": "gemv_kernel (restriction / prolongation)",
    "spmv": "spmv_kernel",
    "diag": "diag_kernel<double>",
    "smoother_reduce": "sym_reduce_kernel (transposed-product sums of the symmetric smoother)",
}
SYM_SMOOTHER_NAME = "sym_gemv_kernel (grain + contact smoother, S = W^T W)"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", choices=["grf", "uneven"], default="grf",
                    help="grf: Gaussian-random-field solid, lognormal E, box subdomains (the headline case); "
                         "uneven: pores + disc fractures, two-phase E, irregular Voronoi subdomains")
    ap.add_argument("--n", type=int, default=64, help="voxels per side")
    ap.add_argument("--box", type=int, default=8)
    ap.add_argument("--dofs-per-cell", type=float, default=1000.0, help="uneven workload: target dofs per subdomain")
    ap.add_argument("--mortar", type=int, default=4,
                    help="mortar nodes per interface (4 minimises set-up + solve time on this workload)")
    ap.add_argument("--precision", type=int, default=64, choices=[64, 32, 16])
    ap.add_argument("--smoother-form", choices=["auto", "factors", "inverse"], default="auto",
                    help="local solves of the smoother as W^T (W x) or as S x with S = W^T W "
                         "(auto: the inverse form, except with bfloat16 storage)")
    ap.add_argument("--assembled", action="store_true",
                    help="products with A from the assembled blocks (default: matrix-free from the voxel grid)")
    ap.add_argument("--autotune-reps", type=int, default=3,
                    help="launch-shape autotuning after the warm-up steps, untimed (0: default shapes)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-full", action="store_true",
                    help="no GPU: time the oracle on the whole workload and print one JSON line")
    ap.add_argument("--cpu-threads", type=int, default=0, help="--cpu-full: BLAS threads (0: as configured)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="run one device-to-device copy of this many MiB first (counter calibration)")
    return ap.parse_args()


def main():
    a = parse()
    if a.cpu_full:
        cpu_full(a)
        return
    if a.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1"}))
        sys.exit(2)
    import torch
    from paper_2509_19777_amd import hplmm as hp, synth

    torch.cuda.set_device(0)
    t0 = time.perf_counter()
    prob = make_problem(a, a.n)
    sysm, part = hp.build_problem(prob)
    S = hp.Solver(sysm, part, n_mortar=a.mortar, smoother_precision=a.precision, smoother_form=a.smoother_form)
    if not a.assembled:
        S.set_voxel_operator(prob)
    t_plan = time.perf_counter() - t0
    sizes = S.sizes()
    print(f"# plan done in {t_plan:.1f} s: {sizes}", file=sys.stderr, flush=True)

    if a.copy_calibration_mib > 0:
        # a plain copy of known size: reads and writes exactly this many bytes,
        # so hardware fetch/write counters of this kernel give their scale
        src = torch.ones(a.copy_calibration_mib * (1 << 20) // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    hbm = measure_triad(torch, hp)
    print(f"# streaming triad: {hbm}", file=sys.stderr, flush=True)

    def step():
        S.setup()
        x, info = S.solve(rtol=1e-8, restart=50, maxit=300)
        return x, info

    for _ in range(a.warmup):
        step()
    tune = None
    if a.autotune_reps > 0:
        # launch shapes depend on the problem's structure only: chosen once,
        # like the plan, before the timed region
        t_t = time.perf_counter()
        if a.warmup == 0:
            S.setup()   # the tuner times the set-up's operators
        recs = S.autotune(a.autotune_reps)
        t_t = time.perf_counter() - t_t
        changed = [r for r in recs if r["variant"] != 0 or r["waves"] != 4]
        tune = {"launches": len(recs), "changed": len(changed), "tuning_s": round(t_t, 3),
                "saved_us_per_apply": round(sum(r["t_default_us"] - r["t_best_us"] for r in changed), 1)}
        print(f"# autotune: {tune}", file=sys.stderr, flush=True)
        step()
    # one untimed step with HIP events around every kernel class: the
    # per-class breakdown and the dominant class
    S.profile(S.PROF_CLASSES)
    step()
    prof_all = S.profile_results()
    S.profile([])
    names = dict(KERNEL_NAMES)
    if S.smoother_form() == "inverse":
        names["gemv_smoother"] = SYM_SMOOTHER_NAME
    meth = S.method_work()
    # the set-up's dense factorisation work runs in two kernels (the tile
    # contractions and the diagonal-tile factorisations): one roofline class
    cls_ms = {k: v for k, v in
              [("setup_dense", prof_all["tile_gemm"]["ms"] + prof_all["diag"]["ms"])] +
              [(k, prof_all[k]["ms"]) for k in ("gemv_smoother", "gemv_coarse", "gemv_basis", "spmv")]
              if v > 0}
    ranked = sorted(cls_ms, key=lambda k: -cls_ms[k])
    dom = ranked[0]
    second = ranked[1] if len(ranked) > 1 else None
    # timed region: the dominant class timed live with HIP events on its stream
    S.profile(CLASS_KERNELS.get(dom, [dom]))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    infos = []
    for _ in range(a.steps):
        x, info = step()
        infos.append(info)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    ms = (t2 - t1) * 1e3 / a.steps
    prof = S.profile_results()
    S.profile([])
    setup_ms = S.setup_times_ms()
    # the same steps without events, for reference
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    for _ in range(a.steps):
        step()
    torch.cuda.synchronize()
    ms_unprof = (time.perf_counter() - t3) * 1e3 / a.steps
    print(f"# step {ms:.1f} ms, iters {infos[-1]['iters']}, rel_res {infos[-1]['rel_res']:.2e}, "
          f"setup {setup_ms}", file=sys.stderr, flush=True)
    roof = class_roofline(dom, prof, meth, a.steps, S, names)
    apply_gbs = (meth["apply_bytes"]["total"] * prof_all["apply"]["launches"] / (prof_all["apply"]["ms"] * 1e-3) / 1e9
                 if prof_all["apply"]["ms"] else None)
    spmv_gbs = prof_all["spmv"]["units"] / (prof_all["spmv"]["ms"] * 1e-3) / 1e9 if prof_all["spmv"]["ms"] else None

    def _rate(k, v):
        # tile_gemm units are issued flops, every other class counts algorithmic bytes
        if not v["ms"]:
            return None
        r = v["units"] / (v["ms"] * 1e-3)
        if k == "diag":
            return None
        return {"tflops": round(r / 1e12, 2)} if k == "tile_gemm" else {"gbs": round(r / 1e9, 1)}

    breakdown = {k: {"ms_per_step": round(v["ms"], 3), "launches_per_step": v["launches"], **(_rate(k, v) or {})}
                 for k, v in prof_all.items() if v["launches"]}
    out = {
        "metric": METRIC, "value": round(ms, 3), "unit": "ms", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": round(ms, 3), "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64" if a.precision == 64 else f"f64+{'f32' if a.precision == 32 else 'bf16'}-smoother",
        "data": "synthetic",
        "config": {"workload": workload_name(a),
                   "dofs": 3 * sizes["n_nodes"], "subdomains": sizes["grain_mats"], "coarse_dofs": sizes["n_coarse"],
                   "fine_operator": "assembled SELL-64" if a.assembled else "matrix-free Q1",
                   "smoother_form": S.smoother_form()},
        "iters": infos[-1]["iters"], "rel_res_true": infos[-1]["rel_res"],
        "setup_ms": {k: round(float(v), 3) for k, v in setup_ms.items()},
        "solve_ms": round(float(np.mean([i["t_solve_ms"] for i in infos])), 3),
        # the paper's Table 3 split of the set-up (they overlap on the device)
        "t_ml_ms": round(float(infos[-1]["t_ml_ms"]), 3), "t_mg_ms": round(float(infos[-1]["t_mg_ms"]), 3),
        "ms_per_step_without_profiler_events": round(ms_unprof, 3),
        "spmv_gbs": None if spmv_gbs is None else round(spmv_gbs, 1),
        "apply_gbs": None if apply_gbs is None else round(apply_gbs, 1),
        "method_work": {"setup_flops": meth["setup_flops"], "issued_setup_flops": meth["issued_setup_flops"],
                        "apply_bytes": meth["apply_bytes"]},
        "spmv_algorithmic_bytes": S.algorithmic_bytes()["spmv"],
        "kernel_breakdown": breakdown,   # one untimed step with events around every class
        "autotune": tune,
        "hbm_measured": hbm,
        "roofline": roof,
        "roofline_secondary": None if second is None else class_roofline(second, prof_all, meth, 1, S, names),
        "cpu_baseline": None if a.no_cpu_baseline else cpu_baseline(a, infos[-1]["iters"], 3 * sizes["n_nodes"], sizes["grain_mats"]),
    }
    for rk in ("roofline", "roofline_secondary"):
        r = out[rk]
        if r and r.get("bound") == "hbm":
            r["frac_of_triad"] = round(r["achieved"] / hbm["triad_gbs_best"], 4)
    print(json.dumps(out), flush=True)


def measure_triad(torch, hp, mib=1024, reps=20):
    """Streaming-triad bandwidth of this GPU (a = b + s c, three arrays of
    `mib` MiB, the library's own kernel): the best and the median of `reps`
    timed launches, beside the vendor's 8 TB/s."""
    n = mib * (1 << 20) // 8
    a = torch.empty(n, dtype=torch.float64, device="cuda")
    b = torch.ones(n, dtype=torch.float64, device="cuda")
    c = torch.full((n,), 0.5, dtype=torch.float64, device="cuda")
    hp.stream_triad(a, b, c, 3.0)
    torch.cuda.synchronize()
    if not bool(torch.all(a == 2.5)):
        raise RuntimeError("streaming triad returned wrong values")
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for e0, e1 in ev:
        e0.record()
        hp.stream_triad(a, b, c, 3.0)
        e1.record()
    torch.cuda.synchronize()
    gbs = sorted(3 * 8 * n / (e0.elapsed_time(e1) * 1e-3) / 1e9 for e0, e1 in ev)
    del a, b, c
    return {"triad_gbs_best": round(gbs[-1], 1), "triad_gbs_median": round(gbs[len(gbs) // 2], 1),
            "vendor_peak_gbs": HBM_PEAK_GBS, "arrays_mib": mib,
            "kernel": "a = b + s c, two reads and one write per element (hplmm_stream_triad)"}


# kernel classes of the built-in profiler behind each roofline class
CLASS_KERNELS = {"setup_dense": ["tile_gemm", "diag"]}


def class_roofline(k, prof, meth, steps, S, names):
    """Roofline of one kernel class over the profiled region: achieved = the
    method's own work (flops of the set-up, or bytes of the applications, from
    unpadded sizes with every operator read once) / the summed duration of
    the class's launches; the work its launches issue (64x64 tile padding,
    explicit inverses, diagonal tiles) is reported beside it."""
    if k == "setup_dense":
        t, d = prof["tile_gemm"], prof["diag"]
        launches = t["launches"] + d["launches"]
        ms = t["ms"] + d["ms"]
        method = meth["setup_flops"]["total"] * steps
        ach = method / (ms * 1e-3) / 1e12
        iss = t["units"] / (t["ms"] * 1e-3) / 1e12 if t["ms"] else None
        r = {"bound": "mfma", "achieved": round(ach, 3), "peak": FP64_MFMA_TFLOPS, "unit": "TFLOP/s",
             "frac": round(ach / FP64_MFMA_TFLOPS, 4),
             "kernel": "tile_gemm_kernel<double> + diag_kernel<double> (set-up tile Cholesky, inverses, basis, "
                       "Galerkin blocks, coarse fronts)",
             "launches": launches, "avg_launch_us": round(ms * 1e3 / launches, 3),
             "units_per_launch": method / launches,
             "units": "method flops: sum N^3/3 + 2 N^2 (k+1) + 2 N k^2 over grains, n^3/3 over contact grids, "
                      "d^3/3 + d^2 u + d u^2 over coarse fronts",
             "issued": {"tile_gemm_tflops": None if iss is None else round(iss, 3),
                        "tile_gemm_frac": None if iss is None else round(iss / FP64_MFMA_TFLOPS, 4),
                        "issued_over_method": round(meth["issued_setup_flops"]["total"] / meth["setup_flops"]["total"], 3)},
             "traffic": traffic_for("setup_dense")}
        return r
    d = prof[k]
    if not d["launches"] or not d["ms"]:
        return None
    per_apply = {"gemv_smoother": (meth["apply_bytes"]["smoother"], 2 if S.smoother_form() == "inverse" else 4),
                 "gemv_basis": (meth["apply_bytes"]["basis"], 2),
                 "gemv_coarse": (meth["apply_bytes"]["coarse"], 1)}
    if k in per_apply:
        mb, lpa = per_apply[k]
        method = mb * d["launches"] / lpa
    else:
        method = d["units"]
    ach = method / (d["ms"] * 1e-3) / 1e9
    key = k + "_inverse" if k == "gemv_smoother" and S.smoother_form() == "inverse" else k
    return {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(ach / HBM_PEAK_GBS, 4), "kernel": names[k], "launches": d["launches"],
            "avg_launch_us": round(d["ms"] * 1e3 / d["launches"], 3), "units_per_launch": method / d["launches"],
            "units": "method bytes: each operator's stored triangle or block read once, vectors in and out",
            "issued": {"bytes_per_launch": d["units"] / d["launches"],
                       "issued_over_method": round(d["units"] / method, 3)},
            "traffic": traffic_for(key)}


def traffic_for(dom):
    """HBM bytes per launch of the dominant kernel class from the committed
    rocprofv3 counter summary, if it was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        t = json.load(open(path))
        rec = t.get(dom)
        if not rec or rec.get("source_sha256") != _source_hash(rec.get("source_files", [])):
            return None
        return rec.get("bytes_per_launch")
    except Exception:
        return None


def _source_hash(files):
    """SHA-256 over the sources of the counted kernel (paths relative to the repository)."""
    import hashlib
    h = hashlib.sha256()
    for f in files:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()


def make_problem(a, n):
    from paper_2509_19777_amd import synth
    if a.workload == "uneven":
        return synth.config_uneven(n, seed=31, n_mortar=a.mortar, dofs_per_cell=a.dofs_per_cell)
    return synth.config_grf(n, a.box, seed=2, n_mortar=a.mortar)


def workload_name(a):
    if a.workload == "uneven":
        return (f"uneven{a.n}^3 pores + 5 disc fractures, E in {{1, 10}}, Voronoi subdomains of ~{a.dofs_per_cell:g} "
                f"dofs, n={a.mortar}, FGMRES(50) to 1e-8")
    return f"grf{a.n}^3 solid 0.6, lognormal E, {a.box}^3-voxel boxes, n={a.mortar}, FGMRES(50) to 1e-8"


ORACLE_FILES = ["oracle/fem.py", "oracle/partition.py", "oracle/mortar.py", "oracle/hplmm.py", "oracle/gmres.py"]
CPU_FULL_RECORD = os.path.join(ROOT, "profiles", "cpu_oracle_grf64_n4.json")


def oracle_timed(problem, mortar, label="", progress=False):
    """The oracle, untuned, on one problem: set-up (the literal W, Q, P, P^
    and dense coarse Cholesky of Eqs. 18-24, grain and contact-grid
    factorisations of Eq. 26) and FGMRES(50) to a 1e-8 true residual, timed by
    phase with the host clock; assembly is excluded, as on the GPU.  A
    subclass only wraps the oracle's set-up stages with timers."""
    from oracle import fem, gmres, hplmm as oh
    A, b, mesh = fem.assemble(problem)
    ph = {}

    def stamp(name, f):
        t0 = time.perf_counter()
        f()
        ph[name] = time.perf_counter() - t0
        if progress:
            print(f"# oracle {label}: {name} {ph[name]:.1f} s", file=sys.stderr, flush=True)

    class Timed(oh.HPLMM):
        def _build_P(self, use_rhs):
            stamp("grains_basis_s", lambda: oh.HPLMM._build_P(self, use_rhs))

        def _coarse_operator(self):
            stamp("coarse_operator_s", lambda: oh.HPLMM._coarse_operator(self))

        def _coarse_factor(self):
            stamp("coarse_factor_s", lambda: oh.HPLMM._coarse_factor(self))

        def _build_smoothers(self):
            stamp("contacts_s", lambda: oh.HPLMM._build_smoothers(self))

    t0 = time.perf_counter()
    H = Timed(problem, A=A, b=b, mesh=mesh, n=mortar)
    t1 = time.perf_counter()
    n_app = [0]

    def M(r):
        n_app[0] += 1
        if progress and n_app[0] % 10 == 0:
            print(f"# oracle {label}: {n_app[0]} applications, {time.perf_counter() - t1:.1f} s", file=sys.stderr,
                  flush=True)
        return H.apply(r)

    r = gmres.gmres(A, b, M, tol=1e-8, restart=50, maxit=300, flexible=True)
    t2 = time.perf_counter()
    return {"setup_s": round(t1 - t0, 3), "phases_s": {k: round(v, 3) for k, v in ph.items()},
            "solve_s": round(t2 - t1, 3), "iters": int(r.iters), "rel_res_true": float(r.rel_res),
            "dofs": int(A.shape[0]), "coarse_dofs": int(H.Acoarse.shape[0]),
            "subdomains": int(sum(1 for g in H.part.grain_nodes if len(g)))}


def _blas_threads():
    """Threads of the BLAS / OpenMP pools loaded in this process (the largest)."""
    try:
        import threadpoolctl
        return max([p.get("num_threads", 1) for p in threadpoolctl.threadpool_info()] or [1])
    except Exception:
        return None


def cpu_full(a):
    """--cpu-full: the oracle on the whole workload (no GPU), with the BLAS
    threads limited to --cpu-threads (0: as configured); prints one JSON line."""
    import contextlib
    # load every BLAS the oracle uses before limiting their threads (a limit
    # reaches only the libraries loaded when it is set)
    import scipy.linalg  # noqa: F401
    import scipy.sparse.linalg  # noqa: F401
    from oracle import fem, gmres, hplmm  # noqa: F401
    try:
        import threadpoolctl
        lim = threadpoolctl.threadpool_limits(a.cpu_threads) if a.cpu_threads > 0 else contextlib.nullcontext()
    except Exception:
        lim = contextlib.nullcontext()
    with lim:
        threads = _blas_threads()
        rec = oracle_timed(make_problem(a, a.n), a.mortar, label=f"{a.n}^3, {threads} threads", progress=True)
    rec.update({"workload": workload_name(a), "blas_threads": threads, "host_cpus": len(os.sched_getaffinity(0)),
                "oracle_sha256": _source_hash(ORACLE_FILES),
                "setup_plus_solve_ms": round((rec["setup_s"] + rec["solve_s"]) * 1e3, 1)})
    print(json.dumps(rec), flush=True)


def cpu_baseline(a, gpu_iters, gpu_dofs, full_grains):
    """The oracle beside the GPU.  Live: the untuned oracle on a bounded sample
    of the workload, the lower 32^3 corner of the same fields with the same
    8^3 boxes (about 10 s of host work), timed by phase.  Measured: the same
    oracle on the whole workload on this host type, all cores and one BLAS
    thread (the paper's serial protocol), from the committed record of
    `bench.py --cpu-full`; it gives `value` when it was taken on the current
    oracle sources, otherwise `value` falls back to the sample scaled by the
    subdomain count (set-up) and by dofs x iterations (solve) -- a lower
    bound, since the oracle's dense coarse factor grows with the cube of the
    coarse size."""
    from paper_2509_19777_amd import synth
    if a.workload == "uneven":
        sub = make_problem(a, CPU_SAMPLE_N)
        what = f"a {CPU_SAMPLE_N}^3 realisation of the same generator"
    else:
        sub = synth.crop(synth.config_grf(a.n, a.box, seed=2, n_mortar=a.mortar), CPU_SAMPLE_N, box=a.box)
        what = f"the {CPU_SAMPLE_N}^3 corner crop of the same fields"
    live = oracle_timed(sub, a.mortar)
    live.update({"what": what, "blas_threads": _blas_threads()})
    full = None
    if os.path.exists(CPU_FULL_RECORD) and a.workload == "grf" and a.n == 64 and a.box == 8 and a.mortar == 4:
        try:
            full = json.load(open(CPU_FULL_RECORD))
            if full.get("oracle_sha256") != _source_hash(ORACLE_FILES):
                full = None
        except Exception:
            full = None
    if full:
        allc, one = full["all_cores"], full["one_thread"]
        return {"value": allc["setup_plus_solve_ms"], "unit": "ms", "cores": allc["blas_threads"],
                "kind": "oracle-measured",
                "sample": (f"the whole workload ({allc['dofs']} dofs, {allc['coarse_dofs']} coarse dofs, "
                           f"{allc['iters']} iterations) measured with bench.py --cpu-full on the box host: "
                           f"set-up {allc['setup_s']:.1f} s + solve {allc['solve_s']:.1f} s with "
                           f"{allc['blas_threads']} BLAS threads; {one['setup_s']:.1f} s + {one['solve_s']:.1f} s "
                           f"with one thread"),
                "one_thread": {"value": one["setup_plus_solve_ms"], "unit": "ms", "cores": 1},
                "record": os.path.relpath(CPU_FULL_RECORD, ROOT),
                "live_sample": live}
    n_sub = live["subdomains"]
    setup_ms = live["setup_s"] * 1e3 * full_grains / n_sub
    solve_ms = live["solve_s"] * 1e3 * (gpu_dofs / live["dofs"]) * (gpu_iters / max(live["iters"], 1))
    return {"value": round(setup_ms + solve_ms, 1), "unit": "ms", "cores": live["blas_threads"], "kind": "oracle",
            "sample": (f"oracle set-up + FGMRES(50) to 1e-8 on {what} ({live['dofs']} dofs, {n_sub} subdomains, "
                       f"{live['iters']} iterations, set-up {live['setup_s']:.2f} s, solve {live['solve_s']:.2f} s); "
                       f"scaled x{full_grains / n_sub:.1f} (set-up), x{gpu_dofs / live['dofs']:.1f} dofs "
                       f"x{gpu_iters / max(live['iters'], 1):.2f} iterations (solve): a lower bound"),
            "live_sample": live}


if __name__ == "__main__":
    main()
