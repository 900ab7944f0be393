#!/usr/bin/env python3
"""Time-to-solution benchmark of the deflated block-AMG CG solve on one MI355X.

Workload: 150^3 7-point Poisson with log-normal cell coefficients (sigma = 2,
seed 0), right-hand side U[-1,1] (seed 1), 64 box subdomains, linear deflation
(4 vectors per subdomain), smoothed-aggregation AMG with SPAI-0, CG to
rtol 1e-8.  One step = one complete solve through the C ABI (permutation in,
initial projection, all Krylov iterations, solution recovery, true residual,
permutation out) with inputs resident in HBM.

The JSON line reports the FP64 path as `value` (seconds per solve), the
mixed-precision path (FP32 hierarchy / FP64 Krylov and deflation) and, unless
--no-batched, the 48-system batched solve (mixed and FP64) next to it, the
32^3 eight-slab Poisson solve (cache-resident), the roofline of the dominant
kernel (the slower of the outer SpMV with its fused epilogue and the level-0
restriction) measured with HIP events inside the timed solves, the rate of
every kernel span against the HBM peak, and the CPU oracle timed on a
bounded sample.

Layouts: the autotuner's choices are read from (and new ones appended to) the
record named by DFAMG_TUNE_CACHE, by default the one shipped with the package,
so that the timed solves and the profiler runs dispatch the same kernels.

    python bench.py [--gpus 1] [--steps 5] [--warmup 1]
"""
import argparse
import hashlib
import json
import os
import re
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "time-to-solution at rtol 1e-8 (FP64 vs mixed vs batched); SpMV HBM GB/s % peak"
# device code of the outer-operator kernel (its launcher, views and body)
KERNEL_SOURCES = ["paper_1710_03940_amd/csrc/kernels.hpp", "paper_1710_03940_amd/csrc/launch_outer.hip",
                  "paper_1710_03940_amd/csrc/launch_vcycle.hip", "paper_1710_03940_amd/csrc/devmat.hpp"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "lognormal150_traffic.json")
TUNE_RECORD = os.path.join(ROOT, "paper_1710_03940_amd", "tuned_layouts_gfx950.txt")
# what each per-span figure covers (DFAMG_KERNEL_* spans of the FP64 CG iteration)
SPAN_DOC = {
    "spmv": "k_outer: outer SpMV q = A p with the fused (p,q) and Z^T q epilogue",
    "project": "t1 sums per system, t2 = E^-1 t1 (one wavefront per row), alpha",
    "update": "y += alpha p, r -= alpha (q - AZ t2), ||r||^2 partials",
    "test": "stopping test (per-system reductions)",
    "presmooth0": "level 0: B0 = R0 (I - A0 diag(m0)) applied to r (pre-smoothing, residual, restriction)",
    "restrict0": "level 0: restriction when it is not fused into presmooth0",
    "coarser": "levels >= 1 and every coarsest direct solve (= restrict1 + deep + up1)",
    "prolong0": "level 0: z = m r + P0 x1",
    "postsmooth0": "level 0: s = z + m (r - A0 z) with (r,s) partials",
    "direction": "beta from (r,s); p = s + beta p",
    "restrict1": "level 1: B1 applied (pre-smoothing, residual, restriction)",
    "deep": "levels >= 2 and all coarsest dense solves",
    "up1": "level 1: prolongation and post-smoothing",
}


def kernel_source_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


# --------------------------------------------------------------------------
# CPU baseline: the oracle, in a child process with one BLAS thread
# --------------------------------------------------------------------------

def cpu_baseline_worker(sample_iters):
    import numpy as np
    from workloads import config_lognormal_poisson
    from oracle import OracleSolver
    P = config_lognormal_poisson()
    t0 = time.perf_counter()
    S = OracleSolver(P.A, P.part, P.nsub, P.Z)
    t_setup = time.perf_counter() - t0
    t0 = time.perf_counter()
    r = S.solve(P.b, maxiter=sample_iters)
    t_solve = time.perf_counter() - t0
    import scipy
    print(json.dumps({"setup_s": t_setup, "sample_iters": r["iters"], "sample_s": t_solve,
                      "numpy": np.__version__, "scipy": scipy.__version__,
                      "threads_env": {k: os.environ.get(k) for k in
                                      ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")}}),
          flush=True)


def start_cpu_baseline(sample_iters):
    env = dict(os.environ)
    for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        env[k] = "1"
    return subprocess.Popen([sys.executable, os.path.abspath(__file__), "--cpu-baseline-worker",
                             "--sample-iters", str(sample_iters)],
                            stdout=subprocess.PIPE, stderr=subprocess.PIPE, env=env, text=True)


# --------------------------------------------------------------------------
# GPU timing
# --------------------------------------------------------------------------

def time_solver(S, b, x, steps, warmup, log):
    import torch
    out = None
    for _ in range(warmup):
        x.zero_()
        out = S.solve(b, x, history=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    iters, each = [], []
    for _ in range(steps):
        t1 = time.perf_counter()
        x.zero_()
        out = S.solve(b, x, history=False)   # returns after the stream is synchronised
        each.append(time.perf_counter() - t1)
        iters.append(out["iters"])
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    out["median_s"] = sorted(each)[len(each) // 2]
    log(f"  {steps} solves: {dt * 1e3:.2f} ms/solve (median {out['median_s'] * 1e3:.2f}), iterations {iters}, "
        f"relres_true {out['relres_true']:.3e}")
    return dt, out, iters


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-breakdown", action="store_true")
    ap.add_argument("--no-oseen", action="store_true")
    ap.add_argument("--no-bicgstab2", action="store_true")
    ap.add_argument("--no-fgmres", action="store_true")
    ap.add_argument("--no-schur", action="store_true")
    ap.add_argument("--no-coarse-inverse", action="store_true")
    ap.add_argument("--no-small", action="store_true")
    ap.add_argument("--only", choices=["oseen", "batched", "small"],
                    help="run one leg alone and print its result (for kernel traces of that workload)")
    ap.add_argument("--record-layouts", metavar="FILE",
                    help="write the layouts the FP64 and mixed handles chose (for --traffic-from)")
    ap.add_argument("--sample-iters", type=int, default=20)
    ap.add_argument("--cpu-baseline-worker", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="time a 2 GiB device copy (streaming ceiling; reference for HBM counters)")
    ap.add_argument("--traffic-from", nargs=5,
                    metavar=("BENCH_FETCH", "BENCH_WRITE", "COPY_FETCH", "COPY_WRITE", "LAYOUTS"),
                    help="rocprofv3 --pmc CSVs of FETCH_SIZE / WRITE_SIZE for bench and for --copy-calibration, "
                         "and the --record-layouts file of the profiled bench run; writes the traffic file "
                         "read by the roofline")
    args = ap.parse_args()
    if args.copy_calibration:
        return copy_calibration()
    if args.traffic_from:
        return write_traffic(*args.traffic_from)

    if args.cpu_baseline_worker:
        cpu_baseline_worker(args.sample_iters)
        return 0
    if args.gpus != 1:
        print("bench.py measures one GPU: the deflated solve is not sharded across GPUs "
              "(run with --gpus 1)", file=sys.stderr)
        return 2

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    if args.only:
        os.environ.setdefault("DFAMG_TUNE_CACHE", TUNE_RECORD)
        leg = {"oseen": bench_oseen, "batched": bench_batched, "small": bench_small}[args.only]
        print(json.dumps({"leg": args.only, "result": leg(args, log)}), flush=True)
        return 0

    cpu_proc = None if args.no_cpu_baseline else start_cpu_baseline(args.sample_iters)

    os.environ.setdefault("DFAMG_TUNE_CACHE", TUNE_RECORD)
    import numpy as np
    import torch
    import paper_1710_03940_amd as dfamg
    from workloads import config_lognormal_poisson

    dev = torch.device("cuda:0")
    log("generating the 150^3 log-normal Poisson problem")
    P = config_lognormal_poisson()
    b = torch.tensor(P.b, device=dev)
    x = torch.zeros(P.n, dtype=torch.float64, device=dev)

    log("setup FP64 (hierarchies built on the GPU)")
    t0 = time.perf_counter()
    S64 = dfamg.Solver(P.A, P.part, P.nsub, P.Z, precision="fp64", profile=1, setup_device=1)
    t_setup64 = time.perf_counter() - t0
    st64 = S64.stats()
    log(f"  setup {t_setup64:.2f} s: host part {st64['setup_host_s']:.2f} s (hierarchies on the GPU "
        f"{st64['setup_hierarchy_s']:.2f} s), device part {st64['setup_device_s']:.2f} s, "
        f"levels {st64['level_rows']}")
    setup = setup_phases(dfamg, P, st64, t_setup64, log)
    log(f"  layouts: {st64['layouts']}")
    if args.record_layouts:
        with open(args.record_layouts, "w") as fh:
            json.dump({"fp64": parse_layouts(st64["layouts"]), "text": st64["layouts"]}, fh, indent=1)
    log("timing FP64")
    t64, out64, it64 = time_solver(S64, b, x, args.steps, args.warmup, log)
    st64 = S64.stats()
    x64 = x.clone()
    golden = load_golden("poisson150_lognormal2_boxes64_linear")
    err64 = error_vs_oracle(x64, golden)
    log(f"  FP64 error against the stored oracle solution (sampled): {err64:.2e}")

    result = {}
    mixed = None
    if not args.no_mixed:
        log("setup mixed")
        Sm = dfamg.Solver(P.A, P.part, P.nsub, P.Z, precision="mixed", profile=1)
        log("timing mixed")
        tm, outm, itm = time_solver(Sm, b, x, args.steps, args.warmup, log)
        stm = Sm.stats()
        diff = float(torch.linalg.norm(x - x64) / torch.linalg.norm(x64))
        mixed = {"s_per_solve": tm, "median_s": outm["median_s"], "iters": itm[-1],
                 "relres_true": outm["relres_true"],
                 "speedup_vs_fp64": t64 / tm, "rel_diff_vs_fp64_solution": diff,
                 "rel_error_vs_oracle_sampled": error_vs_oracle(x, golden),
                 "bytes_per_iter": stm["bytes_per_iter"]}
        Sm.close()

    bicgstab2 = None
    if not args.no_bicgstab2:
        # the solver of the paper's Poisson runs, on the same problem
        bicgstab2 = {}
        g2 = load_golden("poisson150_lognormal2_boxes64_linear_bicgstab2")
        for prec in ("fp64", "mixed"):
            S2 = dfamg.Solver(P.A, P.part, P.nsub, P.Z, solver="bicgstab2", precision=prec)
            log(f"timing BiCGStab(2) {prec}")
            t2s, o2, it2 = time_solver(S2, b, x, args.steps, args.warmup, log)
            S2.close()
            bicgstab2[prec] = {"s_per_solve": t2s, "median_s": o2["median_s"], "iters": it2[-1],
                               "relres_true": o2["relres_true"],
                               "rel_error_vs_oracle_sampled": error_vs_oracle(x, g2)}
        bicgstab2["oracle_iters"] = g2["iters"]
        bicgstab2["note"] = "iterations are BiCGStab(2) cycles, four operator products each"

    fgmres = None
    if not args.no_fgmres:
        # restarted flexible GMRES on A x = b with the deflation as part of
        # the preconditioner: exact FP64 E^{-1} and the inexact FP32 one
        fgmres = {}
        gf = load_golden("poisson150_lognormal2_boxes64_linear_fgmres30_fp32coarse")
        gcg = load_golden("poisson150_lognormal2_boxes64_linear_fgmres30_cgcoarse")
        for coarse, prec in (("exact", "fp64"), ("fp32", "fp64"), ("fp32", "mixed"), ("cg", "fp64")):
            Sf = dfamg.Solver(P.A, P.part, P.nsub, P.Z, solver="fgmres", restart=30, coarse_solve=coarse,
                              precision=prec, coarse_rtol=1e-2, coarse_maxiter=100)
            log(f"timing FGMRES(30) coarse {coarse} {prec}")
            tfs, of, itf = time_solver(Sf, b, x, args.steps, args.warmup, log)
            stf = Sf.stats()
            Sf.close()
            gref = gcg if coarse == "cg" else gf
            fgmres[f"{coarse}_coarse_{prec}"] = {
                "s_per_solve": tfs, "median_s": of["median_s"], "iters": itf[-1],
                "relres_true": of["relres_true"], "rel_error_vs_oracle_sampled": error_vs_oracle(x, gref),
                "oracle_iters": gref["iters"], "bytes_per_iter": stf["bytes_per_iter"]}
            if coarse == "cg":
                fgmres[f"{coarse}_coarse_{prec}"]["coarse_cg_steps"] = stf["coarse_iters"]
        fgmres["note"] = ("oracle: FGMRES(30) with the FP32 coarse solve (exact and fp32 rows) or the CG "
                          "coarse solve to 1e-2 (cg row); the deflated CG on the same problem is the "
                          "headline value")

    oseen = None
    if not args.no_oseen:
        try:
            oseen = bench_oseen(args, log)
        except Exception as exc:  # reported, never silently dropped
            oseen = {"error": str(exc)}

    schur = None
    if not args.no_schur:
        try:
            schur = bench_schur(args, log)
        except Exception as exc:  # reported, never silently dropped
            schur = {"error": str(exc)}

    coarse_inverse = None
    if not args.no_coarse_inverse:
        try:
            coarse_inverse = bench_coarse_inverse(log)
        except Exception as exc:  # reported, never silently dropped
            coarse_inverse = {"error": str(exc)}

    batched = None
    if not args.no_batched:
        try:
            batched = bench_batched(args, log)
        except Exception as exc:  # reported, never silently dropped
            batched = {"error": str(exc)}

    # roofline of the dominant kernel, from events recorded in the timed solves
    copy_gbps = copy_ceiling_gbps()
    log(f"  streaming copy ceiling {copy_gbps:.0f} GB/s")
    layouts64 = parse_layouts(st64["layouts"])
    live = {}
    for name in ("spmv", "presmooth0"):
        k = st64["kernels"][name]
        if k["calls"]:
            avg_s = k["ms"] / k["calls"] * 1e-3
            live[name] = {"avg_us": avg_s * 1e6, "bytes_per_launch": k["bytes"],
                          "achieved": k["bytes"] / avg_s / 1e9, "launches_timed": k["calls"]}
    dom = max(live, key=lambda kname: live[kname]["avg_us"])
    traffic = load_traffic(dom, layouts64)
    roofline = {"bound": "hbm", "achieved": live[dom]["achieved"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": live[dom]["achieved"] / HBM_PEAK_GBS,
                "traffic": traffic["bytes_per_launch"] if traffic else None,
                "kernel": SPAN_DOC[dom], "span": dom, "layout": layouts64.get(dom),
                "avg_us": live[dom]["avg_us"], "bytes_per_launch": live[dom]["bytes_per_launch"],
                "copy_ceiling": copy_gbps, "frac_of_copy": live[dom]["achieved"] / copy_gbps,
                "events_in_graph": st64["profile_in_graph"],
                "other": {kname: dict(v, frac=v["achieved"] / HBM_PEAK_GBS, layout=layouts64.get(kname),
                                      traffic=(load_traffic(kname, layouts64) or {}).get("bytes_per_launch"))
                          for kname, v in live.items() if kname != dom}}
    if dom == "spmv":
        roofline["layout_bytes_per_launch"] = st64["outer_layout_bytes"]
    kernels = kernel_breakdown(P, b, x, log, "fp64") if not args.no_breakdown else None
    kernels_mixed = kernel_breakdown(P, b, x, log, "mixed") if not (args.no_breakdown or args.no_mixed) else None
    small = None if args.no_small else bench_small(args, log)

    cpu = None
    if cpu_proc is not None:
        log("waiting for the CPU oracle baseline")
        outs, errs = cpu_proc.communicate(timeout=900)
        try:
            cb = json.loads(outs.strip().splitlines()[-1])
            per_it = cb["sample_s"] / max(cb["sample_iters"], 1)
            cpu = {"value": per_it * out64["iters"], "unit": "s", "cores": 1, "kind": "oracle",
                   "sample": (f"oracle deflated CG on the full 150^3 problem for {cb['sample_iters']} "
                              f"iterations ({cb['sample_s']:.1f} s, setup {cb['setup_s']:.1f} s "
                              f"excluded), scaled to {out64['iters']} iterations; SciPy sparse "
                              f"products are single-threaded"),
                   "numpy": cb.get("numpy"), "scipy": cb.get("scipy"), "threads_env": cb.get("threads_env"),
                   "host_cores_available": len(os.sched_getaffinity(0))}
        except Exception as exc:
            cpu = {"error": f"{exc}: {errs[-400:]}"}

    line = {
        "metric": METRIC, "value": t64, "unit": "s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": t64 * 1e3, "higher_is_better": False,
        "scaling": "strong", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "poisson150_lognormal2_boxes64_linear_cg",
                   "n": P.n, "nnz": int(P.A.nnz), "subdomains": P.nsub, "deflation": "linear",
                   "rtol": 1e-8, "smoother": "spai0", "solver": "cg"},
        "iters": out64["iters"], "relres_true": out64["relres_true"], "median_s": out64["median_s"],
        "oracle_iters": golden["iters"], "rel_error_vs_oracle_sampled": err64,
        "setup_s": setup,
        "bytes_per_iter": st64["bytes_per_iter"],
        "effective_GBps": st64["bytes_per_iter"] * out64["iters"] / t64 / 1e9,
        "layouts": st64["layouts"],
        "mixed": mixed, "batched": batched, "small": small, "oseen": oseen, "bicgstab2": bicgstab2,
        "fgmres": fgmres, "schur": schur, "coarse_inverse": coarse_inverse,
        "roofline": roofline,
        "kernels": kernels, "kernels_mixed": kernels_mixed,
        "cpu_baseline": cpu,
    }
    S64.close()
    print(json.dumps(line), flush=True)
    return 0


COPY_BYTES = 1 << 31


def load_golden(name):
    """Stored oracle result of a workload (written by tests/golden/make_golden.py)."""
    with open(os.path.join(ROOT, "tests", "golden", name + ".json")) as fh:
        return json.load(fh)


def error_vs_oracle(x, golden):
    """||x - x_oracle|| / ||x_oracle|| over the oracle's stored sample entries."""
    import numpy as np
    idx = np.array(golden["sample_index"])
    xs = x.cpu().numpy()[idx]
    gs = np.array(golden["sample_x"])
    return float(np.linalg.norm(xs - gs) / np.linalg.norm(gs))


def copy_ceiling_gbps(nbytes=1 << 30, reps=10):
    """Read+write bandwidth of a plain device copy (b = -a): the streaming
    ceiling the kernels are compared with besides the spec-sheet peak."""
    import torch
    a = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(3):
        torch.neg(a, out=b)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        torch.neg(a, out=b)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    del a, b
    return 2 * nbytes / dt / 1e9


def copy_calibration():
    """Plain device copy of COPY_BYTES: the streaming ceiling of the device,
    and the known-size reference for the HBM traffic counters."""
    import torch
    n = COPY_BYTES // 8
    # uninitialised on purpose: the only kernels of this run are the copies
    # (b = -a, one ordinary elementwise kernel reading and writing COPY_BYTES)
    a = torch.empty(n, dtype=torch.float64, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(3):
        torch.neg(a, out=b)
    torch.cuda.synchronize()
    reps = 10
    t0 = time.perf_counter()
    for _ in range(reps):
        torch.neg(a, out=b)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    print(json.dumps({"copy_bytes": COPY_BYTES, "s": dt,
                      "GBps_read_plus_write": 2 * COPY_BYTES / dt / 1e9}), flush=True)
    return 0


def parse_layouts(text):
    """Layout strings per profiled span from the stats' layout text, e.g.
    'outer sell1/i32; L0{A sell2/i16/stage, B csr16/t64/glist, P ...} ...':
    spmv -> the outer operator's, presmooth0 -> level 0's B (or A when the
    level-0 restriction is not fused), prolong0 -> P of level 0,
    postsmooth0 -> A of level 0."""
    out = {}
    m = re.search(r"outer ([^;]+);", text)
    if m:
        out["spmv"] = m.group(1).strip()
    m = re.search(r"L0\{([^}]*)\}", text)
    if m:
        parts = dict(p.strip().split(" ", 1) for p in m.group(1).split(",") if " " in p.strip())
        if "B" in parts:
            out["presmooth0"] = "B " + parts["B"]
        elif "A" in parts:
            out["presmooth0"] = "A " + parts["A"]
        if "P" in parts:
            out["prolong0"] = "P " + parts["P"]
        if "A" in parts:
            out["postsmooth0"] = "A " + parts["A"]
    return out


def load_traffic(span, layouts):
    """Counter-derived HBM bytes per launch of `span`, only when they were
    taken on the same kernel source and the same layout as the timed run."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    with open(TRAFFIC_FILE) as fh:
        tf = json.load(fh)
    e = tf.get("kernels", {}).get(span)
    if not e or e.get("kernel_source_hash") != kernel_source_hash():
        return None
    if e.get("layout") != layouts.get(span):
        return None
    return e


# kernels whose launches the counters isolate: span -> (name prefix, rule) of
# each kernel that one launch of the span dispatches; the in-loop instance is
# the most often dispatched (name, grid) group, and of the restriction groups
# (one per level, dispatched as often as each other) the heaviest, the one
# whose launches move the most bytes (level 0).  The level-0 restriction in
# the column-tiled layout ("B seg...") is two kernels: the partial sums per
# column tile and their sum per row.
def traffic_kernels(span, layout):
    if span == "spmv":
        return [("k_outer<0,", "most")]
    if layout and layout.startswith("B seg"):
        return [("k_seg_partial<double, double,", "heaviest"), ("k_seg_combine<double>", "heaviest")]
    return [("k_restrict<double, double,", "heaviest")]


TRAFFIC_SPANS = ("spmv", "presmooth0")


def _pmc_groups(csv_path, prefix, counter):
    """Per-dispatch counter values (KiB) of the kernels whose name contains
    `prefix`, grouped by (kernel name, grid size)."""
    import collections
    import csv
    by = collections.defaultdict(list)
    with open(csv_path) as fh:
        for row in csv.DictReader(fh):
            if prefix in row.get("Kernel_Name", "") and row.get("Counter_Name", counter) == counter:
                by[(row["Kernel_Name"], int(float(row.get("Grid_Size", 0) or 0)))].append(float(row["Counter_Value"]))
    return by


def _pick_group(by, rule):
    import statistics
    if not by:
        return None
    if rule == "most":
        return max(by, key=lambda k: len(by[k]))
    top = max(len(v) for v in by.values())
    busy = [k for k in by if len(by[k]) >= top // 2]
    return max(busy, key=lambda k: statistics.median(by[k]))


def _pmc_kib(csv_path, name_part, counter):
    """Per-dispatch counter values (KiB) of kernels whose name contains name_part."""
    import csv
    vals = []
    with open(csv_path) as fh:
        for row in csv.DictReader(fh):
            if name_part in row.get("Kernel_Name", "") and row.get("Counter_Name", counter) == counter:
                vals.append(float(row["Counter_Value"]))
    return vals


def write_traffic(bench_fetch, bench_write, copy_fetch, copy_write, layouts_file):
    """HBM bytes per launch of the outer SpMV and of the level-0 restriction
    from FETCH_SIZE / WRITE_SIZE, scaled by what the same counters read for the
    plain copy of COPY_BYTES; tagged with the layouts the profiled run used."""
    import statistics
    cf = statistics.median(_pmc_kib(copy_fetch, "elementwise", "FETCH_SIZE"))
    cw = statistics.median(_pmc_kib(copy_write, "elementwise", "WRITE_SIZE"))
    fscale = (COPY_BYTES / 1024.0) / cf      # true KiB per counted KiB
    wscale = (COPY_BYTES / 1024.0) / cw
    with open(layouts_file) as fh:
        lay = json.load(fh)["fp64"]
    out = {"note": "HBM bytes per launch from rocprofv3 FETCH_SIZE / WRITE_SIZE (KiB per dispatch), "
                   "scaled by the counters' reading of a plain copy of known size; only launches that did "
                   "work (above half the group's largest reading) count", "kernels": {}}
    for span in TRAFFIC_SPANS:
        names, grids, counted = [], [], []
        fetch = write = 0.0
        for prefix, rule in traffic_kernels(span, lay.get(span)):
            fg = _pmc_groups(bench_fetch, prefix, "FETCH_SIZE")
            wg = _pmc_groups(bench_write, prefix, "WRITE_SIZE")
            key = _pick_group(fg, rule)
            if key is None or key not in wg:
                names = None
                break
            f, w = fg[key], wg[key]
            fbig = [v for v in f if v > 0.5 * max(f)]
            wbig = [v for v in w if v > 0.5 * max(w)]
            fetch += statistics.median(fbig) * fscale * 1024.0
            write += statistics.median(wbig) * wscale * 1024.0
            names.append(key[0])
            grids.append(key[1])
            counted.append([len(fbig), len(wbig)])
        if not names:
            continue
        one = len(names) == 1
        out["kernels"][span] = {"kernel": names[0] if one else " + ".join(names), "grid": grids[0] if one else grids,
                                "layout": lay.get(span),
                                "bytes_per_launch": fetch + write, "fetch_bytes": fetch, "write_bytes": write,
                                "copy_scale_fetch": fscale, "copy_scale_write": wscale,
                                "launches_counted": counted[0] if one else counted,
                                "kernel_source_hash": kernel_source_hash()}
    os.makedirs(os.path.dirname(TRAFFIC_FILE), exist_ok=True)
    with open(TRAFFIC_FILE, "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out))
    return 0


def setup_phases(dfamg, P, st, total, log):
    """Setup of the timed FP64 handle in phases, and the same plan (validation,
    permutation, hierarchies, AZ, E, packing) built with the hierarchies and AZ
    on the host and on the GPU."""
    out = {"total_s": total, "plan_s": st["setup_host_s"], "hierarchies_s": st["setup_hierarchy_s"],
           "hierarchies_on": "gpu" if st["setup_hierarchy_device"] else "host",
           "device_s": st["setup_device_s"],
           "note": "plan_s: validation, permutation, hierarchies, AZ, E and packing; device_s: uploads, layouts "
                   "(from the layout record), E inversion; the hierarchies are bit-for-bit those of the host"}
    for dev in (0, 1):
        t0 = time.perf_counter()
        p = dfamg.dfamg_plan_create(dfamg.make_params(setup_device=dev), P.A, P.part, P.nsub, P.Z)
        out[("plan_gpu_s" if dev else "plan_host_s")] = time.perf_counter() - t0
        dfamg.dfamg_plan_destroy(p)
    log(f"  plan with host hierarchies {out['plan_host_s']:.2f} s, with GPU hierarchies {out['plan_gpu_s']:.2f} s")
    return out


def span_rates(st):
    """Per-span average time, algorithmic bytes, rate and fraction of the HBM
    peak from a handle's profile."""
    out = {}
    for name, kv in st["kernels"].items():
        if kv["calls"]:
            a = kv["ms"] / kv["calls"] * 1e-3
            gbps = kv["bytes"] / a / 1e9 if kv["bytes"] and a > 0 else None
            out[name] = {"avg_us": a * 1e6, "bytes_per_launch": kv["bytes"] or None, "GBps": gbps,
                         "frac": gbps / HBM_PEAK_GBS if gbps else None}
    return out


def kernel_breakdown(P, b, x, log, precision):
    """Per-kernel spans of one path from a separate, untimed handle that
    records an event pair around every kernel span of each iteration."""
    import paper_1710_03940_amd as dfamg
    S = dfamg.Solver(P.A, P.part, P.nsub, P.Z, precision=precision, profile=2)
    for _ in range(2):
        x.zero_()
        S.solve(b, x, history=False)
    st = S.stats()
    S.close()
    out = span_rates(st)
    # the coarser span encloses the event nodes of its three sub-spans (six
    # per iteration, a few us each): report it as the sum of the sub-spans
    subs = ("restrict1", "deep", "up1")
    if "coarser" in out and all(k in out for k in subs):
        c = out["coarser"]
        a = sum(out[k]["avg_us"] for k in subs) * 1e-6
        gbps = c["bytes_per_launch"] / a / 1e9 if c["bytes_per_launch"] and a > 0 else None
        out["coarser"] = {"avg_us": a * 1e6, "bytes_per_launch": c["bytes_per_launch"], "GBps": gbps,
                          "frac": gbps / HBM_PEAK_GBS if gbps else None, "avg_us_enclosing_span": c["avg_us"],
                          "note": "sum of restrict1, deep and up1"}
    log(f"  per-kernel spans {precision} (us): " + ", ".join(f"{k} {v['avg_us']:.1f}" for k, v in out.items()))
    return out


def bench_small(args, log):
    """32^3 Poisson, 8 slabs, constant deflation, CG, FP64: the whole working
    set (about 20 MB) stays in the caches, so its rate is an effective one, not
    an HBM figure; the solve is bound by launch and synchronisation latency."""
    import torch
    import paper_1710_03940_amd as dfamg
    from workloads import config_small_poisson
    P = config_small_poisson()
    dev = torch.device("cuda:0")
    b = torch.tensor(P.b, device=dev)
    x = torch.zeros(P.n, dtype=torch.float64, device=dev)
    golden = load_golden("poisson32_slabs8_constant")
    S = dfamg.Solver(P.A, P.part, P.nsub, P.Z, precision="fp64")
    log("timing the 32^3 slab problem")
    t, o, its = time_solver(S, b, x, max(args.steps, 10), args.warmup, log)
    st = S.stats()
    S.close()
    return {"workload": "poisson32_unit_slabs8_constant_cg", "n": P.n, "nnz": int(P.A.nnz), "subdomains": P.nsub,
            "s_per_solve": t, "median_s": o["median_s"], "iters": its[-1], "oracle_iters": golden["iters"],
            "relres_true": o["relres_true"], "rel_error_vs_oracle_sampled": error_vs_oracle(x, golden),
            "bytes_per_iter": st["bytes_per_iter"], "us_per_iter": t / max(its[-1], 1) * 1e6,
            "effective_GBps_cache_resident": st["bytes_per_iter"] * its[-1] / t / 1e9,
            "note": "cache-resident working set: effective rate, latency-bound, not an HBM figure"}


def bench_oseen(args, log):
    """Q1 Oseen system (64^3 nodes x 4 fields, 256 subdomains, per-field
    deflation): BiCGStab with the FP32 block-SA preconditioner, and the same
    solve with an FP64 preconditioner for comparison."""
    import torch
    import paper_1710_03940_amd as dfamg
    from workloads import config_oseen
    log("generating the 64^3 Q1 Oseen problem")
    P = config_oseen()
    dev = torch.device("cuda:0")
    b = torch.tensor(P.b, device=dev)
    x = torch.zeros(P.n, dtype=torch.float64, device=dev)
    out = {"workload": P.name, "n": P.n, "nnz": int(P.A.nnz), "subdomains": P.nsub,
           "deflation": "per-field constant (4 per subdomain)", "solver": "bicgstab",
           "block_size": 4}
    golden = load_golden("oseen64_boxes256_field")
    out["oracle_iters"] = golden["iters"]
    for prec in ("mixed", "fp64"):
        S = dfamg.Solver(P.A, P.part, P.nsub, P.Z, solver="bicgstab", block_size=4, precision=prec)
        t, o, its = time_solver(S, b, x, args.steps, args.warmup, log)
        o["rel_error_vs_oracle_sampled"] = error_vs_oracle(x, golden)
        st = S.stats()
        S.close()
        log(f"  oseen {prec} layouts: {st['layouts']}")
        out[prec] = {"s_per_solve": t, "iters": its[-1], "relres_true": o["relres_true"],
                     "rel_error_vs_oracle_sampled": o["rel_error_vs_oracle_sampled"],
                     "setup_host_s": st["setup_host_s"], "setup_device_s": st["setup_device_s"],
                     "bytes_per_iter": st["bytes_per_iter"]}
        log(f"  oseen {prec}: {t * 1e3:.1f} ms, {its[-1]} iterations, relres {o['relres_true']:.2e}")
    out["speedup_mixed_vs_fp64"] = out["fp64"]["s_per_solve"] / out["mixed"]["s_per_solve"]
    # the block SPAI-0 smoother (4 x 4 node blocks) in place of scalar SPAI-0
    gb = load_golden("oseen64_boxes256_field_blockspai0")
    out["block_spai0"] = {"oracle_iters": gb["iters"]}
    for prec in ("mixed", "fp64"):
        S = dfamg.Solver(P.A, P.part, P.nsub, P.Z, solver="bicgstab", block_size=4, precision=prec,
                         smoother="block_spai0")
        t, o, its = time_solver(S, b, x, args.steps, args.warmup, log)
        S.close()
        out["block_spai0"][prec] = {"s_per_solve": t, "iters": its[-1], "relres_true": o["relres_true"],
                                    "rel_error_vs_oracle_sampled": error_vs_oracle(x, gb)}
        log(f"  oseen block SPAI-0 {prec}: {t * 1e3:.1f} ms, {its[-1]} iterations")
    return out


def bench_schur(args, log):
    """The 64^3 Oseen system (one backward-Euler step, dt = 0.1) solved by
    FGMRES(50) with the Schur pressure-correction preconditioner (FP64 and
    FP32 pressure AMG)."""
    import time
    import torch
    import paper_1710_03940_amd as dfamg
    from workloads import config_oseen_schur
    log("generating the 64^3 Oseen system for the Schur pressure correction")
    P, pmask, part_p, nsub, Zp = config_oseen_schur()
    golden = load_golden("oseen64_boxes256_schur")
    dev = torch.device("cuda:0")
    b = torch.tensor(P.b, device=dev)
    out = {"workload": P.name + "_dt0.1_schur", "n": P.n, "pressure_subdomains": nsub,
           "solver": "fgmres(50) + Schur pressure correction", "oracle_iters": golden["iters"]}
    for prec in ("fp64", "mixed"):
        t0 = time.time()
        S = dfamg.SchurSolver(P.A, pmask, part_p, nsub, Zp, precision=prec, rtol=1e-8)
        setup = time.time() - t0
        x = torch.zeros(P.n, dtype=torch.float64, device=dev)
        ts, o, its = time_solver(S, b, x, max(1, min(args.steps, 3)), args.warmup, log)
        st = S.stats()
        S.close()
        out[prec] = {"s_per_solve": ts, "median_s": o["median_s"], "iters": its[-1],
                     "relres_true": o["relres_true"], "rel_error_vs_oracle_sampled": error_vs_oracle(x, golden),
                     "inner_iters_velocity": st["schur_inner_iters"][0],
                     "inner_iters_pressure": st["schur_inner_iters"][1], "setup_s": setup}
        log(f"  schur {prec}: {ts * 1e3:.1f} ms, {its[-1]} iterations, relres {o['relres_true']:.2e}, "
            f"inner {st['schur_inner_iters']}")
    return out


def bench_coarse_inverse(log):
    """Setup on the GPU: the FP64 inverse of dense systems of the sizes the
    coarse operator E = Z^T A Z takes (m = subdomains x vectors), by the
    blocked Gauss-Jordan elimination (panel GEMMs on the FP64 matrix cores)
    and by the unblocked one, host copies included (the second of two calls
    is timed).  Each inverse is checked
    on 64 sampled rows of A X - I (a full host product would disturb the
    single-threaded CPU baseline running beside the benchmark)."""
    import time
    import numpy as np
    import paper_1710_03940_amd as dfamg
    log("dense FP64 inverses (coarse-operator sizes)")
    rows = []
    for n in (256, 1024, 2048, 4096):
        rng = np.random.default_rng(n)
        A = rng.standard_normal((n, n)) + 2.0 * np.sqrt(n) * np.eye(n)
        pick = np.sort(rng.choice(n, size=min(n, 64), replace=False))
        row = {"m": n}
        for name, method in (("blocked", 0), ("unblocked", 1)):
            dt = 0.0
            for _ in range(2):   # the second call is timed (the first loads GEMM kernels of new shapes)
                t0 = time.perf_counter()
                X = dfamg.dfamg_dense_inverse(A, method)
                dt = time.perf_counter() - t0
            res = A[pick] @ X
            res[np.arange(len(pick)), pick] -= 1.0
            row[name + "_ms"] = dt * 1e3
            row[name + "_max_abs_AX_minus_I_sampled"] = float(np.abs(res).max())
        row["blocked_TFLOPs"] = 2.0 * n ** 3 / (row["blocked_ms"] * 1e-3) / 1e12
        rows.append(row)
        log(f"  m={n}: blocked {row['blocked_ms']:.1f} ms, unblocked {row['unblocked_ms']:.1f} ms, "
            f"max|AX-I| {max(row['blocked_max_abs_AX_minus_I_sampled'], row['unblocked_max_abs_AX_minus_I_sampled']):.1e}")
    return {"note": "dfamg_dense_inverse, host copies included; 2 m^3 flops per inverse; the library "
                    "takes the blocked form for systems with m >= 1024", "rows": rows}


def _time_batched(Sb, b, x, steps, warmup):
    import torch
    for _ in range(warmup):
        x.zero_()
        Sb.solve(b, x)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        x.zero_()
        out = Sb.solve(b, x)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps, out


def bench_batched(args, log):
    """48 independent systems in one handle (mixed and FP64) vs the same
    systems one by one (FP64): the batching gain is the FP64 batched time
    against the sequential one, the precision gain mixed against FP64 batched."""
    import numpy as np
    import torch
    import paper_1710_03940_amd as dfamg
    from workloads import config_batched, concat_problems
    probs = config_batched()
    A, part, nsub, Z, bvec, x0, off = concat_problems(probs)
    dev = torch.device("cuda:0")
    log(f"batched: {len(probs)} systems, {A.shape[0]} unknowns")
    b = torch.tensor(bvec, device=dev)
    x = torch.zeros(A.shape[0], dtype=torch.float64, device=dev)
    ns = np.diff(np.asarray(off))
    gsys = load_golden("batched48_sample")["systems"]
    res = {}
    for prec in ("mixed", "fp64"):
        Sb = dfamg.BatchedSolver(A, part, nsub, Z, off, precision=prec)
        tb, outb = _time_batched(Sb, b, x, args.steps, args.warmup)
        st = Sb.stats()
        Sb.close()
        its = np.asarray(outb["iters"])
        # bytes scale with the unknowns of each system: a system stops moving
        # data once it has converged (its tiles exit early)
        moved = st["bytes_per_iter"] * float((ns * its).sum()) / float(ns.sum())
        xs_all = x.cpu().numpy()
        errs = {}
        for key, gs in gsys.items():
            sidx = int(key)
            xs = xs_all[off[sidx] + np.array(gs["sample_index"])]
            ref = np.array(gs["sample_x"])
            errs[key] = float(np.linalg.norm(xs - ref) / np.linalg.norm(ref))
        res[prec] = {"s_per_batch": tb, "iters_max": int(its.max()), "iters_min": int(its.min()),
                     "relres_true_max": float(np.asarray(outb["relres_true"]).max()),
                     "rel_error_vs_oracle_sampled_max": max(errs.values()), "status": int(outb["status"]),
                     "bytes_per_iter_all_systems": st["bytes_per_iter"],
                     "effective_GBps": moved / tb / 1e9, "setup_device_s": st["setup_device_s"],
                     "setup_host_s": st["setup_host_s"]}
        log(f"  batched {prec}: {tb * 1e3:.2f} ms, iterations max {int(its.max())}, "
            f"effective {moved / tb / 1e9:.0f} GB/s")
    # plain FP64 path, one system after another
    solvers = []
    vecs = []
    for p in probs:
        solvers.append(dfamg.Solver(p.A, p.part, p.nsub, p.Z, precision="fp64"))
        vecs.append((torch.tensor(p.b, device=dev), torch.zeros(p.n, dtype=torch.float64, device=dev)))
    for S, (bb, xx) in zip(solvers, vecs):
        xx.zero_()
        S.solve(bb, xx, history=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(max(1, args.steps // 2)):
        for S, (bb, xx) in zip(solvers, vecs):
            xx.zero_()
            S.solve(bb, xx, history=False)
    torch.cuda.synchronize()
    ts = (time.perf_counter() - t0) / max(1, args.steps // 2)
    for S in solvers:
        S.close()
    log(f"  sequential fp64: {ts * 1e3:.2f} ms")
    return {"s_per_batch": res["mixed"]["s_per_batch"], "mixed": res["mixed"], "fp64": res["fp64"],
            "sequential_fp64_s": ts,
            "speedup_batching_fp64": ts / res["fp64"]["s_per_batch"],
            "speedup_precision_batched": res["fp64"]["s_per_batch"] / res["mixed"]["s_per_batch"],
            "speedup_vs_sequential_fp64": ts / res["mixed"]["s_per_batch"],
            "systems": len(probs), "unknowns": int(A.shape[0]),
            "oracle_sampled_systems": sorted(int(k) for k in gsys)}


if __name__ == "__main__":
    sys.exit(main())
