#!/usr/bin/env python3
"""Benchmark of the MI355X pipelined BiCGStab library.

Headline (``value``): p-BiCGStab iterations per second on the 200^3
convection-diffusion workload (N = 8e6, 7-point stencil, convection
(10, 5, 1), Jacobi, FP64, residual replacement every 50 iterations; its
working set of ~0.9 GB lives in HBM, far beyond the 256 MB Infinity Cache).
One *step* is one pbicgstab_solve call of 200 iterations: initialisation, 200
iterations of Algorithm 2 (phase A, v = A M^-1 z, phase B, t = A M^-1 w; the
GLRED finals in the first blocks of the products; 4 replacements), replayed
from HIP graphs, and the final FP64 true residual.  The tolerance 1e-10 is not
reached within 200 iterations (the workload needs ~2500), so every step
performs exactly 200 iterations.  The right-hand side lives in HBM before the
timed region starts.

Printed (one JSON line):
  value            FP64 iterations per second (iterations of the K timed
                   solves / their wall time)
  value_fp32_storage  the same with FP32 storage (FP64 dots, scalars, x and
                   replacement; products fused into the phase kernels)
  roofline         the FP64 phase B kernel (the largest HBM stream of the
                   iteration, 15 vectors of 8 B per row), algorithmic bytes per
                   launch / average launch duration from HIP events on the
                   library's stream; traffic = calibrated FETCH_SIZE +
                   WRITE_SIZE per launch from profiles/ (null when the kernel
                   source changed since the counters were taken)
  hbm_gbps_effective  algorithmic bytes of the whole iteration x iterations/s
  mixed_vs_fp64    time to a 1e-10 true residual, FP32 storage against FP64,
                   at equal replacement periods, without and (where a run
                   breaks down) with restarts
  paper_accuracy_vs_time  the paper's TP2 and TP3 (Table tab:specs) on one
                   GPU: relative true residual against seconds (Section 4.6)
  extras           C2 1000^2 Poisson (cache-resident), C1 32^2 latency
                   (classic vs pipelined), C4 and C5 iteration kernels, C5
                   full-size forward and adjoint outcome
  cpu_baseline     the oracle (NumPy/SciPy FP64, one thread) on 20 iterations
                   of the same 200^3 solve after 2 warm-up iterations
"""

from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published
ITERS_PER_STEP = 200
RR_PERIOD = 50
KERNELS_ONLY_REPS = 20
# FP64 bytes per row of the 200^3 iteration: phase A 13 and phase B 15 vector
# streams, each product 2 (the constant stencil and scalar Jacobi add none)
C3_FP64_BYTES_ROW = 32 * 8
# FP32 storage, products fused: phase A 13 and phase B 15 streams of 4 B, x
# read and written in FP64 (+8 B)
C3_FP32_BYTES_ROW = 28 * 4 + 8
PHASEB_FP64_BYTES_ROW = 15 * 8
PHASEB_FP32_BYTES_ROW = 13 * 4 + 16


# counted kernel per workload: (file prefix, hash key, kernel-name key per
# storage precision, algorithmic bytes per row per precision, rows)
_C4_ROWS, _C4_SLOTS = 2_000_000, 27
COUNTED = {
    "convdiff200": ("phaseB", "phaseB", {"fp64": "k_phaseB", "mixed": "k_phaseB"},
                    {"fp64": 15 * 8, "mixed": 13 * 4 + 16}, 200 ** 3),
    "poisson1000": ("phaseB", "phaseB", {"fp64": "k_phaseB", "mixed": "k_phaseB"},
                    {"fp64": 15 * 8, "mixed": 13 * 4 + 16}, 1000 ** 2),
    # the sliced-ELL product reading M^-1 z: the input and output vectors and
    # 27 (value, int32 column) slots per row
    "random2m": ("spmv_sell_lds", "spmv_sell_lds",
                 {"fp64": "k_spmv_sell_lds<double", "mixed": "k_spmv_sell_lds<float"},
                 {"fp64": 2 * 8 + _C4_SLOTS * 12, "mixed": 2 * 4 + _C4_SLOTS * 8}, _C4_ROWS),
}


def traffic_file(workload, precision):
    return os.path.join(HERE, "profiles",
                        f"{COUNTED[workload][0]}_{workload}_{precision}_traffic.txt")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--skip-cpu", action="store_true", help="omit the CPU oracle baseline")
    ap.add_argument("--skip-mixed", action="store_true", help="omit the mixed-vs-FP64 solves")
    ap.add_argument("--skip-extras", action="store_true",
                    help="omit the paper's accuracy runs and the other workloads")
    ap.add_argument("--cpu-iters", type=int, default=20)
    ap.add_argument("--graph", type=int, default=1, help="replay iteration chunks from HIP graphs")
    ap.add_argument("--kernels-only", action="store_true",
                    help="only launch the iteration kernels of one workload (the short program "
                         "that the rocprofv3 trace and counter runs profile)")
    ap.add_argument("--kernels-workload",
                    choices=("convdiff200", "poisson1000", "random2m", "kappa2048"),
                    default="convdiff200",
                    help="workload of --kernels-only: the 200^3 convection-diffusion problem, "
                         "the 1000^2 Poisson problem, the 2e6-row random matrix with 27 entries "
                         "per row (sliced ELL), or the 2048^2 variable-coefficient DIA5 operator "
                         "with its gradients")
    ap.add_argument("--kernels-precision", choices=("fp64", "mixed"), default="fp64")
    ap.add_argument("--c1-only", action="store_true",
                    help="only the 32^2 latency solves (classic, graphs, one workgroup): the "
                         "short program that the rocprofv3 trace of the single-workgroup "
                         "solve profiles; one JSON line")
    ap.add_argument("--summarize-pmc", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="turn two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE) of "
                         "--kernels-only into the traffic summary under profiles/")
    return ap.parse_args()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


_HASH_COMMON = ("common.hpp", ("double lane_xor(", "double wave_sum(", "void block_partials(",
                                "void ld16(", "void st16(", "void ldc(", "void stc(",
                                "struct XcdWalk"))
_HASH_PARTS = {
    "phaseB": (("kernels_vec.hip", ("struct PhaseBArgs", "struct BTile", "void phaseB_issue(",
                                    "void phaseB_stencil(", "void phaseB_update(",
                                    "void k_phaseB(", "void k_copy(", "bool marchable(",
                                    "auto tile_seq(", "bool march_fused(", "void march_rotate(",
                                    "void march_planes(")),
               _HASH_COMMON,
               ("ops.hpp", ("T prec1(", "void load_chunk(", "struct StParams", "struct TileSeq",
                            "struct RowSeq", "T st_row_sum(", "void st_apply(",
                            "void st_apply3_planes("))),
    "spmv_sell_lds": (("kernels_op.hip", ("struct LdsVis", "void k_spmv_sell_lds(",
                                          "void launch_spmv_lds(")),
                      ("kernels_vec.hip", ("void k_copy(",)),
                      _HASH_COMMON,
                      ("ops.hpp", ("struct SellOp",))),
}


def kernel_source_hash(kernel="phaseB"):
    """Hash of the device code a counted kernel and the copy kernel are built
    from (their definitions and the shared device helpers): a stored counter
    reading is used only while that code is unchanged."""
    import hashlib
    h = hashlib.sha256()
    for fname, starts in _HASH_PARTS[kernel]:
        src = open(os.path.join(HERE, "paper_1809_01948_amd/csrc", fname)).read()
        for start in starts:
            i = src.index(start)
            h.update(src[i:src.index("\n}\n", i)].encode())
    return h.hexdigest()[:16]


def read_pmc_dir(path, counter):
    """Per-dispatch values of one counter from a rocprofv3 --pmc CSV run:
    {kernel name: [value per dispatch]}."""
    import csv
    import glob
    out = {}
    files = glob.glob(os.path.join(path, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise SystemExit(f"no *counter_collection.csv under {path}")
    for fn in files:
        with open(fn) as f:
            for row in csv.DictReader(f):
                if row.get("Counter_Name") != counter:
                    continue
                out.setdefault(row["Kernel_Name"], []).append(float(row["Counter_Value"]))
    return out


def summarize_pmc(fetch_dir, write_dir, workload, precision):
    """FETCH_SIZE and WRITE_SIZE (KiB per dispatch) of the workload's counted
    kernel and of the plain copy kernel; the copy's known bytes calibrate
    each counter."""
    fetch = read_pmc_dir(fetch_dir, "FETCH_SIZE")
    write = read_pmc_dir(write_dir, "WRITE_SIZE")
    label, hkey, keys, per_row, n = COUNTED[workload]
    key = keys[precision]

    def pick(d, key):
        # dispatches of a converged solve's last graph chunk exit at once
        # (a few bytes each): only full launches are averaged
        vals = [v for k, vs in d.items() if key in k for v in vs]
        if not vals:
            raise SystemExit(f"no dispatch of {key} in the counter output")
        vals = [v for v in vals if v >= 0.5 * max(vals)]
        return sum(vals) / len(vals), len(vals)

    npad = (n + 2047) // 2048 * 2048
    copy_bytes = 8 * npad                               # read once, written once
    f_b, nf = pick(fetch, key)
    w_b, nw = pick(write, key)
    f_c, _ = pick(fetch, "k_copy")
    w_c, _ = pick(write, "k_copy")
    kf = copy_bytes / (f_c * 1024.0)
    kw = copy_bytes / (w_c * 1024.0)
    traffic = f_b * 1024.0 * kf + w_b * 1024.0 * kw
    algo = per_row[precision] * (npad if label == "phaseB" else n)
    kflag = "" if workload == "convdiff200" else f" --kernels-workload {workload}"
    pflag = "" if precision == "fp64" or workload == "random2m" \
        else f" --kernels-precision {precision}"
    fd, wd = os.path.relpath(fetch_dir, HERE), os.path.relpath(write_dir, HERE)
    lines = [
        f"# {label} ({key}), {workload} {precision}: HBM traffic per launch",
        f"source_hash {kernel_source_hash(hkey)}",
        "commands (from the repository root R; the profiler runs from /tmp):",
        f"  rocprofv3 --pmc FETCH_SIZE --output-format csv -d R/{fd} -- "
        f"python R/bench.py --kernels-only{kflag}{pflag}",
        f"  rocprofv3 --pmc WRITE_SIZE --output-format csv -d R/{wd} -- "
        f"python R/bench.py --kernels-only{kflag}{pflag}",
        f"  python bench.py --summarize-pmc {fd} {wd}{kflag}"
        f"{'' if precision == 'fp64' else ' --kernels-precision ' + precision}",
        f"full_dispatches {label} fetch {nf} write {nw}",
        f"FETCH_SIZE_KiB {label} {f_b:.1f} copy {f_c:.1f}",
        f"WRITE_SIZE_KiB {label} {w_b:.1f} copy {w_c:.1f}",
        f"copy_algorithmic_bytes_each_way {copy_bytes}",
        f"calibration_fetch {kf:.4f}",
        f"calibration_write {kw:.4f}",
        f"{label}_algorithmic_bytes {algo}",
        f"{label}_traffic_bytes {traffic:.0f}",
        f"traffic_over_algorithmic {traffic / algo:.4f}",
    ]
    with open(traffic_file(workload, precision), "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def stored_traffic(workload, precision):
    """Calibrated HBM bytes per phase B launch, or None when no counter
    reading exists for the current kernel sources."""
    try:
        kv = {}
        with open(traffic_file(workload, precision)) as f:
            for line in f:
                parts = line.split()
                if len(parts) == 2:
                    kv[parts[0]] = parts[1]
        label, hkey = COUNTED[workload][:2]
        if kv.get("source_hash") != kernel_source_hash(hkey):
            return None
        return float(kv[f"{label}_traffic_bytes"])
    except (OSError, KeyError, ValueError):
        return None


def cpu_model():
    """The host CPU's model name from /proc/cpuinfo (platform.processor()
    would start a child process)."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.machine()


def cpu_baseline(iters):
    """The oracle's p-BiCGStab (Algorithm 2) on the host, one thread: 2
    warm-up iterations, then `iters` timed iterations of the same 200^3 solve
    (a full solve would take hours)."""
    from threadpoolctl import threadpool_limits
    from oracle import Float64Ops, pipelined_bicgstab
    from workloads import convdiff3d_c3
    prob = convdiff3d_c3(200, with_csr=True)
    A = prob.scipy_csr()
    ops = Float64Ops(A, 1.0 / A.diagonal())
    with threadpool_limits(limits=1):
        pipelined_bicgstab(ops, prob.b, tol=0.0, maxit=2, rr_period=RR_PERIOD)   # warm-up
        t0 = time.perf_counter()
        res = pipelined_bicgstab(ops, prob.b, tol=0.0, maxit=iters, rr_period=RR_PERIOD)
        dt = time.perf_counter() - t0
    return {"value": res.iterations / dt, "unit": "iter/s", "cores": 1, "kind": "oracle",
            "sample": f"{res.iterations} iterations of the same 200^3 FP64 solve after 2 "
                      f"warm-up iterations (NumPy/SciPy FP64 CSR, 1 thread, {dt:.1f} s)",
            "host_cpus": os.cpu_count(), "cpu_model": cpu_model()}


def timed_steps(S, b, opts, steps, warmup, label):
    """W untimed solves, then K timed ones bracketed by device syncs."""
    import torch
    for w in range(warmup):
        _, st = S.solve(b, **opts)
        log(f"{label} warmup {w}: {st['status_name']} its={st['iterations']} "
            f"{st['elapsed_ms']:.1f} ms")
    torch.cuda.synchronize()
    its = 0
    stats = []
    t0 = time.perf_counter()
    for _ in range(steps):
        _, st = S.solve(b, **opts)
        its += st["iterations"]
        stats.append(st)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    for k, st in enumerate(stats):
        log(f"{label} step {k}: {st['status_name']} its={st['iterations']} "
            f"rr={st['replacements']} {st['elapsed_ms']:.1f} ms")
    if any(st["iterations"] != opts["maxit"] for st in stats):
        log(f"{label}: a timed solve stopped early")
    return its / dt, 1000.0 * dt / steps, stats


def solve_timed(S, b, **kw):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    x, st = S.solve(b, **kw)
    torch.cuda.synchronize()
    return x, st, time.perf_counter() - t0


def mixed_vs_fp64(p3, S_f, S_m, b, x_exact, graph):
    """Time to a 1e-10 true residual on the 200^3 workload's own b, FP32
    storage against FP64, at each replacement period of a common grid (and
    the automated criterion), with the paper's shadow residual r_0 and with a
    random fixed shadow vector (an option outside the paper; b = A 1/sqrt(N)
    vanishes off the boundary layer, since the operator's interior rows sum
    to zero, so r_0 = b is a very particular shadow vector).  Each
    configuration runs without restarts; a run that stops in a breakdown is
    repeated with up to 5 restarts from the current iterate (another option
    outside the paper), reported separately."""
    import numpy as np
    import torch
    periods = (10, 15, 25, 50, 100, "auto")
    rh = torch.from_numpy(np.random.default_rng(56).standard_normal(p3.n)).to(b.device)
    for S in (S_f, S_m):                                   # graph capture per shape
        for P in periods:
            rr = dict(rr_auto=True) if P == "auto" else dict(rr_period=P)
            S.solve(b, tol=1e-10, maxit=100, use_graph=graph, **rr)
    out = {"workload": "convdiff3d 200^3, c=(10,5,1), Jacobi, b = A 1/sqrt(N), tol 1e-10 "
                       "true residual, maxit 20000"}
    for shadow_name, shadow in (("shadow_r0", None), ("shadow_random", rh)):
        rows = {}
        x_ref = None
        for P in periods:
            rr = dict(rr_auto=True) if P == "auto" else dict(rr_period=P)
            row = {}
            for prec, S in (("fp64", S_f), ("mixed", S_m)):
                ent = {}
                for restarts in (0, 5):
                    x, st, sec = solve_timed(S, b, tol=1e-10, maxit=20000, use_graph=graph,
                                             restarts=restarts, rhat=shadow, **rr)
                    key = "no_restart" if restarts == 0 else "with_restarts"
                    ent[key] = {
                        "seconds": sec, "status": st["status_name"],
                        "iterations": st["iterations"], "replacements": st["replacements"],
                        "restarts": st["restarts"], "rel_res_true": st["rel_res_true"],
                        "rel_err_vs_exact": float(torch.linalg.norm(x - x_exact) /
                                                  torch.linalg.norm(x_exact))}
                    if prec == "fp64" and x_ref is None and st["status_name"] == "CONVERGED":
                        x_ref = x.clone()
                    if prec == "mixed" and x_ref is not None:
                        ent[key]["rel_diff_vs_fp64"] = float(torch.linalg.norm(x - x_ref) /
                                                             torch.linalg.norm(x_ref))
                    if st["status_name"] != "BREAKDOWN_RHO":
                        break
                row[prec] = ent
            f0, m0 = row["fp64"]["no_restart"], row["mixed"]["no_restart"]
            ok = f0["status"] == "CONVERGED" and m0["status"] == "CONVERGED"
            row["speedup_no_restart"] = f0["seconds"] / m0["seconds"] if ok else None
            fr = row["fp64"].get("with_restarts", f0)
            mr = row["mixed"].get("with_restarts", m0)
            ok = fr["status"] == "CONVERGED" and mr["status"] == "CONVERGED"
            row["speedup_allowing_restarts"] = fr["seconds"] / mr["seconds"] if ok else None
            rows[f"P_{P}"] = row
            log(f"mixed vs fp64 {shadow_name} P={P}: {json.dumps(row)}")

        def best(prec, allow):
            vals = []
            for P in periods:
                ent = rows[f"P_{P}"][prec]
                e = ent.get("with_restarts", ent["no_restart"]) if allow else ent["no_restart"]
                if e["status"] == "CONVERGED":
                    vals.append((e["seconds"], P))
            return min(vals) if vals else None

        res = {"by_period": rows}
        for allow, key in ((False, "no_restart"), (True, "allowing_restarts")):
            bf, bm = best("fp64", allow), best("mixed", allow)
            res[f"best_{key}"] = {"fp64": bf, "mixed": bm,
                                  "speedup": (bf[0] / bm[0]) if (bf and bm) else None}
        eq = [rows[f"P_{P}"]["speedup_no_restart"] for P in periods]
        eq = [v for v in eq if v is not None]
        res["equal_P_speedups_no_restart"] = {
            "converged_in_both": len(eq), "of": len(periods),
            "median": float(np.median(eq)) if eq else None,
            "min": min(eq) if eq else None, "max": max(eq) if eq else None}
        out[shadow_name] = res
    return out


def accuracy_vs_time(S, b, runs):
    """Relative true residual against time for several methods: solves are
    bitwise repeatable, so stopping the same run after k iterations samples
    its trajectory exactly; the time is the solve's own (HIP events)."""
    out = {}
    for name, kw, ks in runs:
        pts = []
        for k in ks:
            _, st = S.solve(b, tol=0.0, maxit=k, **kw)
            pts.append([st["iterations"], st["elapsed_ms"] / 1e3, st["rel_res_true"]])
            if st["iterations"] < k:            # stopped (breakdown): the trajectory ends
                break
        best = min(pts, key=lambda q: q[2])
        desc = {key: ("random fixed shadow vector, rng(56)" if key == "rhat" else val)
                for key, val in kw.items()}
        out[name] = {"points_iterations_seconds_relres": pts,
                     "best": {"iterations": best[0], "seconds": best[1], "rel_res_true": best[2]},
                     "replacement": desc}
        log(f"accuracy {name}: best {best}")
    return out


def paper_problems(dev):
    import torch
    from paper_1809_01948_amd.solver import Solver
    from workloads import tp2_unsymmetric, tp3_helmholtz
    import numpy as np
    res = {}
    p = tp2_unsymmetric(1000)
    S = Solver.from_problem(p, form="stencil", precond="none")
    b = torch.from_numpy(p.b).to(dev)
    rh = torch.from_numpy(np.random.default_rng(56).standard_normal(p.n)).to(dev)
    ks = list(range(100, 1501, 100))
    res["TP2_1000x1000"] = accuracy_vs_time(S, b, [
        ("classic", dict(method="classic"), ks),
        ("p-BiCGStab", dict(), ks),
        ("p-BiCGStab_rr100", dict(rr_period=100), ks),
        ("p-BiCGStab_auto", dict(rr_auto=True), ks),
        # options outside the paper: the bound's square-root estimate in the
        # products reading, with a random fixed shadow vector
        ("p-BiCGStab_auto_products_estimate_random_shadow",
         dict(rr_auto="products-estimate", rhat=rh), ks),
        # another option outside the paper: every replacement also refreshes
        # n = M^-1 z and v = A n from the replaced z (with the paper's r_0)
        ("p-BiCGStab_rr100_nv", dict(rr_period=100, rr_nv=True), ks),
        ("p-BiCGStab_auto_estimate_nv", dict(rr_auto="estimate", rr_nv=True), ks)])
    S.close()
    p = tp3_helmholtz(500)
    S = Solver.from_problem(p, form="stencil", precond="none")
    b = torch.from_numpy(p.b).to(dev)
    ks = list(range(500, 8001, 500))
    res["TP3_500x500"] = accuracy_vs_time(S, b, [
        ("classic", dict(method="classic"), ks),
        ("p-BiCGStab", dict(), ks),
        ("p-BiCGStab_rr200", dict(rr_period=200), ks),
        ("p-BiCGStab_rr200_nv", dict(rr_period=200, rr_nv=True), ks)])
    S.close()
    res["note"] = ("the paper's TP2/TP3 (Table tab:specs, ||A||_2 = 1, b = A 1/sqrt(N), no "
                   "preconditioner, FP64); paper (120 ranks): TP2 classic ~1e-13 at ~600 "
                   "iterations, p-BiCGStab ~1e-10 then growing, with replacement every 100 "
                   "~1e-13; TP3 classic ~1e-8 at ~4000, p-BiCGStab 8e-5 at ~4000, with "
                   "replacement every 200 ~1e-8 at ~4000")
    return res


def c1_latency(dev):
    """32^2 convection-diffusion (N = 1024): launch-bound; iterations per
    second of full solves to 1e-10, classic (Algorithm 1, 7 launches per
    iteration), pipelined (Algorithm 2 from HIP graphs) and pipelined as one
    kernel in one workgroup (no launches or host polls inside the solve);
    without replacement, every 50 iterations and the automated strategy.
    Also the 45^2 grid (2025 rows), graphs against one workgroup."""
    import torch
    from paper_1809_01948_amd.solver import Solver
    from workloads import convdiff2d_c1
    p = convdiff2d_c1(32)
    b = torch.from_numpy(p.b).to(dev)
    out = {}
    for form in ("csr", "stencil"):
        S = Solver.from_problem(p, form=form, precond="none")
        for name, kw in (("classic", dict(method="classic")),
                         ("pipelined_graph", dict(use_graph=True)),
                         ("pipelined_rr50_graph", dict(use_graph=True, rr_period=50)),
                         ("pipelined_auto_graph", dict(use_graph=True, rr_auto=True)),
                         ("pipelined_single_kernel", dict(single_kernel=True)),
                         ("pipelined_rr50_single_kernel", dict(single_kernel=True,
                                                               rr_period=50)),
                         ("pipelined_auto_single_kernel", dict(single_kernel=True,
                                                               rr_auto=True))):
            S.solve(b, tol=1e-10, maxit=2000, **kw)
            ts, its = [], 0
            for _ in range(20):
                _, st, sec = solve_timed(S, b, tol=1e-10, maxit=2000, **kw)
                ts.append(sec)
                its = st["iterations"]
            ts.sort()
            med = ts[len(ts) // 2]
            out[f"{form}_{name}"] = {"iterations": its, "median_seconds": med,
                                     "iter_per_s": its / med, "status": st["status_name"],
                                     "device_ms": st["elapsed_ms"],
                                     "single_kernel": st["single_kernel"]}
        S.close()
    # the 45^2 grid (2025 rows): one workgroup with four rows per thread
    p45 = convdiff2d_c1(45)
    b45 = torch.from_numpy(p45.b).to(dev)
    for form in ("csr", "stencil"):
        S = Solver.from_problem(p45, form=form, precond="none")
        for name, kw in (("pipelined_graph", dict(use_graph=True)),
                         ("pipelined_single_kernel", dict(single_kernel=True))):
            S.solve(b45, tol=1e-10, maxit=3000, **kw)
            ts = []
            for _ in range(20):
                _, st, sec = solve_timed(S, b45, tol=1e-10, maxit=3000, **kw)
                ts.append(sec)
            ts.sort()
            med = ts[len(ts) // 2]
            out[f"n2025_{form}_{name}"] = {"iterations": st["iterations"], "median_seconds": med,
                                           "iter_per_s": st["iterations"] / med,
                                           "status": st["status_name"],
                                           "device_ms": st["elapsed_ms"],
                                           "single_kernel": st["single_kernel"]}
        S.close()
    log(f"c1 latency: {json.dumps(out)}")
    return out


def c2_cache_resident(dev, graph):
    """1000^2 Poisson (FP64 stencil, Jacobi, replacement every 50): its
    ~110 MB working set fits the 256 MB Infinity Cache, so its bandwidth is
    effective bandwidth, not HBM."""
    import torch
    from paper_1809_01948_amd.solver import Solver
    from workloads import poisson2d_c2
    p = poisson2d_c2(1000, with_csr=False)
    S = Solver.from_problem(p, form="stencil", precision="fp64", precond="jacobi")
    b = torch.from_numpy(p.b).to(dev)
    opts = dict(tol=1e-10, maxit=1000, rr_period=50, use_graph=graph)
    ips, ms, _ = timed_steps(S, b, opts, 5, 1, "c2")
    ms_b = S.time_kernel("phaseB", reps=100)
    out = {"workload": "poisson2d 1000x1000, FP64 stencil, Jacobi, replacement every 50, "
                       "1000 iterations per solve (cache-resident)",
           "iter_per_s": ips, "effective_gbps": 28 * 8 * p.n * ips / 1e9,
           "phaseB_ms": ms_b, "phaseB_effective_gbps": 15 * 8 * p.n / (ms_b * 1e-3) / 1e9}
    x, st, sec = solve_timed(S, b, tol=1e-10, maxit=20000, rr_auto=True, use_graph=graph,
                             restarts=5)
    out["to_1e-10_automated"] = {"seconds": sec, "status": st["status_name"],
                                 "iterations": st["iterations"],
                                 "replacements": st["replacements"], "restarts": st["restarts"]}
    x, st, sec = solve_timed(S, b, tol=1e-10, maxit=20000, method="classic")
    out["to_1e-10_classic"] = {"seconds": sec, "status": st["status_name"],
                               "iterations": st["iterations"]}
    S.close()
    log(f"c2: {json.dumps(out)}")
    return out


def other_kernels(which, dev):
    """Kernel times of the sliced-ELL (2e6 rows x 27) or DIA5 (2048^2)
    iteration in FP64 and with FP32 storage, with algorithmic bytes per row;
    on the DIA5 operator also the two gradient passes."""
    import torch
    from paper_1809_01948_amd.solver import Solver
    from workloads import inverse_problem_c5, random_banded_c4
    if which == "random2m":
        p, form, slots = random_banded_c4(), "csr", 27
    else:
        p, form, slots = inverse_problem_c5(), "dia5", 5
    b = torch.from_numpy(p.b).to(dev)
    out = {"workload": which, "n": p.n, "bytes_per_row": {}, "ms": {}, "GBps": {}, "frac": {}}
    for prec, bv in (("fp64", 8), ("mixed", 4)):
        S = Solver.from_problem(p, form=form, precision=prec, precond="jacobi")
        S.solve(b, tol=1e-10, maxit=50, rr_period=50)       # realistic vector contents
        if form == "csr":
            # separate products; Jacobi with a dinv vector, applied by the phase
            # kernels, which also write the products' input M^-1 z (M^-1 w); values
            # in the storage precision plus int32 columns
            byts = {"phaseA": 15 * bv, "phaseB": 15 * bv + 16,
                    "spmv1": 2 * bv + slots * (bv + 4)}
            it_bytes = byts["phaseA"] + byts["phaseB"] + 2 * byts["spmv1"]
        else:
            # products fused into the phase kernels; five coefficient arrays
            byts = {"phaseA": 14 * bv + slots * bv, "phaseB": 14 * bv + 16 + slots * bv}
            it_bytes = byts["phaseA"] + byts["phaseB"]
        # the copy kernel calibrates the HBM byte counters of the product
        out["ms"][f"{prec}_copy"] = S.time_kernel("copy", reps=KERNELS_ONLY_REPS)
        for k, bpr in byts.items():
            ms = S.time_kernel(k, reps=KERNELS_ONLY_REPS)
            out["bytes_per_row"][f"{prec}_{k}"] = bpr
            out["ms"][f"{prec}_{k}"] = ms
            out["GBps"][f"{prec}_{k}"] = bpr * p.n / (ms * 1e-3) / 1e9
            out["frac"][f"{prec}_{k}"] = out["GBps"][f"{prec}_{k}"] / HBM_PEAK_GBS
        ms_it = S.time_kernel("iteration", reps=KERNELS_ONLY_REPS)
        out["ms"][f"{prec}_iteration"] = ms_it
        out["bytes_per_row"][f"{prec}_iteration"] = it_bytes
        out["frac"][f"{prec}_iteration"] = it_bytes * p.n / (ms_it * 1e-3) / 1e9 / HBM_PEAK_GBS
        if form == "dia5" and prec == "fp64":
            lam = torch.randn(p.n, dtype=torch.float64, device=dev)
            x = torch.randn(p.n, dtype=torch.float64, device=dev)
            for name, fn in (("grad_values", lambda: S.grad_values(lam, x)),
                             ("kappa_grad", lambda: S.kappa_grad(lam, x))):
                fn()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(KERNELS_ONLY_REPS):
                    fn()
                torch.cuda.synchronize()
                out["ms"][name] = (time.perf_counter() - t0) / KERNELS_ONLY_REPS * 1e3
        S.close()
    return out


def c5_full_size(dev):
    """The 2048^2 coefficient-field problem at full size: forward solve for
    the target field, forward solve for the current field, adjoint solve with
    g = 2 (u - u_target); FP64, tolerance 1e-6 (1e-7 for the classic runs
    with a random shadow vector, the accuracy the gradient check needs).
    Classic BiCGStab and p-BiCGStab with automated replacement, each with the
    paper's shadow residual r_0 and with a random fixed shadow vector (an
    option outside the paper: with b = h^2 1 the operator's vanishing
    interior column sums drive (r_0, r_i) to zero), and p-BiCGStab with
    periodic replacement that also refreshes n and v (rr_nv, another option
    outside the paper).  Reported, not asserted: with the six quantities of
    eq:rr alone p-BiCGStab breaks down on this operator at full size."""
    import torch
    from paper_1809_01948_amd.solver import Solver
    from workloads import dia5_from_kappa, inverse_problem_c5
    p = inverse_problem_c5(2048)
    n = 2048
    h = 1.0 / (n + 1)
    b = torch.from_numpy(p.b).to(dev)
    import numpy as np
    rh = torch.from_numpy(np.random.default_rng(56).standard_normal(p.n)).to(dev)
    S_t = Solver.from_stencil("dia5", (n, n), dia5_from_kappa(p.extra["kappa_target"], h))
    S = Solver.from_problem(p, form="dia5", precond="jacobi")
    out = {}
    for name, kw in (("classic_r0", dict(method="classic", tol=1e-6)),
                     ("pipelined_auto_r0", dict(rr_auto=True, tol=1e-6)),
                     ("classic_random_shadow", dict(method="classic", tol=1e-7, rhat=rh)),
                     ("pipelined_auto_random_shadow", dict(rr_auto=True, tol=1e-6, rhat=rh)),
                     ("pipelined_rr50_nv_r0", dict(rr_period=50, rr_nv=True, tol=1e-6)),
                     ("pipelined_rr200_nv_random_shadow",
                      dict(rr_period=200, rr_nv=True, tol=1e-7, rhat=rh))):
        ut, st_t, s_t = solve_timed(S_t, b, maxit=20000, **kw)
        u, st_f, s_f = solve_timed(S, b, maxit=20000, **kw)
        g = 2.0 * (u - ut)
        lam, st_a, s_a = solve_timed(S, g, maxit=20000, transpose=True, **kw)
        out[name] = {k: {"status": st["status_name"], "iterations": st["iterations"],
                         "replacements": st["replacements"],
                         "rel_res_true": st["rel_res_true"], "seconds": sec}
                     for k, st, sec in (("target_forward", st_t, s_t), ("forward", st_f, s_f),
                                        ("adjoint", st_a, s_a))}
        log(f"c5 {name}: {json.dumps(out[name])}")
    S.close()
    S_t.close()
    return out


def kernels_only(args, dev):
    """The iteration kernels of one workload, HIP-event timed (the program
    the rocprofv3 runs profile).  One JSON line."""
    import torch
    from paper_1809_01948_amd.solver import Solver
    from workloads import convdiff3d_c3, poisson2d_c2
    if args.kernels_workload in ("random2m", "kappa2048"):
        print(json.dumps(other_kernels(args.kernels_workload, dev)), flush=True)
        return
    prec = args.kernels_precision
    p = convdiff3d_c3(200) if args.kernels_workload == "convdiff200" else \
        poisson2d_c2(1000, with_csr=False)
    S = Solver.from_problem(p, form="stencil", precision=prec, precond="jacobi")
    S.solve(torch.from_numpy(p.b).to(dev), tol=1e-10, maxit=50, rr_period=RR_PERIOD)
    # (with the products fused into the phase kernels, spmv1/spmv2 time the
    # one-block GLRED finals)
    names = ("phaseA", "spmv1", "phaseB", "spmv2", "copy")
    res = {k: S.time_kernel(k, reps=KERNELS_ONLY_REPS) for k in names}
    res["iteration"] = S.time_kernel("iteration", reps=KERNELS_ONLY_REPS)
    print(json.dumps({"workload": args.kernels_workload, "precision": prec, "ms": res}),
          flush=True)
    S.close()


def main():
    args = parse()
    if args.summarize_pmc:
        summarize_pmc(args.summarize_pmc[0], args.summarize_pmc[1], args.kernels_workload,
                      args.kernels_precision)
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(--gpus must be 1)", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1809_01948_amd.solver import Solver
    from workloads import convdiff3d_c3

    dev = torch.device("cuda:0")
    if args.kernels_only:
        kernels_only(args, dev)
        return
    if args.c1_only:
        print(json.dumps({"c1_latency": c1_latency(dev)}), flush=True)
        return
    graph = bool(args.graph)
    log("generating the 200^3 convection-diffusion workload")
    p3 = convdiff3d_c3(200)
    n = p3.n
    b = torch.from_numpy(p3.b).to(dev)
    xe = torch.from_numpy(p3.x_exact).to(dev)
    S_f = Solver.from_problem(p3, form="stencil", precision="fp64", precond="jacobi")
    opts = dict(tol=1e-10, maxit=ITERS_PER_STEP, rr_period=RR_PERIOD, use_graph=graph)
    value, ms_per_step, stats = timed_steps(S_f, b, opts, args.steps, args.warmup, "fp64")
    eff_gbs = C3_FP64_BYTES_ROW * n * value / 1e9

    # roofline of the dominant kernel: FP64 phase B (15 streams per row)
    phaseB_bytes = PHASEB_FP64_BYTES_ROW * n
    ms = {k: S_f.time_kernel(k, reps=50) for k in ("phaseA", "spmv1", "phaseB", "copy")}
    ms["iteration"] = S_f.time_kernel("iteration", reps=20)
    achieved = phaseB_bytes / (ms["phaseB"] * 1e-3) / 1e9
    kernels = {
        "fp64_phaseA": {"ms": ms["phaseA"], "GBps": 13 * 8 * n / (ms["phaseA"] * 1e-3) / 1e9},
        "fp64_phaseB": {"ms": ms["phaseB"], "GBps": achieved},
        "fp64_spmv": {"ms": ms["spmv1"], "GBps": 2 * 8 * n / (ms["spmv1"] * 1e-3) / 1e9},
        "copy": {"ms": ms["copy"], "GBps": 2 * 8 * n / (ms["copy"] * 1e-3) / 1e9},
        "fp64_iteration_kernels_only_ms": ms["iteration"],
    }

    S_m = Solver.from_problem(p3, form="stencil", precision="mixed", precond="jacobi")
    v32, ms32, _ = timed_steps(S_m, b, opts, args.steps, args.warmup, "fp32-storage")
    m32 = {k: S_m.time_kernel(k, reps=50) for k in ("phaseA", "phaseB")}
    m32["iteration"] = S_m.time_kernel("iteration", reps=20)
    kernels["fp32_phaseA"] = {"ms": m32["phaseA"],
                              "GBps": 13 * 4 * n / (m32["phaseA"] * 1e-3) / 1e9}
    kernels["fp32_phaseB"] = {"ms": m32["phaseB"],
                              "GBps": PHASEB_FP32_BYTES_ROW * n / (m32["phaseB"] * 1e-3) / 1e9}
    kernels["fp32_iteration_kernels_only_ms"] = m32["iteration"]
    log(f"kernels: {json.dumps(kernels)}")

    out = {
        "metric": "p-BiCGStab iter/s + HBM GB/s; time to 1e-10 true residual, mixed vs FP64",
        "value": value,
        "unit": "iter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "convdiff3d 200^3 7-point stencil, convection (10,5,1), N=8e6, "
                               "Jacobi, FP64, residual replacement every 50, "
                               f"{ITERS_PER_STEP} iterations per step",
                   "n": n, "form": "stencil", "precision": "fp64",
                   "iterations_per_solve": stats[-1]["iterations"],
                   "replacements_per_solve": stats[-1]["replacements"],
                   "status": stats[-1]["status_name"], "graph": graph},
        "hbm_gbps_effective": eff_gbs,
        "hbm_frac_effective": eff_gbs / HBM_PEAK_GBS,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": stored_traffic("convdiff200", "fp64"),
                     "kernel": "phaseB (FP64, 200^3)",
                     "algorithmic_bytes_per_launch": phaseB_bytes,
                     "avg_launch_ms": ms["phaseB"]},
        "value_fp32_storage": {
            "iter_per_s": v32, "ms_per_step": ms32,
            "hbm_gbps_effective": C3_FP32_BYTES_ROW * n * v32 / 1e9,
            "hbm_frac_effective": C3_FP32_BYTES_ROW * n * v32 / 1e9 / HBM_PEAK_GBS,
            "roofline_phaseB": {"achieved": kernels["fp32_phaseB"]["GBps"],
                                "frac": kernels["fp32_phaseB"]["GBps"] / HBM_PEAK_GBS,
                                "traffic": stored_traffic("convdiff200", "mixed"),
                                "algorithmic_bytes_per_launch": PHASEB_FP32_BYTES_ROW * n,
                                "avg_launch_ms": m32["phaseB"]}},
        "kernels": kernels,
    }

    if not args.skip_mixed:
        log("200^3: FP64 vs FP32 storage to 1e-10 at equal replacement periods")
        out["mixed_vs_fp64"] = mixed_vs_fp64(p3, S_f, S_m, b, xe, graph)
    S_f.close()
    S_m.close()

    if not args.skip_extras:
        log("the paper's TP2 and TP3: accuracy against time")
        out["paper_accuracy_vs_time"] = paper_problems(dev)
        out["extras"] = {"c2_cache_resident": c2_cache_resident(dev, graph),
                         "c1_latency": c1_latency(dev)}
        log("2e6 x 27 random matrix and 2048^2 DIA5 kernels")
        out["extras"]["c4_random2m_kernels"] = other_kernels("random2m", dev)
        out["extras"]["c5_kappa2048_kernels"] = other_kernels("kappa2048", dev)
        out["extras"]["c5_full_size"] = c5_full_size(dev)

    if not args.skip_cpu:
        log(f"CPU oracle baseline ({args.cpu_iters} iterations of the 200^3 solve)")
        out["cpu_baseline"] = cpu_baseline(args.cpu_iters)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
