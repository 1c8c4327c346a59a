"""Benchmark: MG-preconditioned FCG solves of the SIPG operator on one MI355X.

Workload "hp" (default, the largest configuration whose timed solves fit about a minute):
-div(k grad u) = g on [-1, 1]^3, 32^3 cells, degree p uniform in 2..7 per cell (seed 0),
cells cut by r = 0.5 refined 2:1, k = 1 inside r = 0.5 and 5 outside, manufactured
u = r^2 / k + c_k with Dirichlet data (8,649,651 DOF).  One step = one FP64 solve from u = 0
to a relative residual of 1e-10 (flexible CG, V-cycle with point-Jacobi Chebyshev smoothing,
exact coarse solve): every row of the linear hot path runs inside it.  The same line carries
the mixed-precision solves (FP32 V-cycle inside FP64 FCG), the fine-level apply rate against
the HBM and FP64 roofs, the compactified cubed-sphere shell (p = 5, 1,244,160 DOF, block-Jacobi
smoothing with the fused apply + block step) as a sub-measurement, the committed out-of-cache
apply sweep and the oracle's CPU rate.

Other workloads (``--workload``): "shell" alone, "newton" (the 13-macro cube + compactified
exterior refined around three seeded punctures, p = 6, 12,739,363 DOF, Newton-Krylov to
|R| <= 1e-10 |R_0|), "serving" (the 512-request stream), "sweep" (the out-of-cache apply
rates of the uniform box, written to profiles/), "amr" (the hp-adaptive loop) and "schwarz"
(MG-FCG with the additive Schwarz smoother against point-Jacobi Chebyshev on a uniform box).
Printed: one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
                    [--workload hp|shell|newton|serving|sweep|amr|schwarz]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "DG operator DOF-applies/s (FP64 vs mixed); solves/s + p99 latency at 1e-10 residual"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6  # MI355X FP64 vector
# HBM traffic per launch from rocprofv3 FETCH_SIZE / WRITE_SIZE counters, written by
# --summarize-traffic; valid only while the kernel sources hash to the recorded value
TRAFFIC_FILE = os.path.join("profiles", "solve_hp_hbm_traffic.txt")
# the operator apply of a level with element-centric groups: one fast_kernel launch per degree
# (descending), and for the cells it does not cover (variable k, 2:1 faces) the face traces, the
# mortar kernel and the element kernel per (n, q) bucket
APPLY_EC = ("fast_kernel<double, n, mixed, false> per degree + trace_kernel<double> + mortar_kernel<double> + "
            "apply_kernel<double, n, q, false> per bucket")
SMOOTH_EC = ("fast_kernel<double, n, mixed, true> per degree + trace_kernel<double> + mortar_kernel<double> + "
             "apply_kernel<double, n, q, true> per bucket (fused point-Jacobi Chebyshev step)")
KERNEL_SOURCES = [os.path.join("paper_1907_01572_amd", "csrc", f)
                  for f in ("apply.hip", "fastapply.hip", "apply_common.hpp", "kernels.hip", "blocks.hpp", "device.hpp",
                            "host.hpp")]
COPY_BYTES = 1 << 30  # calibration copy: 1 GiB read, 1 GiB written
# kernel timing inside the timed solves: HIP events around every 8th launch of each kernel
# kind and level (two event records per sampled launch)
TIMING_EVERY = 8
# library timing kinds: the apply, the block-Jacobi step and the two fused in one kernel
TIMED_KINDS = ("apply", "block", "smooth")


def kernel_sources_sha256():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(kernel, alg_bytes):
    """HBM bytes per launch of ``kernel`` from the committed counter summary, or None when
    there is none or the kernel sources changed since the counters were taken."""
    path = os.path.join(ROOT, TRAFFIC_FILE)
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as fh:
        for line in fh:
            if ": " in line and not line.startswith("#"):
                k, v = line.rstrip("\n").split(": ", 1)
                vals[k.strip()] = v.strip()
    if vals.get("sources_sha256") != kernel_sources_sha256():
        return None
    v = vals.get("bytes_per_launch[%s]" % kernel)
    return None if v is None else float(v)


def composite_members(name):
    """Which of a composite apply / step's member kernels a kernel name is (None if it is not one):
    the element-centric groups, the face traces, the mortar kernel and the element kernel."""
    short = name.split("(hpdg::")[0].replace("void hpdg::(anonymous namespace)::", "")
    if not short.endswith(">") or "<double" not in short:
        return None
    if short.startswith("mortar_kernel") and short.endswith("true>"):
        return None  # the estimator's form
    if short.startswith("trace_kernel") or short.startswith("mortar_kernel"):
        return "both"
    if short.startswith("fast_kernel") or short.startswith("apply_kernel"):
        return "step" if short.endswith("true>") else "apply"
    return None


def summarize_trace(stats_csv, out_md, command, trace_csv=None):
    """Top kernels of a rocprofv3 kernel-stats table as markdown (name, calls, total, mean), and
    from the per-dispatch trace (optional) the mean duration of each kernel's fine-level
    dispatches (those with its largest grid)."""
    import csv

    with open(stats_csv) as fh:
        rows = list(csv.DictReader(fh))
    fine = {}
    if trace_csv:
        per = {}
        with open(trace_csv) as fh:
            for r in csv.DictReader(fh):
                g = (int(r["Grid_Size"]) if r.get("Grid_Size") else
                     int(r["Grid_Size_X"]) * int(r["Grid_Size_Y"]) * int(r["Grid_Size_Z"]))
                per.setdefault(r["Kernel_Name"], []).append((g, int(r["End_Timestamp"]) - int(r["Start_Timestamp"])))
        for name, v in per.items():
            g = max(x[0] for x in v)
            d = [x[1] for x in v if x[0] == g]
            fine[name] = (g, len(d), float(np.mean(d)))
    total = sum(float(r["TotalDurationNs"]) for r in rows)
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    lines = ["# rocprofv3 kernel trace", "", "Command (from the repository root, on one MI355X):", "",
             "    " + command, "", "Total kernel time: %.1f ms." % (total / 1e6), "",
             "| kernel | calls | total ms | share | mean us | min us | max us |", "|---|---|---|---|---|---|---|"]
    for r in rows[:20]:
        name = r["Name"].split("(hpdg::")[0].replace("void hpdg::(anonymous namespace)::", "").replace("|", "/")
        lines.append("| `%s` | %s | %.2f | %.1f%% | %.1f | %.1f | %.1f |" % (
            name[:90], r["Calls"], float(r["TotalDurationNs"]) / 1e6, 100 * float(r["TotalDurationNs"]) / total,
            float(r["AverageNs"]) / 1e3, float(r["MinNs"]) / 1e3, float(r["MaxNs"]) / 1e3))
    if fine:
        lines += ["", "Fine-level dispatches (each kernel's largest grid, from the per-dispatch trace):", "",
                  "| kernel | grid (threads) | dispatches | mean us |", "|---|---|---|---|"]
        top = [r["Name"] for r in rows[:24]]
        for nm in top:
            if nm in fine:
                g, c, m = fine[nm]
                name = nm.split("(hpdg::")[0].replace("void hpdg::(anonymous namespace)::", "").replace("|", "/")
                lines.append("| `%s` | %d | %d | %.1f |" % (name[:90], g, c, m / 1e3))
        # composites: one fine-level apply / fused smoother step is one dispatch of each member;
        # the element kernel's buckets run on a side stream beside the element-centric groups, so
        # the step's span is the main stream's chain (face traces, mortar kernel, groups)
        for kind, label in (("apply", APPLY_EC), ("step", SMOOTH_EC)):
            mem = [nm for nm in fine if composite_members(nm) in (kind, "both")]
            if any(composite_members(nm) == kind for nm in mem):
                tot = sum(fine[nm][2] for nm in mem)
                chain = sum(fine[nm][2] for nm in mem if "apply_kernel" not in nm)
                lines += ["", "Fine-level %s (%d kernels): main-stream chain (face traces + mortar kernel + "
                          "element-centric groups) %.1f us; sum over all members %.1f us (the element kernel's "
                          "buckets overlap the groups on the side stream)  [%s]"
                          % ("apply" if kind == "apply" else "fused step", len(mem), chain / 1e3, tot / 1e3, label)]
    with open(out_md, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def summarize_traffic(fetch_csv, write_csv, cal_fetch_csv, cal_write_csv, out, kernels=None):
    """Mean FETCH_SIZE + WRITE_SIZE per dispatch of each kernel (rocprofv3 --pmc CSVs, KiB),
    each scaled by the same counter on a 1 GiB device copy, written as a text summary; for the
    per-bucket FP64 apply (trace kernel + one apply_kernel launch per degree bucket) also the sum
    over its kernels, the traffic of one finest-level apply."""
    import csv

    def per_kernel(path, fine_only=False):
        # fine_only: only the dispatches with the kernel's largest grid (the finest level)
        rows = {}
        with open(path) as fh:
            for r in csv.DictReader(fh):
                rows.setdefault(r["Kernel_Name"], []).append((int(r["Grid_Size"]), float(r["Counter_Value"]) * 1024.0))
        acc = {}
        for name, v in rows.items():
            g = max(x[0] for x in v)
            acc[name] = [x[1] for x in v if x[0] == g or not fine_only]
        return acc

    def copy_value(path):
        acc = per_kernel(path)
        return max(max(v) for k, v in acc.items() if "copyBuffer" in k)

    sf = COPY_BYTES / copy_value(cal_fetch_csv)
    sw = COPY_BYTES / copy_value(cal_write_csv)
    fa, wa = per_kernel(fetch_csv, True), per_kernel(write_csv, True)
    if kernels is None:
        kernels = sorted(k for k in fa if "hpdg" in k)
    lines = ["# HBM traffic per fine-level launch (the kernel's dispatches with the largest grid):",
             "# rocprofv3 FETCH_SIZE and WRITE_SIZE (KiB per dispatch), scaled by the counters read",
             "# on a 1 GiB device-to-device copy",
             "fetch_scale: %.6f" % sf, "write_scale: %.6f" % sw,
             "sources_sha256: %s" % kernel_sources_sha256()]
    for k in kernels:
        full = [n for n in fa if k in n]
        if not full:
            continue
        f = np.mean(fa[full[0]]) * sf
        w = np.mean(wa[full[0]]) * sw if full[0] in wa else float("nan")
        short = k.split("(hpdg::")[0].replace("void hpdg::(anonymous namespace)::", "")
        lines += ["dispatches[%s]: %d" % (short, len(fa[full[0]])),
                  "fetch_bytes_per_launch[%s]: %.0f" % (short, f),
                  "write_bytes_per_launch[%s]: %.0f" % (short, w),
                  "bytes_per_launch[%s]: %.0f" % (short, f + w)]
    # one finest-level FP64 apply / fused step: one fine-level dispatch of each member kernel
    for kind, label in (("apply", APPLY_EC), ("step", SMOOTH_EC)):
        parts = [k for k in fa if composite_members(k) in (kind, "both")]
        if any(composite_members(k) == kind for k in parts):
            tot = sum(np.mean(fa[k]) * sf + (np.mean(wa[k]) * sw if k in wa else 0.0) for k in parts)
            lines.append("bytes_per_launch[%s]: %.0f" % (label, tot))
    with open(out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def make_workload(args, meshgen, hp):
    """Mesh, problem and solver settings of a workload."""
    w = dict(name=args.workload)
    if args.workload == "shell":
        w["mesh"] = meshgen.cubed_sphere_shell(level=args.level, p=args.p)
        w["prob"] = meshgen.problem_config2()
        # four levels: the coarsest (10,368 DOF, 48 cells at p = 5) is solved exactly
        w["upload"] = dict(build_f32=True, max_levels=4)
        w["smoother"] = dict(n_cheb=args.n_cheb or 26, smoother=args.smoother or "block",
                             Lambda=args.Lambda or 600.0)
        w["desc"] = ("cubed-sphere shell r=1..1e9 (compactified), 6x8^3 cells + 2:1 inner layer, p=%d, "
                     "Poisson, MG-FCG to 1e-10" % args.p)
    elif args.workload == "hp":
        w["mesh"] = meshgen.hp_sphere_cube()
        w["prob"] = meshgen.problem_config3()
        w["upload"] = dict(coef=hp.coef_from_problem(w["prob"]), build_f32=True)
        # Chebyshev degree 6 (41 FCG iterations) is the fastest of a sweep over 3..12 and Lambda 10..30
        w["smoother"] = dict(n_cheb=args.n_cheb or 6, smoother=args.smoother or "point", Lambda=args.Lambda or 20.0)
        w["desc"] = ("[-1,1]^3, 32^3 cells, p~U{2..7} (seed 0), cells cut by r=0.5 refined 2:1, k=1|5 across "
                     "r=0.5, -div(k grad u)=-6, MG-FCG to 1e-10")
    else:
        nl = meshgen.puncture_problem()
        w["nl"] = nl
        w["mesh"] = meshgen.puncture_mesh(punctures=nl["params"][1:].reshape(-1, 5)[:, :3])
        w["prob"] = None
        w["upload"] = dict(mass_term=True, build_f32=True)
        w["smoother"] = dict(n_cheb=args.n_cheb or 16, smoother=args.smoother or "point", Lambda=args.Lambda or 400.0)
        w["desc"] = ("cube [-10,10]^3 + cube-to-sphere + compactified shell to 1e11 (13 macros), refined 5x "
                     "around 3 seeded punctures, p=6, -lap u = beta (1 + alpha u)^-7, Newton-Krylov to 1e-10")
    return w


def run_solves(args, W, hp, ctx, steps, warmup, kinds_names, cpu=True):
    """Upload a workload, set up its smoother, time ``steps`` FP64 solves and as many mixed
    (and mixed-bf16 with block smoothing) solves; returns the measurement dictionary."""
    import torch

    mesh, prob = W["mesh"], W["prob"]
    newton = "nl" in W
    dev = torch.device("cuda:0")
    t0 = time.time()
    up = dict(W["upload"])
    if args.max_levels >= 0:
        up["max_levels"] = args.max_levels
    if args.ec_mode:
        up["ec_mode"] = {"auto": hp.EC_AUTO, "always": hp.EC_ALWAYS, "never": hp.EC_NEVER}[args.ec_mode]
    M = ctx.upload(mesh, **up)
    if args.n_cheb_coarse >= 0:
        W["smoother"]["n_cheb_coarse"] = args.n_cheb_coarse
    if args.unfused:
        W["smoother"]["fused"] = False
    lam = M.setup_smoother(**W["smoother"])
    setup_s = time.time() - t0
    N = M.n_dof[0]
    F = torch.zeros(N, dtype=torch.float64, device=dev)
    if prob is not None:
        M.assemble_rhs(prob, F)
    u = torch.zeros_like(F)

    def solve(prec):
        u.zero_()
        if newton:
            st = M.newton_solve(W["nl"], u, tol=1e-10, lin_tol=1e-6, max_lin_iter=args.max_iter, precision=prec)
            st["iterations"] = st["linear_iterations"]
            return st
        return M.solve(F, u, tol=1e-10, max_iter=args.max_iter, precision=prec,
                       solver=hp.SOLVER_FGMRES if args.solver == "fgmres" else hp.SOLVER_FCG)

    for _ in range(warmup):
        solve(hp.PREC_F64)
    torch.cuda.synchronize()
    L = M.n_levels

    def read_timing(prec):
        # per kernel kind: level -> (ms, launches, algorithmic bytes) recorded by the library
        return {kind: [M.kernel_timing(kind, lv, prec) for lv in range(L)] for kind in TIMED_KINDS}

    def timed_solves(prec):
        read_timing(hp.F64), read_timing(hp.F32)  # reset
        M.timing_enable(TIMING_EVERY)
        lat, its, sts = [], [], []
        t_start = time.perf_counter()
        for _ in range(steps):
            a = time.perf_counter()
            st = solve(prec)
            torch.cuda.synchronize()
            lat.append((time.perf_counter() - a) * 1e3)
            its.append(st["iterations"])
            sts.append(st)
        elapsed = time.perf_counter() - t_start
        M.timing_enable(0)
        return elapsed, lat, its, sts, read_timing(hp.F64), read_timing(hp.F32)

    elapsed, lat, iters, sts, t64, _ = timed_solves(hp.PREC_F64)
    st = sts[-1]
    solve(hp.PREC_MIXED)  # warm the FP32 path
    torch.cuda.synchronize()
    el_mx, lat_mx, it_mx, sts_mx, _, t32 = timed_solves(hp.PREC_MIXED)
    stm = sts_mx[-1]
    bf16_info = None
    if W["smoother"]["smoother"] == "block":
        # FP32 V-cycle whose block-Jacobi smoother reads bf16 inverse blocks
        solve(hp.PREC_MIXED_BF16)
        torch.cuda.synchronize()
        el_bf, lat_bf, it_bf, sts_bf, _, _ = timed_solves(hp.PREC_MIXED_BF16)
        bf16_info = {"solves_per_s": round(steps / el_bf, 4), "iterations": it_bf,
                     "final_rel_residual": sts_bf[-1]["rel_residual"],
                     "p50_ms": float(np.percentile(lat_bf, 50)), "p99_ms": float(np.percentile(lat_bf, 99))}

    est_info = None
    if prob is not None and not newton and not args.no_estimator:
        # the a posteriori estimate of the last solution (Eqs. Eta2_*): the first call builds the
        # problem's point data on the host; the timed calls run the kernels only
        eta2 = torch.zeros(M.n_elem[0], dtype=torch.float64, device=dev)
        a = time.perf_counter()
        M.estimate(prob, u, eta2)
        torch.cuda.synchronize()
        build_s = time.perf_counter() - a
        reps = 10
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            M.estimate(prob, u, eta2)
        e1.record()
        torch.cuda.synchronize()
        est_ms = e0.elapsed_time(e1) / reps
        eb, vpts, mpts = M.estimate_info()
        est_info = {"ms": round(est_ms, 4), "dof_per_s": N / (est_ms * 1e-3),
                    "elements_per_s": M.n_elem[0] / (est_ms * 1e-3), "alg_bytes": eb,
                    "gbs": round(eb / (est_ms * 1e-3) / 1e9, 2),
                    "hbm_frac": round(eb / (est_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                    "volume_points": vpts, "mortar_points": mpts, "point_data_build_s": round(build_s, 3),
                    "eta": float(torch.sqrt(eta2.sum())), "reps": reps}

    def totals(entries):
        return (sum(e[0] for e in entries), sum(e[1] for e in entries), sum(e[2] for e in entries))

    kernels = {}
    for kind in TIMED_KINDS:
        ms, n, b = totals(t64[kind])
        if n:
            kernels[kind] = {"kernel": kinds_names[kind], "total_ms": ms, "launches": n, "avg_launch_us": 1e3 * ms / n,
                             "alg_bytes_per_launch": b / n, "gbs": b / (ms * 1e-3) / 1e9,
                             "per_level_launches": [e[1] for e in t64[kind]],
                             "per_level_avg_us": [round(1e3 * e[0] / e[1], 2) if e[1] else None for e in t64[kind]]}
    ms0, n0, b0 = t64["apply"][0]
    ms0_32, n0_32, b0_32 = t32["apply"][0]
    apply_ms64 = ms0 / n0
    apply_ms32 = ms0_32 / n0_32 if n0_32 else float("nan")
    flops = M.apply_flops[0]
    res = {
        "M": M, "N": N, "lam": lam, "setup_s": setup_s, "elapsed": elapsed, "iters": iters, "lat": lat,
        "solves_per_s": steps / elapsed, "ms_per_step": elapsed * 1e3 / steps, "t64": t64, "kernels": kernels,
        "solve": {"iterations": iters, "final_rel_residual": st["rel_residual"],
                  "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                  "setup_s": round(setup_s, 3), "lambda_max": [round(float(v), 4) for v in lam],
                  "setup_retries": list(M.setup_retries())},
        "mixed": {"solves_per_s": round(steps / el_mx, 4), "iterations": it_mx, "final_rel_residual": stm["rel_residual"],
                  "p50_ms": float(np.percentile(lat_mx, 50)), "p99_ms": float(np.percentile(lat_mx, 99))},
        "mixed_bf16_blocks": bf16_info,
        "estimator": est_info,
        # fine-level operator applies inside the timed solves (HIP events on the solve stream)
        "apply": {"dof_applies_per_s_f64": N / (apply_ms64 * 1e-3), "dof_applies_per_s_f32": N / (apply_ms32 * 1e-3),
                  "kernel_ms_f64": apply_ms64, "kernel_ms_f32": apply_ms32,
                  "alg_bytes_f64": b0 / n0, "alg_bytes_f32": b0_32 / n0_32 if n0_32 else None,
                  "gbs_f64": b0 / (ms0 * 1e-3) / 1e9,
                  "gbs_f32": b0_32 / (ms0_32 * 1e-3) / 1e9 if n0_32 else None,
                  "hbm_frac_f64": round(b0 / (ms0 * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                  "flops_f64": flops, "fp64_tflops": flops / (apply_ms64 * 1e-3) / 1e12,
                  "fp64_alu_frac": round(flops / (apply_ms64 * 1e-3) / 1e12 / FP64_PEAK_TFLOPS, 4)},
    }
    if newton:
        res["solve"]["newton_steps"] = [s["newton_steps"] for s in sts]
        res["mixed"]["newton_steps"] = [s["newton_steps"] for s in sts_mx]
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="hp", choices=["hp", "shell", "newton", "serving", "sweep", "amr", "schwarz"])
    ap.add_argument("--schwarz-level", type=int, default=3, help="schwarz: refinement level of the unit cube")
    ap.add_argument("--schwarz-p", type=int, default=3, help="schwarz: degree")
    ap.add_argument("--schwarz-overlap", type=int, default=2, help="schwarz: N_overlap")
    ap.add_argument("--schwarz-mesh", default="box", choices=["box", "shell"],
                    help="schwarz: the unit box or the compactified six-patch shell")
    ap.add_argument("--amr-steps", type=int, default=6, help="amr: adaptation steps")
    ap.add_argument("--amr-fraction", type=float, default=0.2, help="amr: fraction of elements marked")
    ap.add_argument("--requests", type=int, default=512, help="serving: number of requests")
    ap.add_argument("--max-active", type=int, default=8, help="serving: requests in flight")
    ap.add_argument("--arrival-factor", type=float, default=1.0,
                    help="serving: Poisson arrival rate as a multiple of the FP64 sequential capacity")
    ap.add_argument("--solver", choices=["fcg", "fgmres"], default="fcg",
                    help="outer Krylov solver of the linear solves (fgmres: restarted flexible GMRES, 30)")
    ap.add_argument("--n-cheb", type=int, default=0, help="0: the workload's default")
    ap.add_argument("--n-cheb-coarse", type=int, default=-1,
                    help="Chebyshev steps on the levels below the finest; -1: the workload's default")
    ap.add_argument("--Lambda", type=float, default=0.0, help="0: the workload's default")
    ap.add_argument("--max-levels", type=int, default=-1,
                    help="multigrid levels (the last one solved exactly); -1: the workload's default, 0: all")
    ap.add_argument("--smoother", default=None, choices=["none", "point", "block"])
    ap.add_argument("--ec-mode", default=None, choices=["auto", "always", "never"],
                    help="element-centric apply by level (the library's default), everywhere it applies, or nowhere")
    ap.add_argument("--max-iter", type=int, default=1000)
    ap.add_argument("--level", type=int, default=3)
    ap.add_argument("--p", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-shell", action="store_true", help="hp workload: skip the shell sub-measurement")
    ap.add_argument("--no-estimator", action="store_true",
                    help="skip the a posteriori estimate after the solves (profiles of the solve alone)")
    ap.add_argument("--shell-steps", type=int, default=5, help="timed solves of the shell sub-measurement")
    ap.add_argument("--apply-reps", type=int, default=50)
    ap.add_argument("--profile-apply", action="store_true",
                    help="only upload the mesh and run --apply-reps FP64 and FP32 applies (for rocprofv3)")
    ap.add_argument("--profile-estimate", action="store_true",
                    help="only upload the mesh and run --apply-reps a posteriori estimates of a seeded vector "
                         "(for rocprofv3)")
    ap.add_argument("--unfused", action="store_true",
                    help="block smoothing with the apply and the block step in separate kernels")
    ap.add_argument("--sweep-p", default="2,3,4,5,6,7", help="sweep: degrees")
    ap.add_argument("--sweep-gb", type=float, default=2.0, help="sweep: algorithmic GB per FP64 apply (at least)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run one 1 GiB device-to-device copy (counter calibration)")
    ap.add_argument("--summarize-traffic", nargs=4, metavar=("FETCH_CSV", "WRITE_CSV", "CAL_FETCH", "CAL_WRITE"),
                    help="write the HBM traffic summary from rocprofv3 --pmc counter CSVs")
    ap.add_argument("--summarize-trace", nargs="+", metavar="ARG",
                    help="KERNEL_STATS_CSV OUT_MD COMMAND [KERNEL_TRACE_CSV]: write a markdown summary of a "
                         "rocprofv3 --kernel-trace --stats run")
    args = ap.parse_args()
    if args.summarize_trace:
        summarize_trace(*args.summarize_trace)
        return
    if args.summarize_traffic:
        summarize_traffic(*args.summarize_traffic, out=os.path.join(ROOT, TRAFFIC_FILE))
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU only (no multi-GPU path); --gpus %d is not supported" % args.gpus}))
        sys.exit(2)

    import torch

    import meshgen
    import paper_1907_01572_amd as hp

    dev = torch.device("cuda:0")
    if args.copy_calibration:
        x = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device=dev)
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": COPY_BYTES}))
        return
    if args.workload == "serving":
        return run_serving(args, meshgen, hp)
    if args.workload == "sweep":
        return run_sweep(args, meshgen, hp)
    if args.workload == "amr":
        return run_amr(args, meshgen, hp)
    if args.workload == "schwarz":
        return run_schwarz(args, meshgen, hp)
    W = make_workload(args, meshgen, hp)
    ctx = hp.Context(0)
    if args.profile_estimate:
        M = ctx.upload(W["mesh"], **W["upload"])
        u = torch.randn(M.n_dof[0], dtype=torch.float64, device=dev, generator=torch.Generator(dev).manual_seed(0))
        eta2 = torch.zeros(M.n_elem[0], dtype=torch.float64, device=dev)
        for _ in range(args.apply_reps):
            M.estimate(W["prob"], u, eta2)
        torch.cuda.synchronize()
        eb, vp, mp = M.estimate_info()
        print(json.dumps({"profile_estimate": True, "dof": M.n_dof[0], "reps": args.apply_reps, "alg_bytes": eb,
                          "volume_points": vp, "mortar_points": mp}))
        return
    if args.profile_apply:
        up = dict(W["upload"])
        if args.max_levels >= 0:
            up["max_levels"] = args.max_levels
        M = ctx.upload(W["mesh"], **up)
        x64 = torch.randn(M.n_dof[0], dtype=torch.float64, device=dev)
        y64 = torch.zeros_like(x64)
        x32, y32 = x64.float(), torch.zeros_like(x64, dtype=torch.float32)
        for _ in range(args.apply_reps):
            M.apply(x64, y64)
        for _ in range(args.apply_reps):
            M.apply(x32, y32)
        torch.cuda.synchronize()
        print(json.dumps({"profile_apply": True, "dof": M.n_dof[0], "reps": args.apply_reps}))
        return
    names = ({"apply": "apply_kernel<double, 6, 7, true, false>", "block": "block_sym_kernel<double, double, true>",
              "smooth": "apply_kernel<double, 6, 7, true, true>"}
             if args.workload == "shell" else
             {"apply": APPLY_EC, "block": "block_sym_kernel<double, double, true>", "smooth": SMOOTH_EC})
    R = run_solves(args, W, hp, ctx, args.steps, args.warmup, names)
    M, N, kernels, t64 = R["M"], R["N"], R["kernels"], R["t64"]
    dom = max(kernels, key=lambda k: kernels[k]["total_ms"])
    # roofline of the dominant kernel on the finest level (its largest launches): the method's
    # algorithmic bytes per launch (the library's count, see the timing call) over the mean event time
    msR, nR, bR = t64[dom][0]
    R_us, R_bytes = 1e3 * msR / nR, bR / nR
    R_gbs = R_bytes / (R_us * 1e-6) / 1e9
    roof = {"bound": "hbm", "achieved": round(R_gbs, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(R_gbs / HBM_PEAK_GBS, 4),
            "traffic": measured_traffic(kernels[dom]["kernel"], R_bytes),
            "kernel": kernels[dom]["kernel"], "level": "finest", "avg_launch_us": round(R_us, 2),
            "alg_bytes_per_launch": round(R_bytes)}
    if dom == "apply":
        roof["fp64_alu_frac"] = R["apply"]["fp64_alu_frac"]
        roof["fp64_tflops"] = round(R["apply"]["fp64_tflops"], 3)
    out = {
        "metric": METRIC,
        "value": round(R["solves_per_s"], 4),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(R["ms_per_step"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": W["desc"] + " (%d DOF)" % N, "name": args.workload,
                   "elements": M.n_elem[0], "dof": N, "levels": M.n_levels, "level_dof": list(M.n_dof),
                   "n_cheb": W["smoother"]["n_cheb"], "n_cheb_coarse": W["smoother"].get("n_cheb_coarse", 0),
                   "Lambda": W["smoother"]["Lambda"],
                   "smoother": W["smoother"]["smoother"], "solver": args.solver},
        "solve": R["solve"],
        "mixed": R["mixed"],
        "mixed_bf16_blocks": R["mixed_bf16_blocks"],
        "apply": R["apply"],
        "estimator": R["estimator"],
        "kernels_f64_solve": kernels,
        "roofline": roof,
    }
    if not args.no_cpu:
        n_lin = float(np.mean(R["iters"]))
        n_newton = float(np.mean(R["solve"].get("newton_steps", [0])))
        out["cpu_baseline"] = cpu_baseline(W["mesh"], W["prob"], M, W["smoother"]["n_cheb"],
                                           W["smoother"].get("n_cheb_coarse", 0), n_lin, n_newton,
                                           mass="nl" in W)
    M.free()
    if args.workload == "hp" and not args.no_shell:
        # the compactified shell (p = 5, 1,244,160 DOF): its own solves, smoother and fused step
        a2 = argparse.Namespace(**vars(args))
        a2.workload, a2.n_cheb, a2.Lambda, a2.smoother = "shell", 0, 0.0, None
        W2 = make_workload(a2, meshgen, hp)
        n2 = {"apply": "apply_kernel<double, 6, 7, true, false>", "block": "block_sym_kernel<double, double, true>",
              "smooth": "apply_kernel<double, 6, 7, true, true>"}
        S = run_solves(a2, W2, hp, ctx, args.shell_steps, 1, n2)
        k2 = S["kernels"]
        d2 = max(k2, key=lambda k: k2[k]["total_ms"])
        ms2, c2, b2 = S["t64"][d2][0]
        sm = {"workload": W2["desc"] + " (%d DOF)" % S["N"], "steps": args.shell_steps,
              "solves_per_s": round(S["solves_per_s"], 4), "solve": S["solve"], "mixed": S["mixed"],
              "mixed_bf16_blocks": S["mixed_bf16_blocks"], "apply": S["apply"], "estimator": S["estimator"],
              "n_cheb": W2["smoother"]["n_cheb"], "Lambda": W2["smoother"]["Lambda"], "smoother": "block",
              "dominant_kernel": {"kernel": k2[d2]["kernel"], "avg_launch_us": round(1e3 * ms2 / c2, 2),
                                  "alg_bytes_per_launch": round(b2 / c2),
                                  "hbm_frac": round(b2 / c2 / (ms2 / c2 * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}}
        if d2 == "smooth":
            # the fused step's bytes are mostly the packed element-block inverses (the block-Jacobi
            # smoother's own data, N (N + 1) / 2 FP64 values per element, N = (p + 1)^3); the
            # operator's own share is the apply's bytes without the y write
            nb = (S["M"].level_cells(0)["elem_p"].astype(np.float64) + 1) ** 3
            blk = float(8.0 * np.sum(nb * (nb + 1) / 2))
            sm["dominant_kernel"]["block_inverse_bytes_per_launch"] = round(blk)
            sm["dominant_kernel"]["method_bytes_per_launch"] = round(b2 / c2 - blk)
            sm["dominant_kernel"]["method_hbm_frac"] = round((b2 / c2 - blk) / (ms2 / c2 * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
        S["M"].free()
        out["shell"] = sm
    out["sweep"] = committed_sweep()
    print(json.dumps(out))
    ctx.close()


def serving_requests(n, meshgen, hp, seed=0):
    """The request mix: Poisson or variable-k, on a unit cube or a cubed-sphere shell
    (r in [1, 3], linear radial map), target DOF log-uniform in [1e4, 4e6] mapped to the nearest
    level at a degree p uniform in 2..7, source a seeded sum of 8 Gaussians, g_D = 0."""
    rng = np.random.default_rng(seed)
    cache = {}
    reqs = []
    for i in range(n):
        mesh_kind = "cube" if rng.random() < 0.5 else "shell"
        var_k = rng.random() < 0.5
        target = float(np.exp(rng.uniform(np.log(1e4), np.log(4e6))))
        p = int(rng.integers(2, 8))
        per = (p + 1) ** 3 * (1 if mesh_kind == "cube" else 6)
        level = int(np.clip(np.round(np.log(target / per) / np.log(8.0)), 0, 6 if mesh_kind == "cube" else 5))
        key = (mesh_kind, level, p)
        if key not in cache:
            cache[key] = (meshgen.unit_cube(level, p) if mesh_kind == "cube" else
                          meshgen.cubed_sphere_shell(level=level, p=p, r_in=1.0, r_out=3.0, radial_kind=0,
                                                     inner_refine=False))
        lo, hi = ((0, 0, 0), (1, 1, 1)) if mesh_kind == "cube" else ((-3, -3, -3), (3, 3, 3))
        prob = meshgen.gaussian_problem(n=8, lo=lo, hi=hi, seed=seed * 100003 + i)
        coef = (hp.COEF_RADIAL_STEP, [0.5 if mesh_kind == "cube" else 2.0, 1.0, 5.0, 0.0]) if var_k else None
        reqs.append(dict(mesh=cache[key], prob=prob, coef=coef, dof=meshgen.dof_count(cache[key]),
                         key="%s-l%d-p%d%s" % (mesh_kind, level, p, "-k" if var_k else "")))
    return reqs


def run_serving(args, meshgen, hp):
    """Serving stream: requests arrive as a seeded Poisson process at a fixed rate (a multiple of
    the FP64 sequential capacity of the mix: a one-at-a-time server would fall behind);
    solves/s = requests / makespan, latency = completion - arrival."""
    import torch  # noqa: F401 (device init)

    ctx = hp.Context(0)
    reqs = serving_requests(args.requests, meshgen, hp)
    common = dict(n_cheb=4, smoother="point", Lambda=20.0, tol=1e-10, max_iter=args.max_iter)

    def run(precision, max_active, arrivals):
        sv = hp.Server(ctx, max_active=max_active, precision=precision, **common)
        outs = [np.zeros(r["dof"]) for r in reqs]
        t0 = time.perf_counter()
        tickets = []
        for k, (r, o, ta) in enumerate(zip(reqs, outs, arrivals)):
            delay = ta - (time.perf_counter() - t0)
            if delay > 0:
                time.sleep(delay)
            tickets.append(sv.submit(r["mesh"], r["prob"], o, coef=r["coef"]))
            if (k + 1) % 16 == 0:
                print("serving: %d submitted, %.1fs" % (k + 1, time.perf_counter() - t0), file=sys.stderr, flush=True)
        sts = []
        for k, t in enumerate(tickets):
            sts.append(sv.wait(t))
            if (k + 1) % 16 == 0:
                print("serving %s: %d/%d done, %.1fs" % ("f64" if precision == hp.PREC_F64 else "mixed", k + 1,
                                                       len(tickets), time.perf_counter() - t0),
                      file=sys.stderr, flush=True)
        makespan = time.perf_counter() - t0
        sv.close()
        lat = [s["end_ms"] - s["submit_ms"] for s in sts]
        failed = sum(s["state"] != "done" for s in sts)
        for k, s_ in enumerate(sts):
            if s_["state"] != "done":
                print("serving: request %d (%s, %d DOF) failed: status %d: %s"
                      % (k, reqs[k]["key"], reqs[k]["dof"], s_["status"], s_["message"]), file=sys.stderr, flush=True)
        return dict(makespan_s=makespan, solves_per_s=len(reqs) / makespan, p50_ms=float(np.percentile(lat, 50)),
                    p99_ms=float(np.percentile(lat, 99)), failed=failed,
                    iterations_mean=float(np.mean([s["iterations"] for s in sts])),
                    max_rel_residual=float(max(s["rel_residual"] for s in sts)))

    # FP64 sequential capacity of the mix (one request at a time, all submitted at once)
    seq = run(hp.PREC_F64, 1, [0.0] * len(reqs))
    rate = seq["solves_per_s"] * args.arrival_factor
    arrivals = np.cumsum(np.random.default_rng(1).exponential(1.0 / rate, len(reqs)))
    f64 = run(hp.PREC_F64, args.max_active, arrivals)
    mixed = run(hp.PREC_MIXED, args.max_active, arrivals)
    # saturated: every request queued at once, max_active in flight (throughput of the server)
    sat64 = run(hp.PREC_F64, args.max_active, [0.0] * len(reqs))
    satmx = run(hp.PREC_MIXED, args.max_active, [0.0] * len(reqs))
    dofs = [r["dof"] for r in reqs]
    out = {
        "metric": METRIC, "value": round(f64["solves_per_s"], 4), "unit": "solves/s", "n_gpus": 1,
        "steps": len(reqs), "warmup": 0, "ms_per_step": round(1e3 * f64["makespan_s"] / len(reqs), 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "serving stream: %d requests, Poisson arrivals at %.3g x the FP64 sequential "
                               "capacity (%.3f req/s), Poisson/var-k x cube/shell, DOF log-uniform 1e4..4e6 "
                               "(mean %.0f), p 2..7, 8-Gaussian sources, to 1e-10"
                               % (len(reqs), args.arrival_factor, rate, np.mean(dofs)),
                   "name": "serving", "max_active": args.max_active, "arrival_factor": args.arrival_factor,
                   "distinct_meshes": len({r["key"] for r in reqs})},
        "sequential_f64": seq, "served_f64": f64, "served_mixed": mixed,
        "saturated_f64": sat64, "saturated_mixed": satmx,
        "p50_ms": f64["p50_ms"], "p99_ms": f64["p99_ms"],
    }
    print(json.dumps(out))
    ctx.close()


def _oracle_apply_rate(job):
    """One host worker: the oracle's matrix-free apply restricted to ``elems`` (their rows exact),
    repeated for about ``seconds`` on one thread; returns (sample DOF, applies, seconds, setup s)."""
    mesh, prob, elems, mass, seconds, seed = job
    from threadpoolctl import threadpool_limits

    from oracle.operator import SIPG

    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        op = SIPG(mesh, prob, active=elems, mass=(lambda x: np.zeros(x.shape[:-1])) if mass else None)
        t_setup = time.perf_counter() - t0
        x = np.random.default_rng(seed).standard_normal(op.ndof)
        reps = 0
        t0 = time.perf_counter()
        while True:
            op.apply(x)
            reps += 1
            if time.perf_counter() - t0 > seconds or reps >= 400:
                break
        el = time.perf_counter() - t0
    dof = int(np.sum((np.asarray(mesh["elem_p"])[elems].astype(np.int64) + 1) ** 3))
    return dof, reps, el, t_setup


def host_cores():
    """Logical CPUs the host reports, and the workers used (the box's share: at most 16)."""
    n = os.cpu_count() or 1
    try:
        n_aff = len(os.sched_getaffinity(0))
    except AttributeError:
        n_aff = n
    return n, n_aff, max(1, min(n_aff, 16))


def cpu_baseline(mesh, prob, M, n_cheb, n_cheb_coarse, n_lin, n_newton, mass=False):
    """The oracle's matrix-free apply on bounded samples of the same mesh, on the host: one
    thread, and one worker process per core of the box's share (each on its own sample)."""
    import multiprocessing as mp

    rng = np.random.default_rng(0)
    E = len(mesh["elem_p"])
    sample = np.sort(rng.choice(E, size=min(E, 192), replace=False))
    dof1, reps1, el1, setup1 = _oracle_apply_rate((mesh, prob, sample, mass, 10.0, 0))
    rate1 = dof1 * reps1 / el1
    n_cpu, n_aff, workers = host_cores()
    jobs = [(mesh, prob, np.sort(rng.choice(E, size=min(E, 96), replace=False)), mass, 8.0, w + 1)
            for w in range(workers)]
    t0 = time.perf_counter()
    with mp.get_context("spawn").Pool(workers) as pool:  # fresh interpreters: no GPU state
        res = pool.map(_oracle_apply_rate, jobs)
    wall = time.perf_counter() - t0
    rate_all = sum(d * r / e for d, r, e, _ in res)
    # DOF-applies of one GPU solve, counted from its structure: the initial residual, then per
    # FCG iteration one fine apply plus, on every smoothed level, (n_cheb - 1) pre-smoothing
    # applies (the first step starts from zero), one residual and n_cheb post-smoothing applies;
    # per Newton step two residuals and 15 CG-bound applies per smoothed level.  The oracle's
    # rate divided by this count bounds its solves/s from above (smoother block solves,
    # transfers, vector work and the coarse factorisations are not charged to it).
    steps = [n_cheb if lv == 0 or n_cheb_coarse <= 0 else n_cheb_coarse for lv in range(M.n_levels - 1)]
    per_iter = M.n_dof[0] + sum(2 * steps[lv] * M.n_dof[lv] for lv in range(M.n_levels - 1))
    per_newton = 2 * M.n_dof[0] + sum(15 * M.n_dof[lv] for lv in range(M.n_levels - 1))
    dof_applies = M.n_dof[0] + n_lin * per_iter + n_newton * per_newton
    return {"value": rate_all / dof_applies, "unit": "solves/s", "cores": workers, "kind": "oracle",
            "sample": "oracle matrix-free apply (numpy FP64) on seeded element samples of the same mesh: %d worker "
                      "processes of one thread each (%d logical CPUs reported, %d in this process's affinity), "
                      "96 elements each, about 8 s each (%.1f s wall): %.3e DOF-applies/s together; divided by "
                      "the %.3e DOF-applies of one GPU solve" % (workers, n_cpu, n_aff, wall, rate_all, dof_applies),
            "dof_applies_per_s": rate_all,
            "single_thread": {"value": rate1 / dof_applies, "dof_applies_per_s": rate1, "cores": 1,
                              "sample": "%d of %d elements (%d DOF), %d applies in %.1f s (setup %.1f s)"
                                        % (len(sample), E, dof1, reps1, el1, setup1)}}


def run_amr(args, meshgen, hp):
    """hp-adaptive solve (Alg. hpamr) of the k-jump problem on [-1, 1]^3 from 8^3 cells at p = 2:
    per step an MG-FCG solve to 1e-10 (from the previous solution carried over), the a posteriori
    estimate, marking of the largest fraction, smooth-pred decisions and the adapted mesh (2:1
    restored), then upload, smoother setup and solution transfer; every numerical step on the GPU."""
    import torch

    dev = torch.device("cuda:0")
    prob = meshgen.problem_config3()
    coef = hp.coef_from_problem(prob)
    mesh = meshgen.box_grid((1, 1, 1), 3, 2, lo=(-1, -1, -1), hi=(1, 1, 1))
    pred = np.full(len(mesh["elem_p"]), np.inf)
    ctx = hp.Context(0)
    steps, u_prev, M_prev = [], None, None
    t_all = time.perf_counter()
    for k in range(args.amr_steps):
        t0 = time.perf_counter()
        M = ctx.upload(mesh, coef=coef, build_f32=True)
        M.setup_smoother(n_cheb=6, smoother="point", Lambda=20.0)
        N = M.n_dof[0]
        F = torch.zeros(N, dtype=torch.float64, device=dev)
        M.assemble_rhs(prob, F)
        u = torch.zeros_like(F)
        if M_prev is not None:
            M_prev.transfer_to(M, u_prev, u)
            M_prev.free()
        torch.cuda.synchronize()
        t_setup = time.perf_counter() - t0
        st = M.solve(F, u, tol=1e-10, max_iter=args.max_iter, precision=hp.PREC_MIXED)
        torch.cuda.synchronize()
        t_solve = time.perf_counter() - t0 - t_setup
        eta2 = torch.zeros(M.n_elem[0], dtype=torch.float64, device=dev)
        a = time.perf_counter()
        M.estimate(prob, u, eta2)
        torch.cuda.synchronize()
        t_est = time.perf_counter() - a
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        M.estimate(prob, u, eta2)
        e1.record()
        torch.cuda.synchronize()
        est_ms = e0.elapsed_time(e1)
        g = eta2.cpu().numpy()
        a = time.perf_counter()
        marked = hp.amr_mark(g, hp.MARK_FRACTION, args.amr_fraction)
        act, pnew = hp.amr_smooth_pred(g, pred, mesh["elem_p"], marked)
        new, origin = hp.amr_adapt(mesh, act, max_degree=8)
        t_adapt = time.perf_counter() - a
        steps.append({"elements": len(mesh["elem_p"]), "dof": N, "iterations": st["iterations"],
                      "rel_residual": st["rel_residual"], "eta": float(np.sqrt(g.sum())),
                      "h_refined": int(np.sum(act == 1)), "p_refined": int(np.sum(act == 2)),
                      "upload_setup_transfer_s": round(t_setup, 3), "solve_s": round(t_solve, 3),
                      "estimate_ms_first": round(1e3 * t_est, 2), "estimate_ms": round(est_ms, 3),
                      "mark_adapt_ms": round(1e3 * t_adapt, 2)})
        print("amr step %d: %d elements, %d DOF, %d iterations, eta %.4g" % (k, steps[-1]["elements"], N,
              st["iterations"], steps[-1]["eta"]), file=sys.stderr, flush=True)
        pred = pnew[origin]
        u_prev, M_prev = u, M
        mesh = new
    M_prev.free()
    wall = time.perf_counter() - t_all
    out = {"metric": METRIC, "value": round(len(steps) / wall, 4), "unit": "solves/s", "n_gpus": 1,
           "steps": len(steps), "warmup": 0, "ms_per_step": round(1e3 * wall / len(steps), 3),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "hp-adaptive solve of -div(k grad u) = -6 on [-1,1]^3 (k = 1 | 5 across r = 0.5) "
                                  "from 8^3 cells at p = 2: MG-FCG (mixed) to 1e-10, estimate, mark %.0f%%, "
                                  "smooth-pred (gamma_h 0.25, gamma_p 0.1), adapt, transfer; per step"
                                  % (100 * args.amr_fraction), "name": "amr"},
           "amr_steps": steps}
    print(json.dumps(out))
    ctx.close()


def run_schwarz(args, meshgen, hp):
    """Multigrid-preconditioned FCG with the additive Schwarz smoother (N_overlap 2, three cycles
    per smoothing call, the settings of the paper's smoother comparison) against Chebyshev
    smoothing, on the unit box (point Jacobi) or on the six-patch shell compactified to 1e9
    (block and point Jacobi; Sec. III.C): setup time, iterations and solve time of each, and the
    roofline of the Schwarz local-solve kernel (HIP events around every launch during one extra
    solve)."""
    import torch

    dev = torch.device("cuda:0")
    if args.schwarz_mesh == "shell":
        # the six-patch shell compactified to r = 1e9 without the extra inner refinement (the
        # smoother needs 1:1 faces); block Jacobi with the shell settings of the main benchmark
        prob = meshgen.problem_config2()
        mesh = meshgen.cubed_sphere_shell(level=args.schwarz_level, p=args.schwarz_p, r_out=1e9, inner_refine=False)
        label = "cubed-sphere shell compactified to r = 1e9, 6 x %d^3 cells, p = %d" % (2 ** args.schwarz_level,
                                                                                       args.schwarz_p)
        problem = "-lap u = 0, Dirichlet data of u = 1/r + x z / r^5 on both spheres"
        others = (("chebyshev_block", dict(n_cheb=26, Lambda=600.0, smoother="block")),
                  ("chebyshev_point", dict(n_cheb=4, smoother="point")))
    else:
        prob = meshgen.problem_config1()
        mesh = meshgen.unit_cube(args.schwarz_level, args.schwarz_p)
        label = "unit cube, %d^3 affine cells, p = %d" % (2 ** args.schwarz_level, args.schwarz_p)
        problem = "-lap u = 3 pi^2 sin sin sin, u = 0 on the boundary"
        others = (("chebyshev_point", dict(n_cheb=4, smoother="point")),)
    ctx = hp.Context(0)
    M = ctx.upload(mesh, coef=hp.coef_from_problem(prob), build_f32=True)
    N = M.n_dof[0]
    F = torch.zeros(N, dtype=torch.float64, device=dev)
    M.assemble_rhs(prob, F)
    out = {}
    for name, kw in (("schwarz", dict(n_cheb=3, smoother="schwarz", schwarz_overlap=args.schwarz_overlap)),) + others:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        M.setup_smoother(**kw)
        torch.cuda.synchronize()
        setup_s = time.perf_counter() - t0
        times, st = [], None
        for k in range(args.warmup + args.steps):
            u = torch.zeros_like(F)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st = M.solve(F, u, tol=1e-10, max_iter=args.max_iter, raise_on_error=False)
            torch.cuda.synchronize()
            if k >= args.warmup:
                times.append(time.perf_counter() - t0)
            if st["status"] != 0:  # e.g. the iteration cap: reported, not repeated
                break
        out[name] = {"setup_s": round(setup_s, 3), "iterations": st["iterations"],
                     "rel_residual": st["rel_residual"], "converged": st["status"] == 0,
                     "solve_ms": round(1e3 * float(np.median(times)), 3) if times else None}
        print("schwarz workload: %s setup %.2f s, %d iterations (%s), %s ms per solve" %
              (name, setup_s, st["iterations"], "converged" if st["status"] == 0 else "status %d" % st["status"],
               out[name]["solve_ms"]), file=sys.stderr, flush=True)
        if st["status"] == 0:  # the FP32 V-cycle inside FP64 FCG
            mt = []
            for k in range(args.warmup + args.steps):
                u = torch.zeros_like(F)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                stm = M.solve(F, u, tol=1e-10, max_iter=args.max_iter, precision=hp.PREC_MIXED, raise_on_error=False)
                torch.cuda.synchronize()
                if k >= args.warmup:
                    mt.append(time.perf_counter() - t0)
            out[name]["mixed"] = {"iterations": stm["iterations"], "rel_residual": stm["rel_residual"],
                                  "converged": stm["status"] == 0, "solve_ms": round(1e3 * float(np.median(mt)), 3)}
            print("schwarz workload: %s mixed %d iterations, %.3f ms per solve" %
                  (name, stm["iterations"], out[name]["mixed"]["solve_ms"]), file=sys.stderr, flush=True)
        if name == "schwarz":
            M.timing_enable(1)
            u = torch.zeros_like(F)
            M.solve(F, u, tol=1e-10, max_iter=args.max_iter)
            ms, n, b = M.kernel_timing("schwarz", 0)
            u = torch.zeros_like(F)
            M.solve(F, u, tol=1e-10, max_iter=args.max_iter, precision=hp.PREC_MIXED, raise_on_error=False)
            ms32, n32, b32 = M.kernel_timing("schwarz", 0, hp.F32)
            M.timing_enable(0)
            for key, (t, c, by) in (("roofline", (ms, n, b)), ("roofline_fp32", (ms32, n32, b32))):
                if c == 0:
                    continue
                gbs = by / c / (t / c * 1e-3) / 1e9
                out[name][key] = {"kernel": "schwarz_local_kernel<%s> (level 0)" % ("float" if key.endswith("32") else
                                                                                  "double"),
                                  "bound": "hbm", "achieved": round(gbs, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                  "frac": round(gbs / HBM_PEAK_GBS, 4), "launches": c,
                                  "avg_us": round(1e3 * t / c, 2), "alg_bytes_per_launch": by / c}
    retries = list(M.setup_retries())
    M.free()
    res = {"workload": "schwarz", "setup_retries": retries,
           "config": {"mesh": label, "dof": N, "problem": problem, "tol": 1e-10,
                      "schwarz_overlap": args.schwarz_overlap, "schwarz_cycles": 3,
                      "chebyshev": {k: v for k, v in others}, "steps": args.steps, "warmup": args.warmup},
           **out}
    print(json.dumps(res))
    ctx.close()


SWEEP_FILE = os.path.join("profiles", "apply_sweep_uniform_box.json")


def run_sweep(args, meshgen, hp):
    """Out-of-cache apply rates: the unit box as M^3 affine macros refined to a level, degree p
    (the plain-method family), sized so that one FP64 apply moves at least --sweep-gb GB of
    algorithmic bytes; FP64 and FP32 applies timed with HIP events; written to SWEEP_FILE."""
    import torch

    ctx = hp.Context(0)
    rows = []
    for p in [int(v) for v in args.sweep_p.split(",")]:
        n3 = (p + 1) ** 3
        # algorithmic bytes per element: x and y (16 n^3), the 6 metric values, the element
        # record and six face-task records (the library's count)
        per_el = 16.0 * n3 + 48.0 + 88.0 + 6 * 32.0
        need = args.sweep_gb * 1e9 / per_el
        best = None
        for level in range(2, 8):
            for Mm in range(1, 9):
                E = Mm ** 3 * 8 ** level
                if E >= need and (best is None or E < best[0]):
                    best = (E, Mm, level)
        E, Mm, level = best
        t0 = time.time()
        mesh = meshgen.uniform_box((Mm, Mm, Mm), level, p)
        M = ctx.upload(mesh, build_f32=True, max_levels=1)  # applies only: one level
        up = time.time() - t0
        row = {"p": p, "macros": Mm, "level": level, "elements": M.n_elem[0], "dof": M.n_dof[0],
               "cells_per_axis": Mm * 2 ** level, "upload_s": round(up, 1)}
        flops = M.apply_flops[0]
        for dt, tag, sc in ((torch.float64, "f64", 8), (torch.float32, "f32", 4)):
            x = torch.randn(M.n_dof[0], dtype=dt, device="cuda")
            y = torch.zeros_like(x)
            for _ in range(3):
                M.apply(x, y)
            torch.cuda.synchronize()
            M.timing_enable(1)
            M.kernel_timing("apply", 0, hp.F64 if sc == 8 else hp.F32)
            for _ in range(args.apply_reps):
                M.apply(x, y)
            ms, n, b = M.kernel_timing("apply", 0, hp.F64 if sc == 8 else hp.F32)
            M.timing_enable(0)
            t = ms / n * 1e-3
            row[tag] = {"ms": round(ms / n, 4), "gdof_per_s": round(M.n_dof[0] / t / 1e9, 3),
                        "alg_bytes": round(b / n), "gbs": round(b / n / t / 1e9, 1),
                        "hbm_frac": round(b / n / t / 1e9 / HBM_PEAK_GBS, 4)}
            if sc == 8:
                row[tag]["fp64_tflops"] = round(flops / t / 1e12, 3)
                row[tag]["fp64_alu_frac"] = round(flops / t / 1e12 / FP64_PEAK_TFLOPS, 4)
            del x, y
        print(json.dumps(row), flush=True)
        rows.append(row)
        M.free()
        del mesh
    out = {"family": "unit box, M^3 affine macros refined uniformly, degree p, constant k (q = p + 1)",
           "min_alg_gb_per_apply": args.sweep_gb, "reps": args.apply_reps, "rows": rows,
           "sources_sha256": kernel_sources_sha256(),
           "command": "python bench.py --workload sweep --sweep-p %s --sweep-gb %g --apply-reps %d"
                      % (args.sweep_p, args.sweep_gb, args.apply_reps)}
    with open(os.path.join(ROOT, SWEEP_FILE), "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps({"sweep_written": SWEEP_FILE, "rows": len(rows)}))
    ctx.close()


def committed_sweep():
    """The committed out-of-cache sweep (bench.py --workload sweep), or None when the kernel
    sources changed since it was measured."""
    path = os.path.join(ROOT, SWEEP_FILE)
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    if d.get("sources_sha256") != kernel_sources_sha256():
        return None
    return {"source": SWEEP_FILE, "command": d["command"], "family": d["family"],
            "rows": [{"p": r["p"], "dof": r["dof"], "cells_per_axis": r["cells_per_axis"],
                      "alg_gb": round(r["f64"]["alg_bytes"] / 1e9, 3), "f64_gdof_per_s": r["f64"]["gdof_per_s"],
                      "f64_hbm_frac": r["f64"]["hbm_frac"], "f64_alu_frac": r["f64"]["fp64_alu_frac"],
                      "f32_gdof_per_s": r["f32"]["gdof_per_s"], "f32_hbm_frac": r["f32"]["hbm_frac"]}
                     for r in d["rows"]]}


if __name__ == "__main__":
    main()
