"""Benchmark: MG-preconditioned FCG solves of the SIPG operator on one MI355X.

Workload "shell" (default): Poisson on the six-patch cubed-sphere shell r in [1, 1e9]
(linear radial map up to r = 10, inverse-radius compactification beyond), 8^3 cells per
patch, innermost radial layer refined 2:1, degree p = 5 (1,244,160 DOF), manufactured
harmonic solution u = 1/r + x z / r^5 with Dirichlet data.  One step = one solve from u = 0
to a relative residual of 1e-10 (FP64 flexible CG, V-cycle with block-Jacobi Chebyshev
smoothing, exact coarse solve): every row of the linear hot path runs inside it.

Other workloads (``--workload``): "hp" (the [-1,1]^3 cube, 32^3 cells, p uniform in 2..7,
cells cut by r = 0.5 refined, k = 1 / 5 across r = 0.5; 8,649,651 DOF) and "newton" (the
13-macro cube + compactified exterior refined around three seeded punctures, p = 6,
12,739,363 DOF, Newton-Krylov to |R| <= 1e-10 |R_0|).  Printed: one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload shell|hp|newton]
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
# HBM traffic per launch from rocprofv3 FETCH_SIZE / WRITE_SIZE counters, written by
# --summarize-traffic; valid only while the kernel sources hash to the recorded value
TRAFFIC_FILE = os.path.join("profiles", "solve_shell_p5_hbm_traffic.txt")
KERNEL_SOURCES = [os.path.join("paper_1907_01572_amd", "csrc", f)
                  for f in ("apply.hip", "kernels.hip", "blocks.hpp", "device.hpp", "host.hpp")]
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
        top = [r["Name"] for r in rows[:8]]
        for nm in top:
            if nm in fine:
                g, c, m = fine[nm]
                name = nm.split("(hpdg::")[0].replace("void hpdg::(anonymous namespace)::", "").replace("|", "/")
                lines.append("| `%s` | %d | %d | %.1f |" % (name[:90], g, c, m / 1e3))
    with open(out_md, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def summarize_traffic(fetch_csv, write_csv, cal_fetch_csv, cal_write_csv, kernels, out):
    """Mean FETCH_SIZE + WRITE_SIZE per dispatch of each kernel (rocprofv3 --pmc CSVs, KiB),
    each scaled by the same counter on a 1 GiB device copy, written as a text summary."""
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
        lines += ["dispatches[%s]: %d" % (k, len(fa[full[0]])),
                  "fetch_bytes_per_launch[%s]: %.0f" % (k, f),
                  "write_bytes_per_launch[%s]: %.0f" % (k, w),
                  "bytes_per_launch[%s]: %.0f" % (k, f + w)]
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
        w["smoother"] = dict(n_cheb=args.n_cheb or 4, smoother=args.smoother or "point", Lambda=args.Lambda or 20.0)
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="shell", choices=["shell", "hp", "newton", "serving"])
    ap.add_argument("--requests", type=int, default=512, help="serving: number of requests")
    ap.add_argument("--max-active", type=int, default=8, help="serving: requests in flight")
    ap.add_argument("--arrival-factor", type=float, default=2.0,
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
    ap.add_argument("--max-iter", type=int, default=1000)
    ap.add_argument("--level", type=int, default=3)
    ap.add_argument("--p", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--apply-reps", type=int, default=50)
    ap.add_argument("--profile-apply", action="store_true",
                    help="only upload the mesh and run --apply-reps FP64 and FP32 applies (for rocprofv3)")
    ap.add_argument("--unfused", action="store_true",
                    help="block smoothing with the apply and the block step in separate kernels")
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
        summarize_traffic(*args.summarize_traffic,
                          kernels=["apply_kernel<double, 6, 7, true, true>", "apply_kernel<double, 6, 7, true, false>",
                                   "block_sym_kernel<double, double, true>",
                                   "apply_kernel<float, 6, 7, true, true>", "apply_kernel<float, 6, 7, true, false>",
                                   "block_sym_kernel<float, float, true>"],
                          out=os.path.join(ROOT, TRAFFIC_FILE))
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
    W = make_workload(args, meshgen, hp)
    mesh, prob = W["mesh"], W["prob"]
    newton = "nl" in W
    ctx = hp.Context(0)
    t0 = time.time()
    up = dict(W["upload"])
    if args.max_levels >= 0:
        up["max_levels"] = args.max_levels
    M = ctx.upload(mesh, **up)
    if args.profile_apply:
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

    for _ in range(args.warmup):
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
        for _ in range(args.steps):
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
    ms_per_step = elapsed * 1e3 / args.steps
    solves_per_s = args.steps / elapsed
    st = sts[-1]
    solve(hp.PREC_MIXED)  # warm the FP32 path
    torch.cuda.synchronize()
    el_mx, lat_mx, it_mx, sts_mx, _, t32 = timed_solves(hp.PREC_MIXED)
    stm = sts_mx[-1]
    mixed_solves_per_s = args.steps / el_mx
    bf16_info = None
    if W["smoother"]["smoother"] == "block":
        # FP32 V-cycle whose block-Jacobi smoother reads bf16 inverse blocks
        solve(hp.PREC_MIXED_BF16)
        torch.cuda.synchronize()
        el_bf, lat_bf, it_bf, sts_bf, _, _ = timed_solves(hp.PREC_MIXED_BF16)
        bf16_info = {"solves_per_s": round(args.steps / el_bf, 4), "iterations": it_bf,
                     "final_rel_residual": sts_bf[-1]["rel_residual"],
                     "p50_ms": float(np.percentile(lat_bf, 50)), "p99_ms": float(np.percentile(lat_bf, 99))}

    def totals(entries):
        return (sum(e[0] for e in entries), sum(e[1] for e in entries), sum(e[2] for e in entries))

    kernels = {}
    names = ({"apply": "apply_kernel<double, 6, 7, true, false>", "block": "block_sym_kernel<double, double, true>",
              "smooth": "apply_kernel<double, 6, 7, true, true>"}
             if args.workload == "shell" else
             {"apply": "apply_kernel<double, *> (all buckets)", "block": "block_sym_kernel<double, double, true>",
              "smooth": "apply_kernel<double, *, *, true, true>"})
    for kind in TIMED_KINDS:
        ms, n, b = totals(t64[kind])
        if n:
            kernels[kind] = {"kernel": names[kind], "total_ms": ms, "launches": n, "avg_launch_us": 1e3 * ms / n,
                             "alg_bytes_per_launch": b / n, "gbs": b / (ms * 1e-3) / 1e9,
                             "per_level_launches": [e[1] for e in t64[kind]],
                             "per_level_avg_us": [round(1e3 * e[0] / e[1], 2) if e[1] else None for e in t64[kind]]}
    dom = max(kernels, key=lambda k: kernels[k]["total_ms"])
    K = kernels[dom]
    # roofline of the dominant kernel on the finest level (its largest launches)
    msR, nR, bR = t64[dom][0]
    R_us, R_bytes = 1e3 * msR / nR, bR / nR
    R_gbs = R_bytes / (R_us * 1e-6) / 1e9
    ms0, n0, b0 = t64["apply"][0]
    ms0_32, n0_32, b0_32 = t32["apply"][0]
    apply_ms64 = ms0 / n0
    apply_ms32 = ms0_32 / n0_32 if n0_32 else float("nan")

    solve_info = {"iterations": iters, "final_rel_residual": st["rel_residual"],
                  "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                  "setup_s": round(setup_s, 3), "lambda_max": [round(float(v), 4) for v in lam]}
    mixed_info = {"solves_per_s": round(mixed_solves_per_s, 4), "iterations": it_mx,
                  "final_rel_residual": stm["rel_residual"],
                  "p50_ms": float(np.percentile(lat_mx, 50)), "p99_ms": float(np.percentile(lat_mx, 99))}
    if newton:
        solve_info["newton_steps"] = [s["newton_steps"] for s in sts]
        mixed_info["newton_steps"] = [s["newton_steps"] for s in sts_mx]
    out = {
        "metric": METRIC,
        "value": round(solves_per_s, 4),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
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
        "solve": solve_info,
        "mixed": mixed_info,
        "mixed_bf16_blocks": bf16_info,
        # fine-level operator applies inside the timed solves (HIP events on the solve stream)
        "apply": {"dof_applies_per_s_f64": N / (apply_ms64 * 1e-3),
                  "dof_applies_per_s_f32": N / (apply_ms32 * 1e-3),
                  "kernel_ms_f64": apply_ms64, "kernel_ms_f32": apply_ms32,
                  "alg_bytes_f64": b0 / n0, "alg_bytes_f32": b0_32 / n0_32 if n0_32 else None,
                  "gbs_f64": b0 / (ms0 * 1e-3) / 1e9,
                  "gbs_f32": b0_32 / (ms0_32 * 1e-3) / 1e9 if n0_32 else None},
        "kernels_f64_solve": kernels,
        "roofline": {"bound": "hbm", "achieved": round(R_gbs, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(R_gbs / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic(K["kernel"], R_bytes) if args.workload == "shell" else None,
                     "kernel": K["kernel"], "level": "finest", "avg_launch_us": round(R_us, 2),
                     "alg_bytes_per_launch": round(R_bytes)},
    }
    if not args.no_cpu:
        n_lin = float(np.mean(iters))
        n_newton = float(np.mean(solve_info.get("newton_steps", [0])))
        out["cpu_baseline"] = cpu_baseline(mesh, prob, M, W["smoother"]["n_cheb"],
                                           W["smoother"].get("n_cheb_coarse", 0), n_lin, n_newton,
                                           mass=newton)
    print(json.dumps(out))
    M.free()
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


def cpu_baseline(mesh, prob, M, n_cheb, n_cheb_coarse, n_lin, n_newton, mass=False):
    """The oracle's matrix-free apply on a bounded sample of the same mesh, on the host."""
    from threadpoolctl import threadpool_limits

    from oracle.operator import SIPG

    rng = np.random.default_rng(0)
    E = len(mesh["elem_p"])
    sample = np.sort(rng.choice(E, size=min(E, 192), replace=False))
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        op = SIPG(mesh, prob, active=sample, mass=(lambda x: np.zeros(x.shape[:-1])) if mass else None)
        t_setup = time.perf_counter() - t0
        x = rng.standard_normal(op.ndof)
        reps = 0
        t0 = time.perf_counter()
        while True:
            op.apply(x)
            reps += 1
            if time.perf_counter() - t0 > 12.0 or reps >= 400:
                break
        t_apply = (time.perf_counter() - t0) / reps
    sample_dof = int(np.sum((mesh["elem_p"][sample].astype(np.int64) + 1) ** 3))
    dof_apply_per_s = sample_dof / t_apply
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
    return {"value": dof_apply_per_s / dof_applies, "unit": "solves/s", "cores": 1, "kind": "oracle",
            "sample": "oracle matrix-free apply on %d of %d elements (%d DOF), %d reps in %.1fs (setup %.1fs), "
                      "one thread: %.3e DOF-applies/s, divided by the %.3e DOF-applies of one GPU solve"
                      % (len(sample), E, sample_dof, reps, t_apply * reps, t_setup, dof_apply_per_s,
                         dof_applies),
            "dof_applies_per_s": dof_apply_per_s}


if __name__ == "__main__":
    main()
