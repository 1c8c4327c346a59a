"""Benchmark: MG-preconditioned FCG solves of the SIPG operator on one MI355X.

Workload (default): Poisson on the six-patch cubed-sphere shell r in [1, 1e9] (linear radial
map up to r = 10, inverse-radius compactification beyond), 8^3 cells per patch, innermost
radial layer refined 2:1, degree p = 5 (1,244,160 DOF), manufactured harmonic solution
u = 1/r + x z / r^5 with Dirichlet data.  One step = one solve from u = 0 to a relative
residual of 1e-10 (FP64 flexible CG, V-cycle with Jacobi-Chebyshev smoothing, exact coarse
solve): every row of the hot path runs inside it.  Printed: one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
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
                  for f in ("apply.hip", "kernels.hip", "device.hpp", "host.hpp")]
COPY_BYTES = 1 << 30  # calibration copy: 1 GiB read, 1 GiB written
# kernel timing inside the timed solves: HIP events around every 8th launch of each kernel
# kind and level (two event records per sampled launch)
TIMING_EVERY = 8


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


def summarize_traffic(fetch_csv, write_csv, cal_fetch_csv, cal_write_csv, kernels, out):
    """Mean FETCH_SIZE + WRITE_SIZE per dispatch of each kernel (rocprofv3 --pmc CSVs, KiB),
    each scaled by the same counter on a 1 GiB device copy, written as a text summary."""
    import csv

    def per_kernel(path):
        acc = {}
        with open(path) as fh:
            for r in csv.DictReader(fh):
                name = r["Kernel_Name"]
                acc.setdefault(name, []).append(float(r["Counter_Value"]) * 1024.0)
        return acc

    def copy_value(path):
        acc = per_kernel(path)
        return max(max(v) for k, v in acc.items() if "copyBuffer" in k)

    sf = COPY_BYTES / copy_value(cal_fetch_csv)
    sw = COPY_BYTES / copy_value(cal_write_csv)
    fa, wa = per_kernel(fetch_csv), per_kernel(write_csv)
    lines = ["# HBM traffic per launch: rocprofv3 FETCH_SIZE and WRITE_SIZE (KiB per dispatch),",
             "# scaled by the counters read on a 1 GiB device-to-device copy",
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n-cheb", type=int, default=8)
    ap.add_argument("--Lambda", type=float, default=100.0)
    ap.add_argument("--smoother", default="block", choices=["none", "point", "block"])
    ap.add_argument("--max-iter", type=int, default=1000)
    ap.add_argument("--level", type=int, default=3)
    ap.add_argument("--p", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--apply-reps", type=int, default=50)
    ap.add_argument("--profile-apply", action="store_true",
                    help="only upload the mesh and run --apply-reps FP64 and FP32 applies (for rocprofv3)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run one 1 GiB device-to-device copy (counter calibration)")
    ap.add_argument("--summarize-traffic", nargs=4, metavar=("FETCH_CSV", "WRITE_CSV", "CAL_FETCH", "CAL_WRITE"),
                    help="write the HBM traffic summary from rocprofv3 --pmc counter CSVs")
    args = ap.parse_args()
    if args.summarize_traffic:
        summarize_traffic(*args.summarize_traffic,
                          kernels=["apply_kernel<double, 6, 7, true>", "block_kernel<double, true>",
                                   "apply_kernel<float, 6, 7, true>", "block_kernel<float, true>"],
                          out=os.path.join(ROOT, TRAFFIC_FILE))
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus %d is not supported" % args.gpus}))
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
    mesh = meshgen.cubed_sphere_shell(level=args.level, p=args.p)
    prob = meshgen.problem_config2()
    ctx = hp.Context(0)
    t0 = time.time()
    M = ctx.upload(mesh, build_f32=True)
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
    lam = M.setup_smoother(n_cheb=args.n_cheb, smoother=args.smoother, Lambda=args.Lambda)
    setup_s = time.time() - t0
    N = M.n_dof[0]
    F = torch.zeros(N, dtype=torch.float64, device=dev)
    M.assemble_rhs(prob, F)
    u = torch.zeros_like(F)
    stream = torch.cuda.current_stream()

    def solve(prec):
        u.zero_()
        return M.solve(F, u, tol=1e-10, max_iter=args.max_iter, precision=prec)

    for _ in range(args.warmup):
        solve(hp.PREC_F64)
    torch.cuda.synchronize()
    L = M.n_levels

    def read_timing(prec):
        # per kernel kind: level -> (ms, launches, algorithmic bytes) recorded by the library
        return {kind: [M.kernel_timing(kind, l, prec) for l in range(L)] for kind in ("apply", "block")}

    read_timing(hp.F64), read_timing(hp.F32)  # reset
    M.timing_enable(TIMING_EVERY)
    lat = []
    iters = []
    t_start = time.perf_counter()
    for _ in range(args.steps):
        a = time.perf_counter()
        st = solve(hp.PREC_F64)
        torch.cuda.synchronize()
        lat.append((time.perf_counter() - a) * 1e3)
        iters.append(st["iterations"])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    M.timing_enable(0)
    t64 = read_timing(hp.F64)
    ms_per_step = elapsed * 1e3 / args.steps
    solves_per_s = args.steps / elapsed
    final_res = st["rel_residual"]

    # mixed precision (FP32 V-cycle inside FP64 FCG)
    solve(hp.PREC_MIXED)
    torch.cuda.synchronize()
    read_timing(hp.F64), read_timing(hp.F32)
    M.timing_enable(TIMING_EVERY)
    lat_mx, it_mx = [], []
    a0 = time.perf_counter()
    for _ in range(args.steps):
        a = time.perf_counter()
        stm = solve(hp.PREC_MIXED)
        torch.cuda.synchronize()
        lat_mx.append((time.perf_counter() - a) * 1e3)
        it_mx.append(stm["iterations"])
    mixed_solves_per_s = args.steps / (time.perf_counter() - a0)
    M.timing_enable(0)
    t32 = read_timing(hp.F32)

    def totals(entries):
        ms = sum(e[0] for e in entries)
        n = sum(e[1] for e in entries)
        b = sum(e[2] for e in entries)
        return ms, n, b

    kernels = {}
    for kind, name in (("apply", "apply_kernel<double, 6, 7, true>"), ("block", "block_kernel<double, true>")):
        ms, n, b = totals(t64[kind])
        if n:
            kernels[kind] = {"kernel": name, "total_ms": ms, "launches": n, "avg_launch_us": 1e3 * ms / n,
                             "alg_bytes_per_launch": b / n, "gbs": b / (ms * 1e-3) / 1e9,
                             "per_level_launches": [e[1] for e in t64[kind]]}
    dom = max(kernels, key=lambda k: kernels[k]["total_ms"])
    K = kernels[dom]
    ms0, n0, b0 = t64["apply"][0]
    ms0_32, n0_32, b0_32 = t32["apply"][0]
    ndof = N
    apply_ms64 = ms0 / n0
    apply_ms32 = ms0_32 / n0_32 if n0_32 else float("nan")

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
        "config": {"workload": "cubed-sphere shell r=1..1e9 (compactified), 6x8^3 cells + 2:1 inner layer, "
                               "p=%d, %d DOF, Poisson, FP64 MG-FCG to 1e-10" % (args.p, ndof),
                   "elements": M.n_elem[0], "dof": ndof, "levels": M.n_levels, "level_dof": list(M.n_dof),
                   "n_cheb": args.n_cheb, "Lambda": args.Lambda, "smoother": args.smoother},
        "solve": {"iterations": iters, "final_rel_residual": final_res,
                  "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                  "setup_s": round(setup_s, 3), "lambda_max": [round(float(v), 4) for v in lam]},
        "mixed": {"solves_per_s": round(mixed_solves_per_s, 4), "iterations": it_mx,
                  "final_rel_residual": stm["rel_residual"],
                  "p50_ms": float(np.percentile(lat_mx, 50)), "p99_ms": float(np.percentile(lat_mx, 99))},
        # fine-level operator applies inside the timed solves (HIP events on the solve stream)
        "apply": {"dof_applies_per_s_f64": ndof / (apply_ms64 * 1e-3),
                  "dof_applies_per_s_f32": ndof / (apply_ms32 * 1e-3),
                  "kernel_ms_f64": apply_ms64, "kernel_ms_f32": apply_ms32,
                  "alg_bytes_f64": b0 / n0, "alg_bytes_f32": b0_32 / n0_32 if n0_32 else None,
                  "gbs_f64": b0 / (ms0 * 1e-3) / 1e9,
                  "gbs_f32": b0_32 / (ms0_32 * 1e-3) / 1e9 if n0_32 else None},
        "kernels_f64_solve": kernels,
        "roofline": {"bound": "hbm", "achieved": round(K["gbs"], 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(K["gbs"] / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic(K["kernel"], K["alg_bytes_per_launch"]),
                     "kernel": K["kernel"], "avg_launch_us": round(K["avg_launch_us"], 2),
                     "alg_bytes_per_launch": round(K["alg_bytes_per_launch"])},
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(mesh, prob, ndof, iters, M, args.n_cheb)
    print(json.dumps(out))
    M.free()
    ctx.close()


def cpu_baseline(mesh, prob, ndof, iters, M, n_cheb):
    """The oracle's matrix-free apply on a bounded sample of the same mesh, on the host."""
    from threadpoolctl import threadpool_limits

    from oracle.operator import SIPG

    rng = np.random.default_rng(0)
    E = len(mesh["elem_p"])
    sample = np.sort(rng.choice(E, size=min(E, 192), replace=False))
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        op = SIPG(mesh, prob, active=sample)
        t_setup = time.perf_counter() - t0
        x = rng.standard_normal(op.ndof)
        reps = 0
        t0 = time.perf_counter()
        while True:
            op.apply(x)
            reps += 1
            if time.perf_counter() - t0 > 10.0 or reps >= 50:
                break
        t_apply = (time.perf_counter() - t0) / reps
    sample_dof = int(np.sum((mesh["elem_p"][sample].astype(np.int64) + 1) ** 3))
    dof_apply_per_s = sample_dof / t_apply
    # DOF-applies of one GPU solve, counted from its structure: the initial residual, then per
    # FCG iteration one fine apply plus, on every smoothed level, (n_cheb - 1) pre-smoothing
    # applies (the first step starts from zero), one residual and n_cheb post-smoothing applies.
    # The oracle's rate divided by this count bounds its solves/s from above (smoother block
    # solves, transfers and vector work are not charged to it).
    per_iter = M.n_dof[0] + sum(2 * n_cheb * M.n_dof[l] for l in range(M.n_levels - 1))
    dof_applies = M.n_dof[0] + np.mean(iters) * per_iter
    return {"value": dof_apply_per_s / dof_applies, "unit": "solves/s", "cores": 1, "kind": "oracle",
            "sample": "oracle matrix-free apply on %d of %d elements (%d DOF), %d reps in %.1fs (setup %.1fs), "
                      "one thread: %.3e DOF-applies/s, divided by the %.3e DOF-applies of one GPU solve"
                      % (len(sample), E, sample_dof, reps, t_apply * reps, t_setup, dof_apply_per_s,
                         dof_applies),
            "dof_applies_per_s": dof_apply_per_s}


if __name__ == "__main__":
    main()
