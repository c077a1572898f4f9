"""Benchmark of the tensor B-spline implicit heat step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload heat928] [--no-cpu-baseline]

K defaults to the workload's own step count (100 implicit steps at 928^3).  A step is one
implicit Euler step of the whole hot path on the 928^3 cubic Dirichlet workload
(~0.8e9 DoF): right-hand side, initial guess (network guess with FP64 fallback test when
trained weights are present, else u^k), FP64-refined FP32 CG to a relative residual of 1e-8.
value = DoF advanced per second (GDoF/s of implicit stepping, inputs resident in HBM).
Also reported: operator-apply throughput (GDoF/s) in FP64, FP32 and bf16->FP32, seconds per
step of plain FP64 CG and of the refined solver with and without the learned guess, the
roofline of the dominant kernel from HIP events recorded by the library on its own stream,
and the FP64 CPU oracle timed on a bounded sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "GDoF/s of (M+τΣK)u apply; s per implicit step at 0.8B DoF, learned vs plain CG"
HBM_PEAK_GBS = 8000.0
# network trained by paper_1904_03057_amd/train_guess.py on 128^3 windows at this workload's grid
# spacing and time step (h = 1/929, tau = 1e-5), half of the training trajectories without a source
WEIGHTS = os.path.join(ROOT, "paper_1904_03057_amd", "weights", "guess_net_928z")


# solver variants: (precision, use the network, tbs_opts.guess_backoff, tbs_opts.guess_test)
SOLVERS = {
    "learned_cost": ("mixed", True, 2, 0),       # refined FP32 + learned guess (residual test), cost-aware backoff
    "learned_backoff": ("mixed", True, 1, 0),    # refined FP32 + learned guess (residual test), backoff
    "learned_every": ("mixed", True, 0, 0),      # same, network run and judged on every step
    "learned_energy_backoff": ("mixed", True, 1, 1),  # energy test (A-norm-optimal multiple), backoff
    "learned_energy_every": ("mixed", True, 0, 1),    # energy test, every step
    "refined": ("mixed", False, 0, 0),           # refined FP32, plain guess
    "fp64": ("fp64", False, 0, 0),               # plain FP64 CG
}
SOLVER_NAMES = {"learned_cost": "fp64-refined fp32 CG + learned guess (residual test, cost-aware backoff)",
                "learned_backoff": "fp64-refined fp32 CG + learned guess (residual test, backoff)",
                "learned_every": "fp64-refined fp32 CG + learned guess (residual test, every step)",
                "learned_energy_backoff": "fp64-refined fp32 CG + learned guess (energy test, backoff)",
                "learned_energy_every": "fp64-refined fp32 CG + learned guess (energy test, every step)",
                "refined": "fp64-refined fp32 CG", "fp64": "plain fp64 CG"}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="default: the workload's step count")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="heat928")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="only the timed steps (for profiling runs)")
    ap.add_argument("--solver", default="learned_cost", choices=list(SOLVERS),
                    help="solver of the timed steps (the others are timed over the same steps in the extras)")
    ap.add_argument("--probe", default=None,
                    help="run one kernel kind --steps times for counter collection instead of the benchmark: "
                         "apply_f64 | apply_f32 | apply_bf16 | net (network guess) | "
                         "copy (f64->f32 conversion, the traffic calibration) | copy16 (16-byte streaming copy) | "
                         "varcoef_f32 | varcoef_f64 | robin_f32 | robin_f64")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path (the design notes "
              "describe how the z-slab decomposition would shard); use --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.probe:
        if args.steps is None:
            args.steps = 5
        probe(args)
        return

    import numpy as np
    import torch

    import paper_1904_03057_amd as tbs
    import workloads

    w = {"heat928": workloads.HEAT_928_DIRICHLET, "heat256": workloads.HEAT_256_DIRICHLET,
         "heat512": workloads.HEAT_512_EVAL}[args.workload]
    if args.steps is None:
        args.steps = w.steps
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    N = w.grid[0] * w.grid[1] * w.grid[2]
    shape = w.grid[::-1]
    log("workload %s grid %s n=%d tau=%g rtol=%g" % (w.name, w.grid, w.degree, w.tau, w.rtol))

    with torch.cuda.stream(stream):
        params = workloads.initial_field_gaussians(w)
        u0 = workloads.gaussian_sum(w.grid, w.bc, w.h, params, xp=torch, device="cuda", dtype=torch.float64)
        ua, ub = u0.clone(), torch.empty_like(u0)
        ctx = tbs.Context(w.grid, w.degree, w.h, w.tau, w.bc, stream=stream)
        # poll convergence after every CG iteration: no launch ever runs past convergence, so the
        # profiler's per-launch averages and rocprofv3's agree (one 8-byte read per ~ms iteration)
        ctx.set_opts()
        ctx.ensure_workspace(tbs.PREC_MIXED)
    net = None
    if os.path.exists(WEIGHTS + ".f32") and args.workload == "heat928":
        net = tbs.Net(stream=stream)
        net.ensure_workspace(w.grid, 1, False)
        net.set_weights(np.fromfile(WEIGHTS + ".f32", dtype="<f4"))
        net.set_hparams(out_scale=json.load(open(WEIGHTS + ".json"))["out_scale"])
    torch.cuda.synchronize()

    sprec, suse, sbackoff, stest = SOLVERS[args.solver]
    if suse and net is None:
        raise SystemExit("solver %s needs the trained weights %s.f32" % (args.solver, WEIGHTS))
    PREC = tbs.PREC_MIXED if sprec == "mixed" else tbs.PREC_FP64
    ctx.set_opts(guess_backoff=sbackoff, guess_test=stest)
    ctx.ensure_workspace(PREC)

    def step(prec, use_net):
        nonlocal ua, ub
        st = ctx.timestep(ua, None, ub, prec, w.rtol, 5000, net if use_net else None)
        ua, ub = ub, ua
        return st

    log("warmup %d" % args.warmup)
    for _ in range(args.warmup):
        step(PREC, suse)
    torch.cuda.synchronize()
    ua.copy_(u0)
    # the backoff counters restart with the timed steps
    ctx.set_opts(guess_backoff=sbackoff, guess_test=stest)
    ctx.ensure_workspace(PREC)
    torch.cuda.synchronize()

    ctx.prof_enable(True)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    stats = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    step_ms = []
    for i in range(args.steps):
        ts = time.perf_counter()
        stats.append(step(PREC, suse))  # synchronises
        step_ms.append((time.perf_counter() - ts) * 1e3)
        log("step %d: iters %d sweeps %d rel_res %.3e learned %d" % (
            i, stats[-1]["iters"], stats[-1]["sweeps"], stats[-1]["rel_res_fp64"], stats[-1]["used_learned_guess"]))
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_total = e0.elapsed_time(e1)
    prof = ctx.prof_read()
    ctx.prof_enable(False)
    s_step = ms_total / 1e3 / args.steps
    value = N / s_step / 1e9

    # dominant kernel of the timed region: the largest total time among the profiled kinds
    dom = max(prof.items(), key=lambda kv: kv[1][0])
    dname, (dms, dbytes, dcount) = dom
    achieved = dbytes / (dms / 1e3) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(dname), "kernel": dname,
                "avg_launch_ms": round(dms / dcount, 4), "launches": dcount,
                "algorithmic_bytes_per_launch": round(dbytes / dcount)}

    out = {
        "metric": METRIC, "value": round(value, 4), "unit": "GDoF/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_total / args.steps, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": w.name, "grid": list(w.grid), "degree": w.degree, "bc": w.bc, "tau": w.tau,
                   "rtol": w.rtol, "solver": SOLVER_NAMES[args.solver],
                   "global_batch": 1, "parallelism": "none"},
        "wall_s_timed": round(wall, 3),
        "step_ms_host": {"median": round(float(np.median(step_ms)), 3), "min": round(min(step_ms), 3),
                         "max": round(max(step_ms), 3), "first": round(step_ms[0], 3), "last": round(step_ms[-1], 3)},
        "iters_per_step": [s["iters"] for s in stats], "sweeps_per_step": [s["sweeps"] for s in stats],
        "learned_guess_used": [s["used_learned_guess"] for s in stats],
        "learned_guess_skipped": [s["skipped_learned_guess"] for s in stats],
        "learned_gamma": [round(s["learned_gamma"], 4) for s in stats],
        "learned_over_plain_residual": [round(s["rel_res_learned"] / s["rel_res_plain"], 4)
                                        if suse and s["rel_res_plain"] > 0 and s["rel_res_learned"] == s["rel_res_learned"]
                                        else None for s in stats],
        "rel_res_fp64": max(s["rel_res_fp64"] for s in stats),
        "roofline": roofline,
        "kernels": {k: {"ms": round(v[0], 3), "GB/s": round(v[1] / (v[0] / 1e3) / 1e9, 1), "launches": v[2]}
                    for k, v in prof.items()},
    }

    if not args.no_extras:
        out.update(extras(ctx, tbs, torch, w, u0, stream, net, N, args.steps))
        out["roofline_varcoef"] = out.get("varcoef", {}).get("roofline")
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, params, out.get("all_%d_steps" % args.steps, {}),
                                           out.get("s_per_step", {}))
    print(json.dumps(out), flush=True)


# the sources of the stencil kernels and of their launch geometry (the host's tile / z-chunk plan):
# a traffic summary holds only while they hash as measured
STENCIL_SOURCES = ("stencil_kernel.h", "stencil.hip", "stencil.h", "common.h")


def stencil_sources_hash():
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1904_03057_amd", "csrc")
    for f in STENCIL_SOURCES:
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    api = open(os.path.join(csrc, "api.cpp")).read()
    start = api.index("static void plan_geometry(")
    h.update(api[start:api.index("\n}\n", start) + 3].encode())
    return h.hexdigest()


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter summary, or None when
    there is none for it or the stencil sources have changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "%s_heat928_traffic.txt" % kernel)
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel") != kernel or kv.get("source_sha256") != stencil_sources_hash():
        return None
    return int(float(kv["traffic_bytes_per_launch"]))


def probe(args):
    """One kernel kind, --steps launches on the 928^3 field (for rocprofv3 counter passes)."""
    import numpy as np
    import torch

    import paper_1904_03057_amd as tbs
    import workloads

    w = workloads.HEAT_928_DIRICHLET
    torch.cuda.set_device(0)
    N = w.grid[0] * w.grid[1] * w.grid[2]
    u = workloads.gaussian_sum(w.grid, w.bc, w.h, workloads.initial_field_gaussians(w), xp=torch,
                               device="cuda", dtype=torch.float64)
    ctx = tbs.Context(w.grid, w.degree, w.h, w.tau, w.bc)
    ctx.ensure_workspace(-1)
    kind = args.probe
    if kind == "apply_f64":
        src, dst = u, torch.empty_like(u)
        run = lambda: ctx.apply(src, dst)
        nbytes = 16 * N
    elif kind == "apply_f32":
        src = u.to(torch.float32)
        dst = torch.empty_like(src)
        run = lambda: ctx.apply(src, dst)
        nbytes = 8 * N
    elif kind == "apply_bf16":
        src = u.to(torch.bfloat16)
        dst = torch.empty(u.shape, dtype=torch.float32, device="cuda")
        run = lambda: ctx.apply(src, dst)
        nbytes = 6 * N
    elif kind == "net":
        net = tbs.Net()
        net.ensure_workspace(w.grid, 1, False)
        net.set_weights(np.fromfile(WEIGHTS + ".f32", dtype="<f4"))
        net.set_hparams(out_scale=json.load(open(WEIGHTS + ".json"))["out_scale"])
        du = torch.empty(u.shape, dtype=torch.float32, device="cuda")
        run = lambda: net.forward(u, None, du, False, w.tau)
        nbytes = 0
    elif kind == "copy":
        dst = torch.empty(u.shape, dtype=torch.float32, device="cuda")
        run = lambda: ctx.convert(u, dst)
        nbytes = 12 * N
    elif kind == "copy16":
        dst = torch.empty_like(u)
        run = lambda: ctx.stream_copy(u, dst)
        nbytes = 16 * N
    elif kind in ("varcoef_f32", "varcoef_f64"):
        td = torch.float32 if kind.endswith("f32") else torch.float64
        src = u.to(td)
        d = torch.full_like(src, w.tau) * (1.0 + 0.5 * torch.tanh(src))
        m = 1.0 + 0.5 * torch.tanh(src)
        dst = torch.empty_like(src)
        run = lambda: ctx.apply_varcoef(src, d, m, dst)
        nbytes = 4 * src.element_size() * N
    elif kind in ("robin_f32", "robin_f64"):
        n = w.degree
        rctx = tbs.RobinContext(w.grid, n, tuple(1.0 / (g - 1 - 2 * (n // 2)) for g in w.grid), w.tau, 1e-3)
        ctx = rctx
        src = u if kind.endswith("f64") else u.to(torch.float32)
        dst = torch.empty_like(src)
        run = lambda: rctx.apply(src, dst)
        nbytes = 2 * src.element_size() * N
    else:
        raise SystemExit("unknown probe " + kind)
    for _ in range(2):  # warm-up (code-object load, caches)
        run()
    torch.cuda.synchronize()
    ctx.prof_enable(True)
    for i in range(args.steps):
        run()
        log("probe %s launch %d" % (kind, i))
    torch.cuda.synchronize()
    p = ctx.prof_read()
    ms = sum(v[0] for v in p.values())
    print(json.dumps({"probe": kind, "launches": args.steps, "algorithmic_bytes_per_launch": nbytes,
                      "avg_ms": (ms / args.steps) if ms else None}), flush=True)


def extras(ctx, tbs, torch, w, u0, stream, net, N, k_all):
    """Apply throughput per dtype and seconds per step of the other solver variants."""
    import numpy as np

    res = {}
    with torch.cuda.stream(stream):
        y64 = torch.empty_like(u0)
        u32 = u0.to(torch.float32)
        y32 = torch.empty_like(u32)
        u16 = u0.to(torch.bfloat16)
    torch.cuda.synchronize()
    gd = {}
    for name, u, y in (("f64", u0, y64), ("f32", u32, y32), ("bf16_to_f32", u16, y32)):
        for _ in range(5):
            ctx.apply(u, y)
        torch.cuda.synchronize()
        ctx.prof_enable(True)
        reps = 20
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
        for a, b in ev:
            a.record(stream)
            ctx.apply(u, y)
            b.record(stream)
        torch.cuda.synchronize()
        p = ctx.prof_read()
        ctx.prof_enable(False)
        ms, by, cnt = list(p.values())[0]
        med = float(np.median([a.elapsed_time(b) for a, b in ev]))
        gd[name] = {"GDoF/s": round(N / (ms / cnt / 1e3) / 1e9, 1), "GB/s": round(by / (ms / 1e3) / 1e9, 1),
                    "frac_hbm": round(by / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4), "ms": round(ms / cnt, 4),
                    "ms_median_of_%d" % reps: round(med, 4), "GDoF/s_median": round(N / (med / 1e3) / 1e9, 1)}
        log("apply %s: %s" % (name, gd[name]))
    # practical ceiling: the library's 16-byte streaming copy of the FP64 field (read 8 B + write 8 B
    # per DoF), timed like the applies
    for _ in range(2):
        ctx.stream_copy(u0, y64)
    torch.cuda.synchronize()
    cev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(10)]
    for a, b in cev:
        a.record(stream)
        ctx.stream_copy(u0, y64)
        b.record(stream)
    torch.cuda.synchronize()
    cms = float(np.median([a.elapsed_time(b) for a, b in cev]))
    copy_gbs = 16 * N / (cms / 1e3) / 1e9
    res["copy_ceiling"] = {"GB/s": round(copy_gbs, 1), "frac_hbm": round(copy_gbs / HBM_PEAK_GBS, 4),
                           "ms_median_of_10": round(cms, 4),
                           "kernel": "tbs_stream_copy (16-byte accesses) of the FP64 928^3 field"}
    for v in gd.values():
        v["frac_copy"] = round(v["GB/s"] / copy_gbs, 4)
    res["apply"] = gd
    del y64, u32, y32, u16
    res["varcoef"] = varcoef_apply(tbs, torch, w)
    res["robin"] = robin_box(tbs, torch, w)
    res["apply_degree_sweep"] = degree_sweep(tbs, torch)
    res["transforms"] = transforms(tbs, torch, w, u0)
    res.update(workload_steps(tbs, torch))
    res.update(graph_cg(tbs, torch))

    def time_steps(prec, use_net, k):
        ua, ub = u0.clone(), torch.empty_like(u0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sts = []
        for _ in range(k):
            sts.append(ctx.timestep(ua, None, ub, prec, w.rtol, 5000, net if use_net else None))
            ua, ub = ub, ua
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / k, sts

    sp = {}
    variants = [("plain_fp64_cg", tbs.PREC_FP64, False), ("refined_fp32", tbs.PREC_MIXED, False),
                ("refined_fp32_bf16p", tbs.PREC_MIXED_BF16, False)]
    if net is not None:
        variants.append(("refined_fp32_learned", tbs.PREC_MIXED, True))
    ctx.ensure_workspace(tbs.PREC_FP64)
    for name, prec, use_net in variants:
        ctx.set_opts()
        ctx.ensure_workspace(tbs.PREC_FP64)
        t, sts = time_steps(prec, use_net, 2)
        sp[name] = {"s_per_step": round(t, 4), "iters": [s["iters"] for s in sts],
                    "rel_res_fp64": max(s["rel_res_fp64"] for s in sts),
                    "learned_used": [s["used_learned_guess"] for s in sts]}
        log("%s: %s" % (name, sp[name]))
    # the paper's reduced-grid start: coarse-grid guess (halved grid, two-scale prolongation)
    ctx.set_opts(coarse_guess=1, coarse_rtol=1e-2)
    for name, prec in (("refined_fp32_coarse", tbs.PREC_MIXED), ("plain_fp64_cg_coarse", tbs.PREC_FP64)):
        ctx.ensure_workspace(prec)
        t, sts = time_steps(prec, False, 2)
        sp[name] = {"s_per_step": round(t, 4), "iters": [s["iters"] for s in sts],
                    "rel_res_fp64": max(s["rel_res_fp64"] for s in sts),
                    "coarse_used": [s["used_coarse_guess"] for s in sts],
                    "coarse_iters": [s["coarse_iters"] for s in sts],
                    "coarse_over_plain_residual": [round(s["rel_res_coarse"] / s["rel_res_plain"], 4) for s in sts]}
        log("%s: %s" % (name, sp[name]))
    ctx.set_opts()
    res["s_per_step"] = sp
    # every solver variant over the same k_all steps as the timed run, from the same field
    ra = {}
    for key, (prec_s, use_net, backoff, test) in SOLVERS.items():
        if use_net and net is None:
            continue
        prec = tbs.PREC_MIXED if prec_s == "mixed" else tbs.PREC_FP64
        ctx.set_opts(guess_backoff=backoff, guess_test=test)
        ctx.ensure_workspace(tbs.PREC_FP64)
        t, sts = time_steps(prec, use_net, k_all)
        name = {"fp64": "plain_fp64_cg", "refined": "refined_fp32"}.get(key, "refined_fp32_" + key)
        ra[name] = {"solver": SOLVER_NAMES[key], "s_per_step": round(t, 4), "steps": k_all,
                    "iters_total": sum(s["iters"] for s in sts),
                    "iters_first_last": [sts[0]["iters"], sts[-1]["iters"]],
                    "rel_res_fp64_max": max(s["rel_res_fp64"] for s in sts)}
        if use_net:
            ra[name]["net_runs"] = sum(1 - s["skipped_learned_guess"] for s in sts)
            ra[name]["net_kept"] = sum(s["used_learned_guess"] for s in sts)
            ra[name]["gamma_first"] = round(sts[0]["learned_gamma"], 4)
            ra[name]["iters_first_steps"] = [s["iters"] for s in sts[:5]]
            if backoff == 2:
                ran = [s for s in sts if not s["skipped_learned_guess"]]
                ra[name]["saved_vs_cost_iters"] = [[round(s["learned_saved_iters"], 2), round(s["learned_cost_iters"], 2)]
                                                   for s in ran]
        log("%d steps %s: %s" % (k_all, name, ra[name]))
    ctx.set_opts()
    ctx.ensure_workspace(tbs.PREC_MIXED)
    res["all_%d_steps" % k_all] = ra
    if net is not None:
        du = torch.empty(u0.shape, dtype=torch.float32, device="cuda")
        for _ in range(2):
            net.forward(u0, None, du, False, w.tau)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(3):
            net.forward(u0, None, du, False, w.tau)
        torch.cuda.synchronize()
        res["net_forward_s"] = round((time.perf_counter() - t0) / 3, 4)
        log("net forward: %.4f s" % res["net_forward_s"])
        del du
    return res


def varcoef_flops_per_dof(n):
    """Algorithmic flops per coefficient of the sum-factorised variable-coefficient operator: the
    multiply-adds of the interpolations (z: 4 fields, y: 5, x: 6), the x-, y-, z-projections (4, 3,
    2) at 2 flops each, and 10 multiplications per Gauss point (weight, mu phi, D grad phi / h^2)."""
    q, b = (3 * n + 2) // 2, n + 1
    fma = 4 * q * b + 5 * q * q * b + 6 * q ** 3 * b + 4 * q ** 3 * b + 3 * q * q * b + 2 * q * b
    return 2 * fma + 10 * q ** 3


def varcoef_apply(tbs, torch, w):
    """Variable-coefficient operator (the operator the paper timed) on the workload's grid, cubic,
    FP32 and FP64: smooth positive diffusion and absorption fields; ALU roofline (scalar FMA rate,
    packed FP32 not used: 256 CUs x 64 lanes x 2 flops x 2.4 GHz = 78.6 TFLOP/s for FP32 and FP64)."""
    N = w.grid[0] * w.grid[1] * w.grid[2]
    peak = 78.6
    fl = varcoef_flops_per_dof(w.degree)
    ctx = tbs.Context(w.grid, w.degree, w.h, w.tau, w.bc)
    g = torch.Generator(device="cuda")
    g.manual_seed(17)
    out = {"flops_per_dof": fl}
    for dt in ("f32", "f64"):
        td = torch.float32 if dt == "f32" else torch.float64
        c = torch.randn(w.grid[::-1], generator=g, device="cuda", dtype=td)
        d = w.tau * (1.0 + 0.5 * torch.tanh(torch.randn(w.grid[::-1], generator=g, device="cuda", dtype=td)))
        m = 1.0 + 0.5 * torch.tanh(torch.randn(w.grid[::-1], generator=g, device="cuda", dtype=td))
        y = torch.empty_like(c)
        ctx.apply_varcoef(c, d, m, y)
        torch.cuda.synchronize()
        ctx.prof_enable(True)
        reps = 3
        for _ in range(reps):
            ctx.apply_varcoef(c, d, m, y)
        p = ctx.prof_read()
        ctx.prof_enable(False)
        ms, by, cnt = p["varcoef_" + dt]
        t = ms / cnt / 1e3
        tf = fl * N / t / 1e12
        out[dt] = {"GDoF/s": round(N / t / 1e9, 3), "ms": round(ms / cnt, 2), "TFLOP/s": round(tf, 2),
                   "frac_alu": round(tf / peak, 4), "GB/s": round(by / (ms / 1e3) / 1e9, 1)}
        log("varcoef %s: %s" % (dt, out[dt]))
        del c, d, m, y
    out["roofline"] = {"bound": "alu", "achieved": out["f32"]["TFLOP/s"], "peak": peak, "unit": "TFLOP/s",
                       "frac": out["f32"]["frac_alu"], "traffic": None, "kernel": "varcoef_f32",
                       "flops_per_dof": fl, "dofs_per_launch": N}
    out["paper_context"] = ("the paper's on-the-fly cubic operator: 19.1 MDoF/s FP32 at 522^3 on three Radeon "
                            "Vega Frontier Edition GPUs, 3.7 MDoF/s FP64 on a 24-core EPYC 7401P (Sec. 3)")
    del ctx
    return out


def robin_box(tbs, torch, w):
    """Box domain with the Robin / penalty boundary (gamma = 1e-3, the penalty reading of the leg
    example): apply throughput at the workload's size and the first two implicit steps from the
    workload's field, refined FP32 and plain FP64."""
    import workloads
    N = w.grid[0] * w.grid[1] * w.grid[2]
    n, gamma = w.degree, 1e-3
    h = tuple(1.0 / (g - 1 - 2 * (n // 2)) for g in w.grid)
    ctx = tbs.RobinContext(w.grid, n, h, w.tau, gamma)
    u = workloads.gaussian_sum(w.grid, w.bc, w.h, workloads.initial_field_gaussians(w), xp=torch, device="cuda",
                               dtype=torch.float64)
    out = {"gamma": gamma, "h": h[0]}
    for dt in ("f64", "f32"):
        src = u if dt == "f64" else u.float()
        y = torch.empty_like(src)
        for _ in range(2):
            ctx.apply(src, y)
        torch.cuda.synchronize()
        ctx.prof_enable(True)
        for _ in range(10):
            ctx.apply(src, y)
        ms, by, cnt = list(ctx.prof_read().values())[0]
        ctx.prof_enable(False)
        out["apply_" + dt] = {"GDoF/s": round(N / (ms / cnt / 1e3) / 1e9, 1), "ms": round(ms / cnt, 4),
                              "frac_hbm": round(by / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4)}
        del y
    for name, prec in (("refined_fp32", tbs.PREC_MIXED), ("plain_fp64_cg", tbs.PREC_FP64)):
        ctx.set_opts()
        ctx.ensure_workspace(tbs.PREC_FP64)
        ua, ub = u.clone(), torch.empty_like(u)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        its, rr = [], []
        for _ in range(2):
            st = ctx.timestep(ua, None, ub, prec, w.rtol, 5000)
            its.append(st["iters"])
            rr.append(st["rel_res_fp64"])
            ua, ub = ub, ua
        torch.cuda.synchronize()
        out[name] = {"s_per_step": round((time.perf_counter() - t0) / 2, 4), "iters": its, "rel_res_fp64_max": max(rr)}
        del ua, ub
    log("robin: %s" % out)
    del ctx, u
    return out


def degree_sweep(tbs, torch):
    """FP32 apply on the anisotropic periodic 1024 x 512 x 256 grid for quadratic, cubic and
    quintic splines (5, 7, 11 taps per 1-D pass), seeded N(0,1) field."""
    import workloads
    w = workloads.HEAT_1024x512x256_PERIODIC
    N = w.grid[0] * w.grid[1] * w.grid[2]
    g = torch.Generator(device="cuda")
    g.manual_seed(4)
    u = torch.randn(w.grid[::-1], generator=g, device="cuda", dtype=torch.float32)
    y = torch.empty_like(u)
    out = {}
    for n in (2, 3, 5):
        ctx = tbs.Context(w.grid, n, w.h, w.tau, w.bc)
        ctx.ensure_workspace(-1)
        for _ in range(2):
            ctx.apply(u, y)
        torch.cuda.synchronize()
        ctx.prof_enable(True)
        for _ in range(20):
            ctx.apply(u, y)
        ms, by, cnt = list(ctx.prof_read().values())[0]
        ctx.prof_enable(False)
        gbs = by / (ms / 1e3) / 1e9
        out["n%d" % n] = {"taps": 2 * n + 1, "GDoF/s": round(N / (ms / cnt / 1e3) / 1e9, 1), "GB/s": round(gbs, 1),
                          "frac_hbm": round(gbs / HBM_PEAK_GBS, 4), "ms": round(ms / cnt, 4)}
        log("degree sweep n=%d: %s" % (n, out["n%d" % n]))
        del ctx
    out["grid"] = list(w.grid)
    out["bc"] = w.bc
    return out


def graph_cg(tbs, torch):
    """The 32^3 periodic FP64 CG solve (rtol 1e-10) eagerly with host convergence polls, and the
    same number of iterations captured into a HIP graph (poll_every = 0) and replayed: a
    launch-bound solve where the graph removes the host round trips."""
    import workloads
    w = workloads.HEAT_32_PERIODIC
    g = torch.Generator(device="cpu").manual_seed(w.seed)
    b = torch.randn(w.grid[::-1], dtype=torch.float64, generator=g).cuda()
    x = torch.zeros_like(b)
    eager = tbs.Context(w.grid, w.degree, w.h, w.tau, w.bc)
    eager.ensure_workspace(tbs.PREC_FP64)
    reps = 20
    eager.cg_begin(b, x, w.rtol)
    _, iters = eager.cg_step(1000)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        x.zero_()
        eager.cg_begin(b, x, w.rtol)
        eager.cg_step(1000)
    torch.cuda.synchronize()
    t_eager = (time.perf_counter() - t0) / reps
    side = torch.cuda.Stream()
    cap = tbs.Context(w.grid, w.degree, w.h, w.tau, w.bc, stream=side)
    cap.set_opts(poll_every=0)
    cap.ensure_workspace(tbs.PREC_FP64)
    graph = torch.cuda.CUDAGraph()
    torch.cuda.synchronize()
    with torch.cuda.graph(graph, stream=side):
        x.zero_()  # a fill kernel in the graph: every replay solves from x = 0
        cap.cg_begin(b, x, w.rtol)
        cap.cg_step(iters, sync=False)
    torch.cuda.synchronize()
    graph.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        graph.replay()
    torch.cuda.synchronize()
    t_graph = (time.perf_counter() - t0) / reps
    r = {"grid": list(w.grid), "iters": iters, "eager_ms_per_solve": round(t_eager * 1e3, 3),
         "graph_ms_per_solve": round(t_graph * 1e3, 3)}
    log("graph cg: %s" % r)
    del eager, cap, graph
    return {"cg_graph_32": r}


def workload_steps(tbs, torch):
    """The other step workloads: 256^3 Dirichlet with a Gaussian source (10 steps, plain FP64 CG
    vs refined FP32; the arrays fit the 256 MB Infinity Cache, so this is a latency figure), and
    the 1024 x 512 x 256 periodic grid for degrees 2, 3, 5 (20 refined FP32 steps each, with the
    conservation of sum u that a periodic grid without source has)."""
    import numpy as np

    import workloads
    out = {}
    w = workloads.HEAT_256_DIRICHLET
    ctx = tbs.Context(w.grid, w.degree, w.h, w.tau, w.bc)
    ctx.set_opts()
    u = torch.from_numpy(workloads.uniform_field(w.grid[::-1], w.seed)).cuda()
    t = torch.empty_like(u)
    for _ in range(w.smooth_passes):
        ctx.rhs(u, None, t)
        u, t = t, u
    q = workloads.gaussian_sum(w.grid, w.bc, w.h, workloads.source_256(w.seed), xp=torch, device="cuda",
                               dtype=torch.float64)
    r256 = {}
    for name, prec in (("plain_fp64_cg", tbs.PREC_FP64), ("refined_fp32", tbs.PREC_MIXED)):
        ctx.ensure_workspace(prec)
        ua, ub = u.clone(), torch.empty_like(u)
        ctx.timestep(ua, q, ub, prec, w.rtol, 5000)  # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        its, rr = [], []
        for _ in range(w.steps):
            st = ctx.timestep(ua, q, ub, prec, w.rtol, 5000)
            its.append(st["iters"])
            rr.append(st["rel_res_fp64"])
            ua, ub = ub, ua
        torch.cuda.synchronize()
        r256[name] = {"s_per_step": round((time.perf_counter() - t0) / w.steps, 5), "iters": its,
                      "rel_res_fp64_max": max(rr)}
    out["heat256_dirichlet_10_steps"] = r256
    log("heat256: %s" % r256)
    del ctx, u, t, q
    w = workloads.HEAT_1024x512x256_PERIODIC
    g = torch.Generator(device="cuda")
    g.manual_seed(w.seed)
    u0 = torch.randn(w.grid[::-1], generator=g, device="cuda", dtype=torch.float64)
    r4 = {}
    for n in w.degrees:
        ctx = tbs.Context(w.grid, n, w.h, w.tau, w.bc)
        ctx.set_opts()
        ctx.ensure_workspace(tbs.PREC_MIXED)
        ua, ub = u0.clone(), torch.empty_like(u0)
        for _ in range(w.smooth_passes):
            ctx.rhs(ua, None, ub)
            ua, ub = ub, ua
        s0, a0 = float(ua.sum()), float(ua.abs().sum())
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        its, rr = [], []
        for _ in range(w.steps):
            st = ctx.timestep(ua, None, ub, tbs.PREC_MIXED, w.rtol, 5000)
            its.append(st["iters"])
            rr.append(st["rel_res_fp64"])
            ua, ub = ub, ua
        torch.cuda.synchronize()
        r4["n%d" % n] = {"s_per_step": round((time.perf_counter() - t0) / w.steps, 5),
                         "iters_first_last": [its[0], its[-1]], "rel_res_fp64_max": max(rr),
                         "sum_u_drift_rel": abs(float(ua.sum()) - s0) / a0}
        del ctx
    out["heat1024x512x256_periodic_20_steps"] = r4
    log("heat1024x512x256: %s" % r4)
    return out


def transforms(tbs, torch, w, u0):
    """Indirect transform (evaluation at the nodes, FP64) and direct transform (FP64 CG on the
    evaluation operator to 1e-12, started from the samples) of the workload's field, cubic."""
    N = w.grid[0] * w.grid[1] * w.grid[2]
    t = tbs.Transform(w.grid, w.degree, w.bc)
    t.ensure_workspace(tbs.PREC_FP64)
    s = torch.empty_like(u0)
    for _ in range(2):
        t.eval(u0, s)
    torch.cuda.synchronize()
    t.prof_enable(True)
    for _ in range(10):
        t.eval(u0, s)
    ms, by, cnt = list(t.prof_read().values())[0]
    t.prof_enable(False)
    c = s.clone()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    it, rel = t.interp(s, c, rtol=1e-12, max_iter=500)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    err = float(torch.linalg.vector_norm(c - u0) / torch.linalg.vector_norm(u0))
    out = {"eval_f64": {"GDoF/s": round(N / (ms / cnt / 1e3) / 1e9, 1),
                        "frac_hbm": round(by / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4), "ms": round(ms / cnt, 4)},
           "interp_f64": {"s": round(dt, 4), "iters": it, "rel_res": rel, "rel_err_vs_coefficients": err}}
    log("transforms: %s" % out)
    del t, s, c
    return out


def _slab_apply(job):
    """One oracle apply of a z-slab of the workload's field (host worker process; no GPU)."""
    import numpy as np

    import workloads
    from oracle import operator as op
    grid, bc, h, tau, n, params, z0, planes = job
    sub = (grid[0], grid[1], planes + 2 * n)
    shifted = np.array(params, copy=True)
    shifted[:, 4] = params[:, 4] - (z0 - n) * h[2]  # the slab's own coordinates: shift the centres
    u = workloads.gaussian_sum(sub, bc, h, shifted)
    t0 = time.perf_counter()
    op.apply(u, n, h, tau, bc)
    return time.perf_counter() - t0


def cpu_baseline(w, params, allsteps, sp):
    """The FP64 oracle's apply on z-slabs of the same field on the host: one slab in this process
    (one thread), then one slab per worker process on all host cores of the box's share at once;
    scaled to the implicit-step throughput with the plain FP64 CG iteration count the GPU needed
    over the same timed steps (else over the first two steps)."""
    import multiprocessing

    import numpy as np

    n, planes = w.degree, 12
    job = (w.grid, w.bc, w.h, w.tau, n, np.asarray(params), w.grid[2] // 2, planes)
    dofs = w.grid[0] * w.grid[1] * planes  # interior planes of a slab are exact
    t1 = _slab_apply(job)
    nproc = max(1, min(os.cpu_count() or 1, 16))
    jobs = [(w.grid, w.bc, w.h, w.tau, n, np.asarray(params), n + k * planes, planes) for k in range(nproc)]
    # fresh interpreters (spawn): the workers import numpy and the oracle only, never the GPU runtime
    with multiprocessing.get_context("spawn").Pool(nproc) as pool:
        pool.map(_slab_apply, jobs[:1])  # start-up
        t0 = time.perf_counter()
        pool.map(_slab_apply, jobs)
        wall = time.perf_counter() - t0
    per_dof_1 = t1 / dofs
    per_dof_all = wall / (dofs * nproc)
    if "plain_fp64_cg" in allsteps:
        it = allsteps["plain_fp64_cg"]["iters_total"] / float(allsteps["plain_fp64_cg"]["steps"])
    elif "plain_fp64_cg" in sp:
        it = float(np.mean(sp["plain_fp64_cg"]["iters"]))
    else:
        it = 40.0
    applies = it + 3  # CG applies + rhs + initial and final residual
    return {"value": round(1.0 / (per_dof_all * applies) / 1e9, 8), "unit": "GDoF/s", "cores": nproc,
            "kind": "oracle",
            "sample": "numpy FP64 oracle apply of 928x928x18 z-slabs (12 interior planes each) of the 928^3 field, "
                      "one slab per worker process on %d host cores at once: %.2f s wall, %.3g s per DoF-apply "
                      "(one thread: %.2f s, %.3g s per DoF-apply); step rate = 1/(per-DoF apply time x %.1f "
                      "applies per plain-CG step, the GPU's mean plain FP64 CG iteration count over the "
                      "timed steps + 3); host reports %d cores"
                      % (nproc, wall, per_dof_all, t1, per_dof_1, applies, os.cpu_count() or 0),
            "apply_MDoF_per_s": round(dofs * nproc / wall / 1e6, 3),
            "apply_MDoF_per_s_one_thread": round(dofs / t1 / 1e6, 3),
            "value_one_thread": round(1.0 / (per_dof_1 * applies) / 1e9, 8)}


if __name__ == "__main__":
    main()
