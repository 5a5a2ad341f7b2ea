#!/usr/bin/env python3
"""Benchmark: FD-preconditioned space-time PCG on one MI355X.

One step = one PCG solve of A u = F to ||r||/||b|| <= 1e-8 from u = 0 (all
hot-path rows: FD preconditioner applications, matrix-free matvecs, vector
updates and dot products), on the 3-D-space workload: unit cube x (0,1),
p = 4 (C^3) splines, 48 elements per direction, ndof = 50^3 * 51 = 6,375,000,
right-hand side i.i.d. uniform[-1,1] (seed 10026), inputs resident in HBM.

The headline value is the fastest of the mixed-precision solves (FD n-mode
products in FP32, in BF16x3 split products, or asymmetric: FP32 forward and
FP64 backward products, on MFMA inside the FP64 PCG); the FP64-plain solve, per-precision FD application rates and MFMA
fractions, the matvec rate, errors against the FP64 oracle's own solution,
the roofline of the dominant kernel (HIP-event durations measured on the
solver's stream) and the oracle timed on the host cores are printed in the
same JSON line.  Beside it, each with the oracle timed on the host: the
diagonally scaled preconditioner, GPU error norms, the batched solve,
lifting, the mapped domain (Table 2's rotated quarter annulus, P and P^G,
the mapped matvec's roofline) and the adjoint gradient of the misfit.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "FD-prec DOF/s + PCG time-to-1e-8 residual, mixed vs FP64 plain, 1 GPU"
PEAK = {"hbm_GBs": 8000.0, "fp64_TF": 78.6, "fp32_TF": 157.3, "bf16_TF": 2500.0}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# Algorithmic work per unknown (DOF) of each step of one PCG iteration
# (the minimum any implementation must move or compute):
#   FD apply   read r, write s (FP64): 16 B; 4 (d n_s + n_t) flops (§4.5)
#   matvec     read x, write y (FP64): 16 B
STEP_BYTES_PER_DOF = {"fd": 16.0, "matvec": 16.0}
# The kernels of each step (profiling classes of the library).
STEPS = {"matvec": ("mv_inner1", "mv_inner2", "mv_outer"),
         "fd": ("fd_slab_fwd", "fd_slab_bwd", "fd_space", "fd_time")}
# Bytes each kernel of the implementation moves per DOF (every stream read or
# written once).  FD: five passes (FP32 intermediates in the mixed modes,
# FP64 in the FP64 mode).
def impl_bytes(cls, mode):
    w = 8.0 if mode == "fp64" else 4.0
    return {"fd_slab_fwd": 8.0 + w,         # r in, intermediate out
            "fd_slab_bwd": w + 16.0,        # intermediate in, s out, r in for r . s
            "fd_space": 2 * w, "fd_time": 2 * w,
            "mv_inner2": 32.0,              # x in, A, B, C out
            "mv_inner1": 32.0,
            "mv_outer": 40.0,               # A, B, C and the dot operand in, y out
            "vec_xr": 48.0,                 # x, r, p, q in; x, r out
            "vec_p": 24.0}.get(cls)         # z, p in; p out


def measured_traffic(classes):
    """HBM bytes per launch summed over ``classes`` from the committed counter
    summary, if it was taken on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    from paper_1809_10026_amd.profile_summary import source_hash
    with open(path) as f:
        data = json.load(f)
    if data.get("source_sha256") != source_hash():
        return None
    tot = 0.0
    for cls in classes:
        c = data.get("classes", {}).get(cls)
        if c is None:
            return None
        tot += c["fetch_bytes"] + c["write_bytes"]
    return tot


def kernel_table(prof, mode, N):
    """Per-class launches, durations and HBM rates (implementation bytes)."""
    five_pass = prof.get("fd_slab_fwd", (0, 0.0))[0] > 0
    out = []
    for cls, (launches, ms) in prof.items():
        if launches == 0:
            continue
        avg_s = ms / launches / 1e3
        e = dict(kernel=cls, launches=launches, total_ms=round(ms, 4), avg_us=round(avg_s * 1e6, 3))
        ib = impl_bytes(cls, mode)
        if ib is not None and (five_pass or not cls.startswith("fd_")):
            e.update(bytes_per_launch=ib * N, GBs=round(ib * N / avg_s / 1e9, 1),
                     hbm_frac=round(ib * N / avg_s / 1e9 / PEAK["hbm_GBs"], 4))
        out.append(e)
    out.sort(key=lambda e: -e["total_ms"])
    return out


def dominant_roofline(table, prof, mode, N):
    """Roofline of the kernel with the largest total time in the headline
    solve.  A kernel that is one stage of a multi-kernel step (the matvec's
    two stages, the FD's passes) is priced as that step: the step's
    algorithmic bytes over the summed average durations of its kernels per
    application."""
    dom = table[0]["kernel"]
    step = next((st for st, cl in STEPS.items() if dom in cl), None)
    if step is None:
        e = table[0]
        ib = impl_bytes(dom, mode)
        avg_s = e["avg_us"] * 1e-6
        tr = measured_traffic([dom])
        return dict(kernel=dom, bound="hbm", achieved=round(ib * N / avg_s / 1e9, 3), peak=PEAK["hbm_GBs"],
                    unit="GB/s", frac=round(ib * N / avg_s / 1e9 / PEAK["hbm_GBs"], 4),
                    traffic=None if tr is None else round(tr / 1e6, 3), traffic_unit="MB per launch",
                    avg_us=e["avg_us"])
    members = [c for c in STEPS[step] if prof.get(c, (0, 0.0))[0] > 0]
    # launches of the step = launches of its first-stage kernel; durations per application
    napp = max(prof[c][0] for c in members)
    per_app = {c: prof[c][1] / 1e3 / napp for c in members}
    t = sum(per_app.values())
    alg = STEP_BYTES_PER_DOF[step] * N
    impl = sum((impl_bytes(c, mode) or 0.0) * prof[c][0] / napp for c in members) * N
    tr = measured_traffic_per_app(members, prof, napp)
    return dict(kernel=f"{step}: " + " + ".join(members) + f" (dominant: {dom})", bound="hbm",
                achieved=round(alg / t / 1e9, 3), peak=PEAK["hbm_GBs"], unit="GB/s",
                frac=round(alg / t / 1e9 / PEAK["hbm_GBs"], 4),
                traffic=None if tr is None else round(tr / 1e6, 3), traffic_unit="MB per application",
                algorithmic_MB_per_launch=round(alg / 1e6, 3), avg_us=round(t * 1e6, 3),
                impl_MB_per_launch=round(impl / 1e6, 3), impl_achieved=round(impl / t / 1e9, 3),
                impl_frac=round(impl / t / 1e9 / PEAK["hbm_GBs"], 4),
                stage_us={c: round(v * 1e6, 3) for c, v in per_app.items()})


def measured_traffic_per_app(members, prof, napp):
    """Counter traffic of one application of a multi-kernel step."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    from paper_1809_10026_amd.profile_summary import source_hash
    with open(path) as f:
        data = json.load(f)
    if data.get("source_sha256") != source_hash():
        return None
    tot = 0.0
    for c in members:
        e = data["classes"].get(c)
        if e is None:
            return None
        tot += (e["fetch_bytes"] + e["write_bytes"]) * prof[c][0] / napp
    return tot


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--maxit", type=int, default=200)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the solver runs on a single GPU (sharding across GPUs is a "
              "design note, not implemented); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1809_10026_amd as stls
    from stls_inputs import CONFIGS, problem_knots, uniform_pm1

    cfg = CONFIGS["d3_p4_nel48"]
    d, nel, p, rtol = cfg["d"], cfg["n_el"], cfg["p"], cfg["rtol"]
    knots, degs = problem_knots(d, nel, p)
    torch.cuda.init()
    t0 = time.perf_counter()
    S = stls.Solver(knots, degs)
    setup_s = time.perf_counter() - t0
    N, shape = S.ndof, S.shape
    ns = N // shape[d]
    log(f"setup {setup_s:.3f}s ndof={N} shape={shape}")
    b = torch.as_tensor(uniform_pm1(N, cfg["seed"])).cuda()
    x = torch.empty_like(b)
    z = torch.empty_like(b)

    def timed_solves(mode, steps, warmup, profile):
        S.set_fd_precision(mode)
        for _ in range(warmup):
            S.solve(b, rtol, args.maxit, out=x)
        S.profile_reset()
        S.profiling(profile)
        torch.cuda.synchronize()
        t = time.perf_counter()
        its = []
        for _ in range(steps):
            _, it, rel = S.solve(b, rtol, args.maxit, out=x)
            its.append(it)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t) / steps
        prof = S.profile()
        S.profiling(False)
        return dt, its[-1], rel, prof

    def fd_rate(mode, reps=20):
        S.set_fd_precision(mode)
        for _ in range(3):
            S.prec_apply(b, out=z)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            S.prec_apply(b, out=z)
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / reps

    def true_relres(xs):
        r = b - S.matvec(xs)
        return float(torch.linalg.norm(r) / torch.linalg.norm(b))

    modes = {"fp64": stls.STLS_FD_FP64, "fp32": stls.STLS_FD_FP32, "bf16x3": stls.STLS_FD_BF16X3,
             "asym": stls.STLS_FD_ASYM}
    mixed_modes = ("fp32", "bf16x3", "asym")
    res = {}
    sol = {}
    # timed region per precision (no profiling: events would add host work per launch)
    for name, mode in modes.items():
        dt, it, rel, _ = timed_solves(mode, args.steps, args.warmup, profile=False)
        sol[name] = x.clone()
        res[name] = dict(time_s=dt, iters=it, relres=rel, true_relres=true_relres(x))
        log(f"{name}: solve {dt*1e3:.3f} ms, {it} its, relres {rel:.2e}, true {res[name]['true_relres']:.2e}")
    mixed = min(mixed_modes, key=lambda m: res[m]["time_s"])
    log(f"headline mixed mode: {mixed}")
    # the same steps again with HIP events around every launch on the solver's
    # stream: per-kernel durations (every mode)
    for name, mode in modes.items():
        dt_prof, _, _, prof = timed_solves(mode, args.steps, 0, profile=True)
        res[name]["prof"] = prof
        res[name]["prof_step_s"] = dt_prof
        log(f"{name}: profiled repetition {dt_prof*1e3:.3f} ms/step")
    for name, mode in modes.items():
        res[name]["fd_apply_s"] = fd_rate(mode)
        log(f"{name}: FD apply {res[name]['fd_apply_s']*1e6:.1f} us")
    # matvec rate
    for _ in range(3):
        S.matvec(b, out=z)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(20):
        S.matvec(b, out=z)
    torch.cuda.synchronize()
    mv_s = (time.perf_counter() - t) / 20
    err_vs_fp64 = {m: float(torch.linalg.norm(sol[m] - sol["fp64"]) / torch.linalg.norm(sol["fp64"]))
                   for m in mixed_modes}
    # the diagonally scaled preconditioner D^-1/2 P^-1 D^-1/2 (§4.4), same solves
    scaled = {}
    S.set_fd_scaling(True)
    for name in ("fp64", "bf16x3"):
        dt, it, rel, _ = timed_solves(modes[name], args.steps, args.warmup, profile=False)
        scaled[name] = dict(time_to_tol_s=dt, iters=it, relres=rel, true_relres=true_relres(x),
                            err_vs_fp64_solution=float(torch.linalg.norm(x - sol["fp64"]) / torch.linalg.norm(sol["fp64"])),
                            fd_prec_dof_per_s=N / fd_rate(modes[name]))
        log(f"{name} scaled: solve {dt*1e3:.3f} ms, {it} its, true {scaled[name]['true_relres']:.2e}")
    S.set_fd_precision(modes["fp64"])
    scaled_apply = S.prec_apply(b).cpu().numpy()  # for the oracle's scaled FD apply beside it
    S.set_fd_scaling(False)

    kernels = {m: kernel_table(res[m]["prof"], m, N) for m in modes}
    roofline = dominant_roofline(kernels[mixed], res[mixed]["prof"], mixed, N)
    # FD n-mode products against the MFMA peak of their arithmetic: useful
    # flops 4 (d n_s + n_t) N per application (§4.5), x3 for the three bf16
    # products of the split form
    fd_flops = 4.0 * (sum(shape[:d]) + shape[d]) * N
    fd_mfma = {}
    for m, peak, mult in (("fp64", PEAK["fp64_TF"], 1), ("fp32", PEAK["fp32_TF"], 1), ("bf16x3", PEAK["bf16_TF"], 3)):
        tf = mult * fd_flops / res[m]["fd_apply_s"] / 1e12
        fd_mfma[m] = dict(useful_TFLOPs=round(tf, 3), peak_TFLOPs=peak, frac=round(tf / peak, 4),
                          flops_per_apply=mult * fd_flops, apply_us=round(res[m]["fd_apply_s"] * 1e6, 2))

    err_norms = gpu_error_norms(stls, torch)
    batch = gpu_batch(stls, torch)
    lifting = gpu_lifting(stls, torch, knots, degs)
    geometry = gpu_geometry(stls, torch)
    gradient = gpu_gradient(stls, torch)

    cpu = None
    err_vs_oracle = None
    if not args.no_cpu_baseline:
        cpu, xo = cpu_baseline(knots, degs, b.cpu().numpy(), rtol, N)
        import numpy as np
        err_vs_oracle = {}
        for m in modes:
            xs = sol[m].cpu().numpy()
            err_vs_oracle[m] = dict(rel_l2=float(np.linalg.norm(xs - xo) / np.linalg.norm(xo)),
                                    max_abs=float(np.abs(xs - xo).max()), max_abs_oracle=float(np.abs(xo).max()))
            log(f"{m}: error vs oracle solution {err_vs_oracle[m]['rel_l2']:.2e} (relative 2-norm)")
        err_norms["oracle_cpu"] = cpu_error_norms()
        lifting["oracle_cpu"] = cpu_lifting(knots, degs)
        geometry["oracle_cpu"] = cpu_mapped_geometry(geometry)
        gradient["oracle_cpu"] = cpu_gradient(gradient)
        batch["oracle_cpu"] = cpu_batch(batch)
        scaled["oracle_cpu"] = cpu_scaled_apply(knots, degs, b.cpu().numpy(), scaled_apply, scaled)
    geometry.get("small", {}).pop("solution", None)
    batch.pop("sample", None)
    for key in ("grad_f", "grad_kappa"):
        gradient.pop(key, None)

    t_mixed, t_fp64 = res[mixed]["time_s"], res["fp64"]["time_s"]
    out = {
        "metric": METRIC,
        "value": N / t_mixed,
        "unit": "DOF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t_mixed * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64 (PCG) + " + {"fp32": "f32", "bf16x3": "bf16x3/f32-accumulate",
                                   "asym": "f32 forward / f64 backward"}[mixed] + " (FD n-mode products)",
        "data": "synthetic",
        "config": {"workload": "d=3 unit cube x (0,1), p=4 C^3 splines, 48 elements/dir, ndof=6375000 "
                               "(50^3 x 51), RHS U[-1,1] seed 10026, PCG rtol 1e-8 from x0=0",
                   "ndof": N, "unconstrained_dofs": (nel + p) ** (d + 1), "rtol": rtol},
        "headline_mode": mixed,
        "time_to_tol_s": {m: res[m]["time_s"] for m in modes},
        "speedup_mixed_vs_fp64": t_fp64 / t_mixed,
        "iters": {m: res[m]["iters"] for m in modes},
        "true_relres": {m: res[m]["true_relres"] for m in modes},
        "err_vs_fp64_solution": err_vs_fp64,
        "err_vs_oracle": err_vs_oracle,
        "fd_prec_dof_per_s": {k: N / v["fd_apply_s"] for k, v in res.items()},
        "fd_mfma": fd_mfma,
        "matvec_dof_per_s": N / mv_s,
        "diag_scaled_prec": scaled,
        "error_norms": err_norms,
        "batch": batch,
        "lifting": lifting,
        "mapped_domain": geometry,
        "gradient": gradient,
        "setup_s": setup_s,
        "roofline": roofline,
        "roofline_note": "kernel durations from HIP events recorded around every launch on the solver's "
                         "stream in a repetition of the timed steps (%.3f ms/step with events); achieved = "
                         "algorithmic bytes (16 B per unknown for the matvec and for the FD apply) / duration; "
                         "impl_* = the bytes this implementation's kernels move" % (res[mixed]["prof_step_s"] * 1e3),
        "kernels": kernels[mixed],
        "kernels_fp64": kernels["fp64"],
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def _sin_factors(x):
    import numpy as np
    pi = np.pi
    return np.stack([np.sin(pi * x), pi * np.cos(pi * x), -pi * pi * np.sin(pi * x)])


def gpu_error_norms(stls, torch, reps=3):
    """Error norms (§5.1) on the GPU: V0, L2 and H1 errors of a d = 2, p = 3,
    64-element solution (right-hand side U[-1, 1], seed 1809) against
    u = sin(pi x) sin(pi y) sin(pi t), timed per evaluation."""
    import numpy as np

    from stls_inputs import CONFIGS, problem_knots, uniform_pm1
    c = CONFIGS["d2_p3_nel64"]
    S = stls.Solver(*problem_knots(c["d"], c["n_el"], c["p"]))
    b = torch.as_tensor(uniform_pm1(S.ndof, c["seed"])).cuda()
    x, _, _ = S.solve(b, c["rtol"], 300)
    pts = [S.norm_points(k)[0] for k in range(c["d"] + 1)]
    fac = [[_sin_factors(p) for p in pts]]
    S.error_norms(x, fac)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(reps):
        res = S.error_norms(x, fac)
    dt = (time.perf_counter() - t) / reps
    grid = int(np.prod([len(p) for p in pts]))
    log(f"error norms: {dt*1e3:.1f} ms for {grid} grid points")
    return {"workload": "d=2, p=3, 64 elements/dir (N=278,850), u_h solved from a U[-1,1] RHS (seed 1809), "
                        "exact u = sin(pi x) sin(pi y) sin(pi t), p+3 Gauss points per span",
            "seconds": dt, "grid_points": grid, "fields": 2 * c["d"] + 2, "grid_points_per_s": grid / dt,
            "norms": res}


def gpu_batch(stls, torch, steps=3):
    """Batched PCG (256 uneven d = 2 problems: n_el per direction uniform on
    16..96, p uniform on {2..5}, kappa log-uniform on [0.1, 10], right-hand
    sides U[-1, 1] with seeds 20180927 + i), rtol 1e-8, FP64 FD."""
    import numpy as np

    from stls_inputs import batch_params, batch_problem_knots, uniform_pm1
    nel, p, kappa = batch_params()
    probs = [(*batch_problem_knots(nel[i], p[i]), float(kappa[i])) for i in range(len(p))]
    t = time.perf_counter()
    B = stls.Batch(probs)
    setup_s = time.perf_counter() - t
    off = B.offsets
    b = torch.as_tensor(np.concatenate([uniform_pm1(off[i + 1] - off[i], 20180927 + i)
                                        for i in range(len(probs))])).cuda()
    x = torch.empty_like(b)

    def timed():
        B.solve(b, 1e-8, 500, out=x)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            _, its, rels = B.solve(b, 1e-8, 500, out=x)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps, its, rels

    dt_default, _, _ = timed()
    default_tuning = B.tuning
    # autotuner: work-item shapes and launch geometry timed on this batch (no
    # cache here: the bench always measures)
    t = time.perf_counter()
    B.autotune()
    tune_s = time.perf_counter() - t
    dt, its, rels = timed()
    log(f"batch: {dt*1e3:.1f} ms tuned ({dt_default*1e3:.1f} ms default shapes) for {B.total} unknowns, "
        f"{max(its)} iterations; tuning {B.tuning}")
    nsamp = 8
    return {"workload": "256 independent d=2 problems, n_el per direction U{16..96}, p U{2..5}, "
                        "kappa 10^U(-1,1), RHS U[-1,1] (seeds 20180927+i), rtol 1e-8, FP64 FD",
            "sample": {"problems": nsamp, "offsets": [int(v) for v in off[:nsamp + 1]],
                       "x": x[:int(off[nsamp])].cpu().numpy(), "iters": [int(v) for v in its[:nsamp]]},
            "total_dof": int(B.total), "seconds": dt, "dof_per_s": B.total / dt, "max_iters": int(max(its)),
            "iteration_ms": dt / max(its) * 1e3, "graph_replay": bool(B.graph_used), "setup_s": setup_s,
            "max_relres": float(max(rels)),
            "autotune": {"seconds": tune_s, "tuning": B.tuning, "default_tuning": default_tuning,
                         "default_seconds": dt_default}}


def cpu_scaled_apply(knots, degs, b, gpu_apply, scaled):
    """The oracle's diagonally scaled FD apply (ScaledFD, FP64, host cores)
    on the benchmark's right-hand side, and the error of the GPU's FP64
    scaled apply of the same vector."""
    import numpy as np

    from oracle import fd, system
    P = system.Problem(knots, degs)
    t0 = time.perf_counter()
    SF = fd.ScaledFD(P)
    setup = time.perf_counter() - t0
    t0 = time.perf_counter()
    z = system.vec(SF.apply(b))
    dt = time.perf_counter() - t0
    err = float(np.linalg.norm(gpu_apply - z) / np.linalg.norm(z))
    gpu_s = P.ndof / scaled["fp64"]["fd_prec_dof_per_s"]
    log(f"cpu scaled FD apply: {dt:.2f} s (GPU FP64 {gpu_s*1e6:.0f} us); GPU vs oracle {err:.2e}")
    return {"kind": "oracle", "sample": "one FP64 scaled FD apply of the benchmark right-hand side", "seconds": dt,
            "setup_s": setup, "dof_per_s": P.ndof / dt, "gpu_fp64_vs_oracle_rel_l2": err}


def cpu_batch(batch):
    """The oracle's FD-PCG (FP64, host cores) on the first problems of the
    batch, one after the other: time, rate, and the error of the GPU batch's
    solutions of the same problems."""
    import numpy as np

    from oracle import fd, pcg, system
    from stls_inputs import batch_params, batch_problem_knots, uniform_pm1
    smp = batch.pop("sample")
    nel, p, kappa = batch_params()
    off = smp["offsets"]
    errs, iters, dt = [], [], 0.0
    for i in range(smp["problems"]):
        knots, degs = batch_problem_knots(nel[i], p[i])
        t0 = time.perf_counter()
        P = system.Problem(knots, degs, float(kappa[i]))
        F = fd.FD(P)
        b = uniform_pm1(off[i + 1] - off[i], 20180927 + i)
        xo, info = pcg.pcg(lambda v: system.vec(P.matvec(v)), lambda v: system.vec(F.apply(v)), b, 1e-8, maxit=500)
        dt += time.perf_counter() - t0
        xg = smp["x"][off[i]:off[i + 1]]
        errs.append(float(np.linalg.norm(xg - xo) / np.linalg.norm(xo)))
        iters.append(int(info["iters"]))
    log(f"cpu batch sample: {smp['problems']} problems, {off[-1]} unknowns in {dt:.2f} s; GPU solutions vs oracle "
        f"max {max(errs):.2e}; iterations GPU {smp['iters']} oracle {iters}")
    return {"kind": "oracle", "sample": f"problems 0..{smp['problems'] - 1} of the batch, solved one after the other "
                                        "(setup included)", "unknowns": int(off[-1]), "seconds": dt,
            "dof_per_s": off[-1] / dt, "gpu_vs_oracle_max_rel_l2": max(errs), "iters_oracle": iters,
            "iters_gpu": smp["iters"]}


def gpu_geometry(stls, torch, n_sub=32, p=2, reps=3, mv_reps=50, small=12):
    """Mapped domain (§4.4, §5.2 Table 2): the rotated quarter annulus,
    n_sub = 32, p_s = p_t = 2 (ndof 32^3 x 33 = 1,081,344), right-hand side
    U[-1, 1] (seed 1), PCG to 1e-8 with the parametric P and with the
    geometry-aware P^G (FP64 FD; P^G also with bf16x3 FD).  Setup (stencil
    assembly on the device, Algorithm 2 and the eigendecompositions on the
    host) timed apart.  The mapped matvec is priced with its algorithmic
    bytes: the three stencils read once (3 S n_s doubles, S = (2p+1)^3) plus
    x read and y written.  The same P^G solve at n_sub = 12 is timed beside
    the oracle's (cpu_mapped_geometry)."""
    from stls_inputs import problem_knots, uniform_pm1
    knots, degs = problem_knots(3, n_sub, p)
    out = {"workload": f"rotated quarter annulus, n_sub={n_sub}, p={p}, RHS U[-1,1] seed 1, rtol 1e-8",
           "table2_paper_iterations": {"P": 142, "P^G": 42}}
    for name, prec, mode in (("P", stls.STLS_PREC_PARAMETRIC, stls.STLS_FD_FP64),
                             ("P^G", stls.STLS_PREC_GEOMETRY, stls.STLS_FD_FP64),
                             ("P^G bf16x3", stls.STLS_PREC_GEOMETRY, stls.STLS_FD_BF16X3)):
        torch.cuda.synchronize()
        t = time.perf_counter()
        S = stls.Solver(knots, degs, geometry=stls.STLS_GEOM_ROTATED_QUARTER_ANNULUS, prec=prec)
        torch.cuda.synchronize()
        setup_s = time.perf_counter() - t
        S.set_fd_precision(mode)
        b = torch.as_tensor(uniform_pm1(S.ndof, 1)).cuda()
        x = torch.empty_like(b)
        S.solve(b, 1e-8, 3000, out=x)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            _, it, rel = S.solve(b, 1e-8, 3000, out=x)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t) / reps
        out[name] = {"ndof": S.ndof, "iters": it, "relres": rel, "seconds": dt, "setup_s": setup_s,
                     "dof_per_s": S.ndof / dt}
        log(f"mapped domain {name}: {it} iterations, {dt*1e3:.2f} ms, setup {setup_s:.2f} s")
        if name == "P^G":
            y = torch.empty_like(b)
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
            for fn, key in ((lambda: S.matvec(b, out=y), "matvec_us"), (lambda: S.prec_apply(b, out=y), "prec_apply_us")):
                fn()
                torch.cuda.synchronize()
                ev[0].record()
                for _ in range(mv_reps):
                    fn()
                ev[1].record()
                torch.cuda.synchronize()
                out[name][key] = ev[0].elapsed_time(ev[1]) / mv_reps * 1e3
            n_s = S.ndof // (n_sub + p - 1)
            sten = (2 * p + 1) ** 3
            nbytes = 8 * (3 * sten * n_s + 2 * S.ndof)
            achieved = nbytes / (out[name]["matvec_us"] * 1e-6) / 1e9
            out["matvec_roofline"] = {"kernel": "mapped matvec: mapped_space_kernel + mapped_time_kernel",
                                      "bound": "hbm", "algorithmic_bytes": nbytes, "achieved": round(achieved, 1),
                                      "peak": PEAK["hbm_GBs"], "unit": "GB/s",
                                      "frac": round(achieved / PEAK["hbm_GBs"], 4),
                                      "note": "three stencils of (2p+1)^3 entries per spatial row read once, "
                                              "x read and y written; the kernels move U and V (16 B/DOF each way) "
                                              "and re-read stencil rows once per chunk of time slices"}
            log(f"mapped matvec {out[name]['matvec_us']:.1f} us, P^G apply {out[name]['prec_apply_us']:.1f} us, "
                f"{achieved:.0f} GB/s algorithmic")
        S.close()
    # the same P^G solve at n_sub = small, timed beside the oracle's
    knots_s, degs_s = problem_knots(3, small, p)
    S = stls.Solver(knots_s, degs_s, geometry=stls.STLS_GEOM_ROTATED_QUARTER_ANNULUS, prec=stls.STLS_PREC_GEOMETRY)
    b = torch.as_tensor(uniform_pm1(S.ndof, 1)).cuda()
    x = torch.empty_like(b)
    S.solve(b, 1e-8, 3000, out=x)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(reps):
        _, it, rel = S.solve(b, 1e-8, 3000, out=x)
    torch.cuda.synchronize()
    out["small"] = {"n_sub": small, "ndof": S.ndof, "iters": it, "seconds": (time.perf_counter() - t) / reps,
                    "solution": x.cpu().numpy()}
    S.close()
    return out


def cpu_mapped_geometry(geometry, p=2):
    """The oracle's P^G-PCG on the rotated quarter annulus at the small n_sub
    of the GPU leg (numpy, host cores): assembly timed apart, the solve to
    1e-8, and the error of the GPU's solution against it."""
    import numpy as np

    from oracle import geometry as geo, pcg as opcg
    from stls_inputs import problem_knots, uniform_pm1
    small = geometry["small"]
    knots, degs = problem_knots(3, small["n_sub"], p)
    t = time.perf_counter()
    MP = geo.MappedProblem(geo.RotatedQuarterAnnulus(), knots, degs)
    pre = geo.GeometryPreconditioner(MP)
    setup = time.perf_counter() - t
    b = uniform_pm1(MP.ndof, 1)
    t = time.perf_counter()
    xo, info = opcg.pcg(MP.matvec, pre.apply, b, 1e-8, maxit=3000)
    dt = time.perf_counter() - t
    xg = small.pop("solution")
    err = float(np.linalg.norm(xg - xo) / np.linalg.norm(xo))
    log(f"cpu mapped P^G solve (n_sub {small['n_sub']}): {info['iters']} iterations, {dt:.2f} s "
        f"(setup {setup:.1f} s); GPU solution error {err:.2e}")
    return {"kind": "oracle", "workload": f"rotated quarter annulus, n_sub={small['n_sub']}, p={p}, P^G, rtol 1e-8",
            "ndof": MP.ndof, "iters": info["iters"], "seconds": dt, "setup_s": setup,
            "gpu_seconds": small["seconds"], "gpu_iters": small["iters"], "gpu_vs_oracle_rel_l2": err}


def gpu_gradient(stls, torch, reps=3, rtol=1e-8):
    """Adjoint gradient of the space-time misfit (cfg 5): d = 2, p = 3, 128
    elements per direction (ndof 2,163,330; forcing coefficients 131^3 in the
    full spline space), kappa = 1, forcing U[-1, 1] (seed 5), target u* the
    solution for a second forcing (seed 6).  One evaluation = load operator,
    PCG solve, misfit with its gradient, adjoint PCG solve, B^T and the kappa
    derivative (autograd.HeatSolve / Misfit), FP64 FD, solves to 1e-8."""
    from paper_1809_10026_amd import autograd as sag
    from stls_inputs import problem_knots, uniform_pm1
    knots, degs = problem_knots(2, 128, 3)
    S = stls.Solver(knots, degs, kappa=1.0)
    _, nf = S.forcing_shape
    fstar = torch.as_tensor(uniform_pm1(nf, 6)).cuda()
    F = S.load_apply(fstar)
    ustar, _, _ = S.solve(F, rtol=rtol)
    f0 = torch.as_tensor(uniform_pm1(nf, 5)).cuda()

    def evaluate():
        f = f0.clone().requires_grad_(True)
        kt = torch.tensor(1.0, dtype=torch.float64, device="cuda", requires_grad=True)
        L = sag.misfit(sag.heat_solve(f, kt, S, rtol=rtol), ustar, S)
        L.backward()
        return float(L), f.grad, float(kt.grad)

    evaluate()
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(reps):
        L, gf, gk = evaluate()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t) / reps
    log(f"gradient (cfg 5): loss {L:.6e}, dL/dkappa {gk:.6e}, {dt*1e3:.2f} ms per evaluation")
    # one more evaluation with HIP events around every launch: time per kernel class
    stls.stls_set_profiling(S.handle, True)
    stls.stls_profile_reset(S.handle)
    evaluate()
    torch.cuda.synchronize()
    split = {k: round(v[1], 3) for k, v in stls.stls_profile(S.handle).items() if v[0]}
    stls.stls_set_profiling(S.handle, False)
    out = {"workload": "d=2, p=3, 128 elements/dir (ndof 2,163,330, forcing 131^3), kappa 1, f U[-1,1] seed 5, "
                       "target u* from seed 6, FP64 FD, PCG rtol 1e-8: loss and its gradient in f and kappa",
           "ndof": S.ndof, "forcing_size": nf, "seconds": dt, "loss": L, "dL_dkappa": gk,
           "solves_per_evaluation": 2, "ms_per_kernel_class": split,
           "note": "diff = the band products of the load operator, its transpose and the kappa derivative "
                   "(generic banded mode-product kernel); the rest is the two PCG solves",
           "grad_f": gf.cpu().numpy(), "grad_kappa": gk}
    S.close()
    return out


def cpu_gradient(gradient):
    """The oracle's loss and gradient on the host cores (oracle FD-PCG as the
    solver, its own target solve), and the error of the GPU's gradient."""
    import numpy as np

    from oracle import fd, grad as ograd, pcg, system
    from stls_inputs import problem_knots, uniform_pm1
    knots, degs = problem_knots(2, 128, 3)
    t0 = time.perf_counter()
    P = system.Problem(knots, degs)
    Fd = fd.FD(P)
    G = ograd.Misfit(P)
    setup = time.perf_counter() - t0

    def solve(b):
        return np.asarray(pcg.pcg(lambda v: system.vec(P.matvec(v)), lambda v: system.vec(Fd.apply(v)), b, 1e-8,
                                  maxit=300)[0])

    m = [len(k) - q - 1 for k, q in zip(knots, degs)]
    nf = int(np.prod(m))
    ustar = solve(G.load_apply(uniform_pm1(nf, 6).reshape(m, order="F")).ravel(order="F"))
    t0 = time.perf_counter()
    L, gf, dk, _ = G.loss_and_grad(uniform_pm1(nf, 5).reshape(m, order="F"), ustar, solve)
    dt = time.perf_counter() - t0
    gfo = np.asarray(gf).ravel(order="F")
    err_f = float(np.linalg.norm(gradient["grad_f"] - gfo) / np.linalg.norm(gfo))
    err_k = float(abs(gradient["grad_kappa"] - dk) / abs(dk))
    log(f"cpu gradient: {dt:.2f} s per evaluation (setup {setup:.1f} s); GPU vs oracle: dL/df {err_f:.2e}, "
        f"dL/dkappa {err_k:.2e}")
    return {"kind": "oracle", "seconds": dt, "setup_s": setup, "loss": L, "dL_dkappa": dk,
            "gpu_vs_oracle_grad_f_rel_l2": err_f, "gpu_vs_oracle_grad_kappa_rel": err_k}


def gpu_lifting(stls, torch, knots, degs, reps=20):
    """Lifting of non-zero initial data (§2) on the benchmark shape: the
    coupling F -= a(u0_h b_1, B_i) (stls_lift_initial) and the assembly of
    the full-time coefficients (stls_lift_combine), u0 U[-1, 1] (seed 1812).
    Algorithmic bytes: read u0, read and write the first p_t time slices of F."""
    from stls_inputs import uniform_pm1
    S = stls.Solver(knots, degs)
    u0 = torch.as_tensor(uniform_pm1(S.ns, 1812)).cuda()
    F = torch.as_tensor(uniform_pm1(S.ndof, 1813)).cuda()
    w = torch.zeros(S.ndof, dtype=torch.float64, device="cuda")
    S.lift_initial(u0, F)
    u = S.lift_combine(u0, w)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(reps):
        S.lift_initial(u0, F)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t) / reps
    t = time.perf_counter()
    for _ in range(reps):
        S.lift_combine(u0, w, out=u)
    torch.cuda.synchronize()
    dc = (time.perf_counter() - t) / reps
    pt = degs[-1]
    nbytes = 8 * S.ns * (1 + 2 * min(pt, S.shape[-1]))
    d = len(knots) - 1
    # general data: u_B over the full space (boundary and initial coefficients)
    nfull = S.forcing_shape[1]
    ub = torch.as_tensor(uniform_pm1(nfull, 1814)).cuda()
    uf = S.lift_embed(ub, w)
    S.lift_apply(ub, F)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(reps):
        S.lift_apply(ub, F)
    torch.cuda.synchronize()
    dg = (time.perf_counter() - t) / reps
    t = time.perf_counter()
    for _ in range(reps):
        S.lift_embed(ub, w, out=uf)
    torch.cuda.synchronize()
    de = (time.perf_counter() - t) / reps
    gterms = 1 + d * d + 2 * d
    log(f"lifting: coupling {dt*1e6:.1f} us, combine {dc*1e6:.1f} us; general {dg*1e6:.1f} us, embed {de*1e6:.1f} us")
    return {"workload": "d=3, p=4, 48 elements/dir: u0 on the 50^3 spatial coefficients, F of 6,375,000; "
                        "general u_B U[-1,1] (seed 1814) on the 52^4 full space",
            "coupling_s": dt, "combine_s": dc, "algorithmic_bytes": nbytes,
            "coupling_GB_per_s": nbytes / dt / 1e9, "kronecker_terms": 1 + d + d * (d - 1) // 2,
            "launches": (1 + d + d * (d - 1) // 2) * (d + 1),
            "general": {"apply_s": dg, "embed_s": de, "kronecker_terms": gterms,
                        "algorithmic_bytes": 8 * nfull + 16 * S.ndof}}


def cpu_lifting(knots, degs):
    """The oracle's coupling (numpy, host cores) on the same shape."""
    from oracle import lift, system
    from stls_inputs import uniform_pm1
    P = system.Problem(knots, degs)
    u0 = uniform_pm1(int(P.ndof // P.shape[-1]), 1812)
    t = time.perf_counter()
    lift.initial_coupling(P, u0)
    dt = time.perf_counter() - t
    log(f"cpu lifting: {dt:.3f} s")
    return {"kind": "oracle", "coupling_s": dt}


def cpu_error_norms(nel=32):
    """The oracle's error norms (numpy, host cores) on the same kind of
    workload at 32 elements per direction (7.1 M grid points)."""
    import numpy as np

    from oracle import norms, system
    from stls_inputs import problem_knots, uniform_pm1
    pi = np.pi
    ex = dict(u=lambda x, y, t: np.sin(pi * x) * np.sin(pi * y) * np.sin(pi * t),
              ut=lambda x, y, t: np.sin(pi * x) * np.sin(pi * y) * pi * np.cos(pi * t),
              lap=lambda x, y, t: -2 * pi * pi * np.sin(pi * x) * np.sin(pi * y) * np.sin(pi * t),
              grad=[lambda x, y, t: pi * np.cos(pi * x) * np.sin(pi * y) * np.sin(pi * t),
                    lambda x, y, t: pi * np.sin(pi * x) * np.cos(pi * y) * np.sin(pi * t)])
    knots, degs = problem_knots(2, nel, 3)
    P = system.Problem(knots, degs)
    u = uniform_pm1(P.ndof, 1809)
    t = time.perf_counter()
    norms.error_norms(system.unvec(u, P.shape), knots, degs, ex)
    dt = time.perf_counter() - t
    grid = (nel * 6) ** 3
    log(f"cpu error norms: {dt:.2f} s for {grid} grid points")
    return {"kind": "oracle", "workload": f"d=2, p=3, {nel} elements/dir", "seconds": dt, "grid_points": grid,
            "grid_points_per_s": grid / dt}


def cpu_baseline(knots, degs, b, rtol, N):
    """The FP64 oracle's own FD-PCG on the host cores: a full solve to rtol
    from x = 0 on every core the BLAS uses (setup included), then one
    iteration's cost on a single thread (the paper's setting).  Returns the
    baseline record and the oracle's solution."""
    import numpy as np

    from oracle import fd, pcg, system
    import threadpoolctl
    threads = max((i.get("num_threads", 1) for i in threadpoolctl.threadpool_info()), default=None)
    log(f"cpu baseline: oracle PCG to {rtol:g} on {threads} threads")
    t0 = time.perf_counter()
    P = system.Problem(knots, degs)
    F = fd.FD(P)
    setup = time.perf_counter() - t0
    t0 = time.perf_counter()
    xo, info = pcg.pcg(lambda v: system.vec(P.matvec(v)), lambda v: system.vec(F.apply(v)), b, rtol, maxit=200)
    t_solve = time.perf_counter() - t0
    log(f"cpu baseline: setup {setup:.2f} s, solve {t_solve:.2f} s, {info['iters']} iterations")
    # one iteration's operator work (matvec + FD apply) on one thread
    with threadpoolctl.threadpool_limits(limits=1):
        t0 = time.perf_counter()
        q = system.vec(P.matvec(b))
        system.vec(F.apply(q))
        t1 = time.perf_counter() - t0
    log(f"cpu baseline: one matvec + FD apply on 1 thread {t1:.2f} s")
    total = setup + t_solve
    return ({"value": N / total, "unit": "DOF/s", "cores": threads or os.cpu_count(), "kind": "oracle",
             "sample": f"one full solve of the numpy FP64 oracle (setup {setup:.1f} s + PCG {t_solve:.1f} s, "
                       f"{info['iters']} iterations to rtol {rtol:g}, x0 = 0) on the same workload and right-hand side",
             "seconds": total, "iters": int(info["iters"]), "seconds_per_iteration": t_solve / max(1, info["iters"]),
             "one_thread": {"cores": 1, "seconds_matvec_plus_fd": t1,
                            "dof_per_s_estimate": N / (setup + t1 * info["iters"]),
                            "note": "one matvec + one FD apply on one BLAS thread, times the iteration count, "
                                    "plus the all-core setup"}},
            np.asarray(xo))


if __name__ == "__main__":
    main()
