"""Kernel workload for rocprofv3: one calibration copy and a few PCG solves.

    rocprofv3 --kernel-trace --stats -d OUT -o run -- python3 -m paper_1809_10026_amd.kernel_profile
    rocprofv3 --pmc FETCH_SIZE -d OUT -o run -- python3 -m paper_1809_10026_amd.kernel_profile
    rocprofv3 --pmc WRITE_SIZE -d OUT -o run -- python3 -m paper_1809_10026_amd.kernel_profile

The calibration kernel is an elementwise multiply that reads one 256 MiB
FP64 buffer and writes another (a plain copy of known size, launched as a
kernel rather than a DMA-engine copy); its FETCH_SIZE and WRITE_SIZE readings
give the factors that turn the counters into HBM bytes.  Then the d = 3,
p = 4, 48-element workload (ndof 6,375,000) is solved with the BF16x3 FD
preconditioner (the benchmark's headline mode) ``--solves`` times.

With ``--batch`` the workload is instead the batched solve of 256 uneven
d = 2 problems (n_el per direction uniform on 16..96, p uniform on {2..5},
kappa log-uniform on [0.1, 10], right-hand sides U[-1, 1] with seeds
20180927 + i, rtol 1e-8, FP64 FD), solved ``--solves`` times:

    rocprofv3 --kernel-trace --stats -d OUT -o run -- python3 -m paper_1809_10026_amd.kernel_profile --batch

With ``--mapped`` it is, after the calibration copy, the rotated quarter
annulus of Table 2 at n_sub = 32, p = 2 (ndof 1,081,344): setup (stencil
assembly on the device) and ``--solves`` PCG solves to 1e-8 with P^G and
FP64 FD, right-hand side U[-1, 1] (seed 1):

    rocprofv3 --kernel-trace --stats -d OUT -o run -- python3 -m paper_1809_10026_amd.kernel_profile --mapped

With ``--side`` it is, after the calibration copy, ``--solves`` general
liftings (stls_lift_apply) at the benchmark shape (boundary coefficients
U[-1, 1] on the 52^4 full space, seed 1814) and as many error-norm
evaluations of the d = 2, p = 3, 64-element workload (a solution of a
U[-1, 1] right-hand side, seed 1809, against sin(pi x) sin(pi y) sin(pi t)).
"""
from __future__ import annotations

import argparse
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

CALIB_BYTES = 256 * 1024 * 1024


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--solves", type=int, default=2)
    ap.add_argument("--mode", default="bf16x3", choices=["fp64", "fp32", "bf16x3"])
    ap.add_argument("--batch", action="store_true", help="the 256-problem batched solve instead")
    ap.add_argument("--mapped", action="store_true", help="the rotated quarter annulus with P^G instead")
    ap.add_argument("--side", action="store_true", help="general lifting and error norms instead")
    args = ap.parse_args()
    import torch

    import paper_1809_10026_amd as stls
    from stls_inputs import CONFIGS, problem_knots, uniform_pm1

    if args.batch:
        return batch(stls, torch, args.solves)

    src = torch.ones(CALIB_BYTES // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        torch.mul(src, 1.0, out=dst)
    torch.cuda.synchronize()
    print(f"[kernel_profile] calibration copy: {CALIB_BYTES} bytes read and written per launch", flush=True)
    del src, dst
    if args.mapped:
        return mapped(stls, torch, args.solves)
    if args.side:
        return side(stls, torch, args.solves)

    cfg = CONFIGS["d3_p4_nel48"]
    S = stls.Solver(*problem_knots(cfg["d"], cfg["n_el"], cfg["p"]))
    S.set_fd_precision({"fp64": stls.STLS_FD_FP64, "fp32": stls.STLS_FD_FP32, "bf16x3": stls.STLS_FD_BF16X3}[args.mode])
    b = torch.as_tensor(uniform_pm1(S.ndof, cfg["seed"])).cuda()
    x = torch.empty_like(b)
    for i in range(args.solves):
        _, it, rel = S.solve(b, cfg["rtol"], 200, out=x)
        torch.cuda.synchronize()
        print(f"[kernel_profile] solve {i}: {it} iterations, relres {rel:.2e}", flush=True)


def batch(stls, torch, solves):
    import numpy as np

    from stls_inputs import batch_params, batch_problem_knots, uniform_pm1
    nel, p, kappa = batch_params()
    B = stls.Batch([(*batch_problem_knots(nel[i], p[i]), float(kappa[i])) for i in range(len(p))])
    off = B.offsets
    b = torch.as_tensor(np.concatenate([uniform_pm1(off[i + 1] - off[i], 20180927 + i)
                                        for i in range(len(p))])).cuda()
    for i in range(solves):
        _, its, rels = B.solve(b, 1e-8, 500)
        torch.cuda.synchronize()
        print(f"[kernel_profile] batch solve {i}: {max(its)} iterations, max relres {max(rels):.2e}", flush=True)


def mapped(stls, torch, solves, n_sub=32, p=2):
    from stls_inputs import problem_knots, uniform_pm1
    knots, degs = problem_knots(3, n_sub, p)
    S = stls.Solver(knots, degs, geometry=stls.STLS_GEOM_ROTATED_QUARTER_ANNULUS, prec=stls.STLS_PREC_GEOMETRY)
    b = torch.as_tensor(uniform_pm1(S.ndof, 1)).cuda()
    x = torch.empty_like(b)
    for i in range(solves):
        _, it, rel = S.solve(b, 1e-8, 3000, out=x)
        torch.cuda.synchronize()
        print(f"[kernel_profile] mapped solve {i}: {it} iterations, relres {rel:.2e}", flush=True)


def side(stls, torch, reps):
    import numpy as np

    from stls_inputs import CONFIGS, problem_knots, uniform_pm1
    cfg = CONFIGS["d3_p4_nel48"]
    S = stls.Solver(*problem_knots(cfg["d"], cfg["n_el"], cfg["p"]))
    ub = torch.as_tensor(uniform_pm1(S.forcing_shape[1], 1814)).cuda()
    F = torch.zeros(S.ndof, dtype=torch.float64, device="cuda")
    for i in range(reps):
        S.lift_apply(ub, F)
        torch.cuda.synchronize()
        print(f"[kernel_profile] general lifting {i}", flush=True)
    S.close()
    c = CONFIGS["d2_p3_nel64"]
    S = stls.Solver(*problem_knots(c["d"], c["n_el"], c["p"]))
    b = torch.as_tensor(uniform_pm1(S.ndof, c["seed"])).cuda()
    x, _, _ = S.solve(b, c["rtol"], 300)
    pi = np.pi
    fac = [[np.stack([np.sin(pi * q), pi * np.cos(pi * q), -pi * pi * np.sin(pi * q)])
            for q in (S.norm_points(k)[0] for k in range(c["d"] + 1))]]
    for i in range(reps):
        r = S.error_norms(x, fac)
        print(f"[kernel_profile] error norms {i}: {r}", flush=True)


if __name__ == "__main__":
    main()
