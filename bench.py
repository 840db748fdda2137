#!/usr/bin/env python3
"""Benchmark of the FAS heat solver on one MI355X.

Workload: 2D backward-Euler heat steps on a cell-centred 8192^2 grid on [0,1]^2,
h = 1/8192, dt = 1e-4, kappa = 1, homogeneous Neumann BCs; u0 = seeded 64-mode cosine
sum plus uniform(-0.01, 0.01) noise (synthetic).  One step = one solve of
u - dt Lap u = u^n to a relative residual of 1e-10 with V(2,2) X-MCGS cycles down to
4^2, warm-started from u^n.  The plain FP64 solver gives `value` (seconds per step);
the mixed-precision form (FP32 inner cycles inside FP64 defect correction) is timed on
the same steps and reported beside it.

Prints one JSON line.  `roofline` is measured live: HIP events recorded by the library
on its own stream around every finest-level launch inside the timed region.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0  # MI355X HBM3E peak


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10, help="timed heat steps")
    ap.add_argument("--warmup", type=int, default=1, help="untimed heat steps first")
    ap.add_argument("--n", type=int, default=8192, help="cells per axis")
    ap.add_argument("--inner", type=int, default=3, help="FP32 V-cycles per outer correction (mixed form)")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    return ap.parse_args()


def kernel_bytes(s, d):
    """Algorithmic HBM bytes per finest cell of each finest-level kernel class (values
    in bytes; s = bytes per value, c = 2^d children per coarse cell)."""
    c = 2 ** d
    return {
        # one colour phase: half the cells read u and f and write u (3s per full sweep)
        "smooth": 1.5 * s,
        # fused pre-smoothing + residual + restriction: read u, f; write u, u_c, r_c
        "pre": 3 * s + 2 * s / c,
        # fused correction + post-smoothing + norm partials: read u, f, u_c; write u
        "post": 3 * s + s / c,
        # reduction of the per-wave partial sums (a few KB)
        "norm": 0.0,
    }


def cpu_baseline(u0, n, dt, cycles_per_step):
    """The oracle (single thread) on a bounded sample: one V(2,2) cycle of the first
    heat step at full size, scaled to seconds per step by the GPU's cycles per step."""
    import numpy as np

    import oracle

    P = oracle.Problem(n=(n, n), h=1.0 / n, dt=dt, kappa=1.0, bc="neumann", coarsest=4, nuc=2)
    f = np.ascontiguousarray(u0)
    u = f.copy()
    t0 = time.perf_counter()
    oracle.vcycle(P, f, u, 2, 2)
    t_cycle = time.perf_counter() - t0
    return {
        "value": t_cycle * cycles_per_step,
        "unit": "s",
        "cores": 1,
        "kind": "oracle",
        "sample": "one FP64 V(2,2) cycle of step 1 at %d^2 (%.1f s, single thread), times %.2f GPU "
                  "cycles per step" % (n, t_cycle, cycles_per_step),
    }


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only (this solver path is single-GPU); got --gpus %d, WORLD_SIZE %d"
              % (args.gpus, world), file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import fas_inputs
    from paper_2510_11152_amd import Grid, solve_mixed

    n, dt, tol = args.n, 1e-4, 1e-10
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    print("bench: generating %d^2 input" % n, file=sys.stderr, flush=True)
    u0_h = fas_inputs.heat_2d_large(n)
    u0 = torch.from_numpy(u0_h).to(dev)

    g = Grid((n, n), 1.0 / n, dtype=torch.float64, coarsest=4, device=dev)
    rhs = torch.empty_like(u0)

    def step_plain(u):
        rhs.copy_(u)
        st = g.solve(rhs, u, dt, tol=tol, nu1=2, nu2=2)
        if st != 0:
            raise RuntimeError("plain solve did not converge")
        return g.stats()["cycles"]

    # warm-up, then the timed steps
    u = u0.clone()
    for _ in range(args.warmup):
        step_plain(u)
    u = u0.clone()
    g.set(profile=True)
    g.profile(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    cycles = [step_plain(u) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t_plain = (time.perf_counter() - t0) / args.steps
    prof = g.profile(reset=True)
    g.set(profile=False)
    u_plain = u
    print("bench: plain %.4f s/step cycles %s" % (t_plain, cycles), file=sys.stderr, flush=True)

    # roofline of the dominant finest-level kernel class
    kb = kernel_bytes(8, 2)
    dom = max((k for k in prof if kb[k] > 0), key=lambda k: prof[k][1])
    launches, ms = prof[dom]
    avg_s = ms / 1e3 / max(launches, 1)
    achieved = kb[dom] * n * n / avg_s / 1e9
    per_kernel = {k: {"launches": v[0], "avg_us": (v[1] * 1e3 / v[0]) if v[0] else None,
                      "gbs": (kb[k] * n * n / (v[1] / 1e3 / v[0]) / 1e9) if v[0] and kb[k] else None}
                  for k, v in prof.items()}

    result = {
        "metric": "FAS solve s & HBM GB/s, 8192² heat to 1e-10; mixed/batched vs plain FP64",
        "value": t_plain,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t_plain * 1e3,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "2D backward-Euler heat %d^2, h=1/%d, dt=1e-4, kappa=1, Neumann; 64-mode cosine "
                               "+ uniform(-0.01,0.01) noise (seed 1); V(2,2) X-MCGS down to 4^2, relative "
                               "residual 1e-10 per step" % (n, n),
                   "grid": [n, n], "steps_timed": args.steps, "nu1": 2, "nu2": 2, "coarsest": 4, "tol": tol},
        "cycles_per_step": float(np.mean(cycles)),
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": achieved / PEAK_HBM_GBS, "traffic": None},
        "kernels": per_kernel,
    }

    if not args.no_mixed:
        g32 = Grid((n, n), 1.0 / n, dtype=torch.float32, coarsest=4, mixed_inner=True, device=dev)
        outer = []

        def step_mixed(u):
            rhs.copy_(u)
            st = solve_mixed(g, g32, rhs, u, dt, tol=tol, nu1=2, nu2=2, inner=args.inner)
            if st != 0:
                raise RuntimeError("mixed solve did not converge")
            return g.stats()["cycles"]

        u = u0.clone()
        for _ in range(args.warmup):
            step_mixed(u)
        u = u0.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        outer = [step_mixed(u) for _ in range(args.steps)]
        torch.cuda.synchronize()
        t_mixed = (time.perf_counter() - t0) / args.steps
        diff = (u - u_plain).abs().max().item() / u_plain.abs().max().item()
        result["mixed"] = {"s_per_step": t_mixed, "speedup_vs_plain": t_plain / t_mixed, "inner_cycles": args.inner,
                           "outer_per_step": float(np.mean(outer)),
                           "max_rel_diff_vs_plain_fp64": diff}
        print("bench: mixed %.4f s/step outer %s" % (t_mixed, outer), file=sys.stderr, flush=True)
        del g32

    if not args.no_cpu_baseline:
        print("bench: timing the oracle on one cycle", file=sys.stderr, flush=True)
        result["cpu_baseline"] = cpu_baseline(u0_h, n, dt, result["cycles_per_step"])

    result["device"] = torch.cuda.get_device_name(dev)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
