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

# rocprofv3 counter summary of the finest-level pass kernels (FETCH_SIZE / WRITE_SIZE,
# calibrated by a device copy of known size) and the sources it was taken from
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "heat8192_fp64_tile_traffic.md")
PASS_SOURCES = ["paper_2510_11152_amd/csrc/kernels_tile2d.hip", "paper_2510_11152_amd/csrc/fas_device.h",
                "paper_2510_11152_amd/csrc/march_util.h"]


# the same for the staggered solver's red-black sweep kernel (4096^2 projection step)
NS_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "ns4096_sweep_traffic.md")
NS_SOURCES = ["paper_2510_11152_amd/csrc/kernels_stag.hip", "paper_2510_11152_amd/csrc/stag_internal.h",
              "paper_2510_11152_amd/csrc/fas_device.h"]


def pass_sources_sha256(sources=None):
    import hashlib
    h = hashlib.sha256()
    for rel in sources or PASS_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(kernel, n, record=TRAFFIC_FILE, sources=None):
    """HBM bytes per launch of a finest-level kernel class from the committed counter
    summary ('traffic-record:' line), or None when there is none for this grid or the
    kernel sources have changed since the counters were taken."""
    try:
        with open(record) as fh:
            lines = [ln for ln in fh if ln.startswith("traffic-record:")]
    except OSError:
        return None
    if not lines:
        return None
    rec = json.loads(lines[-1].split(":", 1)[1])
    if rec.get("sources_sha256") != pass_sources_sha256(sources) or rec.get("grid") != [n, n]:
        return None
    k = rec.get("kernels", {}).get(kernel)
    return None if k is None else k["read_bytes"] + k["write_bytes"]


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10, help="timed heat steps")
    ap.add_argument("--warmup", type=int, default=1, help="untimed heat steps first")
    ap.add_argument("--n", type=int, default=8192, help="cells per axis")
    ap.add_argument("--inner", type=int, default=2, help="FP32 V-cycles per outer correction (2D mixed form)")
    ap.add_argument("--mixed-nu", type=int, default=2,
                    help="pre- and post-sweeps of the FP32 inner cycles of the 2D mixed form")
    ap.add_argument("--inner3d", type=int, default=4,
                    help="FP32 V-cycles per outer correction (3D mixed form; 4 reaches 1e-10 in two corrections)")
    ap.add_argument("--march3-sweeps", type=int, default=2, choices=(1, 2),
                    help="most sweeps per 3D plane-march pass (identical results)")
    ap.add_argument("--inner3d-next", type=int, default=0,
                    help="FP32 V-cycles in the 3D mixed form's corrections after the first (0: --inner3d)")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-autotune", action="store_true", help="fixed tile-shape rule for the 8192^2 grids")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--ns-dts", default="0.1,0.05,0.025,0.0125,0.00625",
                    help="time steps of the projection convergence study (comma list)")
    ap.add_argument("--ns-sizes", default="1024,2048,4096,8192,16384",
                    help="cavity grids for the memory / time comparison of the two field layouts")
    ap.add_argument("--forms", default="batched,adjoint,3d,orders,ns",
                    help="other workloads timed after the headline (comma list; 'none' to skip; "
                         "'table45' adds per-cycle times at the paper's Table 4/5 sizes)")
    return ap.parse_args()


def _timed(fn, sync):
    sync()
    t0 = time.perf_counter()
    out = fn()
    sync()
    return time.perf_counter() - t0, out


def bench_batched(dev):
    """Uneven batch of 64 2D Neumann heat solves (sizes drawn from 128^2..2048^2, FP64,
    dt = 1e-4, tol 1e-10): one array-form batched solve against looping single solves;
    then one grain-growth step of 1189 fields on 512^2 (periodic, h = 1, dt = 0.1, FP32,
    tol 1e-6): right-hand side + one batched solve."""
    import numpy as np
    import torch

    import fas_inputs
    from paper_2510_11152_amd import GrainGrowth, Grid, UnevenBatch

    sync = torch.cuda.synchronize
    fields = fas_inputs.uneven_batch()
    rhs = [torch.from_numpy(f).to(dev) for f in fields]
    grids = {}
    for r in rhs:
        m = r.shape[0]
        if m not in grids:
            grids[m] = Grid((m, m), 1.0 / m, coarsest=4, device=dev)

    ul = [r.clone() for r in rhs]

    def looped():
        cyc = []
        for r, u in zip(rhs, ul):
            u.copy_(r)
            g = grids[r.shape[0]]
            g.solve(r, u, 1e-4, tol=1e-10)
            cyc.append(g.stats()["cycles"])
        return cyc

    # all 64 problems in one fas_solve_batched call (one launch per pass over every
    # problem), grids planned once; the iterates live in fixed buffers, so the launch
    # descriptors written by the first solve are reused
    ub = UnevenBatch([tuple(r.shape) for r in rhs], device=dev)
    us = [r.clone() for r in rhs]

    def batched():
        for u, r in zip(us, rhs):
            u.copy_(r)
        return ub.solve(rhs, us, 1e-4, tol=1e-10)

    looped()
    batched()
    # best of three for each form (a single timing can catch a host or clock stall)
    loops = [_timed(looped, sync) for _ in range(3)]
    batches = [_timed(batched, sync) for _ in range(3)]
    t_loop, cyc_loop = min(loops, key=lambda x: x[0])
    t_batch, (st, cyc_b) = min(batches, key=lambda x: x[0])
    if list(cyc_b) != list(cyc_loop):
        raise RuntimeError("batched and looped solves ran different cycle counts")
    out = {"uneven": {"problems": len(rhs), "cells": int(sum(r.numel() for r in rhs)),
                      "sizes": sorted(set(int(r.shape[0]) for r in rhs)),
                      "batched_s": t_batch, "looped_s": t_loop, "speedup": t_loop / t_batch,
                      "batched_s_samples": [b[0] for b in batches], "looped_s_samples": [x[0] for x in loops],
                      "all_converged": all(s == 0 for s in st), "max_cycles": int(max(cyc_b))}}
    del rhs, grids, ub
    q, n = 1189, 512
    eta = torch.from_numpy(fas_inputs.grain_init(q, n)).to(dev)
    model = GrainGrowth(q, n, h=1.0, dt=0.1, kappa=1.0, tol=1e-6, device=dev, graph=True, autotune=True)
    model.step(eta.clone())
    steps = 3
    t_grain, cys = _timed(lambda: [model.step(eta) for _ in range(steps)], sync)
    out["grain"] = {"fields": q, "grid": [n, n], "s_per_step": t_grain / steps,
                    "field_cells_per_s": q * n * n * steps / t_grain, "cycles_per_field": float(np.mean(cys[-1]))}
    del eta, model
    torch.cuda.empty_cache()
    out["grain_1e-10"] = bench_grain_tight(dev, q, n)
    return out


def bench_grain_tight(dev, q=1189, n=512, steps=2):
    """The grain-growth step at 1e-10 relative residual per field, from the seeded state:
    the mixed form (FP64 state and right-hand side, defect correction around two FP32
    V-cycles, all fields per launch) against plain FP64 solves looped over the fields (the
    baseline: one fas_solve per field) and the stacked plain FP64 form."""
    import numpy as np
    import torch

    import fas_inputs
    from paper_2510_11152_amd import GrainGrowth, Grid, grain_rhs

    sync = torch.cuda.synchronize
    eta0 = torch.from_numpy(fas_inputs.grain_init(q, n).astype(np.float64)).to(dev)
    kw = dict(h=1.0, dt=0.1, kappa=1.0, tol=1e-10, device=dev)
    mixed = GrainGrowth(q, n, precision="mixed", inner=2, autotune=True, **kw)
    stacked = GrainGrowth(q, n, precision="fp64", autotune=True, **kw)
    g1 = Grid((n, n), 1.0, bc="periodic", coarsest=4, device=dev)
    rhs = torch.empty_like(eta0)

    def looped(eta):
        cyc = []
        for _ in range(steps):
            grain_rhs(eta, 0.1, rhs)
            for i in range(q):
                if g1.solve(rhs[i], eta[i], 0.1, tol=1e-10) != 0:
                    raise RuntimeError("a looped grain solve did not converge")
                cyc.append(g1.stats()["cycles"])
        return cyc

    def run(model, eta):
        return [model.step(eta) for _ in range(steps)]

    res = {}
    for name, fn in (("mixed", lambda e: run(mixed, e)), ("stacked_fp64", lambda e: run(stacked, e)),
                     ("looped_fp64", looped)):
        e = eta0.clone()
        fn(e)  # warm-up (autotuning, descriptors)
        e = eta0.clone()
        t, cyc = _timed(lambda: fn(e), sync)
        res[name] = (t / steps, e, cyc)
    ref = res["looped_fp64"][1]
    scale = ref.abs().max().item()
    out = {"fields": q, "grid": [n, n], "tol": 1e-10, "steps_timed": steps,
           "looped_fp64_s_per_step": res["looped_fp64"][0],
           "stacked_fp64_s_per_step": res["stacked_fp64"][0],
           "mixed_s_per_step": res["mixed"][0],
           "mixed_inner_cycles": 2,
           "mixed_outer_per_field": float(np.mean(res["mixed"][2][-1])),
           "fp64_cycles_per_field": float(np.mean(res["stacked_fp64"][2][-1])),
           "mixed_speedup_vs_looped_fp64": res["looped_fp64"][0] / res["mixed"][0],
           "mixed_speedup_vs_stacked_fp64": res["stacked_fp64"][0] / res["mixed"][0],
           "stacked_fp64_speedup_vs_looped": res["looped_fp64"][0] / res["stacked_fp64"][0],
           "mixed_max_rel_diff_vs_looped_fp64": (res["mixed"][1] - ref).abs().max().item() / scale,
           "stacked_fp64_equals_looped": bool(torch.equal(res["stacked_fp64"][1], ref))}
    del res, ref, mixed, stacked, g1, rhs, eta0
    torch.cuda.empty_cache()
    return out


def bench_orders(dev, sizes=(1024, 2048)):
    """The smoother-ordering study of Section 2.3 in its setting: p - Lap p = f on [0,1]^2
    with Dirichlet boundaries, f from the exact solution prod sin(pi sin(pi x)), a zero
    initial guess, V(2,2) cycles down to 2^2 (meshLevel = log2 n - 1), two sweeps on the
    coarsest level, kMax = 100, stop when the paper's res = h ||f - A p||_2 < 1e-9.  X, U
    and Z set orders, each with the 1234-1234 and 1234-4321 sequences; cycles and time."""
    import torch

    import fas_inputs
    from paper_2510_11152_amd import Grid

    out = {}
    for n in sizes:
        h = 1.0 / n
        f_h, _ = fas_inputs.paper_sine_problem(n)
        f = torch.from_numpy(f_h).to(dev)
        tol = 1e-9 / (h * float(torch.linalg.vector_norm(f)))  # res = h ||r|| as a relative tolerance
        g = Grid((n, n), h, bc="dirichlet", coarsest=2, device=dev).set(coarse_sweeps=2, kmax=100)
        row = {}
        for order in ("x", "u", "z"):
            for sym in (False, True):
                g.set(order=order, symmetric=sym)
                u = torch.zeros_like(f)
                g.solve(f, u, 1.0, tol=tol)  # warm-up (and the cycle count the timed solve reuses)
                u.zero_()
                t, st = _timed(lambda: g.solve(f, u, 1.0, tol=tol), torch.cuda.synchronize)
                s = g.stats()
                row[order.upper() + (" 1234-4321" if sym else " 1234-1234")] = {
                    "cycles": s["cycles"], "converged": st == 0, "s": t,
                    "res": h * s["rel_res"][s["cycles"] - 1] * float(torch.linalg.vector_norm(f))}
        x = row["X 1234-1234"]["cycles"]
        out["%d^2" % n] = {"configs": row,
                           "cycles_vs_x": {k: v["cycles"] / x for k, v in row.items()}}
        del g, f
    torch.cuda.empty_cache()
    return out


def bench_table45(dev, cpu=True, reps=10):
    """Per-V-cycle times at the sizes of the paper's Tables 4 and 5 (2D 1024^2 .. 16384^2,
    3D 128^3 .. 512^3), in their setting: p - Lap p = f (dt = kappa = 1), Dirichlet, the
    sine test solution, zero initial guess, V(2,2) down to 2^d (meshLevel = log2 N - 1).
    GPU: the mean of `reps` cycles after one warm-up cycle (the paper averages ten);
    oracle: one cycle on one thread (sizes up to 8192^2 and 256^3; the larger ones are
    quoted from the paper's own one-core column only)."""
    import numpy as np
    import torch

    import fas_inputs
    from paper_2510_11152_amd import Grid

    out = {"host": host_cpu(), "rows": []}
    for dim, n in ((2, 1024), (2, 2048), (2, 4096), (2, 8192), (2, 16384), (3, 128), (3, 256), (3, 512)):
        f_h, _ = fas_inputs.paper_sine_problem(n, dim)
        f = torch.from_numpy(f_h).to(dev)
        u = torch.zeros_like(f)
        g = Grid((n,) * dim, 1.0 / n, bc="dirichlet", coarsest=2, device=dev).set(coarse_sweeps=2)
        g.vcycle(f, u, 1.0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            g.vcycle(f, u, 1.0)
        torch.cuda.synchronize()
        row = {"dim": dim, "n": n, "gpu_s_per_cycle": (time.perf_counter() - t0) / reps}
        del g, u, f
        torch.cuda.empty_cache()
        if cpu and ((dim == 2 and n <= 8192) or (dim == 3 and n <= 256)):
            import oracle

            P = oracle.Problem(n=(n,) * dim, h=1.0 / n, dt=1.0, kappa=1.0, bc="dirichlet", coarsest=2, nuc=2)
            uh = np.zeros_like(f_h)
            t0 = time.perf_counter()
            oracle.vcycle(P, np.ascontiguousarray(f_h), uh, 2, 2)
            row["oracle_s_per_cycle"] = time.perf_counter() - t0
        print("bench: table 4/5 %dD %d: %s" % (dim, n, row), file=sys.stderr, flush=True)
        out["rows"].append(row)
    return out


def bench_adjoint(dev):
    """Differentiable 2D heat at 2048^2: kappa = exp(0.5 g), 20 steps, dt = 1e-4,
    checkpoint every 4; forward + backward (gradients for u0 and kappa)."""
    import torch

    import fas_inputs
    from paper_2510_11152_amd import Grid, HeatSolveFn

    n, T, dt = 2048, 20, 1e-4
    kap, u0, tgt = (torch.from_numpy(a).to(dev) for a in fas_inputs.adjoint_inputs(n))
    g = Grid((n, n), 1.0 / n, coarsest=4, variable_kappa=True, device=dev)

    def run():
        a = u0.clone().requires_grad_(True)
        k = kap.clone().requires_grad_(True)
        uT = HeatSolveFn.apply(a, k, g, T, dt, 4, 1e-10, 2, 2)
        loss = ((uT - tgt) ** 2).sum()
        loss.backward()
        return float(loss.item())

    run()
    t, loss = _timed(run, torch.cuda.synchronize)
    return {"grid": [n, n], "steps": T, "ckpt": 4, "forward_backward_s": t, "loss": loss}


def bench_3d(dev, steps=5, inner=4, cpu=True, inner_next=0, march3_sweeps=2):
    """3D heat at 512^3 (7-point, 8-set X-MCGS, Neumann, dt = 1e-4): plain FP64 V(2,2)
    steps to 1e-10, then the same steps with FP32 inner cycles in FP64 correction."""
    import numpy as np
    import torch

    import fas_inputs
    from paper_2510_11152_amd import Grid, solve_mixed

    n, dt = 512, 1e-4
    u0_h = fas_inputs.heat_3d(n)
    u0 = torch.from_numpy(u0_h).to(dev)
    g = Grid((n, n, n), 1.0 / n, coarsest=4, device=dev).set(march3_sweeps=march3_sweeps)
    rhs = torch.empty_like(u0)

    def plain(u):
        cyc = []
        for _ in range(steps):
            rhs.copy_(u)
            assert g.solve(rhs, u, dt, tol=1e-10) == 0
            cyc.append(g.stats()["cycles"])
        return cyc

    u = u0.clone()
    plain(u)
    u = u0.clone()
    t_plain, cyc = _timed(lambda: plain(u), torch.cuda.synchronize)
    out = {"grid": [n, n, n], "steps": steps, "plain_s_per_step": t_plain / steps, "cycles_per_step": float(np.mean(cyc)),
           "march3_sweeps_per_pass": march3_sweeps}
    # finest-level plane-march passes of one more (untimed) step, HIP events around each
    # class.  Two sweeps per pass: pre = one sweeps/residual/restriction pass (3s + 2s/8 per
    # cell), post = one correction/sweeps/norm pass (3s + s/8), s = 8 B; one sweep per pass:
    # pre = sweep pass + sweep/residual/restriction pass (3s + 3s + 2s/8), post =
    # correction/sweep pass + sweep/norm pass (3s + s/8 + 3s)
    g.set(profile=True)
    g.profile(reset=True)
    v = u.clone()
    plain(v)
    prof = g.profile(reset=True)
    g.set(profile=False)
    del v
    passes = 1 if march3_sweeps == 2 else 2
    bytes3 = {"pre": 8 * (3 * passes + 2 / 8) * n ** 3, "post": 8 * (3 * passes + 1 / 8) * n ** 3}
    # the bytes the same two sweeps would move as one-sweep passes: a rate for comparing the
    # two pass sizes (the work is the same, only the bytes per pass differ)
    bytes1 = {"pre": 8 * (6 + 2 / 8) * n ** 3, "post": 8 * (6 + 1 / 8) * n ** 3}
    k3 = {}
    for k in ("pre", "post"):
        launches, ms = prof[k]
        if launches:
            sec = ms / 1e3 / launches
            gbs = bytes3[k] / sec / 1e9
            k3[k] = {"passes_per_launch": passes, "avg_us": ms * 1e3 / launches, "algorithmic_bytes": bytes3[k],
                     "gbs": gbs, "frac": gbs / PEAK_HBM_GBS,
                     "one_sweep_pass_bytes": bytes1[k], "one_sweep_pass_equivalent_gbs": bytes1[k] / sec / 1e9}
    out["finest_level_kernels"] = k3
    g32 = Grid((n, n, n), 1.0 / n, dtype=torch.float32, coarsest=4, mixed_inner=True, device=dev).set(
        march3_sweeps=march3_sweeps)

    def mixed(v):
        outer = []
        for _ in range(steps):
            rhs.copy_(v)
            assert solve_mixed(g, g32, rhs, v, dt, tol=1e-10, inner=inner, inner_next=inner_next) == 0
            outer.append(g.stats()["cycles"])
        return outer

    v = u0.clone()
    rhs.copy_(v)
    assert solve_mixed(g, g32, rhs, v, dt, tol=1e-10, inner=inner, inner_next=inner_next) == 0  # warm-up
    v = u0.clone()
    t_mixed, outer = _timed(lambda: mixed(v), torch.cuda.synchronize)
    out.update({"mixed_s_per_step": t_mixed / steps, "mixed_inner_cycles": inner,
                "mixed_inner_cycles_next": inner_next or inner,
                "mixed_outer_per_step": float(np.mean(outer)),
                "mixed_speedup": t_plain / t_mixed,
                "mixed_max_rel_diff": (v - u).abs().max().item() / u.abs().max().item()})
    del g, g32, u0, rhs, u, v
    torch.cuda.empty_cache()
    if cpu:
        # the oracle (one thread) on a bounded sample: the first V(2,2) cycle of step 1
        import oracle

        P = oracle.Problem(n=(n, n, n), h=1.0 / n, dt=dt, kappa=1.0, bc="neumann", coarsest=4, nuc=2)
        f = np.ascontiguousarray(u0_h)
        uh = f.copy()
        t0 = time.perf_counter()
        oracle.vcycle(P, f, uh, 2, 2)
        t_cycle = time.perf_counter() - t0
        value = t_cycle * out["cycles_per_step"]
        out["cpu_baseline"] = {"value": value, "unit": "s", "cores": 1, "kind": "oracle",
                               "sample": "the first FP64 V(2,2) cycle of step 1 at 512^3 (%.1f s, single thread), "
                                         "times %.2f GPU cycles per step" % (t_cycle, out["cycles_per_step"])}
        out["speedup_vs_cpu_baseline"] = value / out["plain_s_per_step"]
    return out


def bench_ns(dev, n=4096, re=10.0, dts=(0.1, 0.05, 0.025, 0.0125, 0.00625), cpu=True, ceiling=None,
             layout_sizes=(1024, 2048, 4096, 8192, 16384)):
    """Section 4.4.3: Scheme 1 (first-order projection) on the staggered 4096^2 grid, Re = 10,
    tol 1e-9, V(2,2), manufactured source at t^{n+1}, t = 0 .. 1 for each dt; L2 errors at
    t = 1 against the exact solution and their orders.  Then both field layouts at one dt
    (fields, workspace, peak device memory, time per step), and the finest level's fused
    pre- and post-smoothing launches of the u solve timed with the library's HIP events."""
    import numpy as np
    import torch

    from oracle import ns as ons
    from paper_2510_11152_amd import NavierStokes2D, StaggeredSolver

    h = 1.0 / n
    Fu, Fv = ons.manufactured_fields(n, n, h, re)
    Fu = [torch.from_numpy(x).to(dev) for x in Fu]
    Fv = [torch.from_numpy(x).to(dev) for x in Fv]
    ue, ve, pe = ons.exact(n, n, h, 1.0)
    u0, v0, p0 = ons.exact(n, n, h, 0.0)
    out = {"grid": [n, n], "re": re, "tol": 1e-9, "rows": []}
    total_steps, total_s, cycles = 0, 0.0, [0, 0, 0]
    prev = None
    for dt in dts:
        G = NavierStokes2D(n, n, h, re)
        G.u.copy_(torch.from_numpy(u0))
        G.v.copy_(torch.from_numpy(v0))
        G.p.copy_(torch.from_numpy(p0))
        steps = int(round(1.0 / dt))

        def run():
            cyc = [0, 0, 0]
            for k in range(steps):
                st, c, _ = G.step(dt, 0.0, Fu, Fv, ons.manufactured_coef((k + 1) * dt), tol=1e-9)
                if st != 0:
                    raise RuntimeError("a projection solve did not converge at step %d" % k)
                cyc = [a + b for a, b in zip(cyc, c)]
            return cyc

        t, cyc = _timed(run, torch.cuda.synchronize)
        u, v, p = G.u.cpu().numpy(), G.v.cpu().numpy(), G.p.cpu().numpy()
        errs = [ons.l2(u - ue, h), ons.l2(v - ve, h), ons.l2((p - p.mean()) - (pe - pe.mean()), h)]
        row = {"dt": dt, "steps": steps, "s": t, "ms_per_step": 1e3 * t / steps, "errors_uvp": errs,
               "cycles_per_step_uvp": [c / steps for c in cyc]}
        if prev is not None:
            row["orders_uvp"] = [float(np.log2(a / b)) for a, b in zip(prev, errs)]
        prev = errs
        out["rows"].append(row)
        total_steps += steps
        total_s += t
        cycles = [a + b for a, b in zip(cycles, cyc)]
        print("bench: ns dt %.5f %.2f ms/step errors %s" % (dt, row["ms_per_step"], errs), file=sys.stderr,
              flush=True)
        del G
    out["ms_per_step"] = 1e3 * total_s / total_steps
    out["cycles_per_step_uvp"] = [c / total_steps for c in cycles]
    # both layouts at dt = 1/40: memory and time
    layouts = {}
    for layout in ("memory_efficient", "classical"):
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        torch.cuda.reset_peak_memory_stats(dev)
        base = torch.cuda.memory_allocated(dev)
        G = NavierStokes2D(n, n, h, re, layout=layout)
        fb, wb = G.memory()
        dt = 0.025

        def run():
            for k in range(40):
                G.step(dt, 0.0, Fu, Fv, ons.manufactured_coef((k + 1) * dt), tol=1e-9)

        t, _ = _timed(run, torch.cuda.synchronize)
        layouts[layout] = {"fields": len(G.fields), "field_bytes": fb, "workspace_bytes": wb,
                           "peak_bytes": torch.cuda.max_memory_allocated(dev) - base, "ms_per_step": 1e3 * t / 40}
        del G
    layouts["field_bytes_saved"] = 1.0 - layouts["memory_efficient"]["field_bytes"] / layouts["classical"]["field_bytes"]
    layouts["time_ratio_classical_over_memory_efficient"] = (layouts["classical"]["ms_per_step"] /
                                                            layouts["memory_efficient"]["ms_per_step"])
    out["layouts_dt_1_40"] = layouts
    # Section 4.4.1-4.4.2 across sizes: device memory and time per step of both layouts,
    # lid-driven cavity (Re = 100, dt = 1e-3, tol 1e-9), 5 timed steps after 2
    sizes = []
    for m in layout_sizes:
        row = {"grid": [m, m]}
        for layout in ("memory_efficient", "classical"):
            torch.cuda.synchronize()
            torch.cuda.empty_cache()
            torch.cuda.reset_peak_memory_stats(dev)
            base = torch.cuda.memory_allocated(dev)
            G = NavierStokes2D(m, m, 1.0 / m, 100.0, layout=layout)
            for _ in range(2):
                G.step(1e-3, lid=1.0)

            def run():
                for _ in range(5):
                    G.step(1e-3, lid=1.0)

            t, _ = _timed(run, torch.cuda.synchronize)
            fb, wb = G.memory()
            row[layout] = {"field_bytes": fb, "workspace_bytes": wb,
                           "peak_bytes": torch.cuda.max_memory_allocated(dev) - base, "ms_per_step": 1e3 * t / 5}
            del G
        row["peak_saved"] = 1.0 - row["memory_efficient"]["peak_bytes"] / row["classical"]["peak_bytes"]
        row["time_ratio_classical_over_memory_efficient"] = (row["classical"]["ms_per_step"] /
                                                            row["memory_efficient"]["ms_per_step"])
        sizes.append(row)
        print("bench: ns cavity %d^2 %.2f / %.2f ms per step, peak %.2f / %.2f GB" % (
            m, row["memory_efficient"]["ms_per_step"], row["classical"]["ms_per_step"],
            row["memory_efficient"]["peak_bytes"] / 1e9, row["classical"]["peak_bytes"] / 1e9), file=sys.stderr,
            flush=True)
    out["layouts_by_size"] = sizes
    # the finest level's fused launches of the u solve, timed by the library's HIP events
    # (FAS_OPT_PROFILE) over a solve of six cycles
    S = StaggeredSolver("edge_x", n, n, h)
    S.set(profile=1)
    f = torch.randn(S.shape, dtype=torch.float64, device=dev)
    w = torch.zeros_like(f)
    S.solve(1.0, 0.025 / re, f, w, 0.0, kmax=6)
    pre_us, post_us, timed = S.profile()
    fine = S.shape[0] * S.shape[1]
    coarse = (n // 2) * (n // 2 - 1)
    alg_pre = 24.0 * fine + 24.0 * coarse    # read w, f; write w; write R w (twice) and R r
    alg_post = 24.0 * fine + 16.0 * coarse   # read w, f and the coarse iterate and its copy; write w
    out["finest_kernels"] = {
        "grid": list(S.shape), "cycles_timed": timed,
        "pre": {"kernel": "k_sweep<2, EDGE_X, RHS=0, RES=1>: two sweeps, residual, restriction",
                "avg_us": pre_us, "algorithmic_bytes": alg_pre, "gbs": alg_pre / (pre_us * 1e-6) / 1e9},
        "post": {"kernel": "k_sweep<2, EDGE_X, CORR=1, NORM=1>: correction, two sweeps, residual norm",
                 "avg_us": post_us, "algorithmic_bytes": alg_post, "gbs": alg_post / (post_us * 1e-6) / 1e9}}
    gbs = alg_pre / (pre_us * 1e-6) / 1e9
    out["roofline"] = {"bound": "hbm", "kernel": out["finest_kernels"]["pre"]["kernel"] + " (finest level)",
                       "achieved": gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": gbs / PEAK_HBM_GBS,
                       "traffic": measured_traffic("pre", n, NS_TRAFFIC_FILE, NS_SOURCES),
                       "algorithmic_bytes": alg_pre}
    if ceiling:
        out["roofline"]["attainable"] = ceiling
        out["roofline"]["frac_of_attainable"] = gbs / ceiling
    del S, f, w
    if cpu:
        out["cpu_baseline"] = ns_cpu_baseline(n, re, out["cycles_per_step_uvp"])
        out["speedup_vs_cpu_baseline"] = out["cpu_baseline"]["value"] / (out["ms_per_step"] / 1e3)
    torch.cuda.empty_cache()
    return out


def ns_cpu_baseline(n, re, cycles_uvp):
    """The oracle on a bounded sample of one 4096^2 projection step: the u momentum
    right-hand side and one V(2,2) cycle of the u solve, extrapolated to a step as two
    right-hand sides and the GPU's mean cycles of the three solves."""
    import numpy as np

    from oracle import ns as ons
    from oracle import staggered as ost

    h = 1.0 / n
    u, v, p = ons.exact(n, n, h, 0.3)
    t0 = time.perf_counter()
    fu = ons.momentum_rhs_u(u, v, p, h, 0.025, 0.0)
    t_rhs = time.perf_counter() - t0
    P = ost.StagProblem(ost.EDGE_X, n, n, h)
    w = np.zeros(P.shape())
    t0 = time.perf_counter()
    ost.vcycle(P, 1.0, 0.025 / re, fu, w)
    t_cyc = time.perf_counter() - t0
    value = 2 * t_rhs + sum(cycles_uvp) * t_cyc
    return {"value": value, "unit": "s", "cores": 1, "kind": "oracle",
            "sample": "one u right-hand side (%.1f s) and one u V(2,2) cycle (%.1f s) at 4096^2, per step "
                      "2 right-hand sides + %.1f cycles (numpy, one thread)" % (t_rhs, t_cyc, sum(cycles_uvp))}


def stream_ceiling(dev, gib=1.0, reps=10):
    """Attainable HBM bandwidth from the library's own streaming probe (fas_stream_probe):
    read, copy and triad (c = a + b) over `gib` GiB arrays, 16 B per lane, best of a few
    grid sizes; GB/s of bytes moved (read 1x, copy 2x, triad 3x the array)."""
    import ctypes

    import torch

    from paper_2510_11152_amd import _lib

    L = _lib.load()
    nbytes = int(gib * 2 ** 30)
    a = torch.full((nbytes // 8,), 1.0, dtype=torch.float64, device=dev)
    b = torch.full_like(a, 2.0)
    c = torch.empty_like(a)
    stream = torch.cuda.current_stream(dev).cuda_stream
    out = {"array_gib": gib}
    for kind, name, moved in ((0, "read", 1), (1, "copy", 2), (2, "triad", 3)):
        best = None
        for blocks in (1024, 2048, 4096, 8192):
            part = torch.empty(blocks, dtype=torch.float64, device=dev)
            ms = ctypes.c_double(0.0)
            _lib.check(L.fas_stream_probe(ctypes.c_void_p(stream), kind, nbytes, ctypes.c_void_p(a.data_ptr()),
                                          ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(c.data_ptr()),
                                          ctypes.c_void_p(part.data_ptr()), blocks, reps, ctypes.byref(ms)),
                       "fas_stream_probe")
            gbs = moved * nbytes / (ms.value / 1e3) / 1e9
            if best is None or gbs > best[0]:
                best = (gbs, blocks, ms.value * 1e3)
        out[name] = {"gbs": best[0], "blocks": best[1], "avg_us": best[2]}
    del a, b, c
    torch.cuda.empty_cache()
    return out


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


def host_cpu():
    """The host the oracle runs on: CPU model (/proc/cpuinfo), logical CPUs, and the CPUs
    this process may use."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for ln in fh:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"model": model, "logical_cpus": os.cpu_count(), "usable_cpus": len(os.sched_getaffinity(0)),
            "oracle_threads": 1}


def cpu_baseline(u0, n, dt, cycles_per_step, cycles=2):
    """The oracle (single thread) on a bounded sample: the first two V(2,2) cycles of the
    first heat step at full size, scaled to seconds per step by the GPU's cycles per step."""
    import numpy as np

    import oracle

    P = oracle.Problem(n=(n, n), h=1.0 / n, dt=dt, kappa=1.0, bc="neumann", coarsest=4, nuc=2)
    f = np.ascontiguousarray(u0)
    u = f.copy()
    t0 = time.perf_counter()
    for _ in range(cycles):
        oracle.vcycle(P, f, u, 2, 2)
    t_all = time.perf_counter() - t0
    t_cycle = t_all / cycles
    return {
        "value": t_cycle * cycles_per_step,
        "unit": "s",
        "cores": 1,
        "kind": "oracle",
        "sample": "the first %d FP64 V(2,2) cycles of step 1 at %d^2 (%.1f s, single thread), per cycle times "
                  "%.2f GPU cycles per step" % (cycles, n, t_all, cycles_per_step),
        "host": host_cpu(),
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

    # tile shapes picked by the library's autotuner on the first (warm-up) solve
    g = Grid((n, n), 1.0 / n, dtype=torch.float64, coarsest=4, device=dev).set(autotune=not args.no_autotune)
    rhs = torch.empty_like(u0)

    def step_plain(u):
        rhs.copy_(u)
        st = g.solve(rhs, u, dt, tol=tol, nu1=2, nu2=2)
        if st != 0:
            raise RuntimeError("plain solve did not converge")
        return g.stats()["cycles"]

    # plan time: with autotuning, one V-cycle times the tile-shape candidates of every level
    # (kept by the grid), then the warm-up steps, then the timed steps
    if not args.no_autotune:
        tune = u0.clone()
        g.vcycle(u0, tune, dt)
        del tune
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

    ceiling = stream_ceiling(dev)
    attain = max(ceiling["copy"]["gbs"], ceiling["triad"]["gbs"])
    for k, v in per_kernel.items():
        v["frac_of_peak"] = v["gbs"] / PEAK_HBM_GBS if v["gbs"] else None
        v["frac_of_attainable"] = v["gbs"] / attain if v["gbs"] else None
    print("bench: stream ceiling read %.0f copy %.0f triad %.0f GB/s" % (
        ceiling["read"]["gbs"], ceiling["copy"]["gbs"], ceiling["triad"]["gbs"]), file=sys.stderr, flush=True)

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
                   "grid": [n, n], "steps_timed": args.steps, "nu1": 2, "nu2": 2, "coarsest": 4, "tol": tol,
                   "autotune": not args.no_autotune},
        "cycles_per_step": float(np.mean(cycles)),
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": achieved / PEAK_HBM_GBS, "traffic": measured_traffic(dom, n),
                     "algorithmic_bytes": kb[dom] * n * n, "attainable": attain,
                     "frac_of_attainable": achieved / attain, "stream_probe": ceiling},
        "kernels": per_kernel,
    }

    if not args.no_mixed:
        g32 = Grid((n, n), 1.0 / n, dtype=torch.float32, coarsest=4, mixed_inner=True, device=dev).set(
            autotune=not args.no_autotune)
        outer = []

        def step_mixed(u):
            rhs.copy_(u)
            st = solve_mixed(g, g32, rhs, u, dt, tol=tol, nu1=args.mixed_nu, nu2=args.mixed_nu, inner=args.inner)
            if st != 0:
                raise RuntimeError("mixed solve did not converge")
            return g.stats()["cycles"]

        if not args.no_autotune:
            # plan time for the FP32 inner grid: one inner V-cycle tunes its levels
            e = torch.zeros(u0.shape, dtype=torch.float32, device=dev)
            g32.vcycle(u0.float(), e, dt, nu1=args.mixed_nu, nu2=args.mixed_nu)
            del e
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
                           "inner_nu": [args.mixed_nu, args.mixed_nu],
                           "outer_per_step": float(np.mean(outer)),
                           "max_rel_diff_vs_plain_fp64": diff}
        print("bench: mixed %.4f s/step outer %s" % (t_mixed, outer), file=sys.stderr, flush=True)
        del g32

    forms = [f for f in args.forms.split(",") if f and f != "none"]
    del g, rhs
    torch.cuda.empty_cache()
    if "batched" in forms:
        print("bench: batched forms", file=sys.stderr, flush=True)
        result["batched"] = bench_batched(dev)
    if "adjoint" in forms:
        print("bench: adjoint form", file=sys.stderr, flush=True)
        result["adjoint"] = bench_adjoint(dev)
    if "table45" in forms:
        print("bench: per-cycle times at the paper's Table 4/5 sizes", file=sys.stderr, flush=True)
        result["table45"] = bench_table45(dev, cpu=not args.no_cpu_baseline)
    if "orders" in forms:
        print("bench: smoother ordering study", file=sys.stderr, flush=True)
        result["orders"] = bench_orders(dev)
    if "3d" in forms:
        print("bench: 3D heat", file=sys.stderr, flush=True)
        result["heat3d"] = bench_3d(dev, inner=args.inner3d, cpu=not args.no_cpu_baseline, inner_next=args.inner3d_next,
                                    march3_sweeps=args.march3_sweeps)
    if "ns" in forms:
        print("bench: staggered projection step (4096^2)", file=sys.stderr, flush=True)
        result["ns"] = bench_ns(dev, dts=tuple(float(x) for x in args.ns_dts.split(",")),
                                cpu=not args.no_cpu_baseline, ceiling=attain,
                                layout_sizes=tuple(int(x) for x in args.ns_sizes.split(",") if x))

    if not args.no_cpu_baseline:
        print("bench: timing the oracle on two cycles", file=sys.stderr, flush=True)
        result["cpu_baseline"] = cpu_baseline(u0_h, n, dt, result["cycles_per_step"])
        result["speedup_vs_cpu_baseline"] = result["cpu_baseline"]["value"] / result["value"]

    result["device"] = torch.cuda.get_device_name(dev)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
