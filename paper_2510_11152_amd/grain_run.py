"""Grain-growth runs (Section 3.3.1): the multi-order-parameter Allen-Cahn system advanced
on the GPU by the stacked batched solver, with the mean grain size measured along the way
and the growth law R^m - R_0^m = k t fitted to it.

    python -m paper_2510_11152_amd.grain_run --dim 2 --q 1189 --n 512 --steps 10000 --every 250 --out run.json

A grain is a connected region (face neighbours, periodic) where one order parameter is the
largest (fas_grain_argmax on the GPU, labelling on the host); R = sqrt(A / pi) in 2D and
(3 V / (4 pi))^(1/3) in 3D from the mean grain size.  Initial state: eta_i uniform in
(-0.001, 0.001) from the seed, h = 1, dt = 0.1, kappa = 1, FP32 solves to a relative
residual of 1e-6, or an absolute one of 1e-6 sqrt(cells) (a field of order one).
"""
import argparse
import json
import math
import sys
import time


def fit_growth_law(t, R, ms=None):
    """Least-squares fits of R^m = R_0^m + k t for each exponent m; returns the best m (the
    smallest relative residual), its k, and the fit quality (R^2) of every m."""
    import numpy as np
    t = np.asarray(t, dtype=np.float64)
    R = np.asarray(R, dtype=np.float64)
    ms = np.arange(1.0, 4.01, 0.05) if ms is None else np.asarray(ms)
    fits = []
    for m in ms:
        y = R ** m
        A = np.stack([np.ones_like(t), t], axis=1)
        coef, *_ = np.linalg.lstsq(A, y, rcond=None)
        pred = A @ coef
        ss_res = float(((y - pred) ** 2).sum())
        ss_tot = float(((y - y.mean()) ** 2).sum())
        fits.append({"m": float(m), "k": float(coef[1]), "r2": 1.0 - ss_res / ss_tot if ss_tot > 0 else 0.0})
    best = max(fits, key=lambda f: f["r2"])
    return best, fits


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--dim", type=int, default=2)
    ap.add_argument("--q", type=int, default=1189)
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--steps", type=int, default=10000)
    ap.add_argument("--every", type=int, default=250)
    ap.add_argument("--fit-from", type=float, default=0.2, help="fit over measurements after this fraction of the run")
    ap.add_argument("--seed", type=int, default=6)
    ap.add_argument("--precision", default="fp32", choices=("fp32", "fp64", "mixed"))
    ap.add_argument("--paper", action="store_true",
                    help="the paper's setting: alpha = beta = gamma = 1, kappa = 2, h = 2, dt = 0.25 (default: "
                         "the grain workload's gamma = 1.5, kappa = 1, h = 1, dt = 0.1)")
    ap.add_argument("--tol", type=float, default=None, help="relative tolerance (default 1e-6 fp32, 1e-10 else)")
    ap.add_argument("--atol-factor", type=float, default=None,
                    help="absolute tolerance as a multiple of sqrt(cells) (default: tol)")
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)

    import numpy as np
    import torch

    from . import GrainGrowth, count_grains, grain_map

    dev = torch.device("cuda", 0)
    shape = (a.q,) + (a.n,) * a.dim
    tdt = np.float32 if a.precision == "fp32" else np.float64
    eta = torch.from_numpy(np.random.default_rng(a.seed).uniform(-0.001, 0.001, shape).astype(tdt)).to(dev)
    tol = a.tol if a.tol is not None else (1e-6 if a.precision == "fp32" else 1e-10)
    # absolute floor: by default tol times the norm of one field of order one over the grid,
    # so a field whose grains have all vanished (its values decaying towards zero) stops
    atol = (tol if a.atol_factor is None else a.atol_factor) * math.sqrt(a.n ** a.dim)
    h, dt, kappa, gamma = (2.0, 0.25, 2.0, 1.0) if a.paper else (1.0, 0.1, 1.0, 1.5)
    model = GrainGrowth(a.q, a.n, h=h, dt=dt, kappa=kappa, tol=tol, device=dev, dim=a.dim, atol=atol,
                        precision=a.precision, gamma=gamma)
    rows = []
    lab = torch.empty(shape[1:], dtype=torch.int32, device=dev)
    t_solve = 0.0
    for k in range(1, a.steps + 1):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        model.step(eta)
        torch.cuda.synchronize()
        t_solve += time.perf_counter() - t0
        if k % a.every == 0 or k == a.steps:
            grains, size = count_grains(grain_map(eta if eta.dtype == torch.float32 else eta.float(), lab).cpu().numpy())
            # grain size in length units (cells of area h^dim)
            R = h * (math.sqrt(size / math.pi) if a.dim == 2 else (3.0 * size / (4.0 * math.pi)) ** (1.0 / 3.0))
            rows.append({"step": k, "t": k * dt, "grains": grains, "mean_size": size, "R": R})
            print("grain run: step %d t %.1f grains %d R %.3f (%.3f ms/step)" % (k, k * dt, grains, R,
                                                                                 1e3 * t_solve / k), flush=True)
    sel = [r for r in rows if r["step"] >= a.fit_from * a.steps and r["grains"] > 1]
    best, fits = fit_growth_law([r["t"] for r in sel], [r["R"] for r in sel])
    m2 = min(fits, key=lambda f: abs(f["m"] - 2.0))
    out = {"dim": a.dim, "fields": a.q, "grid": [a.n] * a.dim, "steps": a.steps, "dt": dt, "kappa": kappa, "h": h,
           "alpha": 1.0, "beta": 1.0, "gamma": gamma,
           "precision": a.precision, "tol": tol, "atol": atol,
           "solve_and_rhs_s_per_step": t_solve / a.steps, "measurements": rows,
           "fit_window_t": [sel[0]["t"], sel[-1]["t"]] if sel else None,
           "best_fit": best, "fit_m2": m2}
    print(json.dumps({k: v for k, v in out.items() if k != "measurements"}), flush=True)
    if a.out:
        with open(a.out, "w") as fh:
            json.dump(out, fh, indent=1)
    return 0


if __name__ == "__main__":
    sys.exit(main())
