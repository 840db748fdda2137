"""Oracle of the grain-growth right-hand side (test infrastructure only).

Section 3.3.1, eq. grain-growth-equations with L = alpha = beta = gamma = 1 (the
free energy sum_i(-eta_i^2/2 + eta_i^4/4) + 3/2 sum_{i<j} eta_i^2 eta_j^2): the
semi-implicit step (1/dt - kappa Lap) eta_i^{n+1} = eta_i^n/dt - df/deta_i(eta^n), times
dt, has the right-hand side

    f_i = eta_i - dt * ((eta_i^3 - eta_i) + 3 eta_i (S - eta_i^2)),  S = sum_j eta_j^2.

Plain numpy in the state's precision (float32 for the FP32 solves, float64 for the FP64
and mixed forms), S summed field by field in index order; each operation rounds in that
precision as written.
"""
import numpy as np


def grain_rhs(eta, dt, dtype=np.float32, alpha=1.0, beta=1.0, gamma=1.5):
    """f_i = eta_i - dt ((beta eta_i^3 - alpha eta_i) + 2 gamma eta_i (S - eta_i^2)); the
    defaults are the grain workload's coefficients (the paper uses alpha = beta = gamma = 1)."""
    eta = np.asarray(eta, dtype=dtype)
    dt, a, b, g2 = dtype(dt), dtype(alpha), dtype(beta), dtype(2.0 * gamma)
    S = eta[0] * eta[0]
    for j in range(1, eta.shape[0]):
        S = S + eta[j] * eta[j]
    out = np.empty_like(eta)
    for i in range(eta.shape[0]):
        e = eta[i]
        e2 = e * e
        g = ((b * e2) * e - a * e) + (g2 * e) * (S - e2)
        out[i] = e - dt * g
    return out


def grain_rhs_reference(eta, dt, alpha=1.0, beta=1.0, gamma=1.5):
    """The same quantity from the free energy in float64 by central differences of
    f(eta) along each eta_i (an independent check of the derivative, not of rounding)."""
    eta = np.asarray(eta, dtype=np.float64)

    def energy(x):
        sq = x * x
        pair = 0.5 * (sq.sum(axis=0) ** 2 - (sq * sq).sum(axis=0))   # sum_{i<j} eta_i^2 eta_j^2
        return (-0.5 * alpha * sq + 0.25 * beta * sq * sq).sum(axis=0) + gamma * pair

    d = np.empty_like(eta)
    h = 1e-5
    for i in range(eta.shape[0]):
        xp, xm = eta.copy(), eta.copy()
        xp[i] += h
        xm[i] -= h
        d[i] = (energy(xp) - energy(xm)) / (2 * h)
    return eta - dt * d
