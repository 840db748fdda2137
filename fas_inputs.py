"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This module only draws numbers and evaluates the closed-form initial fields of the
workloads (sums of cosine modes on cell centres x_i = (i + 1/2) h, uniform noise,
log-normal coefficient fields).  It contains none of the solver's arithmetic and
imports neither the oracle nor the GPU library.

All fields are float64 numpy arrays shaped (ny, nx) or (nz, ny, nx), x fastest.
Generator: numpy.random.default_rng(seed) (PCG64), draws taken in the order stated.
"""
import numpy as np


def centres(n, h=None):
    """Cell centres (i + 1/2) h of an axis with n cells on [0, n h]; h defaults to 1/n."""
    h = 1.0 / n if h is None else h
    return (np.arange(n, dtype=np.float64) + 0.5) * h


def cosine_modes(n, dim, nmodes, rng, kmax=8, scale=1.0):
    """sum_m a_m prod_axes cos(k_{m,axis} pi x_axis) on [0,1]^dim with n cells per axis.

    Draw order: one integer vector per axis (x, then y, then z), each
    rng.integers(1, kmax + 1, nmodes), then a = rng.standard_normal(nmodes) * scale."""
    ks = [rng.integers(1, kmax + 1, nmodes) for _ in range(dim)]
    a = rng.standard_normal(nmodes) * scale
    x = centres(n)
    C = [np.cos(np.pi * np.outer(k, x)) for k in ks]  # each (nmodes, n)
    if dim == 2:
        # u[y, x] = sum_m a_m Cy[m, y] Cx[m, x]
        return (C[1].T * a) @ C[0]
    # u[z, y, x] = sum_m a_m Cz[m, z] Cy[m, y] Cx[m, x]
    yx = (C[1][:, :, None] * C[0][:, None, :]).reshape(nmodes, n * n)
    return ((C[2].T * a) @ yx).reshape(n, n, n)


def heat_2d_small(n=256, seed=0, nmodes=16):
    """256^2 Neumann heat step input: 16 cosine modes, k, l in 1..8, a ~ N(0,1)."""
    return cosine_modes(n, 2, nmodes, np.random.default_rng(seed))


def heat_2d_large(n=8192, seed=1, nmodes=64, noise=0.01):
    """8192^2 heat input: 64 cosine modes plus uniform(-noise, noise) per cell."""
    rng = np.random.default_rng(seed)
    u = cosine_modes(n, 2, nmodes, rng)
    u += rng.uniform(-noise, noise, (n, n))
    return u


def heat_3d(n=512, seed=2, nmodes=32):
    """512^3 heat input: 32 cosine-product modes, k, l, m in 1..8, a ~ N(0,1)."""
    return cosine_modes(n, 3, nmodes, np.random.default_rng(seed))


def kappa_field(n, seed=3, nmodes=16):
    """kappa = exp(0.5 g), g a 16-mode cosine field with amplitudes N(0,1)/4."""
    g = cosine_modes(n, 2, nmodes, np.random.default_rng(seed), scale=0.25)
    return np.exp(0.5 * g)


def adjoint_inputs(n=2048):
    """(kappa, u0, u_target) of the differentiable heat workload (seeds 3, 4, 5)."""
    return kappa_field(n, 3), heat_2d_small(n, 4), heat_2d_small(n, 5)


def grain_init(q=1189, n=512, seed=6, amp=0.001):
    """Order parameters eta_i^0 ~ uniform(-amp, amp), shape (q, n, n), float32."""
    rng = np.random.default_rng(seed)
    out = np.empty((q, n, n), dtype=np.float32)
    for i in range(q):  # one field at a time keeps the float64 draw small
        out[i] = rng.uniform(-amp, amp, (n, n)).astype(np.float32)
    return out


def uneven_sizes(seed=7, count=64, choices=(128, 256, 512, 1024, 2048)):
    """Sizes of the uneven batch: rng.choice(choices, count)."""
    rng = np.random.default_rng(seed)
    return [int(s) for s in rng.choice(np.array(choices), count)]


def uneven_batch(seed=7, count=64, choices=(128, 256, 512, 1024, 2048)):
    """Uneven batch of 2D heat inputs: member b is a 16-mode cosine field of its size
    drawn with seed + 1 + b."""
    sizes = uneven_sizes(seed, count, choices)
    return [cosine_modes(n, 2, 16, np.random.default_rng(seed + 1 + b)) for b, n in enumerate(sizes)]


def random_field(shape, seed, lo=-1.0, hi=1.0):
    """Uniform random field for unit tests."""
    return np.random.default_rng(seed).uniform(lo, hi, shape)


def paper_sine_problem(n, dim=2):
    """The paper's convergence-test problem on [0,1]^dim (Section 3.1): exact solution
    p = prod_axes sin(pi sin(pi x_axis)) on the cell centres and the continuous source
    f = p - Lap p of p - Lap p = f (dt = kappa = 1).  Returns (f, p)."""
    x = centres(n)
    s = np.sin(np.pi * x)
    g = np.sin(np.pi * s)
    # d^2/dx^2 sin(pi sin(pi x)) = -pi^3 sin(pi x) cos(pi s) - pi^4 cos(pi x)^2 sin(pi s)
    g2 = -np.pi ** 3 * s * np.cos(np.pi * s) - np.pi ** 4 * np.cos(np.pi * x) ** 2 * g
    if dim == 2:
        p = np.outer(g, g)
        lap = np.outer(g, g2) + np.outer(g2, g)
    else:
        p = g[:, None, None] * g[None, :, None] * g[None, None, :]
        lap = (g2[:, None, None] * g[None, :, None] * g[None, None, :]
               + g[:, None, None] * g2[None, :, None] * g[None, None, :]
               + g[:, None, None] * g[None, :, None] * g2[None, None, :])
    return p - lap, p
