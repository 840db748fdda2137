"""Independent checks for the oracle (test infrastructure only).

These are different routes to the same discrete objects, used to pin the oracle:
  * dense assembly of A face by face, then numpy.linalg.solve;
  * DCT-II / DST-II / FFT diagonalisations of the constant-coefficient operator with
    Neumann / Dirichlet / periodic boundaries;
  * the X-MCGS smoother of Section 2.3 / Appendix B written literally as the paper's
    four (2D) or eight (3D) strided sub-block updates in the paper's set order;
  * explicit Gauss-Seidel (D + L)^{-1}(b - U x) under the red-black permutation.
Arrays are shaped (ny, nx) / (nz, ny, nx), x fastest.
"""
import numpy as np
import scipy.fft as sfft


def _cells(P):
    shape = P.shape(0)
    return int(np.prod(shape)), shape


def assemble_dense(P, kap=None):
    """A = I + k * sum_faces w_f (e_a - e_b)(e_a - e_b)^T + k * sum_Dirichlet 2 kappa_p e_p e_p^T,
    k = dt/h^2, w_f = kappa (constant) or the harmonic mean of the two cells."""
    N, shape = _cells(P)
    k = P.dt / (P.h * P.h)
    idx = np.arange(N).reshape(shape)
    kc = np.full(shape, float(P.kappa)) if kap is None else np.asarray(kap, dtype=np.float64)
    A = np.eye(N)
    dim = P.dim
    for axis_x in range(dim):  # axis_x: 0 = x, 1 = y, 2 = z
        ax = dim - 1 - axis_x   # numpy axis
        m = shape[ax]
        for c in range(m):
            lo = np.take(idx, c, axis=ax).ravel()
            klo = np.take(kc, c, axis=ax).ravel()
            if c + 1 < m or P.bc == "periodic":
                cn = (c + 1) % m
                hi = np.take(idx, cn, axis=ax).ravel()
                khi = np.take(kc, cn, axis=ax).ravel()
                if kap is None:
                    w = np.full(lo.shape, float(P.kappa))
                else:
                    w = 2 * klo * khi / (klo + khi)
                for a, b, ww in zip(lo, hi, w):
                    A[a, a] += k * ww
                    A[b, b] += k * ww
                    A[a, b] -= k * ww
                    A[b, a] -= k * ww
        if P.bc == "dirichlet":
            for c in (0, m - 1):
                p = np.take(idx, c, axis=ax).ravel()
                kp = np.take(kc, c, axis=ax).ravel()
                for a, ww in zip(p, kp):
                    A[a, a] += k * 2 * ww
    return A


def dense_solve(P, f, kap=None):
    A = assemble_dense(P, kap)
    return np.linalg.solve(A, f.ravel()).reshape(f.shape)


def _eig1d(m, h, bc):
    k = np.arange(m)
    if bc == "neumann":      # DCT-II modes cos(k pi (i+1/2)/m)
        return (4.0 / h**2) * np.sin(k * np.pi / (2 * m)) ** 2
    if bc == "dirichlet":    # DST-II modes sin((k+1) pi (i+1/2)/m)
        return (4.0 / h**2) * np.sin((k + 1) * np.pi / (2 * m)) ** 2
    if bc == "periodic":     # Fourier modes exp(2 pi i k j/m)
        return (4.0 / h**2) * np.sin(k * np.pi / m) ** 2
    raise ValueError(bc)


def spectral_solve(P, f):
    """Exact discrete solution of the constant-coefficient operator by diagonalisation:
    DCT-II (Neumann), DST-II (Dirichlet, ghost = -adjacent), FFT (periodic)."""
    shape = P.shape(0)
    lam = np.zeros(shape)
    for ax in range(P.dim):
        e = _eig1d(shape[ax], P.h, P.bc)
        s = [1] * P.dim
        s[ax] = shape[ax]
        lam = lam + e.reshape(s)
    denom = 1.0 + P.dt * P.kappa * lam
    if P.bc == "neumann":
        return sfft.idctn(sfft.dctn(f, type=2, norm="ortho") / denom, type=2, norm="ortho")
    if P.bc == "dirichlet":
        return sfft.idstn(sfft.dstn(f, type=2, norm="ortho") / denom, type=2, norm="ortho")
    return np.real(sfft.ifftn(sfft.fftn(f) / denom))


def _padded(P, u):
    """u with a one-cell ghost layer: zeros outside non-periodic boundaries, wrapped
    values for periodic ones."""
    mode = "wrap" if P.bc == "periodic" else "constant"
    return np.pad(u, 1, mode=mode)


def _diag_count(P, shape):
    """Diagonal count W per cell for constant kappa (interior face 1, Dirichlet face 2,
    Neumann face 0)."""
    W = np.zeros(shape, dtype=np.int64)
    for ax in range(P.dim):
        m = shape[ax]
        for side in (0, 1):
            inside = np.ones(shape, dtype=bool)
            if P.bc != "periodic":
                sl = [slice(None)] * P.dim
                sl[ax] = 0 if side == 0 else m - 1
                inside[tuple(sl)] = False
            W += np.where(inside, 1, 2 if P.bc == "dirichlet" else 0)
    return W


def xmcgs_sweep_literal(P, lev, f, u, sets=None):
    """One X-MCGS sweep (constant kappa) as the paper's strided sub-block updates.

    2D sets (1-based i along x, j along y), Section 2.3 / Listing of S:
      1: i odd, j even;  2: i even, j odd;  3: i even, j even;  4: i odd, j odd.
    3D sets (Appendix B; the printed upper bound M_1-1 of sets 3 and 7 read as M_1):
      1: (o,e,e) 2: (e,o,e) 3: (e,e,o) 4: (o,o,o) 5: (o,e,o) 6: (e,o,o) 7: (e,e,e) 8: (o,o,e).
    Each set is updated in one vectorised assignment from the current array, with the
    same per-point evaluation tree as the oracle: (f + k*S) * q[W].
    `sets` overrides the order (a list of parity tuples)."""
    dt = u.dtype.type
    hl = P.h * float(1 << lev)
    kd = P.dt * P.kappa / (hl * hl)
    k = dt(kd)
    q = np.array([1.0 / (1.0 + kd * W) for W in range(16)]).astype(u.dtype)
    shape = u.shape
    W = _diag_count(P, shape)
    if sets is None:
        if P.dim == 2:
            sets = [("o", "e"), ("e", "o"), ("e", "e"), ("o", "o")]
        else:
            sets = [("o", "e", "e"), ("e", "o", "e"), ("e", "e", "o"), ("o", "o", "o"),
                    ("o", "e", "o"), ("e", "o", "o"), ("e", "e", "e"), ("o", "o", "e")]
    for s in sets:
        # 1-based odd index -> 0-based even start; paper order (i, j, l) = (x, y, z)
        starts = [0 if c == "o" else 1 for c in s]
        sl = tuple(slice(starts[a], None, 2) for a in reversed(range(P.dim)))
        up = _padded(P, u)
        if P.dim == 2:
            uW, uE = up[1:-1, :-2], up[1:-1, 2:]
            uS, uN = up[:-2, 1:-1], up[2:, 1:-1]
            S = (uW[sl] + uE[sl]) + (uS[sl] + uN[sl])
        else:
            uW, uE = up[1:-1, 1:-1, :-2], up[1:-1, 1:-1, 2:]
            uS, uN = up[1:-1, :-2, 1:-1], up[1:-1, 2:, 1:-1]
            uB, uT = up[:-2, 1:-1, 1:-1], up[2:, 1:-1, 1:-1]
            S = ((uW[sl] + uE[sl]) + (uS[sl] + uN[sl])) + (uB[sl] + uT[sl])
        u[sl] = (f[sl] + k * S) * q[W[sl]]
    return u


def rb_gauss_seidel_dense(A, b, x, first_odd_1based=True, shape=None):
    """One Gauss-Seidel sweep on the dense system with unknowns ordered red-black, each
    colour lexicographic: x <- (D+L)^{-1}(b - U x).  The colour whose 1-based index sum
    is odd comes first when first_odd_1based, else the other one."""
    N = A.shape[0]
    grids = np.indices(shape) + 1          # 1-based indices
    par = (grids.sum(axis=0) & 1).ravel()
    first = 1 if first_odd_1based else 0
    order = np.concatenate([np.nonzero(par == first)[0], np.nonzero(par != first)[0]])
    Ap = A[np.ix_(order, order)]
    DL = np.tril(Ap)
    U = Ap - DL
    xp = x.ravel()[order]
    bp = b.ravel()[order]
    xn = np.linalg.solve(DL, bp - U @ xp)
    out = np.empty(N)
    out[order] = xn
    return out.reshape(x.shape)


def set_gauss_seidel_dense(A, b, x, sets, shape):
    """One Gauss-Seidel sweep on the dense system with unknowns ordered set by set (each
    set lexicographic): x <- (D+L)^{-1}(b - U x) under that permutation.  sets: parity
    tuples of 1-based indices in (x, y[, z]) order, 'o' odd / 'e' even."""
    grids = np.indices(shape) + 1  # 1-based indices, axes (z,) y, x
    dim = len(shape)
    order = []
    for s in sets:
        sel = np.ones(shape, dtype=bool)
        for a in range(dim):
            idx = grids[dim - 1 - a]  # axis a (x first) is the last array axis
            sel &= (idx % 2 == 1) == (s[a] == "o")
        order.append(np.nonzero(sel.ravel())[0])
    order = np.concatenate(order)
    assert len(order) == A.shape[0]
    Ap = A[np.ix_(order, order)]
    DL = np.tril(Ap)
    U = Ap - DL
    xn = np.linalg.solve(DL, b.ravel()[order] - U @ x.ravel()[order])
    out = np.empty(A.shape[0])
    out[order] = xn
    return out.reshape(x.shape)
