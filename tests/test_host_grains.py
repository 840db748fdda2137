"""Host-side grain counting of the grain-growth runs (Section 3.3.1) against a plain
breadth-first search over the periodic grid."""
from collections import deque

import numpy as np
import pytest


def _bfs_count(lab):
    ny, nx = lab.shape
    seen = np.zeros_like(lab, dtype=bool)
    grains = 0
    for y in range(ny):
        for x in range(nx):
            if seen[y, x]:
                continue
            grains += 1
            seen[y, x] = True
            dq = deque([(y, x)])
            while dq:
                a, b = dq.popleft()
                for da, db in ((1, 0), (-1, 0), (0, 1), (0, -1)):
                    c, d = (a + da) % ny, (b + db) % nx
                    if not seen[c, d] and lab[c, d] == lab[a, b]:
                        seen[c, d] = True
                        dq.append((c, d))
    return grains


@pytest.mark.parametrize("seed,k,shape", [(0, 2, (16, 16)), (1, 3, (24, 20)), (2, 5, (32, 32)), (3, 2, (9, 14))])
def test_count_grains_matches_bfs(seed, k, shape):
    from paper_2510_11152_amd.grain import count_grains
    rng = np.random.default_rng(seed)
    # blocky random maps (coarse cells repeated), so grains span several cells and wrap
    coarse = rng.integers(0, k, (shape[0] // 2 + 1, shape[1] // 2 + 1))
    lab = np.repeat(np.repeat(coarse, 2, 0), 2, 1)[: shape[0], : shape[1]]
    lab = np.roll(lab, (1, 1), axis=(0, 1))
    g, area = count_grains(lab)
    assert g == _bfs_count(lab)
    assert area == pytest.approx(lab.size / g)


def test_growth_law_fit_recovers_the_exponent():
    """R^m = R0^m + k t sampled exactly: the fit picks m and k back (m = 2 curvature-driven
    growth in 2D, m = 3 for comparison)."""
    from paper_2510_11152_amd.grain_run import fit_growth_law
    t = np.linspace(50.0, 1000.0, 25)
    for m, r0, k in ((2.0, 3.0, 0.5), (3.0, 2.0, 0.2)):
        best, fits = fit_growth_law(t, (r0 ** m + k * t) ** (1.0 / m))
        assert abs(best["m"] - m) < 1e-9 and abs(best["k"] - k) < 1e-9 and best["r2"] > 1 - 1e-12
