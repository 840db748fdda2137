"""fas_solve_noalloc (the solve whose workspace is the library's static device buffer,
for callers that cannot allocate) against fas_solve on a caller-allocated workspace:
the same kernels on the same inputs, so the same cycle count and identical bits.  Two
calls in a row, the second on a smaller grid, so the second reuses a buffer that the
first left filled."""
import ctypes

import numpy as np
import pytest
import torch

import fas_inputs as I

pytestmark = pytest.mark.gpu

DEV = "cuda"


def _noalloc(L, F, n, h, bc, dtype, coarsest, dt, kappa, kcell, rhs, u, tol, kmax=100):
    n3 = (ctypes.c_int64 * 3)(*(list(n) + [1] * (3 - len(n))))
    cyc = ctypes.c_int(0)
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    st = L.fas_solve_noalloc(len(n), n3, h, F.FAS_BC[bc], dtype, coarsest, stream, dt, kappa,
                             None if kcell is None else ctypes.c_void_p(kcell.data_ptr()),
                             ctypes.c_void_p(rhs.data_ptr()), ctypes.c_void_p(u.data_ptr()), tol, 2, 2, kmax,
                             ctypes.byref(cyc))
    return st, cyc.value


def _reference(n, h, bc, tdtype, coarsest, dt, kappa, kcell, rhs, u0, tol):
    from paper_2510_11152_amd import Grid
    g = Grid(n, h, bc=bc, dtype=tdtype, coarsest=coarsest, variable_kappa=kcell is not None, device=DEV)
    u = u0.clone()
    st = g.solve(rhs, u, dt, kappa=kappa, kappa_cell=kcell, tol=tol)
    return st, g.stats()["cycles"], u


CASES = [  # (n, bc, dtype, coarsest, dt, variable kappa) for the first and the second, smaller call
    (((2048, 2048), "neumann", torch.float64, 4, 1e-4, False), ((256, 256), "neumann", torch.float64, 4, 1e-3, False)),
    (((1024, 512), "dirichlet", torch.float64, 4, 0.05, True), ((128, 64), "periodic", torch.float32, 4, 0.05, False)),
    (((128, 128, 128), "neumann", torch.float64, 4, 1e-3, False), ((32, 32, 32), "periodic", torch.float64, 4, 0.1, True)),
]


@pytest.mark.parametrize("first,second", CASES)
def test_noalloc_equals_solve_twice(first, second):
    from paper_2510_11152_amd import _lib as F
    L = F.load()
    for k, (n, bc, tdtype, coarsest, dt, variable) in enumerate((first, second)):
        h = 1.0 / n[0]
        shape = tuple(reversed(n))
        rhs = torch.from_numpy(I.random_field(shape, 40 + k)).to(DEV, tdtype)
        kcell = torch.from_numpy(np.exp(0.5 * I.random_field(shape, 50 + k))).to(DEV, tdtype) if variable else None
        tol = 1e-10 if tdtype == torch.float64 else 1e-5
        st_ref, cyc_ref, u_ref = _reference(n, h, bc, tdtype, coarsest, dt, 0.9, kcell, rhs, rhs, tol)
        u = rhs.clone()
        dcode = F.FAS_F64 if tdtype == torch.float64 else F.FAS_F32
        st, cyc = _noalloc(L, F, n, h, bc, dcode, coarsest, dt, 0.9, kcell, rhs, u, tol)
        torch.cuda.synchronize()
        print("noalloc call %d: n=%s bc=%s %s status %d/%d cycles %d/%d" % (k, n, bc, tdtype, st, st_ref, cyc, cyc_ref),
              flush=True)
        assert st == 0 and st_ref == 0
        assert cyc == cyc_ref
        assert torch.equal(u, u_ref)


def test_noalloc_rejects_a_grid_beyond_the_buffer():
    from paper_2510_11152_amd import _lib as F
    L = F.load()
    n = (4096, 4096)
    rhs = torch.zeros((1, 1), dtype=torch.float64, device=DEV)  # never touched: rejected first
    u = torch.zeros((1, 1), dtype=torch.float64, device=DEV)
    st, _ = _noalloc(L, F, n, 1.0 / 4096, "neumann", F.FAS_F64, 4, 1e-4, 1.0, None, rhs, u, 1e-10)
    assert st == F.FAS_ERR_NOMEM
    assert b"static buffer" in L.fas_last_error()
