"""jacobi_solve_noalloc (the entry point for callers that cannot allocate
device memory) against the handle path it stands in for: jacobi_create over a
workspace, set_source, set_state, solve, get_state with the same blocks.
Both run the same kernels on the same schedule, so the final states and every
residual must agree bit for bit.  Calls run back to back on one GPU, each
later one on a smaller problem, so what an earlier call left in the shared
scratch array must not leak into a later result; the largest case sits just
under the scratch limit."""
import sys

import numpy as np
import pytest

import synthetic
from gpu_util import bits_equal, first_mismatch, to_device

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def handle_path(U0, f, h2, K, R, blocks, dtype, device):
    import torch
    import paper_2303_02543_amd as jb
    tdt = torch.float32 if dtype == np.float32 else torch.float64
    grid = tuple(reversed([s - 2 for s in U0.shape]))
    s = jb.Solver(grid, blocks, tdt, device=device)
    try:
        if f is not None:
            s.set_source(to_device(f, dtype, device), h2)
        s.set_state(to_device(U0, dtype, device))
        res = s.solve(K, R).cpu().numpy()
        out = s.get_state().cpu().numpy()
        torch.cuda.synchronize()
        return out, res
    finally:
        s.close()


def noalloc_path(U0, f, h2, K, R, blocks, dtype, device):
    import ctypes
    import torch
    import paper_2303_02543_amd as jb
    grid = tuple(reversed([s - 2 for s in U0.shape]))
    u0 = to_device(U0, dtype, device)
    fd = None if f is None else to_device(f, dtype, device)
    out = torch.full_like(u0, float("nan"))
    res = torch.full((jb.residual_count(K, R),), float("nan"), dtype=torch.float64,
                     device=device)
    torch.cuda.synchronize()
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    jb.jacobi_solve_noalloc(len(grid), grid, blocks,
                            jb.JACOBI_F32 if dtype == np.float32 else jb.JACOBI_F64,
                            ctypes.c_void_p(u0.data_ptr()),
                            None if fd is None else ctypes.c_void_p(fd.data_ptr()), h2, K, R,
                            ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(res.data_ptr()),
                            stream)
    torch.cuda.synchronize()
    return out.cpu().numpy(), res.cpu().numpy()


def case(ndim, grid, seed):
    """Seeded Poisson case: U[0,1) interior, ring from another seed, Gaussian
    source (2D) or U[-1,1) source (3D)."""
    shape = tuple(reversed(grid))
    U0 = synthetic.state_with_ring(synthetic.uniform(shape, seed),
                                   synthetic.uniform(tuple(s + 2 for s in shape), seed + 1))
    if ndim == 2 and grid[0] == grid[1]:
        f = synthetic.gaussian_sum(grid[0], 2, seed + 2)
    else:
        f = synthetic.uniform(shape, seed + 2, -1.0, 1.0)
    return U0, f, synthetic.spacing2(max(grid))


# (grid, blocks, dtype, sweeps, check interval): the first sits just under
# the scratch limit (2048^2 FP32 in 4x4 blocks); each later one is smaller
SEQUENCE = [
    ((2048, 2048), (4, 4), np.float32, 60, 25),
    ((700, 433), (3, 2), np.float32, 41, 10),
    ((90, 70, 50), (2, 2, 1), np.float64, 9, 4),
    ((37, 29), (3, 4), np.float64, 13, 5),
]


def test_noalloc_matches_handle_path(device):
    import paper_2303_02543_amd as jb
    for i, (grid, blocks, dtype, K, R) in enumerate(SEQUENCE):
        nbytes = jb.jacobi_workspace_bytes(len(grid), grid, blocks,
                                           jb.JACOBI_F32 if dtype == np.float32 else jb.JACOBI_F64)
        assert nbytes <= jb.JACOBI_NOALLOC_MAX_BYTES
        say("noalloc case %d: grid %s blocks %s %s K=%d R=%d (%d bytes)"
            % (i, grid, blocks, np.dtype(dtype).name, K, R, nbytes))
        U0, f, h2 = case(len(grid), grid, 50 + 10 * i)
        want, want_res = handle_path(U0, f, h2, K, R, blocks, dtype, device)
        got, got_res = noalloc_path(U0, f, h2, K, R, blocks, dtype, device)
        assert bits_equal(got, want), "case %d: state differs, first %s" % (
            i, first_mismatch(got, want))
        assert bits_equal(got_res, want_res), "case %d: residuals %s vs %s" % (
            i, got_res, want_res)
    # a Laplace call (no source) after the Poisson ones
    U0 = synthetic.laplace2d_top_edge(n=96, seed=3)
    want, want_res = handle_path(U0, None, 0.0, 17, 6, (2, 3), np.float64, device)
    got, got_res = noalloc_path(U0, None, 0.0, 17, 6, (2, 3), np.float64, device)
    assert bits_equal(got, want)
    assert bits_equal(got_res, want_res)


def test_noalloc_refuses_too_large(device):
    import ctypes
    import torch
    import paper_2303_02543_amd as jb
    u = torch.zeros(8, dtype=torch.float32, device=device)
    p = ctypes.c_void_p(u.data_ptr())
    with pytest.raises(jb.JacobiError) as ei:
        jb.jacobi_solve_noalloc(2, (4096, 4096), (8, 8), jb.JACOBI_F32, p, p, 1e-6, 1, 1, p, p,
                                None)
    assert ei.value.status == jb.JACOBI_E_NOMEM
    assert "scratch" in str(ei.value)
