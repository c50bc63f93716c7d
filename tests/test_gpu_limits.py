"""Large grids, checked on sampled windows (the oracle computes a window of
the state after K sweeps from a grown copy of that window alone) and on
residuals of whole states.

* A 2D grid whose block columns span 4 GiB or more: the pass kernel keeps
  32-bit lane offsets, so such grids must run the explicit-halo sweep and the
  standalone residual kernel (64-bit offsets), and the adjoint must refuse
  them.  40000 x 27000 FP32 in 2 x 1 blocks: each block stores about 2.2 GB.
* The paper's Jacobi3D domain, 1024 x 1024 x 768, FP32 and FP64.

Windows at domain corners and block seams are bit-exact with the oracle (its
FP32 twin for FP32 runs); the residual of the initial state and of the
device's final state are within 1e-12 of the oracle's FP64 residual of the
same arrays."""
import sys

import numpy as np
import pytest

import oracle
import synthetic
from gpu_util import bits_equal

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def test_wide_block_columns_fall_back(device):
    import torch
    import paper_2303_02543_amd as jb
    nx, ny, K = 40000, 27000, 3
    say("wide grid %dx%d, blocks 2x1, %d sweeps" % (nx, ny, K))
    # seeded tiles repeated over the grid (cheap to build, still irregular)
    ftile = synthetic.uniform((250, 400), 11, -1.0, 1.0).astype(np.float32)
    utile = synthetic.uniform((300, 500), 12, 0.0, 1.0).astype(np.float32)
    f = np.tile(ftile, (ny // 250, nx // 400))
    U0 = np.zeros((ny + 2, nx + 2), dtype=np.float32)
    U0[1:-1, 1:-1] = np.tile(utile, (ny // 300, nx // 500))
    U0[0, :], U0[-1, :], U0[:, 0], U0[:, -1] = 0.5, 1.0, 0.25, 0.75
    h2 = synthetic.spacing2(max(nx, ny))
    s = jb.Solver((nx, ny), (2, 1), torch.float32, device=device)
    try:
        lam = torch.zeros(1, dtype=torch.float32, device=device)
        gb = torch.zeros(1, dtype=torch.float64, device=device)
        with pytest.raises(jb.JacobiError):
            # refused before any device access
            jb.jacobi_adjoint_begin(s.h, lam.data_ptr(), gb.data_ptr())
        s.set_source(torch.from_numpy(f).to(device), h2)
        s.set_state(torch.from_numpy(U0).to(device))
        res = s.solve(K, 1).cpu().numpy()
        got = s.get_state().cpu().numpy()
    finally:
        s.close()
    b = oracle.scale_source(f, h2, np.float32)
    for (x0, x1), (y0, y1) in (((0, 48), (0, 48)), ((19968, 20032), (13000, 13040)),
                               ((39952, 40000), (26952, 27000)), ((19990, 20010), (0, 32))):
        want = oracle.window(U0, b, K, ((x0, x1), (y0, y1)))
        assert bits_equal(got[1 + y0:1 + y1, 1 + x0:1 + x1], want), \
            "window x[%d,%d) y[%d,%d)" % (x0, x1, y0, y1)
    np.testing.assert_allclose(res[0], oracle.residual(U0, b), rtol=1e-12, atol=0)
    np.testing.assert_allclose(res[-1], oracle.residual(got, b), rtol=1e-12, atol=0)


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_paper_domain_3d(device, dtype):
    """The paper's Jacobi3D domain, 1024 x 1024 x 768, in 16 x 16 x 12 blocks
    of 64^3 (Section 4.3's experiment, on one GPU): 6 sweeps with a residual
    every 3; windows at the domain corners, at block seams and inside checked
    bit for bit against the oracle run on those windows alone; residuals of
    the initial and of the device's final state within 1e-12."""
    import torch
    import paper_2303_02543_amd as jb
    nx, ny, nz, K = 1024, 1024, 768, 6
    say("paper domain %dx%dx%d %s, %d sweeps" % (nx, ny, nz, np.dtype(dtype).name, K))
    f = np.tile(synthetic.uniform((48, 64, 64), 13, -1.0, 1.0).astype(dtype), (16, 16, 16))
    U0 = np.zeros((nz + 2, ny + 2, nx + 2), dtype=dtype)
    U0[1:-1, 1:-1, 1:-1] = np.tile(synthetic.uniform((48, 64, 64), 14).astype(dtype),
                                   (16, 16, 16))
    U0[0], U0[-1] = 0.5, 1.0
    U0[:, 0, :], U0[:, -1, :], U0[:, :, 0], U0[:, :, -1] = 0.25, 0.75, 0.125, 0.625
    h2 = synthetic.spacing2(nx)
    tdt = torch.float32 if dtype == np.float32 else torch.float64
    s = jb.Solver((nx, ny, nz), (16, 16, 12), tdt, device=device)
    try:
        s.set_source(torch.from_numpy(f).to(device), h2)
        s.set_state(torch.from_numpy(U0).to(device))
        res = s.solve(K, 3).cpu().numpy()
        got = s.get_state().cpu().numpy()
    finally:
        s.close()
    b = oracle.scale_source(f, h2, dtype)
    for (x0, x1), (y0, y1), (z0, z1) in (((0, 24), (0, 24), (0, 24)),
                                         ((52, 76), (500, 524), (60, 68)),
                                         ((1000, 1024), (1000, 1024), (744, 768)),
                                         ((500, 520), (56, 72), (380, 390))):
        want = oracle.window(U0, b, K, ((x0, x1), (y0, y1), (z0, z1)))
        assert bits_equal(got[1 + z0:1 + z1, 1 + y0:1 + y1, 1 + x0:1 + x1], want), \
            "window x[%d,%d) y[%d,%d) z[%d,%d)" % (x0, x1, y0, y1, z0, z1)
    np.testing.assert_allclose(res[0], oracle.residual(U0, b), rtol=1e-12, atol=0)
    np.testing.assert_allclose(res[-1], oracle.residual(got, b), rtol=1e-12, atol=0)
