"""Deep-halo block storage (every block keeps an H-deep frame, exchanged once
per pass of up to H sweeps, each pass block-local) against the oracle: the
final states bit-exact with the oracle's block-decomposed sweep on the
device's own block boundaries (and with the monolithic sweep), residuals
within 1e-12, for 2D and 3D, FP32 and FP64, every frame depth the shapes
allow, several pass depths and tile heights, Poisson and Laplace."""
import sys

import numpy as np
import pytest

import oracle
import synthetic
from gpu_util import bits_equal, first_mismatch, oracle_residuals, to_device

pytestmark = pytest.mark.gpu

RNG = np.random.default_rng(777)


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def run_deep(U0, f, h2, K, blocks, dtype, device, halo, depth=0, rows=0, flags=0,
             check_every=None):
    import torch
    import paper_2303_02543_amd as jb
    tdt = torch.float32 if dtype == np.float32 else torch.float64
    grid = tuple(reversed([s - 2 for s in U0.shape]))
    s = jb.Solver(grid, blocks, tdt, device=device, halo=halo)
    try:
        s.set_tuning(depth, rows, flags)
        s.set_state(to_device(U0, dtype, device))
        if f is not None:
            s.set_source(to_device(f, dtype, device), h2)
        res = None
        if check_every is None:
            s.sweep(K)
        else:
            res = s.solve(K, check_every).cpu().numpy()
        out = s.get_state().cpu().numpy()
        (nb3, ext3) = s.layout()
        hs = s.halo()
        torch.cuda.synchronize()
        return out, res, nb3, ext3, hs
    finally:
        s.close()


def starts_of(n, nb, e):
    return np.array([min(q * e, n) for q in range(nb)] + [n], dtype=np.int64)


def check(got, want, what):
    assert bits_equal(got, want), "%s: first mismatch %s" % (what, first_mismatch(got, want))


CASES_2D = [
    # (nx, ny, bx, by, K, halos)
    (300, 41, 2, 3, 29, (1, 2, 5, 9, 13)),
    (37, 29, 3, 4, 17, (1, 3, 5)),
    (1000, 130, 4, 3, 31, (4, 13)),
    (8, 8, 1, 1, 7, (1, 5, 13)),      # one block: no exchange partner at all
    (513, 260, 3, 5, 26, (2, 6)),
]


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("case", CASES_2D)
def test_deep_2d_bit_exact(device, dtype, case):
    import paper_2303_02543_amd as jb
    nx, ny, bx, by, K, halos = case
    U0 = RNG.uniform(0, 1, (ny + 2, nx + 2))
    f = RNG.standard_normal((ny, nx)) * 100
    h2 = synthetic.spacing2(max(nx, ny))
    code = jb.JACOBI_F32 if dtype == np.float32 else jb.JACOBI_F64
    want, b = None, None
    for halo in halos:
        try:
            jb.jacobi_deep_workspace_bytes(2, (nx, ny), (bx, by), code, halo)
        except jb.JacobiError as e:
            say("2d deep case=%s halo=%d refused: %s" % (case, halo, e))
            assert e.status == jb.JACOBI_E_INVAL and "exceeds the block extent" in str(e)
            continue
        for depth, rows in ((0, 0), (1, 0), (3, 8), (halo, 0), (16, 64)):
            if depth > jb.jacobi_max_depth(2, code):
                continue
            say("2d deep case=%s dtype=%s halo=%d depth=%d rows=%d"
                % (case, np.dtype(dtype).name, halo, depth, rows))
            got, res, nb3, ext3, hs = run_deep(U0, f, h2, K, (bx, by), dtype, device, halo,
                                              depth=depth, rows=rows, check_every=5)
            assert hs >= halo and (hs - 1) % (16 // np.dtype(dtype).itemsize) == 0
            if want is None:
                b = oracle.scale_source(np.asarray(f, dtype=dtype), h2, dtype)
                starts = [starts_of(nx, nb3[0], ext3[0]), starts_of(ny, nb3[1], ext3[1])]
                want = oracle.blocked_sweep(np.asarray(U0, dtype=dtype), b, K, starts)
                assert bits_equal(want, oracle.sweep(np.asarray(U0, dtype=dtype), b, K))
                ores, _ = oracle_residuals(np.asarray(U0, dtype=dtype), b, K, 5)
            check(got, want, "2d deep %s halo %d depth %d rows %d" % (case, halo, depth, rows))
            np.testing.assert_allclose(res, ores, rtol=1e-12, atol=0)
        # Laplace, and the one-cell explicit exchange on the same storage
        want_l = oracle.sweep(np.asarray(U0, dtype=dtype), None, K)
        got_l, _, _, _, _ = run_deep(U0, None, h2, K, (bx, by), dtype, device, halo)
        check(got_l, want_l, "2d deep laplace %s halo %d" % (case, halo))
        got_e, _, _, _, _ = run_deep(U0, f, h2, K, (bx, by), dtype, device, halo, depth=1,
                                     flags=jb.JACOBI_FLAG_EXPLICIT_HALO)
        check(got_e, want, "2d deep storage, explicit halo %s halo %d" % (case, halo))


CASES_3D = [
    # (nx, ny, nz, bx, by, bz, K, halos)
    (40, 33, 29, 2, 2, 2, 11, (1, 3, 4, 5)),
    (130, 45, 70, 2, 3, 2, 9, (2, 5, 9)),
    (13, 9, 11, 1, 1, 1, 6, (1, 4)),
    (64, 64, 64, 2, 2, 2, 13, (4,)),
]


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("case", CASES_3D)
def test_deep_3d_bit_exact(device, dtype, case):
    import paper_2303_02543_amd as jb
    nx, ny, nz, bx, by, bz, K, halos = case
    U0 = RNG.uniform(0, 1, (nz + 2, ny + 2, nx + 2))
    f = RNG.uniform(-1, 1, (nz, ny, nx))
    h2 = synthetic.spacing2(max(nx, ny, nz))
    code = jb.JACOBI_F32 if dtype == np.float32 else jb.JACOBI_F64
    want = None
    for halo in halos:
        try:
            jb.jacobi_deep_workspace_bytes(3, (nx, ny, nz), (bx, by, bz), code, halo)
        except jb.JacobiError as e:
            say("3d deep case=%s halo=%d refused: %s" % (case, halo, e))
            assert e.status == jb.JACOBI_E_INVAL
            continue
        for depth, rows in ((0, 0), (1, 8), (2, 16), (4, 0)):
            say("3d deep case=%s dtype=%s halo=%d depth=%d rows=%d"
                % (case, np.dtype(dtype).name, halo, depth, rows))
            got, res, nb3, ext3, hs = run_deep(U0, f, h2, K, (bx, by, bz), dtype, device, halo,
                                              depth=depth, rows=rows, check_every=4)
            if want is None:
                b = oracle.scale_source(np.asarray(f, dtype=dtype), h2, dtype)
                starts = [starts_of(n, nb3[a], ext3[a]) for a, n in enumerate((nx, ny, nz))]
                want = oracle.blocked_sweep(np.asarray(U0, dtype=dtype), b, K, starts)
                ores, _ = oracle_residuals(np.asarray(U0, dtype=dtype), b, K, 4)
            check(got, want, "3d deep %s halo %d depth %d rows %d" % (case, halo, depth, rows))
            np.testing.assert_allclose(res, ores, rtol=1e-12, atol=0)
        want_l = oracle.sweep(np.asarray(U0, dtype=dtype), None, K)
        got_l, _, _, _, _ = run_deep(U0, None, h2, K, (bx, by, bz), dtype, device, halo)
        check(got_l, want_l, "3d deep laplace %s halo %d" % (case, halo))


def test_deep_8192_default_schedule(device):
    """The bench's deep-halo form at full size: 8192^2 FP32 in 16x16 blocks of
    512^2, frames of 13, 50 sweeps with a residual every 50 (passes of 13, 13,
    12, 12) bit-exact with the FP32 oracle and its residuals."""
    n, K = 8192, 50
    U0, f = synthetic.poisson2d_gaussians(n)
    U0 = U0.astype(np.float32)
    f = f.astype(np.float32)
    h2 = synthetic.spacing2(n)
    got, res, _, _, hs = run_deep(U0, f, h2, K, (16, 16), np.float32, device, 13,
                                  check_every=50)
    assert hs == 13
    b = oracle.scale_source(f, h2, np.float32)
    want = oracle.sweep(U0, b, K)
    check(got, want, "8192^2 deep halo 13")
    np.testing.assert_allclose(res, [oracle.residual(U0, b), oracle.residual(want, b)],
                               rtol=1e-12, atol=0)
