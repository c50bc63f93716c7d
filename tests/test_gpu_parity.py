"""Device path vs the oracle, element by element, through the C ABI.

FP64 runs must equal the FP64 oracle bit for bit, FP32 runs the FP32 twin of
the oracle bit for bit (same operations in the same order); FP32 runs must be
within 1e-5 norm-relative of the FP64 oracle; residuals within 1e-12 relative.
Sizes span several blocks, several tiles and ragged tails."""
import math
import sys

import numpy as np
import pytest

import oracle
import synthetic
from gpu_util import (bits_equal, first_mismatch, norm_rel_err, oracle_residuals, oracle_run,
                      run_device)

pytestmark = pytest.mark.gpu

RNG = np.random.default_rng(2024)


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def assert_bits(got, want, what):
    if not bits_equal(got, want):
        mm = first_mismatch(got, want)
        raise AssertionError("%s: not bit-exact; first mismatch %s" % (what, mm))


# ------------------------------------------- 256^2 Laplace FP64, 2x2 blocks
@pytest.mark.parametrize("depth,flags", [(1, 0), (2, 0), (3, 0), (4, 0), (1, 1), (1, 9)])
def test_laplace256_fp64_bit_exact(device, depth, flags):
    """2D Laplace 256^2 FP64, 2x2 blocks of 128^2, 100 sweeps, residual every 10:
    bit-exact with the monolithic oracle; residuals within 1e-12."""
    say("laplace 256^2 depth=%d flags=%d" % (depth, flags))
    U0 = synthetic.laplace2d_top_edge()
    got, res = run_device(U0, None, 0.0, 100, (2, 2), np.float64, device, depth=depth,
                          flags=flags, check_every=10)
    want = oracle.sweep(U0, None, 100)
    assert_bits(got, want, "laplace 256^2")
    ores, _ = oracle_residuals(U0, None, 100, 10)
    np.testing.assert_allclose(res, ores, rtol=1e-12, atol=0)


# ------------------------------------------------------- small 2D, all depths
CASES_2D = [
    # (nx, ny, bx, by, K)
    (37, 29, 3, 4, 13),
    (300, 41, 2, 3, 9),
    (1000, 13, 5, 2, 17),
    (8, 8, 1, 1, 7),
    (1, 1, 1, 1, 3),
    (2, 77, 1, 7, 11),
    (513, 260, 3, 5, 25),
]


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("case", CASES_2D)
def test_2d_bit_exact_all_depths(device, dtype, case):
    import paper_2303_02543_amd as jb
    nx, ny, bx, by, K = case
    U0 = RNG.uniform(0, 1, (ny + 2, nx + 2))
    f = RNG.standard_normal((ny, nx)) * 100
    h2 = synthetic.spacing2(max(nx, ny))
    want, _ = oracle_run(U0, f, h2, K, dtype)
    want_l, _ = oracle_run(U0, None, h2, K, dtype)
    code = jb.JACOBI_F32 if dtype == np.float32 else jb.JACOBI_F64
    depths = list(range(1, jb.jacobi_max_depth(2, code) + 1))
    for depth in depths:
        for rows in (0, 8, 64):
            for fl in (0, jb.JACOBI_FLAG_NT_STORES):
                say("2d case=%s dtype=%s depth=%d rows=%d flags=%d"
                    % (case, np.dtype(dtype).name, depth, rows, fl))
                got, _ = run_device(U0, f, h2, K, (bx, by), dtype, device, depth=depth, rows=rows,
                                    flags=fl)
                assert_bits(got, want, "2d %s depth %d rows %d flags %d" % (case, depth, rows, fl))
    for fl in (0, jb.JACOBI_FLAG_NT_STORES):
        got, _ = run_device(U0, None, h2, K, (bx, by), dtype, device, depth=depths[-1], flags=fl)
        assert_bits(got, want_l, "2d laplace %s flags %d" % (case, fl))
    for rg in (0, 1, 3, 5, 64):
        # explicit exchange + block-local sweep; rows = rows per work item
        got, _ = run_device(U0, f, h2, K, (bx, by), dtype, device, rows=rg,
                            flags=jb.JACOBI_FLAG_EXPLICIT_HALO)
        assert_bits(got, want, "2d explicit halo %s rows %d" % (case, rg))
    got, _ = run_device(U0, None, h2, K, (bx, by), dtype, device, rows=3,
                        flags=jb.JACOBI_FLAG_EXPLICIT_HALO)
    assert_bits(got, want_l, "2d explicit halo laplace %s" % (case,))
    for rg in (0, 3):
        # slabs swept and their faces sent on a second stream, overlapped
        got, _ = run_device(U0, f, h2, K, (bx, by), dtype, device, rows=rg,
                            flags=jb.JACOBI_FLAG_EXPLICIT_HALO | jb.JACOBI_FLAG_OVERLAP)
        assert_bits(got, want, "2d overlapped explicit halo %s rows %d" % (case, rg))
    got, _ = run_device(U0, f, h2, K, (bx, by), dtype, device, depth=depths[-1],
                        flags=jb.JACOBI_FLAG_NT_STORES)
    assert_bits(got, want, "2d non-temporal stores %s" % (case,))


# The 2D pass tiling: inner strips get an edge band of hb rows at the top and
# the bottom and tiles of `rows` rows between, outer strips tiles of ho rows,
# with h = max(min(rows, 8), (rows + 2T) * F // 16 - 2T), capped at ny, F = 13
# for hb and 11 for ho.  Tiles of a strip that reaches the ring in x run the
# step with row and column tests, the other tiles that reach it in y the step
# with row tests only.  FP32 strips hold 248 output columns at depth 4 and
# 232 at depth 13.
BAND_CASES = [
    # (nx, ny, bx, by, depth, rows): the tiling case it reaches
    (700, 20, 3, 2, 4, 40),   # 3 strips; ny <= hb (31, capped at 20): one band per inner strip
    (700, 40, 3, 4, 4, 40),   # hb < ny <= 2 hb: a top band and a bottom band only
    (700, 143, 3, 4, 4, 40),  # bands of 31, middle tiles of 40, 40 and a 1-row tail
    (100, 131, 2, 3, 4, 40),  # one strip: outer-strip tiles only
    (300, 131, 2, 3, 4, 40),  # two strips: outer-strip tiles only
    (700, 131, 3, 4, 13, 8),  # depth 13, hb and ho clamped to 8 rows
    (1200, 300, 4, 3, 13, 60),  # six strips, hb = 43, ho = 33, ragged middle tile
    (497, 131, 3, 4, 4, 40),  # the last strip 1 column wide: the inner strip reaches the ring in x
    (470, 131, 2, 3, 13, 40),  # the same at depth 13 (the last strip 6 columns wide)
]


@pytest.mark.parametrize("case", BAND_CASES)
def test_2d_edge_band_tiling(device, case):
    """Every tiling case of the 2D pass (band-only strips, bands with and
    without middle tiles, a ragged middle tile, one and two strips): FP32
    states bit-exact with the oracle's FP32 twin, with the residual folded
    into the passes, for Poisson and Laplace."""
    nx, ny, bx, by, depth, rows = case
    U0 = RNG.uniform(0, 1, (ny + 2, nx + 2))
    f = RNG.standard_normal((ny, nx)) * 100
    h2 = synthetic.spacing2(max(nx, ny))
    K = 2 * depth + 3
    for src in (f, None):
        want, b = oracle_run(U0, src, h2, K, np.float32)
        ores, _ = oracle_residuals(np.asarray(U0, dtype=np.float32), b, K, depth)
        say("2d band tiling case=%s source=%s" % (case, src is not None))
        got, res = run_device(U0, src, h2, K, (bx, by), np.float32, device, depth=depth,
                              rows=rows, check_every=depth)
        assert_bits(got, want, "2d band tiling %s" % (case,))
        np.testing.assert_allclose(res, ores, rtol=1e-12, atol=0)


# 6: non-temporal stores, and the prefetch flag (accepted, no effect)
@pytest.mark.parametrize("flags", [0, 6])
@pytest.mark.parametrize("case", [(37, 29, 3, 4, 13), (513, 260, 3, 5, 25), (1, 1, 1, 1, 3)])
def test_2d_residuals_and_states(device, case, flags):
    """solve() with a residual every 4 sweeps (the residual folded into the
    first pass of each interval): states bit-exact with the FP32 oracle twin,
    residuals within 1e-12 of the FP64 residuals of the oracle's states, for
    Poisson and Laplace, at the deepest depth and at depth 3."""
    import paper_2303_02543_amd as jb
    nx, ny, bx, by, K = case
    U0 = RNG.uniform(0, 1, (ny + 2, nx + 2))
    f = RNG.standard_normal((ny, nx)) * 100
    h2 = synthetic.spacing2(max(nx, ny))
    for src in (f, None):
        want, b = oracle_run(U0, src, h2, K, np.float32)
        ores, _ = oracle_residuals(np.asarray(U0, dtype=np.float32), b, K, 4)
        for depth in (1, 3, jb.jacobi_max_depth(2, jb.JACOBI_F32)):
            say("2d residuals case=%s depth=%d flags=%d source=%s"
                % (case, depth, flags, src is not None))
            got, res = run_device(U0, src, h2, K, (bx, by), np.float32, device, depth=depth,
                                  flags=flags, check_every=4)
            assert_bits(got, want, "2d %s depth %d flags %d" % (case, depth, flags))
            np.testing.assert_allclose(res, ores, rtol=1e-12, atol=0)


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("case", CASES_2D)
def test_2d_plain_sweep_residuals(device, dtype, case):
    """One sweep per pass (the tile kernel reading block-edge neighbours from
    their owning blocks) with the residual every 3 sweeps folded into it:
    states bit-exact with the oracle, residuals within 1e-12; the explicit
    halo order agrees bit for bit."""
    import paper_2303_02543_amd as jb
    nx, ny, bx, by, K = case
    U0 = RNG.uniform(0, 1, (ny + 2, nx + 2))
    f = RNG.standard_normal((ny, nx)) * 100
    h2 = synthetic.spacing2(max(nx, ny))
    for src in (f, None):
        want, b = oracle_run(U0, src, h2, K, dtype)
        ores, _ = oracle_residuals(np.asarray(U0, dtype=dtype), b, K, 3)
        for flags in (0, jb.JACOBI_FLAG_EXPLICIT_HALO):
            say("2d plain residuals case=%s dtype=%s flags=%d source=%s"
                % (case, np.dtype(dtype).name, flags, src is not None))
            got, res = run_device(U0, src, h2, K, (bx, by), dtype, device, depth=1, flags=flags,
                                  check_every=3)
            assert_bits(got, want, "2d plain %s flags %d" % (case, flags))
            np.testing.assert_allclose(res, ores, rtol=1e-12, atol=0)


# --------------------------------------------------------------- small 3D
CASES_3D = [
    (16, 16, 16, 2, 2, 2, 5),
    (13, 9, 11, 1, 2, 3, 7),
    (40, 3, 5, 2, 1, 1, 4),
    (300, 20, 17, 3, 2, 2, 6),
    (1, 1, 1, 1, 1, 1, 2),
    (130, 45, 70, 3, 3, 2, 9),   # several strips, row groups and z segments, ragged
]


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("case", CASES_3D)
def test_3d_bit_exact(device, dtype, case):
    """3D passes of every depth (1 .. the largest) and z segment, the
    explicit-halo and overlapped orders: states bit-exact with the oracle,
    residuals (folded into the first pass of each interval) within 1e-12."""
    nx, ny, nz, bx, by, bz, K = case
    U0 = RNG.uniform(0, 1, (nz + 2, ny + 2, nx + 2))
    f = RNG.uniform(-1, 1, (nz, ny, nx))
    h2 = synthetic.spacing2(max(case[:3]))
    import paper_2303_02543_amd as jb
    code = jb.JACOBI_F32 if dtype == np.float32 else jb.JACOBI_F64
    want, _ = oracle_run(U0, f, h2, K, dtype)
    b = oracle.scale_source(np.asarray(f, dtype=dtype), h2, dtype)
    ores, _ = oracle_residuals(np.asarray(U0, dtype=dtype), b, K, 4)
    scheds = [(d, rows, 0) for d in range(1, jb.jacobi_max_depth(3, code) + 1)
              for rows in (0, 8, 64)]
    scheds += [(2, 16, jb.JACOBI_FLAG_NT_STORES), (1, 0, jb.JACOBI_FLAG_EXPLICIT_HALO),
               (1, 0, jb.JACOBI_FLAG_EXPLICIT_HALO | jb.JACOBI_FLAG_OVERLAP)]
    for depth, rows, flags in scheds:
        say("3d case=%s dtype=%s depth=%d rows=%d flags=%d"
            % (case, np.dtype(dtype).name, depth, rows, flags))
        got, _ = run_device(U0, f, h2, K, (bx, by, bz), dtype, device, depth=depth, rows=rows,
                            flags=flags)
        assert_bits(got, want, "3d %s depth %d rows %d flags %d" % (case, depth, rows, flags))
        got, res = run_device(U0, f, h2, K, (bx, by, bz), dtype, device, depth=depth, rows=rows,
                              flags=flags, check_every=4)
        assert_bits(got, want, "3d solve %s depth %d rows %d flags %d" % (case, depth, rows, flags))
        np.testing.assert_allclose(res, ores, rtol=1e-12, atol=0)
    want_l, _ = oracle_run(U0, None, h2, K, dtype)
    for depth in range(1, jb.jacobi_max_depth(3, code) + 1):
        got_l, _ = run_device(U0, None, h2, K, (bx, by, bz), dtype, device, depth=depth)
        assert_bits(got_l, want_l, "3d laplace %s depth %d" % (case, depth))


# ------------------------------------------------ FP32 against the FP64 oracle
def test_fp32_within_1e5_of_fp64_oracle(device):
    """Gaussian-source Poisson, FP32 inputs widened for the FP64 oracle."""
    import paper_2303_02543_amd as jb
    n, K = 511, 400
    f64 = synthetic.gaussian_sum(n, 2, 2)
    f32 = f64.astype(np.float32)
    U0 = np.zeros((n + 2, n + 2))
    h2 = synthetic.spacing2(n)
    say("fp32 vs fp64 n=%d K=%d" % (n, K))
    got, res = run_device(U0, f32, h2, K, (4, 4), np.float32, device,
                          depth=jb.jacobi_max_depth(2, jb.JACOBI_F32), check_every=50)
    b64 = oracle.scale_source(f32.astype(np.float64), h2, np.float64)
    want = oracle.sweep(U0, b64, K)
    err = norm_rel_err(got, want)
    say("fp32 rel err %.3e" % err)
    assert err <= 1e-5
    # the residual of the FP32 state, computed by the oracle from the same
    # state, matches the device's FP64 residual
    b32 = oracle.scale_source(f32, h2, np.float32)
    assert math.isclose(res[-1], oracle.residual(got.astype(np.float32), b32), rel_tol=1e-12)


# ------------------------------------------------------- state and residual
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_set_get_state_round_trip_and_residual(device, dtype):
    import torch
    import paper_2303_02543_amd as jb
    for ndim, grid, blocks in [(2, (45, 31), (3, 2)), (3, (17, 12, 9), (2, 3, 2))]:
        shape = tuple(n + 2 for n in reversed(grid))
        U = RNG.uniform(-1, 1, shape).astype(dtype)
        f = RNG.uniform(-1, 1, tuple(reversed(grid))).astype(dtype)
        tdt = torch.float32 if dtype == np.float32 else torch.float64
        s = jb.Solver(grid, blocks, tdt, device=device)
        try:
            s.set_state(torch.from_numpy(U).to(device))
            back = s.get_state().cpu().numpy()
            assert_bits(back, U, "round trip %s" % (grid,))   # ring corners included
            h2 = 1e-3
            s.set_source(torch.from_numpy(f).to(device), h2)
            r1 = s.residual()
            r2 = s.residual()
            assert r1 == r2                                   # deterministic
            b = oracle.scale_source(f, h2, dtype)
            assert math.isclose(r1, oracle.residual(U, b), rel_tol=1e-12)
            s.halo_exchange()
            s.halo_exchange()
            assert_bits(s.get_state().cpu().numpy(), U, "halo exchange is idempotent")
            s.set_source(None, 1.0)
            assert math.isclose(s.residual(), oracle.residual(U, None), rel_tol=1e-12)
        finally:
            s.close()


def test_poisoned_workspace_does_not_leak(device):
    """Fill the whole workspace with NaN before set_state: any read of a cell
    that the scatter / halo exchange / sweep should have written first would
    surface as NaN in the result."""
    import torch
    import paper_2303_02543_amd as jb
    nx, ny, K = 203, 150, 12
    U0 = RNG.uniform(0, 1, (ny + 2, nx + 2))
    f = RNG.standard_normal((ny, nx))
    h2 = synthetic.spacing2(nx)
    want, _ = oracle_run(U0, f, h2, K, np.float32)
    for depth, flags in [(1, 0), (3, 0), (8, 0), (1, 1)]:
        s = jb.Solver((nx, ny), (3, 4), torch.float32, device=device)
        try:
            s.workspace.view(torch.float32)[:].fill_(float("nan"))
            s.set_tuning(depth, 8, flags)
            s.set_state(torch.from_numpy(U0.astype(np.float32)).to(device))
            s.set_source(torch.from_numpy(f.astype(np.float32)).to(device), h2)
            s.sweep(K)
            got = s.get_state().cpu().numpy()
            assert_bits(got, want, "poisoned depth %d flags %d" % (depth, flags))
            assert np.isfinite(s.residual())
        finally:
            s.close()


def test_errors_on_device(device):
    import torch
    import paper_2303_02543_amd as jb
    s = jb.Solver((16, 16), (2, 2), torch.float64, device=device)
    try:
        with pytest.raises(jb.JacobiError) as ei:
            s.sweep(1)
        assert ei.value.status == jb.JACOBI_E_STATE
        with pytest.raises(jb.JacobiError):
            s.residual()
        s.set_state(torch.zeros((18, 18), dtype=torch.float64, device=device))
        with pytest.raises(jb.JacobiError) as ei:
            s.sweep(-1)
        assert ei.value.status == jb.JACOBI_E_INVAL
        s.sweep(0)
        with pytest.raises(jb.JacobiError):
            s.set_tuning(99, 0, 0)
        with pytest.raises(jb.JacobiError) as ei:
            s.set_tuning(1, 0, jb.JACOBI_FLAG_OVERLAP)  # needs the explicit-halo flag
        assert ei.value.status == jb.JACOBI_E_INVAL
        with pytest.raises(jb.JacobiError):
            s.set_tuning(1, 0, 64)  # unknown flag bit
        with pytest.raises(jb.JacobiError):
            s.set_source(torch.zeros((16, 16), dtype=torch.float64, device=device), -1.0)
        assert s.residual() == 0.0
    finally:
        s.close()
    # a CPU tensor is refused as workspace memory
    L = jb.lib()
    import ctypes
    t = torch.empty(1 << 20, dtype=torch.uint8)
    out = ctypes.c_void_p()
    rc = L.jacobi_create(2, jb._arr64([8, 8]), jb._arr64([1, 1]), 0,
                         ctypes.c_void_p((t.data_ptr() + 255) // 256 * 256), (1 << 20) - 256, None,
                         ctypes.byref(out))
    assert rc in (jb.JACOBI_E_INVAL, jb.JACOBI_E_HIP)
