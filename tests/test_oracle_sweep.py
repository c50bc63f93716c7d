"""Pins of the oracle's sweep (5-point / 7-point Jacobi update, Section 4.3 of
the paper) against facts fixed by mathematics, not by the oracle's own code:
fixed points, exact eigenmode decay, symmetry, a dense-matrix form built with
numpy, a closed-form Poisson transient, the contraction bound toward the direct
solve, and block decomposition = monolithic bit for bit."""
import math

import numpy as np
import pytest

import oracle
import synthetic

RNG = np.random.default_rng(12345)


def bits_equal(a, b):
    a = np.ascontiguousarray(a)
    b = np.ascontiguousarray(b)
    return a.dtype == b.dtype and a.shape == b.shape and np.array_equal(
        a.view(np.uint8), b.view(np.uint8))


# --------------------------------------------------------------- fixed points
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_constant_field_is_fixed_point_2d(dtype):
    # (c+c)+(c+c) = 4c exactly and 4c*0.25 = c exactly, for any c
    for c in list(RNG.uniform(-100, 100, 20)) + [0.0, 1.0, 1e-300 if dtype == np.float64 else 1e-30]:
        U = np.full((9, 12), c, dtype=dtype)
        assert bits_equal(oracle.sweep(U, None, 7), U)


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("c", [0.0, 0.5, 1.0, 3.0, -2.0])
def test_constant_field_is_fixed_point_3d(dtype, c):
    # 6c exact => 6c * fl(1/6) rounds back to c (fl(1/6) = (1/6)(1 -+ 2^-54 / 2^-25))
    U = np.full((7, 8, 9), c, dtype=dtype)
    assert bits_equal(oracle.sweep(U, None, 5), U)


@pytest.mark.parametrize("dtype,c,fixed", [
    (np.float64, 0.1, True), (np.float64, 0.3, False), (np.float32, 0.1, False)])
def test_constant_field_3d_pins_multiply_by_rounded_sixth(dtype, c, fixed):
    # The 7-point weight is applied as a multiply by fl(1/6), not a divide by
    # 6 (the two round differently).  With the sum 6c formed by exact
    # doublings and one rounded add, fl(6c) * fl(1/6) returns c for FP64 0.1
    # but not for FP64 0.3 or FP32 0.1, while fl(6c) / 6 does the opposite in
    # all three cases; so an oracle that divides fails every one of these.
    c = dtype(c)
    U = np.full((6, 7, 8), c, dtype=dtype)
    V = oracle.sweep(U, None, 1)
    inner = V[1:-1, 1:-1, 1:-1]
    if fixed:
        assert bits_equal(V, U)
    else:
        assert np.all(inner != c)
        # still within an ulp of c: the multiply rounds twice
        assert np.all(np.abs(inner.astype(np.float64) - float(c)) <= float(np.spacing(c)))


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_integer_linear_field_is_fixed_point(dtype):
    # discrete harmonic: neighbour sums are exact integers
    j, i = np.indices((14, 11))
    U = (3 * i - 2 * j + 7).astype(dtype)
    assert bits_equal(oracle.sweep(U, None, 9), U)
    k, j, i = np.indices((8, 9, 10))
    U3 = (3 * i - 2 * j + 5 * k + 7).astype(dtype)
    assert bits_equal(oracle.sweep(U3, None, 6), U3)


def test_real_linear_field_within_an_ulp_per_sweep():
    j, i = np.indices((20, 20))
    U = 0.37 * i - 1.3 * j + 0.1
    V = oracle.sweep(U, None, 1)
    assert np.max(np.abs(V - U)) <= 2 * np.spacing(np.max(np.abs(U)))


# ---------------------------------------------------------------- eigenmodes
def eigenmode(n, ndim):
    x = np.sin(math.pi * synthetic.node_coords(n))
    full = np.zeros(n + 2)
    full[1:-1] = x
    if ndim == 2:
        return np.outer(full, full)
    return full[:, None, None] * full[None, :, None] * full[None, None, :]


@pytest.mark.parametrize("n,K", [(63, 200), (255, 400), (30, 57)])
def test_eigenmode_decays_by_cos_pi_h_2d(n, K):
    # S phi = 4 cos(pi h) phi, so one sweep multiplies the mode by cos(pi h);
    # rounding adds <= 3*2^-53*max|u| per sweep and |G|_inf <= 1
    U = eigenmode(n, 2)
    c = math.cos(math.pi / (n + 1))
    V = oracle.sweep(U, None, K)
    fac = 1.0
    for _ in range(K):
        fac *= c
    err = np.max(np.abs(V - fac * U))
    assert err <= 5 * (K + 1) * 2.0 ** -53 * np.max(np.abs(U))
    # the ring stays exactly zero
    assert np.all(V[0] == 0) and np.all(V[-1] == 0) and np.all(V[:, 0] == 0)


@pytest.mark.parametrize("n,K", [(15, 60), (24, 31)])
def test_eigenmode_decays_by_cos_pi_h_3d(n, K):
    U = eigenmode(n, 3)
    c = math.cos(math.pi / (n + 1))
    V = oracle.sweep(U, None, K)
    fac = c ** 0
    for _ in range(K):
        fac *= c
    assert np.max(np.abs(V - fac * U)) <= 8 * (K + 1) * 2.0 ** -53 * np.max(np.abs(U))


def test_eigenmode_decay_fp32_within_fp32_bound():
    n, K = 63, 100
    U = eigenmode(n, 2).astype(np.float32)
    c = math.cos(math.pi / (n + 1))
    V = oracle.sweep(U, None, K).astype(np.float64)
    assert np.max(np.abs(V - c ** K * U.astype(np.float64))) <= 5 * (K + 1) * 2.0 ** -24


# ------------------------------------------------------------------ symmetry
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_d4_equivariance_2d(dtype):
    n = 23
    U = RNG.uniform(-1, 1, (n + 2, n + 2)).astype(dtype)
    b = RNG.uniform(-1e-3, 1e-3, (n, n)).astype(dtype)
    V = oracle.sweep(U, b, 13)
    assert bits_equal(oracle.sweep(np.ascontiguousarray(U.T), np.ascontiguousarray(b.T), 13),
                      np.ascontiguousarray(V.T))
    assert bits_equal(oracle.sweep(np.ascontiguousarray(U[::-1]), np.ascontiguousarray(b[::-1]), 13),
                      np.ascontiguousarray(V[::-1]))
    assert bits_equal(oracle.sweep(np.ascontiguousarray(U[:, ::-1]),
                                   np.ascontiguousarray(b[:, ::-1]), 13),
                      np.ascontiguousarray(V[:, ::-1]))


def test_flips_and_xy_transpose_3d():
    U = RNG.uniform(-1, 1, (12, 11, 13))
    b = RNG.uniform(-1e-3, 1e-3, (10, 9, 11))
    V = oracle.sweep(U, b, 6)
    for ax in range(3):
        Uf = np.ascontiguousarray(np.flip(U, ax))
        bf = np.ascontiguousarray(np.flip(b, ax))
        assert bits_equal(oracle.sweep(Uf, bf, 6), np.ascontiguousarray(np.flip(V, ax)))
    # x <-> y swap keeps the grouping ((x-pair)+(y-pair)) up to commutativity
    Ut = np.ascontiguousarray(U.transpose(0, 2, 1))
    bt = np.ascontiguousarray(b.transpose(0, 2, 1))
    assert bits_equal(oracle.sweep(Ut, bt, 6), np.ascontiguousarray(V.transpose(0, 2, 1)))


# --------------------------------------------------------- dense-matrix form
def dense_operators(shape):
    """S (neighbour sum over interior nodes, zero ring) and B (ring -> interior
    coupling) as dense matrices for interior shape `shape` (C order)."""
    nint = int(np.prod(shape))
    full = tuple(s + 2 for s in shape)
    nfull = int(np.prod(full))
    S = np.zeros((nint, nint))
    B = np.zeros((nint, nfull))
    for idx in np.ndindex(*shape):
        row = np.ravel_multi_index(idx, shape)
        for ax in range(len(shape)):
            for d in (-1, 1):
                nb = list(idx)
                nb[ax] += d
                if 0 <= nb[ax] < shape[ax]:
                    S[row, np.ravel_multi_index(tuple(nb), shape)] += 1.0
                else:
                    B[row, np.ravel_multi_index(tuple(v + 1 for v in nb), full)] += 1.0
    return S, B


@pytest.mark.parametrize("shape", [(5, 7), (8, 3), (4, 5, 6)])
def test_matches_dense_matrix_form(shape):
    d = len(shape)
    w = 0.25 if d == 2 else 1.0 / 6.0
    S, B = dense_operators(shape)
    U = RNG.uniform(-1, 1, tuple(s + 2 for s in shape))
    b = RNG.uniform(-1, 1, shape)
    u = U[(slice(1, -1),) * d].ravel()
    expect = w * (S @ u + B @ U.ravel() + b.ravel())
    got = oracle.interior(oracle.sweep(U, b, 1)).ravel()
    assert np.max(np.abs(got - expect)) <= 8 * 2.0 ** -53 * np.max(np.abs(expect)) * 4


def test_poisson_eigenmode_transient_closed_form():
    # f = a*phi, u_0 = 0, zero ring:  u_K = h^2 a (1 - c^K) / (4 (1 - c)) * phi,
    # c = cos(pi h): pins the +h^2 f sign and the scaling of the source
    n, K, a = 31, 150, 3.7
    h2 = synthetic.spacing2(n)
    phi = eigenmode(n, 2)
    f = a * oracle.interior(phi)
    b = oracle.scale_source(f, h2)
    V = oracle.sweep(np.zeros((n + 2, n + 2)), b, K)
    c = math.cos(math.pi / (n + 1))
    expect = h2 * a * (1 - c ** K) / (4 * (1 - c)) * phi
    assert np.max(np.abs(V - expect)) <= 1e-13 * np.max(np.abs(expect)) * K


@pytest.mark.parametrize("n", [7, 12, 16])
def test_contraction_toward_direct_solve(n):
    # |u_k - u*|_2 <= cos(pi h)^k |u_0 - u*|_2 since the iteration matrix is
    # symmetric with spectral radius cos(pi h)
    S, B = dense_operators((n, n))
    A = 4 * np.eye(n * n) - S
    U0 = RNG.uniform(-1, 1, (n + 2, n + 2))
    b = RNG.uniform(-1, 1, (n, n))
    ustar = np.linalg.solve(A, b.ravel() + B @ U0.ravel())
    c = math.cos(math.pi / (n + 1))
    e0 = np.linalg.norm(oracle.interior(U0).ravel() - ustar)
    for k in (1, 5, 40, 200):
        ek = np.linalg.norm(oracle.interior(oracle.sweep(U0, b, k)).ravel() - ustar)
        assert ek <= c ** k * e0 * (1 + 1e-9) + 1e-12


# ---------------------------------------------------- blocks = monolithic
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("nx,ny,bx,by", [(256, 256, 2, 2), (37, 29, 3, 4), (10, 17, 1, 5),
                                         (9, 9, 9, 9), (64, 40, 7, 1)])
def test_blocked_equals_monolithic_2d(dtype, nx, ny, bx, by):
    U = RNG.uniform(0, 1, (ny + 2, nx + 2)).astype(dtype)
    b = RNG.uniform(-1e-4, 1e-4, (ny, nx)).astype(dtype)
    mono = oracle.sweep(U, b, 11)
    blk = oracle.blocked_sweep(U, b, 11, [oracle.balanced_starts(nx, bx),
                                          oracle.balanced_starts(ny, by)])
    assert bits_equal(mono, blk)
    # uneven, non-balanced partition
    xs = np.array([0] + sorted(RNG.choice(np.arange(1, nx), size=min(bx, nx) - 1, replace=False).tolist())
                  + [nx]) if bx > 1 else np.array([0, nx])
    ys = oracle.balanced_starts(ny, by)
    assert bits_equal(mono, oracle.blocked_sweep(U, b, 11, [xs, ys]))
    assert bits_equal(oracle.sweep(U, None, 11), oracle.blocked_sweep(U, None, 11, [xs, ys]))


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("n,nb", [((16, 16, 16), (2, 2, 2)), ((13, 9, 11), (3, 2, 4)),
                                  ((8, 8, 8), (1, 8, 1))])
def test_blocked_equals_monolithic_3d(dtype, n, nb):
    nx, ny, nz = n
    U = RNG.uniform(0, 1, (nz + 2, ny + 2, nx + 2)).astype(dtype)
    b = RNG.uniform(-1e-4, 1e-4, (nz, ny, nx)).astype(dtype)
    mono = oracle.sweep(U, b, 7)
    blk = oracle.blocked_sweep(U, b, 7, [oracle.balanced_starts(m, q) for m, q in zip(n, nb)])
    assert bits_equal(mono, blk)


def test_laplace256_blocked_equals_monolithic():
    U = synthetic.laplace2d_top_edge()
    mono = oracle.sweep(U, None, 100)
    blk = oracle.blocked_sweep(U, None, 100, [oracle.balanced_starts(256, 2)] * 2)
    assert bits_equal(mono, blk)


# ------------------------------------------------------------------- window
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_window_equals_full_run(dtype):
    n, K = 61, 17
    U = RNG.uniform(0, 1, (n + 2, n + 2)).astype(dtype)
    b = RNG.uniform(-1e-3, 1e-3, (n, n)).astype(dtype)
    full = oracle.interior(oracle.sweep(U, b, K))
    for (x0, x1), (y0, y1) in [((0, 5), (0, 61)), ((20, 33), (40, 61)), ((60, 61), (0, 1)),
                               ((0, 61), (0, 61))]:
        assert bits_equal(oracle.window(U, b, K, ((x0, x1), (y0, y1))), full[y0:y1, x0:x1])
    n3 = 19
    U3 = RNG.uniform(0, 1, (n3 + 2,) * 3).astype(dtype)
    b3 = RNG.uniform(-1e-3, 1e-3, (n3,) * 3).astype(dtype)
    full3 = oracle.interior(oracle.sweep(U3, b3, 6))
    got = oracle.window(U3, b3, 6, ((2, 9), (0, 4), (15, 19)))
    assert bits_equal(got, full3[15:19, 0:4, 2:9])


# ------------------------------------------------------------ source scaling
def test_scale_source_rounds_once():
    # the FP64 product rounded once to FP32 differs from two FP32 roundings on
    # some inputs; pin the single-rounding reading on values where they differ
    f32 = np.float32(RNG.uniform(-1, 1, 20000))
    h2 = synthetic.spacing2(8192)
    b = oracle.scale_source(f32, h2, np.float32)
    once = (np.float64(h2) * f32.astype(np.float64)).astype(np.float32)
    assert bits_equal(b, once)
    twice = np.float32(h2) * f32
    assert not bits_equal(b, twice)  # the two readings are distinguishable here
    # subnormal products are kept (no flush to zero)
    tiny = oracle.scale_source(np.array([1e-38, -3e-39], np.float32), 1e-4, np.float32)
    assert np.all(tiny != 0)
