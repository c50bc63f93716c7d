"""Pins of the oracle's FP64 residual and relative-residual stop rule: a dense
numpy operator on tiny grids, the eigenmode closed forms in 2D and 3D, the
identity U_{k+1} - U_k = w r_k, and the closed-form stop sweep of a decaying
eigenmode."""
import math

import numpy as np
import pytest

import oracle
from test_oracle_sweep import dense_operators, eigenmode

RNG = np.random.default_rng(777)


@pytest.mark.parametrize("shape", [(6, 4), (3, 9), (4, 3, 5)])
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_residual_matches_dense_operator(shape, dtype):
    d = len(shape)
    S, B = dense_operators(shape)
    A = 2 * d * np.eye(S.shape[0]) - S
    U = RNG.uniform(-1, 1, tuple(s + 2 for s in shape)).astype(dtype)
    b = RNG.uniform(-1, 1, shape).astype(dtype)
    U64 = U.astype(np.float64)
    r = b.astype(np.float64).ravel() + B @ U64.ravel() - A @ U64[(slice(1, -1),) * d].ravel()
    assert math.isclose(oracle.residual(U, b), np.linalg.norm(r), rel_tol=1e-13)
    r0 = B @ U64.ravel() - A @ U64[(slice(1, -1),) * d].ravel()
    assert math.isclose(oracle.residual(U, None), np.linalg.norm(r0), rel_tol=1e-13)


@pytest.mark.parametrize("n,k", [(31, 0), (31, 25), (100, 300)])
def test_residual_eigenmode_closed_form_2d(n, k):
    # r = (4 - S) u = 4 (1 - cos pi h) u for u = c^k phi, and
    # sum_i sin^2(i pi h) = (n+1)/2  =>  res = 4 (1-c) c^k (n+1)/2
    c = math.cos(math.pi / (n + 1))
    U = oracle.sweep(eigenmode(n, 2), None, k)
    expect = 4 * (1 - c) * c ** k * (n + 1) / 2
    assert math.isclose(oracle.residual(U, None), expect, rel_tol=1e-9)


@pytest.mark.parametrize("n,k", [(15, 0), (15, 20)])
def test_residual_eigenmode_closed_form_3d(n, k):
    c = math.cos(math.pi / (n + 1))
    U = oracle.sweep(eigenmode(n, 3), None, k)
    expect = 6 * (1 - c) * c ** k * ((n + 1) / 2) ** 1.5
    assert math.isclose(oracle.residual(U, None), expect, rel_tol=1e-9)


@pytest.mark.parametrize("ndim", [2, 3])
def test_residual_is_scaled_sweep_increment(ndim):
    # U_{k+1} - U_k = w * r_k in exact arithmetic
    n = 20 if ndim == 2 else 9
    U = RNG.uniform(0, 1, (n + 2,) * ndim)
    b = RNG.uniform(-0.1, 0.1, (n,) * ndim)
    w = 0.25 if ndim == 2 else 1.0 / 6.0
    V = oracle.sweep(U, b, 1)
    inc = np.linalg.norm((oracle.interior(V) - oracle.interior(U)).ravel()) / w
    assert math.isclose(oracle.residual(U, b), inc, rel_tol=1e-12)


@pytest.mark.parametrize("n,R,tol", [(15, 1, 1e-6), (15, 7, 1e-6), (15, 50, 1e-6), (9, 10, 1e-3)])
def test_stop_rule_closed_form_on_eigenmode(n, R, tol):
    # rel_k = cos(pi h)^k, so the first checked k with rel <= tol is
    # R * ceil(ln tol / (R ln cos pi h))
    c = math.cos(math.pi / (n + 1))
    kstar = R * math.ceil(math.log(tol) / (R * math.log(c)))
    out = oracle.solve(eigenmode(n, 2), None, 10 ** 6, R, tol)
    assert out["status"] == "converged"
    assert out["sweeps"] == kstar
    assert out["rel"] <= tol
    assert all(kk % R == 0 for kk, _ in out["checks"])


def test_stop_rule_edge_cases():
    n = 8
    # zero residual at k = 0: converged without a sweep
    U = np.full((n + 2, n + 2), 2.5)
    out = oracle.solve(U, None, 100, 10, 1e-6)
    assert out["status"] == "converged" and out["sweeps"] == 0
    # the cap is checked even when it is not a multiple of R
    out = oracle.solve(eigenmode(n, 2), None, 23, 10, 1e-30)
    assert out["status"] == "max_sweeps" and out["sweeps"] == 23
    assert [k for k, _ in out["checks"]] == [0, 10, 20, 23]
    # a non-finite state is reported as diverged
    U = eigenmode(n, 2)
    U[3, 3] = np.nan
    assert oracle.solve(U, None, 100, 10, 1e-6)["status"] == "diverged"
    # max_sweeps = 0 only checks res_0
    out = oracle.solve(eigenmode(n, 2), None, 0, 10, 1e-6)
    assert out["sweeps"] == 0 and out["status"] == "max_sweeps"
