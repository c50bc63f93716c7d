"""Pins of the oracle's FP64 adjoint (reverse-mode derivative of
L = 1/2 |u_K - t|^2 through K sweeps): the dot-product test against the forward
sweep, the K = 1 closed form, the eigenmode closed form, a tangent-linear check
that uses only the forward sweep, and central finite differences."""
import math

import numpy as np
import pytest

import oracle
import synthetic
from test_oracle_sweep import eigenmode

RNG = np.random.default_rng(4242)


def zero_ring(interior):
    return synthetic.state_with_ring(interior)


@pytest.mark.parametrize("K", [1, 3, 17])
def test_dot_product_test(K):
    # <G^K v, w> == <v, (G^T)^K w>: G^K from the forward sweep (zero ring, no
    # source), its transpose from the adjoint recurrence
    ny, nx = 13, 19
    v = RNG.standard_normal((ny, nx))
    w = RNG.standard_normal((ny, nx))
    Gv = oracle.interior(oracle.sweep(zero_ring(v), None, K))
    _, _, GTw = oracle.adjoint2d(w, K)
    lhs, rhs = float(np.sum(Gv * w)), float(np.sum(v * GTw))
    assert math.isclose(lhs, rhs, rel_tol=1e-12, abs_tol=1e-14)


def test_k1_closed_form():
    # u_1 = (S u0 + B g + h^2 f)/4:  dL/df = h^2 (u1 - t)/4,
    # dL/dg_q = (u1 - t)[p(q)]/4, dL/du0 = S (u1 - t)/4
    n = 11
    h2 = synthetic.spacing2(n)
    U0 = RNG.uniform(0, 1, (n + 2, n + 2))
    f = RNG.standard_normal((n, n))
    t = RNG.standard_normal((n, n))
    L, dLdf, dLdU0 = oracle.gradients2d(U0, f, h2, t, 1)
    u1 = oracle.interior(oracle.sweep(U0, oracle.scale_source(f, h2), 1))
    lam = u1 - t
    np.testing.assert_allclose(dLdf, h2 * lam / 4, rtol=1e-14, atol=0)
    np.testing.assert_allclose(dLdU0[0, 1:-1], lam[0] / 4, rtol=1e-14)      # south edge
    np.testing.assert_allclose(dLdU0[-1, 1:-1], lam[-1] / 4, rtol=1e-14)    # north edge
    np.testing.assert_allclose(dLdU0[1:-1, 0], lam[:, 0] / 4, rtol=1e-14)   # west edge
    np.testing.assert_allclose(dLdU0[1:-1, -1], lam[:, -1] / 4, rtol=1e-14)  # east edge
    assert dLdU0[0, 0] == 0 and dLdU0[0, -1] == 0 and dLdU0[-1, 0] == 0 and dLdU0[-1, -1] == 0
    lamfull = zero_ring(lam)
    Slam = (lamfull[1:-1, :-2] + lamfull[1:-1, 2:]) + (lamfull[:-2, 1:-1] + lamfull[2:, 1:-1])
    np.testing.assert_allclose(oracle.interior(dLdU0), Slam / 4, rtol=1e-14, atol=1e-300)
    assert math.isclose(L, 0.5 * float(np.sum(lam ** 2)), rel_tol=1e-15)


@pytest.mark.parametrize("n,K", [(31, 40), (63, 200)])
def test_eigenmode_closed_form(n, K):
    # t = 0, f = 0, g = 0, u0 = phi, c = cos(pi h): u_K = c^K phi,
    # dL/du0 = c^{2K} phi, dL/db = w c^K (1 - c^K)/(1 - c) phi
    c = math.cos(math.pi / (n + 1))
    phi = oracle.interior(eigenmode(n, 2))
    uK = oracle.interior(oracle.sweep(eigenmode(n, 2), None, K))
    Gb, Gring, lam0 = oracle.adjoint2d(uK, K)
    tol = 1e-12 * np.max(np.abs(phi))
    assert np.max(np.abs(lam0 - c ** (2 * K) * phi)) <= tol
    coef = 0.25 * c ** K * (1 - c ** K) / (1 - c)
    assert np.max(np.abs(Gb - coef * phi)) <= 1e-11 * coef
    # ring gradient: coefficient times phi at the adjacent interior node
    np.testing.assert_allclose(Gring[0, 1:-1], coef * phi[0], rtol=1e-10)
    np.testing.assert_allclose(Gring[1:-1, -1], coef * phi[:, -1], rtol=1e-10)


def test_tangent_linear_agrees_with_adjoint():
    # dL[v] computed forward: u_dot_K = sweep^K(U0_dot, source h^2 f_dot)
    # (the map is affine, so its tangent is the same sweep with the tangent
    # inputs); dL = <u_K - t, u_dot_K>.  The adjoint must give the same number.
    n, K = 24, 35
    h2 = synthetic.spacing2(n)
    U0 = RNG.uniform(0, 1, (n + 2, n + 2))
    f = RNG.standard_normal((n, n)) * 50
    t = RNG.standard_normal((n, n)) * 0.01
    fdot = RNG.standard_normal((n, n))
    U0dot = RNG.standard_normal((n + 2, n + 2))
    L, dLdf, dLdU0 = oracle.gradients2d(U0, f, h2, t, K)
    uK = oracle.interior(oracle.sweep(U0, oracle.scale_source(f, h2), K))
    udotK = oracle.interior(oracle.sweep(U0dot, oracle.scale_source(fdot, h2), K))
    forward = float(np.sum((uK - t) * udotK))
    # corners never influence the interior, so their tangent is irrelevant
    reverse = float(np.sum(dLdf * fdot)) + float(np.sum(dLdU0 * U0dot))
    assert math.isclose(forward, reverse, rel_tol=1e-11)


def test_central_finite_differences():
    # L is quadratic in (f, U0): central differences are exact up to rounding
    n, K = 31, 20
    h2 = synthetic.spacing2(n)
    U0 = synthetic.ring_values(n, 2, 7)
    f = synthetic.gaussian_sum(n, 2, 5)
    t = synthetic.gaussian_sum(n, 2, 6) * 1e-3
    L, dLdf, dLdU0 = oracle.gradients2d(U0, f, h2, t, K)
    f_idx, g_idx = synthetic.fd_picks(n, count=6, seed=8)
    for idx in f_idx:
        fd = oracle.fd_grad_source(U0, f, h2, t, K, idx, 1e-3)
        assert math.isclose(fd, dLdf[idx], rel_tol=1e-6, abs_tol=1e-14)
    for idx in g_idx:
        fd = oracle.fd_grad_state(U0, f, h2, t, K, idx, 1e-3)
        assert math.isclose(fd, dLdU0[idx], rel_tol=1e-6, abs_tol=1e-14)


def test_full_state_loss_brute_force_differences():
    # A loss over every node of u_K, ring included: L = 1/2 sum (u_K - T)^2.
    # The ring of u_K is g itself (sweeps copy it), so dL/dg gains dL/du_K on
    # the ring, corners included.  Checked against central differences of
    # every entry of f and U0 on a tiny grid (L is quadratic: differences are
    # exact up to rounding).
    nx, ny, K = 6, 5, 4
    h2 = synthetic.spacing2(max(nx, ny))
    U0 = RNG.uniform(-1, 1, (ny + 2, nx + 2))
    f = RNG.standard_normal((ny, nx))
    T = RNG.standard_normal((ny + 2, nx + 2))
    b = oracle.scale_source(f, h2)
    uK = oracle.sweep(U0, b, K)
    Gb, dU0 = oracle.adjoint2d_full(uK - T, K)
    eps = 1e-3
    for idx in np.ndindex(U0.shape):
        fd = oracle.fd_grad_state(U0, f, h2, T, K, idx, eps)
        assert math.isclose(fd, dU0[idx], rel_tol=1e-9, abs_tol=1e-12), idx
    for idx in np.ndindex(f.shape):
        fd = oracle.fd_grad_source(U0, f, h2, T, K, idx, eps)
        assert math.isclose(fd, h2 * Gb[idx], rel_tol=1e-9, abs_tol=1e-15), idx
    # corners only see the identity: dL/dU0 there is (u_K - T) at the corner
    for c in [(0, 0), (0, -1), (-1, 0), (-1, -1)]:
        assert dU0[c] == (uK - T)[c]
