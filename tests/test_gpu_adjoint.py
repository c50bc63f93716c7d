"""Adjoint (reverse-mode) parity: the device adjoint through the C ABI and the
torch.autograd wrapper against the FP64 oracle adjoint, its finite
differences, and invariance in the checkpoint interval."""
import math
import sys

import numpy as np
import pytest

import oracle
import synthetic
from gpu_util import bits_equal, norm_rel_err

pytestmark = pytest.mark.gpu

RNG = np.random.default_rng(99)


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def device_adjoint(lamK_full, K, h2, blocks, dtype, device, depth=0, rows=0, chunk=None,
                   segments=False):
    """jacobi_adjoint (one call) or, with segments, jacobi_adjoint_begin /
    _sweep / _end; returns numpy arrays."""
    import torch
    import paper_2303_02543_amd as jb
    tdt = torch.float32 if dtype == np.float32 else torch.float64
    ny, nx = lamK_full.shape[0] - 2, lamK_full.shape[1] - 2
    s = jb.Solver((nx, ny), blocks, tdt, device=device)
    try:
        s.set_tuning(depth, rows, 0)
        lam = torch.from_numpy(np.ascontiguousarray(lamK_full, dtype=dtype)).to(device)
        if segments:
            out = s.adjoint_segments(lam, K, h2, chunk=chunk)
        else:
            out = s.adjoint(lam, K, h2, chunk=chunk)
        torch.cuda.synchronize()
        return tuple(t.cpu().numpy() for t in out)
    finally:
        s.close()


CASES = [(37, 29, 3, 4, 13), (130, 70, 2, 3, 40), (8, 8, 1, 1, 5), (1, 1, 1, 1, 3), (300, 9, 4, 1, 21)]


@pytest.mark.parametrize("case", CASES)
def test_adjoint_fp64_bit_exact(device, case):
    """FP64 device adjoint == FP64 oracle adjoint bit for bit (same order of
    accumulation k = K..1), for every chunking of the reverse sweeps.  The
    one-call form takes dL/du_K on every node (its ring passes to dL/dg);
    the three-call form reads the ring of its input as zero."""
    nx, ny, bx, by, K = case
    h2 = synthetic.spacing2(max(nx, ny))
    full = RNG.standard_normal((ny + 2, nx + 2))   # dL/du_K, ring included
    lamK = np.ascontiguousarray(full[1:-1, 1:-1])
    Gb_full, dU0 = oracle.adjoint2d_full(full, K)
    Gb, Gring, lam0 = oracle.adjoint2d(lamK, K)
    assert bits_equal(Gb_full, Gb)
    want_f = h2 * Gb
    for chunk in (None, 1, 7):
        say("adjoint fp64 case=%s chunk=%s" % (case, chunk))
        gf, gU0 = device_adjoint(full, K, h2, (bx, by), np.float64, device, chunk=chunk)
        assert bits_equal(gf, want_f), "dL/df"
        assert bits_equal(gU0, dU0), "dL/dU0"
        gf2, ring2, lam_state = device_adjoint(full, K, h2, (bx, by), np.float64, device,
                                               chunk=chunk, segments=True)
        assert bits_equal(gf2, want_f), "dL/df (segments)"
        assert bits_equal(ring2, Gring), "dL/dg through the sweeps (segments)"
        assert bits_equal(np.ascontiguousarray(lam_state[1:-1, 1:-1]), lam0), "lam_0 (segments)"


def test_adjoint_fp32_within_1e5(device):
    n, K = 255, 300
    h2 = synthetic.spacing2(n)
    lamK = synthetic.gaussian_sum(n, 2, 6).astype(np.float32)
    full = np.zeros((n + 2, n + 2), dtype=np.float32)
    full[1:-1, 1:-1] = lamK
    Gb, Gring, lam0 = oracle.adjoint2d(lamK.astype(np.float64), K)
    gf, gU0 = device_adjoint(full, K, h2, (2, 2), np.float32, device, chunk=50)
    assert np.all(gU0[[0, 0, -1, -1], [0, -1, 0, -1]] == 0.0)  # zero ring in, zero corners
    e_f = np.max(np.abs(gf - h2 * Gb)) / np.max(np.abs(h2 * Gb))
    ring = gU0.copy()
    ring[1:-1, 1:-1] = 0
    e_g = np.max(np.abs(ring - Gring)) / np.max(np.abs(Gring))
    e_l = np.max(np.abs(gU0[1:-1, 1:-1] - lam0)) / np.max(np.abs(lam0))
    say("adjoint fp32 errors f=%.2e g=%.2e u0=%.2e" % (e_f, e_g, e_l))
    assert e_f <= 1e-5 and e_g <= 1e-5 and e_l <= 1e-5


def test_autograd_matches_oracle_and_fd(device):
    """Loss 1/2 |u_K - t|^2 through JacobiK (FP64): gradients equal the
    oracle's FP64 gradients bit for bit, and central finite differences."""
    import torch
    import paper_2303_02543_amd as jb
    from paper_2303_02543_amd.autograd import JacobiK
    n, K = 41, 30
    h2 = synthetic.spacing2(n)
    U0 = synthetic.ring_values(n, 2, 7)
    f = synthetic.gaussian_sum(n, 2, 5)
    t = synthetic.gaussian_sum(n, 2, 6) * 1e-3
    s = jb.Solver((n, n), (2, 3), torch.float64, device=device)
    try:
        fT = torch.from_numpy(f).to(device).requires_grad_(True)
        UT = torch.from_numpy(U0).to(device).requires_grad_(True)
        tT = torch.from_numpy(t).to(device)
        uK = JacobiK.apply(fT, UT, s, K, h2, 7)
        loss = 0.5 * ((uK[1:-1, 1:-1] - tT) ** 2).sum()
        loss.backward()
        gf = fT.grad.cpu().numpy()
        gU = UT.grad.cpu().numpy()
    finally:
        s.close()
    L, dLdf, dLdU0 = oracle.gradients2d(U0, f, h2, t, K)
    assert math.isclose(float(loss), L, rel_tol=1e-12)
    assert bits_equal(gf, dLdf)
    assert bits_equal(gU, dLdU0)
    f_idx, g_idx = synthetic.fd_picks(n, count=6, seed=8)
    for idx in f_idx:
        fd = oracle.fd_grad_source(U0, f, h2, t, K, idx, 1e-3)
        assert math.isclose(fd, gf[idx], rel_tol=1e-6, abs_tol=1e-14)
    for idx in g_idx:
        fd = oracle.fd_grad_state(U0, f, h2, t, K, idx, 1e-3)
        assert math.isclose(fd, gU[idx], rel_tol=1e-6, abs_tol=1e-14)


def test_checkpoint_interval_invariance_and_checkpoints(device):
    """Gradients are bit-identical for C in {1, 7, 50, K}; the forward
    checkpoints equal the oracle's states after 0, C, 2C, ... sweeps."""
    import torch
    import paper_2303_02543_amd as jb
    from paper_2303_02543_amd.autograd import JacobiK
    n, K = 64, 100
    h2 = synthetic.spacing2(n)
    U0 = synthetic.ring_values(n, 2, 7).astype(np.float32)
    f = synthetic.gaussian_sum(n, 2, 5).astype(np.float32)
    t = (synthetic.gaussian_sum(n, 2, 6) * 1e-3).astype(np.float32)
    grads = []
    s = jb.Solver((n, n), (2, 2), torch.float32, device=device)
    try:
        for C in (1, 7, 50, K):
            fT = torch.from_numpy(f).to(device).requires_grad_(True)
            UT = torch.from_numpy(U0).to(device).requires_grad_(True)
            uK = JacobiK.apply(fT, UT, s, K, h2, C, True)
            ckpts = uK.grad_fn.checkpoints
            assert ckpts.shape[0] == -(-K // C)
            loss = 0.5 * ((uK[1:-1, 1:-1] - torch.from_numpy(t).to(device)) ** 2).sum()
            loss.backward()
            grads.append((fT.grad.cpu().numpy(), UT.grad.cpu().numpy()))
            b32 = oracle.scale_source(f, h2, np.float32)
            for i, ck in enumerate(ckpts):
                want = oracle.sweep(U0, b32, i * C)
                assert bits_equal(ck.cpu().numpy(), want), "checkpoint %d (C=%d)" % (i, C)
    finally:
        s.close()
    for gf, gU in grads[1:]:
        assert bits_equal(gf, grads[0][0]) and bits_equal(gU, grads[0][1])


def test_autograd_full_state_loss(device):
    """A loss over every node of u_K, ring and corners included:
    L = 1/2 sum (u_K - T)^2 (FP64).  The ring of u_K is g itself, so dL/dg
    gets dL/du_K on the ring besides what flows through the sweeps, and the
    corners get only that.  Gradients equal the oracle's bit for bit and
    central differences on ring entries (corners included) and source
    entries."""
    import torch
    import paper_2303_02543_amd as jb
    from paper_2303_02543_amd.autograd import JacobiK
    nx, ny, K = 45, 38, 23
    n = max(nx, ny)
    h2 = synthetic.spacing2(n)
    rng = np.random.default_rng(31)
    U0 = rng.uniform(0.0, 1.0, (ny + 2, nx + 2))
    f = rng.standard_normal((ny, nx))
    T = rng.standard_normal((ny + 2, nx + 2)) * 0.1
    s = jb.Solver((nx, ny), (2, 3), torch.float64, device=device)
    try:
        fT = torch.from_numpy(f).to(device).requires_grad_(True)
        UT = torch.from_numpy(U0).to(device).requires_grad_(True)
        uK = JacobiK.apply(fT, UT, s, K, h2, 5)
        loss = 0.5 * ((uK - torch.from_numpy(T).to(device)) ** 2).sum()
        loss.backward()
        gf = fT.grad.cpu().numpy()
        gU = UT.grad.cpu().numpy()
    finally:
        s.close()
    b = oracle.scale_source(f, h2)
    uK_o = oracle.sweep(U0, b, K)
    Gb, dU0 = oracle.adjoint2d_full(uK_o - T, K)
    assert bits_equal(gf, h2 * Gb)
    assert bits_equal(gU, dU0)
    picks = [(0, 0), (0, nx + 1), (ny + 1, 0), (ny + 1, nx + 1), (0, 7), (ny + 1, 13),
             (5, 0), (20, nx + 1), (1, 1), (ny // 2, nx // 2)]
    for idx in picks:
        fd = oracle.fd_grad_state(U0, f, h2, T, K, idx, 1e-3)
        assert math.isclose(fd, gU[idx], rel_tol=1e-7, abs_tol=1e-13), idx
    for idx in [(0, 0), (ny - 1, nx - 1), (10, 20)]:
        fd = oracle.fd_grad_source(U0, f, h2, T, K, idx, 1e-3)
        assert math.isclose(fd, gf[idx], rel_tol=1e-7, abs_tol=1e-15), idx
