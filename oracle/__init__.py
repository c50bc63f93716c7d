"""CPU oracle for the over-decomposed Jacobi sweep (paper Section 4.3,
Proxy Application: Jacobi3D, and Section 4.4, Over-decomposition).

TEST INFRASTRUCTURE ONLY.  Only tests/, the smoke check and the benchmark's
CPU-baseline leg may import this package.  It shares no code with the device
library (paper_2303_02543_amd) and never imports it.

The arithmetic lives in plain C (jacobi_oracle.c, FP64, IEEE, no FMA); this
module marshals numpy arrays and adds the two pieces of control logic that are
clearer in Python: the relative-residual stop rule and the finite-difference
driver.

Readings of points the paper leaves open (it names the Jacobi method, a
cuboid decomposition with one-cell face halos, and a fixed iteration count,
nothing more):
  * PDE -Laplace(u) = f on the unit square/cube, h = 1/(n+1), Dirichlet ring;
    the update adds +h^2 f.
  * 5-point update ((W+E)+(S+N) + b) * 1/4; 7-point
    (((W+E)+(S+N))+(B+F) + b) * fl(1/6); no FMA, no flush-to-zero.
  * residual: sqrt(sum (b - (2d u - s))^2) in FP64 over the interior.
  * stop: first checked sweep count k (multiples of R, and max_sweeps) with
    res_k / res_0 <= tol; res_0 == 0 converges at 0 sweeps; a non-finite
    residual marks the grid diverged.

Parity status of every function is pinned by tests/test_oracle_*.py (closed
forms, invariants, brute force on tiny grids); none is "parity unpinned".
"""
import ctypes
import math
import os

import numpy as np

from . import build as _build

_LIB = None

_F64 = np.float64
_F32 = np.float32

P = ctypes.c_void_p
I64 = ctypes.c_int64
DBL = ctypes.c_double


def lib():
    """Load liboracle.so, compiling it first if it is missing or stale."""
    global _LIB
    if _LIB is None:
        if _build.is_stale():
            _build.build()
        L = ctypes.CDLL(_build.LIB)
        for suf in ("f64", "f32"):
            getattr(L, "orc_scale_source_" + suf).argtypes = [I64, DBL, P, P]
            getattr(L, "orc_sweep2d_" + suf).argtypes = [I64, I64, P, P, I64]
            getattr(L, "orc_sweep3d_" + suf).argtypes = [I64, I64, I64, P, P, I64]
            getattr(L, "orc_blocked_sweep2d_" + suf).argtypes = [I64, I64, I64, P, I64, P, P, P, I64]
            getattr(L, "orc_blocked_sweep3d_" + suf).argtypes = [I64, I64, I64, I64, P, I64, P,
                                                                 I64, P, P, P, I64]
            getattr(L, "orc_residual2d_" + suf).argtypes = [I64, I64, P, P]
            getattr(L, "orc_residual2d_" + suf).restype = DBL
            getattr(L, "orc_residual3d_" + suf).argtypes = [I64, I64, I64, P, P]
            getattr(L, "orc_residual3d_" + suf).restype = DBL
            getattr(L, "orc_window2d_" + suf).argtypes = [I64, I64, P, P, I64, I64, I64, I64, I64, P]
            getattr(L, "orc_window3d_" + suf).argtypes = [I64, I64, I64, P, P, I64, I64, I64, I64,
                                                          I64, I64, I64, P]
        L.orc_adjoint2d_f64.argtypes = [I64, I64, I64, P, P, P, P]
        L.orc_num_threads.argtypes = []
        L.orc_num_threads.restype = ctypes.c_int
        L.orc_set_num_threads.argtypes = [ctypes.c_int]
        L.orc_set_num_threads.restype = None
        _LIB = L
    return _LIB


def num_threads():
    """OpenMP threads the oracle's parallel loops use."""
    return int(lib().orc_num_threads())


def set_num_threads(n):
    """Threads of later oracle calls (results do not depend on the count)."""
    lib().orc_set_num_threads(int(n))


def _suffix(dtype):
    dt = np.dtype(dtype)
    if dt == _F64:
        return "f64"
    if dt == _F32:
        return "f32"
    raise TypeError("oracle supports float64 and float32, got %s" % dt)


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _interior_shape(u):
    return tuple(s - 2 for s in u.shape)


def _check_b(u, b):
    if b is None:
        return None
    b = np.ascontiguousarray(b)
    if b.dtype != u.dtype or b.shape != _interior_shape(u):
        raise ValueError("b must have the interior shape %s and dtype %s"
                         % (_interior_shape(u), u.dtype))
    return b


def scale_source(f, h2, dtype=np.float64):
    """b = fl_T(fl64(h^2) * f), product in FP64, one rounding to the run type T."""
    f = np.ascontiguousarray(f, dtype=dtype)
    b = np.empty_like(f)
    getattr(lib(), "orc_scale_source_" + _suffix(dtype))(f.size, float(h2), _ptr(f), _ptr(b))
    return b


def sweep(u, b, K):
    """K synchronous Jacobi sweeps of the monolithic grid (2D or 3D).

    u: state over all nodes including the Dirichlet ring, shape (ny+2, nx+2)
       or (nz+2, ny+2, nx+2); b: scaled source over the interior or None.
    Returns the new state (u is not modified)."""
    u = np.array(u, copy=True, order="C")
    b = _check_b(u, b)
    suf = _suffix(u.dtype)
    if K < 0:
        raise ValueError("K must be >= 0")
    if u.ndim == 2:
        ny, nx = _interior_shape(u)
        rc = getattr(lib(), "orc_sweep2d_" + suf)(nx, ny, _ptr(b), _ptr(u), K)
    elif u.ndim == 3:
        nz, ny, nx = _interior_shape(u)
        rc = getattr(lib(), "orc_sweep3d_" + suf)(nx, ny, nz, _ptr(b), _ptr(u), K)
    else:
        raise ValueError("u must be 2D or 3D")
    if rc != 0:
        raise MemoryError("oracle sweep failed")
    return u


def balanced_starts(n, nblocks):
    """Block starts 0 = s_0 < s_1 < ... < s_B = n with sizes differing by <= 1."""
    return np.array([(q * n) // nblocks for q in range(nblocks + 1)], dtype=np.int64)


def blocked_sweep(u, b, K, starts):
    """K sweeps of the block-decomposed grid with a halo exchange before each
    sweep.  starts: one array of block starts per axis, x first (each begins
    at 0, ends at n, strictly increasing).  Returns the gathered state."""
    u = np.array(u, copy=True, order="C")
    b = _check_b(u, b)
    suf = _suffix(u.dtype)
    ns = _interior_shape(u)[::-1]  # x first
    st = [np.ascontiguousarray(s, dtype=np.int64) for s in starts]
    if len(st) != u.ndim:
        raise ValueError("need one starts array per axis")
    for s, n in zip(st, ns):
        if s[0] != 0 or s[-1] != n or np.any(np.diff(s) <= 0):
            raise ValueError("bad block starts %s for n=%d" % (s, n))
    if u.ndim == 2:
        rc = getattr(lib(), "orc_blocked_sweep2d_" + suf)(
            ns[0], ns[1], len(st[0]) - 1, _ptr(st[0]), len(st[1]) - 1, _ptr(st[1]),
            _ptr(b), _ptr(u), K)
    else:
        rc = getattr(lib(), "orc_blocked_sweep3d_" + suf)(
            ns[0], ns[1], ns[2], len(st[0]) - 1, _ptr(st[0]), len(st[1]) - 1, _ptr(st[1]),
            len(st[2]) - 1, _ptr(st[2]), _ptr(b), _ptr(u), K)
    if rc != 0:
        raise MemoryError("oracle blocked sweep failed")
    return u


def residual(u, b):
    """FP64 L2 norm of the h^2-scaled residual b - A_h u over the interior."""
    u = np.ascontiguousarray(u)
    b = _check_b(u, b)
    suf = _suffix(u.dtype)
    if u.ndim == 2:
        ny, nx = _interior_shape(u)
        return getattr(lib(), "orc_residual2d_" + suf)(nx, ny, _ptr(b), _ptr(u))
    nz, ny, nx = _interior_shape(u)
    return getattr(lib(), "orc_residual3d_" + suf)(nx, ny, nz, _ptr(b), _ptr(u))


def window(u, b, K, ranges):
    """State after K sweeps on interior nodes ranges = ((x0,x1),(y0,y1)[, (z0,z1)])
    (0-based interior coordinates, half open), computed from a grown copy of
    that region only.  Returns an array of shape (y1-y0, x1-x0) (or 3D)."""
    u = np.ascontiguousarray(u)
    b = _check_b(u, b)
    suf = _suffix(u.dtype)
    ns = _interior_shape(u)[::-1]
    for (lo, hi), n in zip(ranges, ns):
        if not (0 <= lo < hi <= n):
            raise ValueError("window range out of bounds")
    if u.ndim == 2:
        (x0, x1), (y0, y1) = ranges
        out = np.empty((y1 - y0, x1 - x0), dtype=u.dtype)
        rc = getattr(lib(), "orc_window2d_" + suf)(ns[0], ns[1], _ptr(b), _ptr(u), K,
                                                   x0, x1, y0, y1, _ptr(out))
    else:
        (x0, x1), (y0, y1), (z0, z1) = ranges
        out = np.empty((z1 - z0, y1 - y0, x1 - x0), dtype=u.dtype)
        rc = getattr(lib(), "orc_window3d_" + suf)(ns[0], ns[1], ns[2], _ptr(b), _ptr(u), K,
                                                   x0, x1, y0, y1, z0, z1, _ptr(out))
    if rc != 0:
        raise MemoryError("oracle window failed")
    return out


def solve(u, b, max_sweeps, check_every, tol):
    """Sweep with the relative-residual stop rule.

    Residuals are taken on the state after k sweeps for k = 0, R, 2R, ... and
    at max_sweeps.  Stops at the first checked k > 0 with res_k/res_0 <= tol
    (inclusive), else at max_sweeps.  res_0 == 0 means converged at 0 sweeps;
    a non-finite residual ends the solve as diverged.
    Returns dict(u, sweeps, status in {"converged","max_sweeps","diverged"},
    checks=[(k, res_k)], rel)."""
    if max_sweeps < 0 or check_every < 1:
        raise ValueError("max_sweeps >= 0 and check_every >= 1 required")
    res0 = residual(u, b)
    checks = [(0, res0)]
    if not math.isfinite(res0):
        return dict(u=np.array(u), sweeps=0, status="diverged", checks=checks, rel=math.nan)
    if res0 == 0.0:
        return dict(u=np.array(u), sweeps=0, status="converged", checks=checks, rel=0.0)
    k = 0
    cur = np.array(u)
    rel = 1.0
    while k < max_sweeps:
        step = min(check_every, max_sweeps - k)
        cur = sweep(cur, b, step)
        k += step
        r = residual(cur, b)
        checks.append((k, r))
        if not math.isfinite(r):
            return dict(u=cur, sweeps=k, status="diverged", checks=checks, rel=math.nan)
        rel = r / res0
        if rel <= tol:
            return dict(u=cur, sweeps=k, status="converged", checks=checks, rel=rel)
    return dict(u=cur, sweeps=k, status="max_sweeps", checks=checks, rel=rel)


def loss(uK, target):
    """L = 1/2 * sum over the interior of (u_K - t)^2, in FP64.  uK: full state,
    target: interior values."""
    d = interior(uK).astype(np.float64) - np.asarray(target, dtype=np.float64)
    return 0.5 * float(np.sum(d * d))


def interior(u):
    return u[(slice(1, -1),) * u.ndim]


def adjoint2d(lamK, K):
    """Run the FP64 adjoint recurrence through K 2D sweeps.

    lamK: interior array (ny, nx) of dL/du_K.  Returns (Gb, Gring, lam0):
    dL/db over the interior, dL/dg on the ring of a (ny+2, nx+2) array (zero
    at corners and in the interior), and dL/du_0 over the interior."""
    lamK = np.ascontiguousarray(lamK, dtype=np.float64)
    ny, nx = lamK.shape
    Gb = np.empty_like(lamK)
    Gring = np.empty((ny + 2, nx + 2), dtype=np.float64)
    lam0 = np.empty_like(lamK)
    rc = lib().orc_adjoint2d_f64(nx, ny, K, _ptr(lamK), _ptr(Gb), _ptr(Gring), _ptr(lam0))
    if rc != 0:
        raise MemoryError("oracle adjoint failed")
    return Gb, Gring, lam0


def adjoint2d_full(dLduK, K):
    """Adjoint through K 2D sweeps for a loss that reads all of u_K.

    dLduK: full array (ny+2, nx+2) of dL/du_K, ring included.  A sweep copies
    the ring, so the ring of u_K is the boundary data g itself and dL/du_K on
    the ring passes to g unchanged; the interior part runs through the FP64
    recurrence of adjoint2d.  Returns (Gb over the interior, dL/dU0 over all
    nodes: interior lam_0, non-corner ring Gring + dL/du_K, corners dL/du_K)."""
    dLduK = np.asarray(dLduK, dtype=np.float64)
    Gb, Gring, lam0 = adjoint2d(np.ascontiguousarray(interior(dLduK)), K)
    dU0 = Gring.copy()
    ring = np.ones(dLduK.shape, dtype=bool)
    interior(ring)[...] = False
    dU0[ring] = Gring[ring] + dLduK[ring]
    interior(dU0)[...] = lam0
    return Gb, dU0


def gradients2d(U0, f, h2, target, K):
    """FP64 gradients of L = 1/2 ||u_K - t||^2 with respect to the source f and
    the full initial state U0 (ring = boundary values g, interior = u_0).

    Returns (L, dL/df over the interior, dL/dU0 over all nodes: ring entries
    are dL/dg, interior entries dL/du_0, corners 0)."""
    U0 = np.asarray(U0, dtype=np.float64)
    b = scale_source(f, h2, np.float64)
    uK = sweep(U0, b, K)
    lamK = interior(uK) - np.asarray(target, dtype=np.float64)
    Gb, Gring, lam0 = adjoint2d(lamK, K)
    dU0 = Gring.copy()
    interior(dU0)[...] = lam0
    return loss(uK, target), h2 * Gb, dU0


def fd_difference_loss(uplus, uminus, target):
    """L(u+) - L(u-) summed cell by cell as sum (u+ - u-) * ((u+ + u-)/2 - t),
    which avoids cancelling two large sums against each other.  The loss is
    over the interior when target has the interior shape, over every node
    (ring included) when it has the full shape."""
    t = np.asarray(target, dtype=np.float64)
    if t.shape == uplus.shape:
        a = np.asarray(uplus, dtype=np.float64)
        c = np.asarray(uminus, dtype=np.float64)
    else:
        a = interior(uplus).astype(np.float64)
        c = interior(uminus).astype(np.float64)
    return float(np.sum((a - c) * (0.5 * (a + c) - t)))


def fd_grad_source(U0, f, h2, target, K, index, eps):
    """Central finite difference of L with respect to f[index] (FP64)."""
    fp = np.array(f, dtype=np.float64)
    fm = np.array(f, dtype=np.float64)
    fp[index] += eps
    fm[index] -= eps
    up = sweep(np.asarray(U0, dtype=np.float64), scale_source(fp, h2), K)
    um = sweep(np.asarray(U0, dtype=np.float64), scale_source(fm, h2), K)
    return fd_difference_loss(up, um, target) / (2.0 * eps)


def fd_grad_state(U0, f, h2, target, K, index, eps):
    """Central finite difference of L with respect to U0[index] (any node,
    ring entries are boundary values)."""
    b = scale_source(f, h2) if f is not None else None
    Up = np.array(U0, dtype=np.float64)
    Um = np.array(U0, dtype=np.float64)
    Up[index] += eps
    Um[index] -= eps
    return fd_difference_loss(sweep(Up, b, K), sweep(Um, b, K), target) / (2.0 * eps)
