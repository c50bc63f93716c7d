"""Helpers shared by the GPU tests: run the device path through the C ABI and
compare with the oracle.  Inputs come from synthetic/ (seeded); expected
values only ever come from oracle/."""
import numpy as np

import oracle
import synthetic


def bits_equal(a, b):
    a = np.ascontiguousarray(a)
    b = np.ascontiguousarray(b)
    return a.dtype == b.dtype and a.shape == b.shape and np.array_equal(
        a.view(np.uint8), b.view(np.uint8))


def first_mismatch(a, b):
    bad = np.argwhere(a.view(np.uint8 if a.dtype.itemsize == 1 else
                             (np.uint32 if a.dtype == np.float32 else np.uint64))
                      != b.view(np.uint32 if b.dtype == np.float32 else np.uint64))
    if len(bad) == 0:
        return None
    idx = tuple(bad[0])
    return idx, a[idx], b[idx], len(bad)


def norm_rel_err(x, ref):
    """max|x - ref| / max|ref| over the interior (FP64)."""
    xi = oracle.interior(np.asarray(x, dtype=np.float64))
    ri = oracle.interior(np.asarray(ref, dtype=np.float64))
    return float(np.max(np.abs(xi - ri)) / max(np.max(np.abs(ri)), 1e-300))


def to_device(a, dtype, device):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=dtype)).to(device)


def run_device(U0, f, h2, K, blocks, dtype, device, depth=0, rows=0, flags=0, check_every=None):
    """Run K sweeps on the device; returns (final state as numpy, residuals or None)."""
    import torch
    import paper_2303_02543_amd as jb
    tdt = torch.float32 if dtype == np.float32 else torch.float64
    grid = tuple(reversed([s - 2 for s in U0.shape]))
    s = jb.Solver(grid, blocks, tdt, device=device)
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
        torch.cuda.synchronize()
        return out, res
    finally:
        s.close()


def oracle_run(U0, f, h2, K, dtype):
    """The oracle in the run's arithmetic type (FP32 oracle for FP32 runs)."""
    U = np.ascontiguousarray(U0, dtype=dtype)
    b = None if f is None else oracle.scale_source(np.asarray(f, dtype=dtype), h2, dtype)
    return oracle.sweep(U, b, K), b


def oracle_residuals(U0, b, K, R):
    """FP64 residuals of the oracle states after 0, R, 2R, ..., K sweeps."""
    res = [oracle.residual(U0, b)]
    U = U0
    k = 0
    while k < K:
        step = min(R, K - k)
        U = oracle.sweep(U, b, step)
        k += step
        res.append(oracle.residual(U, b))
    return np.array(res), U
