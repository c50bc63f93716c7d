"""The autotuner and the profiling records, through the C ABI.

Autotuning only picks among schedules that compute identical results, so a
tuned run must still equal the oracle bit for bit; its result is cached per
problem shape in the file JACOBI_TUNE_CACHE names, and a cache line the
library cannot use is ignored (the shape is tuned again).  The profiling
records count exactly the passes the host planner issues: a 25-sweep run at
depth 4 is split into passes of 4, 4, 4, 4, 3, 3, 3 sweeps."""
import sys

import numpy as np
import pytest

import oracle
import synthetic
from gpu_util import bits_equal, to_device

pytestmark = pytest.mark.gpu

RNG = np.random.default_rng(77)


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def _problem(nx, ny):
    U0 = RNG.uniform(0, 1, (ny + 2, nx + 2)).astype(np.float32)
    f = (RNG.standard_normal((ny, nx)) * 100).astype(np.float32)
    return U0, f, synthetic.spacing2(max(nx, ny))


def test_autotune_cache_and_bit_neutral(device, tmp_path, monkeypatch):
    import torch
    import paper_2303_02543_amd as jb
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("JACOBI_TUNE_CACHE", str(cache))
    nx, ny, K = 300, 200, 30
    U0, f, h2 = _problem(nx, ny)
    want = oracle.sweep(U0, oracle.scale_source(f, h2, np.float32), K)
    s1 = jb.Solver((nx, ny), (3, 2), torch.float32, device=device)
    s2 = jb.Solver((nx, ny), (3, 2), torch.float32, device=device)
    try:
        tuned = s1.autotune(10, with_source=True)
        say("autotune ->", tuned)
        lines = cache.read_text().splitlines()
        assert len(lines) == 1 and lines[0].endswith("-> %d %d %d" % tuned)
        # a second handle of the same shape takes the cached schedule
        assert s2.autotune(10, with_source=True) == tuned
        assert len(cache.read_text().splitlines()) == 1
        d2, r2, f2 = s2.get_tuning()
        assert (d2, f2) == (tuned[0], tuned[2]) and (tuned[1] == 0 or r2 == tuned[1])
        s2.set_source(to_device(f, np.float32, device), h2)
        s2.set_state(to_device(U0, np.float32, device))
        s2.sweep(K)
        got = s2.get_state().cpu().numpy()
        assert bits_equal(got, want), "tuned schedule %s" % (tuned,)
        # an unusable cache line (flag bits the library does not know) for
        # this shape is skipped: the shape is tuned again and a line added
        key = lines[0].split(" -> ")[0]
        cache.write_text("%s -> 1 0 1024\n" % key)
        again = s1.autotune(10, with_source=True)
        assert again[0] >= 1 and len(cache.read_text().splitlines()) == 2
    finally:
        s1.close()
        s2.close()


def test_profile_records_count_passes(device):
    import torch
    import paper_2303_02543_amd as jb
    nx, ny, K = 513, 260, 25
    U0, f, h2 = _problem(nx, ny)
    cells = nx * ny
    s = jb.Solver((nx, ny), (3, 5), torch.float32, device=device)
    try:
        s.set_source(to_device(f, np.float32, device), h2)
        s.set_state(to_device(U0, np.float32, device))
        s.set_tuning(4, 0, 0)
        s.profile(True)
        s.sweep(K)
        p = s.profile_read(0)
        p4, p3 = s.profile_read(4), s.profile_read(3)
        s.profile(False)
        say("profile", p, p4, p3)
        assert p["launches"] == 7 and p4["launches"] == 4 and p3["launches"] == 3
        assert p["cell_updates"] == cells * K
        assert p["alg_bytes"] == 7 * cells * 4 * 3  # state r+w, source r, FP32
        assert p["ms"] > 0 and p["ms"] == pytest.approx(p4["ms"] + p3["ms"])
        # the explicit-halo schedule records one launch per sweep
        s.set_tuning(1, 0, jb.JACOBI_FLAG_EXPLICIT_HALO)
        s.profile(True)
        s.sweep(5)
        q = s.profile_read(0)
        s.profile(False)
        assert q["launches"] == 5 and q["cell_updates"] == cells * 5
        got = s.get_state().cpu().numpy()
    finally:
        s.close()
    assert bits_equal(got, oracle.sweep(U0, oracle.scale_source(f, h2, np.float32), K + 5))
