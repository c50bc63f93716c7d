"""Batched solver parity: every grid of a ragged batch against the oracle's
solve with the same relative-residual stop rule (same stop sweep, same
status, bit-exact final state), captured hipGraph replays against eager
launches, edge cases of the stop rule, and batched vs single-grid runs."""
import math
import sys

import numpy as np
import pytest

import oracle
import synthetic
from gpu_util import bits_equal

pytestmark = pytest.mark.gpu

RNG = np.random.default_rng(31)


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def make_batch(sizes, dtype, device, seed_base=4000, block=64, ring_seed=None):
    import torch
    import paper_2303_02543_amd as jb
    tdt = torch.float32 if dtype == np.float32 else torch.float64
    B = jb.Batch(sizes, tdt, block=block, device=device)
    inputs = []
    for i, (nx, ny) in enumerate(sizes):
        U0 = np.zeros((ny + 2, nx + 2))
        if ring_seed is not None:
            U0 = synthetic.uniform((ny + 2, nx + 2), ring_seed + i)
            U0[1:-1, 1:-1] = 0.0
        f = np.random.default_rng(seed_base + i).standard_normal((ny, nx)) * 10
        h2 = synthetic.spacing2(max(nx, ny))
        U0d, fd = U0.astype(dtype), f.astype(dtype)
        B.set_grid(i, torch.from_numpy(U0d).to(device), torch.from_numpy(fd).to(device), h2)
        inputs.append((U0d, fd, h2))
    return B, inputs


SIZES = [(17, 17), (33, 21), (64, 64), (100, 37), (9, 130), (257, 257), (5, 5), (48, 200)]


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("use_graph", [True, False])
def test_batch_matches_oracle_stop_rule(device, dtype, use_graph):
    tol, cap, R = 1e-3, 700, 25
    B, inputs = make_batch(SIZES, dtype, device, ring_seed=77)
    try:
        B.set_tuning(0, 0, use_graph)
        say("batch dtype=%s graph=%s" % (np.dtype(dtype).name, use_graph))
        sweeps, rel, status = B.solve(tol, cap, R)
        finals = [B.get_grid(i).cpu().numpy() for i in range(len(SIZES))]
    finally:
        B.close()
    import paper_2303_02543_amd as jb
    stopped_early = 0
    for i, (U0, f, h2) in enumerate(inputs):
        b = oracle.scale_source(f, h2, dtype)
        out = oracle.solve(U0, b, cap, R, tol)
        assert sweeps[i] == out["sweeps"], (i, sweeps[i], out["sweeps"])
        assert jb.STATUS_NAMES[status[i]] == out["status"], (i, status[i], out["status"])
        assert bits_equal(finals[i], out["u"]), "grid %d final state" % i
        assert math.isclose(rel[i], out["rel"], rel_tol=1e-12)
        stopped_early += out["status"] == "converged"
    assert 0 < stopped_early < len(SIZES)   # the rule fires for some grids, not all


def test_graph_replays_match_eager(device):
    """Several solves in a row (graph replays with eager work in between)
    give bit-identical results to eager launches."""
    sizes = [(130, 70), (64, 64), (257, 33)]
    res = []
    for use_graph in (False, True):
        B, _ = make_batch(sizes, np.float32, device)
        try:
            B.set_tuning(3, 16, use_graph)
            runs = []
            for rep in range(3):
                sw, rl, st = B.solve(1e-9, 120, 20)
                runs.append((sw, rl, st, [B.get_grid(i).cpu().numpy() for i in range(len(sizes))]))
                # eager work between replays, then reset the grids
                import torch
                torch.cuda.synchronize()
                for i, (nx, ny) in enumerate(sizes):
                    U0 = np.zeros((ny + 2, nx + 2), np.float32)
                    f = (np.random.default_rng(4000 + i).standard_normal((ny, nx)) * 10).astype(np.float32)
                    B.set_grid(i, torch.from_numpy(U0).to(device), torch.from_numpy(f).to(device),
                               synthetic.spacing2(max(nx, ny)))
            res.append(runs)
        finally:
            B.close()
    base = res[0][0]
    for runs in res:
        for sw, rl, st, fin in runs:
            assert sw == base[0] and st == base[2] and rl == base[1]
            for a, b in zip(fin, base[3]):
                assert bits_equal(a, b)


def test_stop_rule_edge_cases(device):
    import torch
    import paper_2303_02543_amd as jb
    sizes = [(16, 16), (16, 16), (16, 16)]
    B = jb.Batch(sizes, torch.float64, block=64, device=device)
    try:
        # grid 0: exact fixed point (constant ring and interior, no source) -> res_0 = 0
        U = np.full((18, 18), 2.5)
        z = np.zeros((16, 16))
        B.set_grid(0, torch.from_numpy(U).to(device), torch.from_numpy(z).to(device), 1e-3)
        # grid 1: a NaN in the state -> diverged
        U1 = RNG.uniform(0, 1, (18, 18))
        U1[5, 5] = np.nan
        B.set_grid(1, torch.from_numpy(U1).to(device), torch.from_numpy(z).to(device), 1e-3)
        # grid 2: ordinary, runs to the cap (not a multiple of R)
        U2 = RNG.uniform(0, 1, (18, 18))
        B.set_grid(2, torch.from_numpy(U2).to(device), torch.from_numpy(z).to(device), 1e-3)
        sw, rl, st = B.solve(1e-30, 23, 10)
        assert st == [jb.JACOBI_CONVERGED, jb.JACOBI_DIVERGED, jb.JACOBI_MAX_SWEEPS]
        assert sw[0] == 0 and sw[1] == 0 and sw[2] == 23
        assert bits_equal(B.get_grid(0).cpu().numpy(), U)
        assert bits_equal(B.get_grid(2).cpu().numpy(), oracle.sweep(U2, None, 23))
        # max_sweeps = 0: only the initial check
        B.set_grid(2, torch.from_numpy(U2).to(device), torch.from_numpy(z).to(device), 1e-3)
        B.set_grid(0, torch.from_numpy(U).to(device), torch.from_numpy(z).to(device), 1e-3)
        B.set_grid(1, torch.from_numpy(U2).to(device), torch.from_numpy(z).to(device), 1e-3)
        sw, rl, st = B.solve(1e-6, 0, 10)
        assert sw == [0, 0, 0] and st[1] == jb.JACOBI_MAX_SWEEPS
    finally:
        B.close()


def test_autotune_is_bit_neutral_and_batch_equals_single(device):
    import torch
    import paper_2303_02543_amd as jb
    sizes = [(300, 257), (1025, 513), (257, 300)]
    K = 60
    B, inputs = make_batch(sizes, np.float32, device, block=256)
    try:
        d, r = B.autotune(20)
        say("batch autotune depth=%d rows=%d" % (d, r))
        for i, (U0, f, h2) in enumerate(inputs):
            B.set_grid(i, torch.from_numpy(U0).to(device), torch.from_numpy(f).to(device), h2)
        sw, rl, st = B.solve(0.0, K, 20)
        assert sw == [K] * len(sizes)
        finals = [B.get_grid(i).cpu().numpy() for i in range(len(sizes))]
    finally:
        B.close()
    for i, (nx, ny) in enumerate(sizes):
        U0, f, h2 = inputs[i]
        s = jb.Solver((nx, ny), (2, 2), torch.float32, device=device)
        try:
            s.set_state(torch.from_numpy(U0).to(device))
            s.set_source(torch.from_numpy(f).to(device), h2)
            s.sweep(K)
            single = s.get_state().cpu().numpy()
        finally:
            s.close()
        assert bits_equal(finals[i], single), "grid %d batched != single" % i
