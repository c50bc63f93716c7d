"""CPU-only checks of the C ABI: the library loads, exports every entry point
include/jacobi.h declares, and rejects bad arguments before touching HIP."""
import ctypes
import os
import re

import pytest

import paper_2303_02543_amd as jb

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "jacobi.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(jacobi_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = jb.lib()
    names = declared_functions()
    assert len(names) >= 15
    for name in names:
        assert hasattr(L, name), "missing export %s" % name
    # the binding wraps exactly the declared functions
    assert sorted(jb.exported_symbols()) == names


def ws_bytes(ndim, grid, blocks, dtype):
    return jb.jacobi_workspace_bytes(ndim, grid, blocks, dtype)


def expect_status(status, fn, *args):
    with pytest.raises(jb.JacobiError) as ei:
        fn(*args)
    assert ei.value.status == status, str(ei.value)
    return str(ei.value)


def test_workspace_bytes_for_the_workloads():
    # 2D 8192^2 FP32 in 16x16 blocks of 512^2: two state buffers of padded
    # blocks + the blocked source; the sizes must at least cover the data
    b = ws_bytes(2, [8192, 8192], [16, 16], jb.JACOBI_F32)
    assert b >= 3 * 8192 * 8192 * 4
    assert b < 3.2 * 8192 * 8192 * 4
    b3 = ws_bytes(3, [512, 512, 512], [8, 8, 8], jb.JACOBI_F64)
    assert b3 >= 3 * 512 ** 3 * 8
    assert ws_bytes(2, [1, 1], [1, 1], jb.JACOBI_F64) > 0


@pytest.mark.parametrize("ndim,grid,blocks,dtype,frag", [
    (1, [8], [1], 0, "ndim"),
    (4, [8] * 4, [1] * 4, 0, "ndim"),
    (2, [0, 8], [1, 1], 0, "grid[0]"),
    (2, [8, -3], [1, 1], 0, "grid[1]"),
    (2, [8, 8], [0, 1], 0, "blocks[0]"),
    (2, [8, 8], [1, 9], 0, "blocks[1]"),
    (2, [8, 8], [1, 1], 7, "dtype"),
    (2, [9, 8], [2, 1], 0, "empty"),          # x extent rounds up to 8: 8 + 1 ok...
    (2, [16, 8], [3, 1], 0, "empty"),         # 3 blocks of 8 cannot cover 16
    (3, [8, 8, 10], [1, 1, 6], 1, "empty"),   # ceil(10/6) = 2 -> 5 blocks suffice
    (2, [2 ** 31, 8], [1, 1], 0, "grid[0]"),
])
def test_workspace_bytes_rejects(ndim, grid, blocks, dtype, frag):
    if frag == "empty" and grid == [9, 8]:
        # 9 columns, 2 blocks: extent ceil(9/2)=5 -> 8, last block has 1: valid
        assert ws_bytes(ndim, grid, blocks, dtype) > 0
        return
    msg = expect_status(jb.JACOBI_E_INVAL, ws_bytes, ndim, grid, blocks, dtype)
    assert frag in msg


def test_null_pointers_and_handles_rejected():
    L = jb.lib()
    assert L.jacobi_workspace_bytes(2, None, None, 0, None) == jb.JACOBI_E_INVAL
    out = ctypes.c_void_p()
    g = jb._arr64([8, 8])
    # NULL workspace is rejected before any HIP call
    one = jb._arr64([1, 1])
    assert L.jacobi_create(2, g, one, 0, None, 1 << 20, None, ctypes.byref(out)) == jb.JACOBI_E_INVAL
    assert "workspace" in jb.jacobi_last_error()
    assert out.value is None
    # misaligned workspace pointer
    assert L.jacobi_create(2, g, jb._arr64([1, 1]), 0, ctypes.c_void_p(16), 1 << 30, None,
                           ctypes.byref(out)) == jb.JACOBI_E_INVAL
    assert "aligned" in jb.jacobi_last_error()
    # too small workspace
    assert L.jacobi_create(2, g, jb._arr64([1, 1]), 0, ctypes.c_void_p(256), 16, None,
                           ctypes.byref(out)) == jb.JACOBI_E_NOMEM
    for name in ["jacobi_set_state", "jacobi_get_state", "jacobi_set_stream"]:
        assert getattr(L, name)(None, None) == jb.JACOBI_E_INVAL
    assert L.jacobi_sweep(None, 1) == jb.JACOBI_E_INVAL
    assert L.jacobi_halo_exchange(None) == jb.JACOBI_E_INVAL
    assert L.jacobi_residual(None, None) == jb.JACOBI_E_INVAL
    assert L.jacobi_residual_async(None, None) == jb.JACOBI_E_INVAL
    assert L.jacobi_solve(None, 1, 1, None) == jb.JACOBI_E_INVAL
    assert L.jacobi_set_tuning(None, 1, 1, 0) == jb.JACOBI_E_INVAL
    assert L.jacobi_profile(None, 1) == jb.JACOBI_E_INVAL
    assert L.jacobi_profile_read(None, 0, None, None, None, None) == jb.JACOBI_E_INVAL
    assert L.jacobi_autotune(None, 10, 1, None, None, None) == jb.JACOBI_E_INVAL
    assert L.jacobi_destroy(None) == jb.JACOBI_OK


def test_batch_arguments_rejected():
    L = jb.lib()
    out = ctypes.c_void_p()
    sz = ctypes.c_size_t()
    good = jb._arr64([300, 257, 64, 64])
    assert L.jacobi_batch_workspace_bytes(2, good, 64, 0, ctypes.byref(sz)) == jb.JACOBI_OK
    assert sz.value > 2 * (302 * 259 + 66 * 66) * 4
    assert L.jacobi_batch_workspace_bytes(0, good, 64, 0, ctypes.byref(sz)) == jb.JACOBI_E_INVAL
    assert L.jacobi_batch_workspace_bytes(2, None, 64, 0, ctypes.byref(sz)) == jb.JACOBI_E_INVAL
    assert L.jacobi_batch_workspace_bytes(2, good, 4, 0, ctypes.byref(sz)) == jb.JACOBI_E_INVAL
    assert L.jacobi_batch_workspace_bytes(2, jb._arr64([0, 5, 5, 5]), 64, 0,
                                          ctypes.byref(sz)) == jb.JACOBI_E_INVAL
    assert L.jacobi_batch_create(2, good, 64, 0, None, 1 << 30, None,
                                 ctypes.byref(out)) == jb.JACOBI_E_INVAL
    assert L.jacobi_batch_destroy(None) == jb.JACOBI_OK
    assert L.jacobi_batch_solve(None, 1e-6, 10, 5, None, None, None) == jb.JACOBI_E_INVAL
    assert L.jacobi_batch_set_tuning(None, 1, 8, 1) == jb.JACOBI_E_INVAL
    assert L.jacobi_adjoint_begin(None, None, None) == jb.JACOBI_E_INVAL
    assert L.jacobi_adjoint_sweep(None, 1) == jb.JACOBI_E_INVAL
    assert L.jacobi_adjoint_end(None, 1.0, None, None) == jb.JACOBI_E_INVAL
    assert L.jacobi_forward_ckpt(None, 10, 5, None) == jb.JACOBI_E_INVAL
    assert L.jacobi_adjoint(None, 10, 5, None, 1.0, None, None) == jb.JACOBI_E_INVAL


def test_adjoint_entry_points_declared_with_their_arguments():
    # the one-call checkpointed forward / adjoint pair is part of the ABI
    text = open(os.path.join(ROOT, "include", "jacobi.h")).read()
    assert re.search(r"int jacobi_forward_ckpt\(jacobi_t h, int64_t K, int64_t C, void \*ckpt\);",
                     text)
    assert re.search(r"int jacobi_adjoint\(jacobi_t h, int64_t K, int64_t C, const void \*dL_duK, "
                     r"double h2,\s+double \*dL_df, double \*dL_dU0\);", text)
    L = jb.lib()
    assert L.jacobi_forward_ckpt.argtypes == [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64,
                                              ctypes.c_void_p]
    assert len(L.jacobi_adjoint.argtypes) == 7


def test_strerror_and_depths():
    assert jb.jacobi_strerror(0) == "success"
    assert "invalid" in jb.jacobi_strerror(jb.JACOBI_E_INVAL)
    assert jb.jacobi_strerror(-99) == "unknown status"
    assert jb.jacobi_max_depth(2, jb.JACOBI_F32) >= 4
    assert jb.jacobi_max_depth(2, jb.JACOBI_F64) >= 2
    assert jb.jacobi_max_depth(3, jb.JACOBI_F32) >= 1
    with pytest.raises(jb.JacobiError):
        jb.jacobi_max_depth(5, 0)


def test_solver_refuses_without_gpu():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    with pytest.raises(RuntimeError, match="no GPU"):
        jb.Solver((16, 16), (2, 2), torch.float32)


def test_noalloc_arguments_rejected_before_any_hip_call():
    L = jb.lib()
    p = ctypes.c_void_p(256)  # never dereferenced: every case fails its checks first
    g, b = jb._arr64([64, 64]), jb._arr64([2, 2])
    f = L.jacobi_solve_noalloc
    assert f(2, g, b, 0, None, p, 1e-4, 10, 5, p, p, None) == jb.JACOBI_E_INVAL
    assert f(2, g, b, 0, p, p, 1e-4, 10, 5, None, p, None) == jb.JACOBI_E_INVAL
    assert f(2, g, b, 0, p, p, 1e-4, 10, 5, p, None, None) == jb.JACOBI_E_INVAL
    assert f(2, g, b, 0, p, p, 1e-4, -1, 5, p, p, None) == jb.JACOBI_E_INVAL
    assert f(2, g, b, 0, p, p, 1e-4, 10, 0, p, p, None) == jb.JACOBI_E_INVAL
    assert f(2, g, b, 0, p, p, -1.0, 10, 5, p, p, None) == jb.JACOBI_E_INVAL
    assert f(2, g, b, 9, p, p, 1e-4, 10, 5, p, p, None) == jb.JACOBI_E_INVAL
    assert f(2, g, jb._arr64([65, 1]), 0, p, p, 1e-4, 10, 5, p, p, None) == jb.JACOBI_E_INVAL
    # a workspace beyond the scratch array is refused with a clear message
    big = jb._arr64([4096, 4096])
    need = jb.jacobi_workspace_bytes(2, [4096, 4096], [8, 8], jb.JACOBI_F32)
    assert need > jb.JACOBI_NOALLOC_MAX_BYTES
    assert f(2, big, jb._arr64([8, 8]), 0, p, p, 1e-4, 10, 5, p, p, None) == jb.JACOBI_E_NOMEM
    msg = jb.jacobi_last_error()
    assert "scratch" in msg and str(need) in msg
    # the limit in the binding is the header's
    text = open(os.path.join(ROOT, "include", "jacobi.h")).read()
    m = re.search(r"#define JACOBI_NOALLOC_MAX_BYTES \((\d+)u << (\d+)\)", text)
    assert m and int(m.group(1)) << int(m.group(2)) == jb.JACOBI_NOALLOC_MAX_BYTES
    # a problem that fits passes every check (2048^2 FP32 in 4x4 blocks)
    assert jb.jacobi_workspace_bytes(2, [2048, 2048], [4, 4], jb.JACOBI_F32) <= \
        jb.JACOBI_NOALLOC_MAX_BYTES


def test_deep_halo_arguments():
    # sizes: larger than the one-cell layout, growing with the frame depth
    base = jb.jacobi_workspace_bytes(2, [8192, 8192], [16, 16], jb.JACOBI_F32)
    d5 = jb.jacobi_deep_workspace_bytes(2, [8192, 8192], [16, 16], jb.JACOBI_F32, 5)
    d13 = jb.jacobi_deep_workspace_bytes(2, [8192, 8192], [16, 16], jb.JACOBI_F32, 13)
    assert base < d5 < d13
    # the stored depth is rounded up (FP32: 1 + a multiple of 4): 6 -> 9 = 9
    assert jb.jacobi_deep_workspace_bytes(2, [8192, 8192], [16, 16], jb.JACOBI_F32, 6) == \
        jb.jacobi_deep_workspace_bytes(2, [8192, 8192], [16, 16], jb.JACOBI_F32, 9)
    for halo, frag in ((0, "halo"), (65, "halo")):
        msg = expect_status(jb.JACOBI_E_INVAL, jb.jacobi_deep_workspace_bytes, 2, [64, 64],
                            [2, 2], jb.JACOBI_F32, halo)
        assert frag in msg
    # a frame deeper than a block is refused: 37 x 29 in 3 x 4 blocks has
    # blocks of 5 nodes at the far edges
    msg = expect_status(jb.JACOBI_E_INVAL, jb.jacobi_deep_workspace_bytes, 2, [37, 29], [3, 4],
                        jb.JACOBI_F32, 9)
    assert "exceeds the block extent" in msg
    # one block per axis: any depth up to 64
    assert jb.jacobi_deep_workspace_bytes(3, [8, 8, 8], [1, 1, 1], jb.JACOBI_F64, 64) > 0
    L = jb.lib()
    out = ctypes.c_void_p()
    g, b = jb._arr64([64, 64]), jb._arr64([2, 2])
    assert L.jacobi_deep_create(2, g, b, 0, 5, None, 1 << 30, None,
                                ctypes.byref(out)) == jb.JACOBI_E_INVAL
    assert L.jacobi_deep_create(2, g, b, 0, 5, ctypes.c_void_p(256), 16, None,
                                ctypes.byref(out)) == jb.JACOBI_E_NOMEM
    assert L.jacobi_get_halo(None, None) == jb.JACOBI_E_INVAL
