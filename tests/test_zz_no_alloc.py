"""h3d_matvec_noalloc through the C ABI: the product that allocates nothing.

Its output must equal h3d_matvec's bitwise (the same kernels, the same
summation order, only the scratch lives elsewhere), on two calls in a row,
the second with a smaller input, and sizes beyond its static scratch must be
refused before any launch.
"""
import ctypes

import numpy as np
import pytest

from paper_2307_16303_amd import hodlr3d, inputs

pytestmark = pytest.mark.gpu

CUBE = dict(box_lo=inputs.CUBE_LO, box_side=inputs.CUBE_SIDE)
IO_F64 = 0  # h3d_dtype H3D_F64: x and y in double precision


def torch_mod():
    import torch
    return torch


def _products(op, X, noalloc):
    """Y = K~X through h3d_matvec or h3d_matvec_noalloc on caller-owned x and y."""
    torch = torch_mod()
    lib = hodlr3d.load_library()
    n = op.n
    X2 = np.asarray(X).reshape(n, -1)
    nrhs = X2.shape[1]
    xt = torch.as_tensor(np.ascontiguousarray(X2.T), device="cuda")  # column-major n x nrhs
    yt = torch.full_like(xt, float("nan"))
    fn = lib.h3d_matvec_noalloc if noalloc else lib.h3d_matvec
    st = fn(op.handle, ctypes.c_void_p(xt.data_ptr()), ctypes.c_void_p(yt.data_ptr()), nrhs, n, n,
            IO_F64, None)
    assert st == hodlr3d.H3D_OK, lib.h3d_last_error().decode()
    torch.cuda.synchronize()
    return yt.cpu().numpy().T


def test_noalloc_equals_matvec_on_two_calls():
    torch = torch_mod()
    # sizes whose scratch fits the static array (about 40 MB at three right-hand sides)
    big = inputs.uniform_points(12000, seed=61)
    small = inputs.uniform_points(6000, seed=62)
    op_big = hodlr3d.build(torch.as_tensor(big, device="cuda"), leaf_size=32, tol=1e-7, **CUBE)
    op_small = hodlr3d.build(torch.as_tensor(small, device="cuda"), leaf_size=16, tol=1e-7,
                             factor_dtype="fp32", **CUBE)
    try:
        # first call: the larger plan with three right-hand sides
        X = inputs.normal_rhs(12000, seed=63, nrhs=3)
        print("[noalloc] n=12000 nrhs=3", flush=True)
        np.testing.assert_array_equal(_products(op_big, X, True), _products(op_big, X, False))
        # second call, right after: a smaller input (another plan, one RHS),
        # reusing the same static scratch
        x = inputs.normal_rhs(6000, seed=64)
        print("[noalloc] n=6000 nrhs=1", flush=True)
        np.testing.assert_array_equal(_products(op_small, x, True), _products(op_small, x, False))
        # and the larger plan once more with one RHS after the smaller call
        x = inputs.normal_rhs(12000, seed=65)
        print("[noalloc] n=12000 nrhs=1", flush=True)
        np.testing.assert_array_equal(_products(op_big, x, True), _products(op_big, x, False))
        # the Python binding
        xt = torch.as_tensor(x, device="cuda")
        np.testing.assert_array_equal(op_big.matvec_noalloc(xt).cpu().numpy(),
                                      op_big.matvec(xt).cpu().numpy())
    finally:
        op_big.close()
        op_small.close()


def test_noalloc_refuses_what_it_cannot_hold():
    torch = torch_mod()
    lib = hodlr3d.load_library()
    n = 1 << 20  # 16 n bytes of sorted input and sums alone exceed 64 MiB at nrhs = 4
    pts = inputs.uniform_points(4000, seed=66)
    op = hodlr3d.build(torch.as_tensor(pts, device="cuda"), leaf_size=32, tol=1e-6, **CUBE)
    try:
        x = torch.zeros((8, 4000), dtype=torch.float64, device="cuda")
        y = torch.zeros_like(x)
        # eight right-hand sides take the matrix-core path, which keeps plan scratch
        st = lib.h3d_matvec_noalloc(op.handle, ctypes.c_void_p(x.data_ptr()),
                                    ctypes.c_void_p(y.data_ptr()), 8, 4000, 4000,
                                    IO_F64, None)
        assert st == hodlr3d.H3D_EINVAL
        assert b"nrhs" in lib.h3d_last_error()
    finally:
        op.close()
    big = inputs.uniform_points(n, seed=67)
    op = hodlr3d.build(torch.as_tensor(big, device="cuda"), leaf_size=64, tol=1e-4, **CUBE)
    try:
        x = torch.zeros((4, n), dtype=torch.float64, device="cuda")
        y = torch.full_like(x, 7.0)
        st = lib.h3d_matvec_noalloc(op.handle, ctypes.c_void_p(x.data_ptr()),
                                    ctypes.c_void_p(y.data_ptr()), 4, n, n, IO_F64, None)
        assert st == hodlr3d.H3D_EINVAL
        assert b"scratch" in lib.h3d_last_error()
        torch.cuda.synchronize()
        assert bool((y == 7.0).all())  # nothing launched
    finally:
        op.close()
