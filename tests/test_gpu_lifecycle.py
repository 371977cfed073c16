"""Plan and graph lifecycle through the C ABI: rules that keep captured graphs
valid, handles used after release, and an allocator that fails mid-build.

Every failure here is a host-side condition (an argument the library refuses,
an allocator callback returning NULL); no kernel is made to fail.
"""
import ctypes
import gc

import numpy as np
import pytest

from paper_2307_16303_amd import hodlr3d, inputs

pytestmark = pytest.mark.gpu

CUBE = dict(box_lo=inputs.CUBE_LO, box_side=inputs.CUBE_SIDE)


def torch_mod():
    import torch
    return torch


def test_graph_holds_scratch_and_tables():
    """While a graph exists, calls that would reallocate what it captured are
    refused (H3D_EINVAL) and change nothing; the replay stays bitwise equal."""
    torch = torch_mod()
    pts = inputs.uniform_points(15000, seed=50)
    print("[graph guard] n=15000 leaf 32", flush=True)
    op = hodlr3d.build(torch.as_tensor(pts, device="cuda"), leaf_size=32, tol=1e-8, **CUBE)
    x = torch.as_tensor(inputs.normal_rhs(15000, seed=51), device="cuda")
    eager = op.matvec(x).cpu().numpy()
    g = op.graph(x)
    X4 = torch.as_tensor(inputs.normal_rhs(15000, seed=52, nrhs=4), device="cuda")
    X64 = torch.as_tensor(inputs.normal_rhs(15000, seed=53, nrhs=64), device="cuda")
    for call in (lambda: op.matvec(X4), lambda: op.rmatvec(X4), lambda: op.autotune(1),
                 lambda: op.autotune(4), lambda: op.graph(X4), lambda: op.close()):
        with pytest.raises(hodlr3d.H3DError) as e:
            call()
        assert e.value.status == hodlr3d.H3D_EINVAL
    # the many-RHS path allocates its own buffers (nothing the graph holds)
    y64 = op.matvec(X64)
    torch.cuda.synchronize()
    for _ in range(3):
        np.testing.assert_array_equal(g.launch().cpu().numpy(), eager)
        torch.cuda.synchronize()
    # a second graph at the many-RHS width, then growth of that width is refused
    g64 = op.graph(X64)
    X80 = torch.as_tensor(inputs.normal_rhs(15000, seed=54, nrhs=80), device="cuda")
    with pytest.raises(hodlr3d.H3DError) as e:
        op.matvec(X80)
    assert e.value.status == hodlr3d.H3D_EINVAL
    np.testing.assert_array_equal(g64.launch().cpu().numpy(), y64.cpu().numpy())
    g64.close()
    g.close()
    # with no graph left everything works again
    y4 = op.matvec(X4).cpu().numpy()
    op.autotune(1)
    for c in range(4):
        yc = op.matvec(X4[:, c].contiguous()).cpu().numpy()
        assert np.linalg.norm(y4[:, c] - yc) <= 1e-14 * np.linalg.norm(yc)
    assert op.matvec(X80).shape == (15000, 80)
    op.close()


def test_handles_after_release():
    torch = torch_mod()
    lib = hodlr3d.load_library()
    pts = inputs.uniform_points(3000, seed=55)
    op = hodlr3d.build(torch.as_tensor(pts, device="cuda"), leaf_size=32, tol=1e-8, **CUBE)
    x = torch.as_tensor(inputs.normal_rhs(3000, seed=56), device="cuda")
    y = torch.empty_like(x)
    g = op.graph(x)
    gh = ctypes.c_void_p(g._h.value)
    g.close()
    assert lib.h3d_graph_launch(gh, None) == hodlr3d.H3D_EINVAL
    assert lib.h3d_graph_destroy(gh) == hodlr3d.H3D_EINVAL
    h = ctypes.c_void_p(op.handle.value)
    op.close()
    px, py = ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr())
    assert lib.h3d_matvec(h, px, py, 1, 3000, 3000, 0, None) == hodlr3d.H3D_ENOTBUILT
    assert lib.h3d_matvec_adjoint(h, px, py, 1, 3000, 3000, 0, None) == hodlr3d.H3D_ENOTBUILT
    st = hodlr3d.Stats()
    assert lib.h3d_get_stats(h, ctypes.byref(st)) == hodlr3d.H3D_ENOTBUILT
    assert lib.h3d_autotune(h, 1, None) == hodlr3d.H3D_ENOTBUILT
    assert lib.h3d_destroy(h) == hodlr3d.H3D_EINVAL  # no double release
    # a problem of a batch belongs to its batch
    bop = hodlr3d.build_batch([torch.as_tensor(inputs.uniform_points(2000, seed=57),
                                               device="cuda")], leaf_size=32, tol=1e-8, **CUBE)
    sub = ctypes.c_void_p(bop.plans[0].handle.value)
    assert lib.h3d_destroy(sub) == hodlr3d.H3D_EINVAL
    bop.close()
    assert lib.h3d_matvec(sub, px, py, 1, 2000, 2000, 0, None) == hodlr3d.H3D_ENOTBUILT


class _FailingAllocator:
    """h3d_allocator over torch's caching allocator that returns NULL from the
    k-th request on, and counts what is still held."""

    def __init__(self, fail_at: int):
        torch = torch_mod()
        self.fail_at = fail_at
        self.calls = 0
        self.live = {}

        def _alloc(nbytes, stream, ctx):
            self.calls += 1
            if self.calls >= self.fail_at:
                return None
            p = torch.cuda.caching_allocator_alloc(int(nbytes), device=0, stream=int(stream or 0))
            self.live[p] = int(nbytes)
            return p

        def _free(ptr, nbytes, stream, ctx):
            assert ptr in self.live, "free of a pointer the allocator did not hand out"
            del self.live[ptr]
            torch.cuda.caching_allocator_delete(ptr)

        self._a = hodlr3d.ALLOC_FN(_alloc)
        self._f = hodlr3d.FREE_FN(_free)
        self.struct = hodlr3d.Allocator(self._a, self._f, None)


def test_allocator_failure_mid_build_leaks_nothing():
    torch = torch_mod()
    lib = hodlr3d.load_library()
    pts = torch.as_tensor(inputs.uniform_points(6000, seed=58), device="cuda")
    cfg = hodlr3d._make_config("laplace", 1.0, 32, 1e-8, "fp32", 0, 10, inputs.CUBE_LO,
                               inputs.CUBE_SIDE, 0, False, True)
    # how many requests a successful build makes
    ok = _FailingAllocator(1 << 30)
    h = ctypes.c_void_p()
    assert lib.h3d_build(ctypes.c_void_p(pts.data_ptr()), 6000, ctypes.byref(cfg),
                         ctypes.byref(ok.struct), None, ctypes.byref(h)) == hodlr3d.H3D_OK
    total = ok.calls
    assert lib.h3d_destroy(h) == hodlr3d.H3D_OK
    assert not ok.live
    print(f"[alloc failure] a build makes {total} requests", flush=True)
    # tensors of earlier tests that the garbage collector frees in the middle
    # of the loop would change torch's count: collect them first, and keep the
    # collector off while the count is compared
    gc.collect()
    gc.disable()
    try:
        torch.cuda.synchronize()
        base = torch.cuda.memory_allocated()
        for k in sorted({1, 2, 3, total // 4, total // 2, total - 1, total}):
            if k < 1:
                continue
            fa = _FailingAllocator(k)
            h = ctypes.c_void_p(123)
            st = lib.h3d_build(ctypes.c_void_p(pts.data_ptr()), 6000, ctypes.byref(cfg),
                               ctypes.byref(fa.struct), None, ctypes.byref(h))
            assert st == hodlr3d.H3D_ENOMEM, (k, st)
            assert h.value is None  # *out is NULL on failure
            assert not fa.live, f"request {k} failing left {len(fa.live)} allocations held"
            torch.cuda.synchronize()
            assert torch.cuda.memory_allocated() == base
    finally:
        gc.enable()
