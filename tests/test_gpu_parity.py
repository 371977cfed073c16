"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Integer work (tree, permutation, lists) must be bit-exact.  ACA in FP64 takes
the same decisions as the oracle (same entry formula, no FMA contraction,
sequential reductions), so ranks and pivots are compared exactly and factors
to rounding.  Mat-vec results carry relative 2-norm bounds: against the
oracle's HODLR3D with the same factors (summation order only) and against the
exact dense product (compression error, 10 tol).
"""
import numpy as np
import pytest

import oracle
from paper_2307_16303_amd import hodlr3d, inputs

pytestmark = pytest.mark.gpu

CUBE = dict(box_lo=inputs.CUBE_LO, box_side=inputs.CUBE_SIDE)


def torch_mod():
    import torch
    return torch


def gpu_build(pts, **kw):
    torch = torch_mod()
    print(f"[gpu_build] n={len(pts)} {kw}", flush=True)
    return hodlr3d.build(torch.as_tensor(np.ascontiguousarray(pts), device="cuda"), **kw)


def gpu_apply(op, x, adjoint=False, dtype="float64"):
    torch = torch_mod()
    xt = torch.as_tensor(np.asarray(x), device="cuda").to(getattr(torch, dtype))
    y = op.rmatvec(xt) if adjoint else op.matvec(xt)
    torch.cuda.synchronize()
    return y.double().cpu().numpy()


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(b))


def oracle_kw(kw):
    k = dict(kernel=kw.get("kernel", "laplace"), param=kw.get("kernel_param", 1.0),
             leaf_size=kw.get("leaf_size", 64), tol=kw.get("tol", 1e-8),
             max_rank=kw.get("max_rank", 0))
    if "box_side" in kw:
        k.update(box_lo=kw["box_lo"], box_side=kw["box_side"])
    return k


CASES = {
    "grid4096": (lambda: inputs.grid_points(16), dict(leaf_size=64, tol=1e-10, **CUBE)),
    "uniform20k_leaf32": (lambda: inputs.uniform_points(20000, 1),
                          dict(leaf_size=32, tol=1e-8, **CUBE)),
    "uniform9k_leaf8_autobox": (lambda: inputs.uniform_points(9000, 2),
                                dict(leaf_size=8, tol=1e-7)),
    "uniform3000_leaf100": (lambda: inputs.uniform_points(3000, 3),
                            dict(leaf_size=100, tol=1e-9, **CUBE)),
    # mostly tiny leaves with a cluster of full ones: the finest level in one
    # fused pass, with leaves of more than 16 rows taken in several row passes
    "clustered8k_leaf64": (lambda: inputs.clustered_points(6000, 2000, seed=4),
                           dict(leaf_size=64, tol=1e-8, **CUBE)),
}


@pytest.fixture(scope="module", params=sorted(CASES))
def case(request):
    make, kw = CASES[request.param]
    pts = make()
    op = gpu_build(pts, keep_pivots=True, **kw)
    ref = oracle.HODLR3D(pts, **oracle_kw(kw))
    yield request.param, pts, kw, op, ref
    op.close()


def test_tree_and_lists_bit_exact(case):
    name, pts, kw, op, ref = case
    st = op.stats()
    assert st["depth"] == ref.depth
    perm_o, leaf_o = ref.tree()
    np.testing.assert_array_equal(op.export("perm"), perm_o)
    np.testing.assert_array_equal(op.export("leaf_off"), leaf_o)
    far = op.export("far")
    fo = ref.far()
    for i, k in enumerate(("level", "t", "s", "m", "n")):
        np.testing.assert_array_equal(far[i], fo[k], err_msg=k)
    near = op.export("near")
    no = ref.near()
    for i, k in enumerate(("t", "s", "rel")):
        np.testing.assert_array_equal(near[i], no[k], err_msg=k)
    assert st["n_far"] == ref.num_far and st["n_near"] == ref.num_near
    lo, side = ref.box()
    np.testing.assert_array_equal(st["box_lo"], lo)
    assert st["box_side"] == side


def test_aca_decisions_match_oracle(case):
    name, pts, kw, op, ref = case
    far = op.export("far")
    fo = ref.far()
    np.testing.assert_array_equal(far[5], fo["rank"])  # ranks
    piv = op.export("pivots")
    rp, cp = ref.pivots()
    np.testing.assert_array_equal(piv[0], rp)
    np.testing.assert_array_equal(piv[1], cp)
    Ug, Vg = op.export("factors_u"), op.export("factors_v")
    Uo, Vo = ref.factors()
    assert Ug.shape == Uo.shape and Vg.shape == Vo.shape
    scale = max(np.abs(Uo).max(), 1e-300)
    assert np.abs(Ug - Uo).max() <= 1e-14 * scale
    assert np.abs(Vg - Vo).max() <= 1e-14 * max(np.abs(Vo).max(), 1e-300)
    st = op.stats()
    assert st["n_rank_capped"] == 0
    assert st["rank_sum"] == int(fo["rank"].sum()) and st["rank_max"] == int(fo["rank"].max())
    assert st["factor_entries"] == int(((fo["m"] + fo["n"]) * fo["rank"]).sum())


def test_matvec_and_adjoint_vs_oracle(case):
    name, pts, kw, op, ref = case
    x = inputs.normal_rhs(len(pts), seed=5)
    y = gpu_apply(op, x)
    ya = gpu_apply(op, x, adjoint=True)
    assert rel(y, ref.matvec(x)) <= 1e-13
    assert rel(ya, ref.rmatvec(x)) <= 1e-13
    # the GPU's own factors applied by the oracle (robust to any ACA difference)
    U, V = op.export("factors_u"), op.export("factors_v")
    ref2 = oracle.HODLR3D(pts, **oracle_kw(kw))
    ref2.set_factors(op.export("far")[5], U, V)
    assert rel(y, ref2.matvec(x)) <= 1e-13
    assert rel(ya, ref2.rmatvec(x)) <= 1e-13
    # near field and far field separately transposed: dot test
    w = inputs.normal_rhs(len(pts), seed=6)
    assert abs(w @ y - gpu_apply(op, w, adjoint=True) @ x) <= 1e-12 * np.linalg.norm(w) * np.linalg.norm(y)


def test_matvec_vs_dense(case):
    name, pts, kw, op, ref = case
    x = inputs.uniform_rhs(len(pts), seed=0)
    yd = oracle.dense_matvec(pts, x)
    assert rel(gpu_apply(op, x), yd) <= 10 * kw["tol"]


def test_multiple_rhs_are_columns(case):
    name, pts, kw, op, ref = case
    X = inputs.normal_rhs(len(pts), seed=7, nrhs=5)
    Y = gpu_apply(op, X)
    Ya = gpu_apply(op, X, adjoint=True)
    Yo = ref.matvec(X)
    # the multi-column kernels may sum in another order than the (tuned)
    # single-column ones: equal to rounding in the 2-norm
    for c in range(5):
        assert rel(Y[:, c], Yo[:, c]) <= 1e-13
        assert rel(Y[:, c], gpu_apply(op, X[:, c])) <= 1e-14
        assert rel(Ya[:, c], gpu_apply(op, X[:, c], adjoint=True)) <= 1e-14


def test_bitwise_reproducible(case):
    name, pts, kw, op, ref = case
    x = inputs.normal_rhs(len(pts), seed=8)
    a = gpu_apply(op, x)
    b = gpu_apply(op, x)
    np.testing.assert_array_equal(a, b)


def test_float32_io(case):
    name, pts, kw, op, ref = case
    x = inputs.normal_rhs(len(pts), seed=9).astype(np.float32)
    y32 = gpu_apply(op, x, dtype="float32")
    y64 = gpu_apply(op, x.astype(np.float64))
    assert rel(y32, y64) <= 1e-6


# ---------------------------------------------------------------------------
@pytest.mark.parametrize("kernel,param", [("yukawa", 1.0), ("inv_r4", 0.0), ("cos_r", 1.0)])
def test_other_kernels(kernel, param):
    pts = inputs.uniform_points(8000, seed=11)
    kw = dict(kernel=kernel, kernel_param=param, leaf_size=32, tol=1e-9, **CUBE)
    op = gpu_build(pts, **kw)
    x = inputs.normal_rhs(8000, seed=12)
    y = gpu_apply(op, x)
    ref = oracle.HODLR3D(pts, **oracle_kw(kw))
    ref.set_factors(op.export("far")[5], op.export("factors_u"), op.export("factors_v"))
    assert rel(y, ref.matvec(x)) <= 1e-13
    yd = oracle.dense_matvec(pts, x, kernel=kernel, param=param)
    assert rel(y, yd) <= 1e-7
    op.close()


@pytest.mark.parametrize("kernel,param", [("yukawa", 1.0), ("cos_r", 1.0), ("inv_r4", 0.0)])
@pytest.mark.parametrize("nrhs", [1, 16])
def test_other_kernels_fp32_entries(kernel, param, nrhs):
    """FP32 factors: the near field evaluates kernel entries in FP32 (single
    precision exp / cos and one reciprocal square root).  Against the oracle
    with the GPU's own factors (near entries in FP64 there) and against dense."""
    n = 8000
    pts = inputs.uniform_points(n, seed=11)
    kw = dict(kernel=kernel, kernel_param=param, leaf_size=32, tol=1e-9, **CUBE)
    op = gpu_build(pts, factor_dtype="fp32", **kw)
    X = inputs.normal_rhs(n, seed=12, nrhs=None if nrhs == 1 else nrhs)
    Y = gpu_apply(op, X)
    Ya = gpu_apply(op, X, adjoint=True)
    ref = oracle.HODLR3D(pts, **oracle_kw(kw))
    ref.set_factors(op.export("far")[5], op.export("factors_u"), op.export("factors_v"))
    Y2, Yo = Y.reshape(n, -1), ref.matvec(X).reshape(n, -1)
    e2, einf = colwise_errors(Y2, Yo)
    ea2, _ = colwise_errors(Ya.reshape(n, -1), ref.rmatvec(X).reshape(n, -1))
    # the near field alone, where the FP32 entries are
    yn = ref.matvec(X, far=False).reshape(n, -1)
    yd = oracle.dense_matvec(pts, X, kernel=kernel, param=param).reshape(n, -1)
    ed = max(rel(Y2[:, c], yd[:, c]) for c in range(Y2.shape[1]))
    print(f"[fp32 entries] {kernel} nrhs={nrhs}: vs oracle same factors {e2:.3e} (element "
          f"{einf:.3e}, adjoint {ea2:.3e}); vs dense {ed:.3e}; |near|/|y| "
          f"{np.linalg.norm(yn) / np.linalg.norm(Yo):.2f}")
    assert e2 <= 1e-6 and einf <= 1e-6 and ea2 <= 1e-6
    assert ed <= 1e-6
    op.close()


@pytest.mark.parametrize("dtype,bound", [("fp32", 1e-6), ("bf16", 3e-2)])
def test_precision_forms(dtype, bound):
    pts = inputs.uniform_points(20000, seed=13)
    kw = dict(leaf_size=32, tol=1e-8, **CUBE)
    x = inputs.normal_rhs(20000, seed=14)
    op64 = gpu_build(pts, **kw)
    op = gpu_build(pts, factor_dtype=dtype, **kw)
    y64, y = gpu_apply(op64, x), gpu_apply(op, x)
    yd = oracle.dense_matvec(pts, x)
    e = rel(y, yd)
    print(f"[precision] {dtype}: rel err vs dense {e:.3e} (fp64 form {rel(y64, yd):.3e})")
    assert e <= bound
    # same ACA, so the difference isolates storage rounding
    np.testing.assert_array_equal(op.export("far")[5], op64.export("far")[5])
    st, st64 = op.stats(), op64.stats()
    assert st["factor_bytes"] < st64["factor_bytes"]
    ya = gpu_apply(op, x, adjoint=True)
    w = inputs.normal_rhs(20000, seed=15)
    assert abs(w @ y - gpu_apply(op, w, adjoint=True) @ x) <= 1e-10 * np.linalg.norm(w) * np.linalg.norm(y)
    assert rel(ya, yd) <= bound
    op.close()
    op64.close()


def test_rank_cap():
    pts = inputs.grid_points(16)
    kw = dict(leaf_size=64, tol=1e-10, max_rank=12, **CUBE)
    op = gpu_build(pts, **kw)
    ref = oracle.HODLR3D(pts, **oracle_kw(kw))
    assert op.stats()["n_rank_capped"] == ref.num_capped > 0
    np.testing.assert_array_equal(op.export("far")[5], ref.far()["rank"])
    x = inputs.uniform_rhs(4096, seed=0)
    assert rel(gpu_apply(op, x), ref.matvec(x)) <= 1e-13
    op.close()


def test_small_workspace_batches():
    pts = inputs.uniform_points(20000, seed=16)
    kw = dict(leaf_size=32, tol=1e-8, **CUBE)
    a = gpu_build(pts, autotune=False, **kw)
    b = gpu_build(pts, workspace_bytes=1 << 20, autotune=False, **kw)  # many ACA batches, chunks
    x = inputs.normal_rhs(20000, seed=17)
    np.testing.assert_array_equal(gpu_apply(a, x), gpu_apply(b, x))
    np.testing.assert_array_equal(a.export("factors_v"), b.export("factors_v"))
    a.close()
    b.close()


def test_own_allocator_matches_torch_allocator():
    pts = inputs.uniform_points(5000, seed=18)
    a = gpu_build(pts, leaf_size=32, tol=1e-8, autotune=False)
    b = gpu_build(pts, leaf_size=32, tol=1e-8, use_torch_allocator=False, autotune=False)
    x = inputs.normal_rhs(5000, seed=19)
    np.testing.assert_array_equal(gpu_apply(a, x), gpu_apply(b, x))
    a.close()
    b.close()


# ---------------------------------------------------------------------------
def test_degenerate_inputs():
    # a single point: L = 0, K = [0]
    op = gpu_build(np.array([[0.1, 0.2, 0.3]]), leaf_size=4)
    assert op.stats()["depth"] == 0
    np.testing.assert_array_equal(gpu_apply(op, np.array([2.5])), [0.0])
    op.close()
    # everything in one leaf: the dense product exactly (up to summation order)
    pts = inputs.uniform_points(40, seed=20)
    op = gpu_build(pts, leaf_size=64)
    x = inputs.normal_rhs(40, seed=21)
    assert op.stats()["n_far"] == 0
    assert rel(gpu_apply(op, x), oracle.dense_matvec(pts, x)) <= 1e-14
    op.close()
    # two coincident distinct points contribute nothing to each other; no
    # depth can put them in separate leaves, so one leaf must hold both
    pts = np.array([[0.0, 0.0, 0.0], [0.0, 0.0, 0.0], [0.5, 0.0, 0.0], [0.9, 0.9, 0.9]])
    with pytest.raises(hodlr3d.H3DError) as e:
        gpu_build(pts, leaf_size=1, max_depth=3)
    assert e.value.status == hodlr3d.H3D_EDEPTH
    op = gpu_build(pts, leaf_size=2, max_depth=3)
    x = np.array([1.0, 2.0, 3.0, 4.0])
    np.testing.assert_allclose(gpu_apply(op, x), oracle.dense_matvec(pts, x), rtol=1e-14)
    op.close()


def test_error_paths():
    torch = torch_mod()
    same = np.zeros((10, 3))
    with pytest.raises(hodlr3d.H3DError) as e:
        gpu_build(same, leaf_size=2, max_depth=5)
    assert e.value.status == hodlr3d.H3D_EDEPTH
    bad = inputs.uniform_points(100, seed=22)
    bad[17, 1] = np.nan
    with pytest.raises(hodlr3d.H3DError) as e:
        gpu_build(bad, leaf_size=8)
    assert e.value.status == hodlr3d.H3D_EINVAL
    out = inputs.uniform_points(100, seed=23) * 1.5
    with pytest.raises(hodlr3d.H3DError) as e:
        gpu_build(out, leaf_size=8, **CUBE)
    assert e.value.status == hodlr3d.H3D_EINVAL
    op = gpu_build(inputs.uniform_points(100, seed=24), leaf_size=8)
    x = torch.zeros(200, dtype=torch.float64, device="cuda")
    lib = hodlr3d.load_library()
    import ctypes
    p = ctypes.c_void_p(x.data_ptr())
    p2 = ctypes.c_void_p(x.data_ptr() + 8 * 50)
    assert lib.h3d_matvec(op.handle, p, p2, 1, 100, 100, 0, None) == hodlr3d.H3D_EINVAL  # overlap
    assert lib.h3d_matvec(op.handle, p, p2, 1, 99, 100, 0, None) == hodlr3d.H3D_EINVAL  # ldx < n
    assert lib.h3d_matvec(op.handle, p, p2, 0, 100, 100, 0, None) == hodlr3d.H3D_EINVAL
    assert lib.h3d_matvec(op.handle, p, p2, 1, 100, 100, 5, None) == hodlr3d.H3D_EINVAL
    op.close()


def test_autograd_gradients():
    torch = torch_mod()
    pts = inputs.grid_points(16)
    op = gpu_build(pts, leaf_size=64, tol=1e-10, **CUBE)
    x = torch.as_tensor(inputs.uniform_rhs(4096, seed=0), device="cuda").requires_grad_(True)
    b = torch.as_tensor(inputs.normal_rhs(4096, seed=2), device="cuda")
    loss = ((hodlr3d.matvec_autograd(op, x) - b) ** 2).sum()
    loss.backward()
    g = x.grad.cpu().numpy()
    xn, bn = x.detach().cpu().numpy(), b.cpu().numpy()
    # dense FP64 gradient 2 K^T (K x - b), K symmetric
    gd = 2.0 * oracle.dense_matvec(pts, oracle.dense_matvec(pts, xn) - bn)
    assert rel(g, gd) <= 1e-8
    # central difference of the quadratic loss is exact up to rounding
    v = inputs.normal_rhs(4096, seed=3)
    h = 1e-3 * np.linalg.norm(xn) / np.linalg.norm(v)
    f = lambda z: float(np.sum((gpu_apply(op, z) - bn) ** 2))
    fd = (f(xn + h * v) - f(xn - h * v)) / (2 * h)
    assert abs(fd - g @ v) <= 1e-8 * abs(g @ v) + 1e-10 * np.linalg.norm(g) * np.linalg.norm(v)
    op.close()
    # torch's own gradient check on a small cloud
    small = inputs.uniform_points(300, seed=4)
    op2 = gpu_build(small, leaf_size=16, tol=1e-10, **CUBE)
    xs = torch.as_tensor(inputs.normal_rhs(300, seed=5), device="cuda").requires_grad_(True)
    assert torch.autograd.gradcheck(lambda z: hodlr3d.matvec_autograd(op2, z), (xs,))
    op2.close()


# ---------------------------------------------------------------------------
@pytest.mark.parametrize("name", ["uniform262k", "uniform262k_yukawa"])
def test_full_size_sampled_rows(name):
    """The benchmark configuration at full size: sampled rows of y = K~x and of
    K~^T x against the exact dense rows, and the structure against the oracle's
    tree (built without compression)."""
    w = inputs.WORKLOADS[name]
    pts = inputs.workload_points(name)
    x = inputs.workload_rhs(name)
    kw = dict(kernel=w["kernel"], leaf_size=w["leaf_size"], tol=w["tol"], **CUBE)
    op = gpu_build(pts, **kw)
    st = op.stats()
    print(f"[{name}] depth={st['depth']} far={st['n_far']} ranks={st['rank_sum']} "
          f"factor GB={st['factor_bytes'] / 1e9:.2f} build {st['build_ms'] / 1e3:.1f} s "
          f"(ACA {st['aca_ms'] / 1e3:.1f} s)", flush=True)
    ref = oracle.HODLR3D(pts, compress=False, **{k: v for k, v in oracle_kw(kw).items()
                                                  if k not in ("tol", "max_rank")})
    assert st["depth"] == ref.depth and st["n_far"] == ref.num_far and st["n_near"] == ref.num_near
    np.testing.assert_array_equal(op.export("perm"), ref.tree()[0])
    rows = inputs.sample_rows(len(pts), 384, seed=3)
    y = gpu_apply(op, x)
    yd = oracle.dense_rows(pts, x, rows, kernel=w["kernel"])
    e = rel(y[rows], yd)
    ya = gpu_apply(op, x, adjoint=True)
    ea = rel(ya[rows], yd)
    print(f"[{name}] sampled rel err {e:.3e} adjoint {ea:.3e}", flush=True)
    assert e <= 10 * w["tol"] and ea <= 10 * w["tol"]
    op.close()


def test_autotune_changes_only_summation_order():
    pts = inputs.uniform_points(30000, seed=25)
    op = gpu_build(pts, leaf_size=32, tol=1e-8, autotune=False, **CUBE)
    x = inputs.normal_rhs(30000, seed=26)
    X = inputs.normal_rhs(30000, seed=27, nrhs=6)
    y0, Y0, A0 = gpu_apply(op, x), gpu_apply(op, X), gpu_apply(op, X, adjoint=True)
    op.autotune(1)
    op.autotune(6)
    y1, Y1, A1 = gpu_apply(op, x), gpu_apply(op, X), gpu_apply(op, X, adjoint=True)
    assert rel(y1, y0) <= 1e-14 and rel(Y1, Y0) <= 1e-14 and rel(A1, A0) <= 1e-14
    np.testing.assert_array_equal(y1, gpu_apply(op, x))  # still reproducible
    op.close()


# ---------------------------------------------------------------------------
# many right-hand sides: the matrix-core (MFMA) path
@pytest.fixture(scope="module")
def rhs_cloud():
    pts = inputs.uniform_points(12000, seed=30)
    kw = dict(leaf_size=32, tol=1e-8, **CUBE)
    return pts, kw


@pytest.mark.parametrize("nrhs", [8, 16, 64, 70])
def test_many_rhs_fp64_matrix_cores(rhs_cloud, nrhs):
    pts, kw = rhs_cloud
    op = gpu_build(pts, **kw)
    X = inputs.normal_rhs(len(pts), seed=31, nrhs=nrhs)
    Y = gpu_apply(op, X)
    Ya = gpu_apply(op, X, adjoint=True)
    ref = oracle.HODLR3D(pts, **oracle_kw(kw))
    for c in (0, nrhs // 2, nrhs - 1):
        assert rel(Y[:, c], ref.matvec(X[:, c])) <= 1e-13
        assert rel(Ya[:, c], ref.rmatvec(X[:, c])) <= 1e-13
    for c in range(nrhs):
        assert rel(Y[:, c], gpu_apply(op, X[:, c])) <= 1e-13
    np.testing.assert_array_equal(Y, gpu_apply(op, X))  # reproducible
    op.close()


def colwise_errors(Y, Yo):
    """Worst column relative 2-norm error and worst element error relative to
    the column's largest entry."""
    e2 = max(rel(Y[:, c], Yo[:, c]) for c in range(Y.shape[1]))
    einf = max(float(np.abs(Y[:, c] - Yo[:, c]).max() / np.abs(Yo[:, c]).max())
               for c in range(Y.shape[1]))
    return e2, einf


@pytest.mark.parametrize("dtype,bound", [("fp32", 1e-6), ("bf16", 1e-5)])
def test_many_rhs_low_precision(rhs_cloud, dtype, bound):
    """FP32 and BF16 factors on the matrix cores, every column of a 64-RHS
    product and of its adjoint, element by element against the oracle applying
    the GPU's own stored factors in FP64 (exported exactly: FP32 values, or
    BF16 values times their power-of-two scales).  What remains is the
    arithmetic of the GPU path, bounded by `bound`: for FP32 factors x, z and
    the near-field entries rounded to FP32 and FP32 MFMA sums flushed to FP64;
    for BF16 factors the forward far field runs on the BF16 matrix cores with
    x and z carried as BF16 hi + lo pairs (2^-18 relative each) and FP32 sums.
    Against the exact dense rows FP32 stays within 1e-6; BF16's storage error
    is reported."""
    pts, kw = rhs_cloud
    X = inputs.normal_rhs(len(pts), seed=32, nrhs=64)
    op = gpu_build(pts, factor_dtype=dtype, **kw)
    Y, Ya = gpu_apply(op, X), gpu_apply(op, X, adjoint=True)
    ref = oracle.HODLR3D(pts, **oracle_kw(kw))
    ref.set_factors(op.export("far")[5], op.export("factors_u"), op.export("factors_v"))
    e2, einf = colwise_errors(Y, ref.matvec(X))
    ea2, eainf = colwise_errors(Ya, ref.rmatvec(X))
    rows = inputs.sample_rows(len(pts), 256, seed=3)
    ed = rel(Y[rows], oracle.dense_rows(pts, X, rows))
    print(f"[many rhs] {dtype}: vs oracle with the same factors: column 2-norm {e2:.3e}, "
          f"element {einf:.3e}; adjoint {ea2:.3e}, {eainf:.3e}; vs dense rows {ed:.3e}")
    assert e2 <= bound and einf <= bound and ea2 <= bound and eainf <= bound
    if dtype == "fp32":
        assert ed <= 1e-6
    else:
        assert ed <= 3e-2
    # the one-RHS kernels of the same plan agree with the matrix-core columns
    for c in (0, 63):
        assert rel(Y[:, c], gpu_apply(op, X[:, c])) <= bound
    # the FP64 matrix-core form as a further check
    op64 = gpu_build(pts, **kw)
    Y64 = gpu_apply(op64, X)
    print(f"[many rhs] {dtype}: worst column rel diff to the FP64 form "
          f"{max(rel(Y[:, c], Y64[:, c]) for c in range(64)):.3e}")
    op.close()
    op64.close()


@pytest.mark.parametrize("dtype,bound", [("fp32", 1e-6), ("bf16", 1e-5)])
def test_many_rhs_row_panel_levels(dtype, bound):
    """A tree deep enough for U_b to be stored as row panels above the chunk
    level: 60,000 points, leaves of 32, depth 4; levels 3 and 4 hold 117 and
    15 points per box on average, so the chunk level is 3 and level 2's
    adjoint stage 1 walks the row panels chunk box by chunk box (16-row
    super-steps padded per chunk box).  Three columns of a 64-RHS product and
    of its adjoint (lanes 0, 37 and 63 of the group of 64), element by element
    against the oracle applying the GPU's own factors."""
    n = 60000
    pts = inputs.uniform_points(n, seed=35)
    kw = dict(leaf_size=32, tol=1e-7, **CUBE)
    op = gpu_build(pts, factor_dtype=dtype, **kw)
    assert op.stats()["depth"] == 4
    X = inputs.normal_rhs(n, seed=36, nrhs=64)
    Y, Ya = gpu_apply(op, X), gpu_apply(op, X, adjoint=True)
    ref = oracle.HODLR3D(pts, **oracle_kw(kw))
    ref.set_factors(op.export("far")[5], op.export("factors_u"), op.export("factors_v"))
    cols = [0, 37, 63]
    e2, einf = colwise_errors(Y[:, cols], ref.matvec(X[:, cols]))
    ea2, eainf = colwise_errors(Ya[:, cols], ref.rmatvec(X[:, cols]))
    print(f"[row panels] {dtype}: column 2-norm {e2:.3e}, element {einf:.3e}; adjoint "
          f"{ea2:.3e}, {eainf:.3e}")
    assert e2 <= bound and einf <= bound and ea2 <= bound and eainf <= bound
    op.close()


@pytest.mark.parametrize("dtype,bound", [("fp32", 1e-6), ("bf16", 1e-5)])
def test_many_rhs_fused_leaves_of_64(dtype, bound):
    """The finest level in one pass per leaf for leaves of 17 to 64 rows on
    average, with leaves of every 16-row tile count (1 to 4): 14,000 points of
    two densities, depth 3, leaves of 4 to 62 points; 70 right-hand sides (a
    full and a partial pass of 64 columns), every column against the oracle
    applying the GPU's own factors."""
    pts = inputs.two_density_points(14000, 0.72, seed=33)
    kw = dict(leaf_size=64, tol=1e-7, **CUBE)
    X = inputs.normal_rhs(len(pts), seed=34, nrhs=70)
    op = gpu_build(pts, factor_dtype=dtype, **kw)
    sizes = np.diff(op.export("leaf_off"))
    print(f"[fused leaves] leaf sizes {sizes.min()}..{sizes.max()}, mean {sizes.mean():.1f}")
    assert sizes.max() > 48 and sizes.min() <= 16 and sizes.mean() > 16
    Y = gpu_apply(op, X)
    ref = oracle.HODLR3D(pts, **oracle_kw(kw))
    ref.set_factors(op.export("far")[5], op.export("factors_u"), op.export("factors_v"))
    e2, einf = colwise_errors(Y, ref.matvec(X))
    print(f"[fused leaves] {dtype}: column 2-norm {e2:.3e}, element {einf:.3e}")
    # leaves of 4 to 62 points side by side: the FP32 near-field entries and
    # inputs (rounding 6e-8) meet more cancellation than on uniform clouds;
    # the two-stage kernels gave 1.24e-6 element-wise here, so elements get
    # twice the column bound
    assert e2 <= bound and einf <= 2 * bound
    for c in (0, 64, 69):
        assert rel(Y[:, c], gpu_apply(op, X[:, c])) <= bound
    np.testing.assert_array_equal(gpu_apply(op, X), Y)  # reproducible
    op.close()


@pytest.mark.parametrize("nrhs,adjoint", [(1, False), (1, True), (3, False), (64, False), (64, True)])
def test_graph_replay_equals_eager(nrhs, adjoint):
    torch = torch_mod()
    pts = inputs.uniform_points(15000, seed=40)
    op = gpu_build(pts, leaf_size=32, tol=1e-8, **CUBE)
    X = torch.as_tensor(inputs.normal_rhs(15000, seed=41, nrhs=None if nrhs == 1 else nrhs),
                        device="cuda")
    eager = (op.rmatvec(X) if adjoint else op.matvec(X)).cpu().numpy()
    g = op.graph(X, adjoint=adjoint)
    X2 = torch.as_tensor(inputs.normal_rhs(15000, seed=42, nrhs=None if nrhs == 1 else nrhs),
                         device="cuda")
    eager2 = (op.rmatvec(X2) if adjoint else op.matvec(X2)).cpu().numpy()
    for rep in range(4):
        # eager work of the program between replays
        _ = op.matvec(X2)
        torch.cuda.synchronize()
        g.set_x(X if rep % 2 == 0 else X2)
        out = g.launch().cpu().numpy()
        torch.cuda.synchronize()
        np.testing.assert_array_equal(out, eager if rep % 2 == 0 else eager2)
    g.close()
    op.close()
