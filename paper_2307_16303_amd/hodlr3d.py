"""Python binding of libhodlr3d (C ABI in include/hodlr3d.h).

Argument marshalling only: every step of the build and of the mat-vec runs in
the HIP kernels of ``libhodlr3d.so``.  PyTorch provides device memory (through
its caching allocator, handed to the library as an h3d_allocator) and the
stream.  If the library is missing this module raises; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhodlr3d.so")

H3D_OK, H3D_EINVAL, H3D_ENOMEM, H3D_EDEVICE, H3D_ENOTBUILT, H3D_EDEPTH, H3D_ENOTIMPL = range(7)
STATUS_NAMES = {0: "H3D_OK", 1: "H3D_EINVAL", 2: "H3D_ENOMEM", 3: "H3D_EDEVICE",
                4: "H3D_ENOTBUILT", 5: "H3D_EDEPTH", 6: "H3D_ENOTIMPL"}
KERNELS = {"laplace": 0, "yukawa": 1, "inv_r4": 2, "cos_r": 3}
DTYPES = {"fp64": 0, "f64": 0, "fp32": 1, "f32": 1, "bf16": 2, "bf16_scaled": 2}
EXPORTS = {"perm": 0, "leaf_off": 1, "far": 2, "near": 3, "factors_u": 4, "factors_v": 5,
           "pivots": 6, "lu": 7}
FLAG_KEEP_PIVOTS = 1
FLAG_NO_AUTOTUNE = 2
FLAG_TRUNCATE = 4
FLAG_LU_FORM = 8
MAX_LEVELS = 11

EXPORTED_SYMBOLS = (
    "h3d_config_init", "h3d_build", "h3d_matvec", "h3d_matvec_adjoint", "h3d_get_stats",
    "h3d_export", "h3d_destroy", "h3d_last_error", "h3d_profile_enable", "h3d_profile_read",
    "h3d_profile_reset", "h3d_version", "h3d_autotune", "h3d_graph_create",
    "h3d_graph_launch", "h3d_graph_destroy", "h3d_build_batch", "h3d_matvec_batch",
    "h3d_batch_plan", "h3d_batch_check", "h3d_matvec_noalloc", "h3d_solve_gmres",
    "h3d_dense_matvec", "h3d_graph_create_batch",
)


class H3DError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class Config(ctypes.Structure):
    _fields_ = [
        ("kernel", ctypes.c_int32),
        ("kernel_param", ctypes.c_double),
        ("leaf_size", ctypes.c_int32),
        ("tol", ctypes.c_double),
        ("factor_dtype", ctypes.c_int32),
        ("max_rank", ctypes.c_int32),
        ("max_depth", ctypes.c_int32),
        ("box_lo", ctypes.c_double * 3),
        ("box_side", ctypes.c_double),
        ("workspace_bytes", ctypes.c_int64),
        ("flags", ctypes.c_int32),
    ]


class Stats(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64),
        ("depth", ctypes.c_int32),
        ("factor_dtype", ctypes.c_int32),
        ("box_lo", ctypes.c_double * 3),
        ("box_side", ctypes.c_double),
        ("n_far", ctypes.c_int64),
        ("n_near", ctypes.c_int64),
        ("far_per_level", ctypes.c_int64 * MAX_LEVELS),
        ("rank_sum", ctypes.c_int64),
        ("rank_max", ctypes.c_int32),
        ("n_rank_capped", ctypes.c_int64),
        ("factor_entries", ctypes.c_int64),
        ("factor_bytes", ctypes.c_int64),
        ("factor_bytes_per_level", ctypes.c_int64 * MAX_LEVELS),
        ("near_pair_evals", ctypes.c_int64),
        ("device_bytes", ctypes.c_int64),
        ("build_ms", ctypes.c_double),
        ("aca_ms", ctypes.c_double),
        ("tune_source", ctypes.c_int32),
    ]

    def to_dict(self) -> dict:
        out = {}
        for name, _ in self._fields_:
            v = getattr(self, name)
            out[name] = list(v) if hasattr(v, "__len__") else v
        return out


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)


class SolveInfo(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("cycles", ctypes.c_int32),
                ("converged", ctypes.c_int32), ("rel_residual", ctypes.c_double),
                ("est_residual", ctypes.c_double)]


class Allocator(ctypes.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("ctx", ctypes.c_void_p)]


class KernelProfile(ctypes.Structure):
    _fields_ = [
        ("name", ctypes.c_char * 48),
        ("launches", ctypes.c_int64),
        ("total_ms", ctypes.c_double),
        ("bytes_per_launch", ctypes.c_double),
        ("flops_per_launch", ctypes.c_double),
    ]


_lib = None


def library_path() -> str:
    return LIB_PATH


def load_library():
    """Loads libhodlr3d.so (built by ``__graft_entry__.build()``); raises if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -c 'import "
                           f"__graft_entry__ as g; g.build()'` (no fallback path exists)")
    lib = ctypes.CDLL(LIB_PATH)
    P, I32, I64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    S = ctypes.c_int
    lib.h3d_config_init.argtypes = [ctypes.POINTER(Config)]
    lib.h3d_config_init.restype = None
    lib.h3d_build.argtypes = [P, I64, ctypes.POINTER(Config), ctypes.POINTER(Allocator), P,
                              ctypes.POINTER(P)]
    lib.h3d_build.restype = S
    for f in ("h3d_matvec", "h3d_matvec_adjoint", "h3d_matvec_noalloc"):
        getattr(lib, f).argtypes = [P, P, P, I64, I64, I64, I32, P]
        getattr(lib, f).restype = S
    lib.h3d_get_stats.argtypes = [P, ctypes.POINTER(Stats)]
    lib.h3d_get_stats.restype = S
    lib.h3d_export.argtypes = [P, I32, P, ctypes.POINTER(ctypes.c_size_t)]
    lib.h3d_export.restype = S
    lib.h3d_destroy.argtypes = [P]
    lib.h3d_destroy.restype = S
    lib.h3d_last_error.argtypes = []
    lib.h3d_last_error.restype = ctypes.c_char_p
    lib.h3d_profile_enable.argtypes = [P, I32]
    lib.h3d_profile_enable.restype = S
    lib.h3d_profile_reset.argtypes = [P]
    lib.h3d_profile_reset.restype = S
    lib.h3d_profile_read.argtypes = [P, ctypes.POINTER(KernelProfile), I32,
                                     ctypes.POINTER(ctypes.c_int32)]
    lib.h3d_profile_read.restype = S
    lib.h3d_graph_create.argtypes = [P, P, P, I64, I64, I64, I32, I32, P, ctypes.POINTER(P)]
    lib.h3d_graph_create.restype = S
    lib.h3d_graph_create_batch.argtypes = [P, ctypes.POINTER(P), ctypes.POINTER(P), I64, I32, P,
                                           ctypes.POINTER(P)]
    lib.h3d_graph_create_batch.restype = S
    lib.h3d_graph_launch.argtypes = [P, P]
    lib.h3d_graph_launch.restype = S
    lib.h3d_graph_destroy.argtypes = [P]
    lib.h3d_graph_destroy.restype = S
    lib.h3d_autotune.argtypes = [P, I64, P]
    lib.h3d_autotune.restype = S
    lib.h3d_build_batch.argtypes = [I32, ctypes.POINTER(P), ctypes.POINTER(I64),
                                    ctypes.POINTER(Config), ctypes.POINTER(Allocator), P,
                                    ctypes.POINTER(P)]
    lib.h3d_build_batch.restype = S
    lib.h3d_matvec_batch.argtypes = [P, ctypes.POINTER(P), ctypes.POINTER(P), I64, I32, P]
    lib.h3d_matvec_batch.restype = S
    lib.h3d_batch_plan.argtypes = [P, I32, ctypes.POINTER(P)]
    lib.h3d_batch_plan.restype = S
    lib.h3d_batch_check.argtypes = [P, P]
    lib.h3d_batch_check.restype = S
    D = ctypes.c_double
    lib.h3d_solve_gmres.argtypes = [P, D, D, P, P, D, I32, I32, P, ctypes.POINTER(SolveInfo)]
    lib.h3d_solve_gmres.restype = S
    lib.h3d_dense_matvec.argtypes = [P, I64, I32, D, P, P, P]
    lib.h3d_dense_matvec.restype = S
    lib.h3d_version.argtypes = []
    lib.h3d_version.restype = I32
    _lib = lib
    return lib


def _check(status: int) -> None:
    if status != H3D_OK:
        raise H3DError(status, load_library().h3d_last_error().decode())


def default_config() -> Config:
    cfg = Config()
    load_library().h3d_config_init(ctypes.byref(cfg))
    return cfg


def _torch():
    import torch
    return torch


class _TorchAllocator:
    """h3d_allocator backed by torch's caching allocator (kept alive with the plan)."""

    def __init__(self, device: int):
        torch = _torch()
        self.device = device

        def _alloc(nbytes, stream, ctx):
            try:
                return torch.cuda.caching_allocator_alloc(int(nbytes), device=self.device,
                                                          stream=int(stream or 0))
            except Exception:
                return None

        def _free(ptr, nbytes, stream, ctx):
            torch.cuda.caching_allocator_delete(ptr)

        self._a = ALLOC_FN(_alloc)
        self._f = FREE_FN(_free)
        self.struct = Allocator(self._a, self._f, None)


def _check_rhs(x, n: int, device: int) -> None:
    """x must be (n,) or (n, nrhs) with nrhs >= 1, on the operator's GPU."""
    if x.dim() not in (1, 2) or x.shape[0] != n or (x.dim() == 2 and x.shape[1] < 1):
        raise ValueError(f"x must have shape ({n},) or ({n}, nrhs); got {tuple(x.shape)}")
    if x.device.index is not None and x.device.index != device:
        raise ValueError(f"x is on cuda:{x.device.index}, the operator on cuda:{device}")


class Operator:
    """The HODLR3D representation of K on one point cloud, resident on the GPU."""

    def __init__(self, handle, n: int, device: int, allocator, config: Config, owner=None):
        self._h = handle
        self.n = int(n)
        self.device = device
        self._alloc = allocator
        self.config = config
        self._owner = owner  # the batch a problem's plan belongs to (not destroyed here)

    # -- lifecycle --------------------------------------------------------
    def close(self) -> None:
        if self._owner is not None:
            self._h = None
            return
        if getattr(self, "_h", None) is not None and self._h.value:
            _check(load_library().h3d_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    # -- products ---------------------------------------------------------
    def _apply(self, x, adjoint: bool, out=None, noalloc: bool = False):
        torch = _torch()
        if not isinstance(x, torch.Tensor) or not x.is_cuda:
            raise TypeError("x must be a CUDA (HIP) tensor")
        if x.dtype not in (torch.float64, torch.float32):
            raise TypeError("x must be float64 or float32")
        _check_rhs(x, self.n, self.device)
        vec = x.dim() == 1
        x2 = x.reshape(self.n, -1)
        nrhs = x2.shape[1]
        xc = x2.t().contiguous()  # nrhs x n row-major == n x nrhs column-major
        y = torch.empty_like(xc) if out is None else out
        io = 0 if x.dtype == torch.float64 else 1
        stream = torch.cuda.current_stream(x.device).cuda_stream
        lib = load_library()
        fn = (lib.h3d_matvec_noalloc if noalloc else
              lib.h3d_matvec_adjoint if adjoint else lib.h3d_matvec)
        _check(fn(self._h, ctypes.c_void_p(xc.data_ptr()), ctypes.c_void_p(y.data_ptr()), nrhs,
                  self.n, self.n, io, ctypes.c_void_p(stream)))
        return y.reshape(-1) if vec else y.t()

    def matvec(self, x):
        """y = K~ x for x of shape (n,) or (n, nrhs) on the GPU."""
        return self._apply(x, adjoint=False)

    def rmatvec(self, x):
        """y = K~^T x with the same stored blocks."""
        return self._apply(x, adjoint=True)

    def matvec_noalloc(self, x):
        """y = K~ x (nrhs < 8) through h3d_matvec_noalloc: the library allocates
        nothing during the product (its scratch is one static array per GPU)."""
        return self._apply(x, adjoint=False, noalloc=True)

    def __matmul__(self, x):
        return self.matvec(x)

    def solve(self, f, diag: float, scale: float, x0=None, rtol: float = 1e-10,
              restart: int = 50, max_iter: int = 1000):
        """GMRES on (diag I + scale K~) x = f (Sec. 5.2).  f: (n,) float64 on the
        operator's GPU.  Returns (x, info) with info a dict of iterations, cycles,
        converged, rel_residual (true, at exit) and est_residual."""
        torch = _torch()
        if not isinstance(f, torch.Tensor) or not f.is_cuda or f.dtype != torch.float64:
            raise TypeError("f must be a float64 CUDA tensor")
        if f.dim() != 1:
            raise ValueError("f must be a vector")
        _check_rhs(f, self.n, self.device)
        fc = f.contiguous()
        x = torch.zeros_like(fc) if x0 is None else x0.to(torch.float64).contiguous().clone()
        info = SolveInfo()
        stream = torch.cuda.current_stream(f.device).cuda_stream
        _check(load_library().h3d_solve_gmres(
            self._h, float(diag), float(scale), ctypes.c_void_p(fc.data_ptr()),
            ctypes.c_void_p(x.data_ptr()), float(rtol), int(restart), int(max_iter),
            ctypes.c_void_p(stream), ctypes.byref(info)))
        return x, {k: getattr(info, k) for k, _ in SolveInfo._fields_}

    # -- introspection ----------------------------------------------------
    def graph(self, x, adjoint: bool = False) -> "Graph":
        """Captures the product with this x (kept alive) into a replayable HIP graph."""
        return Graph(self, x, adjoint)

    def autotune(self, nrhs: int = 1) -> None:
        """Times the stream-kernel shapes for products with nrhs columns and keeps the fastest."""
        torch = _torch()
        stream = torch.cuda.current_stream(self.device).cuda_stream
        _check(load_library().h3d_autotune(self._h, int(nrhs), ctypes.c_void_p(stream)))

    def stats(self) -> dict:
        s = Stats()
        _check(load_library().h3d_get_stats(self._h, ctypes.byref(s)))
        return s.to_dict()

    def export(self, what: str) -> np.ndarray:
        wid = EXPORTS[what]
        lib = load_library()
        nbytes = ctypes.c_size_t(0)
        _check(lib.h3d_export(self._h, wid, None, ctypes.byref(nbytes)))
        dtype = np.float64 if what.startswith("factors") or what == "lu" else np.int64
        buf = np.empty(max(nbytes.value // 8, 1), dtype=dtype)
        _check(lib.h3d_export(self._h, wid, buf.ctypes.data_as(ctypes.c_void_p), ctypes.byref(nbytes)))
        buf = buf[: nbytes.value // 8]
        if what == "far":
            return buf.reshape(6, -1)
        if what == "near":
            return buf.reshape(3, -1)
        if what == "pivots":
            return buf.reshape(2, -1)
        return buf

    def profile(self, enable=True) -> None:
        """Turns kernel timing on (True or 1), on and level by level (2), or off."""
        _check(load_library().h3d_profile_enable(self._h, int(enable)))

    def profile_reset(self) -> None:
        _check(load_library().h3d_profile_reset(self._h))

    def profile_read(self) -> list[dict]:
        lib = load_library()
        cnt = ctypes.c_int32(0)
        _check(lib.h3d_profile_read(self._h, None, 0, ctypes.byref(cnt)))
        arr = (KernelProfile * max(cnt.value, 1))()
        _check(lib.h3d_profile_read(self._h, arr, cnt.value, ctypes.byref(cnt)))
        return [dict(name=arr[i].name.decode(), launches=arr[i].launches,
                     total_ms=arr[i].total_ms, bytes_per_launch=arr[i].bytes_per_launch,
                     flops_per_launch=arr[i].flops_per_launch) for i in range(cnt.value)]


class Graph:
    """y = K~ x (or K~^T x) for a fixed x buffer, replayed from a captured HIP graph.
    Write new values into ``x`` in place and call ``launch()``; the result is ``y``."""

    def __init__(self, op: Operator, x, adjoint: bool = False):
        torch = _torch()
        if not isinstance(x, torch.Tensor) or not x.is_cuda or x.dtype not in (torch.float64,
                                                                                torch.float32):
            raise TypeError("x must be a float64/float32 CUDA tensor")
        _check_rhs(x, op.n, op.device)
        self.op = op
        self.vec = x.dim() == 1
        self.nrhs = 1 if self.vec else x.shape[1]
        # column-major buffers owned by the graph
        self.x = torch.empty((self.nrhs, op.n), dtype=x.dtype, device=x.device)
        self.x.copy_(x.reshape(op.n, -1).t())
        self._y = torch.empty_like(self.x)
        self._h = ctypes.c_void_p()
        io = 0 if x.dtype == torch.float64 else 1
        stream = torch.cuda.current_stream(x.device).cuda_stream
        _check(load_library().h3d_graph_create(
            op.handle, ctypes.c_void_p(self.x.data_ptr()), ctypes.c_void_p(self._y.data_ptr()),
            self.nrhs, op.n, op.n, io, int(bool(adjoint)), ctypes.c_void_p(stream),
            ctypes.byref(self._h)))

    def set_x(self, x) -> None:
        self.x.copy_(x.reshape(self.op.n, -1).t())

    def launch(self):
        torch = _torch()
        stream = torch.cuda.current_stream(self.x.device).cuda_stream
        _check(load_library().h3d_graph_launch(self._h, ctypes.c_void_p(stream)))
        return self._y.reshape(-1) if self.vec else self._y.t()

    def close(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value:
            _check(load_library().h3d_graph_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def dense_matvec(points, x, kernel="laplace", kernel_param: float = 1.0):
    """The exact dense product y_i = sum_{j != i} f(|p_i - p_j|) x_j on the GPU
    (points (n, 3) and x (n,) float64 CUDA tensors, same order)."""
    torch = _torch()
    points = _device_points(points)
    n = points.shape[0]
    if not isinstance(x, torch.Tensor) or not x.is_cuda or x.dtype != torch.float64 \
            or x.shape != (n,):
        raise TypeError(f"x must be a float64 CUDA tensor of shape ({n},)")
    xc = x.contiguous()
    y = torch.empty_like(xc)
    kid = KERNELS[kernel] if isinstance(kernel, str) else int(kernel)
    stream = torch.cuda.current_stream(points.device).cuda_stream
    _check(load_library().h3d_dense_matvec(ctypes.c_void_p(points.data_ptr()), n, kid,
                                           float(kernel_param), ctypes.c_void_p(xc.data_ptr()),
                                           ctypes.c_void_p(y.data_ptr()), ctypes.c_void_p(stream)))
    return y


def _make_config(kernel, kernel_param, leaf_size, tol, factor_dtype, max_rank, max_depth, box_lo,
                 box_side, workspace_bytes, keep_pivots, autotune, truncate=False,
                 lu_form=False) -> Config:
    cfg = default_config()
    cfg.kernel = KERNELS[kernel] if isinstance(kernel, str) else int(kernel)
    cfg.kernel_param = float(kernel_param)
    cfg.leaf_size = int(leaf_size)
    cfg.tol = float(tol)
    cfg.factor_dtype = DTYPES[factor_dtype] if isinstance(factor_dtype, str) else int(factor_dtype)
    cfg.max_rank = int(max_rank)
    cfg.max_depth = int(max_depth)
    if box_lo is not None:
        for a in range(3):
            cfg.box_lo[a] = float(box_lo[a])
    cfg.box_side = float(box_side)
    cfg.workspace_bytes = int(workspace_bytes)
    cfg.flags = ((FLAG_KEEP_PIVOTS if keep_pivots else 0) | (0 if autotune else FLAG_NO_AUTOTUNE)
                 | (FLAG_TRUNCATE if truncate else 0) | (FLAG_LU_FORM if lu_form else 0))
    return cfg


def _device_points(points):
    torch = _torch()
    if not isinstance(points, torch.Tensor):
        points = torch.as_tensor(np.ascontiguousarray(points, dtype=np.float64))
    if not points.is_cuda:
        points = points.to("cuda")
    points = points.to(torch.float64).contiguous()
    if points.dim() != 2 or points.shape[1] != 3:
        raise ValueError("points must have shape (n, 3)")
    return points


def build(points, kernel="laplace", kernel_param: float = 1.0, leaf_size: int = 64,
          tol: float = 1e-8, factor_dtype="fp64", max_rank: int = 0, max_depth: int = 10,
          box_lo=None, box_side: float = 0.0, workspace_bytes: int = 0,
          keep_pivots: bool = False, use_torch_allocator: bool = True,
          autotune: bool = True, truncate: bool = False, lu_form: bool = False) -> Operator:
    """Builds the HODLR3D operator of the n x 3 FP64 point cloud (moved to the GPU).
    truncate=True recompresses every block's ACA factors to its optimal rank at tol.
    lu_form=True keeps the paper's storage form: per block the ACA pivots and the
    LU factors of K(sigma, tau), with the other entries regenerated in every product."""
    torch = _torch()
    lib = load_library()
    points = _device_points(points)
    cfg = _make_config(kernel, kernel_param, leaf_size, tol, factor_dtype, max_rank, max_depth,
                       box_lo, box_side, workspace_bytes, keep_pivots, autotune, truncate,
                       lu_form)
    device = points.device.index if points.device.index is not None else torch.cuda.current_device()
    alloc = _TorchAllocator(device) if use_torch_allocator else None
    handle = ctypes.c_void_p()
    stream = torch.cuda.current_stream(points.device).cuda_stream
    with torch.cuda.device(device):
        _check(lib.h3d_build(ctypes.c_void_p(points.data_ptr()), points.shape[0], ctypes.byref(cfg),
                             ctypes.byref(alloc.struct) if alloc else None,
                             ctypes.c_void_p(stream), ctypes.byref(handle)))
    return Operator(handle, points.shape[0], device, alloc, cfg)


class BatchOperator:
    """Independent HODLR3D operators (one per point cloud) whose products run together,
    one launch per phase over all problems.  ``plans[i]`` is problem i's own operator."""

    def __init__(self, handle, ns, device: int, allocator, config: Config):
        self._h = handle
        self.ns = [int(v) for v in ns]
        self.device = device
        self._alloc = allocator
        self.config = config
        lib = load_library()
        self.plans = []
        for i, n in enumerate(self.ns):
            sub = ctypes.c_void_p()
            _check(lib.h3d_batch_plan(self._h, i, ctypes.byref(sub)))
            self.plans.append(Operator(sub, n, device, None, config, owner=self))

    def close(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value:
            for p in self.plans:
                p.close()
            _check(load_library().h3d_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def matvec(self, xs, outs=None):
        """[K~_i x_i] for a list of tensors x_i of shape (n_i,) or (n_i, nrhs), one launch."""
        torch = _torch()
        if len(xs) != len(self.ns):
            raise ValueError(f"expected {len(self.ns)} inputs, got {len(xs)}")
        cols, ys, shapes = [], [], []
        nrhs, dtype = None, None
        for x, n in zip(xs, self.ns):
            if not isinstance(x, torch.Tensor) or not x.is_cuda:
                raise TypeError("every x must be a CUDA (HIP) tensor")
            _check_rhs(x, n, self.device)
            x2 = x.reshape(n, -1)
            if nrhs is None:
                nrhs, dtype = x2.shape[1], x.dtype
            if x2.shape[1] != nrhs or x.dtype != dtype:
                raise ValueError("all inputs must share nrhs and dtype")
            xc = x2.t().contiguous()
            cols.append(xc)
            ys.append(torch.empty_like(xc))
            shapes.append(x.dim() == 1)
        if dtype not in (torch.float64, torch.float32):
            raise TypeError("inputs must be float64 or float32")
        P = ctypes.c_void_p * len(self.ns)
        xp = P(*[c.data_ptr() for c in cols])
        yp = P(*[y.data_ptr() for y in ys])
        io = 0 if dtype == torch.float64 else 1
        stream = torch.cuda.current_stream(cols[0].device).cuda_stream
        _check(load_library().h3d_matvec_batch(self._h, xp, yp, nrhs, io, ctypes.c_void_p(stream)))
        return [y.reshape(-1) if vec else y.t() for y, vec in zip(ys, shapes)]

    def graph(self, xs) -> "BatchGraph":
        """Captures the batch product with these inputs (copied into buffers the
        graph owns) into a replayable HIP graph."""
        return BatchGraph(self, xs)

    def check(self) -> None:
        """Raises if a dependency wait of the last product gave up (synchronises)."""
        torch = _torch()
        stream = torch.cuda.current_stream(self.device).cuda_stream
        _check(load_library().h3d_batch_check(self._h, ctypes.c_void_p(stream)))

    def stats(self) -> dict:
        s = Stats()
        _check(load_library().h3d_get_stats(self._h, ctypes.byref(s)))
        return s.to_dict()

    profile = Operator.profile
    profile_reset = Operator.profile_reset
    profile_read = Operator.profile_read


class BatchGraph:
    """The product of a batch for fixed input buffers, replayed from a captured HIP
    graph.  Write new values into ``xs[i]`` (column-major copies, see set_x) and
    call ``launch()``; the results are the returned views of the graph's outputs."""

    def __init__(self, bop: "BatchOperator", xs):
        torch = _torch()
        if len(xs) != len(bop.ns):
            raise ValueError(f"expected {len(bop.ns)} inputs, got {len(xs)}")
        self.bop = bop
        self.vec = xs[0].dim() == 1
        self.nrhs = 1 if self.vec else xs[0].shape[1]
        self.xs, self._ys = [], []
        for x, n in zip(xs, bop.ns):
            _check_rhs(x, n, bop.device)
            xc = torch.empty((self.nrhs, n), dtype=x.dtype, device=x.device)
            xc.copy_(x.reshape(n, -1).t())
            self.xs.append(xc)
            self._ys.append(torch.empty_like(xc))
        io = 0 if xs[0].dtype == torch.float64 else 1
        P = ctypes.c_void_p * len(bop.ns)
        xp = P(*[c.data_ptr() for c in self.xs])
        yp = P(*[y.data_ptr() for y in self._ys])
        self._h = ctypes.c_void_p()
        stream = torch.cuda.current_stream(self.xs[0].device).cuda_stream
        _check(load_library().h3d_graph_create_batch(bop._h, xp, yp, self.nrhs, io,
                                                     ctypes.c_void_p(stream),
                                                     ctypes.byref(self._h)))

    def set_x(self, i: int, x) -> None:
        self.xs[i].copy_(x.reshape(self.bop.ns[i], -1).t())

    def launch(self):
        torch = _torch()
        stream = torch.cuda.current_stream(self.xs[0].device).cuda_stream
        _check(load_library().h3d_graph_launch(self._h, ctypes.c_void_p(stream)))
        return [y.reshape(-1) if self.vec else y.t() for y in self._ys]

    def close(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value:
            _check(load_library().h3d_graph_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def build_batch(points_list, kernel="laplace", kernel_param: float = 1.0, leaf_size: int = 64,
                tol: float = 1e-8, factor_dtype="fp64", max_rank: int = 0, max_depth: int = 10,
                box_lo=None, box_side: float = 0.0, workspace_bytes: int = 0,
                use_torch_allocator: bool = True, lu_form: bool = False,
                autotune: bool = True) -> BatchOperator:
    """Builds one operator per point cloud for products that run together, one launch
    per phase over all problems (explicit factors only: the library refuses
    lu_form=True for batches).  With autotune each member times the launch shapes
    the batch carries on its own factors."""
    torch = _torch()
    lib = load_library()
    pts = [_device_points(p) for p in points_list]
    if not pts:
        raise ValueError("points_list is empty")
    cfg = _make_config(kernel, kernel_param, leaf_size, tol, factor_dtype, max_rank, max_depth,
                       box_lo, box_side, workspace_bytes, False, autotune, lu_form=lu_form)
    device = pts[0].device.index if pts[0].device.index is not None else torch.cuda.current_device()
    alloc = _TorchAllocator(device) if use_torch_allocator else None
    P = ctypes.c_void_p * len(pts)
    N = ctypes.c_int64 * len(pts)
    parr = P(*[p.data_ptr() for p in pts])
    narr = N(*[p.shape[0] for p in pts])
    handle = ctypes.c_void_p()
    stream = torch.cuda.current_stream(pts[0].device).cuda_stream
    with torch.cuda.device(device):
        _check(lib.h3d_build_batch(len(pts), parr, narr, ctypes.byref(cfg),
                                   ctypes.byref(alloc.struct) if alloc else None,
                                   ctypes.c_void_p(stream), ctypes.byref(handle)))
    return BatchOperator(handle, [p.shape[0] for p in pts], device, alloc, cfg)


def _autograd_function():
    torch = _torch()

    class HODLR3DMatVec(torch.autograd.Function):
        """y = K~ x; the backward pass applies K~^T through the adjoint kernels."""

        @staticmethod
        def forward(ctx, op: Operator, x):
            ctx.op = op
            return op.matvec(x)

        @staticmethod
        def backward(ctx, grad_y):
            return None, ctx.op.rmatvec(grad_y.contiguous())

    return HODLR3DMatVec


_AUTOGRAD = None


def matvec_autograd(op: Operator, x):
    """Differentiable y = K~ x (gradient with respect to x only)."""
    global _AUTOGRAD
    if _AUTOGRAD is None:
        _AUTOGRAD = _autograd_function()
    return _AUTOGRAD.apply(op, x)
