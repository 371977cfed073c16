"""Plain CPU FP64 oracle for the HODLR3D mat-vec (arXiv 2307.16303).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  It shares no code
with the GPU library in ``paper_2307_16303_amd/`` and never imports it.

The arithmetic lives in ``h3d_oracle.c`` (plain C, FP64, ``-ffp-contract=off``,
sums in index order); this module only compiles it with gcc and marshals numpy
arrays through ctypes.  See the header of ``h3d_oracle.c`` for the paper
passage each function follows.  The one exception is ``truncate_factors``
(rank truncation of given factors), written here with numpy's LAPACK QR and
SVD as the steps of its definition.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "h3d_oracle.c")
_LIB = os.path.join(_HERE, "libh3d_oracle.so")

KERNELS = {"laplace": 0, "yukawa": 1, "inv_r4": 2, "cos_r": 3}
REL_NAMES = {0: "self", 1: "F", 2: "E", 3: "V", 4: "W"}
_ERR = {1: "invalid argument", 2: "out of memory", 5: "max depth exceeded"}


class OracleError(RuntimeError):
    pass


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C, OpenMP over independent rows/blocks)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        cmd = ["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
               "-fno-fast-math", "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build(force=True)
    lib = ctypes.CDLL(_LIB)
    P = ctypes.c_void_p
    I64 = ctypes.c_int64
    D = ctypes.c_double
    I = ctypes.c_int
    lib.oracle_dense_rows.argtypes = [P, I64, I, D, P, I64, P, I64, P]
    lib.oracle_dense_matvec.argtypes = [P, I64, I, D, P, I64, P]
    lib.oracle_kernel_eval.argtypes = [I, D, P, I64, P]
    lib.oracle_num_threads.restype = I
    lib.oracle_set_num_threads.argtypes = [I]
    lib.oracle_aca_dense.argtypes = [P, I64, I64, D, I64, P, P, P, P, P, P]
    lib.oracle_aca_dense.restype = I64
    lib.oracle_build.argtypes = [P, I64, I, D, I, D, I, I64, P, D, I, ctypes.POINTER(P)]
    lib.oracle_build.restype = I
    lib.oracle_destroy.argtypes = [P]
    lib.oracle_apply.argtypes = [P, P, I64, P, I, I, I]
    lib.oracle_apply.restype = I
    lib.oracle_apply_lu.argtypes = [P, P, I64, P, I, I, I]
    lib.oracle_apply_lu.restype = I
    lib.oracle_export_lu.argtypes = [P, P]
    lib.oracle_set_factors.argtypes = [P, P, P, P]
    lib.oracle_set_factors.restype = I
    lib.oracle_depth.argtypes = [P]
    lib.oracle_depth.restype = I
    for f in ("oracle_num_far", "oracle_num_near", "oracle_num_capped"):
        getattr(lib, f).argtypes = [P]
        getattr(lib, f).restype = I64
    lib.oracle_factor_len.argtypes = [P, I]
    lib.oracle_factor_len.restype = I64
    lib.oracle_box.argtypes = [P, P]
    lib.oracle_export_tree.argtypes = [P, P, P]
    lib.oracle_export_far.argtypes = [P, P, P, P, P, P, P]
    lib.oracle_export_near.argtypes = [P, P, P, P]
    lib.oracle_export_factors.argtypes = [P, P, P]
    lib.oracle_export_pivots.argtypes = [P, P, P]
    lib.oracle_block_dense.argtypes = [P, I64, P]
    lib.oracle_relation.argtypes = [I64] * 6
    lib.oracle_relation.restype = I
    lib.oracle_morton_encode.argtypes = [ctypes.c_uint64] * 3 + [I]
    lib.oracle_morton_encode.restype = ctypes.c_uint64
    lib.oracle_morton_decode.argtypes = [ctypes.c_uint64, I, P]
    _lib = lib
    return lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _kid(kernel) -> int:
    return KERNELS[kernel] if isinstance(kernel, str) else int(kernel)


def set_num_threads(t: int) -> None:
    _load().oracle_set_num_threads(int(t))


def num_threads() -> int:
    return int(_load().oracle_num_threads())


def kernel_eval(kernel, r, param: float = 1.0) -> np.ndarray:
    """f(r) for the kernel id (f(0) := 0)."""
    r = np.ascontiguousarray(r, dtype=np.float64).ravel()
    out = np.empty_like(r)
    _load().oracle_kernel_eval(_kid(kernel), float(param), _ptr(r), r.size, _ptr(out))
    return out


def _as_cols(x: np.ndarray, n: int) -> tuple[np.ndarray, int, bool]:
    x = np.asarray(x, dtype=np.float64)
    vec = x.ndim == 1
    if vec:
        x = x[:, None]
    assert x.shape[0] == n
    return np.asfortranarray(x), x.shape[1], vec


def dense_matvec(points, x, kernel="laplace", param: float = 1.0) -> np.ndarray:
    """Exact y_i = sum_{j != i} f(|r_i - r_j|) x_j, j in index order (O(N^2))."""
    pts = np.ascontiguousarray(points, dtype=np.float64)
    n = pts.shape[0]
    xc, nrhs, vec = _as_cols(x, n)
    y = np.empty((n, nrhs), dtype=np.float64, order="F")
    _load().oracle_dense_matvec(_ptr(pts), n, _kid(kernel), float(param), _ptr(xc), nrhs, _ptr(y))
    return y[:, 0] if vec else y


def dense_rows(points, x, rows, kernel="laplace", param: float = 1.0) -> np.ndarray:
    """Exact y_i of the dense product for the listed target rows only."""
    pts = np.ascontiguousarray(points, dtype=np.float64)
    n = pts.shape[0]
    xc, nrhs, vec = _as_cols(x, n)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    out = np.empty((rows.size, nrhs), dtype=np.float64, order="F")
    _load().oracle_dense_rows(_ptr(pts), n, _kid(kernel), float(param), _ptr(xc), nrhs,
                              _ptr(rows), rows.size, _ptr(out))
    return out[:, 0] if vec else out


def aca_dense(A, tol: float, max_rank: int = 0, return_norm: bool = False):
    """Partially pivoted ACA of an explicit matrix: returns U, V, row pivots, column pivots
    (and, with ``return_norm``, the running |S_k|_F^2 estimate at the stop)."""
    A = np.asfortranarray(A, dtype=np.float64)
    m, n = A.shape
    kcap = min(m, n) if max_rank <= 0 else min(m, n, max_rank)
    U = np.zeros((m, max(kcap, 1)), order="F")
    V = np.zeros((n, max(kcap, 1)), order="F")
    rp = np.zeros(max(kcap, 1), dtype=np.int64)
    cp = np.zeros(max(kcap, 1), dtype=np.int64)
    capped = ctypes.c_int(0)
    norm2 = ctypes.c_double(0.0)
    k = _load().oracle_aca_dense(_ptr(A), m, n, float(tol), kcap, _ptr(U), _ptr(V), _ptr(rp),
                                 _ptr(cp), ctypes.byref(capped), ctypes.byref(norm2))
    out = (U[:, :k].copy(), V[:, :k].copy(), rp[:k].copy(), cp[:k].copy())
    return out + (norm2.value,) if return_norm else out


def truncate_factors(U, V, tol: float):
    """Recompression of low-rank factors to their optimal rank (the step that
    follows ACA in the recompression the references of Sec. 4.1 describe).

    With U = Q_U R_U and V = Q_V R_V (QR) and R_U R_V^T = W diag(s) Z^T (SVD),
    r is the smallest rank with ||(s_{r+1}, ..., s_k)||_2 <= tol ||s||_2, and
    U' = Q_U W_r diag(s_r)^(1/2), V' = Q_V Z_r diag(s_r)^(1/2).  Blocks of rank
    below 2, zero blocks and blocks whose rank does not drop come back as
    given.  Returns (U', V', r).
    """
    U = np.asarray(U, dtype=np.float64)
    V = np.asarray(V, dtype=np.float64)
    k = U.shape[1]
    if k < 2:
        return U.copy(), V.copy(), k
    qu, ru = np.linalg.qr(U)
    qv, rv = np.linalg.qr(V)
    w, sv, zt = np.linalg.svd(ru @ rv.T)
    s2 = sv * sv
    total = float(np.sum(s2))
    if total == 0.0:
        return U.copy(), V.copy(), k
    tail = np.zeros(k + 1)
    tail[:k] = np.cumsum(s2[::-1])[::-1]  # tail[r] = sum of s_i^2 for i >= r (0-based)
    r = next(j for j in range(1, k + 1) if tail[j] <= tol * tol * total)
    if r >= k:
        return U.copy(), V.copy(), k
    root = np.sqrt(sv[:r])
    return qu @ (w[:, :r] * root), qv @ (zt[:r].T * root), r


def relation(a, b) -> str:
    """Relation of two same-level boxes given by integer coordinates."""
    return REL_NAMES[_load().oracle_relation(*[int(v) for v in a], *[int(v) for v in b])]


def morton_encode(q, bits: int) -> int:
    return int(_load().oracle_morton_encode(int(q[0]), int(q[1]), int(q[2]), int(bits)))


def morton_decode(key: int, bits: int) -> tuple[int, int, int]:
    out = np.zeros(3, dtype=np.int64)
    _load().oracle_morton_decode(int(key), int(bits), _ptr(out))
    return int(out[0]), int(out[1]), int(out[2])


class HODLR3D:
    """The oracle's HODLR3D representation of the kernel matrix on a point cloud."""

    def __init__(self, points, kernel="laplace", param: float = 1.0, leaf_size: int = 64,
                 tol: float = 1e-8, max_depth: int = 10, max_rank: int = 0,
                 box_lo=None, box_side: float = 0.0, compress: bool = True):
        lib = _load()
        self.points = np.ascontiguousarray(points, dtype=np.float64)
        self.n = self.points.shape[0]
        self.kernel = _kid(kernel)
        self.param = float(param)
        lo = np.zeros(3) if box_lo is None else np.ascontiguousarray(box_lo, dtype=np.float64)
        h = ctypes.c_void_p()
        rc = lib.oracle_build(_ptr(self.points), self.n, self.kernel, self.param, int(leaf_size),
                              float(tol), int(max_depth), int(max_rank), _ptr(lo),
                              float(box_side), int(bool(compress)), ctypes.byref(h))
        if rc != 0:
            raise OracleError(f"oracle_build failed: {_ERR.get(rc, rc)}")
        self._h = h
        self._lib = lib

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._lib.oracle_destroy(h)
            self._h = None

    @property
    def depth(self) -> int:
        return int(self._lib.oracle_depth(self._h))

    @property
    def num_far(self) -> int:
        return int(self._lib.oracle_num_far(self._h))

    @property
    def num_near(self) -> int:
        return int(self._lib.oracle_num_near(self._h))

    @property
    def num_capped(self) -> int:
        return int(self._lib.oracle_num_capped(self._h))

    def box(self):
        out = np.zeros(4)
        self._lib.oracle_box(self._h, _ptr(out))
        return out[:3].copy(), float(out[3])

    def tree(self):
        perm = np.empty(self.n, dtype=np.int64)
        leaf_off = np.empty(8 ** self.depth + 1, dtype=np.int64)
        self._lib.oracle_export_tree(self._h, _ptr(perm), _ptr(leaf_off))
        return perm, leaf_off

    def far(self) -> dict:
        nb = self.num_far
        cols = {k: np.empty(nb, dtype=np.int64) for k in ("level", "t", "s", "m", "n", "rank")}
        self._lib.oracle_export_far(self._h, *[_ptr(cols[k]) for k in
                                               ("level", "t", "s", "m", "n", "rank")])
        return cols

    def near(self) -> dict:
        nn = self.num_near
        cols = {k: np.empty(nn, dtype=np.int64) for k in ("t", "s", "rel")}
        self._lib.oracle_export_near(self._h, _ptr(cols["t"]), _ptr(cols["s"]), _ptr(cols["rel"]))
        return cols

    def factors(self):
        """Concatenated U_b (m x k) and V_b (n x k) column-major blocks, block order."""
        U = np.empty(self._lib.oracle_factor_len(self._h, 0))
        V = np.empty(self._lib.oracle_factor_len(self._h, 1))
        self._lib.oracle_export_factors(self._h, _ptr(U), _ptr(V))
        return U, V

    def pivots(self):
        tot = int(self.far()["rank"].sum())
        rp = np.empty(tot, dtype=np.int64)
        cp = np.empty(tot, dtype=np.int64)
        self._lib.oracle_export_pivots(self._h, _ptr(rp), _ptr(cp))
        return rp, cp

    def block_factors(self, b: int):
        """U_b, V_b of one block (views into fresh copies)."""
        f = self.far()
        U, V = self.factors()
        uoff = np.concatenate([[0], np.cumsum(f["m"] * f["rank"])])
        voff = np.concatenate([[0], np.cumsum(f["n"] * f["rank"])])
        m, n, k = int(f["m"][b]), int(f["n"][b]), int(f["rank"][b])
        return (U[uoff[b]:uoff[b] + m * k].reshape(k, m).T,
                V[voff[b]:voff[b] + n * k].reshape(k, n).T)

    def block_dense(self, b: int) -> np.ndarray:
        f = self.far()
        m, n = int(f["m"][b]), int(f["n"][b])
        out = np.empty((m, n), order="F")
        self._lib.oracle_block_dense(self._h, int(b), _ptr(out))
        return out

    def set_factors(self, ranks, U, V) -> None:
        ranks = np.ascontiguousarray(ranks, dtype=np.int64)
        U = np.ascontiguousarray(U, dtype=np.float64)
        V = np.ascontiguousarray(V, dtype=np.float64)
        rc = self._lib.oracle_set_factors(self._h, _ptr(ranks), _ptr(U), _ptr(V))
        if rc != 0:
            raise OracleError("oracle_set_factors failed")

    def _apply(self, x, adjoint: bool, near: bool, far: bool, lu_form: bool = False):
        xc, nrhs, vec = _as_cols(x, self.n)
        y = np.empty((self.n, nrhs), order="F")
        fn = self._lib.oracle_apply_lu if lu_form else self._lib.oracle_apply
        st = fn(self._h, _ptr(xc), nrhs, _ptr(y), int(adjoint), int(near), int(far))
        if st != 0:
            raise OracleError(_ERR.get(st, str(st)))
        return y[:, 0] if vec else y

    def matvec(self, x, near: bool = True, far: bool = True, lu_form: bool = False):
        """y = K~ x; lu_form applies every low-rank block as K(X,tau) R^-1 L^-1
        K(sigma,Y) with regenerated entries (Sec. 4.1; Algorithm 2)."""
        return self._apply(x, False, near, far, lu_form)

    def rmatvec(self, x, near: bool = True, far: bool = True, lu_form: bool = False):
        return self._apply(x, True, near, far, lu_form)

    def lu_factors(self):
        """Packed LU factors of K(sigma, tau) per block (k_b x k_b column-major,
        L on and below the diagonal, the unit-diagonal R above it),
        concatenated in block order."""
        r = self.far()["rank"]
        out = np.empty(max(int((r * r).sum()), 1), dtype=np.float64)
        self._lib.oracle_export_lu(self._h, _ptr(out))
        return out[: int((r * r).sum())]

    def block_lu(self, b: int) -> np.ndarray:
        r = self.far()["rank"]
        off = int((r[:b] * r[:b]).sum())
        k = int(r[b])
        return self.lu_factors()[off: off + k * k].reshape(k, k, order="F")
