"""Differentiation form at full size: N = 2,097,152 uniform points, Laplace,
FP32 factors (ACA tol 1e-7, about 219 GB), loss L(x) = ||K~x - b||^2 with
b ~ N(0,1), gradient by autograd through the adjoint kernels.

L is quadratic in x, so its central difference along any direction equals
<grad L, v> up to rounding whatever the step; the gradient's entries are also
compared on sampled rows with 2 (K^T r)_i, r = K~x - b taken from the GPU and
K^T applied exactly (dense rows, CPU oracle): that difference is the
compression error of the adjoint, bounded like the forward's (10 tol).
"""
import time

import numpy as np
import pytest

import oracle
from paper_2307_16303_amd import hodlr3d, inputs

pytestmark = pytest.mark.gpu

N = 2097152
TOL = 1e-7


@pytest.mark.timeout(900)
def test_differentiation_form_full_size():
    import torch
    pts = inputs.uniform_points(N, 0)
    print(f"[diff2m] building n={N} fp32 tol={TOL}", flush=True)
    t0 = time.perf_counter()
    op = hodlr3d.build(torch.as_tensor(pts, device="cuda"), kernel="laplace", leaf_size=64,
                       tol=TOL, factor_dtype="fp32", box_lo=inputs.CUBE_LO,
                       box_side=inputs.CUBE_SIDE)
    torch.cuda.synchronize()
    st = op.stats()
    print(f"[diff2m] depth {st['depth']} far {st['n_far']} factor GB "
          f"{st['factor_bytes'] / 1e9:.1f} build {time.perf_counter() - t0:.1f} s", flush=True)
    try:
        x = torch.as_tensor(inputs.normal_rhs(N, 1), device="cuda")
        b = torch.as_tensor(inputs.normal_rhs(N, 2), device="cuda")
        xg = x.clone().requires_grad_(True)
        loss = ((hodlr3d.matvec_autograd(op, xg) - b) ** 2).sum()
        loss.backward()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        xg2 = x.clone().requires_grad_(True)
        loss2 = ((hodlr3d.matvec_autograd(op, xg2) - b) ** 2).sum()
        loss2.backward()
        torch.cuda.synchronize()
        print(f"[diff2m] forward + backward {1e3 * (time.perf_counter() - t0):.1f} ms", flush=True)
        g = xg.grad
        assert torch.equal(g, xg2.grad)  # reproducible

        v = torch.as_tensor(inputs.normal_rhs(N, 5), device="cuda")
        h = 1e-3 * float(x.norm()) / float(v.norm())

        def L(z):
            r = op.matvec(z) - b
            return float(torch.dot(r, r))

        fd = (L(x + h * v) - L(x - h * v)) / (2 * h)
        gv = float(torch.dot(g, v))
        print(f"[diff2m] central difference {fd:.12e} vs <grad, v> {gv:.12e}", flush=True)
        assert abs(fd - gv) <= 1e-10 * abs(gv)

        # sampled gradient entries against the exact adjoint of the GPU residual
        r = (op.matvec(x) - b).cpu().numpy()
        rows = inputs.sample_rows(N, 24, seed=3)
        gd = 2.0 * oracle.dense_rows(pts, r, rows)  # K symmetric: rows of K^T = rows of K
        e = float(np.linalg.norm(g.cpu().numpy()[rows] - gd) / np.linalg.norm(gd))
        print(f"[diff2m] sampled gradient rel err {e:.3e}", flush=True)
        assert e <= 10 * TOL
    finally:
        op.close()
        del op
        torch.cuda.empty_cache()
