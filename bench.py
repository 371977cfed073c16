"""Benchmark: HODLR3D mat-vec throughput on one MI355X.

A step is one full mat-vec Y = K~X (gather, near-field tiles, both factor
streams, scatter) over the resident operator of the workload; the build
(tree, lists, ACA, packing) happens before the timed region and is reported
separately.  Prints one JSON line.

Headline: the precision + batching form on 1,048,576 i.i.d. uniform points
(Laplace, leaf <= 64, ACA tol 1e-7 in FP64): FP32 factors, 64 right-hand
sides on the matrix cores.  Beside it, on the same points, the plain FP64
form with one right-hand side (the baseline the gain is taken over), and the
relative error of both on sampled rows of the exact dense product (the gate
is 1e-6).

The roofline object describes the dominant kernel of the headline step: its
algorithmic flops per launch (2 per factor entry per right-hand side) over
its average launch time, taken with HIP events recorded by the library on the
launch stream during the timed steps, against the FP32 matrix-core peak; its
algorithmic bytes per launch over the same time are reported beside it.  The
baseline carries its own HBM roofline.

The cpu_baseline object times the CPU oracle's exact dense direct sum on a
bounded sample of target rows of the headline workload (rows x 64 RHS per
second) with every thread of the process's CPU share, and once with one
thread; beside it, the oracle's own HODLR3D product (build and mat-vec) on
the 16^3 grid and on 65,536 uniform points (the oracle cannot hold the
1,048,576-point operator in reasonable time).

The variants object measures the other storage forms (FP32 and BF16 factors,
one and 64 right-hand sides; the paper's own pivot + LU form, whose product
regenerates the kernel entries and is bound by the vector ALUs) on the
headline points, the plain FP64 and LU forms on 262,144 points, the
multi-problem form (32 clouds, N_i in [8192, 131072], FP32 factors, tol 1e-7)
as one batch (one launch per phase over all problems), and the integral-equation solve of Sec. 5.2 on a
64^3 grid (GMRES to a relative residual of 1e-10).

roofline.traffic is the dominant kernel's HBM traffic per launch from the
hardware counters FETCH_SIZE and WRITE_SIZE (rocprofv3 --pmc, one counter per
run), each divided by what the same counter reads for a plain 2 GiB device
copy (--calibration-copy).  Readings hold for the sources they were taken on:
if any library source has changed since, traffic is null.
"""
from __future__ import annotations

import argparse
import glob
import hashlib
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

METRIC = "HODLR3D matvec points·RHS/s vs plain FP64 GPU at rel err ≤1e-6; HBM GB/s"
UNIT = "points·RHS/s"
HBM_PEAK_GBS = 8000.0
# dense matrix-core peaks of MI355X (TFLOP/s); BF16 factors are widened to FP32 tiles
MFMA_PEAK_TFS = {"fp64": 78.6, "fp32": 157.3, "bf16": 157.3}
# FP64 vector ALU peak (TFLOP/s): the pivot + LU form's kernel evaluations
VALU_FP64_PEAK_TFS = 78.6
DTYPE_NAMES = {"fp64": "f64", "fp32": "f32", "bf16": "bf16"}
GATE = 1e-6

# Counter readings, KiB per dispatch (a kernel launched once per level: the
# mean over its dispatches of one product), with the copy-kernel scale of each
# counter.  The runs that produced them are listed in profiles/;
# sources_sha256 identifies the code of the library sources they were taken
# on (sources_digest: comments and layout left out, so that rewording a comment
# keeps them; the compiled code of every source is the same either way).
TRAFFIC = {
    "fetch_scale": 0.500016,
    "write_scale": 1.000000,
    "readings": [
        {"workload": "uniform262k", "factor_dtype": "fp64", "nrhs": 1,
         "sources_sha256": "a0162748c17231bcc1d54d4578e5c26e8a87cea858efad8f47f54f7b3d5a9393",
         "scope": "stream",
         "kernels": {"k_stage2": {"fetch_kib": 10105573.1875, "write_kib": 8198.0938},
                     "k_s1_wide": {"fetch_kib": 2560271.7656, "write_kib": 35383.5391},
                     "k_leaf": {"fetch_kib": 1903345.375, "write_kib": 2846.7188}}},
        # the headline: 64 right-hand sides on the matrix cores (per launch:
        # a level of stage 1 or stage 2; the finest level and the near field
        # are one launch group each)
        {"workload": "uniform1m", "factor_dtype": "fp32", "nrhs": 64,
         "sources_sha256": "d8b3039b713dff9d9fde327c3721087beba4c3bbc1168c8a8e68087c9b5a4d85",
         "scope": "all",
         "kernels": {"k_s1_mfma": {"fetch_kib": 5739502.875, "write_kib": 1019414.4062},
                     "k_s2_mfma": {"fetch_kib": 5461342.0312, "write_kib": 524288.0},
                     "k_leaf_fused": {"fetch_kib": 16546339.9375, "write_kib": 524288.0},
                     "k_near_mfma": {"fetch_kib": 1068406.5625, "write_kib": 524288.125}}},
    ],
}

# library sources of kernels launched on their own, on which the one-RHS
# stream readings do not depend (many right-hand sides, many problems,
# optional rank truncation, the fused finest level)
OTHER_PATHS = ("batched.hip", "batch.hip", "truncate.hip", "leaf.hip")


def code_only(text: str) -> str:
    """C/C++ text without its comments, with each run of blanks outside string
    and character literals made one space, lines trimmed and empty lines left
    out: the code alone, so that a reading stays keyed to the code it was taken
    on, not to the wording or layout of its comments."""
    out, i, n = [], 0, len(text)

    def blank():
        if out and out[-1] not in " \n":
            out.append(" ")

    while i < n:
        c = text[i]
        if text.startswith("//", i):
            j = text.find("\n", i)
            i = n if j < 0 else j
        elif text.startswith("/*", i):
            j = text.find("*/", i + 2)
            blank()
            i = n if j < 0 else j + 2
        elif c in "\"'":
            j = i + 1
            while j < n and text[j] != c:
                j += 2 if text[j] == "\\" else 1
            out.append(text[i:j + 1])
            i = j + 1
        elif c in " \t\r\f\v":
            blank()
            i += 1
        elif c == "\n":
            if out and out[-1] == " ":
                out.pop()
            if out and out[-1] != "\n":
                out.append("\n")
            i += 1
        else:
            out.append(c)
            i += 1
    return "".join(out).strip()


def sources_digest(scope: str = "all") -> str:
    """sha256, in name order, over the code (code_only) of the library sources
    and header.  scope 'stream': without the files of kernels launched on their
    own."""
    h = hashlib.sha256()
    files = sorted(f for f in glob.glob(os.path.join(ROOT, "paper_2307_16303_amd", "csrc", "*"))
                   if scope != "stream" or os.path.basename(f) not in OTHER_PATHS)
    files.append(os.path.join(ROOT, "include", "hodlr3d.h"))
    for f in files:
        h.update(os.path.basename(f).encode())
        with open(f, encoding="utf-8") as fh:
            h.update(code_only(fh.read()).encode())
    return h.hexdigest()


def traffic_bytes(kernel: str, workload: str, factor_dtype: str, nrhs: int,
                  adjoint: bool = False):
    """HBM bytes per launch from the stored counter readings, or None."""
    for r in TRAFFIC["readings"]:
        k = r["kernels"].get(kernel)
        if (k is None or r["workload"] != workload or r["factor_dtype"] != factor_dtype
                or r["nrhs"] != nrhs or r.get("adjoint", False) != adjoint
                or r["sources_sha256"] != sources_digest(r["scope"])):
            continue
        return (k["fetch_kib"] * 1024.0 / TRAFFIC["fetch_scale"]
                + k["write_kib"] * 1024.0 / TRAFFIC["write_scale"])
    return None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="uniform1m")
    ap.add_argument("--factor-dtype", default="fp32", choices=["fp64", "fp32", "bf16"])
    ap.add_argument("--nrhs", type=int, default=64)
    ap.add_argument("--adjoint", action="store_true", help="time the adjoint product instead")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="target CPU time of the oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the baseline and the other forms measured beside the headline")
    ap.add_argument("--profile-levels", action="store_true",
                    help="profile the factor streams level by level (one launch per level)")
    ap.add_argument("--batch-only", action="store_true",
                    help="run only the multi-problem batch variant and print its figures "
                         "(a profiling aid; not the bench line)")
    ap.add_argument("--calibration-copy", action="store_true",
                    help="after the timed steps, fill and copy a 2 GiB buffer: the plain "
                         "kernels that hardware byte counters are scaled by; then time "
                         "torch's sum over it, a plain read stream")
    return ap.parse_args()


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def build_op(pts, w, dt, truncate=False, lu_form=False, tol=None):
    import torch
    from paper_2307_16303_amd import hodlr3d, inputs
    t0 = time.perf_counter()
    op = hodlr3d.build(torch.as_tensor(pts, device="cuda:0"), kernel=w["kernel"],
                       leaf_size=w["leaf_size"], tol=w["tol"] if tol is None else tol,
                       factor_dtype=dt, box_lo=inputs.CUBE_LO, box_side=inputs.CUBE_SIDE,
                       truncate=truncate, lu_form=lu_form)
    torch.cuda.synchronize()
    return op, time.perf_counter() - t0


def time_products(op, x, steps, warmup, adjoint=False, profile=False, levels=False):
    """Mean seconds per product over `steps` after `warmup`; the last output;
    the library's per-kernel profile of the timed steps when asked."""
    import torch
    f = op.rmatvec if adjoint else op.matvec
    for _ in range(warmup):
        y = f(x)
    torch.cuda.synchronize()
    if profile:
        op.profile(2 if levels else True)
        op.profile_reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        y = f(x)
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / steps
    prof = None
    if profile:
        prof = op.profile_read()
        op.profile(False)
    return sec, y, prof


def roofline_of(prof, workload, dt, nrhs, adjoint=False):
    """Roofline object of the dominant kernel of a profiled product: matrix-core
    bound (FLOP/s) for the many-RHS kernels, HBM bound (GB/s) otherwise."""
    dom = max(prof, key=lambda p: p["total_ms"])
    avg_ms = dom["total_ms"] / max(dom["launches"], 1)
    gbs = dom["bytes_per_launch"] / (avg_ms * 1e-3) / 1e9
    traffic = traffic_bytes(dom["name"], workload, dt, nrhs, adjoint)
    common = {"traffic": None if traffic is None else round(traffic, 0), "kernel": dom["name"],
              "avg_launch_ms": round(avg_ms, 4), "bytes_per_launch": dom["bytes_per_launch"]}
    if dom["name"].startswith("k_lu"):
        tfs = dom["flops_per_launch"] / (avg_ms * 1e-3) / 1e12
        return {"bound": "alu", "achieved": round(tfs, 2), "peak": VALU_FP64_PEAK_TFS,
                "unit": "TFLOP/s", "frac": round(tfs / VALU_FP64_PEAK_TFS, 4), **common,
                "flops_per_launch": dom["flops_per_launch"], "hbm_gbs": round(gbs, 1)}
    if "mfma" in dom["name"] or dom["name"].startswith("k_leaf_fused"):
        tfs = dom["flops_per_launch"] / (avg_ms * 1e-3) / 1e12
        peak = MFMA_PEAK_TFS[dt]
        return {"bound": "mfma", "achieved": round(tfs, 2), "peak": peak, "unit": "TFLOP/s",
                "frac": round(tfs / peak, 4), **common,
                "flops_per_launch": dom["flops_per_launch"], "hbm_gbs": round(gbs, 1),
                "hbm_frac": round(gbs / HBM_PEAK_GBS, 4)}
    return {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(gbs / HBM_PEAK_GBS, 4), **common}


def kernel_table(prof):
    return {p["name"]: {"ms": round(p["total_ms"] / max(p["launches"], 1), 4),
                        "launches": p["launches"]} for p in prof}


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def cpu_threads() -> int:
    """Threads of this process's CPU share: its affinity set, capped by
    OMP_NUM_THREADS when that is set."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    env = os.environ.get("OMP_NUM_THREADS", "")
    if env.isdigit() and int(env) > 0:
        n = min(n, int(env))
    return max(1, n)


def integral_equation(k: int, tol: float) -> dict:
    """sigma + int_B sigma(y) / |x - y| dy = f on a k^3 collocation grid of
    [-1,1]^3 (midpoint rule off the diagonal, the exact self-cell integral on
    it): a known sigma, f from the exact dense product on the GPU, GMRES(50)
    with the HODLR3D product to a relative residual of 1e-10."""
    import torch
    from paper_2307_16303_amd import hodlr3d, inputs
    n = k ** 3
    h = 2.0 / k
    s3 = np.sqrt(3.0)
    diag = 1.0 + h * h * (6.0 * np.log((1.0 + s3) / np.sqrt(2.0)) - np.pi / 2.0)
    scale = 4.0 * np.pi * h ** 3  # the library's Laplace kernel is 1/(4 pi r)
    pts = torch.as_tensor(inputs.grid_points(k), device="cuda:0")
    sigma = torch.as_tensor(inputs.normal_rhs(n, seed=98), device="cuda:0")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    f = diag * sigma + scale * hodlr3d.dense_matvec(pts, sigma)
    torch.cuda.synchronize()
    dense_s = time.perf_counter() - t0
    t0 = time.perf_counter()
    op = hodlr3d.build(pts, leaf_size=64, tol=tol, box_lo=inputs.CUBE_LO,
                       box_side=inputs.CUBE_SIDE)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    t0 = time.perf_counter()
    x, info = op.solve(f, diag, scale, rtol=1e-10, restart=50, max_iter=500)
    torch.cuda.synchronize()
    solve_s = time.perf_counter() - t0
    err = float(torch.linalg.norm(x - sigma) / torch.linalg.norm(sigma))
    op.close()
    log(f"ie_grid{k}: {info['iterations']} iterations, solve {solve_s:.3f} s, forward error "
        f"{err:.2e}")
    return {"n": n, "aca_tol": tol, "factor_dtype": "fp64", "rtol": 1e-10,
            "build_s": round(build_s, 2), "solve_s": round(solve_s, 4),
            "exact_rhs_s": round(dense_s, 4), **info, "forward_error": err}


def rel_err(a, b) -> float:
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def batch_variant(args, dev):
    """The bench's multi-problem workload as one batch: its time per product, and
    that of the members' own products in sequence; returns (figures, two
    problems' outputs for the error check)."""
    import torch

    from paper_2307_16303_amd import hodlr3d, inputs
    bw = inputs.BATCH_WORKLOAD
    work = inputs.batch_workload(bw["count"])
    t0 = time.perf_counter()
    bop = hodlr3d.build_batch([torch.as_tensor(p, device=dev) for p, _ in work],
                              kernel=bw["kernel"], leaf_size=bw["leaf_size"], tol=bw["tol"],
                              factor_dtype=bw["factor_dtype"], box_lo=inputs.CUBE_LO,
                              box_side=inputs.CUBE_SIDE)
    torch.cuda.synchronize()
    bbuild = time.perf_counter() - t0
    xs = [torch.as_tensor(x, device=dev) for _, x in work]
    nb = max(3, args.steps // 2)
    for _ in range(max(1, args.warmup // 2)):
        ys = bop.matvec(xs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(nb):
        ys = bop.matvec(xs)
    torch.cuda.synchronize()
    tb = (time.perf_counter() - t0) / nb
    bop.check()
    for p, x in zip(bop.plans, xs):
        p.matvec(x)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(nb):
        for p, x in zip(bop.plans, xs):
            p.matvec(x)
    torch.cuda.synchronize()
    ts = (time.perf_counter() - t0) / nb
    ntot = sum(len(p) for p, _ in work)
    bst = bop.stats()
    fig = {
        "factor_dtype": bw["factor_dtype"], "nrhs": 1, "problems": len(work), "n_total": ntot,
        "ms_per_step": round(1e3 * tb, 4), "value": round(ntot / tb, 1),
        "own_products_in_sequence_ms": round(1e3 * ts, 4),
        "gain_vs_own_products": round(ts / tb, 2),
        "factor_bytes": bst["factor_bytes"],
        "hbm_gbs": round(bst["factor_bytes"] / tb / 1e9, 1), "build_s": round(bbuild, 2)}
    log(f"batch32: {1e3 * tb:.3f} ms ({1e3 * ts:.3f} ms as own products)")
    outs = [(work[i][0], work[i][1], ys[i].detach().cpu().numpy()) for i in (0, 17)]
    bop.close()
    del bop, xs, ys
    torch.cuda.empty_cache()
    return fig, outs


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(the mat-vec would shard by target box with one all-gather of x).", file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2307_16303_amd import hodlr3d, inputs

    if args.batch_only:
        dev = torch.device("cuda:0")
        torch.cuda.set_device(dev)
        fig, _ = batch_variant(args, dev)
        print(json.dumps({"batch32_fp32": fig}), flush=True)
        return

    wname = args.workload
    w = inputs.WORKLOADS[wname]
    n = w["n"]
    nrhs = args.nrhs
    dt = args.factor_dtype
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    pts = inputs.workload_points(wname)
    x1_np = inputs.workload_rhs(wname, None)
    xh_np = x1_np if nrhs == 1 else inputs.workload_rhs(wname, nrhs)
    # target rows whose exact products the oracle computes afterwards
    rows_err = inputs.sample_rows(n, 2048, seed=3)
    sampled = {}  # form -> (rhs id, GPU rows)

    # ---- headline form ---------------------------------------------------
    op, build_s = build_op(pts, w, dt)
    st = op.stats()
    log(f"built {wname} ({dt}): depth {st['depth']}, {st['n_far']} far blocks, "
        f"{st['factor_bytes'] / 1e9:.2f} GB factors, build {build_s:.1f} s")
    xh = torch.as_tensor(xh_np, device=dev)
    sec, y, prof = time_products(op, xh, args.steps, args.warmup, adjoint=args.adjoint,
                                 profile=True, levels=args.profile_levels)
    ms = 1e3 * sec
    value = n * nrhs / sec
    log(f"headline {dt} {nrhs} RHS: {ms:.3f} ms, {value:.3e} {UNIT}")
    roofline = roofline_of(prof, wname, dt, nrhs, args.adjoint)
    kernels = kernel_table(prof)
    head_form = f"{dt}_{nrhs}rhs"
    sampled[head_form] = ("h", y.detach().reshape(n, -1)[torch.as_tensor(rows_err, device=dev)]
                          .cpu().numpy())
    copy_gbs = read_gbs = None
    if args.calibration_copy:
        # 2 GiB written by the fill, then 2 GiB read and 2 GiB written by the copy
        a = torch.ones(2 ** 28, dtype=torch.float64, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(5):
            b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        copy_gbs = 5 * 2 * 2 ** 31 / (e0.elapsed_time(e1) * 1e-3) / 1e9
        log(f"device copy: {copy_gbs:.1f} GB/s (read + write)")
        s = a.sum()
        torch.cuda.synchronize()
        e0.record()
        for _ in range(5):
            s = a.sum()
        e1.record()
        torch.cuda.synchronize()
        read_gbs = 5 * 2 ** 31 / (e0.elapsed_time(e1) * 1e-3) / 1e9
        log(f"device read (sum): {read_gbs:.1f} GB/s")
        del a, b, s
    variants = {}
    rows_t = torch.as_tensor(rows_err, device=dev)

    def run_variant(name, opv, dtv, nr, steps, warmup, extra=None, profile=False, wl=wname,
                    nn=n, xnp=None, adjoint=False):
        xv = torch.as_tensor(xnp, device=dev)
        sec_v, yv, prof_v = time_products(opv, xv, steps, warmup, adjoint=adjoint, profile=profile)
        rec = {"workload": wl, "factor_dtype": dtv, "nrhs": nr, "ms_per_step": round(1e3 * sec_v, 4),
               "value": round(nn * nr / sec_v, 1), "factor_bytes": opv.stats()["factor_bytes"]}
        if adjoint:
            rec["product"] = "adjoint"
        if extra:
            rec.update(extra)
        if prof_v:
            rec["roofline"] = roofline_of(prof_v, wl, dtv, nr, adjoint)
            rec["kernel_ms"] = kernel_table(prof_v)
        variants[name] = rec
        log(f"{name}: {1e3 * sec_v:.3f} ms, {nn * nr / sec_v:.3e} {UNIT}")
        return yv

    if not args.no_variants and nrhs > 1:
        yv = run_variant(f"{dt}_1rhs", op, dt, 1, max(5, args.steps), max(2, args.warmup),
                         xnp=x1_np)
        sampled[f"{dt}_1rhs"] = ("1", yv.reshape(n, -1)[rows_t].cpu().numpy())
        if not args.adjoint:
            # the adjoint product of the headline form on the same plan
            run_variant(f"{dt}_{nrhs}rhs_adjoint", op, dt, nrhs, max(3, args.steps // 4),
                        max(1, args.warmup // 2), profile=True, xnp=xh_np, adjoint=True)
    op.close()
    del op, y, xh
    torch.cuda.empty_cache()

    baseline = None
    if not args.no_variants:
        # ---- the plain FP64 form, one right-hand side (the baseline) -----
        op, bs = build_op(pts, w, "fp64")
        log(f"built {wname} (fp64): {op.stats()['factor_bytes'] / 1e9:.2f} GB factors, "
            f"build {bs:.1f} s")
        yv = run_variant("fp64_1rhs", op, "fp64", 1, max(5, args.steps), max(2, args.warmup),
                         extra={"build_s": round(bs, 2)}, profile=True, xnp=x1_np)
        sampled["fp64_1rhs"] = ("1", yv.reshape(n, -1)[rows_t].cpu().numpy())
        baseline = variants.pop("fp64_1rhs")
        op.close()
        del op, yv
        torch.cuda.empty_cache()
        # ---- BF16 factors with per-factor scale --------------------------
        op, bs = build_op(pts, w, "bf16")
        yv = run_variant("bf16_1rhs", op, "bf16", 1, max(5, args.steps), max(2, args.warmup),
                         extra={"build_s": round(bs, 2)}, xnp=x1_np)
        sampled["bf16_1rhs"] = ("1", yv.reshape(n, -1)[rows_t].cpu().numpy())
        if nrhs > 1:
            yv = run_variant(f"bf16_{nrhs}rhs", op, "bf16", nrhs, max(3, args.steps // 4),
                             max(1, args.warmup // 2), xnp=xh_np)
            sampled[f"bf16_{nrhs}rhs"] = ("h", yv.reshape(n, -1)[rows_t].cpu().numpy())
        op.close()
        del op, yv
        torch.cuda.empty_cache()
        # ---- the paper's storage form: pivots + LU of K(sigma, tau) -------
        op, bs = build_op(pts, w, "fp64", lu_form=True)
        st_lu = op.stats()
        yv = run_variant("lu_fp64_1rhs", op, "fp64", 1, max(5, args.steps // 2),
                         max(2, args.warmup // 2),
                         extra={"build_s": round(bs, 2), "form": "pivots + LU (Sec. 4.1)",
                                "stored_bytes": st_lu["factor_bytes"],
                                "explicit_fp64_bytes": 8 * st_lu["factor_entries"]},
                         profile=True, xnp=x1_np)
        sampled["lu_fp64_1rhs"] = ("1", yv.reshape(n, -1)[rows_t].cpu().numpy())
        op.close()
        del op, yv
        torch.cuda.empty_cache()
        # ---- 262,144 points, plain FP64, one RHS (and FP32 64 RHS) -------
        w2 = inputs.WORKLOADS["uniform262k"]
        pts2 = inputs.workload_points("uniform262k")
        x2 = inputs.workload_rhs("uniform262k", None)
        op, bs = build_op(pts2, w2, "fp64")
        run_variant("uniform262k_fp64_1rhs", op, "fp64", 1, max(5, args.steps),
                    max(2, args.warmup), extra={"build_s": round(bs, 2)}, profile=True,
                    wl="uniform262k", nn=w2["n"], xnp=x2)
        x2h = inputs.workload_rhs("uniform262k", 64)
        run_variant("uniform262k_fp64_64rhs", op, "fp64", 64, max(3, args.steps // 4),
                    max(1, args.warmup // 2), profile=True, wl="uniform262k", nn=w2["n"],
                    xnp=x2h)
        op.close()
        del op
        torch.cuda.empty_cache()
        op, bs = build_op(pts2, w2, "fp32")
        run_variant("uniform262k_fp32_64rhs", op, "fp32", 64, max(3, args.steps // 4),
                    max(1, args.warmup // 2), extra={"build_s": round(bs, 2)}, profile=True,
                    wl="uniform262k", nn=w2["n"], xnp=x2h)
        op.close()
        del op
        torch.cuda.empty_cache()
        op, bs = build_op(pts2, w2, "bf16")
        run_variant("uniform262k_bf16_64rhs", op, "bf16", 64, max(3, args.steps // 4),
                    max(1, args.warmup // 2), extra={"build_s": round(bs, 2)}, profile=True,
                    wl="uniform262k", nn=w2["n"], xnp=x2h)
        op.close()
        del op
        torch.cuda.empty_cache()
        op, bs = build_op(pts2, w2, "fp64", lu_form=True)
        st_lu = op.stats()
        run_variant("uniform262k_lu_fp64_1rhs", op, "fp64", 1, max(5, args.steps),
                    max(2, args.warmup), profile=True, wl="uniform262k", nn=w2["n"], xnp=x2,
                    extra={"build_s": round(bs, 2), "form": "pivots + LU (Sec. 4.1)",
                           "stored_bytes": st_lu["factor_bytes"],
                           "explicit_fp64_bytes": 8 * st_lu["factor_entries"]})
        op.close()
        del op, pts2, x2
        torch.cuda.empty_cache()
        # ---- the integral equation of Sec. 5.2 on a 64^3 grid -------------
        variants["ie_grid64"] = integral_equation(64, 1e-7)
        torch.cuda.empty_cache()

    # ---- many uneven problems multiplied together -------------------------
    batch_ys = None
    if not args.no_variants:
        variants["batch32_fp32"], batch_ys = batch_variant(args, dev)

    # ---- the CPU oracle: exact rows (errors and the baseline) -------------
    cpu = None
    err_head = None
    if not args.no_cpu_baseline:
        import oracle
        oracle.build(force=False)
        threads = cpu_threads()
        oracle.set_num_threads(threads)
        # exact rows of the one-RHS forms
        ref1 = oracle.dense_rows(pts, x1_np.reshape(n, 1), rows_err, kernel=w["kernel"])
        # the headline sample: as many exact rows (all right-hand sides) as the
        # threads finish in about cpu_seconds, measured on a probe first
        xh2 = xh_np.reshape(n, -1)
        probe = inputs.sample_rows(n, min(n, 4 * threads), seed=5)
        t0 = time.perf_counter()
        oracle.dense_rows(pts, xh2, probe, kernel=w["kernel"])
        per_row = (time.perf_counter() - t0) / probe.size
        count = int(min(rows_err.size, max(16, args.cpu_seconds / max(per_row, 1e-9))))
        rows_c = rows_err[:count]
        t0 = time.perf_counter()
        refh = oracle.dense_rows(pts, xh2, rows_c, kernel=w["kernel"])
        cpu_s = time.perf_counter() - t0
        # one thread, on a smaller sample
        oracle.set_num_threads(1)
        c1 = max(2, count // (2 * threads))
        t0 = time.perf_counter()
        oracle.dense_rows(pts, xh2, rows_c[:c1], kernel=w["kernel"])
        cpu1_s = time.perf_counter() - t0
        oracle.set_num_threads(threads)
        for form, (rid, ygpu) in sampled.items():
            if rid == "1":
                e = rel_err(ygpu, ref1)
            else:
                e = rel_err(ygpu[:count], refh)
            if form == head_form:
                err_head = e
            elif form == "fp64_1rhs" and baseline is not None:
                baseline["rel_err_on_sample"] = e
            elif form in variants:
                variants[form]["rel_err_on_sample"] = e
        if batch_ys:
            errs = []
            for pts_i, x_i, y_i in batch_ys:
                r_i = inputs.sample_rows(len(pts_i), 64, seed=3)
                ref = oracle.dense_rows(pts_i, x_i, r_i, kernel=inputs.BATCH_WORKLOAD["kernel"])
                errs.append(rel_err(y_i[r_i], ref))
            variants["batch32_fp32"]["rel_err_on_sample"] = max(errs)
        # the oracle's own HODLR3D product where it finishes: the 16^3 grid and
        # 65,536 uniform points (same kernel, leaf and tolerance rules)
        hod = {}
        for hname, hp, hx, htol in (
                ("grid4096_tol1e-10", inputs.grid_points(16), inputs.uniform_rhs(4096, 0), 1e-10),
                ("uniform65536_tol1e-7", inputs.uniform_points(65536, 0),
                 inputs.normal_rhs(65536, 1), 1e-7)):
            t0 = time.perf_counter()
            H = oracle.HODLR3D(hp, kernel=w["kernel"], leaf_size=w["leaf_size"], tol=htol,
                               box_lo=inputs.CUBE_LO, box_side=inputs.CUBE_SIDE)
            hb = time.perf_counter() - t0
            t0 = time.perf_counter()
            H.matvec(hx)
            hm = time.perf_counter() - t0
            oracle.set_num_threads(1)
            t0 = time.perf_counter()
            H.matvec(hx)
            hm1 = time.perf_counter() - t0
            oracle.set_num_threads(threads)
            hod[hname] = {"n": len(hp), "build_s": round(hb, 2), "matvec_s": round(hm, 4),
                          "matvec_s_1thread": round(hm1, 4),
                          "value": round(len(hp) / hm, 1)}
            del H
        cpu = {"value": round(count * nrhs / cpu_s, 1), "unit": UNIT, "cores": threads,
               "kind": "oracle",
               "sample": f"exact FP64 direct sum, all {nrhs} right-hand sides, for {count} "
                         f"sampled target rows of the same N={n} workload ({cpu_s:.1f} s)",
               "value_1thread": round(c1 * nrhs / cpu1_s, 1),
               "sample_1thread": f"{c1} of the same rows on one thread ({cpu1_s:.1f} s)",
               "cpu_model": cpu_model(), "host_cpus": os.cpu_count(),
               "oracle_hodlr3d_matvec": hod}

    if baseline is not None:
        baseline["gain"] = round(value / baseline["value"], 2)
    out = {
        "metric": METRIC, "value": round(value, 1), "unit": UNIT, "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": DTYPE_NAMES[dt], "data": "synthetic",
        "config": {
            "workload": f"{wname}: N={n} i.i.d. uniform points in [-1,1]^3, "
                        f"{w['kernel']} kernel, leaf <= {w['leaf_size']}, ACA tol {w['tol']} "
                        f"(FP64), {dt} factors, {nrhs} RHS"
                        + (" (adjoint)" if args.adjoint else ""),
            "n": n, "nrhs": nrhs, "depth": st["depth"], "far_blocks": st["n_far"],
            "factor_bytes": st["factor_bytes"], "rank_max": st["rank_max"],
            "build_s": round(build_s, 2), "aca_s": round(st["aca_ms"] / 1e3, 2),
            "kernel_ms": kernels, "parallelism": "single GPU",
        },
        "rel_err_on_sample": err_head,
        "meets_gate": None if err_head is None else bool(err_head <= GATE),
        "gain_vs_fp64_1rhs": None if baseline is None else baseline["gain"],
        "baseline_fp64_1rhs": baseline,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "device_copy_gbs": None if copy_gbs is None else round(copy_gbs, 1),
        "device_read_gbs": None if read_gbs is None else round(read_gbs, 1),
        "variants": variants or None,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
