"""Benchmark: HODLR3D mat-vec throughput on one MI355X.

A step is one full mat-vec y = K~x (gather, near-field tiles, both factor
streams, scatter) over the resident operator of the workload; the build
(tree, lists, ACA, packing) happens before the timed region and is reported
separately.  Prints one JSON line.

The roofline object describes the dominant kernel of the step: its
algorithmic bytes per launch (factor bytes it streams plus the x/z/y vectors
it must touch) over its average launch time, taken with HIP events recorded
by the library on the launch stream during the timed steps.

The cpu_baseline object times the CPU oracle's exact dense direct sum on a
bounded sample of target rows of the same workload (rows per second), and
reports the GPU result's relative error on those rows.

The variants object measures the same workload with FP32 and BF16 factors,
with FP32 factors recompressed to their optimal ranks (rank truncation), and
with 64 right-hand sides (matrix-core path), each with its relative error
on sampled rows of the exact product and its gain over the plain FP64 form,
and the multi-problem form: 32 independent clouds (N_i in [8192, 131072],
FP32 factors, tol 1e-7) multiplied in one persistent launch, beside the same
problems' own products run one after another.

roofline.traffic is the dominant kernel's HBM traffic per launch from the
hardware counters FETCH_SIZE and WRITE_SIZE (rocprofv3 --pmc, one counter per
run, on this workload), each divided by what the same counter reads for a
plain 2 GiB device copy (--calibration-copy).  Readings are kept for the two
kernels that take the largest share of the product (stage 2, and stage 1
whose per-launch figure is the mean over its launches, one per level).  They
hold for the sources they were taken on: if any library source that these
kernels' code, their launches or the factor layout depend on has changed
since, traffic is null.
"""
from __future__ import annotations

import argparse
import glob
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

METRIC = "HODLR3D matvec points·RHS/s vs plain FP64 GPU at rel err ≤1e-6; HBM GB/s"
UNIT = "points·RHS/s"
HBM_PEAK_GBS = 8000.0
DTYPE_NAMES = {"fp64": "f64", "fp32": "f32", "bf16": "bf16"}

# Counter readings on uniform262k (FP64 factors, one RHS), KiB per dispatch
# (stage 1: the mean over the four dispatches of one product), with the
# copy-kernel scale of each counter.  The runs that produced them are listed in
# profiles/; sources_sha256 identifies the library sources they were taken on
# (see sources_digest).
TRAFFIC = {
    "workload": "uniform262k",
    "fetch_scale": 0.500016,
    "write_scale": 1.000000,
    "kernels": {
        "k_stage2": {"fetch_kib": 10105475.4375, "write_kib": 8198.3229},
        "k_s1_wide": {"fetch_kib": 2551872.3438, "write_kib": 35194.4089},
    },
    "sources_sha256": "56043d14438b5b9a3065bde2e48fb7b01c5bfe4361b96bf4191d5524db659a6a",
}


# library sources of kernels launched on their own, on which the counter
# readings above do not depend (many right-hand sides, many problems, optional
# rank truncation, the fused finest level)
OTHER_PATHS = ("batched.hip", "batch.hip", "truncate.hip", "leaf.hip")


def sources_digest() -> str:
    """sha256, in name order, over the library sources and header that the
    stream kernels' code and launches and the factor layout depend on."""
    h = hashlib.sha256()
    files = sorted(f for f in glob.glob(os.path.join(ROOT, "paper_2307_16303_amd", "csrc", "*"))
                   if os.path.basename(f) not in OTHER_PATHS)
    files.append(os.path.join(ROOT, "include", "hodlr3d.h"))
    for f in files:
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def traffic_bytes(kernel: str, workload: str, factor_dtype: str, nrhs: int):
    """HBM bytes per launch from the stored counter readings, or None."""
    t = TRAFFIC
    k = None if t is None else t["kernels"].get(kernel)
    if (k is None or t["workload"] != workload or factor_dtype != "fp64" or nrhs != 1
            or t["sources_sha256"] != sources_digest()):
        return None
    return k["fetch_kib"] * 1024.0 / t["fetch_scale"] + k["write_kib"] * 1024.0 / t["write_scale"]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="uniform262k")
    ap.add_argument("--factor-dtype", default="fp64", choices=["fp64", "fp32", "bf16"])
    ap.add_argument("--nrhs", type=int, default=1)
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="target CPU time of the oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the FP32 / BF16 / 64-RHS forms measured beside the headline")
    ap.add_argument("--calibration-copy", action="store_true",
                    help="after the timed steps, fill and copy a 2 GiB buffer: the plain "
                         "kernels that hardware byte counters are scaled by; then time "
                         "torch's sum over it, a plain read stream")
    return ap.parse_args()


def time_products(op, x, steps, warmup):
    import torch
    for _ in range(warmup):
        y = op.matvec(x)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        y = op.matvec(x)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps, y


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(the mat-vec would shard by target box with one all-gather of x).", file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2307_16303_amd import hodlr3d, inputs

    w = inputs.WORKLOADS[args.workload]
    n = w["n"]
    pts = inputs.workload_points(args.workload)
    x_np = inputs.workload_rhs(args.workload, None if args.nrhs == 1 else args.nrhs)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    t0 = time.perf_counter()
    op = hodlr3d.build(torch.as_tensor(pts, device=dev), kernel=w["kernel"],
                       leaf_size=w["leaf_size"], tol=w["tol"], factor_dtype=args.factor_dtype,
                       box_lo=inputs.CUBE_LO, box_side=inputs.CUBE_SIDE)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    st = op.stats()
    print(f"[bench] built {args.workload}: depth {st['depth']}, {st['n_far']} far blocks, "
          f"{st['factor_bytes'] / 1e9:.2f} GB factors, build {build_s:.1f} s", file=sys.stderr,
          flush=True)
    x = torch.as_tensor(x_np, device=dev)
    for _ in range(args.warmup):
        y = op.matvec(x)
    torch.cuda.synchronize()
    op.profile(True)
    op.profile_reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        y = op.matvec(x)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = op.profile_read()
    op.profile(False)
    ms = 1e3 * elapsed / args.steps
    value = n * args.nrhs / (elapsed / args.steps)

    dom = max(prof, key=lambda p: p["total_ms"])
    avg_ms = dom["total_ms"] / max(dom["launches"], 1)
    achieved = dom["bytes_per_launch"] / (avg_ms * 1e-3) / 1e9
    traffic = traffic_bytes(dom["name"], args.workload, args.factor_dtype, args.nrhs)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": None if traffic is None else round(traffic, 0),
                "kernel": dom["name"], "avg_launch_ms": round(avg_ms, 4),
                "bytes_per_launch": dom["bytes_per_launch"]}
    kernels = {p["name"]: round(p["total_ms"] / max(p["launches"], 1), 4) for p in prof}
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
        print(f"[bench] device copy: {copy_gbs:.1f} GB/s (read + write)", file=sys.stderr,
              flush=True)
        # a plain read stream: torch's sum over the same 2 GiB
        s = a.sum()
        torch.cuda.synchronize()
        e0.record()
        for _ in range(5):
            s = a.sum()
        e1.record()
        torch.cuda.synchronize()
        read_gbs = 5 * 2 ** 31 / (e0.elapsed_time(e1) * 1e-3) / 1e9
        print(f"[bench] device read (sum): {read_gbs:.1f} GB/s", file=sys.stderr, flush=True)
        del a, b, s
    y_head = y.detach().cpu().numpy().reshape(n, -1)
    op.close()
    del op
    torch.cuda.empty_cache()

    # the same workload in the other storage forms and with 64 right-hand sides
    variants = {}
    var_y = {}
    if not args.no_variants and args.factor_dtype == "fp64" and args.nrhs == 1:
        x64_np = inputs.workload_rhs(args.workload, 64)
        for name, dt, nr in (("fp32_1rhs", "fp32", 1), ("bf16_1rhs", "bf16", 1),
                             ("fp64_64rhs", "fp64", 64), ("fp32_64rhs", "fp32", 64),
                             ("bf16_64rhs", "bf16", 64)):
            opv = hodlr3d.build(torch.as_tensor(pts, device=dev), kernel=w["kernel"],
                                leaf_size=w["leaf_size"], tol=w["tol"], factor_dtype=dt,
                                box_lo=inputs.CUBE_LO, box_side=inputs.CUBE_SIDE)
            xv = torch.as_tensor(x_np if nr == 1 else x64_np, device=dev)
            sec, yv = time_products(opv, xv, max(3, args.steps // (4 if nr > 1 else 1)),
                                    max(1, args.warmup // 2))
            var_y[name] = yv.detach().cpu().numpy().reshape(n, -1)
            variants[name] = {"factor_dtype": dt, "nrhs": nr, "ms_per_step": round(1e3 * sec, 4),
                              "value": round(n * nr / sec, 1),
                              "gain_vs_fp64_1rhs": round(n * nr / sec / value, 2),
                              "factor_bytes": opv.stats()["factor_bytes"]}
            print(f"[bench] {name}: {1e3 * sec:.3f} ms, {n * nr / sec:.3e} {UNIT}", file=sys.stderr,
                  flush=True)
            opv.close()
            del opv, xv, yv
            torch.cuda.empty_cache()
        # FP32 factors recompressed in FP64 to their optimal ranks at tol
        opv = hodlr3d.build(torch.as_tensor(pts, device=dev), kernel=w["kernel"],
                            leaf_size=w["leaf_size"], tol=w["tol"], factor_dtype="fp32",
                            box_lo=inputs.CUBE_LO, box_side=inputs.CUBE_SIDE, truncate=True)
        for name, nr in (("fp32_trunc_1rhs", 1), ("fp32_trunc_64rhs", 64)):
            xv = torch.as_tensor(x_np if nr == 1 else x64_np, device=dev)
            sec, yv = time_products(opv, xv, max(3, args.steps // (4 if nr > 1 else 1)),
                                    max(1, args.warmup // 2))
            var_y[name] = yv.detach().cpu().numpy().reshape(n, -1)
            variants[name] = {"factor_dtype": "fp32", "truncated": True, "nrhs": nr,
                              "ms_per_step": round(1e3 * sec, 4), "value": round(n * nr / sec, 1),
                              "gain_vs_fp64_1rhs": round(n * nr / sec / value, 2),
                              "factor_bytes": opv.stats()["factor_bytes"]}
            print(f"[bench] {name}: {1e3 * sec:.3f} ms, {n * nr / sec:.3e} {UNIT}", file=sys.stderr,
                  flush=True)
            del xv, yv
        opv.close()
        del opv
        torch.cuda.empty_cache()

    # many uneven problems in one persistent launch
    batch_ys = None
    if not args.no_variants and args.factor_dtype == "fp64" and args.nrhs == 1:
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
        variants["batch32_fp32"] = {
            "factor_dtype": bw["factor_dtype"], "nrhs": 1, "problems": len(work), "n_total": ntot,
            "ms_per_step": round(1e3 * tb, 4), "value": round(ntot / tb, 1),
            "own_products_in_sequence_ms": round(1e3 * ts, 4),
            "gain_vs_own_products": round(ts / tb, 2),
            "factor_bytes": bst["factor_bytes"], "build_s": round(bbuild, 2)}
        print(f"[bench] batch32: {1e3 * tb:.3f} ms ({1e3 * ts:.3f} ms as own products)",
              file=sys.stderr, flush=True)
        batch_ys = [(work[i][0], work[i][1], ys[i].detach().cpu().numpy()) for i in (0, 17)]
        bop.close()
        del bop, xs, ys
        torch.cuda.empty_cache()

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        oracle.build(force=False)
        threads = min(16, os.cpu_count() or 1)
        oracle.set_num_threads(threads)
        y_np = y_head
        xs = x_np.reshape(n, -1)
        # a probe large enough for every thread to stay busy: the rate of a
        # few dozen rows understates what the threads sustain several times
        probe = inputs.sample_rows(n, min(n, 2048), seed=3)
        t0 = time.perf_counter()
        oracle.dense_rows(pts, xs, probe, kernel=w["kernel"])
        per_row = (time.perf_counter() - t0) / probe.size
        count = int(min(n, max(64, args.cpu_seconds / max(per_row, 1e-9))))
        rows = inputs.sample_rows(n, count, seed=4)
        t0 = time.perf_counter()
        yd = oracle.dense_rows(pts, xs, rows, kernel=w["kernel"])
        cpu_s = time.perf_counter() - t0
        err = float(np.linalg.norm(y_np[rows] - yd) / np.linalg.norm(yd))
        # accuracy of the other forms on sampled rows of the exact product
        if var_y:
            r64 = rows[:64]
            yd64 = oracle.dense_rows(pts, inputs.workload_rhs(args.workload, 64), r64,
                                     kernel=w["kernel"])
            for name, yv in var_y.items():
                ref = yd if yv.shape[1] == 1 else yd64
                rr = rows if yv.shape[1] == 1 else r64
                variants[name]["rel_err_on_sample"] = float(
                    np.linalg.norm(yv[rr] - ref) / np.linalg.norm(ref))
        if batch_ys:
            errs = []
            for pts_i, x_i, y_i in batch_ys:
                r_i = inputs.sample_rows(len(pts_i), 64, seed=3)
                ref = oracle.dense_rows(pts_i, x_i, r_i, kernel=inputs.BATCH_WORKLOAD["kernel"])
                errs.append(float(np.linalg.norm(y_i[r_i] - ref) / np.linalg.norm(ref)))
            variants["batch32_fp32"]["rel_err_on_sample"] = max(errs)
        cpu = {"value": round(rows.size * args.nrhs / cpu_s, 1), "unit": UNIT,
               "cores": oracle.num_threads(), "kind": "oracle",
               "sample": f"exact FP64 direct sum for {rows.size} sampled target rows of the "
                         f"same N={n} workload ({cpu_s:.1f} s)",
               "gpu_rel_err_on_sample": err}

    out = {
        "metric": METRIC, "value": round(value, 1), "unit": UNIT, "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": DTYPE_NAMES[args.factor_dtype], "data": "synthetic",
        "config": {
            "workload": f"{args.workload}: N={n} i.i.d. uniform points in [-1,1]^3, "
                        f"{w['kernel']} kernel, leaf <= {w['leaf_size']}, ACA tol {w['tol']}, "
                        f"{args.factor_dtype} factors, {args.nrhs} RHS",
            "n": n, "nrhs": args.nrhs, "depth": st["depth"], "far_blocks": st["n_far"],
            "factor_bytes": st["factor_bytes"], "rank_max": st["rank_max"],
            "build_s": round(build_s, 2), "aca_s": round(st["aca_ms"] / 1e3, 2),
            "kernel_ms": kernels, "parallelism": "single GPU",
        },
        "roofline": roofline,
        "cpu_baseline": cpu,
        "device_copy_gbs": None if copy_gbs is None else round(copy_gbs, 1),
        "device_read_gbs": None if read_gbs is None else round(read_gbs, 1),
        "variants": variants or None,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
