#!/usr/bin/env python3
"""Throughput benchmark of the fused MinxEnt-LBM stream-and-collide step.

Workload: D2Q9 lid-driven cavity, 4096 x 4096 nodes, lid velocity 0.05,
Re = 5000 (tau = 0.62288), rho0 = 1 with seeded 1e-6 noise (seed 1803),
MinxEnt4 collision.  Headline form: populations stored in FP32, every node
computed in FP64 (moments, logarithms, Newton step, correction).  The same
steps are also timed for the plain FP64 form; the headline form's field error
against it is reported.

One step = one fused launch over all 16.8 M nodes.  Inputs are resident in
HBM before timing starts.  MLUPS = nodes * timed steps / seconds / 1e6.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
Prints one JSON line.
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
PROFILE_TRAFFIC = os.path.join(ROOT, "profiles", "traffic_d2q9_fp32n64_cavity4096.txt")


def kernel_source_digest():
    h = hashlib.sha256()
    for name in ("collide.hpp", "kernels.hip", "kernels.hpp"):
        with open(os.path.join(ROOT, "paper_1801_03863_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def read_traffic(digest):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel source."""
    if not os.path.exists(PROFILE_TRAFFIC):
        return None
    txt = open(PROFILE_TRAFFIC).read()
    m_src = re.search(r"kernel_source_sha256_16:\s*([0-9a-f]+)", txt)
    m_b = re.search(r"hbm_bytes_per_launch_scaled:\s*([0-9.eE+]+)", txt)
    if not m_src or not m_b or m_src.group(1) != digest:
        return None
    return float(m_b.group(1))


def fluid_errors(a, b, n):
    import numpy as np
    out = {}
    for k in ("rho", "ux", "uy"):
        x = a[k].reshape(n, n)[1:-1, 1:-1]
        y = b[k].reshape(n, n)[1:-1, 1:-1]
        d = x - y
        out[k] = {"max_rel": float(np.max(np.abs(d)) / np.max(np.abs(y))),
                  "l2_rel": float(np.sqrt(np.sum(d * d) / np.sum(y * y)))}
    return out


def time_form(B, torch, precision, n, tau, u_lid, fields, steps, warmup, tune_cache):
    p = B.make_params("d2q9", "minxent4", "cavity", precision, n, n, tau, 0.0, u_lid, 1.0)
    ws = torch.empty(B.lbm_workspace_bytes(p), dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()
    ctx = B.lbm_init(p, *fields, workspace=ws, stream=stream)
    variant = B.lbm_autotune(ctx, tune_cache)
    B.lbm_step(ctx, warmup)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    B.lbm_step(ctx, steps)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev_ms = e0.elapsed_time(e1)
    info = B.lbm_info(ctx)
    r, u, v = B.lbm_moments(ctx)
    st = B.lbm_status(ctx)
    shape = B.lbm_variant_name(ctx, variant)
    B.lbm_free(ctx)
    del ws
    return {"wall_s": wall, "event_ms": ev_ms, "variant": shape,
            "nodes": info["nodes"], "bytes_per_step": info["bytes_per_step"],
            "fields": {"rho": r, "ux": u, "uy": v}, "status": st}


def copy_bandwidth(B, torch, nbytes=2 << 30, reps=10):
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        B.lbm_copy_kernel(dst, src, nbytes)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        B.lbm_copy_kernel(dst, src, nbytes)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    return 2 * nbytes / ms / 1e6


def cpu_baseline(n, tau, u_lid, seed, rows=512, steps=8):
    """The FP64 oracle, single-threaded, on rows [0, rows) of the same cavity
    (bottom wall included) for `steps` steps; init and read-back cost removed
    by subtracting a zero-step run of the same window."""
    from oracle import oracle as O
    from paper_1801_03863_amd import inputs as I
    r, u, v = I.cavity_fields_window(n, 0, 0, n, rows, 1.0, seed)
    O.build(force=False)
    t0 = time.perf_counter()
    O.run(O.D2Q9, O.MINXENT4, O.BC_CAVITY, n, n, tau, r, u, v, steps=0, u_lid=u_lid, window=(0, 0, n, rows))
    t_init = time.perf_counter() - t0
    t0 = time.perf_counter()
    O.run(O.D2Q9, O.MINXENT4, O.BC_CAVITY, n, n, tau, r, u, v, steps=steps, u_lid=u_lid, window=(0, 0, n, rows))
    t_run = time.perf_counter() - t0
    secs = max(t_run - t_init, 1e-9)
    return {"value": round(n * rows * steps / secs / 1e6, 4), "unit": "MLUPS", "cores": 1, "kind": "oracle",
            "sample": "rows 0-%d of the %dx%d cavity (full width, bottom wall included), %d steps, "
                      "FP64 single-threaded C oracle; init/read-back subtracted" % (rows - 1, n, n, steps)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=4096)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--tune-cache", default=None)
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: this build measures the single-GPU kernel; "
              "use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1801_03863_amd import binding as B
    from paper_1801_03863_amd import inputs as I

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    cfg = I.cavity_4096_params()
    n = args.n
    tau = I.tau_from_re(cfg["u_lid"], n, cfg["re"])
    fields = I.cavity_fields(n, 1.0, cfg["seed"])

    head = time_form(B, torch, "fp32_newton64", n, tau, cfg["u_lid"], fields, args.steps, args.warmup,
                     args.tune_cache)
    nodes = head["nodes"]
    ms_event = head["event_ms"] / args.steps
    value = nodes * args.steps / head["wall_s"] / 1e6
    achieved = head["bytes_per_step"] / (ms_event * 1e-3) / 1e9

    out = {
        "metric": "MLUPS and % of HBM roofline, FP64 vs FP32/batched at stated field error",
        "value": round(value, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(head["wall_s"] * 1e3 / args.steps, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 storage, f64 compute",
        "data": "synthetic (seeded noise on rho0=1, fluid at rest)",
        "config": {"workload": "d2q9 lid-driven cavity %dx%d, MinxEnt4, lid 0.05, Re 5000, tau %.5f, seed %d"
                               % (n, n, tau, cfg["seed"]),
                   "nodes": nodes, "form": "fp32_newton64", "launch_shape": head["variant"]},
    }
    digest = kernel_source_digest()
    traffic = read_traffic(digest)
    out["roofline"] = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                       "algorithmic_bytes_per_launch": head["bytes_per_step"],
                       "kernel_ms_per_launch": round(ms_event, 5)}
    out["status"] = head["status"]
    if not args.no_fp64:
        ref = time_form(B, torch, "fp64", n, tau, cfg["u_lid"], fields, args.steps, args.warmup, args.tune_cache)
        fp64_mlups = nodes * args.steps / ref["wall_s"] / 1e6
        out["fp64"] = {"mlups": round(fp64_mlups, 1),
                       "achieved_gbs": round(ref["bytes_per_step"] / (ref["event_ms"] / args.steps * 1e-3) / 1e9, 1),
                       "speedup_of_headline": round(value / fp64_mlups, 3)}
        out["field_error_vs_fp64"] = fluid_errors(head["fields"], ref["fields"], n)
    out["copy_kernel_gbs"] = round(copy_bandwidth(B, torch), 1)
    out["kernel_source_sha256_16"] = digest
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(n, tau, cfg["u_lid"], cfg["seed"])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
