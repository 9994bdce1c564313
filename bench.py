#!/usr/bin/env python3
"""Throughput benchmark of the fused MinxEnt-LBM stream-and-collide step.

Workload: D2Q9 lid-driven cavity, 4096 x 4096 nodes, lid velocity 0.05,
Re = 5000 (tau = 0.62288), rho0 = 1 with seeded 1e-6 noise (seed 1803),
MinxEnt4 collision.  Headline form: populations stored in FP32, every node
computed in FP64 (moments, logarithms, Newton step, correction).  The same
steps are also timed for the plain FP64 form; the headline form's field error
against it is reported.

One step = one pass of the fused update over all 16.8 M nodes; the launch
shape the autotuner picks takes one or two steps per launch (the two-step
shapes keep the intermediate step in on-chip memory; results are bitwise the
same).  Inputs are resident in HBM before timing starts.  MLUPS = nodes *
timed steps / seconds / 1e6.

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
# Algorithmic bytes per lattice update: nine populations read once and written
# once per step, at the stored width.
BYTES_PER_LU = {"fp64": 144, "fp32": 72, "fp32_newton64": 72, "fp16dev": 36}
# VALU issue peak: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz lane-operations per
# second (one wave64 VALU instruction is 64 lane-operations issued over four
# cycles); equal to the FP64 vector FMA rate, 78.6 TFLOP/s / 2.
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
PROFILE_TRAFFIC = os.path.join(ROOT, "profiles", "traffic_fused_kernels_bench_workloads.txt")
PROFILE_VALU = os.path.join(ROOT, "profiles", "valu_fused_kernels_bench_workloads.txt")
# The single-step shape quoted beside a two-step headline: 256 x 1 tiles,
# non-temporal loads of the unshifted planes and non-temporal stores, an
# 8-wave register budget, raised issue priority while the loads issue.
SINGLE_STEP_SHAPE = 25


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


def read_valu(digest):
    """VALU lane-operations per node and step of the headline kernel from the
    committed rocprofv3 counter summary, if it was taken on the current kernel
    source."""
    if not os.path.exists(PROFILE_VALU):
        return None
    txt = open(PROFILE_VALU).read()
    m_src = re.search(r"kernel_source_sha256_16:\s*([0-9a-f]+)", txt)
    m_v = re.search(r"headline_valu_per_node_step:\s*([0-9.eE+]+)", txt)
    if not m_src or not m_v or m_src.group(1) != digest:
        return None
    return float(m_v.group(1))


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


def settle_clocks(B, torch, ctx, spl, seconds):
    """Untimed launches of the context's own shape for about `seconds` of wall
    time, so that the timed steps start at the clock the card holds under this
    load (the first launches after idle run while the clock ramps up; under
    sustained FP64 work it then settles at the power limit).  Whole launches
    only, so the state the timed region starts from is a valid step count.
    Returns (settle seconds, settle steps)."""
    if seconds <= 0:
        return (0.0, 0)
    chunk = 64 * spl
    done = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        B.lbm_step(ctx, chunk)
        torch.cuda.synchronize()
        done += chunk
    return (round(time.perf_counter() - t0, 3), done)


def time_form(B, torch, precision, n, tau, u_lid, fields, steps, warmup, tune_cache, force_variant=None,
              settle_s=0.0):
    """Autotune (or read the cache), optionally replace the chosen shape by
    force_variant (the tuned plane pad stays), settle the clock for settle_s
    seconds of untimed launches, then time `steps` steps."""
    p = B.make_params("d2q9", "minxent4", "cavity", precision, n, n, tau, 0.0, u_lid, 1.0)
    ws = torch.empty(B.lbm_workspace_bytes(p), dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()
    ctx = B.lbm_init(p, *fields, workspace=ws, stream=stream)
    variant = B.lbm_autotune(ctx, tune_cache)
    if force_variant is not None:
        variant = force_variant
        B.lbm_set_variant(ctx, variant)
    spl = B.lbm_variant_steps(ctx, variant)
    B.lbm_step(ctx, warmup)
    torch.cuda.synchronize()
    settle = settle_clocks(B, torch, ctx, spl, settle_s)
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
    pad = B.lbm_get_layout(ctx)[1]
    if pad >= 0:
        shape += ", plane pad %d B" % pad
    B.lbm_free(ctx)
    del ws
    return {"wall_s": wall, "event_ms": ev_ms, "variant": shape, "steps_per_launch": spl,
            "nodes": info["nodes"], "bytes_per_step": info["bytes_per_step"],
            "fields": {"rho": r, "ux": u, "uy": v}, "status": st, "settle": settle}


def time_batch(B, torch, params, rho, ux, uy, total, warmup, tune_cache=None, graph_chunk=0):
    """Run a batched context for `total` steps and time the last ones: one
    launch per step (or per several steps) over every instance, replayed from
    captured HIP graphs of graph_chunk steps when graph_chunk > 0.  The
    untimed first steps are `warmup`, or with graphs two chunks (one graph of
    each buffer parity is captured before timing), at most half the run."""
    ws = torch.empty(B.lbm_workspace_bytes_batch(params), dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()
    ctx = B.lbm_init_batch(params, rho, ux, uy, workspace=ws, stream=stream)
    variant = B.lbm_autotune(ctx, tune_cache)
    spl = B.lbm_variant_steps(ctx, variant)
    if graph_chunk > 0:
        # a whole number of launches per graph
        graph_chunk = -(-graph_chunk // spl) * spl
        B.lbm_set_graph_chunk(ctx, graph_chunk)
    warm = min(2 * graph_chunk if graph_chunk > 0 else warmup, total // 2)
    steps = total - warm
    B.lbm_step(ctx, warm)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    B.lbm_step(ctx, steps)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    info = B.lbm_info(ctx)
    r, u, v = B.lbm_moments(ctx)
    st = B.lbm_status(ctx)
    per = B.lbm_status_batch(ctx, len(params))
    shape = B.lbm_variant_name(ctx, variant)
    if graph_chunk > 0:
        shape += ", HIP graphs of %d steps" % graph_chunk
    B.lbm_free(ctx)
    del ws
    return {"wall_s": wall, "event_ms": e0.elapsed_time(e1), "variant": shape, "nodes": info["nodes"],
            "bytes_per_step": info["bytes_per_step"], "fields": {"rho": r, "ux": u, "uy": v}, "status": st,
            "per_instance": per, "steps_per_launch": spl, "graph_chunk": graph_chunk, "timed_steps": steps,
            "total_steps": total}


def launches(steps, spl, chunk):
    """Launches that run `steps` steps with a shape taking up to `spl` steps
    per launch, in HIP graphs of `chunk` steps (0: plain launches)."""
    ceil = lambda a, b: -(-a // b)
    if chunk > 0:
        return steps // chunk * ceil(chunk, spl) + ceil(steps % chunk, spl)
    return ceil(steps, spl)


def rate(res, steps):
    """MLUPS; the algorithmic HBM rate (every stored population read once and
    written once per step, over the event time of the timed steps); and the
    per-launch rate (one read and one write per launch, whatever number of
    steps the launch takes: the bytes HBM must move)."""
    mlups = res["nodes"] * steps / res["wall_s"] / 1e6
    spl = res["steps_per_launch"]
    n = launches(steps, spl, res.get("graph_chunk", 0))
    gbs = res["bytes_per_step"] * n / (res["event_ms"] * 1e-3) / 1e9
    # the method's bytes: every population read and written once per step
    alg = res["bytes_per_step"] * steps / (res["event_ms"] * 1e-3) / 1e9
    return {"mlups": round(mlups, 1), "alg_gbs": round(alg, 1), "alg_hbm_frac": round(alg / HBM_PEAK_GBS, 4),
            "per_launch_gbs": round(gbs, 1), "per_launch_hbm_frac": round(gbs / HBM_PEAK_GBS, 4),
            "steps_per_launch": spl, "launch_shape": res["variant"], "unstable": res["status"]["unstable"]}


def rel_errors(a, b, mask):
    import numpy as np
    out = {}
    for k in ("rho", "ux", "uy"):
        x, y = a[k][mask], b[k][mask]
        if not np.any(y):
            continue
        d = x - y
        out[k] = {"max_rel": float(np.max(np.abs(d)) / np.max(np.abs(y))),
                  "l2_rel": float(np.sqrt(np.sum(d * d) / np.sum(y * y)))}
    return out


def batched_cavities(B, torch, I, steps, warmup, tune_cache=None, graph_chunk=0):
    """512 cavities, sides log-uniform in [32, 512], Re uniform in [100, 1e4],
    lid 0.1, FP32, one launch per step (replayed from HIP graphs when
    graph_chunk > 0); error against the same batch in FP64."""
    import numpy as np
    insts = I.cavity_batch(count=512)
    fields = [I.cavity_fields(n, 1.0, 1804 * 1000 + i) for i, (n, tau, re) in enumerate(insts)]
    rho = np.concatenate([f[0].ravel() for f in fields])
    ux = np.zeros_like(rho)
    masks = []
    for n, tau, re in insts:
        m = np.zeros((n, n), bool)
        m[1:-1, 1:-1] = True
        masks.append(m.ravel())
    mask = np.concatenate(masks)
    out = {}
    res = {}
    for prec in ("fp32", "fp64"):
        params = [B.make_params("d2q9", "minxent4", "cavity", prec, n, n, tau, 0.0, 0.1, 1.0) for n, tau, re in insts]
        res[prec] = time_batch(B, torch, params, rho, ux, ux, steps, warmup, tune_cache, graph_chunk)
        out[prec] = rate(res[prec], res[prec]["timed_steps"])
    out["field_error_fp32_vs_fp64"] = rel_errors(res["fp32"]["fields"], res["fp64"]["fields"], mask)
    out["instances"] = len(insts)
    out["nodes"] = res["fp32"]["nodes"]
    out["total_steps"] = steps
    return out


def moving_flow(B, torch, I, n, tau, steps, warmup, tune_cache):
    """The headline form on the same lattice, started from a vortex that
    fills the cavity (max |u| 0.02) instead of from rest, so that every wave
    evaluates its logarithms on arguments of a developed flow."""
    fields = I.vortex_fields(n, 0.02)
    res = time_form(B, torch, "fp32_newton64", n, tau, 0.05, fields, steps, warmup, tune_cache)
    out = rate(res, steps)
    out["init"] = "vortex filling the cavity, max |u| 0.02, lid 0.05"
    out["timed_steps"] = steps
    return out


def launch_bound(B, torch, I, tune_cache):
    """The two small configurations, whose steps are a few microseconds of
    work: the 800-node D1Q3 shock tube (400 steps, FP64) and the 256^2 cavity
    (20000 steps, FP64 and FP32), each timed with one launch per step and replayed
    from captured HIP graphs of 100 steps (the whole run is one timed
    region; results are bitwise the same)."""
    out = {}
    for name, c, prec in (("tube800_fp64", I.shock_tube_800(), "fp64"), ("cavity256_fp64", I.cavity_256(), "fp64"),
                          ("cavity256_fp32", I.cavity_256(), "fp32")):
        lat = c.get("lattice", "d2q9")
        coll = "srt" if lat == "d1q3" else "minxent4"
        p = B.make_params(lat, coll, c.get("bc", "cavity"), prec, c["nx"], c["ny"], c["tau"], 0.0, c["u_lid"], 1.0)
        res = {}
        for chunk in (0, 100):
            ctx = B.lbm_init(p, c["rho"], c["ux"], c["uy"])
            B.lbm_autotune(ctx, tune_cache)
            if chunk:
                B.lbm_set_graph_chunk(ctx, chunk)
            B.lbm_step(ctx, min(c["steps"], 200))  # warm-up (and graph capture)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            B.lbm_step(ctx, c["steps"])
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            nodes = B.lbm_info(ctx)["nodes"]
            B.lbm_free(ctx)
            res["graph%d" % chunk if chunk else "plain"] = {
                "mlups": round(nodes * c["steps"] / wall / 1e6, 1), "us_per_step": round(wall / c["steps"] * 1e6, 2)}
        res["nodes"] = nodes
        res["steps"] = c["steps"]
        out[name] = res
    return out


def fp16_cavity(B, torch, I, steps, warmup, tune_cache):
    """8192^2 cavity, lid 0.05, Re 5000: FP16 deviation storage against FP64."""
    import numpy as np
    c = I.cavity_8192_params()
    n = c["nx"]
    fields = I.cavity_fields(n, 1.0, c["seed"])
    out, res = {}, {}
    warm = min(warmup, steps // 2)  # the fields compare after `steps` steps in all
    for prec in ("fp16dev", "fp64"):
        res[prec] = time_form(B, torch, prec, n, c["tau"], c["u_lid"], fields, steps - warm, warm, tune_cache)
        out[prec] = rate(res[prec], steps - warm)
        out[prec]["timed_steps"] = steps - warm
    m = np.zeros((n, n), bool)
    m[1:-1, 1:-1] = True
    out["field_error_fp16dev_vs_fp64"] = rel_errors(res["fp16dev"]["fields"], res["fp64"]["fields"], m.ravel())
    out["nodes"] = n * n
    out["total_steps"] = steps
    return out


def fp16_tubes(B, torch, I, steps, warmup, tune_cache=None, graph_chunk=0):
    """4096 D1Q3 shock tubes, lengths log-uniform in [1024, 65536], density
    ratio in [1.5, 4], tau in [0.505, 0.6], 1000 steps: FP16 deviations
    against FP64.  On D1Q3 the method is SRT, which breaks down for the
    sharpest tubes near tau = 1/2; errors are taken per instance over the
    instances stable in both forms, and the unstable ones are counted."""
    import numpy as np
    tubes = I.tube_batch(count=4096)
    rho = np.concatenate([I.tube_fields(n, rl, rr)[0] for n, rl, rr, tau in tubes])
    ux = np.zeros_like(rho)
    out, res = {}, {}
    for prec in ("fp16dev", "fp64"):
        params = [B.make_params("d1q3", "srt", "tube", prec, n, 1, tau, 0.0, 0.0, 0.5 * (rl + rr))
                  for n, rl, rr, tau in tubes]
        res[prec] = time_batch(B, torch, params, rho, ux, None, steps, warmup, tune_cache, graph_chunk)
        out[prec] = rate(res[prec], res[prec]["timed_steps"])
        out[prec]["unstable_instances"] = int(sum(s_["unstable"] for s_ in res[prec]["per_instance"]))
    # Errors per instance on the instances stable in both forms (the stated
    # bounds: L2 rho <= 0.04, u <= 0.2; max-relative rho <= 0.05, u <= 0.1 on
    # resolved fronts, <= 0.75 and 1.5 on the under-resolved ones).
    pre = np.r_[0, np.cumsum([t[0] for t in tubes])]
    R, U = res["fp64"]["fields"]["rho"], res["fp64"]["fields"]["ux"]
    r16, u16 = res["fp16dev"]["fields"]["rho"], res["fp16dev"]["fields"]["ux"]
    worst = {"l2_rho": 0.0, "l2_u": 0.0, "max_rho_resolved": 0.0, "max_u_resolved": 0.0,
             "max_rho_under_resolved": 0.0, "max_u_under_resolved": 0.0}
    l2r_all, l2u_all = [], []
    n_res = n_both = 0
    for k, (n, rl, rr, tau) in enumerate(tubes):
        if res["fp16dev"]["per_instance"][k]["unstable"] or res["fp64"]["per_instance"][k]["unstable"]:
            continue
        n_both += 1
        sl = slice(pre[k] + 1, pre[k + 1] - 1)
        dr, du = r16[sl] - R[sl], u16[sl] - U[sl]
        l2r = float(np.sqrt((dr ** 2).sum() / (R[sl] ** 2).sum()))
        l2u = float(np.sqrt((du ** 2).sum() / (U[sl] ** 2).sum()))
        l2r_all.append(l2r)
        l2u_all.append(l2u)
        mr = float(np.abs(dr).max() / np.abs(R[sl]).max())
        mu = float(np.abs(du).max() / np.abs(U[sl]).max())
        resolved = np.abs(np.diff(R[sl])).sum() <= 1.2 * (rl - rr)
        n_res += bool(resolved)
        tag = "resolved" if resolved else "under_resolved"
        worst["l2_rho"] = max(worst["l2_rho"], l2r)
        worst["l2_u"] = max(worst["l2_u"], l2u)
        worst["max_rho_" + tag] = max(worst["max_rho_" + tag], mr)
        worst["max_u_" + tag] = max(worst["max_u_" + tag], mu)
    worst = {k: float("%.3g" % v) for k, v in worst.items()}
    worst["median_l2_rho"] = float("%.3g" % np.median(l2r_all))
    worst["median_l2_u"] = float("%.3g" % np.median(l2u_all))
    worst["instances_stable_in_both"] = n_both
    worst["instances_resolved"] = n_res
    out["field_error_fp16dev_vs_fp64_per_instance_worst"] = worst
    out["stability_outcome_differs"] = int(sum(a["unstable"] != b["unstable"] for a, b in
                                               zip(res["fp16dev"]["per_instance"], res["fp64"]["per_instance"])))
    out["instances"] = len(tubes)
    out["nodes"] = res["fp16dev"]["nodes"]
    out["total_steps"] = steps
    return out


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


ORACLE_WINDOW_CHILD = r"""
import sys, time
sys.path.insert(0, sys.argv[1])
from oracle import oracle as O
from paper_1801_03863_amd import inputs as I
n, y0, rows, steps, tau, u_lid, seed = (int(sys.argv[2]), int(sys.argv[3]), int(sys.argv[4]), int(sys.argv[5]),
                                        float(sys.argv[6]), float(sys.argv[7]), int(sys.argv[8]))
r, u, v = I.cavity_fields_window(n, 0, y0, n, rows, 1.0, seed)
w = (0, y0, n, rows)
t0 = time.perf_counter()
O.run(O.D2Q9, O.MINXENT4, O.BC_CAVITY, n, n, tau, r, u, v, steps=0, u_lid=u_lid, window=w)
t1 = time.perf_counter()
O.run(O.D2Q9, O.MINXENT4, O.BC_CAVITY, n, n, tau, r, u, v, steps=steps, u_lid=u_lid, window=w)
t2 = time.perf_counter()
print(max((t2 - t1) - (t1 - t0), 1e-9))
"""


def host_cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_all_cores(n, tau, u_lid, seed, steps=8):
    """One single-threaded oracle process per usable host core (at most 16,
    the host share of one GPU), each over its own block of rows of the same
    cavity.  The processes are children started fresh (no fork of this
    process, which holds the GPU); each times its own run minus a zero-step
    run of its window.  Aggregate MLUPS = all lattice updates / the slowest
    child's time."""
    import subprocess
    cores = max(1, min(len(os.sched_getaffinity(0)), 16))
    rows = max(1, min(256, n // cores))
    env = dict(os.environ, OMP_NUM_THREADS="1")
    procs = [subprocess.Popen([sys.executable, "-c", ORACLE_WINDOW_CHILD, ROOT, str(n), str(k * rows), str(rows),
                               str(steps), repr(tau), repr(u_lid), str(seed)],
                              stdout=subprocess.PIPE, stderr=subprocess.PIPE, env=env, text=True)
             for k in range(cores)]
    secs = []
    for p in procs:
        o, e = p.communicate()
        if p.returncode != 0:
            raise RuntimeError("oracle child failed: " + e[-400:])
        secs.append(float(o.strip().splitlines()[-1]))
    lu = n * rows * steps * cores
    return {"value": round(lu / max(secs) / 1e6, 4), "unit": "MLUPS", "cores": cores,
            "cpu_model": host_cpu_model(), "nproc": os.cpu_count(),
            "sample": "%d processes, rows [%d k, %d k + %d) of the %dx%d cavity (k = process), %d steps each, "
                      "FP64 single-threaded C oracle per process; init subtracted; slowest process %.2f s"
                      % (cores, rows, rows, rows, n, n, steps, max(secs))}


def oracle_tube_800():
    """The 800-node D1Q3 shock tube (tau 0.51, 400 steps), whole, in the oracle."""
    from oracle import oracle as O
    from paper_1801_03863_amd import inputs as I
    c = I.shock_tube_800()
    t0 = time.perf_counter()
    O.run(O.D1Q3, O.SRT, O.BC_TUBE, c["nx"], 1, c["tau"], c["rho"], c["ux"], steps=c["steps"])
    secs = time.perf_counter() - t0
    return {"value": round(c["nx"] * c["steps"] / secs / 1e6, 3), "unit": "MLUPS", "seconds": round(secs, 4),
            "cores": 1, "sample": "whole run, %d nodes x %d steps" % (c["nx"], c["steps"])}


def oracle_cavity_256_stored():
    """The oracle time of the whole 256^2, 20000-step cavity, stored when the
    golden file of the full-length parity test was written (one core of the
    machine that wrote it, not this host)."""
    path = os.path.join(ROOT, "tests", "golden", "cavity256_re1000_20000.json")
    with open(path) as fh:
        g = json.load(fh)
    n, steps, secs = g["n"], g["steps"], g["oracle_seconds"]
    return {"value": round(n * n * steps / secs / 1e6, 3), "unit": "MLUPS", "seconds": secs, "cores": 1,
            "sample": "whole run, %dx%d x %d steps; stored in tests/golden (measured when it was written, "
                      "on the build host)" % (n, n, steps)}


def oracle_batch_subsets(cavities=3, tubes=16):
    """Seeded subsets of the two batches run whole in the oracle (one core):
    the smallest cavities of the 512-cavity batch for their 5000 steps and the
    shortest tubes of the 4096-tube batch for their 1000 steps; the rate is
    extrapolated to the whole batch by lattice updates."""
    from oracle import oracle as O
    from paper_1801_03863_amd import inputs as I
    out = {}
    insts = I.cavity_batch(count=512)
    order = sorted(range(len(insts)), key=lambda i: insts[i][0])[:cavities]
    lu = secs = 0.0
    for i in order:
        m, tau, re = insts[i]
        r, u, v = I.cavity_fields(m, 1.0, 1804 * 1000 + i)
        t0 = time.perf_counter()
        O.run(O.D2Q9, O.MINXENT4, O.BC_CAVITY, m, m, tau, r, u, v, steps=5000, u_lid=0.1)
        secs += time.perf_counter() - t0
        lu += m * m * 5000
    total = sum(m * m for m, tau, re in insts) * 5000
    rate = lu / secs / 1e6
    out["cavities_512_fp64"] = {
        "value": round(rate, 3), "unit": "MLUPS", "cores": 1, "seconds": round(secs, 2),
        "extrapolated_whole_batch_hours": round(total / (rate * 1e6) / 3600, 2),
        "sample": "the %d smallest cavities of the 512-cavity batch (sides %s), 5000 steps each, whole; "
                  "extrapolated to the batch by lattice updates" % (cavities, [insts[i][0] for i in order])}
    tb = I.tube_batch(count=4096)
    order = sorted(range(len(tb)), key=lambda i: tb[i][0])[:tubes]
    lu = secs = 0.0
    for i in order:
        m, rl, rr, tau = tb[i]
        r, u = I.tube_fields(m, rl, rr)[:2]
        t0 = time.perf_counter()
        O.run(O.D1Q3, O.SRT, O.BC_TUBE, m, 1, tau, r, u, steps=1000)
        secs += time.perf_counter() - t0
        lu += m * 1000
    total = sum(t[0] for t in tb) * 1000
    rate = lu / secs / 1e6
    out["tubes_4096_fp64"] = {
        "value": round(rate, 3), "unit": "MLUPS", "cores": 1, "seconds": round(secs, 2),
        "extrapolated_whole_batch_hours": round(total / (rate * 1e6) / 3600, 3),
        "sample": "the %d shortest tubes of the 4096-tube batch (%d-%d nodes), 1000 steps each, whole; "
                  "extrapolated to the batch by lattice updates" % (tubes, tb[order[0]][0], tb[order[-1]][0])}
    return out


def cpu_baseline(n, tau, u_lid, seed, rows=512, steps=8, all_cores=True):
    """The FP64 oracle, single-threaded, on rows [0, rows) of the same cavity
    (bottom wall included) for `steps` steps; init and read-back cost removed
    by subtracting a zero-step run of the same window.  Beside it: the
    all-cores figure, the whole 800-node tube, the stored 256^2 time and
    whole-length subsets of the two batches."""
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
    out = {"value": round(n * rows * steps / secs / 1e6, 4), "unit": "MLUPS", "cores": 1, "kind": "oracle",
           "cpu_model": host_cpu_model(),
           "sample": "rows 0-%d of the %dx%d cavity (full width, bottom wall included), %d steps, "
                     "FP64 single-threaded C oracle; init/read-back subtracted" % (rows - 1, n, n, steps)}
    if all_cores:
        out["all_cores"] = oracle_all_cores(n, tau, u_lid, seed, steps)
    out["tube800_full"] = oracle_tube_800()
    out["cavity256_20000_stored"] = oracle_cavity_256_stored()
    out.update(oracle_batch_subsets())
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--settle", type=float, default=0.5,
                    help="seconds of untimed headline launches before its timed steps")
    ap.add_argument("--n", type=int, default=4096)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--tune-cache", default=os.path.join(ROOT, "paper_1801_03863_amd", "tune_cache_gfx950.txt"),
                    help="autotuner cache (entries are keyed by a hash of the kernel sources)")
    ap.add_argument("--no-extra", action="store_true", help="skip the batched and FP16 workloads")
    ap.add_argument("--extra-steps", type=int, default=500)
    ap.add_argument("--no-launch-bound", action="store_true", help="skip the two small launch-bound configurations")
    ap.add_argument("--batch-graph-chunk", type=int, default=50,
                    help="steps per captured HIP graph for the batched workloads (0: plain launches)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: it measures the fused kernel on one GPU's lattice "
              "(no multi-GPU path is implemented); use --gpus 1", file=sys.stderr)
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

    head_form = "fp32_newton64"
    head = time_form(B, torch, head_form, n, tau, cfg["u_lid"], fields, args.steps, args.warmup,
                     args.tune_cache, settle_s=args.settle)
    settle_s, settle_steps = head["settle"]
    nodes = head["nodes"]
    spl = head["steps_per_launch"]
    n_launch = launches(args.steps, spl, 0)
    ms_launch = head["event_ms"] / n_launch   # HIP events on the context's stream over the timed launches
    value = nodes * args.steps / head["wall_s"] / 1e6
    lu_per_launch = nodes * args.steps / n_launch
    # Per-launch HBM view: one read and one write of every stored population
    # per launch, whatever number of steps the launch takes.
    per_launch_bytes = head["bytes_per_step"]
    per_launch_gbs = per_launch_bytes / (ms_launch * 1e-3) / 1e9
    # The HBM roofline of the method's work: 72 B per lattice update (every
    # population read and written once per step, FP32 storage) times the
    # lattice updates one launch performs, over the launch time.
    alg_bytes = BYTES_PER_LU[head_form] * lu_per_launch
    alg_gbs = alg_bytes / (ms_launch * 1e-3) / 1e9

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
        "dtype": "f32 storage, f64 compute (refinements stopped four orders below the f32 rounding: "
                 "hardware reciprocal for the 4x4 pivots, log series truncated at 2^-42)",
        "data": "synthetic (seeded noise on rho0=1, fluid at rest)",
        "config": {"workload": "d2q9 lid-driven cavity %dx%d, MinxEnt4, lid 0.05, Re 5000, tau %.5f, seed %d"
                               % (n, n, tau, cfg["seed"]),
                   "nodes": nodes, "form": "fp32_newton64", "launch_shape": head["variant"]},
    }
    digest = kernel_source_digest()
    traffic = read_traffic(digest)
    out["roofline"] = {
        "bound": "hbm", "achieved": round(alg_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": round(alg_gbs / HBM_PEAK_GBS, 4), "traffic": traffic,
        "algorithmic_bytes_per_launch": int(alg_bytes), "bytes_per_lattice_update": BYTES_PER_LU[head_form],
        "lattice_updates_per_launch": int(lu_per_launch), "kernel_ms_per_launch": round(ms_launch, 5),
        "steps_per_launch": spl, "launches_timed": n_launch,
        # One read and one write of every stored population per launch: the
        # bytes HBM must move when a launch takes several steps.
        "per_launch_hbm": {"bytes": per_launch_bytes, "achieved": round(per_launch_gbs, 1),
                           "frac": round(per_launch_gbs / HBM_PEAK_GBS, 4)},
    }
    if spl > 1:
        # Several steps per launch cut the HBM bytes per step; what binds the
        # kernel is then VALU issue.  Lane-operations per node and step come
        # from the committed counter summary of the same kernel sources.
        valu = read_valu(digest)
        alu = None if valu is None else valu * lu_per_launch / (ms_launch * 1e-3) / 1e12
        out["roofline"]["binding_roof"] = "valu"
        out["roofline"]["valu"] = {"achieved": None if alu is None else round(alu, 3),
                                   "peak": round(VALU_PEAK_TOPS, 3), "unit": "T VALU lane-ops/s",
                                   "frac": None if alu is None else round(alu / VALU_PEAK_TOPS, 4),
                                   "lane_ops_per_lattice_update": valu}
    else:
        out["roofline"]["binding_roof"] = "hbm"
    out["settle"] = {"seconds": settle_s, "steps": settle_steps,
                     "note": "untimed launches of the headline shape before its timed steps"}
    out["status"] = head["status"]
    # The best single-step shape on the same lattice, the fused kernel as a
    # pure HBM stream (one read and one write of every population per step).
    single = time_form(B, torch, "fp32_newton64", n, tau, cfg["u_lid"], fields, args.extra_steps, args.warmup,
                       args.tune_cache, force_variant=SINGLE_STEP_SHAPE)
    out["single_step_fused_kernel"] = rate(single, args.extra_steps)
    if not args.no_fp64:
        # Same step count as the headline (its settle steps run as warm-up
        # here), so that the fields compare at the same time step.
        ref = time_form(B, torch, "fp64", n, tau, cfg["u_lid"], fields, args.steps, args.warmup + settle_steps,
                        args.tune_cache)
        fp64_mlups = nodes * args.steps / ref["wall_s"] / 1e6
        out["fp64"] = rate(ref, args.steps)
        out["fp64"]["speedup_of_headline"] = round(value / fp64_mlups, 3)
        out["field_error_vs_fp64"] = fluid_errors(head["fields"], ref["fields"], n)
    if not args.no_extra:
        ref32 = time_form(B, torch, "fp32", n, tau, cfg["u_lid"], fields, args.extra_steps, args.warmup,
                          args.tune_cache)
        out["fp32"] = rate(ref32, args.extra_steps)
        out["moving_flow_4096"] = moving_flow(B, torch, I, n, tau, args.extra_steps, args.warmup, args.tune_cache)
        # The batched and FP16 configurations run for their own step counts
        # (5000 and 1000 steps), which take a few seconds each.
        out["batched_cavities_512"] = batched_cavities(B, torch, I, 5000, args.warmup, args.tune_cache,
                                                       args.batch_graph_chunk)
        out["fp16dev_cavity_8192"] = fp16_cavity(B, torch, I, 1000, args.warmup, args.tune_cache)
        out["fp16dev_tubes_4096"] = fp16_tubes(B, torch, I, 1000, 0, args.tune_cache, args.batch_graph_chunk)
        if not args.no_launch_bound:
            out["launch_bound"] = launch_bound(B, torch, I, args.tune_cache)
    out["copy_kernel_gbs"] = round(copy_bandwidth(B, torch), 1)
    out["kernel_source_sha256_16"] = digest
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(n, tau, cfg["u_lid"], cfg["seed"])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
