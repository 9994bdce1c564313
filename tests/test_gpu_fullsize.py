"""Parity at the benchmark sizes and for the batched launch form.

- 4096^2 cavity (the benchmark workload) in FP64 and FP32-storage forms,
  run on the GPU at full size and compared with windowed oracle runs at
  sampled nodes (each window covers the node's dependency cone, so the
  oracle value is exact).
- 256^2 cavity for its full 20000 steps against stored oracle values.
- Batched cavities and shock tubes against the oracle per instance and
  bitwise against single-instance contexts.
"""
import json
import os
import shutil

import numpy as np
import pytest

from paper_1801_03863_amd import inputs as I
from tests.gpu_helpers import B, fluid_mask, gpu_run, orc_run

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CACHE = os.path.join(ROOT, "paper_1801_03863_amd", "tune_cache_gfx950.txt")


def bench_tuning(b, ctx, tmp_path):
    """The launch configuration bench.py times: launch shape and plane pad
    from the committed tuning cache, read through a copy so that a missing
    key is tuned without touching the package's file."""
    path = tmp_path / "tune_cache.txt"
    if os.path.exists(CACHE):
        shutil.copy(CACHE, path)
    return b.lbm_autotune(ctx, str(path))


def sample_points(n, count, seed):
    idx = np.arange(count, dtype=np.uint64)
    xs = np.floor(I.splitmix_uniform(seed, 2 * idx) * n).astype(int)
    ys = np.floor(I.splitmix_uniform(seed, 2 * idx + np.uint64(1)) * n).astype(int)
    pts = list(zip(xs.tolist(), ys.tolist()))
    # corners, walls, lid-adjacent row, centre
    pts += [(1, 1), (n - 2, 1), (1, n - 2), (n - 2, n - 2), (n // 2, n - 2), (n // 2, 1), (1, n // 2),
            (n - 2, n // 2), (n // 2, n // 2), (2, n - 2), (n - 3, n - 2)]
    return [(x, y) for x, y in pts if 0 < x < n - 1 and 0 < y < n - 1]


def windowed_oracle(c, n, steps, x, y):
    k = steps + 1
    x0, x1 = max(0, x - k), min(n, x + k + 1)
    y0, y1 = max(0, y - k), min(n, y + k + 1)
    r, u, v = I.cavity_fields_window(n, x0, y0, x1 - x0, y1 - y0, 1.0, c["seed"])
    o = orc_run("d2q9", "minxent4", "cavity", n, n, c["tau"], r, u, v, steps=steps, u_lid=c["u_lid"],
                window=(x0, y0, x1 - x0, y1 - y0))
    return {f: o[f][y - y0, x - x0] for f in ("rho", "ux", "uy")}


@pytest.mark.parametrize("n,precision,tol_rho,tol_u", [
    (4096, "fp64", 1e-12, 1e-12), (4096, "fp32_newton64", 1e-7, 5e-6), (4096, "fp32", 1e-6, 1e-5),
    (8192, "fp16dev", 5e-5, 2e-3)])
def test_benchmark_cavity_sampled(n, precision, tol_rho, tol_u, tmp_path):
    c = I.cavity_4096_params() if n == 4096 else I.cavity_8192_params()
    n, steps = c["nx"], 6
    r, u, v = I.cavity_fields(n, 1.0, c["seed"])
    b = B()
    p = b.make_params("d2q9", "minxent4", "cavity", precision, n, n, c["tau"], 0.0, c["u_lid"], 1.0)
    ctx = b.lbm_init(p, r, u, v)
    try:
        bench_tuning(b, ctx, tmp_path)
        b.lbm_step(ctx, steps)
        gr, gu, gv = (a.reshape(n, n) for a in b.lbm_moments(ctx))
        st = b.lbm_status(ctx)
    finally:
        b.lbm_free(ctx)
    assert not st["unstable"] and st["guarded"] == 0
    pts = sample_points(n, 24, 99)
    umax = 0.0
    worst = {"rho": 0.0, "u": 0.0}
    for x, y in pts:
        o = windowed_oracle(c, n, steps, x, y)
        worst["rho"] = max(worst["rho"], abs(gr[y, x] - o["rho"]) / abs(o["rho"]))
        worst["u"] = max(worst["u"], abs(gu[y, x] - o["ux"]), abs(gv[y, x] - o["uy"]))
        umax = max(umax, abs(o["ux"]), abs(o["uy"]))
    worst["u"] /= max(umax, 1e-300)
    print(precision, worst, "umax", umax, flush=True)
    assert worst["rho"] <= tol_rho and worst["u"] <= tol_u


def test_cavity_256_full_length_against_stored_oracle():
    path = os.path.join(ROOT, "tests", "golden", "cavity256_re1000_20000.json")
    if not os.path.exists(path):
        pytest.skip("stored oracle values not generated")
    g = json.load(open(path))
    c = I.cavity_256()
    n = c["nx"]
    b = B()
    p = b.make_params("d2q9", "minxent4", "cavity", "fp64", n, n, c["tau"], 0.0, c["u_lid"], 1.0)
    ctx = b.lbm_init(p, c["rho"], c["ux"], c["uy"])
    try:
        b.lbm_set_graph_chunk(ctx, 100)
        b.lbm_step(ctx, g["steps"])
        fr, fu, fv = (a.reshape(n, n) for a in b.lbm_moments(ctx))
        st = b.lbm_status(ctx)
    finally:
        b.lbm_free(ctx)
    assert not st["unstable"] and st["guarded"] == g["guarded"] == 0
    fields = {"rho": fr, "ux": fu, "uy": fv}
    for k in ("rho", "ux", "uy"):
        ref = np.array([float.fromhex(h) for h in g[k]])
        got = np.array([fields[k][y, x] for x, y in g["nodes"]])
        emax = np.max(np.abs(got - ref)) / float.fromhex(g["fluid_max_abs"][k])
        el2 = np.sqrt(np.sum((got - ref) ** 2) / np.sum(ref ** 2))
        print(k, "max %.2e l2 %.2e" % (emax, el2), flush=True)
        assert emax <= 1e-12 and el2 <= 1e-12, k
    fl = (slice(1, n - 1), slice(1, n - 1))
    assert abs(fr[fl].sum() - float.fromhex(g["fluid_sum_rho"])) <= 1e-12 * (n - 2) ** 2


def cavity_batch_subset(count=12):
    insts = I.cavity_batch(count=512)
    # the smallest instances (the oracle runs them whole) plus a spread of sizes
    order = sorted(range(512), key=lambda i: insts[i][0])
    pick = order[:count // 2] + order[::512 // (count // 2)][: count // 2]
    return [insts[i] + (i,) for i in pick]


@pytest.mark.parametrize("precision", ["fp64"])
def test_batched_cavities_match_oracle_and_single_runs(precision):
    sel = cavity_batch_subset()
    b = B()
    params, rs, us, vs, fields = [], [], [], [], []
    for (n, tau, re, i) in sel:
        r, u, v = I.cavity_fields(n, 1.0, 1804 * 1000 + i)
        params.append(b.make_params("d2q9", "minxent4", "cavity", precision, n, n, tau, 0.0, 0.1, 1.0))
        rs.append(r.ravel()); us.append(u.ravel()); vs.append(v.ravel()); fields.append((r, u, v))
    steps = 60
    ctx = b.lbm_init_batch(params, np.concatenate(rs), np.concatenate(us), np.concatenate(vs))
    try:
        b.lbm_step(ctx, steps)
        R, U, V = b.lbm_moments(ctx)
        F = b.lbm_get_populations(ctx, 9)
        sts = b.lbm_status_batch(ctx, len(sel))
    finally:
        b.lbm_free(ctx)
    off = 0
    foff = 0
    for k, (n, tau, re, i) in enumerate(sel):
        m = n * n
        g = {"rho": R[off:off + m].reshape(n, n), "ux": U[off:off + m].reshape(n, n),
             "uy": V[off:off + m].reshape(n, n)}
        fl = fluid_mask("d2q9", "cavity", n, n)
        if n <= 64:
            o = orc_run("d2q9", "minxent4", "cavity", n, n, tau, *fields[k], steps=steps, u_lid=0.1)
            for f in ("rho", "ux", "uy"):
                err = np.max(np.abs(g[f] - o[f])[fl]) / np.max(np.abs(o[f][fl]))
                assert err <= 1e-12, (n, f, err)
        single = gpu_run("d2q9", "minxent4", "cavity", precision, n, n, tau, *fields[k], steps=steps,
                         u_lid=0.1, want_f=True)
        assert np.array_equal(single["f"], F[foff:foff + 9 * m]), (k, n)
        assert not sts[k]["unstable"]
        off += m
        foff += 9 * m


@pytest.mark.parametrize("precision", ["fp64", "fp16dev"])
def test_batched_tubes(precision):
    tubes = I.tube_batch(count=4096)[:10] + [(3, 1.5, 0.75, 0.55), (1024, 4.0 * 0.75, 0.75, 0.505)]
    b = B()
    params, rs, us = [], [], []
    for (n, rl, rr, tau) in tubes:
        r, u = I.tube_fields(n, rl, rr)
        # FP16 deviations are taken from the mean of the two densities.
        params.append(b.make_params("d1q3", "srt", "tube", precision, n, 1, tau, 0.0, 0.0, 0.5 * (rl + rr)))
        rs.append(r); us.append(u)
    steps = 150
    ctx = b.lbm_init_batch(params, np.concatenate(rs), np.concatenate(us), None)
    try:
        b.lbm_step(ctx, steps)
        R, U, _ = b.lbm_moments(ctx)
        sts = b.lbm_status_batch(ctx, len(tubes))
    finally:
        b.lbm_free(ctx)
    off = 0
    # FP64: 1e-12 against the oracle.  FP16 deviations: the stated bounds of
    # the tube batch (the reasoning is in the full-length test of that batch):
    # L2-relative rho <= 0.04 and u <= 0.2; max-relative rho <= 0.05 and
    # u <= 0.1 where the fronts are resolved (total variation of rho at most
    # 1.2 times the initial jump), else rho <= 0.75 and u <= 1.5.
    for k, (n, rl, rr, tau) in enumerate(tubes):
        o = orc_run("d1q3", "srt", "tube", n, 1, tau, rs[k], us[k], steps=steps)
        if o["unstable"]:
            # After a blow-up the fields diverge chaotically; the status and
            # the first unstable step are what is compared.
            assert sts[k]["unstable"], (k, n)
            if precision == "fp64":
                assert sts[k]["first_step"] == o["first_step"], (k, n)
                assert sts[k]["first_node"] == o["first_node"], (k, n)
            off += n
            continue
        fl = fluid_mask("d1q3", "tube", n, 1)
        dr, du = (R[off:off + n] - o["rho"])[fl], (U[off:off + n] - o["ux"])[fl]
        orho, oux = o["rho"][fl], o["ux"][fl]
        er = np.max(np.abs(dr)) / np.max(np.abs(orho))
        eu = np.max(np.abs(du)) / max(np.max(np.abs(oux)), 1e-300)
        print(precision, n, "rho %.2e u %.2e" % (er, eu), flush=True)
        if precision == "fp64":
            assert er <= 1e-12 and eu <= 1e-12, (k, n, er, eu)
        else:
            l2r = np.sqrt((dr ** 2).sum() / (orho ** 2).sum())
            l2u = np.sqrt((du ** 2).sum() / max((oux ** 2).sum(), 1e-300))
            resolved = np.abs(np.diff(orho)).sum() <= 1.2 * (rl - rr)
            mr, mu = (0.05, 0.1) if resolved else (0.75, 1.5)
            assert l2r <= 0.04 and l2u <= 0.2 and er <= mr and eu <= mu, (k, n, l2r, l2u, er, eu, resolved)
        assert not sts[k]["unstable"]
        off += n


def test_batched_launch_shapes_and_graph_bitwise():
    sel = cavity_batch_subset(8)
    b = B()
    params, rs, us, vs = [], [], [], []
    for (n, tau, re, i) in sel:
        r, u, v = I.cavity_fields(n, 1.0, 1804 * 1000 + i)
        params.append(b.make_params("d2q9", "minxent4", "cavity", "fp32", n, n, tau, 0.0, 0.1, 1.0))
        rs.append(r.ravel()); us.append(u.ravel()); vs.append(v.ravel())
    ref = None
    ctx = b.lbm_init_batch(params, np.concatenate(rs), np.concatenate(us), np.concatenate(vs))
    nv = b.lbm_variant_count(ctx)
    b.lbm_free(ctx)
    assert nv >= 2
    for variant in range(nv):
        for graph in (0, 9):
            ctx = b.lbm_init_batch(params, np.concatenate(rs), np.concatenate(us), np.concatenate(vs))
            try:
                b.lbm_set_variant(ctx, variant)
                if graph:
                    b.lbm_set_graph_chunk(ctx, graph)
                b.lbm_step(ctx, 40)
                F = b.lbm_get_populations(ctx, 9)
            finally:
                b.lbm_free(ctx)
            if ref is None:
                ref = F
            assert np.array_equal(ref, F), (variant, graph)


def test_reduced_precision_forms_long_run_error():
    # 256^2 cavity, 20000 steps: each reduced-precision form against the FP64
    # GPU path on fluid nodes.  Bounds are the stated errors of each form.
    c = I.cavity_256()
    n, steps = c["nx"], c["steps"]
    # measured: fp32_newton64 rho 1.1e-6 u 1.9e-5; fp32 rho 6.4e-6 u 1.4e-4;
    # fp16dev rho 2.0e-4 u 3.0e-2 (max over fluid nodes, relative)
    bounds = {"fp32_newton64": (5e-6, 1e-4), "fp32": (3e-5, 1e-3), "fp16dev": (1e-3, 0.1)}
    runs = {}
    for prec in ("fp64", "fp32_newton64", "fp32", "fp16dev"):
        b = B()
        p = b.make_params("d2q9", "minxent4", "cavity", prec, n, n, c["tau"], 0.0, c["u_lid"], 1.0)
        ctx = b.lbm_init(p, c["rho"], c["ux"], c["uy"])
        try:
            b.lbm_set_graph_chunk(ctx, 100)
            b.lbm_step(ctx, steps)
            runs[prec] = [a.reshape(n, n)[1:-1, 1:-1] for a in b.lbm_moments(ctx)]
            assert not b.lbm_status(ctx)["unstable"], prec
        finally:
            b.lbm_free(ctx)
    ref = runs["fp64"]
    for prec, (tol_rho, tol_u) in bounds.items():
        got = runs[prec]
        e_rho = np.max(np.abs(got[0] - ref[0])) / np.max(np.abs(ref[0]))
        umax = max(np.max(np.abs(ref[1])), np.max(np.abs(ref[2])))
        e_u = max(np.max(np.abs(got[1] - ref[1])), np.max(np.abs(got[2] - ref[2]))) / umax
        l2_u = np.sqrt((np.sum((got[1] - ref[1]) ** 2) + np.sum((got[2] - ref[2]) ** 2)) /
                       (np.sum(ref[1] ** 2) + np.sum(ref[2] ** 2)))
        print(prec, "rho max %.2e  u max %.2e  u L2 %.2e" % (e_rho, e_u, l2_u), flush=True)
        assert e_rho <= tol_rho and e_u <= tol_u, prec


def test_batched_tube_shapes_and_graph_bitwise():
    tubes = I.tube_batch(count=4096)[:40]
    b = B()
    params = [b.make_params("d1q3", "srt", "tube", "fp16dev", n, 1, tau, 0.0, 0.0, 0.5 * (rl + rr))
              for n, rl, rr, tau in tubes]
    rho = np.concatenate([I.tube_fields(n, rl, rr)[0] for n, rl, rr, tau in tubes])
    ux = np.zeros_like(rho)
    ref = None
    ctx = b.lbm_init_batch(params, rho, ux, None)
    nv = b.lbm_variant_count(ctx)
    b.lbm_free(ctx)
    assert nv >= 4
    for v in range(nv):
        # every launch shape, plain launches and HIP-graph replay (30 steps =
        # four graphs of 7 steps + 2 plain launches)
        for graph in (0, 7):
            ctx = b.lbm_init_batch(params, rho, ux, None)
            try:
                b.lbm_set_variant(ctx, v)
                if graph:
                    b.lbm_set_graph_chunk(ctx, graph)
                b.lbm_step(ctx, 30)
                F = b.lbm_get_populations(ctx, 3)
            finally:
                b.lbm_free(ctx)
            ref = F if ref is None else ref
            assert np.array_equal(ref, F), (v, graph)


@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp16dev"])
@pytest.mark.parametrize("steps", [1, 50, 77])
def test_lds_resident_persistent_batch_is_bitwise(precision, steps):
    # Small cavities (the stability study's 17^2 and a few others, one of
    # them driven to instability) run all steps in one launch with the
    # lattices in LDS; the result equals per-step launches bit for bit.
    b = B()
    spec = [(17, 0.55, 0.1), (17, 0.5025, 0.9), (23, 0.6, 0.2), (30, 0.52, 0.05), (11, 0.7, 0.3)]
    params = [b.make_params("d2q9", "minxent4", "cavity", precision, n, n, tau, 0.0, u, 1.0) for n, tau, u in spec]
    rho = np.concatenate([np.ones(n * n) for n, _, _ in spec])
    z = np.zeros_like(rho)
    out = {}
    for mode in ("per_step", "lds"):
        ctx = b.lbm_init_batch(params, rho, z, z)
        try:
            names = [b.lbm_variant_name(ctx, v) for v in range(b.lbm_variant_count(ctx))]
            lds = [v for v, nm in enumerate(names) if "LDS" in nm]
            assert lds, names
            b.lbm_set_variant(ctx, lds[0] if mode == "lds" else 0)
            b.lbm_step(ctx, steps)
            b.lbm_step(ctx, 3)
            out[mode] = (b.lbm_get_populations(ctx, 9), b.lbm_status_batch(ctx, len(spec)),
                         b.lbm_info(ctx)["steps_done"])
        finally:
            b.lbm_free(ctx)
    F1, S1, n1 = out["per_step"]
    F2, S2, n2 = out["lds"]
    assert n1 == n2 == steps + 3
    assert np.array_equal(F1, F2, equal_nan=True)
    for a_, b_ in zip(S1, S2):
        assert a_["unstable"] == b_["unstable"] and a_["first_step"] == b_["first_step"]
        assert a_["first_node"] == b_["first_node"]
        assert a_["guarded"] == b_["guarded"]


def test_full_cavity_batch_5000_steps_against_oracle(tmp_path):
    # The whole 512-cavity batch (22.3 M nodes, sides 32..512, Re 100..10000,
    # lid 0.1) for its full 5000 steps in FP64; the oracle reruns the four
    # smallest instances whole.  Instances that blow up are compared by status
    # and first unstable step.
    insts = I.cavity_batch(count=512)
    b = B()
    params, rs, us, vs = [], [], [], []
    for i, (n, tau, re) in enumerate(insts):
        r, u, v = I.cavity_fields(n, 1.0, 1804 * 1000 + i)
        params.append(b.make_params("d2q9", "minxent4", "cavity", "fp64", n, n, tau, 0.0, 0.1, 1.0))
        rs.append(r.ravel()); us.append(u.ravel()); vs.append(v.ravel())
    steps = 5000
    ctx = b.lbm_init_batch(params, np.concatenate(rs), np.concatenate(us), np.concatenate(vs))
    try:
        bench_tuning(b, ctx, tmp_path)
        b.lbm_set_graph_chunk(ctx, 50)  # as bench.py times batches
        b.lbm_step(ctx, steps)
        R, U, V = b.lbm_moments(ctx)
        sts = b.lbm_status_batch(ctx, len(insts))
    finally:
        b.lbm_free(ctx)
    offs = np.concatenate([[0], np.cumsum([n * n for n, _, _ in insts])])
    pick = sorted(range(len(insts)), key=lambda i: insts[i][0])[:4]
    for i in pick:
        n, tau, re = insts[i]
        o = orc_run("d2q9", "minxent4", "cavity", n, n, tau, rs[i].reshape(n, n), us[i].reshape(n, n),
                    vs[i].reshape(n, n), steps=steps, u_lid=0.1)
        assert sts[i]["unstable"] == o["unstable"], (i, n, re)
        if o["unstable"]:
            assert sts[i]["first_step"] == o["first_step"], (i, n, re)
            assert sts[i]["first_node"] == o["first_node"], (i, n, re)
            continue
        m = n * n
        g = {"rho": R[offs[i]:offs[i] + m].reshape(n, n), "ux": U[offs[i]:offs[i] + m].reshape(n, n),
             "uy": V[offs[i]:offs[i] + m].reshape(n, n)}
        fl = fluid_mask("d2q9", "cavity", n, n)
        for f in ("rho", "ux", "uy"):
            err = np.max(np.abs(g[f] - o[f])[fl]) / np.max(np.abs(o[f][fl]))
            print("cavity", i, n, round(re), f, "%.2e" % err, flush=True)
            assert err <= 1e-12, (i, n, f, err)


def test_full_tube_batch_1000_steps_against_oracle(tmp_path):
    # The whole 4096-tube batch (62.6 M nodes) for its full 1000 steps in
    # FP64; the oracle reruns the six shortest tubes whole.
    tubes = I.tube_batch(count=4096)
    b = B()
    params, rs, us = [], [], []
    for (n, rl, rr, tau) in tubes:
        r, u = I.tube_fields(n, rl, rr)
        params.append(b.make_params("d1q3", "srt", "tube", "fp64", n, 1, tau, 0.0, 0.0, 0.5 * (rl + rr)))
        rs.append(r); us.append(u)
    steps = 1000
    ctx = b.lbm_init_batch(params, np.concatenate(rs), np.concatenate(us), None)
    try:
        v = bench_tuning(b, ctx, tmp_path)
        # as bench.py times batches: graphs of 50 steps rounded up to whole
        # launches (256 steps for the tuned 256-step shape)
        spl = b.lbm_variant_steps(ctx, v)
        b.lbm_set_graph_chunk(ctx, -(-50 // spl) * spl)
        b.lbm_step(ctx, steps)
        R, U, _ = b.lbm_moments(ctx)
        sts = b.lbm_status_batch(ctx, len(tubes))
    finally:
        b.lbm_free(ctx)
    offs = np.concatenate([[0], np.cumsum([t[0] for t in tubes])])
    pick = sorted(range(len(tubes)), key=lambda i: tubes[i][0])[:6]
    for i in pick:
        n, rl, rr, tau = tubes[i]
        o = orc_run("d1q3", "srt", "tube", n, 1, tau, rs[i], us[i], steps=steps)
        assert sts[i]["unstable"] == o["unstable"], (i, n)
        if o["unstable"]:
            assert sts[i]["first_step"] == o["first_step"], (i, n)
            assert sts[i]["first_node"] == o["first_node"], (i, n)
            continue
        fl = fluid_mask("d1q3", "tube", n, 1)
        er = np.max(np.abs(R[offs[i]:offs[i] + n] - o["rho"])[fl]) / np.max(np.abs(o["rho"][fl]))
        eu = np.max(np.abs(U[offs[i]:offs[i] + n] - o["ux"])[fl]) / np.max(np.abs(o["ux"][fl]))
        print("tube", i, n, "rho %.2e u %.2e" % (er, eu), flush=True)
        assert er <= 1e-12 and eu <= 1e-12, (i, n, er, eu)


def test_benchmark_cavity_fp64_60_steps_sampled(tmp_path):
    # The 4096^2 benchmark cavity in FP64 for 60 steps in the autotuned shape;
    # 12 sampled nodes (corners, lid row, walls, interior) against windowed
    # oracle runs of (2*61+1)^2 nodes each.
    c = I.cavity_4096_params()
    n, steps = c["nx"], 60
    r, u, v = I.cavity_fields(n, 1.0, c["seed"])
    b = B()
    p = b.make_params("d2q9", "minxent4", "cavity", "fp64", n, n, c["tau"], 0.0, c["u_lid"], 1.0)
    ctx = b.lbm_init(p, r, u, v)
    try:
        bench_tuning(b, ctx, tmp_path)
        b.lbm_step(ctx, steps)
        gr, gu, gv = (a.reshape(n, n) for a in b.lbm_moments(ctx))
        assert not b.lbm_status(ctx)["unstable"]
    finally:
        b.lbm_free(ctx)
    pts = [(1, 1), (n - 2, 1), (1, n - 2), (n - 2, n - 2), (n // 2, n - 2), (n // 3, n - 3), (2 * n // 3, n - 2),
           (1, n // 2), (n - 2, n // 2), (n // 2, 1), (n // 2, n // 2), (257, n - 5)]
    worst = {"rho": 0.0, "u": 0.0}
    umax = 0.0
    for x, y in pts:
        o = windowed_oracle(c, n, steps, x, y)
        worst["rho"] = max(worst["rho"], abs(gr[y, x] - o["rho"]) / abs(o["rho"]))
        worst["u"] = max(worst["u"], abs(gu[y, x] - o["ux"]), abs(gv[y, x] - o["uy"]))
        umax = max(umax, abs(o["ux"]), abs(o["uy"]))
    worst["u"] /= umax
    print("fp64 60 steps", worst, "umax", umax, flush=True)
    assert worst["rho"] <= 1e-12 and worst["u"] <= 1e-12


def _limits_case(b, lattice, sizes, limits, variants, graph):
    """Batch with per-instance step limits, stepped 5 + 7 times, against the
    oracle run of each instance for min(limit, 12) steps."""
    rng = np.random.default_rng(77)
    params, fields = [], []
    for n in sizes:
        if lattice == "d2q9":
            r = 1.0 + 0.02 * rng.uniform(-1, 1, (n, n))
            u = 0.02 * rng.uniform(-1, 1, (n, n))
            v = 0.02 * rng.uniform(-1, 1, (n, n))
            params.append(b.make_params("d2q9", "minxent4", "cavity", "fp64", n, n, 0.6, 0.0, 0.05, 1.0))
        else:
            r = 1.0 + 0.2 * rng.uniform(-1, 1, n)
            u = 0.05 * rng.uniform(-1, 1, n)
            v = None
            params.append(b.make_params("d1q3", "srt", "tube", "fp64", n, 1, 0.7, 0.0, 0.0, 1.0))
        fields.append((r, u, v))
    cat = lambda k: np.concatenate([f[k].ravel() for f in fields]) if fields[0][k] is not None else None
    for variant in variants:
        ctx = b.lbm_init_batch(params, cat(0), cat(1), cat(2))
        try:
            if variant == "lds":
                v = b.lbm_variant_count(ctx) - 1
                assert "LDS" in b.lbm_variant_name(ctx, v)
            else:
                v = variant
            b.lbm_set_variant(ctx, v)
            if graph:
                b.lbm_set_graph_chunk(ctx, graph)
            b.lbm_set_batch_steps(ctx, limits)
            b.lbm_step(ctx, 5)
            b.lbm_step(ctx, 7)
            R, U, V = b.lbm_moments(ctx)
            sts = b.lbm_status_batch(ctx, len(sizes))
        finally:
            b.lbm_free(ctx)
        off = 0
        for k, n in enumerate(sizes):
            m = n * n if lattice == "d2q9" else n
            steps = 12 if limits[k] < 0 else min(limits[k], 12)
            ny = n if lattice == "d2q9" else 1
            shape = (n, n) if lattice == "d2q9" else (n,)
            o = orc_run(lattice, "minxent4" if lattice == "d2q9" else "srt", "cavity" if lattice == "d2q9" else "tube",
                        n, ny, 0.6 if lattice == "d2q9" else 0.7, fields[k][0], fields[k][1], fields[k][2],
                        steps=steps, u_lid=0.05 if lattice == "d2q9" else 0.0)
            fl = fluid_mask(lattice, "cavity" if lattice == "d2q9" else "tube", n, ny)
            for name, G in (("rho", R), ("ux", U)):
                g = G[off:off + m].reshape(shape)
                e = np.max(np.abs(g - o[name])[fl]) / np.max(np.abs(o[name][fl]))
                assert e <= 1e-12, (variant, k, n, limits[k], name, e)
            assert sts[k]["unstable"] == o["unstable"]
            off += m


@pytest.mark.parametrize("graph", [0, 4])
def test_batch_step_limits_d2q9(graph):
    b = B()
    # launch shapes of the tiled batch kernel, and (small instances) the
    # LDS-resident persistent shape
    # (9, 10 and 13 take two steps per launch, 13 one tile per wave: limits 3
    # and 10 fall between the two steps of a launch, so those instances take
    # only the first)
    _limits_case(b, "d2q9", [20, 33, 47, 64, 90], [3, 10, 0, 7, -1], [0, 4, 5, 9, 10, 13], graph)
    _limits_case(b, "d2q9", [12, 20, 25, 30], [3, -1, 0, 11], [0, "lds"], graph)


def test_batch_step_limits_d1q3():
    b = B()
    # (10 and 12 take up to 16 and 64 steps per launch: the limits fall inside
    # a launch)
    _limits_case(b, "d1q3", [100, 1000, 2500, 37], [3, 10, 0, -1], [0, 1, 5, 8, 10, 12], 0)
    ctx = b.lbm_init_batch([b.make_params("d1q3", "srt", "tube", "fp64", 50, 1, 0.7)] * 2,
                           np.ones(100), np.zeros(100), None)
    try:
        with pytest.raises(b.LbmError):
            b.lbm_set_batch_steps(ctx, [1, 2, 3])  # one per instance
        b.lbm_set_batch_steps(ctx, None)
    finally:
        b.lbm_free(ctx)
    single = b.lbm_init(b.make_params("d1q3", "srt", "tube", "fp64", 50, 1, 0.7), np.ones(50), np.zeros(50), None)
    try:
        with pytest.raises(b.LbmError):
            b.lbm_set_batch_steps(single, [1])  # batches only
    finally:
        b.lbm_free(single)
