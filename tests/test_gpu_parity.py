"""GPU parity: the HIP library (through its C ABI) against the FP64 oracle on
the same seeded inputs, element by element on fluid nodes.

FP64 tolerance: relative max-abs and relative L2 error of rho, u_x, u_y over
fluid nodes <= 1e-12 each.
"""
import os

import numpy as np
import pytest

from paper_1801_03863_amd import inputs as I
from tests.gpu_helpers import B, field_errors, fluid_mask, gpu_run, orc_run, smooth_fields

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

pytestmark = pytest.mark.gpu
TOL64 = 1e-12


def assert_close(g, o, mask, tol, fields=("rho", "ux", "uy"), label=""):
    errs = field_errors(g, o, mask, fields)
    print(label, {k: ("%.2e" % v[0], "%.2e" % v[1]) for k, v in errs.items()}, flush=True)
    for k, (emax, el2) in errs.items():
        assert emax <= tol and el2 <= tol, (label, k, emax, el2)
    return errs


# --------------------------------------------------------------------------
# D1Q3
# --------------------------------------------------------------------------

def test_d1q3_shock_tube_800_fp64():
    c = I.shock_tube_800()
    g = gpu_run("d1q3", "srt", "tube", "fp64", 800, 1, c["tau"], c["rho"], c["ux"], steps=c["steps"])
    o = orc_run("d1q3", "srt", "tube", 800, 1, c["tau"], c["rho"], c["ux"], steps=c["steps"])
    assert_close(g, o, fluid_mask("d1q3", "tube", 800, 1), TOL64, ("rho", "ux"), "tube800")
    assert not g["status"]["unstable"] and not o["unstable"]


def test_d1q3_shock_tube_800_fp64_in_the_benchmark_shape(tmp_path):
    # The launch shape the committed tuning cache gives this tube (the whole
    # tube in LDS for up to 256 steps per launch: 400 steps in two launches),
    # plain and from graphs of 100 steps as the benchmark times it.
    import shutil
    c = I.shock_tube_800()
    o = orc_run("d1q3", "srt", "tube", 800, 1, c["tau"], c["rho"], c["ux"], steps=c["steps"])
    cache = tmp_path / "tune_cache.txt"
    shutil.copy(os.path.join(ROOT, "paper_1801_03863_amd", "tune_cache_gfx950.txt"), cache)
    b = B()
    p = b.make_params("d1q3", "srt", "tube", "fp64", 800, 1, c["tau"], 0.0, 0.0, 1.0)
    for graph in (0, 100):
        ctx = b.lbm_init(p, c["rho"], c["ux"], None)
        try:
            b.lbm_autotune(ctx, str(cache))
            if graph:
                b.lbm_set_graph_chunk(ctx, graph)
            b.lbm_step(ctx, c["steps"])
            r, u, _ = b.lbm_moments(ctx)
            st = b.lbm_status(ctx)
        finally:
            b.lbm_free(ctx)
        g = {"rho": r, "ux": u, "uy": np.zeros_like(r), "status": st}
        assert_close(g, o, fluid_mask("d1q3", "tube", 800, 1), TOL64, ("rho", "ux"), "tube800 tuned")
        assert not st["unstable"]


@pytest.mark.parametrize("nx,bc,steps", [(3, "tube", 5), (1000, "periodic", 77), (257, "cavity", 60)])
def test_d1q3_sizes_and_boundaries(nx, bc, steps):
    rng = np.random.default_rng(nx)
    rho = 1 + 0.2 * rng.uniform(-1, 1, nx)
    ux = 0.05 * rng.uniform(-1, 1, nx)
    g = gpu_run("d1q3", "srt", bc, "fp64", nx, 1, 0.53, rho, ux, steps=steps)
    o = orc_run("d1q3", "srt", bc, nx, 1, 0.53, rho, ux, steps=steps)
    assert_close(g, o, fluid_mask("d1q3", bc, nx, 1), TOL64, ("rho", "ux"), "d1q3 %d %s" % (nx, bc))


# --------------------------------------------------------------------------
# D2Q9, every collision rule and boundary kind, ragged sizes
# --------------------------------------------------------------------------

COLLISIONS = ["minxent4", "minxent2", "srt", "trt", "mrt"]


@pytest.mark.parametrize("collision", COLLISIONS)
@pytest.mark.parametrize("bc", ["cavity", "periodic", "tube", "box"])
def test_d2q9_small_fp64(collision, bc):
    nx, ny, steps, tau = 45, 37, 30, 0.57
    seed = 10 * COLLISIONS.index(collision) + ["cavity", "periodic", "tube", "box"].index(bc)
    rho, ux, uy = smooth_fields(nx, ny, seed=seed)
    g = gpu_run("d2q9", collision, bc, "fp64", nx, ny, tau, rho, ux, uy, steps=steps, u_lid=0.08)
    o = orc_run("d2q9", collision, bc, nx, ny, tau, rho, ux, uy, steps=steps, u_lid=0.08)
    assert_close(g, o, fluid_mask("d2q9", bc, nx, ny), TOL64, label="%s/%s" % (collision, bc))
    assert g["status"]["unstable"] == o["unstable"]
    assert g["status"]["guarded"] == o["guarded"]


@pytest.mark.parametrize("nx,ny", [(3, 3), (4, 3), (3, 7), (65, 3), (300, 257)])
def test_d2q9_edge_sizes(nx, ny):
    rho, ux, uy = smooth_fields(nx, ny, seed=nx * 1000 + ny)
    g = gpu_run("d2q9", "minxent4", "cavity", "fp64", nx, ny, 0.6, rho, ux, uy, steps=12, u_lid=0.1)
    o = orc_run("d2q9", "minxent4", "cavity", nx, ny, 0.6, rho, ux, uy, steps=12, u_lid=0.1)
    assert_close(g, o, fluid_mask("d2q9", "cavity", nx, ny), TOL64, label="%dx%d" % (nx, ny))


def test_zero_steps_returns_the_initial_fields():
    nx, ny = 70, 33
    rho, ux, uy = smooth_fields(nx, ny, seed=5, amp=0.05)
    g = gpu_run("d2q9", "minxent4", "periodic", "fp64", nx, ny, 0.6, rho, ux, uy, steps=0)
    m = np.ones((ny, nx), bool)
    # u = j / rho is recovered from populations of size ~rho/9: its absolute
    # round-off is a few eps*rho, i.e. ~1e-15 relative to |u|max = 0.05.
    assert_close(g, {"rho": rho, "ux": ux, "uy": uy}, m, 1e-13, label="t=0")


def test_cavity_noise_input_matches_oracle():
    c = I.cavity(96, 0.1, 1000.0, 1802, 200)
    g = gpu_run("d2q9", "minxent4", "cavity", "fp64", 96, 96, c["tau"], c["rho"], c["ux"], c["uy"],
                steps=c["steps"], u_lid=0.1)
    o = orc_run("d2q9", "minxent4", "cavity", 96, 96, c["tau"], c["rho"], c["ux"], c["uy"], steps=c["steps"],
                u_lid=0.1)
    assert_close(g, o, fluid_mask("d2q9", "cavity", 96, 96), TOL64, label="cavity96")
    assert g["status"]["guarded"] == 0 and o["guarded"] == 0


def test_homogeneous_density_scaling_on_gpu():
    # f -> 2 f scales every population; velocities are unchanged.
    nx = 40
    rho, ux, uy = smooth_fields(nx, nx, seed=9)
    a = gpu_run("d2q9", "minxent4", "cavity", "fp64", nx, nx, 0.6, rho, ux, uy, steps=25, u_lid=0.1, rho0=1.0)
    b = gpu_run("d2q9", "minxent4", "cavity", "fp64", nx, nx, 0.6, 2 * rho, ux, uy, steps=25, u_lid=0.1, rho0=2.0)
    m = fluid_mask("d2q9", "cavity", nx, nx)
    assert np.max(np.abs(b["rho"] - 2 * a["rho"])[m]) <= 1e-14
    assert np.max(np.abs(b["ux"] - a["ux"])[m]) <= 1e-14


# --------------------------------------------------------------------------
# Status word
# --------------------------------------------------------------------------

def test_unstable_flag_and_first_step_match_oracle():
    n = 16
    z = np.zeros((n, n))
    g = gpu_run("d2q9", "srt", "cavity", "fp64", n, n, 0.5001, np.ones((n, n)), z, z, steps=300, u_lid=0.4)
    o = orc_run("d2q9", "srt", "cavity", n, n, 0.5001, np.ones((n, n)), z, z, steps=300, u_lid=0.4)
    assert o["unstable"] and g["status"]["unstable"]
    assert g["status"]["first_step"] == o["first_step"]
    assert g["status"]["first_node"] == o["first_node"] >= 0


@pytest.mark.parametrize("precision", ["fp64", "fp32_newton64", "fp32", "fp16dev"])
def test_first_unstable_node_is_the_perturbed_one(precision):
    # As in the oracle pin: only node (5, 3) starts with negative start-point
    # populations, so every form reports step 0 at node 3*nx + 5.
    nx, ny = 300, 70  # several tiles per row, several rows per launch shape
    rho = np.ones((ny, nx))
    ux = np.zeros((ny, nx))
    ux[3, 5] = 0.9
    z = np.zeros((ny, nx))
    g = gpu_run("d2q9", "minxent4", "periodic", precision, nx, ny, 0.8, rho, ux, z, steps=3)
    assert g["status"]["unstable"] and g["status"]["first_step"] == 0
    assert g["status"]["first_node"] == 3 * nx + 5


def test_guarded_nodes_counted_like_oracle():
    # A strongly perturbed start leaves p > 0 at some nodes: both count them.
    n = 24
    rng = np.random.default_rng(3)
    rho = 1 + 0.6 * rng.uniform(-1, 1, (n, n))
    ux = 0.35 * rng.uniform(-1, 1, (n, n))
    uy = 0.35 * rng.uniform(-1, 1, (n, n))
    g = gpu_run("d2q9", "minxent4", "periodic", "fp64", n, n, 0.52, rho, ux, uy, steps=3)
    o = orc_run("d2q9", "minxent4", "periodic", n, n, 0.52, rho, ux, uy, steps=3)
    assert g["status"]["guarded"] == o["guarded"]
    assert g["status"]["unstable"] == o["unstable"]


# --------------------------------------------------------------------------
# Launch forms give bitwise identical results
# --------------------------------------------------------------------------

@pytest.mark.parametrize("precision", ["fp64", "fp32_newton64", "fp32", "fp16dev"])
def test_launch_shapes_are_bitwise_identical(precision):
    nx, ny = 300, 131
    rho, ux, uy = smooth_fields(nx, ny, seed=11)
    b = B()
    ref = None
    p = b.make_params("d2q9", "minxent4", "cavity", precision, nx, ny, 0.6, 0.0, 0.1, 1.0)
    ctx = b.lbm_init(p, rho, ux, uy)
    nv = b.lbm_variant_count(ctx)
    b.lbm_free(ctx)
    for v in range(nv):
        g = gpu_run("d2q9", "minxent4", "cavity", precision, nx, ny, 0.6, rho, ux, uy, steps=9, u_lid=0.1,
                    variant=v, want_f=True)
        if ref is None:
            ref = g["f"]
        else:
            assert np.array_equal(g["f"], ref), v


@pytest.mark.parametrize("nx,ny", [(700, 70), (2048, 40)])
def test_launch_shapes_interior_tiles_are_bitwise_identical(nx, ny):
    # 700 columns: three tiles of 256, so the middle tile takes the interior
    # neighbour offsets while the two edge tiles apply the wall rule.  2048
    # columns: every tile but the first and last of a row is interior, for
    # every block width.
    rho, ux, uy = smooth_fields(nx, ny, seed=21)
    b = B()
    ctx = b.lbm_init(b.make_params("d2q9", "minxent4", "cavity", "fp32_newton64", nx, ny, 0.6, 0.0, 0.1, 1.0),
                     rho, ux, uy)
    nv = b.lbm_variant_count(ctx)
    b.lbm_free(ctx)
    ref = None
    for v in range(nv):
        g = gpu_run("d2q9", "minxent4", "cavity", "fp32_newton64", nx, ny, 0.6, rho, ux, uy, steps=7, u_lid=0.1,
                    variant=v, want_f=True)
        ref = g["f"] if ref is None else ref
        assert np.array_equal(g["f"], ref), v


def test_tall_lattice_one_dimensional_grid_matches_oracle():
    # 70001 rows: one-row tiles exceed the grid's y limit, so those launch
    # shapes fall back to a one-dimensional grid of tiles.
    nx, ny = 6, 70001
    rho, ux, uy = smooth_fields(nx, ny, seed=22)
    b = B()
    ctx = b.lbm_init(b.make_params("d2q9", "minxent4", "cavity", "fp64", nx, ny, 0.6, 0.0, 0.05, 1.0),
                     rho, ux, uy)
    nv = b.lbm_variant_count(ctx)
    b.lbm_free(ctx)
    ref = None
    for v in range(nv):
        g = gpu_run("d2q9", "minxent4", "cavity", "fp64", nx, ny, 0.6, rho, ux, uy, steps=3, u_lid=0.05,
                    variant=v, want_f=True)
        if ref is None:
            ref = g
        else:
            assert np.array_equal(g["f"], ref["f"]), v
    o = orc_run("d2q9", "minxent4", "cavity", nx, ny, 0.6, rho, ux, uy, steps=3, u_lid=0.05)
    m = fluid_mask("d2q9", "cavity", nx, ny)
    e = field_errors(ref, o, m)
    assert all(v[0] <= 1e-12 for v in e.values()), e


def test_d1q3_launch_shapes_are_bitwise_identical():
    nx = 5000
    rho, ux = I.tube_fields(nx, 2.0, 0.75)
    ref = None
    b = B()
    ctx = b.lbm_init(b.make_params("d1q3", "srt", "tube", "fp64", nx, 1, 0.52), rho, ux)
    nv = b.lbm_variant_count(ctx)
    b.lbm_free(ctx)
    assert nv >= 4
    for v in range(nv):
        g = gpu_run("d1q3", "srt", "tube", "fp64", nx, 1, 0.52, rho, ux, steps=33, variant=v, want_f=True)
        ref = g["f"] if ref is None else ref
        assert np.array_equal(g["f"], ref), v


@pytest.mark.parametrize("chunk", [1, 7, 10])
def test_graph_replay_is_bitwise_identical(chunk):
    nx, ny = 77, 64
    rho, ux, uy = smooth_fields(nx, ny, seed=12)
    a = gpu_run("d2q9", "minxent4", "cavity", "fp64", nx, ny, 0.58, rho, ux, uy, steps=41, u_lid=0.1,
                want_f=True)
    g = gpu_run("d2q9", "minxent4", "cavity", "fp64", nx, ny, 0.58, rho, ux, uy, steps=41, u_lid=0.1,
                graph=chunk, want_f=True)
    assert np.array_equal(a["f"], g["f"])


def test_graph_replays_repeated_with_eager_work_between():
    nx, ny = 50, 40
    rho, ux, uy = smooth_fields(nx, ny, seed=13)
    b = B()
    p = b.make_params("d2q9", "minxent4", "cavity", "fp64", nx, ny, 0.6, 0.0, 0.1, 1.0)
    c1 = b.lbm_init(p, rho, ux, uy)
    c2 = b.lbm_init(p, rho, ux, uy)
    try:
        b.lbm_set_graph_chunk(c2, 6)
        for k in range(5):
            b.lbm_step(c1, 6)
            b.lbm_step(c2, 6)
            assert np.array_equal(b.lbm_get_populations(c1, 9), b.lbm_get_populations(c2, 9)), k
            b.lbm_step(c1, 1)  # eager step between replays
            b.lbm_step(c2, 1)
        assert b.lbm_info(c2)["steps_done"] == 35
    finally:
        b.lbm_free(c1)
        b.lbm_free(c2)


def test_checkpoint_restore_is_bitwise():
    nx, ny = 64, 48
    rho, ux, uy = smooth_fields(nx, ny, seed=14)
    b = B()
    p = b.make_params("d2q9", "minxent4", "cavity", "fp64", nx, ny, 0.6, 0.0, 0.1, 1.0)
    c1 = b.lbm_init(p, rho, ux, uy)
    c2 = b.lbm_init(p, np.ones(nx * ny), np.zeros(nx * ny), np.zeros(nx * ny))
    try:
        b.lbm_step(c1, 10)
        b.lbm_set_populations(c2, b.lbm_get_populations(c1, 9))
        b.lbm_step(c1, 15)
        b.lbm_step(c2, 15)
        assert np.array_equal(b.lbm_get_populations(c1, 9), b.lbm_get_populations(c2, 9))
    finally:
        b.lbm_free(c1)
        b.lbm_free(c2)


def test_autotune_keeps_the_state_and_caches(tmp_path):
    nx, ny = 200, 150
    rho, ux, uy = smooth_fields(nx, ny, seed=15)
    b = B()
    p = b.make_params("d2q9", "minxent4", "cavity", "fp64", nx, ny, 0.6, 0.0, 0.1, 1.0)
    c1 = b.lbm_init(p, rho, ux, uy)
    c2 = b.lbm_init(p, rho, ux, uy)
    cache = str(tmp_path / "tune.txt")
    try:
        b.lbm_step(c1, 5)
        b.lbm_step(c2, 5)
        v = b.lbm_autotune(c2, cache)
        assert 0 <= v < b.lbm_variant_count(c2)
        assert b.lbm_autotune(c2, cache) == v  # second call reads the cache
        b.lbm_step(c1, 5)
        b.lbm_step(c2, 5)
        assert np.array_equal(b.lbm_get_populations(c1, 9), b.lbm_get_populations(c2, 9))
        assert not b.lbm_status(c2)["unstable"]
    finally:
        b.lbm_free(c1)
        b.lbm_free(c2)


def test_caller_workspace_and_stream():
    import torch
    nx, ny = 60, 50
    rho, ux, uy = smooth_fields(nx, ny, seed=16)
    b = B()
    p = b.make_params("d2q9", "minxent4", "cavity", "fp64", nx, ny, 0.6, 0.0, 0.1, 1.0)
    ws = torch.empty(b.lbm_workspace_bytes(p), dtype=torch.uint8, device="cuda")
    s = torch.cuda.Stream()
    ctx = b.lbm_init(p, rho, ux, uy, workspace=ws, stream=s)
    try:
        b.lbm_step(ctx, 20)
        r, u, v = b.lbm_moments(ctx)
    finally:
        b.lbm_free(ctx)
    o = orc_run("d2q9", "minxent4", "cavity", nx, ny, 0.6, rho, ux, uy, steps=20, u_lid=0.1)
    g = {"rho": r.reshape(ny, nx), "ux": u.reshape(ny, nx), "uy": v.reshape(ny, nx)}
    assert_close(g, o, fluid_mask("d2q9", "cavity", nx, ny), TOL64, label="caller ws")
    small = torch.empty(16, dtype=torch.uint8, device="cuda")
    with pytest.raises(b.LbmError):
        b.lbm_init(p, rho, ux, uy, workspace=small)
    # A workspace that is not 256-byte aligned is rejected before any device work.
    big = torch.empty(b.lbm_workspace_bytes(p) + 256, dtype=torch.uint8, device="cuda")
    with pytest.raises(b.LbmError) as ei:
        b.lbm_init(p, rho, ux, uy, workspace=big[8:])
    assert ei.value.code == b.LBM_EINVAL


def test_argument_errors_leave_the_context_usable():
    nx, ny = 40, 30
    rho, ux, uy = smooth_fields(nx, ny, seed=23)
    b = B()
    p = b.make_params("d2q9", "minxent4", "cavity", "fp64", nx, ny, 0.6, 0.0, 0.1, 1.0)
    ctx = b.lbm_init(p, rho, ux, uy)
    try:
        nv = b.lbm_variant_count(ctx)
        for call in (lambda: b.lbm_set_variant(ctx, nv), lambda: b.lbm_set_variant(ctx, -1),
                     lambda: b.lbm_step(ctx, -1), lambda: b.lbm_set_graph_chunk(ctx, -1)):
            with pytest.raises(b.LbmError) as ei:
                call()
            assert ei.value.code == b.LBM_EINVAL
        b.lbm_step(ctx, 12)
        r, u, v = b.lbm_moments(ctx)
    finally:
        b.lbm_free(ctx)
    o = orc_run("d2q9", "minxent4", "cavity", nx, ny, 0.6, rho, ux, uy, steps=12, u_lid=0.1)
    g = {"rho": r.reshape(ny, nx), "ux": u.reshape(ny, nx), "uy": v.reshape(ny, nx)}
    assert_close(g, o, fluid_mask("d2q9", "cavity", nx, ny), TOL64, label="after errors")


@pytest.mark.parametrize("nbytes", [0, 16, 4096, 16384 + 48, (1 << 22) + 16 * 1023, 3 << 20])
def test_copy_kernel(nbytes):
    """Whole blocks, a ragged last block and sizes below one block; the bytes
    after the copied range keep their value."""
    import torch
    b = B()
    n = nbytes // 4
    src = torch.arange(n + 64, dtype=torch.int32, device="cuda")
    dst = torch.full_like(src, -7)
    b.lbm_copy_kernel(dst, src, nbytes)
    torch.cuda.synchronize()
    assert torch.equal(src[:n], dst[:n])
    assert bool((dst[n:] == -7).all())


# --------------------------------------------------------------------------
# Plane pad (single lattices with planes of at least 1 MiB)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("nx", [1024, 1000])
def test_plane_pad_moves_the_state_bitwise(nx):
    # nx x 300 FP32: 1.2 MB planes, so the context takes a pad.  Pads
    # changed mid-run (with graph replay around them) leave the trajectory
    # bitwise equal to a run that keeps the default pad.  1000 columns are
    # stored at a pitch of 1024 (whole 128-byte lines), and the move copies
    # the padded rows.
    ny = 300
    pitch = (nx + 31) // 32 * 32
    rho, ux, uy = smooth_fields(nx, ny, seed=31)
    b = B()
    p = b.make_params("d2q9", "minxent4", "cavity", "fp32", nx, ny, 0.6, 0.0, 0.1, 1.0)
    ref = b.lbm_init(p, rho, ux, uy)
    c = b.lbm_init(p, rho, ux, uy)
    try:
        base = (pitch * ny + 63) // 64 * 64
        assert b.lbm_get_layout(c) == (base + 2048 // 4, 2048)
        b.lbm_step(ref, 25)
        b.lbm_set_graph_chunk(c, 4)
        b.lbm_step(c, 7)
        for pad in (0, 8192, 256, 4096):
            b.lbm_set_plane_pad(c, pad)
            assert b.lbm_get_layout(c) == (base + pad // 4, pad)
            b.lbm_step(c, 6 if pad != 4096 else 0)
        assert b.lbm_info(c)["steps_done"] == 25
        assert np.array_equal(b.lbm_get_populations(ref, 9), b.lbm_get_populations(c, 9))
        r1, r2 = b.lbm_status(ref), b.lbm_status(c)
        assert r1 == r2 and not r1["unstable"]
    finally:
        b.lbm_free(ref)
        b.lbm_free(c)


def test_plane_pad_fp64_against_oracle():
    # The FP64 path with a non-default pad still matches the oracle.
    nx, ny = 520, 260  # 1.08 MB planes
    rho, ux, uy = smooth_fields(nx, ny, seed=32)
    b = B()
    p = b.make_params("d2q9", "minxent4", "cavity", "fp64", nx, ny, 0.6, 0.0, 0.1, 1.0)
    ctx = b.lbm_init(p, rho, ux, uy)
    try:
        b.lbm_set_plane_pad(ctx, 1024)
        b.lbm_step(ctx, 12)
        r, u, v = b.lbm_moments(ctx)
    finally:
        b.lbm_free(ctx)
    o = orc_run("d2q9", "minxent4", "cavity", nx, ny, 0.6, rho, ux, uy, steps=12, u_lid=0.1)
    g = {"rho": r.reshape(ny, nx), "ux": u.reshape(ny, nx), "uy": v.reshape(ny, nx)}
    assert_close(g, o, fluid_mask("d2q9", "cavity", nx, ny), TOL64, label="pad 1024")


def test_plane_pad_argument_errors():
    b = B()
    big = b.make_params("d2q9", "minxent4", "cavity", "fp32", 1024, 300, 0.6, 0.0, 0.1, 1.0)
    small = b.make_params("d2q9", "minxent4", "cavity", "fp32", 45, 37, 0.6, 0.0, 0.1, 1.0)
    r, u, v = smooth_fields(1024, 300, seed=33)
    c = b.lbm_init(big, r, u, v)
    rs, us, vs = smooth_fields(45, 37, seed=34)
    s = b.lbm_init(small, rs, us, vs)
    bt = b.lbm_init_batch([big], r, u, v)
    try:
        for bad in (-256, 100, 8448):
            with pytest.raises(b.LbmError) as ei:
                b.lbm_set_plane_pad(c, bad)
            assert ei.value.code == b.LBM_EINVAL
        for ctx in (s, bt):
            with pytest.raises(b.LbmError):
                b.lbm_set_plane_pad(ctx, 0)
            assert b.lbm_get_layout(ctx)[1] == -1
        assert b.lbm_get_layout(c)[1] == 2048  # errors left the pad alone
        b.lbm_step(c, 3)
        assert not b.lbm_status(c)["unstable"]
    finally:
        b.lbm_free(c)
        b.lbm_free(s)
        b.lbm_free(bt)


def test_autotune_tunes_the_plane_pad_and_keeps_the_state(tmp_path):
    nx, ny = 1024, 300
    rho, ux, uy = smooth_fields(nx, ny, seed=35)
    b = B()
    p = b.make_params("d2q9", "minxent4", "cavity", "fp32_newton64", nx, ny, 0.6, 0.0, 0.1, 1.0)
    c1 = b.lbm_init(p, rho, ux, uy)
    c2 = b.lbm_init(p, rho, ux, uy)
    c3 = b.lbm_init(p, rho, ux, uy)
    cache = str(tmp_path / "tune.txt")
    try:
        for c in (c1, c2, c3):
            b.lbm_step(c, 5)
        v = b.lbm_autotune(c2, cache)
        pad = b.lbm_get_layout(c2)[1]
        assert pad in (0, 1024, 2048, 4096, 8192)
        fields = open(cache).read().split()
        assert len(fields) == 3 and int(fields[1]) == v and int(fields[2]) == pad
        assert b.lbm_autotune(c3, cache) == v and b.lbm_get_layout(c3)[1] == pad  # from the cache
        for c in (c1, c2, c3):
            b.lbm_step(c, 5)
        f1 = b.lbm_get_populations(c1, 9)
        assert np.array_equal(f1, b.lbm_get_populations(c2, 9))
        assert np.array_equal(f1, b.lbm_get_populations(c3, 9))
    finally:
        for c in (c1, c2, c3):
            b.lbm_free(c)
