"""Several steps per launch: the temporally blocked D2Q9 MinxEnt4 shapes (two
steps, single lattices and batches) and the D1Q3 shapes that keep 1024-node
segments in LDS for up to 16, 32, 64 or 256 steps.

Each such launch computes one step into LDS and the next from there, so its
results must be bitwise equal to two single-step launches: for every boundary
kind, for lattices smaller than, equal to and ragged against one tile, for odd
step counts (the last launch then takes one step), under graph replay, and
with the same status records (first unstable step and node, guarded count),
wherever the event falls inside a launch.  Batches add instances of uneven
size sharing one tile table, and per-instance step limits (in the full-size
step-limit tests).  D1Q3 adds periodic lattices narrower than a segment's
window, which then wraps several times.
"""

import numpy as np
import pytest

from paper_1801_03863_amd import inputs as I
from tests.gpu_helpers import B, field_errors, fluid_mask, gpu_run, orc_run, smooth_fields

pytestmark = pytest.mark.gpu

SINGLE = 0  # a single-step shape


def two_step_shapes():
    b = B()
    z = np.zeros((8, 8))
    ctx = b.lbm_init(b.make_params("d2q9", "minxent4", "cavity", "fp64", 8, 8, 0.6, 0.0, 0.1, 1.0),
                     np.ones((8, 8)), z, z)
    try:
        vs = [v for v in range(b.lbm_variant_count(ctx)) if "two steps" in b.lbm_variant_name(ctx, v)]
    finally:
        b.lbm_free(ctx)
    assert vs
    return vs


def _status(s):
    return (s["unstable"], s["first_step"], s["first_node"], s["guarded"])


@pytest.mark.parametrize("bc", ["cavity", "box", "tube", "periodic"])
@pytest.mark.parametrize("nx,ny", [(300, 131), (257, 65), (33, 17), (3, 3)])
def test_two_step_shapes_bitwise_every_boundary(bc, nx, ny):
    rho, ux, uy = smooth_fields(nx, ny, seed=nx + ny)
    for steps in (10, 7):
        ref = gpu_run("d2q9", "minxent4", bc, "fp32_newton64", nx, ny, 0.6, rho, ux, uy, steps=steps, u_lid=0.1,
                      variant=SINGLE, want_f=True)
        for v in two_step_shapes():
            g = gpu_run("d2q9", "minxent4", bc, "fp32_newton64", nx, ny, 0.6, rho, ux, uy, steps=steps, u_lid=0.1,
                        variant=v, want_f=True)
            assert np.array_equal(g["f"], ref["f"]), (v, steps)
            assert _status(g["status"]) == _status(ref["status"]), (v, steps)


@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp16dev"])
def test_two_step_shapes_bitwise_every_form(precision):
    nx, ny = 530, 97  # ragged in both directions for every tile shape
    rho, ux, uy = smooth_fields(nx, ny, seed=31)
    ref = gpu_run("d2q9", "minxent4", "cavity", precision, nx, ny, 0.58, rho, ux, uy, steps=12, u_lid=0.1,
                  variant=SINGLE, want_f=True)
    for v in two_step_shapes():
        g = gpu_run("d2q9", "minxent4", "cavity", precision, nx, ny, 0.58, rho, ux, uy, steps=12, u_lid=0.1,
                    variant=v, want_f=True)
        assert np.array_equal(g["f"], ref["f"]), v


def test_two_step_fp64_matches_oracle():
    nx, ny = 270, 70
    rho, ux, uy = smooth_fields(nx, ny, seed=32)
    o = orc_run("d2q9", "minxent4", "cavity", nx, ny, 0.6, rho, ux, uy, steps=6, u_lid=0.1)
    m = fluid_mask("d2q9", "cavity", nx, ny)
    for v in two_step_shapes():
        g = gpu_run("d2q9", "minxent4", "cavity", "fp64", nx, ny, 0.6, rho, ux, uy, steps=6, u_lid=0.1, variant=v)
        e = field_errors(g, o, m)
        assert all(x[0] <= 1e-12 for x in e.values()), (v, e)


@pytest.mark.parametrize("chunk", [1, 2, 5, 8])
def test_two_step_graph_replay_is_bitwise(chunk):
    nx, ny = 77, 64
    rho, ux, uy = smooth_fields(nx, ny, seed=33)
    v = two_step_shapes()[0]
    a = gpu_run("d2q9", "minxent4", "cavity", "fp32_newton64", nx, ny, 0.58, rho, ux, uy, steps=41, u_lid=0.1,
                variant=SINGLE, want_f=True)
    g = gpu_run("d2q9", "minxent4", "cavity", "fp32_newton64", nx, ny, 0.58, rho, ux, uy, steps=41, u_lid=0.1,
                variant=v, graph=chunk, want_f=True)
    assert np.array_equal(a["f"], g["f"])
    assert _status(a["status"]) == _status(g["status"])


# Periodic 40 x 30 lattices, MinxEnt4 at tau = 0.501, whose first unstable
# event falls on step 1, 2 or 3 (found with the oracle; seeds of
# smooth_fields with density amplitude 0.2).
UNSTABLE = [(0.38, 3, 1), (0.36, 3, 2), (0.36, 0, 3)]


@pytest.mark.parametrize("amp,seed,first", UNSTABLE)
@pytest.mark.parametrize("lead", [0, 1])
def test_two_step_status_matches_oracle_wherever_the_event_falls(amp, seed, first, lead):
    # lead = 1 takes one single step first, so that every two-step launch
    # starts on an odd step and the event moves to the other half of a launch.
    nx, ny = 40, 30
    rho, ux, uy = smooth_fields(nx, ny, seed=seed, amp=amp, rho_amp=0.2)
    o = orc_run("d2q9", "minxent4", "periodic", nx, ny, 0.501, rho, ux, uy, steps=9)
    assert o["unstable"] and o["first_step"] == first
    b = B()
    p = b.make_params("d2q9", "minxent4", "periodic", "fp64", nx, ny, 0.501, 0.0, 0.0, 1.0)
    for v in two_step_shapes():
        ctx = b.lbm_init(p, rho, ux, uy)
        try:
            b.lbm_set_variant(ctx, v)
            if lead:
                b.lbm_step(ctx, 1)
            b.lbm_step(ctx, 9 - lead)
            s = b.lbm_status(ctx)
        finally:
            b.lbm_free(ctx)
        assert s["unstable"], v
        assert (s["first_step"], s["first_node"], s["guarded"]) == (o["first_step"], o["first_node"], o["guarded"]), v


# --------------------------------------------------------------------------
# Batches
# --------------------------------------------------------------------------

def _batch(b, sizes, precision="fp32_newton64", seed=41, amp=0.05, bc="cavity"):
    rng = np.random.default_rng(seed)
    params, rs, us, vs = [], [], [], []
    for (nx, ny) in sizes:
        params.append(b.make_params("d2q9", "minxent4", bc, precision, nx, ny, 0.58, 0.0, 0.1, 1.0))
        rs.append(1.0 + 0.01 * rng.uniform(-1, 1, nx * ny))
        us.append(amp * rng.uniform(-1, 1, nx * ny))
        vs.append(amp * rng.uniform(-1, 1, nx * ny))
    return params, np.concatenate(rs), np.concatenate(us), np.concatenate(vs)


def batch_two_step_shapes(b, params, r, u, v):
    ctx = b.lbm_init_batch(params, r, u, v)
    try:
        vs = [k for k in range(b.lbm_variant_count(ctx)) if b.lbm_variant_steps(ctx, k) == 2]
    finally:
        b.lbm_free(ctx)
    assert vs
    return vs


def _run_batch(b, params, r, u, v, variant, steps, graph=0):
    ctx = b.lbm_init_batch(params, r, u, v)
    try:
        b.lbm_set_variant(ctx, variant)
        if graph:
            b.lbm_set_graph_chunk(ctx, graph)
        b.lbm_step(ctx, steps)
        f = b.lbm_get_populations(ctx, 9)
        st = [_status(s) for s in b.lbm_status_batch(ctx, len(params))]
    finally:
        b.lbm_free(ctx)
    return f, st


@pytest.mark.parametrize("precision", ["fp32_newton64", "fp64", "fp16dev"])
def test_batch_two_step_shapes_bitwise(precision):
    # widths below, equal to and ragged against 64, 128 and 256; a tall
    # instance; the smallest lattice; 320 wide, whose second tile of 192
    # columns (balanced tile widths) ends its instance 128 columns in, so the
    # column just past the edge is the first lane of a wave
    sizes = [(3, 3), (64, 17), (65, 40), (130, 33), (300, 21), (7, 150), (257, 64), (320, 9)]
    b = B()
    params, r, u, v = _batch(b, sizes, precision)
    for steps, graph in ((10, 0), (9, 0), (11, 4)):
        ref = _run_batch(b, params, r, u, v, 0, steps, graph)
        for k in batch_two_step_shapes(b, params, r, u, v):
            got = _run_batch(b, params, r, u, v, k, steps, graph)
            assert np.array_equal(got[0], ref[0]), (k, steps, graph)
            assert got[1] == ref[1], (k, steps, graph)


def test_batch_two_step_status_of_an_unstable_instance():
    # one instance starts far from equilibrium and turns unstable; the others
    # stay stable: equal status records in every shape, FP64 against the oracle
    b = B()
    sizes = [(40, 30), (70, 20), (33, 33)]
    params, r, u, v = _batch(b, sizes, "fp64", bc="periodic")
    n0 = 40 * 30
    rr, uu, vv = smooth_fields(40, 30, seed=3, amp=0.36, rho_amp=0.2)
    r[:n0], u[:n0], v[:n0] = rr.ravel(), uu.ravel(), vv.ravel()
    params[0] = b.make_params("d2q9", "minxent4", "periodic", "fp64", 40, 30, 0.501, 0.0, 0.0, 1.0)
    o = orc_run("d2q9", "minxent4", "periodic", 40, 30, 0.501, rr, uu, vv, steps=9)
    assert o["unstable"]
    ref = _run_batch(b, params, r, u, v, 0, 9)
    assert ref[1][0] == (True, o["first_step"], o["first_node"], o["guarded"])
    assert not ref[1][1][0] and not ref[1][2][0]
    for k in batch_two_step_shapes(b, params, r, u, v):
        got = _run_batch(b, params, r, u, v, k, 9)
        assert got[1] == ref[1], k


# --------------------------------------------------------------------------
# D1Q3, up to K steps per launch (K = 16, 32, 64 or 256)
# --------------------------------------------------------------------------

def d1q3_k_step_shapes(b, batch=False):
    p = b.make_params("d1q3", "srt", "tube", "fp64", 50, 1, 0.7)
    ctx = (b.lbm_init_batch([p, p], np.ones(100), np.zeros(100), None) if batch
           else b.lbm_init(p, np.ones(50), np.zeros(50), None))
    try:
        vs = [k for k in range(b.lbm_variant_count(ctx)) if b.lbm_variant_steps(ctx, k) > 2]
    finally:
        b.lbm_free(ctx)
    assert vs
    return vs


@pytest.mark.parametrize("bc", ["tube", "periodic", "cavity"])
@pytest.mark.parametrize("precision", ["fp64", "fp32_newton64", "fp16dev"])
def test_d1q3_k_step_shapes_bitwise(bc, precision):
    # lattices shorter than, equal to and ragged against a 1024-node segment;
    # periodic lattices narrower than the window; step counts below, at and
    # above each shape's steps per launch
    b = B()
    rng = np.random.default_rng(5)
    for n in (3, 100, 1024, 1025, 5000):
        rho = 1.0 + 0.3 * rng.uniform(-1, 1, n)
        ux = 0.1 * rng.uniform(-1, 1, n)
        # 256 and 300 steps on the longest lattice: the deepest window shrink
        # of the 256-step shape inside one launch, on several segments
        for steps in (1, 15, 16, 17, 70) + ((256, 300) if n == 5000 else ()):
            ref = gpu_run("d1q3", "srt", bc, precision, n, 1, 0.6, rho, ux, steps=steps, variant=0, want_f=True)
            for v in d1q3_k_step_shapes(b):
                g = gpu_run("d1q3", "srt", bc, precision, n, 1, 0.6, rho, ux, steps=steps, variant=v, want_f=True)
                assert np.array_equal(g["f"], ref["f"]), (n, steps, v)
                assert _status(g["status"]) == _status(ref["status"]), (n, steps, v)


@pytest.mark.parametrize("chunk", [5, 16, 40])
def test_d1q3_k_step_graph_replay_is_bitwise(chunk):
    n = 3000
    rho, ux = I.tube_fields(n, 2.0, 0.75)
    ref = gpu_run("d1q3", "srt", "tube", "fp32", n, 1, 0.52, rho, ux, steps=123, variant=0, want_f=True)
    for v in d1q3_k_step_shapes(B()):
        g = gpu_run("d1q3", "srt", "tube", "fp32", n, 1, 0.52, rho, ux, steps=123, variant=v, graph=chunk,
                    want_f=True)
        assert np.array_equal(g["f"], ref["f"]), (chunk, v)


@pytest.mark.parametrize("ratio,tau,first", [(4.0, 0.5001, 12), (3.0, 0.505, 127), (6.0, 0.501, 1)])
def test_d1q3_k_step_status_matches_oracle(ratio, tau, first):
    # 300-node shock tubes that turn unstable at steps 12, 127 and 1 (found
    # with the oracle): every K-step shape reports the oracle's first step and
    # node, wherever in a launch the step falls
    n = 300
    rho, ux = I.tube_fields(n, ratio * 0.75, 0.75)
    o = orc_run("d1q3", "srt", "tube", n, 1, tau, rho, ux, steps=200)
    assert o["unstable"] and o["first_step"] == first
    for v in d1q3_k_step_shapes(B()):
        g = gpu_run("d1q3", "srt", "tube", "fp64", n, 1, tau, rho, ux, steps=200, variant=v)
        assert g["status"]["unstable"], v
        assert (g["status"]["first_step"], g["status"]["first_node"]) == (o["first_step"], o["first_node"]), v


def test_d1q3_k_step_batch_bitwise():
    b = B()
    rng = np.random.default_rng(6)
    sizes = [3, 500, 1024, 1500, 4097, 64]
    params, rs, us = [], [], []
    for n in sizes:
        params.append(b.make_params("d1q3", "srt", "tube", "fp64", n, 1, 0.55, 0.0, 0.0, 1.0))
        rs.append(1.0 + 0.3 * rng.uniform(-1, 1, n))
        us.append(0.1 * rng.uniform(-1, 1, n))
    r, u = np.concatenate(rs), np.concatenate(us)

    def run(v, steps, graph=0):
        ctx = b.lbm_init_batch(params, r, u, None)
        try:
            b.lbm_set_variant(ctx, v)
            if graph:
                b.lbm_set_graph_chunk(ctx, graph)
            b.lbm_step(ctx, steps)
            return b.lbm_get_populations(ctx, 3), [_status(s) for s in b.lbm_status_batch(ctx, len(params))]
        finally:
            b.lbm_free(ctx)

    for steps, graph in ((33, 0), (64, 0), (45, 20), (300, 0), (600, 256)):
        ref = run(0, steps, graph)
        for v in d1q3_k_step_shapes(b, batch=True):
            got = run(v, steps, graph)
            assert np.array_equal(got[0], ref[0]), (v, steps, graph)
            assert got[1] == ref[1], (v, steps, graph)
