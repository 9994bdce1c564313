"""Shared helpers of the GPU tests: run the HIP library through its C ABI and
run the FP64 oracle on the same seeded inputs."""
import numpy as np

from oracle import oracle as O

COLL_ORC = {"minxent4": O.MINXENT4, "minxent2": O.MINXENT2, "srt": O.SRT, "trt": O.TRT, "mrt": O.MRT}
BC_ORC = {"periodic": O.BC_PERIODIC, "tube": O.BC_TUBE, "cavity": O.BC_CAVITY, "box": O.BC_BOX}


def B():
    from paper_1801_03863_amd import binding
    return binding


def gpu_run(lattice, collision, bc, precision, nx, ny, tau, rho, ux, uy=None, steps=1, u_lid=0.0, rho0=1.0,
            tau2=0.0, variant=None, graph=0, want_f=False, fp16_exp=0):
    b = B()
    p = b.make_params(lattice, collision, bc, precision, nx, ny, tau, tau2, u_lid, rho0, fp16_exp)
    ctx = b.lbm_init(p, rho, ux, uy)
    try:
        if variant is not None:
            b.lbm_set_variant(ctx, variant)
        if graph:
            b.lbm_set_graph_chunk(ctx, graph)
        b.lbm_step(ctx, steps)
        r, u, v = b.lbm_moments(ctx)
        st = b.lbm_status(ctx)
        f = b.lbm_get_populations(ctx, 3 if lattice == "d1q3" else 9) if want_f else None
    finally:
        b.lbm_free(ctx)
    shape = (nx,) if lattice == "d1q3" else (ny, nx)
    out = {"rho": r.reshape(shape), "ux": u.reshape(shape), "uy": v.reshape(shape), "status": st}
    if want_f:
        out["f"] = f
    return out


def orc_run(lattice, collision, bc, nx, ny, tau, rho, ux, uy=None, steps=1, u_lid=0.0, rho0=1.0, tau2=0.0,
            window=None):
    lat = O.D1Q3 if lattice == "d1q3" else O.D2Q9
    if collision in ("minxent2", "trt", "mrt") and tau2 <= 0.0:
        tau2 = (8 * tau - 1) / (2 * tau - 1)
    return O.run(lat, COLL_ORC[collision], BC_ORC[bc], nx, ny, tau, rho, ux, uy, steps=steps, tau2=tau2,
                 u_lid=u_lid, rho0=rho0, window=window)


def fluid_mask(lattice, bc, nx, ny):
    if lattice == "d1q3":
        m = np.ones(nx, bool)
        if bc != "periodic":
            m[0] = m[-1] = False
        return m
    m = np.ones((ny, nx), bool)
    if bc in ("tube", "cavity", "box"):
        m[:, 0] = m[:, -1] = False
    if bc in ("cavity", "box"):
        m[0, :] = m[-1, :] = False
    return m


def rel_err(a, b, mask):
    """(max-abs, L2) error of a against b over mask, relative to b's max-abs
    and L2 norm (absolute if b vanishes)."""
    d = (a - b)[mask]
    ref = b[mask]
    mx = np.max(np.abs(ref)) if ref.size else 0.0
    l2 = np.sqrt(np.sum(ref * ref))
    e_max = np.max(np.abs(d)) / (mx if mx > 0 else 1.0) if d.size else 0.0
    e_l2 = np.sqrt(np.sum(d * d)) / (l2 if l2 > 0 else 1.0) if d.size else 0.0
    return float(e_max), float(e_l2)


def field_errors(g, o, mask, fields=("rho", "ux", "uy")):
    return {k: rel_err(g[k], o[k], mask) for k in fields}


def smooth_fields(nx, ny, seed, amp=0.03, rho_amp=0.01):
    rng = np.random.default_rng(seed)
    y, x = np.mgrid[0:ny, 0:nx]
    px, py = rng.uniform(0, 2 * np.pi, 2)
    ux = amp * np.sin(2 * np.pi * y / ny + px) * np.cos(2 * np.pi * x / nx)
    uy = amp * np.cos(2 * np.pi * x / nx + py) * np.sin(2 * np.pi * y / ny + 0.3)
    rho = 1.0 + rho_amp * np.cos(2 * np.pi * (x / nx + 2 * y / ny))
    return rho, ux, uy
