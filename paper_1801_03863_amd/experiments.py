"""The paper's benchmark studies, driven through the C ABI (Sec. IV.F-H).

- lid-driven cavity accuracy study (Sec. IV.H, Table II): run to steady
  state, stream function by Simpson's rule, vortex centres and strengths;
- lid-driven cavity stability study (Sec. IV.G): largest stable lid speed
  per relaxation time, many cavities in one batched context;
- one-dimensional shock tube in the paper's D2Q9 form (Sec. IV.F).

Every time step runs in the HIP library; this module only prepares inputs
and post-processes fields read back with lbm_moments.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.integrate

from . import binding as B


# --------------------------------------------------------------------------
# Sec. IV.H: accuracy study
# --------------------------------------------------------------------------

def stream_function(uy: np.ndarray) -> np.ndarray:
    """psi(x, y) = -int_0^x u_y dx' along each row (lattice units, dx = 1),
    composite Simpson's rule on the uniform lattice, starting at the left
    wall column, where u_y = 0 (the wall nodes' own moments are not fluid
    velocities and are replaced by zero)."""
    v = np.array(uy, dtype=np.float64, copy=True)
    v[:, 0] = 0.0
    v[:, -1] = 0.0
    return -scipy.integrate.cumulative_simpson(v, dx=1.0, axis=1, initial=0.0)


def vortex_summary(rho, ux, uy, u_lid, rho0):
    """Centres and strengths of the main, lower-right and lower-left vortices.

    psi_hat = psi / (U L) with L = n - 2, the distance between the half-way
    bounce-back walls.  Positions use the normalisation that reproduces the
    printed grid positions of Table II: x = (i - 1/2)/(n - 2),
    y = (j - 1/2)/(n - 1).  Vorticity omega = dv/dx - du/dy (central
    differences), omega_hat = omega L / U; pressure deviation from the mean,
    dpi_hat = (rho - mean rho) / (3 rho0 U^2).  Those last two formulas are
    not given in the paper (it cites another work for them)."""
    n = rho.shape[0]
    L = n - 2
    psi = stream_function(uy) / (u_lid * L)
    dvdx = np.gradient(uy, axis=1)
    dudy = np.gradient(ux, axis=0)
    omega = (dvdx - dudy) * L / u_lid
    fl = np.zeros_like(rho, bool)
    fl[1:-1, 1:-1] = True
    dpi = (rho - rho[fl].mean()) / (3.0 * rho0 * u_lid * u_lid)
    j, i = np.mgrid[0:n, 0:n]
    xs = (i - 0.5) / (n - 2)
    ys = (j - 0.5) / (n - 1)

    def pick(mask, fn):
        vals = np.where(mask & fl, psi, np.nan)
        k = fn(vals)
        jj, ii = np.unravel_index(k, psi.shape)
        return {"psi_hat": float(psi[jj, ii]), "i": int(ii), "j": int(jj), "x": float(xs[jj, ii]),
                "y": float(ys[jj, ii]), "dpi_hat": float(dpi[jj, ii]), "omega_hat": float(omega[jj, ii])}

    return {
        "main": pick(np.ones_like(fl), np.nanargmin),
        "lower_right": pick((xs > 0.6) & (ys < 0.4), np.nanargmax),
        "lower_left": pick((xs < 0.4) & (ys < 0.4), np.nanargmax),
    }


def run_cavity_steady(n=257, re=1000.0, u_lid=0.1, rho0=2.7, precision="fp64", check_every=1000, tol=1e-5,
                      max_steps=400000, length=None, min_steps=0, trace=None):
    """Lid-driven cavity from rest (Sec. IV.H): run until psi_hat_min changes
    by less than tol between checks.  nu = U L / Re with L = n (node count)
    unless `length` is given; tau = 3 nu + 1/2 (Sec. IV.C)."""
    L = n if length is None else length
    tau = 3.0 * u_lid * L / re + 0.5
    p = B.make_params("d2q9", "minxent4", "cavity", precision, n, n, tau, 0.0, u_lid, rho0)
    rho = np.full(n * n, rho0)
    z = np.zeros(n * n)
    ctx = B.lbm_init(p, rho, z, z)
    last = None
    steps = 0
    try:
        B.lbm_set_graph_chunk(ctx, min(check_every, 500))
        while steps < max_steps:
            B.lbm_step(ctx, check_every)
            steps += check_every
            r, u, v = (a.reshape(n, n) for a in B.lbm_moments(ctx))
            psi_min = float(np.min(stream_function(v)[1:-1, 1:-1])) / (u_lid * (n - 2))
            if trace is not None:
                trace.append((steps, psi_min))
            if last is not None and abs(psi_min - last) < tol and steps >= min_steps:
                break
            last = psi_min
        st = B.lbm_status(ctx)
    finally:
        B.lbm_free(ctx)
    return {"steps": steps, "tau": tau, "status": st, "rho": r, "ux": u, "uy": v,
            "summary": vortex_summary(r, u, v, u_lid, rho0)}


# --------------------------------------------------------------------------
# Sec. IV.G: stability study
# --------------------------------------------------------------------------

def tau2_of(tau, rule="printed"):
    """The second relaxation time of the heat-flux moments (MinxEnt2, TRT,
    MRT).  'printed': (8 tau - 1)/(2 tau - 1) as Sec. IV.C prints it;
    'luo': (8 tau - 1)/(8 (2 tau - 1)), the rate 8(2 - s)/(8 - s) with
    s = 1/tau of the MRT literature the paper cites for Table III, a factor 8
    apart from the printed one."""
    if rule == "printed":
        return (8.0 * tau - 1.0) / (2.0 * tau - 1.0)
    if rule == "luo":
        return (8.0 * tau - 1.0) / (8.0 * (2.0 * tau - 1.0))
    raise ValueError(rule)


def stability_sweep(collision, inv_taus, lids, n=17, rho0=2.7, steps=1000, precision="fp64", tau2_rule="printed"):
    """Run one n x n cavity per (1/tau, lid speed) pair, all in one batched
    context, for `steps` steps from rest at density rho0.  A run is stable if
    every post-collision population stayed finite and non-negative (the
    criterion of Sec. IV.G).  tau2 follows `tau2_rule` (see tau2_of).
    Returns (stable[len(inv_taus), len(lids)], first_step array, max stable
    lid speed per 1/tau scanning downwards)."""
    params = []
    for it in inv_taus:
        for u in lids:
            tau = 1.0 / it
            params.append(B.make_params("d2q9", collision, "cavity", precision, n, n, tau, tau2_of(tau, tau2_rule),
                                        u, rho0))
    m = len(params)
    rho = np.full(m * n * n, rho0)
    z = np.zeros(m * n * n)
    ctx = B.lbm_init_batch(params, rho, z, z)
    try:
        # All lattices are tiny: run every step in one launch with the
        # lattices resident in LDS when the device allows it.
        names = [B.lbm_variant_name(ctx, v) for v in range(B.lbm_variant_count(ctx))]
        lds = [v for v, nm in enumerate(names) if "LDS" in nm]
        if lds:
            B.lbm_set_variant(ctx, lds[0])
        else:
            B.lbm_set_graph_chunk(ctx, 100)
        B.lbm_step(ctx, steps)
        st = B.lbm_status_batch(ctx, m)
    finally:
        B.lbm_free(ctx)
    stable = np.array([not s["unstable"] for s in st]).reshape(len(inv_taus), len(lids))
    first = np.array([s["first_step"] for s in st]).reshape(len(inv_taus), len(lids))
    order = np.argsort(lids)[::-1]
    max_stable = []
    for row in stable:
        best = 0.0
        for k in order:  # decreasing lid speed: the first stable one
            if row[k]:
                best = float(lids[k])
                break
        max_stable.append(best)
    return stable, first, np.array(max_stable)


# --------------------------------------------------------------------------
# Sec. IV.F: shock tube, paper form
# --------------------------------------------------------------------------

def shock_tube_d2q9(collision, nx=800, ny=4, rho_left=1.0, rho_right=0.5, tau=0.5 + 1e-9, steps=400,
                    precision="fp64"):
    """D2Q9 on an nx x ny periodic lattice with data constant in y: density
    rho_left on x < nx/2 and rho_right elsewhere, fluid at rest.  Returns the
    density and velocity profiles (row 0) and the status."""
    x = np.arange(nx)
    rho = np.tile(np.where(x < nx // 2, rho_left, rho_right).astype(np.float64), (ny, 1))
    z = np.zeros((ny, nx))
    p = B.make_params("d2q9", collision, "periodic", precision, nx, ny, tau, 0.0, 0.0, 1.0)
    ctx = B.lbm_init(p, rho, z, z)
    try:
        B.lbm_step(ctx, steps)
        r, u, v = (a.reshape(ny, nx) for a in B.lbm_moments(ctx))
        st = B.lbm_status(ctx)
    finally:
        B.lbm_free(ctx)
    return {"rho": r[0], "ux": u[0], "status": st, "rows_equal": bool(np.all(r == r[0]))}


def total_variation(a):
    return float(np.sum(np.abs(np.diff(a))))
