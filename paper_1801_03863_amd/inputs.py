"""Seeded synthetic inputs for the benchmark problems of MinxEnt-LBM.

This module holds no arithmetic of the method: it only draws the initial
macroscopic fields and the per-instance problem parameters.  The HIP library
and the FP64 oracle receive the same arrays from here.

Random numbers come from SplitMix64 (G. L. Steele, D. Lea, C. H. Flood, "Fast
splittable pseudorandom number generators", OOPSLA 2014) used as a
counter-based generator: draw k of stream `seed` is the SplitMix64 output
mixer applied to seed * 2^32 + (k + 1) * 0x9E3779B97F4A7C15 (mod 2^64), and
its top 53 bits give a uniform double in [0, 1).

Problem shapes follow the paper's benchmarks (Sec. IV.F-H): a density step at
the middle of a tube at rest, and a lid-driven cavity that starts at rest with
the lid moving in +x.  Viscosity and relaxation time are related by
nu = (2 tau - 1) / 6 (Sec. IV.C); a cavity of N nodes with lid speed U at
Reynolds number Re uses nu = U N / Re.
"""
from __future__ import annotations

import math

import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix_uniform(seed: int, index) -> np.ndarray:
    """Uniform doubles in [0, 1) for the given counter values of stream `seed`."""
    k = np.asarray(index, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64((seed << 32) & 0xFFFFFFFFFFFFFFFF) + (k + np.uint64(1)) * _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return (z >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


def tau_from_re(u_lid: float, n: int, re: float) -> float:
    """Relaxation time for a cavity of n nodes, lid speed u_lid, Reynolds re."""
    nu = u_lid * n / re
    return 3.0 * nu + 0.5


def cavity_fields(n: int, rho0: float = 1.0, seed: int = 1802, amp: float = 1e-6,
                  ny: int | None = None):
    """rho = rho0 (1 + xi), xi ~ U[-amp, amp) iid per node (counter = node
    index y*n + x); u = 0.  Returns (rho, ux, uy), each shape (ny, n)."""
    ny = n if ny is None else ny
    idx = np.arange(n * ny, dtype=np.uint64)
    xi = (2.0 * splitmix_uniform(seed, idx) - 1.0) * amp
    rho = (rho0 * (1.0 + xi)).reshape(ny, n)
    z = np.zeros((ny, n))
    return rho, z, z.copy()


def cavity_fields_window(n: int, x0: int, y0: int, wx: int, wy: int, rho0: float = 1.0,
                         seed: int = 1802, amp: float = 1e-6, ny: int | None = None):
    """The same fields as cavity_fields, restricted to a window."""
    ys, xs = np.meshgrid(np.arange(y0, y0 + wy), np.arange(x0, x0 + wx), indexing="ij")
    idx = (ys.astype(np.uint64) * np.uint64(n) + xs.astype(np.uint64)).reshape(-1)
    xi = (2.0 * splitmix_uniform(seed, idx) - 1.0) * amp
    rho = (rho0 * (1.0 + xi)).reshape(wy, wx)
    z = np.zeros((wy, wx))
    return rho, z, z.copy()


def vortex_fields(n: int, u_max: float, rho0: float = 1.0):
    """A lattice-filling vortex with zero velocity on the walls: stream
    function psi = -A sin^2(pi x/L) sin^2(pi y/L), L = n - 1, u_x = d psi/dy,
    u_y = -d psi/dx, with A set so that max |u| is about u_max; rho = rho0.
    A flow that moves everywhere (the cavity benchmark itself starts at
    rest)."""
    L = n - 1.0
    x = np.arange(n, dtype=np.float64)
    sx, s2x = np.sin(np.pi * x / L) ** 2, np.sin(2.0 * np.pi * x / L)
    # max over the lattice of |d/dy sin^2(pi y/L)| = pi/L at y = L/4
    amp = u_max * L / np.pi
    ux = -amp * (np.pi / L) * np.outer(s2x, sx)    # [y, x]: sin^2 in x, sin(2 .) in y
    uy = amp * (np.pi / L) * np.outer(sx, s2x)
    return np.full((n, n), rho0), ux, uy


def tube_fields(n: int, rho_left: float, rho_right: float, split: int | None = None):
    """Density step: rho_left for x < split, rho_right for x >= split; u = 0."""
    split = n // 2 if split is None else split
    rho = np.where(np.arange(n) < split, rho_left, rho_right).astype(np.float64)
    return rho, np.zeros(n)


# --------------------------------------------------------------------------
# Benchmark problem recipes.
# --------------------------------------------------------------------------

def shock_tube_800():
    """D1Q3 tube: 800 nodes (walls at both ends), rho 1.5 | 0.75 split at
    x = 400, u = 0, tau = 0.51, 400 steps."""
    rho, ux = tube_fields(800, 1.5, 0.75, 400)
    return dict(name="d1q3_tube800", lattice="d1q3", bc="tube", nx=800, ny=1, tau=0.51,
                rho=rho, ux=ux, uy=None, steps=400, u_lid=0.0, rho0=1.0)


def cavity(n: int, u_lid: float, re: float, seed: int, steps: int, rho0: float = 1.0):
    rho, ux, uy = cavity_fields(n, rho0, seed)
    return dict(name="d2q9_cavity%d" % n, lattice="d2q9", bc="cavity", nx=n, ny=n,
                tau=tau_from_re(u_lid, n, re), rho=rho, ux=ux, uy=uy, steps=steps,
                u_lid=u_lid, rho0=rho0, seed=seed, re=re)


def cavity_256():
    """256^2 cavity, lid 0.1, Re 1000, rho0 = 1 with 1e-6 noise, 20000 steps."""
    return cavity(256, 0.1, 1000.0, 1802, 20000)


def cavity_4096_params():
    """4096^2 cavity, lid 0.05, Re 5000, rho0 = 1 with 1e-6 noise (seed 1803)."""
    n, u, re = 4096, 0.05, 5000.0
    return dict(name="d2q9_cavity4096", nx=n, ny=n, u_lid=u, re=re, seed=1803,
                tau=tau_from_re(u, n, re), rho0=1.0, steps=2000)


def cavity_8192_params():
    """8192^2 cavity, lid 0.05, Re 5000 (seed 1805), 1000 steps."""
    n, u, re = 8192, 0.05, 5000.0
    return dict(name="d2q9_cavity8192", nx=n, ny=n, u_lid=u, re=re, seed=1805,
                tau=tau_from_re(u, n, re), rho0=1.0, steps=1000)


def cavity_batch(count: int = 512, seed: int = 1804, n_min: int = 32, n_max: int = 512,
                 re_min: float = 100.0, re_max: float = 10000.0, u_lid: float = 0.1):
    """Cavities with side log-uniform in [n_min, n_max] and Re uniform in
    [re_min, re_max].  Returns a list of (n, tau, re) per instance."""
    k = np.arange(count, dtype=np.uint64)
    a = splitmix_uniform(seed, 2 * k)
    b = splitmix_uniform(seed, 2 * k + np.uint64(1))
    sides = np.floor(np.exp(math.log(n_min) + a * (math.log(n_max) - math.log(n_min)))).astype(int)
    sides = np.clip(sides, n_min, n_max)
    res = re_min + b * (re_max - re_min)
    return [(int(n), tau_from_re(u_lid, int(n), float(r)), float(r)) for n, r in zip(sides, res)]


def tube_batch(count: int = 4096, seed: int = 1806, n_min: int = 1024, n_max: int = 65536,
               ratio_min: float = 1.5, ratio_max: float = 4.0, rho_right: float = 0.75,
               tau_min: float = 0.505, tau_max: float = 0.6):
    """Shock tubes with length log-uniform in [n_min, n_max], density ratio
    uniform in [ratio_min, ratio_max] (right density fixed) and tau uniform in
    [tau_min, tau_max].  Returns a list of (n, rho_left, rho_right, tau)."""
    k = np.arange(count, dtype=np.uint64)
    a = splitmix_uniform(seed, 3 * k)
    b = splitmix_uniform(seed, 3 * k + np.uint64(1))
    c = splitmix_uniform(seed, 3 * k + np.uint64(2))
    lens = np.floor(np.exp(math.log(n_min) + a * (math.log(n_max) - math.log(n_min)))).astype(int)
    lens = np.clip(lens, n_min, n_max)
    ratios = ratio_min + b * (ratio_max - ratio_min)
    taus = tau_min + c * (tau_max - tau_min)
    return [(int(n), float(r * rho_right), rho_right, float(t)) for n, r, t in zip(lens, ratios, taus)]
