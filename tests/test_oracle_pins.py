"""Pins of the FP64 oracle against what the paper and mathematics fix.

Each test checks the oracle against something other than itself: the
printed tables (tests/golden/paper_tables.json), closed forms, invariants of
the collision and of the whole run, an independent arbitrary-precision
minimiser (mpmath), a library optimiser (scipy), the viscosity relation of
Sec. IV.C and the exact isothermal Riemann solution.
"""
from fractions import Fraction

import mpmath
import numpy as np
import pytest
import scipy.optimize

EPS = np.finfo(np.float64).eps
NORM2 = np.array([9, 36, 36, 6, 12, 6, 12, 4, 4], dtype=float)


# --------------------------------------------------------------------------
# Helpers built from the printed tables only (never from the oracle).
# --------------------------------------------------------------------------

def printed_T(golden):
    return np.array(golden["moment_matrix_T"]["rows"], dtype=float)


def printed_columns(golden):
    """Velocity of each column of the printed T: rows 4 and 6 are j_x, j_y."""
    T = printed_T(golden)
    return T[3].astype(int), T[5].astype(int)


def printed_weights_by_velocity(golden):
    t = golden["table_I_d2q9"]
    return {tuple(v): Fraction(n, d) for v, n, d in zip(t["velocities"], t["weights_num"], t["weights_den"])}


def printed_weights_in_T_order(golden):
    wmap = printed_weights_by_velocity(golden)
    vx, vy = printed_columns(golden)
    return np.array([float(wmap[(int(a), int(b))]) for a, b in zip(vx, vy)])


def random_nodes(rng, n, umax=0.1, noise=0.05):
    """Near-equilibrium populations: polynomial equilibrium of a random
    (rho, u) times (1 + noise*U[-1,1]) per population, built from Table I."""
    out = []
    for _ in range(n):
        rho = rng.uniform(0.5, 3.0)
        ux, uy = rng.uniform(-umax, umax, 2)
        out.append((rho, ux, uy))
    return out


# --------------------------------------------------------------------------
# Lattice constants
# --------------------------------------------------------------------------

def test_T_is_the_printed_matrix(orc, golden):
    T, _, _, _, _ = orc.constants()
    assert np.array_equal(T, printed_T(golden))


def test_oracle_velocity_order_matches_T_columns(orc, golden):
    # Each row of T is a polynomial of its column's velocity; this fixes the
    # order of the velocities (rest first, unlike Table I).
    T, _, _, vx, vy = orc.constants()
    pvx, pvy = printed_columns(golden)
    assert np.array_equal(vx, pvx) and np.array_equal(vy, pvy)
    v2 = vx ** 2 + vy ** 2
    rows = np.array([np.ones(9), -4 + 3 * v2, 4 - 10.5 * v2 + 4.5 * v2 ** 2, vx, (-5 + 3 * v2) * vx,
                     vy, (-5 + 3 * v2) * vy, vx ** 2 - vy ** 2, vx * vy])
    assert np.array_equal(T, rows)
    # The set of velocities is Table I's.
    tab = {tuple(v) for v in golden["table_I_d2q9"]["velocities"]}
    assert {(int(a), int(b)) for a, b in zip(vx, vy)} == tab


def test_weights_are_table_I_and_a_tensor_product(orc, golden):
    _, _, W, vx, vy = orc.constants()
    wmap = printed_weights_by_velocity(golden)
    for a in range(9):
        assert W[a] == float(wmap[(int(vx[a]), int(vy[a]))])
    w1 = {0: Fraction(2, 3), 1: Fraction(1, 6), -1: Fraction(1, 6)}
    for a in range(9):
        assert W[a] == float(w1[int(vx[a])] * w1[int(vy[a])])
    assert sum(wmap.values()) == 1


def test_T_rows_orthogonal_and_inverse_closed_form(orc):
    T, Ti, _, _, _ = orc.constants()
    assert np.array_equal(T @ T.T, np.diag(NORM2))
    closed = T.T / NORM2[None, :]
    assert np.max(np.abs(Ti - closed)) <= 1e-17
    assert np.max(np.abs(Ti @ T - np.eye(9))) <= 4 * EPS


def test_equilibrium_moments_closed_form(orc, golden):
    T = printed_T(golden)
    rng = np.random.default_rng(1)
    for _ in range(200):
        rho = rng.uniform(0.3, 3.0)
        ux, uy = rng.uniform(-0.3, 0.3, 2)
        feq = orc.feq_d2q9(rho, ux, uy)
        uu = ux * ux + uy * uy
        want = rho * np.array([1, -2 + 3 * uu, 1 - 3 * uu, ux, -ux, uy, -uy, ux * ux - uy * uy, ux * uy])
        assert np.max(np.abs(T @ feq - want)) <= 16 * EPS * rho
        # Pressure tensor: sum f v v = rho (I/3 + u u), i.e. pi = rho/3 (Sec. IV.C).
        vx, vy = printed_columns(golden)
        assert abs(feq @ (vx * vx) - rho * (1 / 3 + ux * ux)) <= 16 * EPS * rho
        assert abs(feq @ (vx * vy) - rho * ux * uy) <= 16 * EPS * rho


# --------------------------------------------------------------------------
# Per-node collision invariants
# --------------------------------------------------------------------------

def perturbed(orc, rng, rho, ux, uy, noise):
    return orc.feq_d2q9(rho, ux, uy) * (1 + noise * rng.uniform(-1, 1, 9))


def test_collision_conserves_mass_and_momentum(orc, golden):
    vx, vy = printed_columns(golden)
    rng = np.random.default_rng(2)
    for rho, ux, uy in random_nodes(rng, 2000):
        f = perturbed(orc, rng, rho, ux, uy, 0.05)
        tau = rng.uniform(0.5005, 1.5)
        g, guarded = orc.collide_minxent(f, tau)
        assert not guarded
        scale = np.abs(f).sum()
        assert abs(g.sum() - f.sum()) <= 8 * EPS * scale
        assert abs(g @ vx - f @ vx) <= 8 * EPS * scale
        assert abs(g @ vy - f @ vy) <= 8 * EPS * scale


def test_stress_constraints_hold_after_the_step(orc, golden):
    T = printed_T(golden)
    rng = np.random.default_rng(3)
    for rho, ux, uy in random_nodes(rng, 1000):
        f = perturbed(orc, rng, rho, ux, uy, 0.05)
        tau = rng.uniform(0.5005, 1.5)
        g, _ = orc.collide_minxent(f, tau)
        p = f / f.sum()
        u_x, u_y = T[3] @ p, T[5] @ p
        # Constraints C8, C9: stress moments relaxed by 1/tau toward the
        # equilibrium values u_x^2 - u_y^2 and u_x u_y.
        c8 = T[7] @ p + (u_x * u_x - u_y * u_y - T[7] @ p) / tau
        c9 = T[8] @ p + (u_x * u_y - T[8] @ p) / tau
        q = g / g.sum()
        assert abs(T[7] @ q - c8) <= 16 * EPS
        assert abs(T[8] @ q - c9) <= 16 * EPS


def test_start_point_free_moments_are_equilibrium(orc, golden):
    T = printed_T(golden)
    rng = np.random.default_rng(4)
    for rho, ux, uy in random_nodes(rng, 300):
        f = perturbed(orc, rng, rho, ux, uy, 0.05)
        p0 = orc.minxent_start(f, 0.7) / f.sum()
        p = f / f.sum()
        u_x, u_y = T[3] @ p, T[5] @ p
        uu = u_x ** 2 + u_y ** 2
        M = T @ p0
        assert abs(M[1] - (-2 + 3 * uu)) <= 32 * EPS
        assert abs(M[2] - (1 - 3 * uu)) <= 32 * EPS
        assert abs(M[4] + u_x) <= 32 * EPS
        assert abs(M[6] + u_y) <= 32 * EPS


def test_rest_equilibrium_is_a_fixed_point(orc):
    _, _, W, _, _ = orc.constants()
    for rho in (1.0, 2.7, 0.3):
        f = rho * W
        g, _ = orc.collide_minxent(f, 0.57)
        assert np.max(np.abs(g - f)) <= 2 * EPS * rho


def test_moving_equilibrium_is_fixed_only_to_third_order(orc):
    # ln(f_eq/W) has cubic terms outside the span of the constrained rows, so
    # the single step moves a moving polynomial equilibrium by O(|u|^3).
    d = np.array([0.6, 0.8])
    speeds = np.geomspace(0.0125, 0.1, 6)
    errs = []
    for s in speeds:
        feq = orc.feq_d2q9(1.0, *(s * d))
        g, _ = orc.collide_minxent(feq, 0.6)
        errs.append(np.max(np.abs(g - feq)))
    slope = np.polyfit(np.log(speeds), np.log(errs), 1)[0]
    assert abs(slope - 3.0) < 0.1, slope


def test_divergence_does_not_increase_and_minimiser_beats_other_rules(orc):
    rng = np.random.default_rng(5)
    bad = 0
    for rho, ux, uy in random_nodes(rng, 2000):
        f = perturbed(orc, rng, rho, ux, uy, 0.05)
        tau = rng.uniform(0.5005, 1.5)
        tau2 = (8 * tau - 1) / (2 * tau - 1)
        r = f.sum()
        H = lambda g: orc.kld(g / g.sum())
        p0 = orc.minxent_start(f, tau)
        p1, _ = orc.collide_minxent(f, tau)
        ps, _ = orc.converged_minxent(f, tau)
        srt = orc.collide_srt_d2q9(f, tau)
        trt = orc.collide_mrt_d2q9(f, [0, 1 / tau, 1 / tau, 0, 1 / tau2, 0, 1 / tau2, 1 / tau, 1 / tau])
        mrt = orc.collide_mrt_d2q9(f, [0, 1.64, 1.54, 0, 1 / tau2, 0, 1 / tau2, 1 / tau, 1 / tau])
        tol = 1e-15
        bad += H(p1) > H(p0) + tol
        bad += H(ps) > H(p1) + tol
        for other in (srt, trt, mrt):
            if np.all(other > 0):
                bad += H(ps) > H(other) + tol
        assert abs(r - ps.sum()) < 1e-13 * r
    assert bad == 0


# --------------------------------------------------------------------------
# Converged minimiser by independent routes, and the single step against it
# --------------------------------------------------------------------------

def dual_minimiser(golden, f, tau, tau2, variant, dps=40):
    """Exponential-family (dual) route in mpmath: p = W exp(sum_c l_c T_c - 1)
    with the multipliers l solving the constraints by Newton's method."""
    mpmath.mp.dps = dps
    T = printed_T(golden)
    W = printed_weights_in_T_order(golden)
    rows = [0, 3, 5, 7, 8] if variant == 4 else [0, 3, 4, 5, 6, 7, 8]
    fm = [mpmath.mpf(float(x)) for x in f]
    rho = sum(fm)
    p = [x / rho for x in fm]
    Tm = [[mpmath.mpf(int(T[i][a])) for a in range(9)] for i in range(9)]
    mom = lambda q, i: sum(Tm[i][a] * q[a] for a in range(9))
    ux, uy = mom(p, 3), mom(p, 5)
    eq = {7: ux * ux - uy * uy, 8: ux * uy, 4: -ux, 6: -uy}
    target = {0: mpmath.mpf(1), 3: ux, 5: uy,
              7: mom(p, 7) + (eq[7] - mom(p, 7)) / tau, 8: mom(p, 8) + (eq[8] - mom(p, 8)) / tau}
    if variant == 2:
        target[4] = mom(p, 4) + (eq[4] - mom(p, 4)) / tau2
        target[6] = mom(p, 6) + (eq[6] - mom(p, 6)) / tau2
    Wm = [mpmath.mpf(Fraction(w).limit_denominator(100).numerator) / Fraction(w).limit_denominator(100).denominator
          for w in W]
    lam = [mpmath.mpf(0)] * len(rows)
    lam[0] = mpmath.mpf(1)
    for _ in range(100):
        q = [Wm[a] * mpmath.exp(sum(lam[k] * Tm[rows[k]][a] for k in range(len(rows))) - 1) for a in range(9)]
        res = [mom(q, rows[k]) - target[rows[k]] for k in range(len(rows))]
        if max(abs(x) for x in res) < mpmath.mpf(10) ** (-dps + 5):
            break
        J = mpmath.matrix(len(rows), len(rows))
        for i in range(len(rows)):
            for j in range(len(rows)):
                J[i, j] = sum(Tm[rows[i]][a] * Tm[rows[j]][a] * q[a] for a in range(9))
        d = mpmath.lu_solve(J, mpmath.matrix(res))
        lam = [lam[k] - d[k] for k in range(len(rows))]
    return np.array([float(rho * x) for x in q])


@pytest.mark.parametrize("variant", [4, 2])
def test_converged_minimiser_two_routes(orc, golden, variant):
    rng = np.random.default_rng(6 + variant)
    for rho, ux, uy in random_nodes(rng, 12):
        f = perturbed(orc, rng, rho, ux, uy, 0.08)
        tau = rng.uniform(0.51, 1.2)
        tau2 = (8 * tau - 1) / (2 * tau - 1)
        ps, _ = orc.converged_minxent(f, tau, tau2, variant)
        pd = dual_minimiser(golden, f, tau, tau2, variant)
        assert np.max(np.abs(ps - pd)) <= 1e-13 * f.sum()


def test_converged_minimiser_meets_optimality_conditions(orc, golden):
    # At the minimiser, ln(p/W) lies in the span of the constrained rows.
    T = printed_T(golden)
    W = printed_weights_in_T_order(golden)
    C = T[[0, 3, 5, 7, 8]]
    Q, _ = np.linalg.qr(C.T)
    rng = np.random.default_rng(8)
    for rho, ux, uy in random_nodes(rng, 50):
        f = perturbed(orc, rng, rho, ux, uy, 0.08)
        ps, _ = orc.converged_minxent(f, rng.uniform(0.51, 1.2))
        L = np.log(ps / ps.sum() / W)
        resid = L - Q @ (Q.T @ L)
        assert np.max(np.abs(resid)) <= 1e-12


def test_minxent2_library_optimiser(orc, golden):
    # MinxEnt2 leaves two free moments: minimise S over them with scipy.
    T = printed_T(golden)
    W = printed_weights_in_T_order(golden)
    Ti = np.linalg.inv(T)
    rng = np.random.default_rng(9)
    for rho, ux, uy in random_nodes(rng, 10):
        f = perturbed(orc, rng, rho, ux, uy, 0.05)
        tau = rng.uniform(0.55, 1.2)
        tau2 = (8 * tau - 1) / (2 * tau - 1)
        ps, _ = orc.converged_minxent(f, tau, tau2, 2)
        M = T @ (ps / ps.sum())

        def S(m):
            Mm = M.copy()
            Mm[1], Mm[2] = m
            p = Ti @ Mm
            if np.any(p <= 0):
                return 1e3
            return float(np.sum(p * np.log(p / W)))

        m0 = np.array([M[1], M[2]]) + rng.uniform(-0.02, 0.02, 2)
        r = scipy.optimize.minimize(S, m0, method="Nelder-Mead",
                                    options={"xatol": 1e-12, "fatol": 1e-18, "maxiter": 4000})
        assert np.max(np.abs(r.x - M[[1, 2]])) <= 1e-7


def test_single_step_converges_quadratically(orc):
    # One Newton step from the start point: error ~ K * (start error)^2.
    # From a rest base the start error scales with the perturbation, so the
    # log-log slope of the one-step error against the start error is 2.
    _, _, W, _, _ = orc.constants()
    rng = np.random.default_rng(10)
    for trial in range(4):
        rho = rng.uniform(0.5, 2.0)
        base = rho * W
        delta = base * rng.uniform(-1, 1, 9)
        ds, es = [], []
        for s in np.geomspace(2e-3, 2e-1, 8):
            f = base + s * delta
            fs, _ = orc.converged_minxent(f, 0.8)
            f0 = orc.minxent_start(f, 0.8)
            f1, _ = orc.collide_minxent(f, 0.8)
            ds.append(np.max(np.abs(f0 - fs)))
            es.append(np.max(np.abs(f1 - fs)))
        slope = np.polyfit(np.log(ds), np.log(es), 1)[0]
        assert abs(slope - 2.0) < 0.15, (trial, slope)
        assert max(es) < 0.1 * max(ds)


def test_single_step_error_bounded_by_square_of_start_error(orc):
    rng = np.random.default_rng(18)
    for rho, ux, uy in random_nodes(rng, 200, umax=0.1, noise=0.05):
        f = perturbed(orc, rng, rho, ux, uy, 0.05)
        fs, _ = orc.converged_minxent(f, 0.8)
        f0 = orc.minxent_start(f, 0.8)
        f1, _ = orc.collide_minxent(f, 0.8)
        d = np.max(np.abs(f0 - fs)) / rho
        e = np.max(np.abs(f1 - fs)) / rho
        assert e <= 50.0 * d * d + 1e-15


# --------------------------------------------------------------------------
# D1Q3 and cross-lattice reductions
# --------------------------------------------------------------------------

def test_d1q3_srt_equals_moment_form(orc):
    rng = np.random.default_rng(11)
    for _ in range(2000):
        rho = rng.uniform(0.3, 3)
        u = rng.uniform(-0.3, 0.3)
        f = orc.feq_d1q3(rho, u) * (1 + 0.1 * rng.uniform(-1, 1, 3))
        tau = rng.uniform(0.5001, 2.0)
        a = orc.collide_srt_d1q3(f, tau)
        b = orc.collide_moment_d1q3(f, tau)
        assert np.max(np.abs(a - b)) <= 4 * EPS * f.sum()


def test_d2q9_srt_tube_marginalises_to_d1q3(orc):
    nx, ny, steps, tau = 96, 4, 120, 0.53
    rho1 = np.where(np.arange(nx) < nx // 2, 1.5, 0.75)
    r1 = orc.run(orc.D1Q3, orc.SRT, orc.BC_TUBE, nx, 1, tau, rho1, np.zeros(nx), steps=steps)
    rho2 = np.tile(rho1, (ny, 1))
    r2 = orc.run(orc.D2Q9, orc.SRT, orc.BC_TUBE, nx, ny, tau, rho2, np.zeros((ny, nx)), np.zeros((ny, nx)),
                 steps=steps)
    fl = slice(1, nx - 1)
    for y in range(ny):
        assert np.max(np.abs(r2["rho"][y, fl] - r1["rho"][fl])) <= 1e-13
        assert np.max(np.abs(r2["ux"][y, fl] - r1["ux"][fl])) <= 1e-13
        assert np.max(np.abs(r2["uy"][y, fl])) <= 1e-13


def test_riemann_plateau_of_the_d1q3_tube(orc):
    # Exact isothermal Riemann problem with c_s^2 = 1/3 (pi = rho/3, Sec. IV.C):
    # left rarefaction u* = c ln(rho_L/rho*), right shock u* = c (rho* - rho_R)/sqrt(rho* rho_R).
    c = 1 / np.sqrt(3)
    rl, rr = 1.5, 0.75
    fn = lambda r: c * np.log(rl / r) - c * (r - rr) / np.sqrt(r * rr)
    rs = scipy.optimize.brentq(fn, rr, rl)
    us = c * np.log(rl / rs)
    rho = np.where(np.arange(800) < 400, rl, rr)
    r = orc.run(orc.D1Q3, orc.SRT, orc.BC_TUBE, 800, 1, 0.51, rho, np.zeros(800), steps=400)
    tail = int(400 + 400 * (us - c)) + 20
    shock = int(400 + 400 * us * rs / (rs - rr)) - 40
    assert tail < shock
    plateau = slice(tail, shock)
    assert abs(np.median(r["rho"][plateau]) / rs - 1) < 0.02
    assert abs(np.median(r["ux"][plateau]) / us - 1) < 0.02
    assert not r["unstable"]


def test_tube_mirror_symmetry(orc):
    n = 200
    rho = np.where(np.arange(n) < 100, 1.5, 0.75)
    a = orc.run(orc.D1Q3, orc.SRT, orc.BC_TUBE, n, 1, 0.52, rho, np.zeros(n), steps=150)
    b = orc.run(orc.D1Q3, orc.SRT, orc.BC_TUBE, n, 1, 0.52, rho[::-1].copy(), np.zeros(n), steps=150)
    assert np.max(np.abs(a["rho"] - b["rho"][::-1])) <= 1e-14
    assert np.max(np.abs(a["ux"] + b["ux"][::-1])) <= 1e-14


# --------------------------------------------------------------------------
# Whole-run invariants of the D2Q9 MinxEnt4 cycle
# --------------------------------------------------------------------------

def smooth_field(n, rng, amp=0.03):
    y, x = np.mgrid[0:n, 0:n] * (2 * np.pi / n)
    kx, ky = rng.integers(1, 3, 2)
    ux = amp * np.sin(kx * y + 0.3) * np.cos(x)
    uy = amp * np.cos(ky * x + 0.1) * np.sin(y + 0.2)
    rho = 1 + 0.01 * np.cos(x + 2 * y)
    return rho, ux, uy


def test_periodic_run_conserves_mass_and_momentum(orc):
    rng = np.random.default_rng(12)
    n = 20
    rho, ux, uy = smooth_field(n, rng)
    r = orc.run(orc.D2Q9, orc.MINXENT4, orc.BC_PERIODIC, n, n, 0.53, rho, ux, uy, steps=100)
    m0, m1 = rho.sum(), r["rho"].sum()
    assert abs(m1 - m0) <= 1e-13 * m0
    assert abs((r["rho"] * r["ux"]).sum() - (rho * ux).sum()) <= 1e-13 * m0
    assert abs((r["rho"] * r["uy"]).sum() - (rho * uy).sum()) <= 1e-13 * m0


def test_box_bounce_back_conserves_mass(orc, golden):
    # Mass in fluid nodes plus the populations parked on wall nodes that came
    # from fluid nodes is conserved by full-way bounce-back.
    vx, vy = printed_columns(golden)
    rng = np.random.default_rng(13)
    n = 18
    rho, ux, uy = smooth_field(n, rng)
    total = None
    for steps in (0, 1, 7, 40):
        r = orc.run(orc.D2Q9, orc.MINXENT4, orc.BC_BOX, n, n, 0.56, rho, ux, uy, steps=steps, want_f=True)
        f = r["f"]
        m = 0.0
        for y in range(n):
            for x in range(n):
                wall = x in (0, n - 1) or y in (0, n - 1)
                if not wall:
                    m += f[:, y, x].sum()
                else:
                    for a in range(9):
                        sx, sy = x - vx[a], y - vy[a]
                        if 0 < sx < n - 1 and 0 < sy < n - 1:
                            m += f[a, y, x]
        if steps == 0:
            total = m
        else:
            assert abs(m - total) <= 1e-13 * total, steps


def test_rotation_equivariance(orc):
    rng = np.random.default_rng(14)
    n = 16
    rho, ux, uy = smooth_field(n, rng, amp=0.05)
    a = orc.run(orc.D2Q9, orc.MINXENT4, orc.BC_PERIODIC, n, n, 0.6, rho, ux, uy, steps=30)
    # Rotate by +90 degrees: new(x', y') with x' = -y, y' = x (array rot90
    # over (y, x) axes), velocity (ux, uy) -> (-uy, ux).
    R = lambda A: np.rot90(A, 1, axes=(1, 0)).copy()
    b = orc.run(orc.D2Q9, orc.MINXENT4, orc.BC_PERIODIC, n, n, 0.6, R(rho), R(-uy), R(ux), steps=30)
    assert np.max(np.abs(b["rho"] - R(a["rho"]))) <= 1e-14
    assert np.max(np.abs(b["ux"] - R(-a["uy"]))) <= 1e-14
    assert np.max(np.abs(b["uy"] - R(a["ux"]))) <= 1e-14


def test_cavity_mirror_symmetry(orc):
    n = 20
    rng = np.random.default_rng(15)
    rho = 1 + 1e-3 * rng.uniform(-1, 1, (n, n))
    z = np.zeros((n, n))
    a = orc.run(orc.D2Q9, orc.MINXENT4, orc.BC_CAVITY, n, n, 0.55, rho, z, z, steps=60, u_lid=0.1)
    b = orc.run(orc.D2Q9, orc.MINXENT4, orc.BC_CAVITY, n, n, 0.55, rho[:, ::-1].copy(), z, z, steps=60,
                u_lid=-0.1)
    fl = (slice(1, n - 1), slice(1, n - 1))
    assert np.max(np.abs(a["rho"][fl] - b["rho"][:, ::-1][fl])) <= 1e-14
    assert np.max(np.abs(a["ux"][fl] + b["ux"][:, ::-1][fl])) <= 1e-14
    assert np.max(np.abs(a["uy"][fl] - b["uy"][:, ::-1][fl])) <= 1e-14


def test_homogeneity_in_density(orc):
    n = 16
    rng = np.random.default_rng(16)
    rho = 1 + 1e-3 * rng.uniform(-1, 1, (n, n))
    z = np.zeros((n, n))
    a = orc.run(orc.D2Q9, orc.MINXENT4, orc.BC_CAVITY, n, n, 0.6, rho, z, z, steps=40, u_lid=0.1, rho0=1.0)
    b = orc.run(orc.D2Q9, orc.MINXENT4, orc.BC_CAVITY, n, n, 0.6, 2 * rho, z, z, steps=40, u_lid=0.1, rho0=2.0)
    fl = (slice(1, n - 1), slice(1, n - 1))
    assert np.max(np.abs(b["rho"][fl] - 2 * a["rho"][fl])) <= 1e-14
    assert np.max(np.abs(b["ux"][fl] - a["ux"][fl])) <= 1e-14


@pytest.mark.parametrize("direction", ["axis", "diagonal"])
def test_shear_wave_decay_gives_the_viscosity_relation(orc, direction):
    # nu = (2 tau - 1)/6 (Sec. IV.C).  An axis-aligned shear wave loads the
    # xy stress (C9); a diagonal transverse wave loads xx - yy (C8).
    n, tau, amp = 48, 0.8, 1e-4
    nu = (2 * tau - 1) / 6
    y, x = np.mgrid[0:n, 0:n]
    if direction == "axis":
        k2 = (2 * np.pi / n) ** 2
        ux, uy = amp * np.sin(2 * np.pi * y / n), np.zeros((n, n))
        proj = lambda r: (r["ux"] * np.sin(2 * np.pi * y / n)).sum()
    else:
        k2 = 2 * (2 * np.pi / n) ** 2
        ph = 2 * np.pi * (x + y) / n
        ux, uy = amp * np.sin(ph), -amp * np.sin(ph)
        proj = lambda r: ((r["ux"] - r["uy"]) * np.sin(ph)).sum()
    rho = np.ones((n, n))
    t1, t2 = 100, 400
    a1 = proj(orc.run(orc.D2Q9, orc.MINXENT4, orc.BC_PERIODIC, n, n, tau, rho, ux, uy, steps=t1))
    a2 = proj(orc.run(orc.D2Q9, orc.MINXENT4, orc.BC_PERIODIC, n, n, tau, rho, ux, uy, steps=t2))
    rate = np.log(a1 / a2) / (t2 - t1)
    assert abs(rate / (nu * k2) - 1) < 0.02, rate / (nu * k2)


def test_unstable_flag_on_negative_populations(orc):
    # SRT near tau = 1/2 with a fast lid breaks down; the run reports it.
    n = 16
    z = np.zeros((n, n))
    r = orc.run(orc.D2Q9, orc.SRT, orc.BC_CAVITY, n, n, 0.5001, np.ones((n, n)), z, z, steps=300, u_lid=0.4)
    assert r["unstable"] and r["first_step"] >= 0


def test_first_unstable_node_is_the_perturbed_one(orc):
    # Every node at rest except (5, 3), whose velocity 0.9 gives its start
    # point negative populations: it alone can fail the stability test in the
    # first collision, so the first event is step 0 at node 3*8 + 5.
    nx, ny = 8, 6
    rho = np.ones((ny, nx))
    ux = np.zeros((ny, nx))
    ux[3, 5] = 0.9
    r = orc.run(orc.D2Q9, orc.MINXENT4, orc.BC_PERIODIC, nx, ny, 0.8, rho, ux, np.zeros((ny, nx)), steps=3)
    assert r["unstable"] and r["first_step"] == 0 and r["first_node"] == 3 * nx + 5
    # The same node seen through a window that starts at (2, 1).
    w = orc.run(orc.D2Q9, orc.MINXENT4, orc.BC_PERIODIC, nx, ny, 0.8, rho[1:5, 2:8], ux[1:5, 2:8],
                np.zeros((4, 6)), steps=1, window=(2, 1, 6, 4))
    assert w["first_step"] == 0 and w["first_node"] == 3 * nx + 5
    # A stable run reports no node.
    q = orc.run(orc.D2Q9, orc.MINXENT4, orc.BC_PERIODIC, nx, ny, 0.8, rho, np.zeros((ny, nx)),
                np.zeros((ny, nx)), steps=3)
    assert not q["unstable"] and q["first_step"] == -1 and q["first_node"] == -1


def test_rejects_tau_at_or_below_one_half(orc):
    with pytest.raises(ValueError):
        orc.run(orc.D1Q3, orc.SRT, orc.BC_TUBE, 10, 1, 0.5, np.ones(10), np.zeros(10), steps=1)


def test_window_run_matches_whole_run_inside_the_cone(orc):
    n, steps = 40, 5
    rng = np.random.default_rng(17)
    rho = 1 + 1e-3 * rng.uniform(-1, 1, (n, n))
    z = np.zeros((n, n))
    full = orc.run(orc.D2Q9, orc.MINXENT4, orc.BC_CAVITY, n, n, 0.6, rho, z, z, steps=steps, u_lid=0.1)
    for (x0, y0, wx, wy) in [(0, 0, 14, 14), (10, 12, 17, 15), (25, 25, 15, 15)]:
        w = orc.run(orc.D2Q9, orc.MINXENT4, orc.BC_CAVITY, n, n, 0.6, rho[y0:y0 + wy, x0:x0 + wx],
                    z[y0:y0 + wy, x0:x0 + wx], z[y0:y0 + wy, x0:x0 + wx], steps=steps, u_lid=0.1,
                    window=(x0, y0, wx, wy))
        for yy in range(wy):
            for xx in range(wx):
                gx, gy = x0 + xx, y0 + yy
                open_l = xx - steps if x0 > 0 else 1
                open_r = (wx - 1 - xx) - steps if x0 + wx < n else 1
                open_b = yy - steps if y0 > 0 else 1
                open_t = (wy - 1 - yy) - steps if y0 + wy < n else 1
                if min(open_l, open_r, open_b, open_t) < 0 or not (0 < gx < n - 1 and 0 < gy < n - 1):
                    continue
                assert w["rho"][yy, xx] == full["rho"][gy, gx]
                assert w["ux"][yy, xx] == full["ux"][gy, gx]
