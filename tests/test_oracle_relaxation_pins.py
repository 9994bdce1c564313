"""Pins of the oracle's SRT, TRT and MRT collisions against Table III, and of
its divergence H against an independent evaluation.

Sec. II.B.2 writes every comparator as f + T^{-1} B T (f^eq - f) with a
diagonal B, and Table III prints B for each rule.  The rates are read here
from the printed table (tests/golden/paper_tables.json), never from the
oracle, and checked through the per-node rule that the oracle's whole runs
apply (`collide_node`):

* mode by mode: a rest equilibrium perturbed along one non-conserved moment
  keeps rho and j, so its equilibrium is unchanged and one collision scales
  that moment by exactly 1 - b_k and leaves every other moment alone; a rate
  in the wrong slot (1.64 and 1.54 swapped, 1/tau2 on the energy rows) moves
  the scaled moment;
* reductions: Table III's SRT row is the BGK rule of Sec. II.B.1, and TRT
  with tau2 = tau is SRT;
* invariants: rho and j are conserved for any populations;
* the viscosity relation nu = (2 tau - 1)/6 (Sec. IV.C) from the decay of a
  shear wave, since every rule relaxes the stress rows at 1/tau.
"""
import mpmath
import numpy as np
import pytest

NORM2 = np.array([9, 36, 36, 6, 12, 6, 12, 4, 4], dtype=float)
NONCONSERVED = (1, 2, 4, 6, 7, 8)


def printed_T(golden):
    return np.array(golden["moment_matrix_T"]["rows"], dtype=float)


def printed_Tinv(golden):
    # Rows of the printed T are orthogonal with squared norms NORM2, so
    # T^{-1} = T^T diag(1/NORM2) (checked against the printed T below).
    T = printed_T(golden)
    return T.T / NORM2


def printed_weights(golden):
    t = golden["table_I_d2q9"]
    wmap = {tuple(v): n / d for v, n, d in zip(t["velocities"], t["weights_num"], t["weights_den"])}
    T = printed_T(golden)
    return np.array([wmap[(int(a), int(b))] for a, b in zip(T[3], T[5])])


def table_III_rates(golden, rule, tau, tau2):
    """Diagonal of B for `rule`, evaluated from the printed entries."""
    env = {"tau": tau, "tau2": tau2}
    return np.array([float(eval(e, {"__builtins__": {}}, env))
                     for e in golden["table_III_relaxation"][rule]])


def oracle_rule(orc, name):
    return {"SRT": orc.SRT, "TRT": orc.TRT, "MRT": orc.MRT}[name]


def test_printed_T_inverse_is_an_inverse(golden):
    T = printed_T(golden)
    assert np.max(np.abs(T @ printed_Tinv(golden) - np.eye(9))) <= 4e-16


@pytest.mark.parametrize("rule", ["SRT", "TRT", "MRT"])
@pytest.mark.parametrize("tau", [0.52, 0.8, 1.3])
def test_each_moment_relaxes_at_its_table_III_rate(orc, golden, rule, tau):
    tau2 = (8 * tau - 1) / (2 * tau - 1)
    b = table_III_rates(golden, rule, tau, tau2)
    T, Ti, W = printed_T(golden), printed_Tinv(golden), printed_weights(golden)
    rho, eps = 1.7, 1e-3
    base = T @ (rho * W)
    for k in NONCONSERVED:
        f = rho * W + eps * rho * Ti[:, k]
        out, guarded = orc.collide_node(oracle_rule(orc, rule), f, tau, tau2)
        assert not guarded
        m = T @ out
        want = base.copy()
        want[k] += (1.0 - b[k]) * eps * rho
        assert np.max(np.abs(m - want)) <= 1e-14 * rho, (rule, k, m - want)


def test_rates_differ_between_the_perturbed_moments(golden):
    # The mode test can tell the slots apart only where Table III gives them
    # different rates; it does for every pair a plausible mix-up would swap.
    tau = 0.8
    tau2 = (8 * tau - 1) / (2 * tau - 1)
    mrt = table_III_rates(golden, "MRT", tau, tau2)
    trt = table_III_rates(golden, "TRT", tau, tau2)
    assert mrt[1] != mrt[2] and mrt[1] != mrt[4] and mrt[2] != mrt[7] and mrt[4] != mrt[7]
    assert trt[1] != trt[4] and trt[4] == trt[6] and trt[7] == trt[8] == trt[1]


def random_populations(rng, W, n, umax=0.1, noise=0.05):
    out = []
    for _ in range(n):
        rho = rng.uniform(0.5, 3.0)
        ux, uy = rng.uniform(-umax, umax, 2)
        vx = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1])
        vy = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1])
        cu = vx * ux + vy * uy
        feq = W * rho * (1 + 3 * cu + 4.5 * cu * cu - 1.5 * (ux * ux + uy * uy))
        out.append(feq * (1 + noise * rng.uniform(-1, 1, 9)))
    return out


@pytest.mark.parametrize("rule", ["TRT", "MRT"])
def test_comparators_conserve_mass_and_momentum(orc, golden, rule):
    T, W = printed_T(golden), printed_weights(golden)
    rng = np.random.default_rng(11)
    for f in random_populations(rng, W, 300):
        tau = rng.uniform(0.505, 1.5)
        tau2 = (8 * tau - 1) / (2 * tau - 1)
        out, _ = orc.collide_node(oracle_rule(orc, rule), f, tau, tau2)
        d = T @ (out - f)
        assert np.max(np.abs(d[[0, 3, 5]])) <= 8 * np.finfo(float).eps * np.abs(f).sum()


def test_srt_row_is_the_bgk_rule_and_trt_with_equal_times_is_srt(orc, golden):
    W = printed_weights(golden)
    rng = np.random.default_rng(12)
    for f in random_populations(rng, W, 300):
        tau = rng.uniform(0.505, 1.5)
        srt, _ = orc.collide_node(orc.SRT, f, tau)
        via_b = orc.collide_mrt_d2q9(f, table_III_rates(golden, "SRT", tau, tau))
        trt, _ = orc.collide_node(orc.TRT, f, tau, tau)
        scale = np.abs(f).max()
        assert np.max(np.abs(via_b - srt)) <= 1e-15 * 16 * scale
        assert np.max(np.abs(trt - srt)) <= 1e-15 * 16 * scale


def test_runs_apply_the_same_rule(orc, golden):
    # One step of a uniform periodic lattice streams nothing that changes a
    # node, so the run's populations are the per-node rule's output.
    n, tau = 5, 0.7
    tau2 = (8 * tau - 1) / (2 * tau - 1)
    rho, ux, uy = 1.3, 0.04, -0.03
    feq = orc.feq_d2q9(rho, ux, uy)
    for rule in ("SRT", "TRT", "MRT"):
        r = orc.run(orc.D2Q9, oracle_rule(orc, rule), orc.BC_PERIODIC, n, n, tau,
                    np.full((n, n), rho), np.full((n, n), ux), np.full((n, n), uy), steps=1,
                    tau2=tau2, want_f=True)
        node, _ = orc.collide_node(oracle_rule(orc, rule), feq, tau, tau2)
        assert np.max(np.abs(r["f"][:, 2, 2] - node)) <= 1e-15


def shear_wave_rate(orc, coll, n, tau, tau2, direction, t1=50, t2=250, amp=1e-4):
    """Decay rate of a shear wave of wavelength n over [t1, t2], and k^2."""
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
    a1 = proj(orc.run(orc.D2Q9, coll, orc.BC_PERIODIC, n, n, tau, rho, ux, uy, steps=t1, tau2=tau2))
    a2 = proj(orc.run(orc.D2Q9, coll, orc.BC_PERIODIC, n, n, tau, rho, ux, uy, steps=t2, tau2=tau2))
    return np.log(a1 / a2) / (t2 - t1), k2


@pytest.mark.parametrize("rule", ["SRT", "TRT", "MRT", "MINXENT2"])
@pytest.mark.parametrize("direction", ["axis", "diagonal"])
def test_shear_wave_decay_gives_the_viscosity_relation(orc, rule, direction):
    # nu = (2 tau - 1)/6 (Sec. IV.C); every rule relaxes rows 8 and 9 at 1/tau
    # (Table III, and C8/C9 of Sec. IV.C for MinxEnt2).  An axis-aligned wave
    # loads the xy stress, a diagonal transverse wave loads xx - yy.  The
    # measured rate is nu k^2 (1 + c k^2 + ...), where c depends on the other
    # rates (tau2 here), so the rate is taken at two wavelengths and
    # extrapolated to k -> 0 (Richardson).
    tau = 0.8
    tau2 = (8 * tau - 1) / (2 * tau - 1)
    nu = (2 * tau - 1) / 6
    coll = getattr(orc, rule)
    r1, k1 = shear_wave_rate(orc, coll, 48, tau, tau2, direction)
    r2, k2 = shear_wave_rate(orc, coll, 96, tau, tau2, direction)
    q1, q2 = r1 / (nu * k1), r2 / (nu * k2)
    limit = (4 * q2 - q1) / 3
    assert abs(q2 - 1) < 0.01, (q1, q2)
    assert abs(limit - 1) < 0.002, (q1, q2, limit)


def test_kld_value_pins(orc, golden):
    W = printed_weights(golden)
    # H(W) = 0: the weights are the divergence's reference distribution.
    assert orc.kld(W) == 0.0 or abs(orc.kld(W)) <= 1e-16
    # Against a 40-digit evaluation of sum p ln(p/W) from the printed weights.
    mpmath.mp.dps = 40
    t = golden["table_I_d2q9"]
    wmap = {tuple(v): mpmath.mpf(n) / d for v, n, d in zip(t["velocities"], t["weights_num"], t["weights_den"])}
    T = printed_T(golden)
    Wm = [wmap[(int(a), int(b))] for a, b in zip(T[3], T[5])]
    rng = np.random.default_rng(13)
    for _ in range(50):
        p = rng.uniform(0.01, 1.0, 9)
        p /= p.sum()
        exact = mpmath.fsum(mpmath.mpf(pa) * mpmath.log(mpmath.mpf(pa) / w) for pa, w in zip(p, Wm))
        assert abs(orc.kld(p) - float(exact)) <= 1e-14 * max(1.0, abs(float(exact)))
        # Gibbs' inequality: H(p) >= 0 for any distribution p.
        assert orc.kld(p) >= -1e-16
    # A closed form: all mass on the rest velocity gives H = ln(9/4).
    p = np.zeros(9)
    p[int(np.argmax(W))] = 1.0
    q = np.where(p > 0, p, 1e-300)
    assert abs(orc.kld(q) - np.log(9 / 4)) <= 1e-15
