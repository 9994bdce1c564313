"""The paper's studies on the GPU path (Sec. IV.F-H).

- Table II (Sec. IV.H): the 257^2 MinxEnt4 cavity at Re = 1000, rho = 2.7,
  lid speed 0.01, run to steady state; vortex centres and strengths against
  the printed MinxEnt4 row.
- Stability study (Sec. IV.G): the ranking of the collision rules by the
  largest stable lid speed near 1/tau = 2, with each outcome's status checked
  against the oracle on sampled runs.
- Shock tube in the paper's D2Q9 form (Sec. IV.F): oscillation at the front
  for SRT/TRT, none for MinxEnt, and oracle parity of the profiles.
"""
import numpy as np
import pytest

from tests.gpu_helpers import orc_run

pytestmark = pytest.mark.gpu


def E():
    from paper_1801_03863_amd import experiments
    return experiments


# Table II prints the secondary-vortex columns without their powers of ten:
# psi_hat x 1e3 (lower right) and x 1e4 (lower left), dpi_hat x 1e2, and the
# lower-left omega_hat x 10 (the values are otherwise those of the standard
# Re = 1000 cavity).
SCALE = {"main": {"psi_hat": 1.0, "dpi_hat": 1.0, "omega_hat": 1.0},
         "lower_right": {"psi_hat": 1e3, "dpi_hat": 1e2, "omega_hat": 1.0},
         "lower_left": {"psi_hat": 1e4, "dpi_hat": 1e2, "omega_hat": 10.0}}


@pytest.fixture(scope="module")
def table2_run():
    return E().run_cavity_steady(n=257, re=1000.0, u_lid=0.01, rho0=2.7, check_every=20000, tol=3e-6,
                                 min_steps=1500000, max_steps=3000000)


def test_table_II_vortex_centres(table2_run, golden):
    paper = golden["table_II_minxent4"]
    s = table2_run["summary"]
    assert not table2_run["status"]["unstable"] and table2_run["status"]["guarded"] == 0
    n = 257
    for name in ("main", "lower_right", "lower_left"):
        want_i = paper[name]["x"] * (n - 2) + 0.5
        want_j = paper[name]["y"] * (n - 1) + 0.5
        print(name, s[name], "paper cell", want_i, want_j, flush=True)
        assert abs(s[name]["i"] - want_i) <= 1.01 and abs(s[name]["j"] - want_j) <= 1.01, name


@pytest.mark.parametrize("name,field,rel", [
    ("main", "psi_hat", 0.025), ("lower_right", "psi_hat", 0.05), ("lower_left", "psi_hat", 0.08),
    ("main", "omega_hat", 0.03), ("lower_right", "omega_hat", 0.05),
])
def test_table_II_values(table2_run, golden, name, field, rel):
    paper = golden["table_II_minxent4"][name][field]
    got = table2_run["summary"][name][field] * SCALE[name][field]
    print(name, field, got, paper, flush=True)
    assert abs(got / paper - 1) <= rel


def test_table_II_lid_speed_reading(table2_run, golden):
    # The paper names both 0.01 and 0.1 as lid speeds.  At U = 0.1 every
    # strength falls further from the printed MinxEnt4 row than at U = 0.01
    # (by 4-14% against 1-5%): Table II is read as the U = 0.01 run.
    fast = E().run_cavity_steady(n=257, re=1000.0, u_lid=0.1, rho0=2.7, check_every=20000, tol=3e-6,
                                 min_steps=200000, max_steps=1500000)
    assert not fast["status"]["unstable"]
    for name, field in (("main", "psi_hat"), ("lower_right", "psi_hat"), ("lower_left", "psi_hat"),
                        ("main", "omega_hat"), ("lower_right", "omega_hat")):
        paper = golden["table_II_minxent4"][name][field]
        slow_err = abs(table2_run["summary"][name][field] * SCALE[name][field] / paper - 1)
        fast_err = abs(fast["summary"][name][field] * SCALE[name][field] / paper - 1)
        print(name, field, "U=0.01 %.4f  U=0.1 %.4f" % (slow_err, fast_err), flush=True)
        assert fast_err > slow_err + 0.01, (name, field)


def test_table_II_closer_to_minxent4_than_to_ef3_row(table2_run, golden):
    # The run reproduces the paper's MinxEnt4 main vortex, not its EF3 one.
    got = table2_run["summary"]["main"]["psi_hat"]
    assert abs(got - golden["table_II_minxent4"]["main"]["psi_hat"]) < abs(got - (-0.13746))


INV = np.array([1.4, 1.6, 1.8, 1.9, 1.95, 1.99])
LIDS = np.round(np.arange(0.02, 1.001, 0.02), 4)


@pytest.fixture(scope="module")
def sweep():
    out = {}
    for coll in ("srt", "trt", "mrt", "minxent2", "minxent4"):
        out[coll] = E().stability_sweep(coll, INV, LIDS)
    return out


@pytest.fixture(scope="module")
def sweep_luo():
    # The same sweep with tau2 = (8 tau - 1)/(8 (2 tau - 1)), the other reading
    # of the tau2 relation (R2); SRT and MinxEnt4 do not use tau2.
    out = {}
    for coll in ("trt", "mrt", "minxent2"):
        out[coll] = E().stability_sweep(coll, INV, LIDS, tau2_rule="luo")
    return out


def test_stability_ranking_near_zero_viscosity(sweep):
    mx = {c: v[2] for c, v in sweep.items()}
    print({c: dict(zip(INV.tolist(), m.tolist())) for c, m in mx.items()}, flush=True)
    k = int(np.where(INV == 1.99)[0][0])
    # Sec. IV.G / IV.I ranking: MinxEnt4, then MRT, MinxEnt2, TRT; SRT last.
    assert mx["minxent4"][k] > mx["mrt"][k] > mx["minxent2"][k] > mx["trt"][k] > mx["srt"][k]
    for c in ("srt", "trt", "mrt", "minxent2"):
        assert np.all(mx["minxent4"] >= mx[c]), c


@pytest.mark.parametrize("reading", ["printed", "luo"])
def test_stability_claims_at_every_viscosity(sweep, sweep_luo, reading):
    # Sec. IV.G results: MinxEnt4 consistently at least as stable as MRT, and
    # MinxEnt2 consistently at least as stable as its counterpart TRT, at
    # every 1/tau of the sweep under either reading of tau2.  (That SRT is the
    # least stable holds only near zero viscosity, 1/tau = 1.99, under either
    # reading: see the previous test.)
    mx = {c: v[2] for c, v in sweep.items()}
    if reading == "luo":
        mx.update({c: v[2] for c, v in sweep_luo.items()})
    print(reading, {c: m.tolist() for c, m in mx.items()}, flush=True)
    assert np.all(mx["minxent4"] >= mx["mrt"])
    assert np.all(mx["minxent2"] >= mx["trt"])
    k = int(np.where(INV == 1.99)[0][0])
    assert mx["srt"][k] < min(mx[c][k] for c in ("trt", "mrt", "minxent2", "minxent4"))


@pytest.mark.parametrize("coll", ["srt", "mrt", "minxent4"])
def test_stability_outcomes_match_oracle(sweep, coll):
    stable, first, mx = sweep[coll]
    k = int(np.where(INV == 1.99)[0][0])
    inv = INV[k]
    n = 17
    checked = 0
    for u in (mx[k], min(mx[k] + 0.1, 1.0)):
        j = int(np.argmin(np.abs(LIDS - u)))
        rho = np.full((n, n), 2.7)
        z = np.zeros((n, n))
        o = orc_run("d2q9", coll, "cavity", n, n, 1.0 / inv, rho, z, z, steps=1000, u_lid=float(LIDS[j]), rho0=2.7)
        assert o["unstable"] == (not stable[k, j]), (coll, LIDS[j])
        if o["unstable"]:
            assert first[k, j] == o["first_step"], (coll, LIDS[j], first[k, j], o["first_step"])
        checked += 1
    assert checked == 2


@pytest.fixture(scope="module")
def tubes():
    return {c: E().shock_tube_d2q9(c) for c in ("srt", "trt", "mrt", "minxent2", "minxent4")}


def test_shock_tube_oscillation_ranking(tubes):
    tv = {c: E().total_variation(t["rho"]) for c, t in tubes.items()}
    print(tv, flush=True)
    # The initial profile has two jumps of 0.5 (one across the periodic wrap),
    # so a profile that does not oscillate has TV at most 1.
    assert tv["minxent4"] <= 1.0 + 1e-6 and tv["minxent2"] <= 1.0 + 1e-6
    assert tv["srt"] > 10 * tv["minxent4"] and tv["trt"] > 10 * tv["minxent4"]
    assert tv["mrt"] < tv["srt"]
    for t in tubes.values():
        assert t["rows_equal"] and not t["status"]["unstable"]


def test_shock_tube_trt_equals_srt_in_one_dimension(tubes):
    # For data constant in y the state keeps product form, the heat-flux
    # non-equilibrium vanishes, and TRT (which differs only there) is SRT.
    assert np.max(np.abs(tubes["trt"]["rho"] - tubes["srt"]["rho"])) <= 1e-10


@pytest.mark.parametrize("coll", ["minxent4", "srt"])
def test_shock_tube_matches_oracle(tubes, coll):
    nx, ny = 800, 4
    x = np.arange(nx)
    rho = np.tile(np.where(x < nx // 2, 1.0, 0.5), (ny, 1))
    z = np.zeros((ny, nx))
    o = orc_run("d2q9", coll, "periodic", nx, ny, 0.5 + 1e-9, rho, z, z, steps=400)
    g = tubes[coll]
    e_rho = np.max(np.abs(g["rho"] - o["rho"][0])) / np.max(o["rho"][0])
    e_u = np.max(np.abs(g["ux"] - o["ux"][0])) / np.max(np.abs(o["ux"][0]))
    print(coll, e_rho, e_u, flush=True)
    assert e_rho <= 1e-12 and e_u <= 1e-12
