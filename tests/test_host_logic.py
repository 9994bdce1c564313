"""Host-side logic that the GPU studies rely on (CPU only).

- The counter-based input generator is SplitMix64: its first draws of stream 0
  are the published seed-0 outputs of that generator.
- The stream function of the accuracy study (Sec. IV.H) integrates an
  analytic velocity field to its analytic stream function, and the vortex
  search finds the analytic centre.
"""
import math

import numpy as np

from paper_1801_03863_amd import inputs as I


def test_splitmix_stream0_matches_published_outputs():
    # SplitMix64 started from state 0 (Steele, Lea and Flood 2014) outputs
    # 0xe220a8397b1dcdaf, 0x6e789e6aa1b965f4, 0x06c45d188009454f,
    # 0xf88bb8a8724c81ec; the uniform double is the top 53 bits / 2^53.
    want = [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F, 0xF88BB8A8724C81EC]
    got = I.splitmix_uniform(0, np.arange(4, dtype=np.uint64))
    assert [int(g * 2.0 ** 53) for g in got] == [w >> 11 for w in want]


def test_splitmix_streams_are_uniform_and_distinct():
    u = I.splitmix_uniform(1802, np.arange(200000, dtype=np.uint64))
    v = I.splitmix_uniform(1803, np.arange(200000, dtype=np.uint64))
    assert 0.0 <= u.min() and u.max() < 1.0
    assert abs(u.mean() - 0.5) < 3e-3 and abs(u.var() - 1.0 / 12.0) < 2e-3
    assert abs(np.corrcoef(u, v)[0, 1]) < 1e-2


def _vortex_field(n, amp=0.01):
    # psi = -A sin^2(pi x / L) sin^2(pi y / L) on x, y in [0, L], L = n - 1;
    # u_y = -d psi / dx vanishes on the side walls, u_x = d psi / dy.
    L = n - 1.0
    y, x = np.mgrid[0:n, 0:n].astype(np.float64)
    sx, sy = np.sin(math.pi * x / L), np.sin(math.pi * y / L)
    psi = -amp * sx ** 2 * sy ** 2
    uy = amp * (math.pi / L) * np.sin(2 * math.pi * x / L) * sy ** 2
    ux = -amp * (math.pi / L) * sx ** 2 * np.sin(2 * math.pi * y / L)
    return psi, ux, uy


def test_stream_function_of_analytic_field():
    from paper_1801_03863_amd.experiments import stream_function
    n = 129
    psi, ux, uy = _vortex_field(n)
    got = stream_function(uy)
    err = np.max(np.abs(got - psi)) / np.max(np.abs(psi))
    assert err < 1e-6, err


def test_stream_function_exact_for_low_degree_rows():
    # Composite Simpson is exact for cubics over whole double intervals (even
    # points) and, with the half-interval rule at odd points, for quadratics
    # everywhere.
    from paper_1801_03863_amd.experiments import stream_function
    n = 33
    x = np.arange(n, dtype=np.float64)
    a = float(n - 1)
    quad = x * (a - x)
    got = stream_function(np.tile(quad, (3, 1)))
    exact = -(a * x ** 2 / 2 - x ** 3 / 3)
    assert np.max(np.abs(got - exact)) <= 1e-12 * np.max(np.abs(exact))
    cubic = x * (a - x) * (x + 1)
    got = stream_function(np.tile(cubic, (3, 1)))
    exact = -(a * x ** 2 / 2 + (a - 1) * x ** 3 / 3 - x ** 4 / 4)
    assert np.max(np.abs(got[:, ::2] - exact[::2])) <= 1e-12 * np.max(np.abs(exact))


def test_vortex_summary_finds_the_analytic_centre():
    from paper_1801_03863_amd.experiments import vortex_summary
    n = 65
    psi, ux, uy = _vortex_field(n)
    rho = np.ones((n, n))
    s = vortex_summary(rho, ux, uy, u_lid=0.01, rho0=1.0)
    assert (s["main"]["i"], s["main"]["j"]) == (n // 2, n // 2)
    # psi_hat = psi / (U L) with L = n - 2 at the centre
    assert abs(s["main"]["psi_hat"] - psi[n // 2, n // 2] / (0.01 * (n - 2))) < 1e-6 * abs(s["main"]["psi_hat"])
    # positions use x = (i - 1/2)/(n - 2), y = (j - 1/2)/(n - 1)
    assert abs(s["main"]["x"] - (n // 2 - 0.5) / (n - 2)) < 1e-15
    assert abs(s["main"]["y"] - (n // 2 - 0.5) / (n - 1)) < 1e-15


def test_total_variation():
    from paper_1801_03863_amd.experiments import total_variation
    assert total_variation(np.array([1.0, 1.0, 0.5, 0.5, 1.0])) == 1.0
    assert total_variation(np.linspace(0.0, 2.0, 11)) == 2.0
