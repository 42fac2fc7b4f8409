"""Pins of the temperature-dependent rebound law and the capture efficiency (Section 4.4, Eqs. CoR and CE)."""

import numpy as np

from oracle import physics as ph
from oracle.sim import OracleSim
from synthetic import make_workload
from synthetic.field import bulk_velocity_plus
from synthetic.workloads import physical_params, q_max

T_MELT = 1000.0 + 200.0 / 0.225      # theta = 1: the yield stress reaches zero


def test_yield_stress_and_theta_map():
    assert ph.yield_stress(1000.0) == 200e6
    assert abs(ph.yield_stress(ph.temperature_of_theta(0.5)) - 100e6) < 1e-6
    assert abs(ph.yield_stress(T_MELT)) < 1e-6
    assert ph.yield_stress(2000.0) == 0.0                           # theta > 1: floored
    assert np.isclose(ph.temperature_of_theta(1.0), T_MELT, rtol=1e-15)


def test_cor_closed_forms_and_monotonicity():
    """Without cohesion CoR_n = min(1, V_y / V_n1) with the yield speed V_y = sigma_y / sqrt(rho_p E);
    CoR_n is in [0, 1] and falls with cohesion (zeta) and temperature (theta) at every impact speed
    (the trends of Fig. 12); at theta = 1 every particle sticks."""
    p = physical_params(180.0, acont_coef=1e-3)
    d = 5e-6
    m = ph.particle_mass(d, p["rho_p"])
    v = np.geomspace(0.01, 100.0, 400)
    for T in (1000.0, 1500.0, 1850.0):
        vy = ph.yield_stress(T) / np.sqrt(p["rho_p"] * p["E_young"])
        assert np.allclose(ph.cor_n(v, T, d, m, 0.0, p), np.minimum(1.0, vy / v), rtol=1e-14)
    prev = None
    for zeta in np.linspace(0.0, 1.0, 11):
        c = ph.cor_n(v, ph.temperature_of_theta(0.5), d, m, zeta * 1e-18, p)
        assert np.all((c >= 0) & (c <= 1))
        if prev is not None:
            assert np.all(c <= prev) and np.any(c < prev)
        prev = c
    prev = None
    for theta in np.linspace(0.0, 1.0, 11):
        c = ph.cor_n(v, ph.temperature_of_theta(theta), d, m, 1e-18, p)
        if prev is not None:
            assert np.all(c <= prev)
        prev = c
    assert np.all(ph.cor_n(v, T_MELT, d, m, 1e-18, p) == 0.0)
    # sticking threshold below the yield speed: V_n1^2 = 2 A_cont gamma_c / m = A acont / (8 pi delta_c^2 rho_p d)
    A = 1e-19
    vs = np.sqrt(A * p["acont_coef"] / (8 * np.pi * p["delta_c"] ** 2 * p["rho_p"] * d))
    c = ph.cor_n(np.array([0.999 * vs, 1.001 * vs]), 1000.0, d, m, A, p)
    assert c[0] == 0.0 and c[1] > 0.0


def test_capture_efficiency_mass_flow_identity():
    """Eq. CE: (4L/D)(u*/U_b) V_dep+ equals deposited over total particle mass flow, m_dep L / (M dt U_b),
    the ratio the oracle's tally computes directly."""
    rng = np.random.default_rng(4)
    n = 300
    p = physical_params(180.0, dt=2e-7)
    d = rng.choice([5e-6, 10e-6], n)
    x, er = _near_wall(rng, n, p, d)
    v0 = 1.5 * er + rng.normal(0, 0.1, (n, 3))
    f = make_workload("plain-1k", n=4, field_n=32).field()
    o = OracleSim(p, f, x, d, q_max(d), np.array([0, n]), np.array([[0.05, 1e-19, 300.0]]), v0=v0)
    o.step(40)
    t = o.tally()[0]
    assert t["n_dep"] > 10
    u_star = ph.friction_velocity(p["re_tau"], p["nu"], p["R"])
    ce = ph.capture_efficiency(t["v_dep_plus"], p["L"], 2 * p["R"], u_star, p["u_bulk"])
    assert np.isclose(t["ce"], ce, rtol=1e-13)


def test_bulk_velocity_of_the_synthetic_field():
    """U_b (the area-mean axial velocity) of the sampled field agrees with the mean profile's U_b+ u*."""
    p = physical_params(180.0)
    f = make_workload("plain-1k", n=4, field_n=64).field()
    from oracle.gather import trilinear
    rng = np.random.default_rng(0)
    n = 400000
    r = p["R"] * np.sqrt(rng.uniform(0, 1, n))
    phi = rng.uniform(0, 2 * np.pi, n)
    x = np.stack([rng.uniform(0, p["L"], n), r * np.cos(phi), r * np.sin(phi)], 1)
    ub = trilinear(f, p["R"], p["L"], x)[:, 0].mean()
    assert abs(ub / p["u_bulk"] - 1) < 0.02
    assert np.isclose(p["u_bulk"], bulk_velocity_plus(180.0) * 180.0 * p["nu"] / p["R"], rtol=1e-15)


def _near_wall(rng, n, p, d, band=100e-6):
    rr = p["R"] - 0.5 * d - rng.uniform(0.0, band, n)
    phi = rng.uniform(0.0, 2 * np.pi, n)
    x = np.stack([rng.uniform(0, p["L"], n), rr * np.cos(phi), rr * np.sin(phi)], 1)
    return x, np.stack([np.zeros(n), np.cos(phi), np.sin(phi)], 1)


def test_rebound_end_points_on_trajectories():
    """theta = 1 (yield stress 0): the rebound law sticks every impact, so the run equals the all-stick
    run exactly; theta = 0 without cohesion: impacts at pipe speeds are far below the yield speed
    (~24 m/s) and fully elastic, so nothing deposits and every impact reverses the normal velocity."""
    rng = np.random.default_rng(6)
    n = 200
    f = make_workload("plain-1k", n=4, field_n=32).field()
    d = rng.choice([5e-6, 10e-6], n)
    base = physical_params(180.0, dt=2e-7, acont_coef=1e-3, wall_vdw=False, vdw=False)
    x, er = _near_wall(rng, n, base, d)
    v0 = 1.5 * er + rng.normal(0, 0.1, (n, 3))
    q = q_max(d)
    runs = {}
    for key, rebound, T, A in (("stick", False, 300.0, 1e-19), ("melt", True, T_MELT, 1e-19),
                               ("cold", True, 1000.0, 0.0)):
        p = dict(base, rebound_osu=rebound)
        o = OracleSim(p, f, x, d, q, np.array([0, n]), np.array([[0.02, A, T]]), v0=v0)
        o.step(40)
        runs[key] = o
    assert runs["stick"].tally()[0]["n_dep"] > 10
    assert np.array_equal(runs["stick"].dep_step, runs["melt"].dep_step)
    assert runs["melt"].tally()[0]["ce"] == runs["stick"].tally()[0]["ce"]
    assert runs["cold"].tally()[0]["n_dep"] == 0 and runs["cold"].tally()[0]["ce"] == 0.0
    rr = np.hypot(runs["cold"].x[:, 1], runs["cold"].x[:, 2])
    assert np.all(rr + 0.5 * d < p["R"])                               # reflected back inside
