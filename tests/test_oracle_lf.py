"""Checks of the 1D Eulerian low-fidelity oracle (Appendix B).

The paper defers the model's closures to other publications, so the oracle
uses stated substitutes and its numbers are parity unpinned; these tests pin
the solver parts by closed forms and the model by the invariants the paper
states (constant flux across y+, deposition growing with charge and Hamaker
constant, Section 2.2 / Fig. 4 trends)."""

import math

import numpy as np
import pytest
from scipy.integrate import quad

from oracle import lf_eulerian as lf
from oracle.physics import q_max_charge
from synthetic.workloads import physical_params


def test_flux_pure_diffusion_is_resistances_in_series():
    """V = 0: J = 1 / (1/h_w + int dy / D) for any D(y)."""
    y = np.linspace(0.1, 50.0, 4001)
    D = 0.01 + 0.002 * y ** 2
    J, rho = lf.flux(y, np.zeros_like(y), D, hw=0.3)
    res = quad(lambda t: 1.0 / (0.01 + 0.002 * t * t), 0.1, 50.0)[0]
    assert np.isclose(J, 1.0 / (1.0 / 0.3 + res), rtol=1e-5)
    assert np.isclose(rho[-1], 1.0)


def test_flux_constant_drift_closed_form():
    """Constant V and D: rho(y) = J/V + (rho_w - J/V) exp(-V (y - y_w)/D), rho(centre) = 1, J = rho_w h."""
    y = np.linspace(0.0, 20.0, 301)
    V, D, h = 0.02, 0.5, 0.07
    J, rho = lf.flux(y, np.full_like(y, V), np.full_like(y, D), h)
    e = math.exp(-V * 20.0 / D)
    rho_w = 1.0 / (h / V + (1.0 - h / V) * e)
    assert np.isclose(J, rho_w * h, rtol=1e-12)
    # the flux J = D drho/dy + V rho is the same everywhere (exact per cell)
    r = rho_w * (h / V + (1.0 - h / V) * np.exp(-V * y / D))
    assert np.allclose(rho, r / r[-1] * 1.0, rtol=1e-12)


def test_momentum_reaches_drag_equilibrium():
    """Uniform driving G and drag time tau: the implicit march reaches V = tau G away from the centre."""
    y = np.linspace(0.0, 100.0, 20001)
    G, tau = 0.004, 2.0
    work = G * np.diff(y)
    V = lf.momentum(y, np.zeros_like(y), work, tau)
    assert np.isclose(V[0], tau * G, rtol=1e-6)
    assert V[-1] == 0.0


def test_wall_flux_factor_limits():
    assert np.isclose(lf.wall_flux_factor(0.0, 0.5), 0.5 / math.sqrt(2 * math.pi))
    assert np.isclose(lf.wall_flux_factor(10.0, 1e-3), 10.0, rtol=1e-9)     # ballistic


@pytest.mark.parametrize("d", [1.6e-6, 5e-6, 16e-6])
def test_deposition_grows_with_charge_and_cohesion(d):
    p = physical_params(180.0, rho_p=2650.0)
    xs = [lf.solve(p, d, xi * q_max_charge(d), 0.0) for xi in (0.0, 0.025, 0.05, 0.1)]
    zs = [lf.solve(p, d, 0.0, z * 1e-18) for z in (0.0, 0.25, 0.5, 1.0)]
    assert all(b >= a for a, b in zip(xs, xs[1:])) and xs[-1] > xs[0]
    assert all(b >= a for a, b in zip(zs, zs[1:])) and zs[-1] > zs[0]


def test_constant_flux_profile_and_grid_convergence():
    p = physical_params(180.0, rho_p=2650.0)
    d = 5e-6
    r = lf.solve(p, d, 0.1 * q_max_charge(d), 1e-18, return_profiles=True)
    y, rho, V, D = r["y_plus"], r["rho"], r["V"], r["D"]
    J = r["vdep_plus"]
    # discrete flux through the core cells equals V_dep+ (the paper's dV_dep+/dy+ = 0)
    k = slice(900, 1500)
    Jk = 0.5 * (D[k] + D[1:][k]) * np.diff(rho)[k] / np.diff(y)[k] + 0.5 * (V[k] + V[1:][k]) * 0.5 * (rho[k] + rho[1:][k])
    assert np.allclose(Jk, J, rtol=1e-2)
    # first-order grid convergence: successive refinements change V_dep+ by shrinking amounts
    a, b, c = (lf.solve(p, d, 0.1 * q_max_charge(d), 1e-18, n_wall=n, n_core=n) for n in (1600, 3200, 6400))
    assert abs(a - c) / c < 0.04
    assert 1.5 < abs(a - b) / abs(b - c) < 2.5


def test_momentum_heavy_drag_equilibrium():
    """Drag time far below the cell transit time (tiny particles): V = tau G still, to rounding; the
    cancellation-prone root -a + sqrt(a^2 + 2 rhs) would return 0 here."""
    y = np.linspace(0.0, 100.0, 20001)
    G, tau = 0.004, 1e-6
    V = lf.momentum(y, np.zeros_like(y), G * np.diff(y), tau)
    assert np.isclose(V[0], tau * G, rtol=1e-6)


def test_diffusivity_is_stokes_einstein_plus_eddy():
    """D+ = D_B / nu + eps / nu: the Brownian part is k_B T / (3 pi mu d) / nu with mu = rho_f nu,
    T = 293 K (Stokes-Einstein), the eddy part tau_L+ Rr V'_fy+^2 (substitute closures)."""
    p = physical_params(180.0)
    for d in (0.05e-6, 1.6e-6, 16e-6):
        r = lf.solve(p, d, 0.0, 0.0, return_profiles=True)
        mu = p["rho_f"] * p["nu"]
        db = 1.380649e-23 * 293.0 / (3 * np.pi * mu * d) / p["nu"]
        rr = 1.0 / (1.0 + r["taup_plus"] / 10.0)
        eddy = 10.0 * rr * lf.vfy_plus(r["y_plus"]) ** 2
        assert np.allclose(r["D"] - eddy, db, rtol=1e-9)


def test_brownian_limit_is_resistances_in_series():
    """A tiny force-free particle (0.01 um): turbophoresis is negligible, so V_dep+ is the diffusion
    resistance 1 / (1/h_w + int dy+ / D+) with D+ = D_B/nu + eps/nu (quadrature of the closed form)."""
    p = physical_params(180.0)
    d = 0.01e-6
    r = lf.solve(p, d, 0.0, 0.0, n_wall=4000, n_core=16000, return_profiles=True)
    assert np.max(np.abs(r["V"])) < 1e-3 * r["vdep_plus"]
    db = 1.380649e-23 * 293.0 / (3 * np.pi * p["rho_f"] * p["nu"] * d) / p["nu"]
    rr = 1.0 / (1.0 + r["taup_plus"] / 10.0)
    y0, yc = r["y_plus"][0], r["y_plus"][-1]
    pts = [y0, y0 + 1e-6, y0 + 1e-3, y0 + 1, y0 + 10, y0 + 40]
    res = sum(quad(lambda t: 1.0 / (db + 10.0 * rr * float(lf.vfy_plus(t)) ** 2), a, b, limit=200)[0]
              for a, b in zip(pts + [], pts[1:] + [yc]))
    assert np.isclose(r["vdep_plus"], 1.0 / (1.0 / r["h_w"] + res), rtol=1e-3)
