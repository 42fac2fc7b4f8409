"""Pins of the FP64 oracle against what the paper and the mathematics fix (CPU only).

Each test names the passage it checks.  None of them re-types the oracle's own
formula: they use values printed in the paper, closed-form solutions,
conservation laws, library routines or brute force.
"""

import numpy as np
import pytest
from scipy.interpolate import RegularGridInterpolator
from scipy.optimize import brentq

from oracle import physics as ph
from oracle.gather import trilinear
from oracle.sim import OracleSim
from synthetic import make_workload
from synthetic.field import bulk_velocity_plus, make_field, node_coordinates
from synthetic.workloads import physical_params
from tests.oracle_helpers import one_sample, quiet_params, uniform_field


# ------------------------------------------------------------------------------------------ units

def test_tau_p_plus_printed_values():
    """Section 2.1: d = 1.6, 5, 16 um at 2650 kg/m^3 give tau_p+ = 0.1, 1, 10 (with rho_f = 1.2)."""
    nu, R = 1.5e-5, 0.01
    tf = ph.friction_time(180.0, nu, R)
    tpp = ph.response_time(np.array([1.6e-6, 5e-6, 16e-6]), 2650.0, 1.2, nu) / tf
    assert np.allclose(tpp, [0.1, 1.0, 10.0], rtol=0.025)
    # printed Re = U_b D / nu = 5333 with U_b = 4 m/s, D = 20 mm
    assert abs(4.0 * 0.02 / nu - 5333.0) < 1.0


def test_friction_velocity_and_bulk():
    """Re_tau = 180 with R = 10 mm and nu = 1.5e-5 gives u* = 0.27 m/s; the Reichardt profile's U_b+ is 13.96."""
    assert abs(ph.friction_velocity(180.0, 1.5e-5, 0.01) - 0.27) < 1e-12
    assert abs(bulk_velocity_plus(180.0) - 13.96) < 0.01


def test_q_max_eq1():
    """Eq. 1: a 10 um particle carries at most 500 e per um^2 -> 8e-15 C."""
    assert abs(ph.q_max_charge(10e-6) - 8e-15) < 1e-28


# ------------------------------------------------------------------------------------------ gather

def test_trilinear_matches_scipy_and_periodic_seam():
    rng = np.random.default_rng(7)
    n, R, L = 12, 0.01, 0.04
    f = rng.normal(size=(n, n, n, 3))
    xs, ys, zs = node_coordinates(n, R, L)
    # extend periodically in x for the library interpolator
    fx = np.concatenate([f, f[:1]], axis=0)
    xe = np.append(xs, L)
    pts = np.stack([rng.uniform(0, L, 500), rng.uniform(-R, R, 500), rng.uniform(-R, R, 500)], axis=1)
    ref = np.stack([RegularGridInterpolator((xe, ys, zs), fx[..., c], method="linear")(pts) for c in range(3)], 1)
    got = trilinear(f, R, L, pts)
    assert np.max(np.abs(got - ref)) < 1e-12
    # continuity across the periodic seam x = L -> 0
    a = trilinear(f, R, L, np.array([[L - 1e-13, 0.001, -0.002]]))
    b = trilinear(f, R, L, np.array([[0.0, 0.001, -0.002]]))
    assert np.max(np.abs(a - b)) < 1e-9


def test_trilinear_reproduces_affine_field():
    n, R, L = 9, 0.01, 0.04
    xs, ys, zs = node_coordinates(n, R, L)
    X, Y, Z = np.meshgrid(xs, ys, zs, indexing="ij")
    f = np.stack([2.0 + 3.0 * Y - Z, 0.5 * Z, -Y + 4.0 * Z], axis=-1)   # affine in y, z; constant in x
    rng = np.random.default_rng(1)
    pts = np.stack([rng.uniform(0, L, 200), rng.uniform(-R, R, 200), rng.uniform(-R, R, 200)], 1)
    y, z = pts[:, 1], pts[:, 2]
    ref = np.stack([2.0 + 3.0 * y - z, 0.5 * z, -y + 4.0 * z], 1)
    assert np.max(np.abs(trilinear(f, R, L, pts) - ref)) < 1e-13


# ------------------------------------------------------------------------------------------ field

def test_synthetic_field_invariants():
    """Field recipe: zero outside the pipe, every fluctuation mode averages to zero along x."""
    n, R, L, nu = 32, 0.01, 0.04, 1.5e-5
    f = make_field(n, 180.0, R, L, nu, seed=180)
    xs, ys, zs = node_coordinates(n, R, L)
    Y, Z = np.meshgrid(ys, zs, indexing="ij")
    outside = np.sqrt(Y * Y + Z * Z) >= R
    assert np.all(f[:, outside, :] == 0.0)
    # x-mean of the cross-stream components is zero (mean flow is streamwise only)
    assert np.max(np.abs(f[..., 1:].mean(axis=0))) < 1e-12
    # streamwise: x-mean equals the Reichardt mean profile exactly
    from synthetic.field import reichardt_uplus
    us = 180.0 * nu / R
    yp = (R - np.sqrt(Y * Y + Z * Z)) * us / nu
    mean = np.where(~outside, us * reichardt_uplus(yp), 0.0)
    assert np.max(np.abs(f[..., 0].mean(axis=0) - mean)) < 1e-12


# ------------------------------------------------------------------------------------------ drag

def _single_particle(p, field, x, v, d=10e-6):
    return OracleSim(p, field, np.array([x]), np.array([d]), np.zeros(1), one_sample(1),
                     np.array([[1.0, 0.0, 300.0]]), v0=np.array([v]))


def test_schiller_naumann_relaxation_closed_form():
    """Eq. part_source in a uniform flow: the slip s obeys ds/dt = -(1 + c s^a) s / tau_p,
    whose solution is s = (K / (1 - c K))^(1/a) with K = u0/(1 + c u0) e^(-a t / tau_p), u = s^a."""
    d, U = 40e-6, np.array([3.0, 0.0, 0.0])
    p = quiet_params(drag=True)
    taup = ph.response_time(d, p["rho_p"], p["rho_f"], p["nu"])
    a, c = 0.687, 0.15 * (d / p["nu"]) ** 0.687
    s0 = 2.5
    t_end = 1.0 * taup

    def run(nsteps):
        q = dict(p, dt=t_end / nsteps)
        sim = _single_particle(q, uniform_field(8, U), [0.01, 0.0, 0.0], U - np.array([s0, 0, 0]), d)
        sim.step(nsteps)
        return U[0] - sim.v[0, 0]

    u0 = s0 ** a
    K = u0 / (1.0 + c * u0) * np.exp(-a * t_end / taup)
    s_exact = (K / (1.0 - c * K)) ** (1.0 / a)
    e1 = abs(run(200) - s_exact)
    e2 = abs(run(400) - s_exact)
    assert e1 / s_exact < 1e-3
    assert e1 / e2 > 1.8          # converges as dt -> 0


def test_stokes_limit_exact_exponential():
    """Creeping slip (Re_p -> 0, f -> 1): v(t) = U + (v0 - U) e^(-t/tau_p), exact for the exponential kick."""
    d, U = 1e-6, np.array([0.5, -0.2, 0.1])
    p = quiet_params(drag=True)
    taup = ph.response_time(d, p["rho_p"], p["rho_f"], p["nu"])
    v0 = U + np.array([1e-7, 2e-7, -1e-7])          # Re_p ~ 1e-8
    q = dict(p, dt=taup / 10)
    sim = _single_particle(q, uniform_field(8, U), [0.01, 0.0, 0.0], v0, d)
    sim.step(10)
    ref = U + (v0 - U) * np.exp(-1.0)
    assert np.max(np.abs(sim.v[0] - ref)) < 1e-13 + 1e-5 * 3e-7


def test_terminal_velocity():
    """With a body force g and still fluid the particle settles at v_t f(v_t d / nu) = g tau_p."""
    d, gy = 20e-6, 9.81
    p = quiet_params(drag=True, body_force=True, g_body=(0.0, 0.0, -gy))
    taup = ph.response_time(d, p["rho_p"], p["rho_f"], p["nu"])
    vt = brentq(lambda v: v * ph.schiller_naumann(v * d / p["nu"]) - gy * taup, 0.0, 10.0, xtol=1e-15)
    q = dict(p, dt=taup / 20)
    sim = _single_particle(q, uniform_field(8, (0, 0, 0)), [0.01, 0.0, 0.003], [0, 0, 0], d)
    sim.step(1000)                                 # 50 tau_p: transient decays below 1e-20
    assert abs(-sim.v[0, 2] - vt) / vt < 1e-12


# ------------------------------------------------------------------------------------------ Coulomb

def test_two_charges_energy_conserved():
    """Coulomb's law (Eq. coulomb) is conservative: kinetic + k_e q1 q2 / r is conserved by the
    drag-free kick-drift-kick to O(dt^2) with no secular drift."""
    p = quiet_params(coulomb=True)
    d = np.array([10e-6, 10e-6])
    m = ph.particle_mass(d, p["rho_p"])
    q = np.array([3e-15, 2e-15])
    ke = ph.coulomb_constant(p["eps0"])
    r0 = 60e-6
    x0 = np.array([[0.02, 0.0, 0.0], [0.02 + r0, 0.0, 0.0]])
    # time scale: sqrt(m r^3 / (k q q))
    tsc = np.sqrt(m[0] * r0 ** 3 / (ke * q[0] * q[1]))

    def energy(sim):
        r = np.linalg.norm(sim.x[0] - sim.x[1])
        return 0.5 * np.sum(m[:, None] * sim.v ** 2) + ke * q[0] * q[1] / r

    drifts = []
    for nst in (2000, 4000):
        sim = OracleSim(dict(p, dt=3 * tsc / nst), uniform_field(8, (0, 0, 0)), x0, d, q, one_sample(2),
                        np.array([[1.0, 0.0, 300.0]]), v0=np.zeros((2, 3)))
        e0 = energy(sim)
        es = []
        for _ in range(10):
            sim.step(nst // 10)
            es.append(energy(sim))
        drifts.append(max(abs(e - e0) for e in es) / e0)
        assert np.linalg.norm(sim.x[1] - sim.x[0]) > 2 * r0      # they really flew apart
    assert drifts[0] < 1e-5
    assert drifts[0] / drifts[1] > 3.0                            # second order


def test_pair_forces_newton_third_law():
    """All pair forces (Coulomb, contact, cohesion) are equal and opposite: sum_i m_i a_i = 0."""
    rng = np.random.default_rng(11)
    n = 300
    p = quiet_params(coulomb=True, collide=True, vdw=True)
    d = rng.choice([5e-6, 10e-6, 20e-6], n)
    # a tight cluster across the periodic seam so that many pairs touch
    x = np.stack([np.mod(rng.normal(0.0, 60e-6, n), p["L"]), rng.normal(0, 60e-6, n), rng.normal(0, 60e-6, n)], 1)
    v = rng.normal(0, 0.1, (n, 3))
    q = rng.normal(0, 2e-15, n)
    sim = OracleSim(p, uniform_field(8, (0, 0, 0)), x, d, q, one_sample(n), np.array([[1.0, 1e-19, 300.0]]), v0=v)
    f = sim.m[:, None] * sim.a
    scale = np.sum(np.abs(f))
    assert np.max(np.abs(f.sum(axis=0))) / scale < 1e-13
    # the cluster really exercises contacts and cohesion
    r = sim.x[:, None, :] - sim.x[None, :, :]
    r[..., 0] -= p["L"] * np.round(r[..., 0] / p["L"])
    dist = np.linalg.norm(r, axis=-1) + np.eye(n)
    assert np.sum(dist < 0.5 * (d[:, None] + d[None, :])) > 20


def test_coulomb_brute_force_small():
    """Direct sum of Eq. coulomb over a handful of particles, written out pair by pair."""
    p = quiet_params(coulomb=True)
    x = np.array([[0.001, 0.0, 0.0], [0.0392, 1e-4, 0.0], [0.002, -2e-4, 3e-4], [0.0015, 0.0, 5e-6]])
    d = np.array([10e-6, 20e-6, 5e-6, 10e-6])
    q = np.array([1e-15, -2e-15, 3e-15, 1.5e-15])
    sim = OracleSim(p, uniform_field(8, (0, 0, 0)), x, d, q, one_sample(4), np.array([[1.0, 0.0, 300.0]]),
                    v0=np.zeros((4, 3)))
    eps0 = p["eps0"]
    m = p["rho_p"] * np.pi * d ** 3 / 6
    for i in range(4):
        acc = np.zeros(3)
        for j in range(4):
            if i == j:
                continue
            r = x[i] - x[j]
            if r[0] > p["L"] / 2:
                r[0] -= p["L"]
            if r[0] < -p["L"] / 2:
                r[0] += p["L"]
            dist = np.sqrt(r @ r)
            acc += q[i] * q[j] / (4 * np.pi * eps0 * max(dist, (d[i] + d[j]) / 2) ** 2) * (r / dist) / m[i]
        assert np.allclose(sim.a[i], acc, rtol=1e-13, atol=0)


# ------------------------------------------------------------------------------------------ contact

def test_head_on_collision_restitution_and_duration():
    """Appendix A.2.2: e = 0.9 and a contact lasting tau_col = 15 dt (linear spring-dashpot closed form)."""
    p = quiet_params(collide=True)
    d = np.array([10e-6, 10e-6])
    vrel = 0.02
    gap0 = 3 * vrel * p["dt"]
    x0 = np.array([[0.02, 0.0, 0.0], [0.02 + d[0] + gap0, 0.0, 0.0]])
    v0 = np.array([[vrel / 2, 0, 0], [-vrel / 2, 0, 0]])
    sim = OracleSim(p, uniform_field(8, (0, 0, 0)), x0, d, np.zeros(2), one_sample(2),
                    np.array([[1.0, 0.0, 300.0]]), v0=v0)
    in_contact = []
    for _ in range(60):
        sim.step(1)
        in_contact.append(abs(sim.x[1, 0] - sim.x[0, 0]) < d[0])
    e_num = (sim.v[1, 0] - sim.v[0, 0]) / vrel
    assert abs(e_num - 0.9) < 0.9 * 5e-3
    assert abs(sum(in_contact) - p["tau_col_steps"]) <= 1


# ------------------------------------------------------------------------------------------ van der Waals

def test_vdw_hamaker_equals_printed_eq_for_equal_spheres():
    """Eq. vdw (equal diameters) versus the general two-sphere Hamaker force used for all pairs."""
    for d in (1e-6, 10e-6, 20e-6):
        delta = np.geomspace(1e-10, d / 4, 40)
        assert np.allclose(ph.vdw_hamaker(delta, d, d, 1e-19), ph.vdw_equal_printed(delta, d, 1e-19),
                           rtol=1e-10, atol=0)


def test_vdw_is_minus_potential_gradient():
    """F = -dU/dr of Hamaker's two-sphere potential, checked by central differences for unequal spheres."""
    A = 5e-20
    for d1, d2 in ((10e-6, 5e-6), (1e-6, 20e-6), (7e-6, 7e-6)):
        for delta in (3e-9, 1e-8, 1e-7, 1e-6):
            r = 0.5 * (d1 + d2) + delta
            h = delta * 1e-5
            dU = (ph.hamaker_potential(r + h, d1, d2, A) - ph.hamaker_potential(r - h, d1, d2, A)) / (2 * h)
            assert np.isclose(ph.vdw_hamaker(delta, d1, d2, A), dU, rtol=1e-6)


def test_vdw_limits_and_saturation():
    """Small-gap limit A d / (24 delta^2); F(d/4) = 0.2697 A / d; saturation at delta_min (k_r/k)^(1/4); cutoff d/4."""
    A, d = 1e-18, 10e-6
    assert np.isclose(ph.vdw_hamaker(1e-10, d, d, A), A * d / (24 * 1e-20), rtol=1e-4)
    assert np.isclose(ph.vdw_hamaker(d / 4, d, d, A) * d / A, 0.2697, rtol=2e-4)
    p = physical_params()
    ds = ph.vdw_saturation_gap(p)
    assert np.isclose(ds, 1e-9 * 700 ** 0.25) and abs(ds - 5.14e-9) < 0.01e-9
    f = ph.vdw_pair_force(np.array([-2e-6, 0.0, 1e-9, ds, 2.4e-6, 2.6e-6]), d, d, A, ds)
    assert f[0] == f[1] == f[2] == f[3] > 0      # constant below the saturation gap, also in overlap
    assert f[4] > 0 and f[5] == 0.0               # cut off beyond d/4 = 2.5 um


def test_wall_terms_match_appendix_b():
    """Appendix B.2: image force 3 q^2 / (8 pi^2 eps0 rho_p d^3 y^2); wall cohesion A d / (12 m (y - d/2)^2) =
    twice the small-gap pair force (Section 2.2)."""
    eps0, rho_p, d, q, A = 8.854e-12, 2650.0, 5e-6, 4e-16, 1e-19
    m = ph.particle_mass(d, rho_p)
    for y in (3e-6, 1e-5, 1e-4):
        ref = 3 * q * q / (8 * np.pi ** 2 * eps0 * rho_p * d ** 3 * y ** 2)
        assert np.isclose(ph.wall_image_accel(y, q, m, ph.coulomb_constant(eps0)), ref, rtol=1e-12)
    g = 2e-8
    assert np.isclose(ph.wall_vdw_accel(g, d, A, m, 1e-9), A * d / (12 * m * g * g), rtol=1e-12)
    assert np.isclose(ph.wall_vdw_accel(g, d, A, m, 1e-9) * m, 2 * ph.vdw_hamaker(g, d, d, A), rtol=2e-2)


# ------------------------------------------------------------------------------------------ wall test / tally

def test_deposition_fraction_brute_force():
    """Forces off, constant outward radial speed: particle i deposits at the first step n with
    r_i + n dt v_r + d/2 >= R (brute force), and V_dep follows Eq. 2 with the alive-mass time integral."""
    rng = np.random.default_rng(5)
    n = 400
    p = quiet_params()
    d = np.full(n, 10e-6)
    w = make_workload("plain-1k", n=n, seed=9)
    x = w.x
    rho = np.hypot(x[:, 1], x[:, 2])
    er = np.stack([np.zeros(n), x[:, 1] / rho, x[:, 2] / rho], 1)
    vr = 50.0                                     # m/s outward
    nst = 40
    sim = OracleSim(p, uniform_field(8, (0, 0, 0)), x, d, np.zeros(n), one_sample(n),
                    np.array([[1.0, 0.0, 300.0]]), v0=vr * er)
    sim.step(nst)
    R, dt = p["R"], p["dt"]
    exp_step = np.zeros(n, dtype=np.int64)
    for i in range(n):
        for k in range(1, nst + 1):
            if np.hypot(*(x[i, 1:] + k * dt * vr * er[i, 1:])) + d[i] / 2 >= R:
                exp_step[i] = k
                break
    assert np.array_equal(sim.dep_step, exp_step)
    m = ph.particle_mass(d, p["rho_p"])
    alive_steps = np.where(exp_step > 0, exp_step - 1, nst)
    m_alive_dt = dt * np.sum(m * alive_steps)
    t = sim.tally()[0]
    assert t["n_dep"] == int(np.sum(exp_step > 0)) > 0
    assert np.isclose(t["m_alive_dt"], m_alive_dt, rtol=1e-13)
    assert np.isclose(t["v_dep"], R / 2 * np.sum(m[exp_step > 0]) / m_alive_dt, rtol=1e-13)
    # expected deposited fraction for particles uniform in the disk r <= R_e
    Re = R - d[0] / 2
    frac = 1 - ((Re - vr * nst * dt) / Re) ** 2
    assert abs(t["n_dep"] / n - frac) < 4 * np.sqrt(frac / n)


def test_rebound_law_values():
    """Eq. CoR: sigma_y(1000 K) = 200 MPa; cohesion-free impacts below the yield speed rebound elastically;
    strong cohesion makes slow particles stick (CoR = 0)."""
    p = physical_params()
    d = 10e-6
    m = ph.particle_mass(d, p["rho_p"])
    vy = 200e6 / np.sqrt(p["rho_p"] * p["E_young"])
    assert np.isclose(ph.osu_rebound_speed_sq(2 * vy, 1000.0, d, m, 0.0, p), vy * vy)
    assert np.isclose(ph.osu_rebound_speed_sq(0.5, 1000.0, d, m, 0.0, p), 0.25)
    # theta = 1 (T ~ 1889 K) removes the yield speed entirely
    assert ph.osu_rebound_speed_sq(0.5, 1000.0 + 200.0 / 0.225, d, m, 0.0, p) <= 1e-12
    g = 1e-18 / (24 * np.pi * (0.165e-9) ** 2)
    vstick = np.sqrt(2 * np.pi * d * d / 4 * g / m)
    assert ph.osu_rebound_speed_sq(0.99 * vstick, 300.0, d, m, 1e-18, p) < 0
    assert ph.osu_rebound_speed_sq(1.01 * vstick, 300.0, d, m, 1e-18, p) > 0


def test_rebound_reflects_and_conserves_speed_without_cohesion():
    p = quiet_params(rebound_osu=True)
    d = np.array([10e-6])
    R = p["R"]
    x0 = np.array([[0.01, R - d[0] / 2 - 1e-8, 0.0]])
    v0 = np.array([[0.0, 1.0, 0.0]])
    sim = OracleSim(p, uniform_field(8, (0, 0, 0)), x0, d, np.zeros(1), one_sample(1),
                    np.array([[1.0, 0.0, 300.0]]), v0=v0)
    sim.step(1)
    assert sim.alive[0] and np.isclose(sim.v[0, 1], -1.0)
    assert sim.x[0, 1] + d[0] / 2 < R


def test_soft_tally_stationary_particle():
    """Smoothed tally: a particle held at gap g accrues l = n sigma(-g/eps_s)/soft_tau."""
    p = quiet_params(soft_tally=True)
    d = np.array([10e-6])
    g = 0.3e-6
    x0 = np.array([[0.01, p["R"] - d[0] / 2 - g, 0.0]])
    sim = OracleSim(p, uniform_field(8, (0, 0, 0)), x0, d, np.zeros(1), one_sample(1),
                    np.array([[1.0, 0.0, 300.0]]), v0=np.zeros((1, 3)))
    sim.step(7)
    sig = 1.0 / (1.0 + np.exp(g / (0.05 * d[0])))
    assert np.isclose(sim.ell[0], 7 * sig / 10.0, rtol=1e-12)
    m = ph.particle_mass(d[0], p["rho_p"])
    assert np.isclose(sim.tally()[0]["j_soft"], m * (1 - np.exp(-sim.ell[0])), rtol=1e-12)
