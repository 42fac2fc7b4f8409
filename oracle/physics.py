"""Force laws of the particle step, float64 (Appendix A.2, Section 2.2, Appendix B.2, Section 4.4).

Each function states the passage it follows.  Readings of points the paper
leaves open are marked "Reading"; they are the same readings the HIP path
implements.
"""

from __future__ import annotations

import numpy as np


# ----------------------------------------------------------------------------- constants, units

def coulomb_constant(eps0: float) -> float:
    """k_e = 1 / (4 pi eps0), the prefactor of Coulomb's law (Eq. coulomb, Section 2.2)."""
    return 1.0 / (4.0 * np.pi * eps0)


def particle_mass(d, rho_p):
    """Mass of a sphere of diameter d and density rho_p."""
    return rho_p * np.pi * np.asarray(d, dtype=np.float64) ** 3 / 6.0


def response_time(d, rho_p, rho_f, nu):
    """tau_p = rho_p d^2 / (18 rho_f nu) (Appendix A.2.1, after the drag law)."""
    return rho_p * np.asarray(d, dtype=np.float64) ** 2 / (18.0 * rho_f * nu)


def friction_velocity(re_tau, nu, R):
    """u* from Re_tau = u* R / nu (pipe radius as the outer scale, Section 2.1)."""
    return re_tau * nu / R


def friction_time(re_tau, nu, R):
    """tau_f = nu / u*^2 (Section 2.1)."""
    us = friction_velocity(re_tau, nu, R)
    return nu / (us * us)


def q_max_charge(d):
    """q_max = 500 * 1.6e-19 * (d / 1e-6)^2 coulomb (Eq. 1)."""
    return 500.0 * 1.6e-19 * (np.asarray(d, dtype=np.float64) / 1e-6) ** 2


# ----------------------------------------------------------------------------- drag

def schiller_naumann(re_p):
    """Drag correction f = 1 + 0.15 Re_p^0.687 (Eq. part_source)."""
    return 1.0 + 0.15 * np.power(np.asarray(re_p, dtype=np.float64), 0.687)


def drag_half_kick(v, u, a, d, h, rho_p, rho_f, nu, drag_on=True):
    """Advance dv/dt = f (u - v) / tau_p + a over a time h with f, u and a frozen.

    Drag law of Eq. part_source with Re_p = |u - v| d / nu.  Reading: the
    integrator is not stated in the paper; the exact exponential solution of
    the linear ODE over the sub-step is used, with the Schiller-Naumann
    factor evaluated at the start of the sub-step.  With drag off this is a
    plain kick v + a h.
    """
    v = np.asarray(v, dtype=np.float64)
    if not drag_on:
        return v + a * h
    w = u - v
    re_p = np.linalg.norm(w, axis=-1) * d / nu
    tau = response_time(d, rho_p, rho_f, nu) / schiller_naumann(re_p)
    v_inf = u + a * tau[:, None]
    return v_inf + (v - v_inf) * np.exp(-h / tau)[:, None]


# ----------------------------------------------------------------------------- Coulomb

def coulomb_pair_accel(r_vec, dist, d_i, d_j, q_i, q_j, m_i, k_e):
    """Acceleration of i due to j: k_e q_i q_j r_ij / (m_i |r_ij| max(|r_ij|, d_ij)^2).

    Eq. coulomb with the centre distance squared (the second of its two printed
    forms) and F_i = sum_j F_ij n_ij (Appendix A.2.4), repulsive for like
    signs.  Reading: the magnitude uses max(|r|, d_ij) with
    d_ij = (d_i + d_j)/2, so overlapping spheres do not see the point-charge
    singularity (exact Gauss's law for non-overlapping uniformly charged
    spheres); pairs at zero distance contribute nothing.
    """
    dij = 0.5 * (d_i + d_j)
    rc = np.maximum(dist, dij)
    with np.errstate(divide="ignore", invalid="ignore"):
        coef = np.where(dist > 0.0, k_e * q_i * q_j / (m_i * dist * rc * rc), 0.0)
    return coef[..., None] * r_vec


# ----------------------------------------------------------------------------- van der Waals

def vdw_equal_printed(delta, d, A):
    """Eq. vdw exactly as printed, for two spheres of the same diameter d at surface gap delta."""
    delta = np.asarray(delta, dtype=np.float64)
    br = delta * (2.0 * d + delta) / (d + delta) ** 2 - 1.0
    return A / 6.0 * d * d * (d + delta) / (delta ** 2 * (2.0 * d + delta) ** 2) * br * br


def hamaker_potential(r, d1, d2, A):
    """Hamaker's interaction energy of two spheres (radii d1/2, d2/2) at centre distance r.

    Reading: the paper prints the pair force only for equal diameters (Eq. vdw);
    for unequal diameters the force is taken as -dU/dr of this potential,
    which reduces to Eq. vdw when d1 = d2.
    """
    R1, R2 = 0.5 * d1, 0.5 * d2
    s, t = R1 + R2, R1 - R2
    P = r * r - s * s
    Q = r * r - t * t
    return -A / 6.0 * (2.0 * R1 * R2 / P + 2.0 * R1 * R2 / Q + np.log(P / Q))


def vdw_hamaker(delta, d1, d2, A):
    """Attractive force magnitude -dU/dr of ``hamaker_potential`` at surface gap delta (four-term form)."""
    delta = np.asarray(delta, dtype=np.float64)
    R1, R2 = 0.5 * np.asarray(d1, dtype=np.float64), 0.5 * np.asarray(d2, dtype=np.float64)
    s, t = R1 + R2, R1 - R2
    r = delta + s
    a = delta * (delta + 2.0 * s)
    b = (delta + s - t) * (delta + s + t)
    return A / 6.0 * (4.0 * R1 * R2 * r / (a * a) + 4.0 * R1 * R2 * r / (b * b) - 2.0 * r / a + 2.0 * r / b)


def vdw_saturation_gap(p):
    """Gap below which the cohesive force is held constant (Section 2.2 and Appendix A.2.3).

    The paper saturates Eq. vdw at delta_min = 1 nm and, for soft spheres,
    modifies the saturation distance so that the cohesive work at contact does
    not depend on the stiffness (k_r / k = 700).  Reading: with the force
    ~ A d / (24 delta^2) near contact, scaling the in-contact force by
    sqrt(k / k_r) is the same as moving the saturation gap to
    delta_min (k_r / k)^(1/4); the Hamaker constant is unchanged.
    """
    if p.get("vdw_gu", True):
        return p["delta_min"] * p["kr_over_k"] ** 0.25
    return p["delta_min"]


def vdw_pair_force(delta, d1, d2, A, delta_sat):
    """Saturated, cut-off pair cohesion: F_H(max(delta, delta_sat)) for delta <= min(d1, d2)/4, else 0."""
    delta = np.asarray(delta, dtype=np.float64)
    cut = 0.25 * np.minimum(d1, d2)
    ds = np.maximum(delta, delta_sat)
    with np.errstate(divide="ignore", invalid="ignore"):
        f = vdw_hamaker(ds, d1, d2, A)
    return np.where(delta <= cut, f, 0.0)


# ----------------------------------------------------------------------------- soft-sphere contact

def contact_coefficients(m_eff, tau_col, e):
    """Linear spring-dashpot stiffness and damping (Appendix A.2.2).

    The paper fixes the restitution coefficient e = 0.9 and the collision time
    tau_col = 15 dt.  Reading: a normal linear spring-dashpot whose contact
    lasts tau_col and rebounds with e: k = m_eff (pi^2 + ln^2 e) / tau_col^2,
    eta = -2 m_eff ln e / tau_col.
    """
    le = np.log(e)
    k = m_eff * (np.pi ** 2 + le * le) / (tau_col * tau_col)
    eta = -2.0 * m_eff * le / tau_col
    return k, eta


# ----------------------------------------------------------------------------- wall terms

def wall_image_accel(h, q, m, k_e):
    """Image-charge attraction toward the wall: k_e q^2 / (2h)^2 / m (Section 2.2; Appendix B.2).

    The image particle of opposite charge sits mirrored across the wall, so the
    wall force is the pair force at twice the centre-to-wall distance h.
    """
    return k_e * q * q / (4.0 * h * h) / m


def wall_vdw_accel(g, d, A, m, delta_sat):
    """Sphere-plane cohesion A d / (12 max(g, delta_sat)^2) / m for gap g <= d/4, else 0 (Appendix B.2).

    Equals twice the small-gap pair force (Section 2.2).  Reading: saturated and
    cut off like the pair force.
    """
    gs = np.maximum(g, delta_sat)
    return np.where(g <= 0.25 * d, A * d / (12.0 * gs * gs) / m, 0.0)


# ----------------------------------------------------------------------------- rebound law

def yield_stress(T):
    """Particle yield stress sigma_y(T) = 200 - 0.225 (T - 1000) MPa (Section 4.4), in Pa.

    Reading: floored at 0.  The paper's input theta = 0.225 (T - 1000) / 200 lies in [0, 1], so the
    law is only defined up to T = 1000 + 200 / 0.225 K, where sigma_y reaches 0; beyond it a negative
    yield stress would square to a spurious elastic rebound."""
    return np.maximum(200.0 - 0.225 * (np.asarray(T, dtype=np.float64) - 1000.0), 0.0) * 1e6


def temperature_of_theta(theta):
    """T = 1000 + 200 theta / 0.225 K, the inverse of theta = 0.225 (T - 1000) / 200 (Section 4.4)."""
    return 1000.0 + 200.0 * np.asarray(theta, dtype=np.float64) / 0.225


def osu_rebound_speed_sq(vn1, T, d, m, A, p):
    """Squared rebound normal speed of the temperature-dependent rebound law (Eq. CoR, Section 4.4).

    sigma_y(T) as ``yield_stress``, gamma_c = A / (24 pi delta_c^2),
    A_cont = acont_coef * pi d^2 / 4.  Reading: the printed CoR does not
    depend on V_n1 for V_n1 below the yield limit (it would exceed 1), so the
    elastic part is capped by the impact energy:
    V_n2^2 = min(V_n1^2, sigma_y^2 / (rho_p E)) - 2 A_cont gamma_c / m.
    The particle sticks when this is <= 0.
    """
    sigma_y = yield_stress(T)
    gamma_c = A / (24.0 * np.pi * p["delta_c"] ** 2)
    a_cont = p["acont_coef"] * np.pi * d * d / 4.0
    return np.minimum(vn1 * vn1, sigma_y * sigma_y / (p["rho_p"] * p["E_young"])) - 2.0 * a_cont * gamma_c / m


def cor_n(vn1, T, d, m, A, p):
    """Normal coefficient of restitution V_n2 / V_n1 of the rebound law (Eq. CoR); 0 means the particle sticks."""
    vn2sq = osu_rebound_speed_sq(vn1, T, d, m, A, p)
    return np.sqrt(np.maximum(vn2sq, 0.0)) / vn1


def capture_efficiency(v_dep_plus_stick, L, D, u_star, u_bulk):
    """CE = (4 L / D) (u* / U_b) V_dep+|stick (Eq. CE): deposited over total particle mass flow rate."""
    return 4.0 * L / D * u_star / u_bulk * v_dep_plus_stick