"""One-dimensional Eulerian deposition model (Appendix B) — test infrastructure.

Equations taken from the paper:

* particle momentum (Eq. mom_modified):
  V dV/dy+ + V/tau_1+ = -d(Rr V'_fy+^2)/dy+ + F_elec+ + F_vdw+;
* constant particle flux (Eq. continuity), D_T = 0 (isothermal):
  V_dep+ = (D_B/nu + eps/nu) d rho+/dy+ + rho+ (-V), the same at every y+;
* kinetic-theory wall condition (Young & Leeming): the diffusive flux at the
  wall equals rho_w V_w (exp(-M^2)/(2 sqrt(pi) M) - (1 - erf M)/2), so the
  total wall flux is the flux of a half-Maxwellian velocity distribution;
* wall forces per unit mass (Appendix B.2): image charge
  -3 q^2 / (8 pi^2 eps0 rho_p d^3 y^2) and sphere-plane cohesion
  -A d / (12 m (y - d/2)^2) with the gap floored at 1e-12 m; scaled to wall
  units by nu / u*^3.

Readings where the paper is silent (the closures are deferred to Guha's
papers, which are not reproduced here; every one is a stated substitute):

* y+ is the particle-centre distance from the wall, from d+/2 (contact) to
  the pipe centre Re_tau; V = -V_py+ >= 0 is the speed toward the wall, with
  V = 0 at the centre; the deposition velocity is the flux toward the wall,
  relative to the centre-line particle density;
* tau_1+ = tau_p+;
* V'_fy+(y+) = 0.005 y+^2 / (1 + 0.002923 y+^2.128) (a near-wall fit of the
  wall-normal fluid rms velocity);
* Rr = 1 / (1 + tau_p+ / tau_L+), tau_L+ = 10 (particle / fluid velocity
  variance ratio), particle rms V'_py+ = sqrt(Rr) V'_fy+;
* eps/nu = tau_L+ Rr V'_fy+^2 (particle eddy diffusivity);
* D_B/nu = k_B T / (3 pi rho_f nu^2 d), T = 293 K;
* the particle wall-normal velocity variance at the wall adds the thermal
  part k_B T / m to the turbulent part: V'_py+^2 = Rr V'_fy+^2 + k_B T / (m u*^2)
  (without it a Brownian particle could never reach the wall);
* M_r = V_w / (sqrt(2) V'_py+(wall)).

Numerics (as the paper describes: near-wall grid refinement, implicit drag):
the momentum equation in K = V^2/2 is marched from the centre to the wall
with the drag term implicit (a quadratic per cell) and the force terms
integrated exactly over each cell; the flux equation is integrated from the
wall outwards with the exact solution of each constant-coefficient cell.

Parity unpinned: the closures are not the paper's, so no printed number can
be reproduced.  Tests check invariants and closed-form limits only.
"""

from __future__ import annotations

import math

import numpy as np

from . import physics as ph

K_B = 1.380649e-23
TAU_L_PLUS = 10.0
G_MIN = 1e-12   # vdW gap floor [m] (Appendix B.2)


def vfy_plus(yp):
    """Wall-normal fluid rms velocity in wall units (substitute closure)."""
    yp = np.asarray(yp, dtype=np.float64)
    return 0.005 * yp ** 2 / (1.0 + 0.002923 * yp ** 2.128)


def momentum(y, Phi, work, tau1):
    """Speed toward the wall V(y) from the momentum equation, marched from the centre (V = 0) to the wall.

    In K = V^2/2 the equation reads dK/ds = G - V / tau1 (s = distance from the centre); per cell
    the drag is implicit (a quadratic in V) and the driving term int G ds = (Phi_k - Phi_{k-1}) + work
    is integrated exactly (``work`` = minus the integral of the attractive force over the cell)."""
    n = y.shape[0]
    V = np.zeros(n)
    K = 0.0
    for k in range(n - 1, 0, -1):
        h = y[k] - y[k - 1]
        rhs = K + (Phi[k] - Phi[k - 1]) + work[k - 1]
        if rhs > 0.0:
            # positive root of v^2/2 + a v = rhs, written without the cancellation of -a + sqrt(a^2 + 2 rhs)
            a = h / tau1
            v = 2.0 * rhs / (a + math.sqrt(a * a + 2.0 * rhs))
        else:
            v = 0.0
        V[k - 1] = v
        K = 0.5 * v * v
    return V


def wall_flux_factor(Vw, vp_w):
    """Flux per unit wall density of a half-Maxwellian: vp e^(-M^2)/sqrt(2 pi) + Vw (1 + erf M)/2, M = Vw/(sqrt2 vp)."""
    if vp_w <= 0.0:
        return Vw
    M = Vw / (math.sqrt(2.0) * vp_w)
    return vp_w * math.exp(-M * M) / math.sqrt(2.0 * math.pi) + Vw * (1.0 + math.erf(M)) / 2.0


def flux(y, V, D, hw):
    """Constant flux toward the wall J = D drho/dy + V rho with rho(centre) = 1 and J = rho_w hw.

    Written rho = rho_w phi, phi(wall) = 1, d phi/dy = (hw - V phi)/D, integrated outwards with the
    exact solution of each cell (V, D frozen at the cell average); J = hw / phi(centre)."""
    n = y.shape[0]
    phi = np.empty(n)
    phi[0] = 1.0
    for k in range(n - 1):
        dy = y[k + 1] - y[k]
        Vm = 0.5 * (V[k] + V[k + 1])
        Dm = 0.5 * (D[k] + D[k + 1])
        x = Vm * dy / Dm
        if x > 0.0:
            # hw/Vm + (phi - hw/Vm) e^-x, arranged so that a tiny drift does not cancel catastrophically
            phi[k + 1] = phi[k] * math.exp(-x) + hw * dy / Dm * (-math.expm1(-x) / x)
        else:
            phi[k + 1] = phi[k] + hw * dy / Dm
    return hw / phi[-1], phi / phi[-1]


def solve(params, d, q, A, n_wall=800, n_core=800, return_profiles=False):
    """V_dep+ of particles of diameter d [m], charge q [C] and Hamaker constant A [J]."""
    R, nu, rho_f, rho_p = params["R"], params["nu"], params["rho_f"], params["rho_p"]
    us = ph.friction_velocity(params["re_tau"], nu, R)
    lw = nu / us                                  # wall unit [m]
    taup_plus = ph.response_time(d, rho_p, rho_f, nu) * us * us / nu
    m = ph.particle_mass(d, rho_p)
    k_e = ph.coulomb_constant(params["eps0"])
    Rr = 1.0 / (1.0 + taup_plus / TAU_L_PLUS)
    db_plus = K_B * 293.0 / (3.0 * math.pi * rho_f * nu * nu * d)   # D_B / nu (Stokes-Einstein)
    yw = 0.5 * d / lw
    yc = R / lw
    # gaps (y - d/2) in wall units: geometric from the 1e-12 m floor to 1, then uniform to the centre
    gw = np.geomspace(G_MIN / lw, 1.0, n_wall)
    gc = np.linspace(1.0, yc - yw, n_core + 1)[1:]
    g = np.concatenate([gw, gc])                  # gap in wall units
    y = yw + g                                    # increasing: wall -> centre
    gap = g * lw                                  # metres (from g itself: y - yw would round away the 1e-12 m gaps)
    ym = y * lw
    Phi = Rr * vfy_plus(y) ** 2
    E = k_e * q * q / (4.0 * m)                   # image:  F = -E / y^2   [m^3/s^2]
    C = A * d / (12.0 * m)                        # vdW:    F = -C / g^2   [m^3/s^2]
    work = (E * (1.0 / ym[:-1] - 1.0 / ym[1:]) + C * (1.0 / gap[:-1] - 1.0 / gap[1:])) / (us * us)
    V = momentum(y, Phi, work, taup_plus)
    D = db_plus + TAU_L_PLUS * Rr * vfy_plus(y) ** 2
    vp_wall = math.sqrt(Rr * float(vfy_plus(y[0])) ** 2 + K_B * 293.0 / (m * us * us))
    hw = wall_flux_factor(V[0], vp_wall)
    vdep, rho = flux(y, V, D, hw)
    if return_profiles:
        return dict(vdep_plus=vdep, y_plus=y, V=V, rho=rho, D=D, h_w=hw, taup_plus=taup_plus)
    return vdep
