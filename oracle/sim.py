"""The particle step of the high-fidelity model, float64 (Appendix A.2, Section 2.1, Eq. 2).

One step advances every alive particle of every Monte Carlo sample; samples
share the carrier field and never interact.  Following Newton's law
(Eq. newtonlaw) the particle feels drag (Eq. part_source), soft-sphere
contact (Appendix A.2.2), van der Waals cohesion (Eq. vdw, Appendix A.2.3)
and Coulomb forces (Eq. coulomb, Appendix A.2.4), plus the wall image charge
and wall cohesion of Section 2.2 / Appendix B.2.  Particles touching the wall
are removed and tallied (Appendix A, "removed after impact").

Reading of the time integrator (not stated in the paper): kick-drift-kick.

1. half kick with the stored non-drag acceleration a^n and u_f(x^n);
2. drift x += dt v, x wrapped into [0, L);
3. wall test: a particle with r + d/2 >= R deposits (all-stick), or, with
   the rebound law on, sticks or reflects (Section 4.4);
4. non-drag acceleration a^{n+1} at the new positions, alive particles only
   (contact damping uses the half-step velocities);
5. half kick with a^{n+1} and u_f(x^{n+1});
6. tally: m_alive_dt += dt * sum of alive masses.

V_dep = J_w / rho_pm (Eq. 2) with J_w = m_dep / (2 pi R L t) and
rho_pm = (m_alive_dt / t) / (pi R^2 L), i.e. V_dep = (R/2) m_dep / m_alive_dt;
V_dep+ = V_dep / u*.

Parity status: each force law and the integrator are pinned in the tests by
closed forms, invariants and brute force (Stokes relaxation, Schiller-Naumann
relaxation, terminal velocity, two-charge energy, momentum, head-on contact,
van der Waals identities, deposition fraction).  The coupled many-particle
trajectory itself has no closed form: parity unpinned beyond those pins.
"""

from __future__ import annotations

import numpy as np

from . import physics as ph
from .gather import trilinear


class OracleSim:
    """Plain float64 simulation of one or more Monte Carlo samples sharing one field."""

    def __init__(self, params: dict, field: np.ndarray, x0, d, qbase, offsets, sample_params, v0=None,
                 evaluate: bool = True):
        """Seed the particles; with ``evaluate`` the initial acceleration a^0 is computed (all pairs)."""
        p = dict(params)
        self.p = p
        self.field = np.asarray(field, dtype=np.float64)
        self.R, self.L, self.dt = float(p["R"]), float(p["L"]), float(p["dt"])
        self.offsets = np.asarray(offsets, dtype=np.int64)
        self.sp = np.asarray(sample_params, dtype=np.float64).reshape(-1, 3)
        S = self.offsets.shape[0] - 1
        if self.sp.shape[0] != S:
            raise ValueError("sample_params must have one row per sample")
        N = int(self.offsets[-1])
        self.sample = np.repeat(np.arange(S), np.diff(self.offsets))
        self.x = np.array(x0, dtype=np.float64).reshape(N, 3)
        self.x[:, 0] = np.mod(self.x[:, 0], self.L)
        self.d = np.array(d, dtype=np.float64).reshape(N)
        self.qbase = np.array(qbase, dtype=np.float64).reshape(N)
        self.m = ph.particle_mass(self.d, p["rho_p"])
        self.k_e = ph.coulomb_constant(p["eps0"])
        self.delta_sat = ph.vdw_saturation_gap(p)
        self.alive = np.ones(N, dtype=bool)
        self.dep_step = np.zeros(N, dtype=np.int64)
        self.ell = np.zeros(N, dtype=np.float64)
        self.nstep = 0
        self.m_dep = np.zeros(S)
        self.n_dep = np.zeros(S, dtype=np.int64)
        self.m_alive_dt = np.zeros(S)
        self.uf = trilinear(self.field, self.R, self.L, self.x)
        self.v = self.uf.copy() if v0 is None else np.array(v0, dtype=np.float64).reshape(N, 3)
        self.a = self.accelerations() if evaluate else np.zeros((N, 3))

    # ------------------------------------------------------------------ per-sample parameters
    @property
    def charge(self):
        return self.sp[self.sample, 0] * self.qbase

    def hamaker(self, i):
        return self.sp[self.sample[i], 1]

    # ------------------------------------------------------------------ forces
    def accelerations(self, targets=None, chunk: int = 256) -> np.ndarray:
        """Non-drag acceleration of each target at the current state (zero for dead targets)."""
        p = self.p
        N = self.x.shape[0]
        tg = np.arange(N) if targets is None else np.asarray(targets, dtype=np.int64)
        out = np.zeros((tg.shape[0], 3))
        q = self.charge
        tau_col = p["tau_col_steps"] * self.dt
        for s in range(self.offsets.shape[0] - 1):
            b, e = int(self.offsets[s]), int(self.offsets[s + 1])
            A = self.sp[s, 1]
            sel = np.nonzero((tg >= b) & (tg < e))[0]
            sel = sel[self.alive[tg[sel]]]
            src = np.arange(b, e)[self.alive[b:e]]
            for c0 in range(0, sel.shape[0], chunk):
                rows = sel[c0:c0 + chunk]
                i = tg[rows]
                r = self.x[i, None, :] - self.x[None, src, :]
                r[..., 0] -= self.L * np.round(r[..., 0] / self.L)
                dist = np.sqrt(np.sum(r * r, axis=-1))
                di, dj = self.d[i][:, None], self.d[src][None, :]
                mi, mj = self.m[i][:, None], self.m[src][None, :]
                acc = np.zeros((i.shape[0], 3))
                if p["coulomb"]:
                    acc += np.sum(ph.coulomb_pair_accel(r, dist, di, dj, q[i][:, None], q[src][None, :],
                                                        mi, self.k_e), axis=1)
                if p["vdw"] or p["collide"]:
                    dij = 0.5 * (di + dj)
                    gap = dist - dij
                    near = (gap <= 0.25 * np.minimum(di, dj)) & (dist > 0.0)
                    if np.any(near):
                        ii, jj = np.nonzero(near)
                        rh = r[ii, jj] / dist[ii, jj][:, None]
                        mi_, mj_ = mi[ii, 0], mj[0, jj]
                        if p["vdw"]:
                            f = ph.vdw_pair_force(gap[ii, jj], di[ii, 0], dj[0, jj], A, self.delta_sat)
                            np.add.at(acc, ii, -(f / mi_)[:, None] * rh)
                        if p["collide"]:
                            ov = gap[ii, jj] < 0.0
                            if np.any(ov):
                                i2, j2, rh2 = ii[ov], jj[ov], rh[ov]
                                meff = mi_[ov] * mj_[ov] / (mi_[ov] + mj_[ov])
                                k, eta = ph.contact_coefficients(meff, tau_col, p["e_pp"])
                                vn = np.sum((self.v[i[i2]] - self.v[src[j2]]) * rh2, axis=1)
                                f = k * (-gap[i2, j2]) - eta * vn
                                np.add.at(acc, i2, (f / mi_[ov])[:, None] * rh2)
                acc += self._wall_accel(i, q[i], A)
                if p.get("body_force", False):
                    acc += np.asarray(p["g_body"], dtype=np.float64)[None, :]
                out[rows] = acc
        return out

    def _wall_accel(self, i, qi, A):
        p = self.p
        y, z = self.x[i, 1], self.x[i, 2]
        rho = np.hypot(y, z)
        acc = np.zeros((i.shape[0], 3))
        if not (p["wall_image"] or p["wall_vdw"]):
            return acc
        di, mi = self.d[i], self.m[i]
        h = np.maximum(self.R - rho, 0.5 * di)        # centre-to-wall distance, never below contact
        g = self.R - rho - 0.5 * di                    # surface gap to the wall
        mag = np.zeros(i.shape[0])
        if p["wall_image"]:
            mag += ph.wall_image_accel(h, qi, mi, self.k_e)
        if p["wall_vdw"]:
            mag += ph.wall_vdw_accel(g, di, A, mi, self.delta_sat)
        ok = rho > 0.0
        acc[ok, 1] = mag[ok] * y[ok] / rho[ok]
        acc[ok, 2] = mag[ok] * z[ok] / rho[ok]
        return acc

    # ------------------------------------------------------------------ time step
    def _kick(self, idx, h):
        p = self.p
        self.v[idx] = ph.drag_half_kick(self.v[idx], self.uf[idx], self.a[idx], self.d[idx], h,
                                        p["rho_p"], p["rho_f"], p["nu"], p["drag"])

    def step(self, n: int = 1):
        p = self.p
        dt = self.dt
        for _ in range(int(n)):
            self.nstep += 1
            al = np.nonzero(self.alive)[0]
            self._kick(al, 0.5 * dt)
            self.x[al] += dt * self.v[al]
            self.x[al, 0] = np.mod(self.x[al, 0], self.L)
            if not p.get("soft_tally", False):
                self._wall_test(al)
            al = np.nonzero(self.alive)[0]
            self.a[al] = self.accelerations(al)
            self.uf[al] = trilinear(self.field, self.R, self.L, self.x[al])
            self._kick(al, 0.5 * dt)
            np.add.at(self.m_alive_dt, self.sample[al], dt * self.m[al])
            if p.get("soft_tally", False):
                self._soft_tally(al)

    def _wall_test(self, al):
        p = self.p
        rho = np.hypot(self.x[al, 1], self.x[al, 2])
        hit = rho + 0.5 * self.d[al] >= self.R
        if not np.any(hit):
            return
        idx, rho_h = al[hit], rho[hit]
        stick = np.ones(idx.shape[0], dtype=bool)
        if p.get("rebound_osu", False):
            er = np.zeros((idx.shape[0], 3))
            er[:, 1] = self.x[idx, 1] / rho_h
            er[:, 2] = self.x[idx, 2] / rho_h
            vn1 = np.sum(self.v[idx] * er, axis=1)
            s = self.sample[idx]
            vn2sq = ph.osu_rebound_speed_sq(vn1, self.sp[s, 2], self.d[idx], self.m[idx], self.sp[s, 1], p)
            stick = vn2sq <= 0.0
            rb = ~stick
            if np.any(rb):
                j = idx[rb]
                self.v[j] -= (vn1[rb] + np.sqrt(vn2sq[rb]))[:, None] * er[rb]
                pen = rho_h[rb] + 0.5 * self.d[j] - self.R
                scale = (rho_h[rb] - 2.0 * pen) / rho_h[rb]
                self.x[j, 1] *= scale
                self.x[j, 2] *= scale
        j = idx[stick]
        self.alive[j] = False
        self.dep_step[j] = self.nstep
        np.add.at(self.m_dep, self.sample[j], self.m[j])
        np.add.at(self.n_dep, self.sample[j], 1)

    def _soft_tally(self, al):
        """Smoothed deposition: l_i += dt sigma(-g_i / eps_s) / tau_s with eps_s = soft_eps d_i, tau_s = soft_tau dt."""
        p = self.p
        rho = np.hypot(self.x[al, 1], self.x[al, 2])
        g = self.R - rho - 0.5 * self.d[al]
        z = -g / (p["soft_eps"] * self.d[al])
        sig = 0.5 * (1.0 + np.tanh(0.5 * z))
        self.ell[al] += self.dt * sig / (p["soft_tau"] * self.dt)

    # ------------------------------------------------------------------ outputs
    def tally(self):
        """Per-sample deposition tally and V_dep (Eq. 2), with the Poisson standard error of V_dep."""
        u_star = ph.friction_velocity(self.p["re_tau"], self.p["nu"], self.R)
        out = []
        for s in range(self.offsets.shape[0] - 1):
            b, e = int(self.offsets[s]), int(self.offsets[s + 1])
            dep = (self.dep_step[b:e] > 0)
            m2 = float(np.sum(self.m[b:e][dep] ** 2))
            vdep = 0.5 * self.R * self.m_dep[s] / self.m_alive_dt[s] if self.m_alive_dt[s] > 0 else 0.0
            se = vdep * np.sqrt(m2) / self.m_dep[s] if self.m_dep[s] > 0 else 0.0
            # capture efficiency (Eq. CE) as the ratio of mass flow rates: deposition m_dep / t over the
            # axial flux of the suspended mass at the bulk velocity, (m_alive_dt / t) U_b / L
            ub = float(self.p.get("u_bulk", 0.0))
            ce = self.m_dep[s] * self.L / (self.m_alive_dt[s] * ub) if (ub > 0 and self.m_alive_dt[s] > 0) else 0.0
            j_soft = float(np.sum(self.m[b:e] * (-np.expm1(-self.ell[b:e]))))
            out.append(dict(m_dep=float(self.m_dep[s]), n_dep=int(self.n_dep[s]),
                            m_alive_dt=float(self.m_alive_dt[s]), t=self.nstep * self.dt,
                            v_dep=vdep, v_dep_plus=vdep / u_star, v_dep_se=se, j_soft=j_soft,
                            n_alive=int(np.sum(self.alive[b:e])), ce=float(ce)))
        return out
