"""Physical parameters and seeded particle sets of the benchmark workloads.

Units are SI throughout.  The pipe of the paper (Section 2.1) has diameter
D = 20 mm, air with nu = 1.5e-5 m^2/s, Re_tau = 180; particles are seeded
uniformly in the pipe.  The workloads here use a periodic pipe section of
radius R = D/2 = 10 mm and length L = 4 R, and particle sets of 1k to 1M.

The fluid density is not printed in the paper; 1.2 kg/m^3 reproduces the
printed tau_p+ values of its three particle sizes (Section 2.1).  The time
step is 1e-4 of the response time of a 10 um, 1000 kg/m^3 particle for every
workload but the temperature study.

Workloads (name: content):

* ``plain-1k``: 1,024 particles, d = 10 um, q = +1e-15 C, A = 1e-20 J,
  64^3 field, Re_tau = 180, 200 steps.
* ``plain-1k-dep``: ``plain-1k`` with dt = 3e-5 s (about 0.1 of the 10 um
  particles' response time), so that the 200 steps span 6 ms and some twenty
  particles reach the wall: the deposition tally has something to count.
* ``single-65k``: 65,536 particles, d lognormal(ln 10 um, 0.3),
  q ~ N(0, (2e-15 C)^2), A = 5e-20 J, 128^3 field, all forces, 2,000 steps.
* ``batched-256``: 256 Monte Carlo samples; per sample xi ~ U[0, 0.1],
  zeta ~ U[0, 1] (A = zeta * 1e-18 J), T ~ U[280, 360] K and
  N_s ~ U{2048..32768}; q = xi * q_max(d) (Eq. 1); shared 128^3 field;
  rebound law on; 1,000 steps.
* ``adjoint-64x16k``: 64 samples of 16,384 particles, parameters drawn as in
  ``batched-256``; smoothed deposition tally; 100 steps.
* ``rebound-theta-64``: the temperature study of Section 4.4: 64 samples of
  16,384 particles, xi and zeta as in ``batched-256``, theta ~ U[0, 1]
  (T = 1000 + 200 theta / 0.225 K, 1000 to 1889 K), rebound law on with a
  wall contact area of 1e-3 of the particle cross-section, 128^3 field,
  dt = 1e-5 s (0.05 viscous time units, so that 1,000 steps span ~50 of
  them and several percent of the particles reach the wall); its quantity
  of interest is the capture efficiency.
* ``large-1m``: 1,048,576 particles, d in {1, 5, 10, 20} um equal mix,
  q ~ N(0, (2e-15 C)^2), A = 5e-20 J, 256^3 field at Re_tau = 300, 500 steps.

Every generator takes size overrides so that the same recipe yields the small
instances the parity tests use.
"""

from __future__ import annotations

from dataclasses import dataclass, field as dc_field
from typing import Optional

import numpy as np

R_PIPE = 0.01
L_PIPE = 4.0 * R_PIPE
NU = 1.5e-5
RHO_F = 1.2
RHO_P = 1000.0
# time step: 1e-4 of the response time of a 10 um particle of 1000 kg/m^3
DT = 1e-4 * RHO_P * (10e-6) ** 2 / (18.0 * RHO_F * NU)

FORCE_FLAGS = ("drag", "coulomb", "collide", "vdw", "vdw_gu", "wall_image", "wall_vdw")


def physical_params(re_tau: float = 180.0, **overrides) -> dict:
    """Parameter dictionary (SI) consumed by both the oracle and the library binding."""
    p = dict(
        R=R_PIPE, L=L_PIPE, nu=NU, rho_f=RHO_F, rho_p=RHO_P, dt=DT, re_tau=float(re_tau),
        e_pp=0.9, tau_col_steps=15,
        delta_min=1e-9, kr_over_k=700.0, eps0=8.854e-12,
        g_body=(0.0, 0.0, 0.0),
        E_young=70e9, delta_c=0.165e-9, acont_coef=1.0,
        soft_eps=0.05, soft_tau=10.0,
        drag=True, coulomb=True, collide=True, vdw=True, vdw_gu=True,
        wall_image=True, wall_vdw=True,
        rebound_osu=False, soft_tally=False, body_force=False,
        u_bulk=None,
    )
    for k, v in overrides.items():
        if k not in p:
            raise KeyError(f"unknown parameter {k!r}")
        p[k] = v
    if p["u_bulk"] is None:
        # bulk velocity of the synthetic field's mean profile (its fluctuations have zero mean)
        from .field import bulk_velocity_plus
        p["u_bulk"] = bulk_velocity_plus(p["re_tau"]) * p["re_tau"] * p["nu"] / p["R"]
    return p


def q_max(d: np.ndarray) -> np.ndarray:
    """Maximum particle charge of Eq. (1): 500 elementary charges per um^2 of d^2."""
    return 500.0 * 1.6e-19 * (np.asarray(d) / 1e-6) ** 2


def seed_positions(rng, d: np.ndarray, R: float, L: float) -> np.ndarray:
    """x ~ U[0, L); (y, z) uniform over the disk r <= R - d/2 (no overlap rejection)."""
    n = d.shape[0]
    x = rng.uniform(0.0, L, n)
    rr = (R - 0.5 * d) * np.sqrt(rng.uniform(0.0, 1.0, n))
    ph = rng.uniform(0.0, 2.0 * np.pi, n)
    return np.stack([x, rr * np.cos(ph), rr * np.sin(ph)], axis=1)


@dataclass
class Workload:
    name: str
    params: dict
    field_n: int
    field_seed: int
    steps: int
    offsets: np.ndarray                 # int64 [S+1]
    sample_params: np.ndarray           # float64 [S, 3]: charge_scale, hamaker, temperature
    x: np.ndarray                       # float64 [N, 3]
    d: np.ndarray                       # float64 [N]
    qbase: np.ndarray                   # float64 [N]
    extra: dict = dc_field(default_factory=dict)

    @property
    def n_particles(self) -> int:
        return int(self.offsets[-1])

    @property
    def n_samples(self) -> int:
        return int(self.offsets.shape[0] - 1)

    def field(self) -> np.ndarray:
        from .field import make_field
        p = self.params
        return make_field(self.field_n, p["re_tau"], p["R"], p["L"], p["nu"], self.field_seed)


def _lognormal_d(rng, n):
    return np.exp(rng.normal(np.log(10e-6), 0.3, n))


def _plain_1k(n=1024, steps=200, field_n=64, seed=1, **kw):
    rng = np.random.default_rng(seed)
    p = physical_params(180.0, **kw)
    d = np.full(n, 10e-6)
    x = seed_positions(rng, d, p["R"], p["L"])
    qb = np.full(n, 1e-15)
    sp = np.array([[1.0, 1e-20, 300.0]])
    return Workload("plain-1k", p, field_n, 180, steps, np.array([0, n], np.int64), sp, x, d, qb)


def _plain_1k_dep(dt=3e-5, **kw):
    w = _plain_1k(dt=dt, **kw)
    w.name = "plain-1k-dep"
    return w


def _single_65k(n=65536, steps=2000, field_n=128, seed=2, **kw):
    rng = np.random.default_rng(seed)
    p = physical_params(180.0, **kw)
    d = _lognormal_d(rng, n)
    x = seed_positions(rng, d, p["R"], p["L"])
    qb = rng.normal(0.0, 2e-15, n)
    sp = np.array([[1.0, 5e-20, 300.0]])
    return Workload("single-65k", p, field_n, 180, steps, np.array([0, n], np.int64), sp, x, d, qb)


def _mc_batch(name, seed, n_samples, n_lo, n_hi, steps, field_n, fixed_n=None, theta_range=False, **kw):
    rng = np.random.default_rng(seed)
    p = physical_params(180.0, **kw)
    xi = rng.uniform(0.0, 0.1, n_samples)
    zeta = rng.uniform(0.0, 1.0, n_samples)
    if theta_range:
        temp = 1000.0 + 200.0 * rng.uniform(0.0, 1.0, n_samples) / 0.225
    else:
        temp = rng.uniform(280.0, 360.0, n_samples)
    if fixed_n is None:
        ns = rng.integers(n_lo, n_hi + 1, n_samples)
    else:
        ns = np.full(n_samples, fixed_n, dtype=np.int64)
    offsets = np.concatenate([[0], np.cumsum(ns)]).astype(np.int64)
    d = _lognormal_d(rng, int(offsets[-1]))
    x = seed_positions(rng, d, p["R"], p["L"])
    qb = q_max(d)
    sp = np.stack([xi, zeta * 1e-18, temp], axis=1)
    return Workload(name, p, field_n, 180, steps, offsets, sp, x, d, qb,
                    extra=dict(xi=xi, zeta=zeta, temperature=temp))


def _batched_256(n_samples=256, n_lo=2048, n_hi=32768, steps=1000, field_n=128, seed=3, **kw):
    kw.setdefault("rebound_osu", True)
    return _mc_batch("batched-256", seed, n_samples, n_lo, n_hi, steps, field_n, **kw)


def _adjoint_64x16k(n_samples=64, n_per=16384, steps=100, field_n=128, seed=4, **kw):
    kw.setdefault("rebound_osu", True)
    kw.setdefault("soft_tally", True)
    w = _mc_batch("adjoint-64x16k", seed, n_samples, 0, 0, steps, field_n, fixed_n=n_per, **kw)
    w.extra["ckpt_every"] = 10
    return w


def _large_1m(n=1 << 20, steps=500, field_n=256, seed=5, **kw):
    rng = np.random.default_rng(seed)
    p = physical_params(300.0, **kw)
    d = np.repeat(np.array([1e-6, 5e-6, 10e-6, 20e-6]), (n + 3) // 4)[:n]
    rng.shuffle(d)
    x = seed_positions(rng, d, p["R"], p["L"])
    qb = rng.normal(0.0, 2e-15, n)
    sp = np.array([[1.0, 5e-20, 300.0]])
    return Workload("large-1m", p, field_n, 300, steps, np.array([0, n], np.int64), sp, x, d, qb)


def _rebound_theta_64(n_samples=64, n_per=16384, steps=1000, field_n=128, seed=6, **kw):
    kw.setdefault("rebound_osu", True)
    kw.setdefault("acont_coef", 1e-3)
    kw.setdefault("dt", 1e-5)
    return _mc_batch("rebound-theta-64", seed, n_samples, 0, 0, steps, field_n, fixed_n=n_per,
                     theta_range=True, **kw)


WORKLOADS = {
    "plain-1k": _plain_1k,
    "plain-1k-dep": _plain_1k_dep,
    "single-65k": _single_65k,
    "batched-256": _batched_256,
    "adjoint-64x16k": _adjoint_64x16k,
    "large-1m": _large_1m,
    "rebound-theta-64": _rebound_theta_64,
}


def make_workload(name: str, **overrides) -> Workload:
    """Build a workload by name; keyword overrides change sizes, seeds or physical parameters."""
    if name not in WORKLOADS:
        raise KeyError(f"unknown workload {name!r}; known: {sorted(WORKLOADS)}")
    return WORKLOADS[name](**overrides)
