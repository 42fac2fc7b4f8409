"""Frozen synthetic turbulent pipe field (stand-in for the paper's DNS carrier flow).

The paper's high-fidelity model advances particles through a DNS of turbulent
pipe flow at Re_tau = 180 (Section 2.1, Appendix A.1).  No DNS data exists
here, so the carrier flow is replaced by a seeded, frozen field on a Cartesian
node grid:

* nodes ``x_i = i L / nx`` (periodic in x), ``y_j = -R + 2 R j / (ny - 1)``,
  ``z_k = -R + 2 R k / (nz - 1)``;
* mean streamwise velocity ``U_x = u* U+(y+)`` from Reichardt's law of the
  wall (kappa = 0.41) with ``y+ = (R - r) u*/nu``;
* fluctuations: a sum of ``n_modes`` random Fourier modes
  ``a_m e_m cos(k_m . x + phi_m)`` with ``k_x`` a non-zero integer multiple
  of ``2 pi / L`` (so the field is periodic in x and every mode averages to
  zero along x), amplitude direction ``e_m`` perpendicular to ``k_m``
  (divergence free before the wall envelope), amplitudes from a von Karman
  type spectrum, scaled so that the per-component rms over the pipe interior
  equals ``u*``, and damped by the envelope ``1 - exp(-y+/10)``;
* every node with ``r >= R`` is set to zero (no-slip wall, fluid at rest
  outside the pipe).

The grid is evaluated with dense complex products (the field is separable per
mode in x, y and z), so a 256^3 field takes a few seconds.
"""

from __future__ import annotations

import numpy as np

KAPPA = 0.41


def reichardt_uplus(yplus: np.ndarray) -> np.ndarray:
    """Reichardt's smooth law of the wall U+(y+), valid from the wall to the log layer."""
    yp = np.maximum(np.asarray(yplus, dtype=np.float64), 0.0)
    return (np.log1p(KAPPA * yp) / KAPPA
            + 7.8 * (1.0 - np.exp(-yp / 11.0) - (yp / 11.0) * np.exp(-yp / 3.0)))


def node_coordinates(n: int, R: float, L: float):
    """Node coordinates of the field grid: x periodic over [0, L), y and z spanning [-R, R]."""
    xs = np.arange(n, dtype=np.float64) * (L / n)
    ys = -R + 2.0 * R * np.arange(n, dtype=np.float64) / (n - 1)
    return xs, ys, ys.copy()


def _draw_modes(rng, n: int, R: float, L: float, n_modes: int):
    dx = L / n
    dyz = 2.0 * R / (n - 1)
    k0 = 2.0 * np.pi / L
    kmin = k0
    kmax = np.pi / (2.0 * max(dx, dyz))          # four nodes per shortest wavelength
    ke = 2.0 * np.pi / R                          # energy-containing scale ~ pipe radius
    nx_max = max(1, n // 2 - 1)
    logk = rng.uniform(np.log(kmin), np.log(kmax), n_modes)
    kmag = np.exp(logk)
    cost = rng.uniform(-1.0, 1.0, n_modes)
    phi = rng.uniform(0.0, 2.0 * np.pi, n_modes)
    sint = np.sqrt(1.0 - cost * cost)
    kvec = np.stack([kmag * cost, kmag * sint * np.cos(phi), kmag * sint * np.sin(phi)], axis=1)
    nxi = np.rint(kvec[:, 0] / k0).astype(np.int64)
    nxi = np.where(nxi == 0, np.where(kvec[:, 0] >= 0.0, 1, -1), nxi)
    nxi = np.clip(nxi, -nx_max, nx_max)
    nxi = np.where(nxi == 0, 1, nxi)
    kvec[:, 0] = nxi * k0
    # amplitude direction: a random unit vector projected perpendicular to k
    g = rng.normal(size=(n_modes, 3))
    kh = kvec / np.linalg.norm(kvec, axis=1, keepdims=True)
    e = g - np.sum(g * kh, axis=1, keepdims=True) * kh
    e /= np.linalg.norm(e, axis=1, keepdims=True)
    phase = rng.uniform(0.0, 2.0 * np.pi, n_modes)
    kk = np.linalg.norm(kvec, axis=1)
    spec = (kk / ke) ** 4 / (1.0 + (kk / ke) ** 2) ** (17.0 / 6.0)
    # log-uniform draws have density ~ 1/k, so weight each mode by E(k) k
    amp = np.sqrt(spec * kk)
    return kvec, e, amp, phase


def make_field(n: int, re_tau: float, R: float, L: float, nu: float, seed: int,
               n_modes: int = 256) -> np.ndarray:
    """Return the frozen synthetic field as float64 ``[n, n, n, 3]`` (x, y, z, component; z fastest)."""
    if n < 4:
        raise ValueError("field grid needs at least 4 nodes per axis")
    rng = np.random.default_rng(seed)
    u_star = re_tau * nu / R
    xs, ys, zs = node_coordinates(n, R, L)
    kvec, e, amp, phase = _draw_modes(rng, n, R, L, n_modes)

    X = np.exp(1j * np.outer(xs, kvec[:, 0]))               # (n, M)
    Y = np.exp(1j * np.outer(ys, kvec[:, 1]))               # (n, M)
    Z = np.exp(1j * np.outer(zs, kvec[:, 2]))               # (n, M)
    coef = amp * np.exp(1j * phase)                          # (M,)

    fluct = np.empty((n, n, n, 3), dtype=np.float64)
    for c in range(3):
        cm = coef * e[:, c]                                  # (M,)
        YZc = Y * cm[None, :]                                # (n_y, M)
        for i0 in range(0, n, 16):
            i1 = min(n, i0 + 16)
            # T[i, j, m] = X[i, m] * Y[j, m] * cm[m]; contract m with Z[k, m]
            T = X[i0:i1, None, :] * YZc[None, :, :]          # (b, n_y, M)
            blk = T.reshape(-1, T.shape[-1]) @ Z.T           # (b*n_y, n_z)
            fluct[i0:i1, :, :, c] = blk.real.reshape(i1 - i0, n, n)

    Yg, Zg = np.meshgrid(ys, zs, indexing="ij")
    r = np.sqrt(Yg * Yg + Zg * Zg)
    inside = r < R
    rms = np.sqrt(np.mean(fluct[:, inside, :] ** 2))
    fluct *= u_star / rms
    yplus = (R - r) * u_star / nu
    envelope = np.where(inside, 1.0 - np.exp(-np.maximum(yplus, 0.0) / 10.0), 0.0)
    field = fluct * envelope[None, :, :, None]
    field[:, :, :, 0] += np.where(inside, u_star * reichardt_uplus(yplus), 0.0)[None, :, :]
    field[:, ~inside, :] = 0.0
    return field


def bulk_velocity_plus(re_tau: float, n_r: int = 20001) -> float:
    """Bulk velocity of the Reichardt mean profile in wall units, U_b / u* (area average over the pipe)."""
    s = np.linspace(0.0, 1.0, n_r)                  # r / R
    up = reichardt_uplus((1.0 - s) * re_tau)
    f = up * s
    return float(2.0 * np.sum(0.5 * (f[1:] + f[:-1]) * np.diff(s)))
