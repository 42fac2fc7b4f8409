"""Particle-particle particle-mesh electrostatics (Appendix A.2.4, Eq. coulomb_force) — test infrastructure.

The paper computes the Coulomb field with Hockney's P3M method: the interaction
is split at a cutoff radius into a short-range part summed directly and a
long-range part solved with FFTs on a mesh, at O(N log N) cost.  The paper
defers the details (and its non-periodic extension) to other publications;
this module states its own reading:

* Geometry: the pipe section is periodic in x with period L and unbounded in
  y and z (free space: the wall is not a conductor; its image-charge force is
  a separate wall term).  The quantity computed is therefore the 1-periodic
  lattice sum
      S_i = sum_j q~_j sum_n (r_ij + n L e_x) / |r_ij + n L e_x|^3,
  where the nearest-image term of an overlapping pair uses the overlap clamp
  r / (|r| max(|r|, d_ij)^2) of the direct sum.  (The direct kernels keep the
  nearest image only; the lattice sum adds every further image.)
* Split (Ewald/Gaussian): 1/r = erfc(alpha r)/r + erf(alpha r)/r.  The field of
  the erf part of one unit charge, E_l(r) = r_hat [erf(alpha r)/r^2 -
  (2 alpha / sqrt(pi)) exp(-alpha^2 r^2) / r], is smooth and goes to the mesh;
  the rest, E_s = (Coulomb) - E_l, vanishes beyond r_max and is summed over
  nearest-image pairs closer than r_max.
* Mesh: nx nodes along x at x_i = i hx (hx = L / nx, periodic); nc nodes across
  [-R, R] in y and z at y_j = -R + (j - 1) hy, hy = 2R / (nc - 3), so that a
  particle's 3-point stencil stays inside; zero-padded to P = 2 nc for the
  aperiodic convolution.
* Charge assignment and field interpolation: triangular-shaped cloud (TSC), the
  same weights both ways.
* Green's function: E_l sampled on the padded mesh and summed over the x images
  n = -M..M (pairs of images cancel to O(n^-3), M = 256), transformed, and
  divided by the square of the TSC transfer function sinc^3 per axis
  (deconvolution of assignment and interpolation).
* Convolution: E_mesh = IFFT(FFT(rho) * G_hat), one inverse transform per
  component.

Pins (tests/test_oracle_p3m.py): the brute-force lattice sum is checked by
image-count convergence, periodicity, Newton's third law and the
single-image limit; P3M is checked against it (relative RMS error of the field
below a bound that shrinks with mesh refinement), and its parts by closed forms
(the erf/erfc split reassembles Coulomb's law, the TSC weights sum to one and
reproduce the first moment).
"""

from __future__ import annotations

import math

import numpy as np
from scipy.special import erf, erfc

M_IMAGES = 256


# ----------------------------------------------------------------------------- exact lattice sum

def lattice_sum(x, q, d, L, images=2000):
    """Brute-force S_i = sum_j q_j sum_n r_n / |r_n|^3 over x images |n| <= images (nearest image clamped).

    x: (N, 3) positions [m] with x[:, 0] in [0, L); q: scaled charges; d: diameters [m]."""
    x = np.asarray(x, dtype=np.float64)
    n = x.shape[0]
    S = np.zeros((n, 3))
    shifts = np.arange(-images, images + 1, dtype=np.float64) * L
    for i in range(n):
        r = x[i] - x
        r[:, 0] -= L * np.round(r[:, 0] / L)           # nearest image first
        dij = 0.5 * (d[i] + d)
        mask = np.arange(n) != i
        # nearest image with the overlap clamp
        rr = np.sqrt(np.sum(r * r, axis=1))
        rc = np.maximum(rr, dij)
        with np.errstate(divide="ignore", invalid="ignore"):
            w = np.where(mask & (rr > 0), q / (rr * rc * rc), 0.0)
        S[i] += (w[:, None] * r).sum(axis=0)
        # further images (n != 0), summed in symmetric pairs
        for j in np.nonzero(mask)[0]:
            rx = r[j, 0] + shifts
            rx = rx[shifts != 0.0]
            rho2 = r[j, 1] ** 2 + r[j, 2] ** 2
            inv3 = (rx * rx + rho2) ** -1.5
            S[i, 0] += q[j] * np.sum(rx * inv3)
            S[i, 1] += q[j] * r[j, 1] * np.sum(inv3)
            S[i, 2] += q[j] * r[j, 2] * np.sum(inv3)
    return S


# ----------------------------------------------------------------------------- split kernels

def long_field(r_vec, alpha):
    """E_l(r) of a unit charge: r_hat [erf(a r)/r^2 - (2a/sqrt(pi)) exp(-a^2 r^2)/r]; 0 at r = 0."""
    r_vec = np.asarray(r_vec, dtype=np.float64)
    r = np.sqrt(np.sum(r_vec * r_vec, axis=-1))
    with np.errstate(divide="ignore", invalid="ignore"):
        mag = erf(alpha * r) / r ** 2 - 2.0 * alpha / math.sqrt(math.pi) * np.exp(-(alpha * r) ** 2) / r
        out = np.where(r[..., None] > 0, (mag / r)[..., None] * r_vec, 0.0)
    return out


def short_field_mag(r, alpha):
    """|E_s| of a unit charge for non-overlapping pairs: erfc(a r)/r^2 + (2a/sqrt(pi)) exp(-a^2 r^2)/r."""
    return erfc(alpha * r) / r ** 2 + 2.0 * alpha / math.sqrt(math.pi) * np.exp(-(alpha * r) ** 2) / r


# ----------------------------------------------------------------------------- mesh

class Mesh:
    """Mesh geometry for a pipe section of radius R and period L (see the module docstring)."""

    def __init__(self, R, L, nx, nc, alpha_h, rmax_alpha):
        self.R, self.L, self.nx, self.nc = float(R), float(L), int(nx), int(nc)
        self.P = 2 * self.nc
        self.hx = self.L / self.nx
        self.hy = 2.0 * self.R / (self.nc - 3)
        self.alpha = alpha_h / max(self.hx, self.hy)
        self.rmax = rmax_alpha / self.alpha

    def grid_coords(self, x):
        """Continuous mesh coordinates (gx periodic in [0, nx); gy, gz in [1, nc - 2])."""
        gx = np.mod(x[:, 0] / self.hx, self.nx)
        gy = (x[:, 1] + self.R) / self.hy + 1.0
        gz = (x[:, 2] + self.R) / self.hy + 1.0
        return gx, gy, gz


def tsc_weights(g):
    """Nearest node i = round(g) and the TSC weights of nodes i - 1, i, i + 1."""
    i = np.floor(g + 0.5)
    dl = g - i
    w = np.stack([0.5 * (0.5 - dl) ** 2, 0.75 - dl ** 2, 0.5 * (0.5 + dl) ** 2], axis=-1)
    return i.astype(np.int64), w


def assign(mesh, x, q):
    """Charge on the padded mesh (nx, P, P): TSC of every particle's q."""
    rho = np.zeros((mesh.nx, mesh.P, mesh.P))
    gx, gy, gz = mesh.grid_coords(x)
    ix, wx = tsc_weights(gx)
    iy, wy = tsc_weights(gy)
    iz, wz = tsc_weights(gz)
    for a in range(3):
        for b in range(3):
            for c in range(3):
                w = wx[:, a] * wy[:, b] * wz[:, c] * q
                np.add.at(rho, (np.mod(ix + a - 1, mesh.nx), iy + b - 1, iz + c - 1), w)
    return rho


def interpolate(mesh, E, x):
    """TSC interpolation of the three field components E[c] (padded mesh) at the particles."""
    gx, gy, gz = mesh.grid_coords(x)
    ix, wx = tsc_weights(gx)
    iy, wy = tsc_weights(gy)
    iz, wz = tsc_weights(gz)
    out = np.zeros((x.shape[0], 3))
    for a in range(3):
        for b in range(3):
            for c in range(3):
                w = wx[:, a] * wy[:, b] * wz[:, c]
                idx = (np.mod(ix + a - 1, mesh.nx), iy + b - 1, iz + c - 1)
                for comp in range(3):
                    out[:, comp] += w * E[comp][idx]
    return out


def green_hat(mesh):
    """FFT of the image-summed long-range field on the padded mesh, divided by the squared TSC transfer."""
    nx, P = mesh.nx, mesh.P
    ix = np.arange(nx)
    dx = ix * mesh.hx
    dx = np.where(dx >= 0.5 * mesh.L, dx - mesh.L, dx)
    iy = np.arange(P)
    dy = np.where(iy < P // 2, iy, iy - P) * mesh.hy
    DX, DY, DZ = np.meshgrid(dx, dy, dy, indexing="ij")
    G = np.zeros((3, nx, P, P))
    for n in range(-M_IMAGES, M_IMAGES + 1):
        r = np.stack([DX + n * mesh.L, DY, DZ], axis=-1)
        G += np.moveaxis(long_field(r, mesh.alpha), -1, 0)
    kx = np.fft.fftfreq(nx)          # cycles per node
    ky = np.fft.fftfreq(P)
    sx = np.sinc(kx) ** 3            # numpy sinc(u) = sin(pi u) / (pi u): TSC transfer per axis
    sy = np.sinc(ky) ** 3
    W = sx[:, None, None] * sy[None, :, None] * sy[None, None, :]
    return np.fft.fftn(G, axes=(1, 2, 3)) / (W * W)[None]


def mesh_field(mesh, x, q, ghat=None):
    """Long-range part of S at the particles: interpolate IFFT(FFT(rho) G_hat)."""
    ghat = green_hat(mesh) if ghat is None else ghat
    rho_hat = np.fft.fftn(assign(mesh, x, q))
    E = [np.real(np.fft.ifftn(rho_hat * ghat[c])) for c in range(3)]
    return interpolate(mesh, E, x)


def short_range(mesh, x, q, d, targets=None):
    """Short-range part over nearest-image pairs closer than r_max: Coulomb (overlap clamp) minus E_l.
    Rows for every particle, or for the particles listed in ``targets`` (every particle is a source)."""
    n = x.shape[0]
    targets = np.arange(n) if targets is None else np.asarray(targets, dtype=np.int64)
    S = np.zeros((targets.shape[0], 3))
    a = mesh.alpha
    for k, i in enumerate(targets):
        r = x[i] - x
        r[:, 0] -= mesh.L * np.round(r[:, 0] / mesh.L)
        rr = np.sqrt(np.sum(r * r, axis=1))
        sel = (rr < mesh.rmax) & (np.arange(n) != i) & (rr > 0)
        if not np.any(sel):
            continue
        rs, qs = rr[sel], q[sel]
        dij = 0.5 * (d[i] + d[sel])
        full = 1.0 / np.maximum(rs, dij) ** 2
        lng = erf(a * rs) / rs ** 2 - 2.0 * a / math.sqrt(math.pi) * np.exp(-(a * rs) ** 2) / rs
        S[k] += ((qs * (full - lng) / rs)[:, None] * r[sel]).sum(axis=0)
    return S


def p3m_sums(mesh, x, q, d, ghat=None):
    """S_i of the lattice sum by P3M: mesh (long range) plus direct short range."""
    x = np.asarray(x, dtype=np.float64)
    return mesh_field(mesh, x, q, ghat) + short_range(mesh, x, q, d)
