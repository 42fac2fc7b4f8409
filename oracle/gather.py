"""Fluid velocity at the particle, u_f[x_p] (Appendix A.2.1, drag law).

The paper interpolates the fluid velocity to the particle position without
naming the scheme; the reading used here is trilinear interpolation on the
collocated node grid of the synthetic field (periodic in x, clamped cells in
y and z).  Pinned in the tests against ``scipy.interpolate.RegularGridInterpolator``
(method "linear") and against exact reproduction of affine fields.
"""

from __future__ import annotations

import numpy as np


def trilinear(field: np.ndarray, R: float, L: float, pts: np.ndarray) -> np.ndarray:
    """Interpolate ``field[nx, ny, nz, 3]`` (nodes x_i = iL/nx, y_j = -R + 2Rj/(ny-1), same for z) at ``pts[n, 3]``."""
    nx, ny, nz = field.shape[:3]
    pts = np.asarray(pts, dtype=np.float64)
    sx = pts[:, 0] / (L / nx)
    fl = np.floor(sx)
    fx = sx - fl
    ix0 = np.mod(fl.astype(np.int64), nx)
    ix1 = np.mod(ix0 + 1, nx)

    def axis(c, n):
        s = (pts[:, c] + R) / (2.0 * R / (n - 1))
        i0 = np.clip(np.floor(s).astype(np.int64), 0, n - 2)
        f = np.clip(s - i0, 0.0, 1.0)
        return i0, f

    iy0, fy = axis(1, ny)
    iz0, fz = axis(2, nz)
    out = np.zeros((pts.shape[0], 3), dtype=np.float64)
    for cx, wx in ((ix0, 1.0 - fx), (ix1, fx)):
        for cy, wy in ((iy0, 1.0 - fy), (iy0 + 1, fy)):
            for cz, wz in ((iz0, 1.0 - fz), (iz0 + 1, fz)):
                out += (wx * wy * wz)[:, None] * field[cx, cy, cz, :]
    return out
