"""Small builders of hand-made particle sets for the oracle pins (test code only)."""

import numpy as np

from synthetic.workloads import physical_params


def quiet_params(**kw):
    """All forces off; individual tests switch on what they pin."""
    base = dict(drag=False, coulomb=False, collide=False, vdw=False, vdw_gu=True,
                wall_image=False, wall_vdw=False, rebound_osu=False, soft_tally=False)
    base.update(kw)
    return physical_params(180.0, **base)


def uniform_field(n, U):
    f = np.zeros((n, n, n, 3))
    f[..., 0], f[..., 1], f[..., 2] = U
    return f


def one_sample(n):
    return np.array([0, n], dtype=np.int64)
