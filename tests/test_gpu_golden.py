"""Trajectory parity against stored FP64-oracle states (Appendix A.2 step sequence, Eq. 2 tally).

The stored states under tests/golden/ were written by tests/golden/make_golden.py, which runs only the
FP64 oracle on the seeded inputs; each file carries a digest of those inputs, checked here.  Metric
(positions): max over the particles alive in both runs of |x_gpu - x_oracle| / R (minimum image in x);
particles whose deposition step differs are left out of it and counted.
"""

import os
import sys

import numpy as np
import pytest

from synthetic import make_workload
from tests.gpu_common import position_error, seeded_pair
from tests.golden.make_golden import input_digest

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def load(name, w, f):
    path = os.path.join(GOLDEN, name)
    gold = np.load(path)
    assert str(gold["digest"]) == input_digest(w, f), f"{name} was made from other inputs; rerun make_golden.py"
    return gold


def compare(g, gold, w, tol_x, max_event_diff):
    R, L = w.params["R"], w.params["L"]
    dep_o = gold["dep_step"]
    both = (g["dep_step"] == 0) & (dep_o == 0)
    n_diff = int(np.sum(g["dep_step"] != dep_o))
    err = position_error(g["x"][both], gold["x"][both], L, R)
    vmax = np.abs(gold["v"][both]).max()
    dv = np.abs(g["v"][both] - gold["v"][both]).max() / vmax
    say(f"alive in both {int(both.sum())}, deposited (oracle) {int((dep_o > 0).sum())}, event differences {n_diff}, "
        f"max |dx|/R {err.max():.3e}, median {np.median(err):.3e}, max |dv|/max|v| {dv:.3e}")
    assert n_diff <= max_event_diff
    assert err.max() < tol_x
    return err, dv


@pytest.mark.parametrize("real_bytes", [4, 8])
def test_single_65k_20_steps_against_stored_oracle(real_bytes):
    """The headline workload (65,536 particles, lognormal diameters, Gaussian charges, 128^3 field, all
    forces) through 20 steps of the default stepping path (captured step graph; FP32: symmetric pair kernel
    (4, 2)), every particle against the stored FP64-oracle state.  FP32: positions within 1e-5 R, at most 2
    particles with a different deposition step, velocities within 1e-5 of the largest.  FP64: positions
    within 1e-12 R, identical deposition steps, velocities within 1e-12 of the largest."""
    w = make_workload("single-65k")
    f = w.field()
    gold = load("single65k_fp64_step20.npz", w, f)
    steps = int(gold["steps"])
    say(f"case: single-65k, {steps} steps against the stored oracle state, fp{8 * real_bytes}")
    sim, _ = seeded_pair(w.params, f, w.x, w.d, w.qbase, w.offsets, w.sample_params, real_bytes, oracle=False)
    sim.step(steps)
    g = sim.read()
    if real_bytes == 4:
        err, dv = compare(g, gold, w, 1e-5, 2)
        assert dv < 1e-5
    else:
        err, dv = compare(g, gold, w, 1e-12, 0)
        assert dv < 1e-12


def test_large_recipe_4096_particles_500_steps_against_stored_oracle():
    """4,096 particles drawn by the 2^20-particle recipe (d in {1, 5, 10, 20} um, 256^3 field at
    Re_tau = 300) through 500 steps of the FP32 default path, every particle against the stored
    FP64-oracle state: positions within 1e-5 R, at most 2 particles with a different deposition step."""
    w = make_workload("large-1m", n=4096)
    f = w.field()
    gold = load("large1m_n4096_fp64_step500.npz", w, f)
    steps = int(gold["steps"])
    say(f"case: large-1m recipe, 4,096 particles, {steps} steps fp32")
    sim, _ = seeded_pair(w.params, f, w.x, w.d, w.qbase, w.offsets, w.sample_params, 4, oracle=False)
    for _ in range(steps // 100):
        sim.step(100)
    sim.step(steps % 100)
    compare(sim.read(), gold, w, 1e-5, 2)
