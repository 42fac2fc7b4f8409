"""The 2^20-particle workload (d in {1, 5, 10, 20} um, Gaussian charges, 256^3 field at Re_tau = 300):
the FP32 Coulomb sums against the FP64 oracle over all 1,048,576 sources (Appendix A.2.4, Eq. coulomb).

One FP32 run of the default configuration (symmetric pair kernel, float source records, every force on)
is taken to steps 0, 250 and 500.  At each of these steps its state is copied (checkpoint blob) into a
second simulation with the Coulomb force alone, whose accelerations of 4,096 targets (index = 0 mod 256)
are evaluated with four pair kernels and compared with the oracle's Coulomb accelerations, in FP64, on the
same snapshot.  Error metric per target: e = |a_gpu - a_oracle| / sum_j |a_ij|.

* Symmetric kernel with integer y/z source records (every coordinate difference exact): e <= 1e-6 against
  the oracle evaluated at the positions the records hold (each coordinate rounded to one x quantum u_x,
  since x is the fixed-point value and y, z are rounded to integers in x quanta): the kernel's own
  arithmetic.  Against the oracle at the snapshot's positions (fixed point plus remainder) that rounding
  adds up to 1.5 u_x / r_nearest (half a quantum per coordinate on the nearest pair's direction):
  e <= 1e-6 + 1.5 u_x / r_nearest.
* Symmetric kernel with float records (the default) and the one-sided Kahan kernel (same records): the
  float records hold y and z in x quanta u_x to 24 bits, a spacing of up to 64 u_x near the wall, so a
  pair at distance r carries a relative error up to ~3 * 64 u_x / r; each target is held to
  1e-6 + 3 * 64 u_x / r_nearest, and the median to 5e-8.
* One-sided kernel with plain (uncompensated) FP32 block sums: reported beside Kahan; the median of the
  compensated errors is not above the plain one.
"""

import sys

import numpy as np
import pytest

from synthetic import make_workload
from tests.gpu_common import oracle_from_snapshot, seeded_pair
from tests.oracle_pool import pooled_force_check

pytestmark = pytest.mark.gpu

TARGETS = np.arange(0, 1 << 20, 256)
KERNELS = {"symmetric-int": (4, 2, 64, 4), "kahan": (1, 16, 32, 1), "plain": (1, 16, 32, 0),
           "symmetric": (4, 2, 64, 2)}   # the default last: the run continues from its evaluation


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


COULOMB_ONLY = dict(drag=False, collide=False, vdw=False, wall_image=False, wall_vdw=False)


@pytest.fixture(scope="module")
def large_run():
    from paper_2205_04979_amd.depo import Simulation
    w = make_workload("large-1m")
    f = w.field()
    say("case: large-1m fp32 default run, seeding 2^20 particles")
    sim, _ = seeded_pair(w.params, f, w.x, w.d, w.qbase, w.offsets, w.sample_params, 4, oracle=False)
    pc = dict(w.params, **COULOMB_ONLY)
    probe = Simulation(pc, w.offsets, f.shape[:3], real_bytes=4)
    probe.init_field(f)
    state = dict(w=w, f=f, sim=sim, probe=probe, pc=pc, step=0, report={})
    yield state
    say("large-1m Coulomb force errors (max, median) per step and kernel:", state["report"])
    probe.close()
    sim.close()


def check_at(state, step):
    w, f, sim, probe = state["w"], state["f"], state["sim"], state["probe"]
    if step > state["step"]:
        for k in range(state["step"], step, 50):
            sim.step(min(50, step - k))
            sim.read()
            say(f"  step {min(k + 50, step)}")
        state["step"] = step
    probe.state_upload(sim.state_download())
    errs = {}
    for name, cfg in KERNELS.items():
        probe.set_kernel_config(*cfg)
        probe.eval_accel()
        g = probe.read()
        if name == "symmetric-int":
            snap = g
            alive = g["dep_step"][TARGETS] == 0
            t = TARGETS[alive]
            ora = oracle_from_snapshot(state["pc"], f, g, w.d, w.qbase, w.offsets, w.sample_params, g["dep_step"])
            chk = pooled_force_check(ora, t)
            a_ora, scale, r_min = chk[:, :3], chk[:, 3], chk[:, 4]
            # the same snapshot at the positions the integer records hold
            ux = w.params["L"] / 2.0 ** 32
            lat = dict(g, x=np.round(g["x"] / ux) * ux)
            lat["x"][:, 0] = np.mod(lat["x"][:, 0], w.params["L"])
            ora_l = oracle_from_snapshot(state["pc"], f, lat, w.d, w.qbase, w.offsets, w.sample_params, g["dep_step"])
            a_lat = pooled_force_check(ora_l, t)[:, :3]
            say(f"step {step}: {t.size} targets, oracle done; nearest source from {r_min.min():.3e} m")
            e_lat = np.linalg.norm(g["a"][t] - a_lat, axis=1) / scale
            say(f"step {step} symmetric-int at the record positions: max {e_lat.max():.3e} "
                f"median {np.median(e_lat):.3e}")
        assert np.array_equal(g["x"], snap["x"]) and np.array_equal(g["v"], snap["v"])
        errs[name] = np.linalg.norm(g["a"][t] - a_ora, axis=1) / scale
        k = int(np.argmax(errs[name]))
        say(f"step {step} {name}: max {errs[name].max():.3e} (target {int(t[k])}, nearest source {r_min[k]:.3e} m) "
            f"median {np.median(errs[name]):.3e}")
    state["report"][step] = {k: (float(v.max()), float(np.median(v))) for k, v in errs.items()}
    state["report"][step]["symmetric-int at the record positions"] = (float(e_lat.max()), float(np.median(e_lat)))
    bound = 1e-6 + 3.0 * 64.0 * ux / r_min
    assert t.size >= 4000
    assert e_lat.max() <= 1e-6
    assert np.all(errs["symmetric-int"] <= 1e-6 + 1.5 * ux / r_min)
    for name in ("symmetric", "kahan"):
        assert np.all(errs[name] <= bound), (name, np.max(errs[name] / bound))
        assert np.median(errs[name]) < 5e-8
    assert np.median(errs["kahan"]) <= np.median(errs["plain"])


def test_large_1m_force_error_step_0(large_run):
    check_at(large_run, 0)


def test_large_1m_force_error_step_250(large_run):
    check_at(large_run, 250)


def test_large_1m_force_error_step_500(large_run):
    check_at(large_run, 500)
