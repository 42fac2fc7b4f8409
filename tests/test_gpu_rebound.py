"""Temperature study (Section 4.4): the rebound law over theta in [0, 1] and the capture efficiency
(Eqs. CoR and CE) on the HIP path, against the FP64 oracle."""

import sys

import numpy as np
import pytest

from synthetic import make_workload
from synthetic.workloads import physical_params, q_max
from tests.gpu_common import near_wall_particles, position_error, seeded_pair

pytestmark = pytest.mark.gpu

T_MELT = 1000.0 + 200.0 / 0.225


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def theta_grid_case(n=150, seed=21):
    """Six samples of one near-wall particle set driven at the wall with normal speeds of 0.1-3 m/s,
    so that the yield speed 23.9 (1 - theta) m/s falls inside the impact-speed range for the top
    temperatures; the cohesion term ranges from none to sticking below ~0.3 m/s."""
    rng = np.random.default_rng(seed)
    p = physical_params(180.0, rebound_osu=True, acont_coef=1e-3, dt=2e-7)
    d1 = rng.choice([5e-6, 10e-6], n)
    x1, er = near_wall_particles(rng, n, p, d1, band=100e-6)
    v1 = rng.uniform(0.1, 3.0, n)[:, None] * er + rng.normal(0, 0.05, (n, 3))
    temps = np.array([1000.0, 1500.0, 1850.0, 1870.0, 1880.0, T_MELT + 0.5])
    zetas = np.array([0.0, 0.3, 0.05, 0.0, 0.2, 0.5])
    S = temps.size
    sp = np.stack([np.full(S, 0.02), zetas * 1e-18, temps], 1)
    x, d, v = np.tile(x1, (S, 1)), np.tile(d1, S), np.tile(v1, (S, 1))
    f = make_workload("plain-1k", n=4, field_n=32).field()
    return p, f, x, d, q_max(d), np.arange(S + 1) * n, sp, v


def test_fp64_theta_grid_matches_oracle():
    p, f, x, d, q, off, sp, v = theta_grid_case()
    say("case: rebound theta grid fp64, 6 samples x 150, 60 steps")
    sim, ora = seeded_pair(p, f, x, d, q, off, sp, 8, v0=v)
    sim.step(60)
    ora.step(60)
    g = sim.read()
    assert np.array_equal(g["dep_step"], ora.dep_step)
    tg, to = sim.tally(), ora.tally()
    for s in range(sp.shape[0]):
        assert tg[s]["n_dep"] == to[s]["n_dep"]
        for k in ("m_dep", "m_alive_dt", "v_dep_plus", "ce"):
            assert np.isclose(tg[s][k], to[s][k], rtol=1e-13, atol=0), (s, k)
    al = ora.alive
    assert np.max(position_error(g["x"][al], ora.x[al], ora.L, ora.R)) < 1e-11
    n_dep = [t["n_dep"] for t in tg]
    say("n_dep per sample", n_dep, "ce", [t["ce"] for t in tg])
    # no cohesion and theta < 1: V_n2 = min(V_n1, V_y) > 0, every impact rebounds
    assert n_dep[0] == 0 and n_dep[3] == 0
    assert n_dep[-1] > n_dep[4] > 0            # theta = 1 sticks everything; 1880 K the slow impacts


def test_fp32_theta_grid_within_error_bars():
    p, f, x, d, q, off, sp, v = theta_grid_case()
    say("case: rebound theta grid fp32")
    sim, ora = seeded_pair(p, f, x, d, q, off, sp, 4, v0=v)
    sim.step(60)
    ora.step(60)
    tg, to = sim.tally(), ora.tally()
    for s in range(sp.shape[0]):
        se = max(tg[s]["v_dep_se"], to[s]["v_dep_se"])
        assert abs(tg[s]["v_dep"] - to[s]["v_dep"]) <= se + 1e-30, s
        ce_se = tg[s]["ce"] * (se / tg[s]["v_dep"]) if tg[s]["v_dep"] > 0 else 0.0
        assert abs(tg[s]["ce"] - to[s]["ce"]) <= ce_se + 1e-30, s


def test_theta_study_full_size_melt_equals_all_stick():
    """At the study's full size (64 x 16,384, FP32, the launch the benchmark times): with every
    temperature at theta = 1 the rebound law sticks every impact, so the run is bit-identical to the
    all-stick run."""
    base = make_workload("rebound-theta-64")
    f = base.field()
    n_steps = 300
    res = {}
    for key in ("sampled", "melt", "stick"):
        w = make_workload("rebound-theta-64", rebound_osu=(key != "stick"))
        sp = w.sample_params.copy()
        if key == "melt":
            sp[:, 2] = T_MELT + 0.5
        say("case: rebound-theta-64 full size,", key, n_steps, "steps")
        sim, _ = seeded_pair(w.params, f, w.x, w.d, w.qbase, w.offsets, sp, 4, oracle=False)
        sim.step(n_steps)
        res[key] = (sim.read()["dep_step"], sim.tally())
        sim.close()
    assert np.array_equal(res["melt"][0], res["stick"][0])
    assert res["melt"][1] == res["stick"][1]
    n_stick = np.array([t["n_dep"] for t in res["stick"][1]])
    n_samp = np.array([t["n_dep"] for t in res["sampled"][1]])
    say("deposits all-stick", int(n_stick.sum()), "sampled theta", int(n_samp.sum()))
    assert n_stick.sum() > 0
