"""GPU parity of the HIP path (through the C-ABI) against the FP64 oracle.

FP64 runs are compared at round-off tolerances; the FP32 form is compared at
the stated error bars: positions within 1e-5 R after 200 steps, force error
relative to the sum of pair magnitudes within 1e-5, V_dep within its Monte
Carlo standard error.  Particles whose discrete events differ between the two
runs (deposition step) are excluded from position metrics and counted.
"""

import sys

import numpy as np
import pytest

from oracle.sim import OracleSim
from synthetic import make_workload
from synthetic.workloads import physical_params
from tests.gpu_common import (coulomb_scale, force_error, near_wall_particles, oracle_from_snapshot,
                              position_error, seeded_pair)
from tests.oracle_helpers import uniform_field

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


# ------------------------------------------------------------------------------------------ FP64 parity

def test_fp64_plain_trajectory_matches_oracle():
    w = make_workload("plain-1k", n=320, field_n=32)
    f = w.field()
    say("case: plain-1k n=320 fp64")
    sim, ora = seeded_pair(w.params, f, w.x, w.d, w.qbase, w.offsets, w.sample_params, 8)
    g = sim.read()
    scale = np.linalg.norm(ora.a, axis=1).max()
    assert np.max(np.abs(g["a"] - ora.a)) <= 1e-10 * scale
    assert np.max(np.abs(g["v"] - ora.v)) <= 1e-12
    for chunk in (1, 4, 15):
        sim.step(chunk)
        ora.step(chunk)
    g = sim.read()
    assert np.array_equal(g["dep_step"], ora.dep_step)
    al = ora.alive
    assert np.max(position_error(g["x"][al], ora.x[al], ora.L, ora.R)) < 1e-12
    assert np.max(np.abs(g["v"][al] - ora.v[al])) < 1e-9
    assert np.max(np.abs(g["a"][al] - ora.a[al])) <= 1e-9 * scale


def test_fp64_dense_cluster_contacts_and_neighbours():
    """Tight cluster across the periodic seam next to the wall: contact, cohesion and Coulomb all active;
    the cell-list neighbour counts equal brute force exactly."""
    rng = np.random.default_rng(21)
    n = 300
    p = physical_params(180.0)
    R, L = p["R"], p["L"]
    d = rng.choice([5e-6, 10e-6, 20e-6], n)
    x = np.stack([np.mod(rng.normal(0.0, 50e-6, n), L), R - 0.4e-3 + rng.normal(0, 50e-6, n),
                  rng.normal(0, 50e-6, n)], 1)
    q = rng.normal(0, 2e-15, n)
    v0 = rng.normal(0, 0.05, (n, 3))
    sp = np.array([[1.0, 2e-19, 300.0]])
    f = make_workload("plain-1k", n=4, field_n=16).field()
    off = np.array([0, n])
    say("case: dense cluster n=300 fp64")
    sim, ora = seeded_pair(p, f, x, d, q, off, sp, 8, v0=v0)
    g = sim.read()
    # brute-force neighbour counts (gap <= min(d_i, d_j)/4)
    r = x[:, None, :] - x[None, :, :]
    r[..., 0] -= L * np.round(r[..., 0] / L)
    dist = np.linalg.norm(r, axis=-1)
    gap = dist - 0.5 * (d[:, None] + d[None, :])
    near = (gap <= 0.25 * np.minimum(d[:, None], d[None, :])) & (dist > 0)
    assert np.array_equal(g["neighbours"], near.sum(axis=1))
    assert near.sum() > 50 and (gap[near] < 0).sum() > 10
    scale = np.linalg.norm(ora.a, axis=1)
    assert np.max(np.linalg.norm(g["a"] - ora.a, axis=1) / (scale + 1e-30)) < 1e-9
    sim.step(30)
    ora.step(30)
    g = sim.read()
    assert np.array_equal(g["dep_step"], ora.dep_step)
    al = ora.alive
    assert np.max(position_error(g["x"][al], ora.x[al], L, R)) < 1e-10
    assert np.max(np.linalg.norm(g["a"][al] - ora.a[al], axis=1) / (np.linalg.norm(ora.a[al], axis=1) + 1e-3)) < 1e-7


@pytest.mark.parametrize("real_bytes", [8, 4])
def test_seed_without_velocity_ignores_stale_workspace(real_bytes):
    """Seeding with v^0 = u_f(x^0) into a workspace that holds NaN bytes from earlier use: the first
    force evaluation (collision damping reads the neighbours' v^0) equals the oracle's."""
    import torch
    from oracle.sim import OracleSim
    from tests.gpu_common import make_sim
    rng = np.random.default_rng(23)
    n = 300
    p = physical_params(180.0)
    R, L = p["R"], p["L"]
    d = rng.choice([5e-6, 10e-6, 20e-6], n)
    x = np.stack([np.mod(rng.normal(0.0, 50e-6, n), L), R - 0.4e-3 + rng.normal(0, 50e-6, n),
                  rng.normal(0, 50e-6, n)], 1)
    q = rng.normal(0, 2e-15, n)
    sp = np.array([[1.0, 2e-19, 300.0]])
    f = make_workload("plain-1k", n=4, field_n=16).field()
    off = np.array([0, n])
    say("case: stale-workspace seed n=300, real_bytes", real_bytes)
    probe = make_sim(p, off, f, real_bytes)
    nbytes = probe._ws.numel()
    del probe
    torch.cuda.synchronize()
    # a block of the workspace's own size, filled with NaN bytes and returned to the caching allocator
    dirty = torch.full((nbytes,), 0xFF, dtype=torch.uint8, device="cuda")
    lo, hi = dirty.data_ptr(), dirty.data_ptr() + dirty.numel()
    torch.cuda.synchronize()
    del dirty
    sim = make_sim(p, off, f, real_bytes)
    if not (lo <= sim._ws.data_ptr() < hi):
        pytest.skip("the caching allocator did not hand back the dirtied block")
    sim.init_field(f)
    sim.seed(sp, x, d, q)
    ora = OracleSim(p, f, x, d, q, off, sp)
    g = sim.read()
    r = x[:, None, :] - x[None, :, :]
    r[..., 0] -= L * np.round(r[..., 0] / L)
    gap = np.linalg.norm(r, axis=-1) - 0.5 * (d[:, None] + d[None, :])
    assert (gap[np.triu_indices(n, 1)] < 0).sum() > 10       # overlapping pairs: damping is active
    assert np.all(np.isfinite(g["a"])) and np.all(np.isfinite(g["v"]))
    scale = np.linalg.norm(ora.a, axis=1)
    if real_bytes == 8:
        assert np.max(np.linalg.norm(g["a"] - ora.a, axis=1) / (scale + 1e-30)) < 1e-9
        assert np.max(np.abs(g["v"] - ora.v)) <= 1e-12
    else:
        assert np.max(np.linalg.norm(g["a"] - ora.a, axis=1) / (scale + 1e-3 * scale.max())) < 1e-4
        assert np.max(np.abs(g["v"] - ora.v)) <= 1e-5 * np.abs(ora.v).max()


def _cell_grid(R, L, n, reach):
    """The short-range cell grid the library builds for one sample (cells sized for about one particle)."""
    h = max(reach, (4.0 * R * R * L / max(n, 1)) ** (1.0 / 3.0))
    while True:
        ncx = max(3, int(np.floor(L / h)))
        ncy = max(1, int(np.floor(2.0 * R / h)))
        if ncx * ncy * ncy <= n + 64:
            return ncx, ncy
        h *= 1.05


@pytest.mark.parametrize("real_bytes", [8, 4])
def test_short_range_pairs_across_cell_faces(real_bytes):
    """Pairs straddling x, y and z cell faces (and the periodic seam), closer to the face than the reach:
    the walk visits a neighbour cell only when the face is within the reach, and still finds every pair
    (counts equal brute force; pairs well outside the range are not counted); accelerations match the oracle."""
    rng = np.random.default_rng(31)
    p = physical_params(180.0)
    R, L = p["R"], p["L"]
    n_pairs, n_free = 150, 100
    n = 2 * n_pairs + n_free
    d = np.full(n, 10e-6)
    reach = 1.25 * d.max()
    ncx, ncy = _cell_grid(R, L, n, reach)
    hx, hy = L / ncx, 2 * R / ncy
    x = np.zeros((n, 3))
    gaps = np.where(np.arange(n_pairs) % 3 == 2, rng.uniform(0.3, 0.6, n_pairs), rng.uniform(-0.05, 0.2, n_pairs)) * d[0]
    for k in range(n_pairs):
        axis = k % 3
        c = np.array([rng.uniform(0, L), rng.uniform(-0.5 * R, 0.5 * R), rng.uniform(-0.5 * R, 0.5 * R)])
        if axis == 0:
            c[0] = rng.integers(0, ncx) * hx                       # includes the seam x = 0
        else:
            j = rng.integers(ncy // 4, 3 * ncy // 4 + 1)
            c[axis] = -R + j * hy
        # a face point c; the pair centre straddles it, direction mostly across the face
        u = rng.normal(0, 0.3, 3)
        u[axis] = 1.0 if rng.random() < 0.5 else -1.0
        u /= np.linalg.norm(u)
        sep = d[0] + gaps[k]
        off = rng.uniform(0.1, 0.9) * sep
        x[2 * k] = c + u * off
        x[2 * k + 1] = c - u * (sep - off)
    x[2 * n_pairs:] = np.stack([rng.uniform(0, L, n_free), rng.uniform(-0.6 * R, 0.6 * R, n_free),
                                rng.uniform(-0.6 * R, 0.6 * R, n_free)], 1)
    x[:, 0] = np.mod(x[:, 0], L)
    q = rng.normal(0, 2e-15, n)
    sp = np.array([[1.0, 2e-19, 300.0]])
    f = make_workload("plain-1k", n=4, field_n=16).field()
    off_ = np.array([0, n])
    say("case: pairs across cell faces, grid", ncx, ncy, "real_bytes", real_bytes)
    sim, ora = seeded_pair(p, f, x, d, q, off_, sp, real_bytes, v0=np.zeros((n, 3)))
    g = sim.read()
    r = x[:, None, :] - x[None, :, :]
    r[..., 0] -= L * np.round(r[..., 0] / L)
    dist = np.linalg.norm(r, axis=-1)
    gap = dist - 0.5 * (d[:, None] + d[None, :])
    near = (gap <= 0.25 * np.minimum(d[:, None], d[None, :])) & (dist > 0)
    assert near.sum() >= 150                                  # the in-range pairs (both members)
    assert np.array_equal(g["neighbours"], near.sum(axis=1))
    scale = np.linalg.norm(ora.a, axis=1)
    if real_bytes == 8:
        assert np.max(np.linalg.norm(g["a"] - ora.a, axis=1) / (scale + 1e-30)) < 1e-9
    else:
        assert np.max(np.linalg.norm(g["a"] - ora.a, axis=1) / (scale + 1e-3 * scale.max())) < 1e-4


@pytest.mark.parametrize("real_bytes", [8, 4])
def test_short_range_pairs_at_and_near_saturation_per_particle(real_bytes):
    """Isolated pairs (contact and van der Waals cohesion only, Appendix A.2.2-A.2.3) with surface gaps from
    a small overlap through the saturation gap delta_M = delta_min (k_r/k)^(1/4) up to near the d/4
    cutoff, unequal and equal diameters, small relative velocities: every particle's acceleration is its
    one pair force, compared with the oracle per particle relative to |a| alone.  FP64: 1e-12; FP32: 5e-6
    (the gap is formed in FP64 from the fixed-point differences, the force in FP32); plus, for pairs in
    contact, what the double-precision input positions alone can move a contact force."""
    from oracle.physics import vdw_saturation_gap
    rng = np.random.default_rng(41)
    p = physical_params(180.0, drag=False, coulomb=False, wall_image=False, wall_vdw=False)
    R, L = p["R"], p["L"]
    dm = vdw_saturation_gap(p)
    # touching pairs are left out: at gap 0 the contact damping switches on or off with the last bit
    factors = np.array([-40.0, -0.5, -1e-3, 1e-3, 0.2, 0.9, 0.999, 1.001, 1.1, 3.0, 30.0, 100.0, 200.0])
    n_pairs = 96
    centres = []
    while len(centres) < n_pairs:     # pair centres at least 0.3 mm apart, inside |y|, |z| < R/2
        c = np.array([rng.uniform(0, L), rng.uniform(-0.5 * R, 0.5 * R), rng.uniform(-0.5 * R, 0.5 * R)])
        if all(np.linalg.norm(c - o) > 3e-4 for o in centres):
            centres.append(c)
    x = np.zeros((2 * n_pairs, 3))
    d = np.zeros(2 * n_pairs)
    for k, c in enumerate(centres):
        di, dj = (10e-6, 10e-6) if k % 2 == 0 else (rng.choice([5e-6, 20e-6]), 10e-6)
        gap = factors[k % factors.size] * dm
        u = rng.normal(size=3)
        u /= np.linalg.norm(u)
        sep = 0.5 * (di + dj) + gap
        x[2 * k], x[2 * k + 1] = c + 0.5 * sep * u, c - 0.5 * sep * u
        d[2 * k], d[2 * k + 1] = di, dj
    x[:, 0] = np.mod(x[:, 0], L)
    v0 = rng.normal(0.0, 0.01, (2 * n_pairs, 3))
    q = np.zeros(2 * n_pairs)
    sp = np.array([[1.0, 4e-19, 300.0]])
    f = make_workload("plain-1k", n=4, field_n=16).field()
    say("case: isolated pairs at and near saturation, fp", 8 * real_bytes)
    sim, ora = seeded_pair(p, f, x, d, q, np.array([0, 2 * n_pairs]), sp, real_bytes, v0=v0)
    g = sim.read()
    assert np.array_equal(g["neighbours"], np.ones(2 * n_pairs, dtype=np.int32))
    an = np.linalg.norm(ora.a, axis=1)
    assert np.all(an > 0)
    e = np.linalg.norm(g["a"] - ora.a, axis=1) / an
    worst = int(np.argmax(e))
    say(f"per particle: max {e.max():.3e} (pair {worst // 2}, gap / delta_M {factors[(worst // 2) % factors.size]}) "
        f"median {np.median(e):.3e}")
    # the positions reach both sides as doubles (spacing 1.7e-18 m at |y| = 1 cm; the FP64 form holds
    # them to 2.2e-21 m): at the contact stiffness K (tau_col = 15 dt) a contact force may differ by
    # K * 4e-18 m from that alone
    tau = p["tau_col_steps"] * p["dt"]
    k_contact = (np.pi ** 2 + np.log(p["e_pp"]) ** 2) / tau ** 2
    bound = (1e-12 if real_bytes == 8 else 5e-6) + k_contact * 4e-18 / an
    say("largest error / bound", float(np.max(e / bound)))
    assert np.all(e <= bound)


def test_fp64_batched_samples_with_rebound():
    w = make_workload("batched-256", n_samples=5, n_lo=60, n_hi=300, field_n=32)
    f = w.field()
    say("case: batched 5 samples fp64, N =", w.n_particles)
    sim, ora = seeded_pair(w.params, f, w.x, w.d, w.qbase, w.offsets, w.sample_params, 8)
    sim.step(25)
    ora.step(25)
    g = sim.read()
    assert np.array_equal(g["dep_step"], ora.dep_step)
    al = ora.alive
    assert np.max(position_error(g["x"][al], ora.x[al], ora.L, ora.R)) < 1e-12
    scale = np.linalg.norm(ora.a[al], axis=1).max()
    assert np.max(np.abs(g["a"][al] - ora.a[al])) < 1e-9 * scale


def test_fp64_wall_removal_tally_and_rebound():
    """Particles driven into the wall: removal step, tally and V_dep exactly as the oracle; with the
    rebound law and weak cohesion some particles bounce back instead."""
    rng = np.random.default_rng(3)
    n = 400
    for rebound in (False, True):
        p = physical_params(180.0, rebound_osu=rebound, dt=2e-7)
        d = rng.choice([5e-6, 10e-6], n)
        x, er = near_wall_particles(rng, n, p, d, band=100e-6)
        v0 = 1.5 * er + rng.normal(0, 0.1, (n, 3))
        q = rng.normal(0, 1e-15, n)
        sp = np.array([[1.0, 1e-22 if rebound else 1e-19, 300.0]])
        f = make_workload("plain-1k", n=4, field_n=32).field()
        say("case: wall tally fp64 rebound =", rebound)
        sim, ora = seeded_pair(p, f, x, d, q, np.array([0, n]), sp, 8, v0=v0)
        sim.step(60)
        ora.step(60)
        g = sim.read()
        assert np.array_equal(g["dep_step"], ora.dep_step)
        tg, to = sim.tally()[0], ora.tally()[0]
        assert tg["n_dep"] == to["n_dep"]
        if not rebound:
            assert to["n_dep"] > 10
        assert np.isclose(tg["m_dep"], to["m_dep"], rtol=1e-14)
        assert np.isclose(tg["m_alive_dt"], to["m_alive_dt"], rtol=1e-13)
        assert np.isclose(tg["v_dep"], to["v_dep"], rtol=1e-13)
        assert np.isclose(tg["v_dep_plus"], to["v_dep_plus"], rtol=1e-13)
        assert tg["n_alive"] == to["n_alive"]
        al = ora.alive
        assert np.max(position_error(g["x"][al], ora.x[al], ora.L, ora.R)) < 1e-11
        if rebound:
            # weak cohesion: impacts at ~1.5 m/s rebound (stick speed ~0.1 m/s), so particles come back inward
            vr = np.sum(g["v"] * er, axis=1)
            assert np.sum(vr < -1.0) > 10
            assert np.allclose(vr, np.sum(ora.v * er, axis=1), rtol=0, atol=1e-9)


def test_fp64_soft_tally():
    rng = np.random.default_rng(4)
    n = 256
    p = physical_params(180.0, soft_tally=True, dt=1e-7)
    d = np.full(n, 10e-6)
    x, er = near_wall_particles(rng, n, p, d, band=20e-6)
    v0 = 0.3 * er
    sp = np.array([[0.05, 3e-19, 300.0]])
    q = np.full(n, 8e-15)
    f = make_workload("plain-1k", n=4, field_n=32).field()
    say("case: soft tally fp64")
    sim, ora = seeded_pair(p, f, x, d, q, np.array([0, n]), sp, 8, v0=v0)
    sim.step(40)
    ora.step(40)
    tg, to = sim.tally()[0], ora.tally()[0]
    assert to["j_soft"] > 0
    assert np.isclose(tg["j_soft"], to["j_soft"], rtol=1e-11)
    assert tg["n_dep"] == 0 and tg["n_alive"] == n


# ------------------------------------------------------------------------------------------ FP32 form

def test_fp32_plain_1k_200_steps_within_error_bars():
    """The FP32 form on the full 1,024-particle workload over 200 steps: positions within 1e-5 R of
    the FP64 oracle, same deposition events, V_dep within its Monte Carlo standard error."""
    w = make_workload("plain-1k")
    f = w.field()
    say("case: plain-1k fp32 200 steps")
    sim, ora = seeded_pair(w.params, f, w.x, w.d, w.qbase, w.offsets, w.sample_params, 4)
    g0 = sim.read()
    tg = np.arange(w.n_particles)
    scale = coulomb_scale(ora, tg)
    e0 = force_error(g0["a"], ora.a, scale)
    say("seed force error max", e0.max())
    assert e0.max() < 1e-5
    sim.step(200)
    ora.step(200)
    g = sim.read()
    both = (g["dep_step"] == 0) & ora.alive
    n_event_diff = int(np.sum(g["dep_step"] != ora.dep_step))
    err = position_error(g["x"][both], ora.x[both], ora.L, ora.R)
    say("fp32 position error max/R", err.max(), "event differences", n_event_diff)
    assert err.max() < 1e-5
    assert n_event_diff <= 1
    # nothing reaches the wall within these 200 steps (6.2 us): the tallies agree on that; the V_dep
    # comparison within its standard error runs on the depositing variant below
    tgp, to = sim.tally()[0], ora.tally()[0]
    assert tgp["n_dep"] == to["n_dep"] == 0 and tgp["n_alive"] == to["n_alive"] == w.n_particles


def test_fp64_plain_1k_full_size_200_steps():
    """The 1,024-particle workload at full size (64^3 field, 200 steps) in the FP64 form against the FP64
    oracle: positions within 1e-12 R, velocities and accelerations to rounding, identical events and
    tallies."""
    w = make_workload("plain-1k")
    f = w.field()
    say("case: plain-1k full size fp64, 200 steps")
    sim, ora = seeded_pair(w.params, f, w.x, w.d, w.qbase, w.offsets, w.sample_params, 8)
    for chunk in (1, 49, 150):
        sim.step(chunk)
        ora.step(chunk)
    g = sim.read()
    assert np.array_equal(g["dep_step"], ora.dep_step)
    al = ora.alive
    err = position_error(g["x"][al], ora.x[al], ora.L, ora.R)
    scale = np.linalg.norm(ora.a[al], axis=1).max()
    say("position error max / R", err.max(), "max |dv|", np.abs(g["v"][al] - ora.v[al]).max())
    assert err.max() < 1e-12
    assert np.max(np.abs(g["v"][al] - ora.v[al])) < 1e-9
    assert np.max(np.abs(g["a"][al] - ora.a[al])) <= 1e-9 * scale
    tg, to = sim.tally()[0], ora.tally()[0]
    assert tg["n_dep"] == to["n_dep"] and tg["n_alive"] == to["n_alive"]
    assert np.isclose(tg["m_alive_dt"], to["m_alive_dt"], rtol=1e-13)


@pytest.mark.parametrize("real_bytes", [8, 4])
def test_plain_1k_dep_deposition_tally(real_bytes):
    """The depositing variant of the 1,024-particle workload (dt = 3e-5 s, 200 steps: about twenty
    particles reach the wall): n_dep > 0 on both sides.  FP64: identical deposition steps, tallies to
    rounding, positions within 1e-12 R.  FP32: positions within 1e-5 R over the particles alive in both
    runs, at most 2 particles whose deposition step differs, and V_dep (Eq. 2) within its Poisson
    standard error of the oracle's."""
    w = make_workload("plain-1k-dep")
    f = w.field()
    say("case: plain-1k-dep, fp", 8 * real_bytes)
    sim, ora = seeded_pair(w.params, f, w.x, w.d, w.qbase, w.offsets, w.sample_params, real_bytes)
    sim.step(w.steps)
    ora.step(w.steps)
    g = sim.read()
    tg, to = sim.tally()[0], ora.tally()[0]
    both = (g["dep_step"] == 0) & ora.alive
    err = position_error(g["x"][both], ora.x[both], ora.L, ora.R)
    n_event_diff = int(np.sum(g["dep_step"] != ora.dep_step))
    say("n_dep gpu", tg["n_dep"], "oracle", to["n_dep"], "V_dep gpu", tg["v_dep"], "oracle", to["v_dep"],
        "se", to["v_dep_se"], "position error max / R", err.max(), "event differences", n_event_diff)
    assert to["n_dep"] > 5 and tg["n_dep"] > 5
    if real_bytes == 8:
        assert np.array_equal(g["dep_step"], ora.dep_step)
        assert err.max() < 1e-12
        assert tg["n_dep"] == to["n_dep"]
        for k in ("m_dep", "m_alive_dt", "v_dep", "v_dep_plus", "v_dep_se"):
            assert np.isclose(tg[k], to[k], rtol=1e-12), k
    else:
        assert err.max() < 1e-5
        assert n_event_diff <= 2
        assert abs(tg["v_dep"] - to["v_dep"]) <= to["v_dep_se"]


@pytest.mark.parametrize("cfg", [None, (1, 8, 64, 2), (4, 2, 64, 2)])
def test_fp32_single_65k_sampled_forces(cfg):
    """Full 65,536-particle workload in the launch configurations the benchmark times (one-sided and
    symmetric pair kernels): force error of sampled targets against the oracle evaluated on the GPU's
    own snapshot, at seed and after 20 steps."""
    w = make_workload("single-65k")
    f = w.field()
    say("case: single-65k fp32 sampled forces", cfg)
    sim, _ = seeded_pair(w.params, f, w.x, w.d, w.qbase, w.offsets, w.sample_params, 4, oracle=False)
    if cfg:
        sim.set_kernel_config(*cfg)
        sim.eval_accel()
    rng = np.random.default_rng(0)
    targets = np.sort(rng.choice(w.n_particles, 96, replace=False))
    for steps in (0, 20):
        if steps:
            sim.step(steps)
            sim.eval_accel()
        g = sim.read()
        ora = oracle_from_snapshot(w.params, f, g, w.d, w.qbase, w.offsets, w.sample_params, g["dep_step"])
        ok = targets[g["dep_step"][targets] == 0]
        a_ora = ora.accelerations(ok)
        e = force_error(g["a"][ok], a_ora, coulomb_scale(ora, ok))
        say("steps", steps, "force error max", e.max(), "median", np.median(e))
        assert e.max() < 1e-5


@pytest.mark.parametrize("cfg", [None, (1, 8, 64, 2)])
def test_fp32_bitwise_deterministic_and_checkpoint_roundtrip(cfg):
    """Repeated runs are bitwise equal (the symmetric kernel combines its items with integer atomics,
    whose order does not matter), and a checkpoint restores the exact trajectory."""
    w = make_workload("single-65k", n=8192, field_n=32)
    f = w.field()
    say("case: determinism / checkpoint fp32 n=8192", cfg)
    runs = []
    for _ in range(2):
        sim, _ = seeded_pair(w.params, f, w.x, w.d, w.qbase, w.offsets, w.sample_params, 4, oracle=False)
        if cfg:
            sim.set_kernel_config(*cfg)
        sim.step(10)
        runs.append(sim.read())
    for k in ("x", "v", "a", "dep_step"):
        assert np.array_equal(runs[0][k], runs[1][k]), k
    blob = sim.state_download()
    sim.step(7)
    ref = sim.read()
    tref = sim.tally()
    sim.state_upload(blob)
    sim.step(7)
    got = sim.read()
    for k in ("x", "v", "a", "dep_step"):
        assert np.array_equal(ref[k], got[k]), k
    assert sim.tally() == tref
    from paper_2205_04979_amd.depo import DepoError, E_CORRUPT
    bad = bytearray(blob)
    bad[-5] ^= 0xFF
    with pytest.raises(DepoError) as ei:
        sim.state_upload(bytes(bad))
    assert ei.value.status == E_CORRUPT
    with pytest.raises(DepoError):
        sim.state_upload(blob[:-8])


@pytest.mark.parametrize("p3m", [False, True])
def test_checkpoint_restores_into_a_fresh_context_on_a_dirty_workspace(p3m):
    """A checkpoint written by one context and restored into another that was never seeded, whose workspace
    is a block the caching allocator hands back full of 0xFF bytes (stale memory): the restore rebuilds
    every table seeding builds (sample ids, pair-kernel work lists, zeroed accumulators, P3M histogram and
    charge mesh), so both contexts then step bitwise alike (FP32 default pair mode, or P3M)."""
    import torch
    from paper_2205_04979_amd.depo import Simulation
    w = make_workload("single-65k", n=3000, field_n=32)
    f = w.field()
    cfg = dict(mesh_x=32, mesh_yz=16, alpha_h=0.5, rmax_alpha=3.5) if p3m else None
    say("case: checkpoint into a fresh context on a dirty workspace, p3m =", p3m)
    src = Simulation(w.params, w.offsets, f.shape[:3], real_bytes=4, p3m=cfg)
    src.set_reorder(4)
    src.init_field(f)
    src.seed(w.sample_params, w.x, w.d, w.qbase)
    src.step(5)
    blob = src.state_download()
    nbytes = src._ws.numel()
    torch.cuda.synchronize()
    dirty = torch.full((nbytes,), 0xFF, dtype=torch.uint8, device="cuda")
    lo, hi = dirty.data_ptr(), dirty.data_ptr() + dirty.numel()
    torch.cuda.synchronize()
    del dirty
    dst = Simulation(w.params, w.offsets, f.shape[:3], real_bytes=4, p3m=cfg)
    dst.set_reorder(4)
    if not (lo <= dst._ws.data_ptr() < hi):
        pytest.skip("the caching allocator did not hand back the dirtied block")
    dst.init_field(f)
    dst.state_upload(blob)
    src.step(7)
    dst.step(7)
    a, b = src.read(), dst.read()
    for k in ("x", "v", "a", "dep_step"):
        assert np.array_equal(a[k], b[k]), k
    assert src.tally() == dst.tally()


@pytest.mark.parametrize("cfg", [(1, 8, 32), (4, 2, 64, 2), (4, 2, 64, 4)])
def test_graph_replay_equals_direct_launch(cfg):
    """The captured step (forked into the pair-sum branch and the cell + short-range branch) gives
    bitwise the state of the same kernels launched one after another, for the one-sided and the
    symmetric (integer-combined) pair kernels."""
    w = make_workload("single-65k", n=4096, field_n=32)
    f = w.field()
    say("case: graph replay vs direct launches fp32", cfg)
    out = []
    for graph in (True, False):
        sim, _ = seeded_pair(w.params, f, w.x, w.d, w.qbase, w.offsets, w.sample_params, 4, oracle=False)
        sim.set_kernel_config(*cfg, use_graph=graph)
        sim.set_reorder(5)        # storage reorders at 5 and 10 steps, between and inside the replays
        for _ in range(3):
            sim.step(4)
            out_k = sim.read()   # eager synchronisation between replays
        out.append(out_k)
    for k in ("x", "v", "a"):
        assert np.array_equal(out[0][k], out[1][k]), k


@pytest.mark.parametrize("real_bytes", [8, 4])
def test_storage_reorder_keeps_the_trajectory(real_bytes):
    """Storage reorders into cell order every 3 steps against none, on a workload with removals (the
    depositing 1,024-particle variant, 60 steps) and on batched samples of uneven size with the rebound
    law: every particle, returned in the caller's order, at the same place (FP64: 1e-13 R; FP32: 1e-6 R,
    the sums that follow the storage order round differently), identical deposition steps and per-sample
    counts; the FP64 form also against the oracle."""
    cases = [make_workload("plain-1k-dep"),
             make_workload("batched-256", n_samples=5, n_lo=60, n_hi=400, field_n=32)]
    for w in cases:
        f = w.field()
        say("case: storage reorder,", w.name, "fp", 8 * real_bytes)
        runs = {}
        for every in (0, 3):
            sim, _ = seeded_pair(w.params, f, w.x, w.d, w.qbase, w.offsets, w.sample_params, real_bytes, oracle=False)
            sim.set_reorder(every)
            sim.step(60)
            runs[every] = (sim.read(), sim.tally())
            # the storage permutation, as the checkpoint blob carries it (after a 48-byte header: positions,
            # 12 per-particle reals, 3 doubles and the deposition step, then the permutation)
            n = w.n_particles
            off = 48 + n * (3 * real_bytes + 12 * real_bytes + 3 * 8 + 4)
            perm = np.frombuffer(sim.state_download(), dtype=np.int32, count=n, offset=off)
            assert np.array_equal(np.sort(perm), np.arange(n))
            assert np.array_equal(perm, np.arange(n)) == (every == 0), "reordered storage expected"
            for s in range(w.n_samples):   # every sample keeps its slots
                sl = slice(w.offsets[s], w.offsets[s + 1])
                assert np.all((perm[sl] >= w.offsets[s]) & (perm[sl] < w.offsets[s + 1]))
        (a, ta), (b, tb) = runs[0], runs[3]
        assert np.array_equal(a["dep_step"], b["dep_step"])
        assert [t["n_dep"] for t in ta] == [t["n_dep"] for t in tb]
        both = a["dep_step"] == 0
        err = position_error(b["x"][both], a["x"][both], w.params["L"], w.params["R"])
        say("reordered vs fixed order: max |dx|/R", err.max(), "deposited", int((a["dep_step"] > 0).sum()))
        assert err.max() < (1e-13 if real_bytes == 8 else 1e-6)
        assert np.array_equal(a["neighbours"] >= 0, b["neighbours"] >= 0)
        if real_bytes == 8:
            ora = OracleSim(w.params, f, w.x, w.d, w.qbase, w.offsets, w.sample_params)
            ora.step(60)
            assert np.array_equal(b["dep_step"], ora.dep_step)
            al = ora.alive
            assert position_error(b["x"][al], ora.x[al], ora.L, ora.R).max() < 1e-12


@pytest.mark.parametrize("cfg", [(1, 4, 32), (2, 8, 32), (4, 4, 32), (2, 16, 32), (1, 16, 64), (2, 8, 64),
                                 (1, 4, 64, 2), (1, 8, 64, 2), (2, 2, 64, 2), (2, 4, 64, 2), (4, 1, 64, 2),
                                 (4, 2, 64, 2), (4, 4, 64, 2), (8, 1, 64, 2), (1, 4, 64, 4), (1, 8, 64, 4),
                                 (2, 2, 64, 4), (2, 4, 64, 4), (4, 1, 64, 4), (4, 2, 64, 4), (4, 4, 64, 4),
                                 (8, 1, 64, 4)])
def test_fp32_kernel_shapes_agree(cfg):
    """Every compiled pair-kernel shape, one-sided or symmetric (modes 2 and 4, float and integer source
    records: 3,000 particles = 6 items of 512 or 3 of 1,024 per side, ragged last tile), gives the oracle's
    forces up to FP32 summation order."""
    w = make_workload("single-65k", n=3000, field_n=32)
    f = w.field()
    say("case: pair-kernel shape", cfg)
    sim, ora = seeded_pair(w.params, f, w.x, w.d, w.qbase, w.offsets, w.sample_params, 4)
    sim.set_kernel_config(*cfg)
    sim.eval_accel()
    g = sim.read()
    tg = np.arange(0, w.n_particles, 7)
    e = force_error(g["a"][tg], ora.a[tg], coulomb_scale(ora, tg))
    assert e.max() < 1e-5


@pytest.mark.parametrize("cfg", [(1, 4, 16), (1, 8, 16), (2, 4, 16), (1, 16, 16)])
def test_fp64_kernel_shapes_agree(cfg):
    """Every compiled FP64 pair-kernel shape (3,000 particles: 47 tiles of 64 targets, ragged last
    tile; 4 to 16 waves splitting the sources) gives the oracle's forces to FP64 rounding."""
    w = make_workload("single-65k", n=3000, field_n=32)
    f = w.field()
    say("case: fp64 pair-kernel shape", cfg)
    sim, ora = seeded_pair(w.params, f, w.x, w.d, w.qbase, w.offsets, w.sample_params, 8)
    sim.set_kernel_config(*cfg)
    sim.eval_accel()
    g = sim.read()
    e = force_error(g["a"], ora.a, coulomb_scale(ora, np.arange(w.n_particles)))
    say("force error max", e.max())
    assert e.max() < 1e-9


def test_nonfinite_is_reported():
    """A non-finite input velocity is flagged on the device and reported by the next synchronising call."""
    from paper_2205_04979_amd.depo import DepoError, E_NONFINITE
    w = make_workload("plain-1k", n=64, field_n=16)
    f = w.field()
    q = w.qbase.copy()
    q[5] = 1e30                      # finite on the host; its scaled charge overflows FP32 in the pair sums
    sim, _ = seeded_pair(w.params, f, w.x, w.d, q, w.offsets, w.sample_params, 4, oracle=False)
    sim.step(1)
    with pytest.raises(DepoError) as ei:
        sim.tally()
    assert ei.value.status == E_NONFINITE


def test_autotune_restores_state_and_picks_a_compiled_shape():
    from paper_2205_04979_amd.autotune import FP32_SHAPES, FP32_SYM_SHAPES, autotune
    w = make_workload("single-65k", n=4096, field_n=32)
    f = w.field()
    sim, _ = seeded_pair(w.params, f, w.x, w.d, w.qbase, w.offsets, w.sample_params, 4, oracle=False)
    sim.step(3)
    before = sim.read()
    best, times = autotune(sim, steps=2)
    after = sim.read()
    assert best in FP32_SHAPES + FP32_SYM_SHAPES and set(times) == set(FP32_SHAPES + FP32_SYM_SHAPES)
    for k in ("x", "v", "a", "dep_step"):
        assert np.array_equal(before[k], after[k]), k
    sim.step(2)            # still steps normally with the chosen shape


@pytest.mark.parametrize("cfg", [None, (1, 8, 64, 2)])
def test_fp32_batched_samples_sampled_forces(cfg):
    """Many Monte Carlo samples of uneven size in one launch: per-sample force parity on sampled targets
    (sources restricted to the target's own sample), at seed and after 10 steps."""
    w = make_workload("batched-256", n_samples=24, n_lo=512, n_hi=6000, field_n=64)
    f = w.field()
    say("case: batched fp32, S =", w.n_samples, "N =", w.n_particles, cfg)
    sim, _ = seeded_pair(w.params, f, w.x, w.d, w.qbase, w.offsets, w.sample_params, 4, oracle=False)
    if cfg:
        sim.set_kernel_config(*cfg)
        sim.eval_accel()
    rng = np.random.default_rng(1)
    targets = np.sort(np.concatenate([rng.choice(np.arange(w.offsets[s], w.offsets[s + 1]), 3, replace=False)
                                      for s in range(w.n_samples)]))
    for steps in (0, 10):
        if steps:
            sim.step(steps)
            sim.eval_accel()
        g = sim.read()
        ora = oracle_from_snapshot(w.params, f, g, w.d, w.qbase, w.offsets, w.sample_params, g["dep_step"])
        ok = targets[g["dep_step"][targets] == 0]
        e = force_error(g["a"][ok], ora.accelerations(ok), coulomb_scale(ora, ok))
        say("steps", steps, "force error max", e.max())
        assert e.max() < 1e-5
    t = sim.tally()
    assert len(t) == w.n_samples and all(x["n_alive"] + x["n_dep"] == w.offsets[s + 1] - w.offsets[s]
                                         for s, x in enumerate(t))


@pytest.mark.parametrize("cfg", [(4, 2, 64, 2), (4, 4, 64, 2)])
def test_fp32_batched_256_full_size_sampled_forces(cfg):
    """The full 256-sample workload the benchmark times (about 4.45 M particles, sample sizes uniform on
    2,048..32,768) with the two symmetric shapes its autotuner chooses between: force error of two sampled
    targets in each of 64 samples against the oracle over the target's own sample, at seed and after 10
    steps, and per-sample particle conservation in the tally."""
    w = make_workload("batched-256")
    f = w.field()
    say("case: batched-256 full size fp32, S =", w.n_samples, "N =", w.n_particles, cfg)
    sim, _ = seeded_pair(w.params, f, w.x, w.d, w.qbase, w.offsets, w.sample_params, 4, oracle=False)
    sim.set_kernel_config(*cfg)
    sim.eval_accel()
    rng = np.random.default_rng(2)
    samples = np.sort(rng.choice(w.n_samples, 64, replace=False))
    targets = np.sort(np.concatenate([rng.choice(np.arange(w.offsets[s], w.offsets[s + 1]), 2, replace=False)
                                      for s in samples]))
    for steps in (0, 10):
        if steps:
            sim.step(steps)
            sim.eval_accel()
        g = sim.read()
        ora = oracle_from_snapshot(w.params, f, g, w.d, w.qbase, w.offsets, w.sample_params, g["dep_step"])
        ok = targets[g["dep_step"][targets] == 0]
        e = force_error(g["a"][ok], ora.accelerations(ok), coulomb_scale(ora, ok))
        say("steps", steps, "targets", ok.size, "force error max", e.max(), "median", np.median(e))
        assert ok.size >= 120 and e.max() < 1e-5
    t = sim.tally()
    assert len(t) == w.n_samples and all(x["n_alive"] + x["n_dep"] == w.offsets[s + 1] - w.offsets[s]
                                         for s, x in enumerate(t))


@pytest.mark.parametrize("cfg", [(1, 8, 64, 2), (4, 1, 64, 2), (4, 4, 64, 2), (4, 2, 64, 4)])
def test_fp32_symmetric_every_particle_of_uneven_samples(cfg):
    """Symmetric pair sums over samples smaller than one item, of one item and of several with ragged
    tails: every particle's acceleration at seed against the oracle, and Newton's third law: the
    charge-weighted Coulomb sums of each sample add up to zero (up to rounding)."""
    w = make_workload("batched-256", n_samples=6, n_lo=100, n_hi=2200, field_n=32)
    f = w.field()
    say("case: symmetric every particle, sizes", np.diff(w.offsets).tolist(), cfg)
    sim, ora = seeded_pair(w.params, f, w.x, w.d, w.qbase, w.offsets, w.sample_params, 4)
    sim.set_kernel_config(*cfg)
    sim.eval_accel()
    g = sim.read()
    tg = np.arange(w.n_particles)
    e = force_error(g["a"], ora.a, coulomb_scale(ora, tg))
    say("force error max", e.max())
    assert e.max() < 1e-5
    # with collisions, cohesion, wall terms and drag off, m_i a_i are pairwise equal and opposite
    p = dict(w.params, drag=False, collide=False, vdw=False, wall_image=False, wall_vdw=False)
    sim2, _ = seeded_pair(p, f, w.x, w.d, w.qbase, w.offsets, w.sample_params, 4, oracle=False)
    sim2.set_kernel_config(*cfg)
    sim2.eval_accel()
    a = sim2.read()["a"].astype(np.float64)
    m = w.params["rho_p"] * np.pi * w.d ** 3 / 6
    scale = m * coulomb_scale(ora, tg)          # sum_j |F_ij| per particle
    for s in range(w.n_samples):
        sl = slice(w.offsets[s], w.offsets[s + 1])
        F = m[sl, None] * a[sl]
        assert np.all(np.abs(F.sum(0)) <= 1e-6 * scale[sl].sum()), s


@pytest.mark.parametrize("reorder", [0, 2])
@pytest.mark.parametrize("real_bytes", [4, 8])
def test_empty_single_and_pair_samples(real_bytes, reorder):
    """Samples of 0, 1, 2, 0, 65 and 300 particles in one layout (the default pair mode of the
    precision): every particle's acceleration at seed against the oracle, positions after 5 steps
    (FP64: round-off; FP32: within 1e-5 R), and per-sample tallies that conserve particles (the empty
    samples tally nothing and report V_dep = 0); with and without the storage reorder (every 2 steps)."""
    w = make_workload("batched-256", n_samples=6, n_lo=100, n_hi=400, field_n=16)
    f = w.field()
    sizes = [0, 1, 2, 0, 65, 300]
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    n = int(off[-1])
    x, d, q = w.x[:n], w.d[:n], w.qbase[:n]
    say("case: empty / single / pair samples, sizes", sizes, "fp", 8 * real_bytes, "reorder", reorder)
    sim, ora = seeded_pair(w.params, f, x, d, q, off, w.sample_params, real_bytes)
    sim.set_reorder(reorder)
    g = sim.read()
    tg = np.arange(n)
    e = force_error(g["a"], ora.a, coulomb_scale(ora, tg))
    say("force error max", e.max())
    assert e.max() < (1e-9 if real_bytes == 8 else 1e-5)
    sim.step(5)
    ora.step(5)
    g = sim.read()
    both = (g["dep_step"] == 0) & ora.alive
    err = position_error(g["x"][both], ora.x[both], ora.L, ora.R)
    say("position error max / R", err.max(), "alive in both", int(both.sum()))
    assert err.max() < (1e-12 if real_bytes == 8 else 1e-5)
    t = sim.tally()
    for s, size in enumerate(sizes):
        assert t[s]["n_alive"] + t[s]["n_dep"] == size, s
        if size == 0:
            assert t[s]["n_dep"] == 0 and t[s]["m_alive_dt"] == 0.0 and t[s]["v_dep"] == 0.0


@pytest.mark.parametrize("real_bytes", [4, 8])
def test_layout_without_particles(real_bytes):
    """A layout whose samples hold no particles at all seeds, steps (graph and direct launches),
    evaluates forces and tallies zeros."""
    f = make_workload("plain-1k", n=4, field_n=16).field()
    p = physical_params(180.0)
    off = np.array([0, 0, 0], dtype=np.int64)
    say("case: layout without particles, fp", 8 * real_bytes)
    sim, _ = seeded_pair(p, f, np.zeros((0, 3)), np.zeros(0), np.zeros(0), off,
                         np.array([[1.0, 1e-20, 300.0]] * 2), real_bytes, oracle=False)
    sim.step(2)            # the precision's default pair mode, captured graph
    for graph in (True, False):
        sim.set_kernel_config(*((1, 8, 32) if real_bytes == 4 else (1, 4, 16)), use_graph=graph)
        sim.step(3)
    sim.eval_accel()
    t = sim.tally()
    assert len(t) == 2 and all(x["n_alive"] == 0 and x["n_dep"] == 0 and x["v_dep"] == 0.0 for x in t)
    assert sim.read()["x"].shape == (0, 3)


@pytest.mark.parametrize("use_graph", [True, False])
def test_step_converts_the_pair_sums_like_the_evaluation(use_graph):
    """In the step, k_finish turns the symmetric pair kernel's fixed-point sums into FP32 and clears the
    accumulators; outside it (a force evaluation) k_pair_finish does.  After 7 steps (graph replay or
    direct launches; 6,000 particles of the 65k recipe, every force on), the stored acceleration equals
    bitwise that of a fresh evaluation at the same positions, twice in a row (the accumulators were
    left at zero by both)."""
    w = make_workload("single-65k", n=6000, field_n=32)
    f = w.field()
    sim, _ = seeded_pair(w.params, f, w.x, w.d, w.qbase, w.offsets, w.sample_params, 4, oracle=False)
    sim.set_kernel_config(4, 2, 64, 2, use_graph=use_graph)
    say("case: pair-sum conversion in the step, graph", use_graph)
    sim.step(7)
    a_step = sim.read()["a"]
    for _ in range(2):
        sim.eval_accel()
        assert np.array_equal(sim.read()["a"], a_step)
