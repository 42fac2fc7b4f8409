"""P3M electrostatics on the GPU (Appendix A.2.4, Eq. coulomb_force) against the P3M oracle (same
algorithm, FP64) and against the exact x-periodic lattice sum it approximates."""

import sys

import numpy as np
import pytest

from oracle import p3m as op3m
from oracle.physics import coulomb_constant, particle_mass
from synthetic import make_workload
from synthetic.workloads import physical_params

pytestmark = pytest.mark.gpu

COULOMB_ONLY = dict(drag=False, collide=False, vdw=False, wall_image=False, wall_vdw=False)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def gpu_accel(w, f, real_bytes, cfg, steps=0, offsets=None):
    from paper_2205_04979_amd.depo import Simulation
    sim = Simulation(w.params, w.offsets if offsets is None else offsets, f.shape[:3], real_bytes=real_bytes,
                     p3m=cfg)
    sim.init_field(f)
    sim.seed(w.sample_params, w.x, w.d, w.qbase)
    if steps:
        sim.step(steps)
        sim.eval_accel()
    return sim, sim.read()


def accel_from_sums(p, sp, qbase, d, S):
    """a_i = k_e q_i S_i / m_i with S in C / m^2."""
    q = sp[0, 0] * qbase
    return coulomb_constant(p["eps0"]) * (q / particle_mass(d, p["rho_p"]))[:, None] * S


def rel_rms(a, ref):
    return np.sqrt(np.mean(np.sum((a - ref) ** 2, 1)) / np.mean(np.sum(ref ** 2, 1)))


def p3m_fp32_bound(w, r_min):
    """Per-target bound of the FP32 form against the P3M oracle, relative to sum_j |a_ij|: 2e-6 for the
    FP32 mesh and FFTs (relative rounding ~1e-6 of the long-range field, which is at most sum_j |a_ij|)
    and the tabulated short-range profile (at most 4.4e-7 of a pair force), plus 3 * 64 u_x / r_min for
    the short-range source records, which hold y and z as floats in position quanta (spacing up to 64
    quanta near the wall): a relative direction error of that size on the nearest pair."""
    ux = w.params["L"] / 2.0 ** 32
    return 2e-6 + 3.0 * 64.0 * ux / r_min


@pytest.mark.parametrize("real_bytes", [8, 4])
def test_p3m_matches_oracle_p3m(real_bytes):
    """Same algorithm, same inputs (the GPU's own positions): every particle's acceleration against the
    FP64 P3M oracle, relative to sum_j |a_ij|.  FP64: 1e-9 per particle.  FP32: the stated per-particle
    bound (FP32 mesh and FFTs, tabulated short-range profile, float short-range records)."""
    from tests.oracle_pool import coulomb_magnitude_sum, nearest_distance
    from oracle.sim import OracleSim
    w = make_workload("single-65k", n=600, field_n=16, **COULOMB_ONLY)
    f = w.field()
    cfg = dict(mesh_x=32, mesh_yz=16, alpha_h=0.5, rmax_alpha=3.5)
    say("case: p3m vs oracle p3m, n=600, fp", 8 * real_bytes)
    sim, g = gpu_accel(w, f, real_bytes, cfg)
    mesh = op3m.Mesh(w.params["R"], w.params["L"], 32, 16, 0.5, 3.5)
    q = w.sample_params[0, 0] * w.qbase
    S = op3m.p3m_sums(mesh, g["x"], q, w.d)
    a_ora = accel_from_sums(w.params, w.sample_params, w.qbase, w.d, S)
    ora = OracleSim(w.params, f, g["x"], w.d, w.qbase, w.offsets, w.sample_params, evaluate=False)
    tg = np.arange(w.n_particles)
    e = np.linalg.norm(g["a"] - a_ora, axis=1) / coulomb_magnitude_sum(ora, tg)
    say("per particle: max", e.max(), "median", np.median(e))
    if real_bytes == 8:
        assert e.max() < 1e-9
    else:
        assert np.all(e <= p3m_fp32_bound(w, nearest_distance(ora, tg)))


@pytest.mark.parametrize("real_bytes", [8, 4])
def test_p3m_single_65k_every_particle_against_stored_p3m_oracle(real_bytes):
    """The 65,536-particle workload in the P3M configuration the benchmark times (mesh 128 x 128 x 128
    with the zero padding, alpha h = 0.5, r_max = 3.5 / alpha), at seed: every particle's acceleration
    against the P3M oracle (stored by tests/golden/make_golden.py from the same seeded inputs), relative
    to sum_j |a_ij|.  FP64: 1e-9 per particle.  FP32: the stated per-particle bound."""
    import os
    from tests.golden.make_golden import P3M_65K, input_digest
    w = make_workload("single-65k")
    f = w.field()
    gold = np.load(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "p3m_single65k_seed.npz"))
    assert str(gold["digest"]) == input_digest(w, f)
    cfg = dict(P3M_65K)
    assert np.array_equal(gold["config"], [cfg["mesh_x"], cfg["mesh_yz"], cfg["alpha_h"], cfg["rmax_alpha"]])
    say("case: p3m single-65k every particle vs stored p3m oracle, fp", 8 * real_bytes)
    wc = make_workload("single-65k", **COULOMB_ONLY)
    sim, g = gpu_accel(wc, f, real_bytes, cfg)
    a_ora = accel_from_sums(w.params, w.sample_params, w.qbase, w.d, gold["S"])
    e = np.linalg.norm(g["a"] - a_ora, axis=1) / gold["scale"]
    k = int(np.argmax(e))
    say(f"per particle: max {e.max():.3e} (particle {k}, nearest {gold['r_min'][k]:.3e} m), median {np.median(e):.3e}")
    if real_bytes == 8:
        assert e.max() < 1e-9
    else:
        bound = p3m_fp32_bound(w, gold["r_min"])
        say("largest error / bound", float(np.max(e / bound)))
        assert np.all(e <= bound)
        assert np.median(e) < 1e-6


@pytest.mark.parametrize("real_bytes", [8, 4])
def test_p3m_large_1m_targets_against_stored_p3m_oracle(real_bytes):
    """The 2^20-particle workload in the P3M configuration the benchmark times (mesh 256 x 256 x 256
    with the zero padding, alpha h = 0.5, r_max = 3.5 / alpha), at seed: the accelerations of the 4,096
    targets i = 0 mod 256 against the P3M oracle (stored by tests/golden/make_golden.py from the same
    seeded inputs, every particle a source), relative to sum_j |a_ij|.  FP64: 1e-9 per target.  FP32:
    the stated per-target bound."""
    import os
    from tests.golden.make_golden import P3M_1M, P3M_1M_TARGETS, input_digest
    w = make_workload("large-1m")
    f = w.field()
    gold = np.load(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "p3m_large1m_seed_targets.npz"))
    assert str(gold["digest"]) == input_digest(w, f)
    cfg = dict(P3M_1M)
    assert np.array_equal(gold["config"], [cfg["mesh_x"], cfg["mesh_yz"], cfg["alpha_h"], cfg["rmax_alpha"]])
    tg = P3M_1M_TARGETS
    assert np.array_equal(gold["targets"], tg)
    say("case: p3m large-1m targets vs stored p3m oracle, fp", 8 * real_bytes)
    wc = make_workload("large-1m", **COULOMB_ONLY)
    sim, g = gpu_accel(wc, f, real_bytes, cfg)
    a_ora = accel_from_sums(w.params, w.sample_params, w.qbase[tg], w.d[tg], gold["S"])
    e = np.linalg.norm(g["a"][tg] - a_ora, axis=1) / gold["scale"]
    k = int(np.argmax(e))
    say(f"per target: max {e.max():.3e} (target {int(tg[k])}, nearest {gold['r_min'][k]:.3e} m), "
        f"median {np.median(e):.3e}")
    if real_bytes == 8:
        assert e.max() < 1e-9
    else:
        bound = p3m_fp32_bound(w, gold["r_min"])
        say("largest error / bound", float(np.max(e / bound)))
        assert np.all(e <= bound)
        assert np.median(e) < 1e-6
    sim.close()


def test_p3m_close_to_the_lattice_sum_and_deterministic():
    """Against the exact lattice sum (brute force over 100 x images; the tail beyond is ~1e-8 of the
    field): relative RMS error at the level of the oracle's pinned P3M accuracy; repeated runs are
    bitwise equal."""
    w = make_workload("single-65k", n=1000, field_n=16, **COULOMB_ONLY)
    f = w.field()
    cfg = dict(mesh_x=64, mesh_yz=32, alpha_h=0.4, rmax_alpha=3.5)
    say("case: p3m vs lattice sum, n=1000")
    _, g = gpu_accel(w, f, 4, cfg)
    _, g2 = gpu_accel(w, f, 4, cfg)
    assert np.array_equal(g["a"], g2["a"])
    q = w.sample_params[0, 0] * w.qbase
    S = op3m.lattice_sum(g["x"], q, w.d, w.params["L"], images=100)
    a_ref = accel_from_sums(w.params, w.sample_params, w.qbase, w.d, S)
    err = rel_rms(g["a"], a_ref)
    say("rel rms vs lattice sum", err)
    assert err < 3e-3


def lattice_sums_at(x, q, d, L, targets, images):
    """Raw Coulomb sums of the targets over every source and its x images |n| <= images (the nearest
    image with the overlap clamp |r| >= d_ij, the others as point charges), in FP64."""
    S = np.zeros((len(targets), 3))
    for k, i in enumerate(targets):
        r = x[i] - x
        r[:, 0] -= L * np.round(r[:, 0] / L)
        m = np.arange(x.shape[0]) != i
        r, qm = r[m], q[m]
        t2 = r[:, 1] ** 2 + r[:, 2] ** 2
        dij = 0.5 * (d[i] + d[m])
        for n in range(-images, images + 1):
            rx = r[:, 0] + n * L
            r2 = rx * rx + t2
            rc2 = np.maximum(r2, dij * dij) if n == 0 else r2
            w = qm / (np.sqrt(r2) * rc2)
            S[k] += (w @ rx, w @ r[:, 1], w @ r[:, 2])
    return S


def test_p3m_large_1m_sampled_against_lattice_sum():
    """The 2^20-particle workload in the P3M configuration the benchmark times (mesh 256 x 128 across,
    alpha h 0.5, r_max = 3.5 / alpha): 8 sampled targets against the x-periodic lattice sum over all
    1,048,576 sources (images |n| <= 40), at seed."""
    w = make_workload("large-1m")
    f = w.field()
    cfg = dict(mesh_x=256, mesh_yz=128, alpha_h=0.5, rmax_alpha=3.5)
    say("case: p3m large-1m vs lattice sum")
    from paper_2205_04979_amd.depo import Simulation
    sim = Simulation(dict(w.params, **COULOMB_ONLY), w.offsets, f.shape[:3], real_bytes=4, p3m=cfg)
    sim.init_field(f)
    sim.seed(w.sample_params, w.x, w.d, w.qbase)
    g = sim.read()
    sim.close()
    tg = np.sort(np.random.default_rng(4).choice(w.n_particles, 8, replace=False))
    q = w.sample_params[0, 0] * w.qbase
    S = lattice_sums_at(g["x"], q, w.d, w.params["L"], tg, 40)
    a_ref = accel_from_sums(w.params, w.sample_params, w.qbase[tg], w.d[tg], S)
    err = rel_rms(g["a"][tg], a_ref)
    say("large-1m sampled rel rms vs lattice sum", err)
    assert err < 5e-3


def test_p3m_single_65k_sampled_against_lattice_sum_and_steps():
    """The 65,536-particle workload with P3M (mesh 128 x 64, alpha h 0.5): sampled targets against the
    lattice sum over all sources, at seed and after 10 steps of the full step with every force on."""
    w = make_workload("single-65k")
    f = w.field()
    cfg = dict(mesh_x=128, mesh_yz=64, alpha_h=0.5, rmax_alpha=3.5)
    say("case: p3m single-65k")
    pc = dict(w.params, **COULOMB_ONLY)
    from paper_2205_04979_amd.depo import Simulation
    sim = Simulation(pc, w.offsets, f.shape[:3], real_bytes=4, p3m=cfg)
    sim.init_field(f)
    sim.seed(w.sample_params, w.x, w.d, w.qbase)
    g = sim.read()
    rng = np.random.default_rng(3)
    tg = np.sort(rng.choice(w.n_particles, 24, replace=False))
    q = w.sample_params[0, 0] * w.qbase
    L = w.params["L"]
    S = np.zeros((tg.size, 3))
    for k, i in enumerate(tg):
        r = g["x"][i] - g["x"]
        r[:, 0] -= L * np.round(r[:, 0] / L)
        m = np.arange(w.n_particles) != i
        for n in range(-100, 101):
            rn = r[m] + np.array([n * L, 0.0, 0.0])
            r2 = np.sum(rn * rn, 1)
            dij = 0.5 * (w.d[i] + w.d[m])
            rc2 = np.maximum(r2, dij * dij) if n == 0 else r2
            S[k] += ((q[m] / (np.sqrt(r2) * rc2))[:, None] * rn).sum(0)
    a_ref = accel_from_sums(w.params, w.sample_params, w.qbase[tg], w.d[tg], S)
    err = rel_rms(g["a"][tg], a_ref)
    say("single-65k sampled rel rms vs lattice sum", err)
    assert err < 5e-3
    sim.close()
    sim2 = Simulation(w.params, w.offsets, f.shape[:3], real_bytes=4, p3m=cfg)
    sim2.init_field(f)
    sim2.seed(w.sample_params, w.x, w.d, w.qbase)
    sim2.step(10)
    t = sim2.tally()[0]
    assert t["n_alive"] + t["n_dep"] == w.n_particles and np.all(np.isfinite(sim2.read()["a"]))


@pytest.mark.parametrize("real_bytes", [8, 4])
def test_p3m_storage_reorder_keeps_the_trajectory(real_bytes):
    """P3M with every other force on, the particle storage permuted into cell order every 3 steps against
    none (the P3M cell lists, their per-wave counters and the short-range lists are rebuilt from the
    storage at every evaluation): the depositing 1,024-particle variant (3 short-range cells along x) and
    6,000 particles of the 65k recipe (17 cells along x), 30 steps.  Every particle, in the caller's
    order, at the same place (FP64: 1e-13 R; FP32: 1e-6 R, sums that follow the storage order round
    differently) and the same deposition steps (FP32: at most one particle whose event moved by a step,
    counted and left out of the position check).  Where each 4 x 4 x 4 sub-cell of the P3M cells holds at
    most one particle, as here, the P3M summation order does not depend on the storage and the two runs
    agree bitwise."""
    from paper_2205_04979_amd.depo import Simulation
    from tests.gpu_common import position_error
    cases = [(make_workload("plain-1k-dep"), dict(mesh_x=32, mesh_yz=16, alpha_h=0.5, rmax_alpha=3.5)),
             (make_workload("single-65k", n=6000, field_n=32), dict(mesh_x=128, mesh_yz=64, alpha_h=0.5,
                                                                     rmax_alpha=3.5))]
    for w, cfg in cases:
        f = w.field()
        say("case: p3m storage reorder,", w.name, w.n_particles, "fp", 8 * real_bytes)
        runs = {}
        for every in (0, 3):
            sim = Simulation(w.params, w.offsets, f.shape[:3], real_bytes=real_bytes, p3m=cfg)
            sim.init_field(f)
            sim.seed(w.sample_params, w.x, w.d, w.qbase)
            sim.set_reorder(every)
            sim.step(30)
            runs[every] = sim.read()
            # the storage permutation, as the checkpoint blob carries it (after a 48-byte header: positions,
            # 12 per-particle reals, 3 doubles and the deposition step, then the permutation)
            n = w.n_particles
            off = 48 + n * (3 * real_bytes + 12 * real_bytes + 3 * 8 + 4)
            perm = np.frombuffer(sim.state_download(), dtype=np.int32, count=n, offset=off)
            assert np.array_equal(np.sort(perm), np.arange(n))
            assert np.array_equal(perm, np.arange(n)) == (every == 0), "reordered storage expected"
            sim.close()
        a, b = runs[0], runs[3]
        moved = a["dep_step"] != b["dep_step"]
        say("deposited", int((a["dep_step"] > 0).sum()), "events moved", int(moved.sum()))
        assert moved.sum() == 0 if real_bytes == 8 else moved.sum() <= 1
        both = (a["dep_step"] == 0) & (b["dep_step"] == 0)
        err = position_error(b["x"][both], a["x"][both], w.params["L"], w.params["R"])
        say("reordered vs fixed order: max |dx|/R", err.max())
        assert err.max() < (1e-13 if real_bytes == 8 else 1e-6)


@pytest.mark.parametrize("real_bytes", [8, 4])
def test_p3m_crowded_cells_against_oracle_p3m(real_bytes):
    """Large P3M cells: 12,300 particles on a 32 x 16 mesh, whose r_max leaves 3 short-range cells of
    about 4,100 particles each.  This takes the kernels' large-cell paths: the one-thread sort of cells
    above 2,048 particles, several staged chunks of the 27-cell neighbourhood and several target passes
    (FP32: 4,096 targets per pass, one cell holds 4,122; FP64: 512 per block).  Every particle against
    the FP64 P3M oracle, relative to sum_j |a_ij|: FP64 1e-9, FP32 the stated per-particle bound."""
    from tests.oracle_pool import pooled_coulomb_scale, pooled_nearest
    from oracle.sim import OracleSim
    w = make_workload("single-65k", n=12300, field_n=16, **COULOMB_ONLY)
    f = w.field()
    cfg = dict(mesh_x=32, mesh_yz=16, alpha_h=0.5, rmax_alpha=3.5)
    say("case: p3m crowded cells, n=12300, fp", 8 * real_bytes)
    sim, g = gpu_accel(w, f, real_bytes, cfg)
    mesh = op3m.Mesh(w.params["R"], w.params["L"], 32, 16, 0.5, 3.5)
    q = w.sample_params[0, 0] * w.qbase
    S = op3m.p3m_sums(mesh, g["x"], q, w.d)
    a_ora = accel_from_sums(w.params, w.sample_params, w.qbase, w.d, S)
    ora = OracleSim(w.params, f, g["x"], w.d, w.qbase, w.offsets, w.sample_params, evaluate=False)
    tg = np.arange(w.n_particles)
    e = np.linalg.norm(g["a"] - a_ora, axis=1) / pooled_coulomb_scale(ora, tg)
    say("per particle: max", e.max(), "median", np.median(e))
    if real_bytes == 8:
        assert e.max() < 1e-9
    else:
        assert np.all(e <= p3m_fp32_bound(w, pooled_nearest(ora, tg)))
    sim.close()
