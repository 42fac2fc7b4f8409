"""Hand-written adjoint of the step (smoothed tally) against finite differences.

References: central differences (relative step 1e-4 per parameter) of the FP64
oracle's smoothed deposited mass, and of the library's own FP64 forward run.
The workload places particles next to the wall so that the image charge
(charge scale squared) and the wall and pair cohesion (Hamaker constant) move
them measurably through the smoothed tally within the horizon.
"""

import sys

import numpy as np
import pytest

from oracle.sim import OracleSim
from synthetic import make_workload
from synthetic.workloads import physical_params, q_max
from tests.gpu_common import near_wall_particles

pytestmark = pytest.mark.gpu

H_REL = 1e-4


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def sensitive_case(n_per=120, S=2, seed=8):
    rng = np.random.default_rng(seed)
    p = physical_params(180.0, soft_tally=True, rebound_osu=True, dt=1e-6)
    d = rng.choice([5e-6, 10e-6, 20e-6], n_per * S)
    x, er = near_wall_particles(rng, n_per * S, p, d, band=6e-6)
    # every 7th particle gets a partner at a surface gap of a fraction of a diameter (cohesion and
    # Coulomb pairs; some overlap slightly, so contact forces act too)
    a_idx = np.arange(0, n_per * S - 1, 7)
    b_idx = a_idx + 1
    gap = rng.uniform(-0.05, 0.2, a_idx.size) * np.minimum(d[a_idx], d[b_idx])
    x[b_idx] = x[a_idx]
    x[b_idx, 0] += 0.5 * (d[a_idx] + d[b_idx]) + gap
    rr = np.hypot(x[:, 1], x[:, 2])
    bad = rr + 0.5 * d >= p["R"] - 1e-7
    x[bad, 1:] *= ((p["R"] - 0.5 * d[bad] - 2e-6) / rr[bad])[:, None]
    v0 = 0.02 * er
    q = q_max(d)
    off = np.arange(S + 1) * n_per
    sp = np.array([[0.08, 4e-19, 300.0], [0.05, 9e-19, 340.0]])[:S]
    f = make_workload("plain-1k", n=4, field_n=32).field()
    return p, f, x, d, q, off, sp, v0


def oracle_J(p, f, x, d, q, off, sp, v0, n):
    o = OracleSim(p, f, x, d, q, off, sp, v0=v0)
    o.step(n)
    return np.array([t["j_soft"] for t in o.tally()])


def fd_oracle(p, f, x, d, q, off, sp, v0, n, h=None):
    h = H_REL if h is None else h
    g = np.zeros((sp.shape[0], 2))
    for c in range(2):
        hp, hm = sp.copy(), sp.copy()
        hp[:, c] *= 1 + h
        hm[:, c] *= 1 - h
        g[:, c] = (oracle_J(p, f, x, d, q, off, hp, v0, n) - oracle_J(p, f, x, d, q, off, hm, v0, n)) / (
            2 * h * sp[:, c])
    return g


def gpu_sim(p, f, off, real_bytes):
    from paper_2205_04979_amd.depo import Simulation
    sim = Simulation(p, off, f.shape[:3], real_bytes=real_bytes)
    sim.init_field(f)
    return sim


def test_fp64_adjoint_single_particle_image_force_closed_form():
    """One particle, the wall image force only (no drag, pair or cohesion forces), one step of the
    smoothed tally: with a0 = k_e s^2 qb^2 / (4 h0^2 m) radially outward and v0 = 0, the step moves the
    particle to rho1 = rho0 + dt^2 a0 / 2 and J = m (1 - exp(-l1)), l1 = sigma(z1) / tau_s,
    z1 = -(R - rho1 - d/2) / (eps d).  So dJ/ds = m exp(-l1) sigma'(z1) / tau_s * dt^2 a0 / (s eps d)
    (the image force is proportional to s^2), dJ/dA = 0 (no cohesion term) and dJ/dT = 0."""
    from oracle.physics import coulomb_constant, particle_mass
    from paper_2205_04979_amd.depo import Simulation
    p = physical_params(180.0, soft_tally=True, drag=False, collide=False, vdw=False, wall_vdw=False,
                        coulomb=False, rebound_osu=False, dt=1e-5)
    R, L = p["R"], p["L"]
    d, qb, s = 10e-6, 1e-14, 0.7
    rho0 = R - 0.5 * d - 1e-6
    x = np.array([[0.5 * L, rho0, 0.0]])
    f = make_workload("plain-1k", n=4, field_n=16).field()
    sp = np.array([[s, 3e-19, 300.0]])
    say("case: adjoint closed form, single particle, image force")
    sim = Simulation(p, np.array([0, 1]), f.shape[:3], real_bytes=8)
    sim.init_field(f)
    sim.seed(sp, x, np.array([d]), np.array([qb]), v=np.zeros((1, 3)))
    g = sim.adjoint(1, 1)[0]
    m = particle_mass(d, p["rho_p"])
    h0 = R - rho0
    a0 = coulomb_constant(p["eps0"]) * (s * qb) ** 2 / (4.0 * h0 * h0 * m)
    dt, eps, tau = p["dt"], p["soft_eps"], p["soft_tau"]
    rho1 = rho0 + 0.5 * dt * dt * a0
    z1 = -(R - rho1 - 0.5 * d) / (eps * d)
    sig = 1.0 / (1.0 + np.exp(-z1))
    l1 = sig / tau
    dJ_ds = m * np.exp(-l1) * sig * (1.0 - sig) / tau * dt * dt * a0 / (s * eps * d)
    say("adjoint", g.tolist(), "closed form", dJ_ds)
    assert 0.1 < sig < 0.9                      # the step lands where the smoothed tally is sensitive
    assert g[0] == pytest.approx(dJ_ds, rel=1e-8)
    assert g[1] == 0.0 and g[2] == 0.0


def test_fp64_adjoint_matches_oracle_finite_differences():
    """The cohesion cutoff (a jump of 0.27 A/d at gap d/4) makes J piecewise smooth; the adjoint
    differentiates the smooth branch, so the seeded case is one where no cutoff crossing falls inside
    the +-h interval: asserted here by the agreement of the h = 1e-4 and h = 1e-6 differences."""
    p, f, x, d, q, off, sp, v0 = sensitive_case(seed=12)
    n, ce = 30, 7
    say("case: adjoint fp64 S=2 n=30 ckpt=7")
    sim = gpu_sim(p, f, off, 8)
    sim.seed(sp, x, d, q, v=v0)
    g = sim.adjoint(n, ce)
    fd = fd_oracle(p, f, x, d, q, off, sp, v0, n)
    fd_fine = fd_oracle(p, f, x, d, q, off, sp, v0, n, h=1e-6)
    assert np.max(np.abs(fd / fd_fine - 1)) < 2e-4
    say("adjoint", g[:, :2].tolist(), "oracle FD", fd.tolist())
    assert np.all(g[:, 2] == 0.0)
    for s in range(sp.shape[0]):
        for c in range(2):
            assert abs(fd[s, c]) > 0
            assert abs(g[s, c] - fd[s, c]) <= 1e-3 * abs(fd[s, c]), (s, c, g[s, c], fd[s, c])
    # the context ends exactly where a plain forward run of n steps ends
    after = sim.read()
    ref = gpu_sim(p, f, off, 8)
    ref.seed(sp, x, d, q, v=v0)
    ref.step(n)
    r = ref.read()
    for k in ("x", "v", "a"):
        assert np.array_equal(after[k], r[k]), k
    assert sim.tally() == ref.tally()


def test_fp64_adjoint_matches_gpu_finite_differences_and_is_checkpoint_invariant():
    p, f, x, d, q, off, sp, v0 = sensitive_case(seed=9)
    n = 24
    say("case: adjoint fp64 vs gpu FD, checkpoint invariance")
    sim = gpu_sim(p, f, off, 8)
    grads = []
    for ce in (1, 5, 24):
        sim.seed(sp, x, d, q, v=v0)
        grads.append(sim.adjoint(n, ce))
    assert np.array_equal(grads[0], grads[1]) and np.array_equal(grads[0], grads[2])

    def J(spp):
        sim.seed(spp, x, d, q, v=v0)
        sim.step(n)
        return np.array([t["j_soft"] for t in sim.tally()])

    for c in range(2):
        fds = []
        for h in (H_REL, 3 * H_REL):
            hp, hm = sp.copy(), sp.copy()
            hp[:, c] *= 1 + h
            hm[:, c] *= 1 - h
            fds.append((J(hp) - J(hm)) / (2 * h * sp[:, c]))
        assert np.allclose(fds[0], fds[1], rtol=2e-4, atol=0)      # smooth over the +-3h interval
        assert np.allclose(grads[0][:, c], fds[0], rtol=1e-3, atol=0), (c, grads[0][:, c], fds[0])


def snap_to_fp32_lattice(x, p):
    """Positions rounded to the FP32 form's fixed-point lattice (x to L/2^32, y and z to R/2^30), which
    the FP64 form holds exactly: both forms then start from the same positions."""
    ux, ur = p["L"] / 2.0 ** 32, p["R"] / 2.0 ** 30
    y = np.array(x, dtype=np.float64)
    y[:, 0] = np.round(np.mod(y[:, 0], p["L"]) / ux) * ux
    y[:, 1:] = np.round(y[:, 1:] / ur) * ur
    return y


@pytest.mark.parametrize("name", ["drag+image", "coulomb", "contact+pair-vdw", "drag+wall-vdw", "all"])
def test_fp32_adjoint_per_force_family(name):
    """Each force family alone, and all together, from the same start in both forms (positions on the FP32
    lattice): the FP32 adjoint against the FP64 adjoint per entry after one step (the reverse kernels'
    own arithmetic) and after 16 steps (plus the FP32 trajectory's departure from the FP64 one), within
    1e-5.  The Coulomb family's bound is 5e-4: its pairs sit within a diameter of each other next to the
    wall, where the FP32 pair records hold y and z to 64 position quanta (relative 6e-5 of a 10 um
    separation, about 3x that in the Jacobian of the pair force)."""
    fam = FORCE_SETS.get(name, {})
    tol = 5e-4 if name == "coulomb" else 1e-5
    say("case: fp32 vs fp64 adjoint, family", name)
    for n in (1, 16):
        p, f, x, d, q, off, sp, v0 = sensitive_case(seed=17)
        p.update(fam)
        x = snap_to_fp32_lattice(x, p)
        g = {}
        for rb in (8, 4):
            sim = gpu_sim(p, f, off, rb)
            sim.seed(sp, x, d, q, v=v0)
            g[rb] = sim.adjoint(n, min(n, 5))
        ref = g[8][:, :2]
        used = np.abs(ref) > 0
        rel = np.abs(g[4][:, :2] - ref)[used] / np.abs(ref)[used]
        say(name, "steps", n, "fp64", ref.tolist(), "largest relative deviation per entry", rel.max())
        assert used.sum() >= 2
        assert np.all(g[4][:, :2][~used] == 0.0)
        assert rel.max() < tol, (name, n, rel)


def test_fp32_adjoint_close_to_fp64_adjoint():
    p, f, x, d, q, off, sp, v0 = sensitive_case(seed=10)
    n, ce = 20, 10
    say("case: adjoint fp32 vs fp64")
    g = {}
    for rb in (8, 4):
        sim = gpu_sim(p, f, off, rb)
        sim.seed(sp, x, d, q, v=v0)
        g[rb] = sim.adjoint(n, ce)
    say("fp64", g[8][:, :2].tolist(), "fp32", g[4][:, :2].tolist())
    assert np.allclose(g[4][:, :2], g[8][:, :2], rtol=5e-4, atol=0)


@pytest.mark.parametrize("shape", [(4, 1), (2, 2), (4, 2), (8, 1)])
def test_fp32_symmetric_pair_adjoint_matches_one_sided(shape):
    """Two samples of uneven size (several tiles each, ragged last tile): the symmetric pair adjoint
    (each pair once, antisymmetric reaction) agrees with the one-sided pair adjoint and with the FP64
    adjoint; a second symmetric run with another checkpoint interval (ragged segments) agrees to FP64
    rounding of the atomic combination."""
    from paper_2205_04979_amd.depo import PAIR_KAHAN, PAIR_SYMMETRIC
    p, f, x, d, q, off, sp, v0 = sensitive_case(n_per=1000, seed=12)
    off = np.array([0, 1300, 2000])
    n, ce = 20, 10
    say("case: symmetric pair adjoint, shape", shape, "samples", np.diff(off).tolist())
    g = {}
    for key in ("sym", "sym2", "one", "fp64"):
        sim = gpu_sim(p, f, off, 8 if key == "fp64" else 4)
        if key.startswith("sym"):
            sim.set_kernel_config(shape[0], shape[1], 64, mode=PAIR_SYMMETRIC)
        elif key == "one":
            sim.set_kernel_config(1, 8, 32, mode=PAIR_KAHAN)
        sim.seed(sp, x, d, q, v=v0)
        g[key] = sim.adjoint(n, 7 if key == "sym2" else ce)[:, :2]
    say({k: v.tolist() for k, v in g.items()})
    assert np.all(np.abs(g["fp64"]) > 0)
    assert np.allclose(g["sym"], g["sym2"], rtol=1e-12, atol=0)
    assert np.allclose(g["sym"], g["one"], rtol=5e-4, atol=0)
    assert np.allclose(g["sym"], g["fp64"], rtol=5e-4, atol=0)


def test_autograd_function_backward():
    import torch
    from paper_2205_04979_amd.depo import DepositionFn
    p, f, x, d, q, off, sp, v0 = sensitive_case(seed=11)
    n, ce = 12, 4
    sim = gpu_sim(p, f, off, 8)
    cs = torch.tensor(sp[:, 0], dtype=torch.float64, requires_grad=True)
    A = torch.tensor(sp[:, 1], dtype=torch.float64, requires_grad=True)
    T = torch.tensor(sp[:, 2], dtype=torch.float64, requires_grad=True)
    J = DepositionFn.apply(cs, A, T, sim, dict(x=x, d=d, qbase=q, v=v0), n, ce)
    w = torch.tensor([2.0, -0.5], dtype=torch.float64)
    (J * w).sum().backward()
    sim.seed(sp, x, d, q, v=v0)
    g = sim.adjoint(n, ce)
    assert np.allclose(cs.grad.numpy(), w.numpy() * g[:, 0], rtol=1e-12)
    assert np.allclose(A.grad.numpy(), w.numpy() * g[:, 1], rtol=1e-12)
    assert np.all(T.grad.numpy() == 0.0)
    # forward runs only the checkpointed forward: J equals a plain forward run's, and a state change
    # between forward and backward (here one more step) makes the backward an error, not a wrong answer
    from paper_2205_04979_amd.depo import DepoError, E_STATE
    J2 = DepositionFn.apply(cs, A, T, sim, dict(x=x, d=d, qbase=q, v=v0), n, ce)
    ref = gpu_sim(p, f, off, 8)
    ref.seed(sp, x, d, q, v=v0)
    ref.step(n)
    assert np.array_equal(J2.detach().numpy(), np.array([t["j_soft"] for t in ref.tally()]))
    sim.step(1)
    with pytest.raises(DepoError) as ei:
        J2.sum().backward()
    assert ei.value.status == E_STATE


FORCE_SETS = {
    "drag+image": dict(drag=True, coulomb=False, collide=False, vdw=False, wall_image=True, wall_vdw=False),
    "coulomb": dict(drag=False, coulomb=True, collide=False, vdw=False, wall_image=False, wall_vdw=False),
    "contact+pair-vdw": dict(drag=False, coulomb=False, collide=True, vdw=True, wall_image=False, wall_vdw=False),
    "drag+wall-vdw": dict(drag=True, coulomb=False, collide=False, vdw=False, wall_image=False, wall_vdw=True),
}


@pytest.mark.parametrize("name", list(FORCE_SETS))
def test_fp64_adjoint_per_force_family(name):
    """Each force family alone: adjoint against central differences of the library's FP64 forward run
    (itself at round-off parity with the oracle); parameters a family does not use have gradient 0.
    Smoothness over the interval is checked with a second, coarser step (3h): a finer step would move
    particles by only a few 64-bit fixed-point position quanta and measure rounding instead."""
    p, f, x, d, q, off, sp, v0 = sensitive_case(seed=17)
    p.update(FORCE_SETS[name])
    n, ce = 16, 5
    say("case: adjoint family", name)
    sim = gpu_sim(p, f, off, 8)
    sim.seed(sp, x, d, q, v=v0)
    g = sim.adjoint(n, ce)

    def J(spp):
        sim.seed(spp, x, d, q, v=v0)
        sim.step(n)
        return np.array([t["j_soft"] for t in sim.tally()])

    for c in range(2):
        fds = []
        for h in (H_REL, 3 * H_REL):
            hp, hm = sp.copy(), sp.copy()
            hp[:, c] *= 1 + h
            hm[:, c] *= 1 - h
            fds.append((J(hp) - J(hm)) / (2 * h * sp[:, c]))
        say(name, "param", c, "adjoint", g[:, c].tolist(), "fd", fds[0].tolist(), fds[1].tolist())
        if np.all(fds[0] == 0.0) and np.all(fds[1] == 0.0):
            assert np.all(g[:, c] == 0.0)
            continue
        assert np.allclose(fds[0], fds[1], rtol=2e-4, atol=0)
        assert np.allclose(g[:, c], fds[0], rtol=1e-3, atol=0), (name, c, g[:, c], fds[0])


def test_adjoint_64x16k_full_size():
    """The adjoint workload the benchmark times, at full size (64 samples x 16,384 particles, 100 steps,
    checkpoints every 10).  FP32 with the symmetric pair adjoint (the benchmark's configuration): its own
    forward run gives bitwise the J of a plain forward run, and its gradient agrees with the one-sided FP32
    pair adjoint and with the FP64 adjoint.  FP64: the adjoint agrees with central differences of the
    library's FP64 forward run, for all samples at once (a sample's J depends only on its own parameters),
    on the samples whose J is smooth over the difference interval.  Every comparison is per entry
    (relative to the FP64 adjoint's entry) over the entries larger than 1e-3 of their column's largest,
    held to 1e-3."""
    from paper_2205_04979_amd.depo import PAIR_KAHAN, PAIR_SYMMETRIC
    w = make_workload("adjoint-64x16k")
    f = w.field()
    n, ce = w.steps, w.extra["ckpt_every"]
    sp = w.sample_params
    say("case: adjoint-64x16k full size, S =", w.n_samples, "N =", w.n_particles, "steps", n, "ckpt", ce)

    def J(sim, spp):
        sim.seed(spp, w.x, w.d, w.qbase)
        sim.step(n)
        return np.array([t["j_soft"] for t in sim.tally()])

    g = {}
    for key in ("sym", "one", "fp64"):
        sim = gpu_sim(w.params, f, w.offsets, 8 if key == "fp64" else 4)
        if key == "sym":
            sim.set_kernel_config(4, 1, 64, mode=PAIR_SYMMETRIC)
        elif key == "one":
            sim.set_kernel_config(1, 8, 32, mode=PAIR_KAHAN)
        j_fwd = J(sim, sp) if key != "one" else None
        sim.seed(sp, w.x, w.d, w.qbase)
        g[key] = sim.adjoint(n, ce)
        if j_fwd is not None:
            assert np.array_equal(j_fwd, np.array([t["j_soft"] for t in sim.tally()])), key
        say(key, "gradient of sample 0", g[key][0].tolist())
        if key == "fp64":
            fd = np.zeros((2, w.n_samples, 2))
            for c in range(2):
                for k, h in enumerate((H_REL, 3 * H_REL)):
                    hp, hm = sp.copy(), sp.copy()
                    hp[:, c] *= 1 + h
                    hm[:, c] *= 1 - h
                    fd[k, :, c] = (J(sim, hp) - J(sim, hm)) / (2 * h * sp[:, c])
        del sim
    for c in range(2):
        ref = g["fp64"][:, c]
        scale = np.abs(ref).max()
        assert scale > 0
        # per entry, wherever the gradient is not negligible against the column's largest entry
        big = np.abs(ref) > 1e-3 * scale
        dev = {k: (np.abs(v[:, c] - ref) / np.abs(ref))[big].max() for k, v in g.items() if k != "fp64"}
        dev["sym-one"] = (np.abs(g["sym"][:, c] - g["one"][:, c]) / np.abs(ref))[big].max()
        # finite differences measure the derivative only where J is smooth over the +-3h interval (a
        # cohesion cutoff crossing inside it is a jump): such samples show as disagreeing h and 3h
        # differences and are left out of the FD comparison, and counted
        smooth = big & (np.abs(fd[0, :, c] - fd[1, :, c]) <= 2e-4 * np.abs(fd[0, :, c]))
        dev["fd"] = (np.abs(fd[0, :, c] - ref) / np.abs(ref))[smooth].max()
        say("column", c, "entries", int(big.sum()), "smooth over +-3h", int(smooth.sum()),
            "largest relative deviation per entry", dev)
        assert big.sum() >= 32 and smooth.sum() >= 0.75 * big.sum()
        assert dev["fd"] < 1e-3 and dev["sym"] < 1e-3 and dev["one"] < 1e-3 and dev["sym-one"] < 5e-4, (c, dev)
    assert np.all(g["sym"][:, 2] == 0) and np.all(g["fp64"][:, 2] == 0)
