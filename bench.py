"""Benchmark of the particle-deposition step on one MI355X.

A step is one pass of the whole hot path over every particle: half kick with
exponential drag, drift, wall test and removal, cell-list build, direct
Coulomb sums, short-range contact and cohesion, wall terms, trilinear gather,
second half kick.  The default workload is the 65,536-particle single sample
(lognormal diameters, Gaussian charges, 128^3 field, all forces) timed over
2,000 steps with inputs resident in HBM.

Prints one JSON line with the throughput (particle-steps/s), the roofline of
the dominant kernel (the Coulomb pair sums, bound by FP32 vector ALU; its
average launch duration is measured with HIP events on the launch stream
during the timed region) and the FP64 CPU oracle timed on a bounded sample of
the same workload on the host cores.
"""

from __future__ import annotations

import argparse
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_FP32_VECTOR_TFLOPS = 157.3       # MI355X published FP32 vector peak (packed FP32 FMA)
NONPACKED_FMA_TFLOPS = 78.6           # 256 CU x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz: one FMA per lane per cycle
FLOPS_PER_PAIR = 20                   # customary N-body count per interaction
HOST_CORE_SHARE = 16                  # host cores that go with one GPU on the benchmark machine
REORDER = 16                          # steps between storage reorders in the batched, large and p3m legs


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def _oracle_worker(args):
    sim, targets = args
    t0 = time.perf_counter()
    from oracle.gather import trilinear
    from oracle import physics as ph
    idx = np.asarray(targets)
    # the O(N) parts of the step for these targets, then their O(N) pair sums
    p = sim.p
    v = ph.drag_half_kick(sim.v[idx], sim.uf[idx], sim.a[idx], sim.d[idx], 0.5 * sim.dt,
                          p["rho_p"], p["rho_f"], p["nu"], p["drag"])
    sim.accelerations(idx, chunk=32)
    u = trilinear(sim.field, sim.R, sim.L, sim.x[idx])
    ph.drag_half_kick(v, u, sim.a[idx], sim.d[idx], 0.5 * sim.dt, p["rho_p"], p["rho_f"], p["nu"], p["drag"])
    return time.perf_counter() - t0


_SIM = None


def _run_chunk(targets):
    return _oracle_worker((_SIM, targets))


def cpu_baseline(w, field, n_targets: int):
    """Time the FP64 oracle on n_targets particles of the workload (all N sources each)."""
    global _SIM
    from oracle.sim import OracleSim
    _SIM = OracleSim(w.params, field, w.x, w.d, w.qbase, w.offsets, w.sample_params, evaluate=False)
    visible = len(os.sched_getaffinity(0))
    cores = min(HOST_CORE_SHARE, visible)
    rng = np.random.default_rng(12345)
    n_targets = min(n_targets, w.n_particles)
    targets = np.sort(rng.choice(w.n_particles, n_targets, replace=False))
    which = (f"all {n_targets} particles" if n_targets == w.n_particles
             else f"{n_targets} randomly chosen particles")
    chunks = np.array_split(targets, cores * 2)
    ctx = mp.get_context("fork")
    t0 = time.perf_counter()
    with ctx.Pool(cores) as pool:
        pool.map(_run_chunk, chunks)
    wall = time.perf_counter() - t0
    return dict(value=n_targets / wall, unit="particle-steps/s", cores=cores, kind="oracle",
                sample=f"{which} of the {w.name} workload, one full step each "
                       f"(drag kicks, gather, all {w.n_particles} Coulomb sources, short-range and wall terms), "
                       f"FP64 NumPy, {cores} processes on {cores} host cores (every core of this GPU's host share; "
                       f"{visible} visible)",
                seconds=wall)


def _force_chunk(targets):
    _SIM.accelerations(np.asarray(targets), chunk=8)   # 8 x 2^20 pair arrays per pass (~0.2 GB each)
    return len(targets)


def oracle_timings() -> dict:
    """The FP64 oracle on the host cores, as context for the GPU figures: the 1,024-particle FP64
    workload run in full (200 steps, one process: each step is one vectorised pass over all pairs),
    and the 2^20-particle force check (4,096 targets, index = 0 mod 256, over all sources, on a pool of
    processes)."""
    global _SIM
    from oracle.sim import OracleSim
    from synthetic import make_workload
    cores = min(HOST_CORE_SHARE, len(os.sched_getaffinity(0)))
    out = {"cores": cores}
    w = make_workload("plain-1k")
    f = w.field()
    sim = OracleSim(w.params, f, w.x, w.d, w.qbase, w.offsets, w.sample_params)
    t0 = time.perf_counter()
    sim.step(w.steps)
    wall = time.perf_counter() - t0
    n = w.n_particles
    out["plain-1k"] = {"steps": w.steps, "seconds": round(wall, 2), "particle_steps_per_s": round(n * w.steps / wall, 1),
                       "ordered_pairs_per_s": round(n * (n - 1) * w.steps / wall, 1), "processes": 1}
    log(f"[bench] oracle plain-1k: {out['plain-1k']}")
    w = make_workload("large-1m")
    f = w.field()
    _SIM = OracleSim(w.params, f, w.x, w.d, w.qbase, w.offsets, w.sample_params, evaluate=False)
    targets = np.arange(0, w.n_particles, 256)
    chunks = np.array_split(targets, cores * 4)
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(cores) as pool:
        pool.map(_force_chunk, chunks)
    wall = time.perf_counter() - t0
    out["large-1m force check"] = {"targets": int(targets.size), "sources": w.n_particles, "seconds": round(wall, 2),
                                   "ordered_pairs_per_s": round(targets.size * (w.n_particles - 1) / wall, 1),
                                   "processes": cores}
    log(f"[bench] oracle large-1m force check: {out['large-1m force check']}")
    return out


def kernel_source_digest(name: str) -> str:
    import hashlib
    src = os.path.join(ROOT, "paper_2205_04979_amd", "csrc", name)
    return hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]


def pair_kernel_source(shape) -> str:
    """Source file of the pair kernel a shape selects (4th entry 2: the symmetric kernel)."""
    return "k_coulomb_sym.hip" if len(shape) > 3 and shape[3] == 2 else "k_coulomb.hip"


def pair_kernel_name(shape) -> str:
    if len(shape) > 3 and shape[3] == 2:
        return f"k_coulomb_sym<{shape[0]}, {shape[1]}> + k_pair_finish (symmetric direct pair sums)"
    return f"k_coulomb<float, {shape[0]}, {shape[1]}, {shape[2]}> (one-sided direct pair sums)"


def measured_traffic(shape):
    """HBM bytes per pair-kernel launch from the committed counter summary, if it was taken on this
    exact kernel source and shape; otherwise None."""
    path = os.path.join(ROOT, "profiles", "pair_kernel_single65k_hbm_counters.json")
    if not os.path.exists(path):
        return None
    src = pair_kernel_source(shape)
    for rec in json.load(open(path))["records"]:
        if rec.get("source") == src and rec.get("sha256_16") == kernel_source_digest(src) and \
                tuple(rec.get("shape", ())) == tuple(shape):
            return rec.get("bytes_per_launch")
    return None


def sequential_estimate(w, field, steps: int = 20, strata: int = 8, per_stratum: int = 2) -> dict:
    """Per-step time of running the batch's samples one after another as single-sample simulations (the
    plain single-sample step, library defaults, graph replay), estimated from a stratified subset: the
    samples are sorted by size into equal strata, ``per_stratum`` of each (seeded choice) are timed over
    ``steps`` steps, and each stratum's total is its size times the mean time of its picks."""
    import torch
    from paper_2205_04979_amd.depo import Simulation
    sizes = np.diff(w.offsets)
    order = np.argsort(sizes, kind="stable")
    rng = np.random.default_rng(2024)
    total_ms, picked = 0.0, []
    for grp in np.array_split(order, strata):
        picks = rng.choice(grp, min(per_stratum, grp.size), replace=False)
        times = []
        for s in picks:
            b, e = int(w.offsets[s]), int(w.offsets[s + 1])
            sim = Simulation(w.params, np.array([0, e - b]), field.shape[:3], real_bytes=4, device="cuda:0")
            sim.init_field(field)
            sim.seed(w.sample_params[s:s + 1], w.x[b:e], w.d[b:e], w.qbase[b:e])
            sim.step(3)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            sim.step(steps)
            torch.cuda.synchronize()
            times.append(1e3 * (time.perf_counter() - t0) / steps)
            picked.append([int(s), e - b, round(times[-1], 4)])
            sim.close()
        total_ms += grp.size * float(np.mean(times))
    return {"ms_per_step": round(total_ms, 4), "steps_timed_per_sample": steps,
            "timed_samples": picked,
            "method": f"{strata} size strata of the {w.n_samples} samples, {per_stratum} timed per stratum as "
                      f"single-sample simulations; stratum total = its size x the mean of its picks"}


def batched_run(steps: int = 0) -> dict:
    """The 256-sample Monte Carlo batch (uneven sample sizes, one launch per kernel family, graph replay):
    the whole run (``steps`` = 0: the workload's 1,000 steps) timed, against the same samples stepped one
    after another as single-sample simulations (estimated from a stratified subset)."""
    import torch
    from paper_2205_04979_amd.autotune import autotune
    from paper_2205_04979_amd.depo import Simulation
    from synthetic import make_workload
    w = make_workload("batched-256")
    field = w.field()
    steps = steps or w.steps
    log(f"[bench] batched-256: S={w.n_samples} N={w.n_particles}, {steps} steps timed")
    sim = Simulation(w.params, w.offsets, field.shape[:3], real_bytes=4, device="cuda:0")
    sim.init_field(field)
    sim.seed(w.sample_params, w.x, w.d, w.qbase)
    shape, _ = autotune(sim, steps=1)
    sim.set_reorder(REORDER)
    sim.step(2)                       # warm the kernels up, then start the run from the seeded state
    sim.seed(w.sample_params, w.x, w.d, w.qbase)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    n_ph = 20
    ph = sim.step_timed(n_ph)
    ms = 1e3 * wall / steps
    pairs = float(np.sum(np.diff(w.offsets).astype(np.float64) ** 2))
    coul = ph["coulomb"] / n_ph
    del sim
    torch.cuda.empty_cache()
    seq = sequential_estimate(w, field)
    res = {"workload": w.name, "samples": w.n_samples, "particles": w.n_particles, "steps_timed": steps,
           "wall_s": round(wall, 4), "ms_per_step": round(ms, 4),
           "samples_per_s": round(w.n_samples * steps / (w.steps * wall), 4),
           "sample_steps_per_s": round(w.n_samples * 1e3 / ms, 1),
           "particle_steps_per_s": round(w.n_particles * 1e3 / ms, 1),
           "coulomb_ms": round(coul, 4), "ordered_pairs_per_s": round(pairs / (coul * 1e-3), 1),
           "pair_kernel_shape": list(shape), "reorder_every": REORDER,
           "sequential_single_sample": seq,
           "batched_speedup_over_sequential": round(seq["ms_per_step"] / ms, 3),
           "note": (f"samples/s = {w.n_samples} samples / wall time of the {w.steps}-step run"
                    + ("" if steps == w.steps else f" (scaled from {steps} timed steps)"))}
    log(f"[bench] batched: {res}")
    return res


def large_run(steps: int = 5) -> dict:
    """The 2^20-particle single sample with the direct O(N^2) Coulomb sums (the FP32 default pair kernel):
    particle-steps/s over ``steps`` graph-replayed steps and the pair kernel's roofline fraction."""
    import torch
    from paper_2205_04979_amd.autotune import autotune
    from paper_2205_04979_amd.depo import Simulation
    from synthetic import make_workload
    w = make_workload("large-1m")
    field = w.field()
    log(f"[bench] large-1m direct: N={w.n_particles}, {steps} steps")
    sim = Simulation(w.params, w.offsets, field.shape[:3], real_bytes=4, device="cuda:0")
    sim.init_field(field)
    sim.seed(w.sample_params, w.x, w.d, w.qbase)
    # the two symmetric shapes that lead at this size (a step takes ~0.2 s, so not the full list);
    # tuning restores the state, and the storage reorder is enabled after it
    shape, _ = autotune(sim, steps=1, shapes=[(4, 2, 64, 2), (4, 4, 64, 2)], refine=2, rounds=2)
    sim.set_reorder(REORDER)
    sim.step(2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ph = sim.step_timed(steps)
    N = w.n_particles
    coul = ph["coulomb"] / steps
    achieved = float(N) * (N - 1) / 2.0 * FLOPS_PER_PAIR / (coul * 1e-3) / 1e12
    res = {"workload": w.name, "particles": N, "steps_timed": steps, "ms_per_step": round(1e3 * wall / steps, 3),
           "particle_steps_per_s": round(N * steps / wall, 1), "pair_kernel": pair_kernel_name(shape),
           "pair_kernel_shape": list(shape),
           "coulomb_ms": round(coul, 3), "achieved_tflops": round(achieved, 3),
           "frac": round(achieved / PEAK_FP32_VECTOR_TFLOPS, 4),
           "frac_of_nonpacked_fma_peak": round(achieved / NONPACKED_FMA_TFLOPS, 4),
           "phase_ms_per_step": {k: round(v / steps, 4) for k, v in ph.items()}, "reorder_every": REORDER}
    log(f"[bench] large: {res}")
    sim.close()
    del sim
    torch.cuda.empty_cache()
    return res


def adjoint_run() -> dict:
    """Adjoint/forward cost on the 64 x 16,384 workload: 100 steps, checkpoints every 10 steps."""
    import torch
    from paper_2205_04979_amd.autotune import FP32_SYM_SHAPES, autotune
    from paper_2205_04979_amd.depo import Simulation
    from synthetic import make_workload
    w = make_workload("adjoint-64x16k")
    field = w.field()
    n, ce = w.steps, w.extra["ckpt_every"]
    log(f"[bench] adjoint-64x16k: S={w.n_samples} N={w.n_particles} steps={n} ckpt={ce}")
    sim = Simulation(w.params, w.offsets, field.shape[:3], real_bytes=4, device="cuda:0")
    sim.init_field(field)
    sim.seed(w.sample_params, w.x, w.d, w.qbase)
    # symmetric shapes only (the pair adjoint runs the forward's items); tuning restores the state
    shape, _ = autotune(sim, steps=1, shapes=FP32_SYM_SHAPES)
    sim.step(2)                       # warm the kernels up
    sim.seed(w.sample_params, w.x, w.d, w.qbase)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(n)
    torch.cuda.synchronize()
    fwd = time.perf_counter() - t0
    j_fwd = [t["j_soft"] for t in sim.tally()]
    sim.seed(w.sample_params, w.x, w.d, w.qbase)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    g = sim.adjoint(n, ce)
    torch.cuda.synchronize()
    adj = time.perf_counter() - t1
    j_adj = [t["j_soft"] for t in sim.tally()]
    res = {"workload": w.name, "samples": w.n_samples, "particles": w.n_particles, "steps": n, "ckpt_every": ce,
           "pair_kernel_shape": list(shape),
           "forward_s": round(fwd, 4), "adjoint_s": round(adj, 4), "adjoint_over_forward": round(adj / fwd, 3),
           "note": "adjoint_s includes its own forward run with checkpoints, the per-segment recomputation "
                   "and the reverse sweep; both start from the seeded state",
           "same_J_as_forward": bool(j_fwd == j_adj),
           "grad_charge_scale_sample0": g[0, 0], "grad_hamaker_sample0": g[0, 1],
           "grad_temperature_all_zero": bool(np.all(g[:, 2] == 0.0))}
    log(f"[bench] adjoint: {res}")
    del sim
    torch.cuda.empty_cache()
    return res


def rebound_run() -> dict:
    """The temperature study of Section 4.4: 64 samples x 16,384 particles, theta ~ U[0, 1], rebound law,
    the whole 1,000-step run timed; reports throughput and the capture efficiency (Eq. CE) per sample."""
    import torch
    from paper_2205_04979_amd.autotune import FP32_SYM_SHAPES, autotune
    from paper_2205_04979_amd.depo import Simulation
    from synthetic import make_workload
    w = make_workload("rebound-theta-64")
    field = w.field()
    log(f"[bench] rebound-theta-64: S={w.n_samples} N={w.n_particles} steps={w.steps}")
    sim = Simulation(w.params, w.offsets, field.shape[:3], real_bytes=4, device="cuda:0")
    sim.init_field(field)
    sim.seed(w.sample_params, w.x, w.d, w.qbase)
    # symmetric shapes only (the pair adjoint runs the forward's items); tuning restores the state
    shape, _ = autotune(sim, steps=1, shapes=FP32_SYM_SHAPES)
    sim.step(2)                       # warm the kernels up
    sim.seed(w.sample_params, w.x, w.d, w.qbase)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(w.steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    tal = sim.tally()
    ce = np.array([t["ce"] for t in tal])
    theta = 0.225 * (w.sample_params[:, 2] - 1000.0) / 200.0
    hot = theta >= 0.9
    res = {"workload": w.name, "samples": w.n_samples, "particles": w.n_particles, "steps": w.steps,
           "dt": w.params["dt"], "pair_kernel_shape": list(shape), "wall_s": round(wall, 4), "ms_per_step": round(1e3 * wall / w.steps, 4),
           "samples_per_s": round(w.n_samples / wall, 4),
           "particle_steps_per_s": round(w.n_particles * w.steps / wall, 1),
           "deposited": int(sum(t["n_dep"] for t in tal)),
           "ce_mean": float(ce.mean()), "ce_std": float(ce.std(ddof=1)),
           "ce_mean_theta_below_0.9": float(ce[~hot].mean()) if np.any(~hot) else None,
           "ce_mean_theta_above_0.9": float(ce[hot].mean()) if np.any(hot) else None,
           "ce_corr_with_theta": float(np.corrcoef(theta, ce)[0, 1]),
           "ce_corr_with_zeta": float(np.corrcoef(w.extra["zeta"], ce)[0, 1])}
    log(f"[bench] rebound: {res}")
    del sim
    torch.cuda.empty_cache()
    return res


def plain_run() -> dict:
    """The 1,024-particle workload in the FP64 form (plain sums), run in full: 200 steps by graph
    replay.  Small enough that launch latency, not arithmetic, sets the time."""
    import torch
    from paper_2205_04979_amd.depo import Simulation
    from synthetic import make_workload
    w = make_workload("plain-1k")
    field = w.field()
    sim = Simulation(w.params, w.offsets, field.shape[:3], real_bytes=8, device="cuda:0")
    sim.init_field(field)
    sim.seed(w.sample_params, w.x, w.d, w.qbase)
    from paper_2205_04979_amd.autotune import autotune
    shape, tune = autotune(sim, steps=5)
    sim.step(w.steps)                 # warm-up run (graph capture, clocks)
    sim.seed(w.sample_params, w.x, w.d, w.qbase)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(w.steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ph = sim.step_timed(20)
    res = {"workload": w.name, "particles": w.n_particles, "steps": w.steps, "dtype": "f64",
           "wall_s": round(wall, 5), "ms_per_step": round(1e3 * wall / w.steps, 4),
           "particle_steps_per_s": round(w.n_particles * w.steps / wall, 1),
           "coulomb_ms_per_step": round(ph["coulomb"] / 20, 4), "pair_kernel_shape": list(shape),
           "autotune_ms_per_step": {",".join(map(str, k)): round(v, 4) for k, v in tune.items()}}
    log(f"[bench] plain: {res}")
    sim.close()
    del sim
    torch.cuda.empty_cache()
    return res


def lf_run() -> dict:
    """The low-fidelity model (Appendix B) over the LF-only Monte Carlo budget of Table 3 at p = 36:
    25,920 particle classes (d in {1.6, 5, 16} um, xi ~ U[0, 0.1], zeta ~ U[0, 1]) per launch."""
    import torch
    from paper_2205_04979_amd.depo import lf_solve
    from synthetic.workloads import physical_params, q_max
    rng = np.random.default_rng(11)
    n = 25920
    p = physical_params(180.0)
    d = rng.choice([1.6e-6, 5e-6, 16e-6], n)
    q = rng.uniform(0, 0.1, n) * q_max(d)
    A = rng.uniform(0, 1, n) * 1e-18
    dev = [torch.from_numpy(a).to("cuda:0") for a in (d, q, A)]
    out = torch.empty(n, dtype=torch.float64, device="cuda:0")
    from paper_2205_04979_amd import depo as dp
    import ctypes as C
    cp = dp.make_params(p)
    args = [C.byref(cp), n] + [C.c_void_p(t.data_ptr()) for t in dev] + [800, 800, C.c_void_p(out.data_ptr()),
                                                                         C.c_void_p(torch.cuda.current_stream().cuda_stream)]
    L = dp.lib()
    assert L.depo_lf_solve(*args) == 0
    torch.cuda.synchronize()
    reps = 5
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(reps):
        assert L.depo_lf_solve(*args) == 0
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / reps
    res = {"classes": n, "nodes": 1600, "ms_per_launch": round(ms, 4), "classes_per_s": round(n / (ms * 1e-3), 1),
           "vdep_plus_median": float(np.median(out.cpu().numpy())),
           "note": "one lane per class, single inward pass (momentum march with the flux carried as an affine map)"}
    log(f"[bench] lf: {res}")
    return res


def mfmc_run(budget: float = 36.0, n_pilot: int = 16, hf_steps: int = 200) -> dict:
    """The multi-fidelity estimator of Section 3 end to end on the GPU models: V_dep+ of the particle
    step (16,384 particles of the temperature-study recipe, rebound law, 200 steps of 1e-5 s; every
    input point one sample of one batched launch) as the high-fidelity model and the one-dimensional
    Eulerian model (d = 10 um) as the low-fidelity one, inputs (xi, zeta, T) with xi ~ U[0, 0.1],
    zeta ~ U[0, 1], T ~ U[1000, 1889] K.  A pilot of 16 points on both models gives sigma, rho_12 and
    the cost ratio (measured wall time per point); the budget of 36 high-fidelity runs (the budget
    of Table 3) is split as p / (d + 2) for the Sobol' indices; the whole estimator is timed."""
    import torch
    from paper_2205_04979_amd import mfmc as pmf
    from synthetic import make_workload
    w = make_workload("rebound-theta-64", n_samples=1, steps=hf_steps)
    field = w.field()
    hf = pmf.HighFidelityGPU(w.params, field, w.x, w.d, steps=hf_steps, real_bytes=4)
    lf = pmf.LowFidelityGPU(w.params, 10e-6)

    def sample(rng, m):
        return np.stack([rng.uniform(0.0, 0.1, m), rng.uniform(0.0, 1.0, m),
                         1000.0 + 200.0 * rng.uniform(0.0, 1.0, m) / 0.225], axis=1)

    log(f"[bench] mfmc: HF {w.n_particles} particles x {hf_steps} steps per input point, pilot {n_pilot}")
    hf(sample(np.random.default_rng(20), 2))          # warm the kernels up
    lf(sample(np.random.default_rng(20), 2))
    pilot = sample(np.random.default_rng(21), n_pilot)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    yh = hf(pilot)
    t1 = time.perf_counter()
    yl = lf(pilot)
    t2 = time.perf_counter()
    w_hf, w_lf = (t1 - t0) / n_pilot, (t2 - t1) / n_pilot
    sigma = (float(yh.std(ddof=1)), float(yl.std(ddof=1)))
    rho12 = float(np.corrcoef(yh, yl)[0, 1])
    res = {"hf_particles": w.n_particles, "hf_steps": hf_steps, "dt": w.params["dt"], "pilot": n_pilot,
           "sigma": sigma, "rho12": rho12, "hf_s_per_point_in_pilot": round(w_hf, 5),
           "lf_s_per_point_in_pilot": round(w_lf, 6), "budget_hf_runs": budget, "inputs": 3}
    try:
        t3 = time.perf_counter()
        r = pmf.mfmc_sobol([hf, lf], sigma, (1.0, rho12), (1.0, w_lf / w_hf), budget, sample, 3,
                           np.random.default_rng(22))
        torch.cuda.synchronize()
        wall = time.perf_counter() - t3
        m1, m2 = int(r.counts[0]), int(r.counts[1])
        res.update({"counts": [m1, m2], "alpha": [float(a) for a in r.alpha], "wall_s": round(wall, 4),
                    "hf_points": 5 * m1, "lf_points": 5 * m2,
                    "hf_particle_steps_per_s": round(5 * m1 * w.n_particles * hf_steps / wall, 1),
                    "mean_vdep_plus": r.mean, "variance": r.variance,
                    "main_effects": [float(v) for v in r.main], "total_effects": [float(v) for v in r.total],
                    "gamma_predicted": pmf.gamma(abs(rho12), 1.0, w_lf / w_hf) if abs(rho12) < 1 else None,
                    "precondition_holds": bool(pmf.precondition_holds((1.0, rho12), (1.0, w_lf / w_hf))),
                    "note": "one batched HF launch and one LF launch per estimator call; wall_s includes "
                            "seeding, field upload and tally readback of the HF batch; the indices come from "
                            "m1 = counts[0] HF samples, so the estimators (Owen's main effect can be negative) "
                            "are noisy at this budget"})
    except ValueError as e:   # degenerate pilot statistics
        res["error"] = str(e)
    log(f"[bench] mfmc: {res}")
    torch.cuda.empty_cache()
    return res


P3M_CONFIGS = {"single-65k": dict(mesh_x=128, mesh_yz=64, alpha_h=0.5, rmax_alpha=3.5),
               "large-1m": dict(mesh_x=256, mesh_yz=128, alpha_h=0.5, rmax_alpha=3.5)}


def p3m_run(steps: int = 5, names=None) -> dict:
    """P3M electrostatics (the x-periodic lattice sum, O(N log N)) against the direct symmetric sums
    (nearest image, O(N^2)): per-step Coulomb-phase time of the full step on the single-65k and
    large-1m workloads."""
    import torch
    from paper_2205_04979_amd.depo import Simulation
    from synthetic import make_workload
    out = {}
    for name, cfg in P3M_CONFIGS.items():
        if names is not None and name not in names:
            continue
        w = make_workload(name)
        field = w.field()
        res = {"particles": w.n_particles, "mesh": [cfg["mesh_x"], 2 * cfg["mesh_yz"], 2 * cfg["mesh_yz"]],
               "alpha_h": cfg["alpha_h"], "rmax_alpha": cfg["rmax_alpha"], "reorder_every": REORDER}
        for kind in ("p3m", "direct"):
            log(f"[bench] p3m leg: {name} {kind}")
            sim = Simulation(w.params, w.offsets, field.shape[:3], real_bytes=4, device="cuda:0",
                             p3m=cfg if kind == "p3m" else None)
            sim.set_reorder(REORDER)
            sim.init_field(field)
            if kind == "direct":
                sim.set_kernel_config(4, 2, 64, 2)
            sim.seed(w.sample_params, w.x, w.d, w.qbase)
            sim.step(1)
            torch.cuda.synchronize()
            # warm up for about 0.3 s of steps: the clock ramps up over the first tens of milliseconds
            t0 = time.perf_counter()
            sim.step(1)
            torch.cuda.synchronize()
            sim.step(min(300, int(0.3 / max(time.perf_counter() - t0, 1e-6))))
            torch.cuda.synchronize()
            ph = sim.step_timed(steps)
            res[f"{kind}_coulomb_ms"] = round(ph["coulomb"] / steps, 4)
            res[f"{kind}_step_ms"] = round(sum(ph.values()) / steps, 4)
            sim.close()
            del sim
            torch.cuda.empty_cache()
        res["coulomb_speedup"] = round(res["direct_coulomb_ms"] / res["p3m_coulomb_ms"], 2)
        out[name] = res
        log(f"[bench] p3m leg {name}: {res}")
    out["note"] = ("P3M computes the lattice sum over all x images (relative RMS deviation 4e-4..1.2e-3 from the "
                   "exact lattice sum in the parity tests), the direct modes the nearest-image sum")
    return out


def main():
    global REORDER
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="single-65k")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-targets", type=int, default=65536,
                    help="particles of the workload the CPU oracle steps once (capped at the workload size)")
    ap.add_argument("--kernel", default=None, help="pair-kernel shape ipl,waves,block (skips autotuning)")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--legs", default="single,batched,adjoint,rebound,plain,lf,mfmc,p3m,large",
                    help="which measurements to run: single (the headline), batched, adjoint, rebound, plain, lf, "
                         "p3m, large")
    ap.add_argument("--secondary-steps", type=int, default=1000,
                    help="steps timed for the batched Monte Carlo workload (its whole run is 1,000; 0 disables "
                         "the secondary legs)")
    ap.add_argument("--large-steps", type=int, default=5, help="steps timed in the 2^20-particle direct leg")
    ap.add_argument("--reorder", type=int, default=REORDER,
                    help="steps between storage reorders into cell order in the batched, large and p3m legs "
                         "(0: none); set after the autotuner has run")
    ap.add_argument("--single-reorder", type=int, default=0,
                    help="steps between storage reorders in the headline leg (0: none, the library default)")
    ap.add_argument("--clock-warmup-ms", type=float, default=200.0,
                    help="GPU busy time (matrix products, not steps) right before the warm-up steps")
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="also run one device-to-device copy of this size (reference for HBM counters)")
    ap.add_argument("--p3m-workloads", default=",".join(P3M_CONFIGS),
                    help="workloads of the p3m leg (comma-separated)")
    ap.add_argument("--p3m-steps", type=int, default=5, help="steps timed per workload in the p3m leg")
    ap.add_argument("--oracle-timings", action="store_true",
                    help="only time the FP64 oracle on the host cores (plain-1k in full, the large-1m force "
                         "check); no GPU")
    args = ap.parse_args()
    REORDER = args.reorder
    p3m_names = args.p3m_workloads.split(",")
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only: the library has no multi-GPU path "
                                   "(samples would shard across GPUs with no per-step exchange; a single large "
                                   "sample would all-gather its source records every step)", "n_gpus": args.gpus}))
        sys.exit(2)
    if args.oracle_timings:
        print(json.dumps({"oracle_timings": oracle_timings()}), flush=True)
        return

    legs = set(args.legs.split(","))
    if "single" not in legs:
        # profiling runs of the secondary legs only (no headline line)
        import torch
        assert torch.cuda.is_available(), "bench.py needs a GPU"
        out = {}
        if "batched" in legs:
            out["batched"] = batched_run(args.secondary_steps)
        if "adjoint" in legs:
            out["adjoint"] = adjoint_run()
        if "rebound" in legs:
            out["rebound"] = rebound_run()
        if "plain" in legs:
            out["plain"] = plain_run()
        if "lf" in legs:
            out["lf"] = lf_run()
        if "mfmc" in legs:
            out["mfmc"] = mfmc_run()
        if "p3m" in legs:
            out["p3m"] = p3m_run(args.p3m_steps, p3m_names)
        if "large" in legs:
            out["large"] = large_run(args.large_steps)
        print(json.dumps(out), flush=True)
        return

    from synthetic import make_workload

    log(f"[bench] building inputs for {args.workload}")
    w = make_workload(args.workload)
    field = w.field()
    N = w.n_particles
    cb = None
    if not args.no_cpu_baseline:
        # runs before anything initialises the GPU (the worker processes are forked)
        log(f"[bench] CPU oracle baseline on {args.cpu_targets} targets")
        cb = cpu_baseline(w, field, args.cpu_targets)
        log(f"[bench] CPU oracle {cb['seconds']:.1f} s on {cb['cores']} processes")

    import torch
    from paper_2205_04979_amd.depo import Simulation

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    sim = Simulation(w.params, w.offsets, field.shape[:3], real_bytes=4, device="cuda:0")
    sim.init_field(field)
    sim.seed(w.sample_params, w.x, w.d, w.qbase)
    tune = None
    if args.kernel:
        sim.set_kernel_config(*[int(v) for v in args.kernel.split(",")])
        shape = tuple(int(v) for v in args.kernel.split(","))
    elif not args.no_autotune:
        from paper_2205_04979_amd.autotune import autotune
        shape, tune = autotune(sim, steps=10)
        log(f"[bench] autotuned pair kernel (ms per step): {shape} " +
            ", ".join(f"{k}:{v:.3f}ms" for k, v in tune.items()))
    else:
        shape = (4, 2, 64, 2)          # the library default in FP32
    if args.copy_probe_mb:
        src = torch.empty(args.copy_probe_mb << 20, dtype=torch.uint8, device="cuda:0").fill_(1)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.single_reorder:
        sim.set_reorder(args.single_reorder)
    if args.clock_warmup_ms > 0:
        # keep the GPU busy (plain matrix products, no simulation state touched) until the clocks have
        # ramped up, so that a short timed region does not measure the ramp
        a = torch.rand(2048, 2048, device="cuda:0")
        b = torch.rand(2048, 2048, device="cuda:0")
        t_w = time.perf_counter()
        while time.perf_counter() - t_w < 1e-3 * args.clock_warmup_ms:
            for _ in range(8):
                a = torch.mm(a, b).clamp_(-1.0, 1.0)
            torch.cuda.synchronize()
        del a, b
    log(f"[bench] seeded N={N}; warmup {args.warmup} steps")
    if args.warmup:
        sim.step(args.warmup)
    torch.cuda.synchronize()

    log(f"[bench] timing {args.steps} steps (graph replay, the default stepping path)")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(args.steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    log(f"[bench] {wall:.3f} s")

    # per-phase breakdown with HIP events on the launch stream (direct launches between events), the
    # source of the pair kernel's live duration in the roofline
    p_steps = max(1, args.steps // 4)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    phase_ms = sim.step_timed(p_steps)
    torch.cuda.synchronize()
    wall_phases = time.perf_counter() - t1
    log(f"[bench] {p_steps} instrumented steps: {wall_phases:.3f} s; phases {phase_ms}")
    tal = sim.tally()
    n_alive = sum(t["n_alive"] for t in tal)

    ms_per_step = 1e3 * wall / args.steps
    value = N * args.steps / wall
    coul_ms = phase_ms["coulomb"] / p_steps
    pairs = float(N) * (N - 1) / 2.0
    achieved = pairs * FLOPS_PER_PAIR / (coul_ms * 1e-3) / 1e12
    roofline = {
        "bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP32_VECTOR_TFLOPS, "unit": "TFLOP/s",
        "frac": round(achieved / PEAK_FP32_VECTOR_TFLOPS, 4), "traffic": measured_traffic(shape),
        "kernel": pair_kernel_name(shape), "kernel_ms": round(coul_ms, 5),
        "algorithmic": f"{FLOPS_PER_PAIR} flop per unordered pair x N(N-1)/2 pairs per launch",
        "ordered_pairs_per_s": round(2 * pairs / (coul_ms * 1e-3), 1),
        "frac_of_nonpacked_fma_peak": round(achieved / NONPACKED_FMA_TFLOPS, 4),
    }
    out = {
        "metric": "particle-steps/s at 65k particles; batched samples/s; adjoint/forward cost", "value": round(value, 1), "unit": "particle-steps/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "particles": N, "samples": w.n_samples,
                   "field": f"{w.field_n}^3", "forces": "drag+coulomb+contact+vdw+wall",
                   "alive_at_end": int(n_alive), "pair_kernel_shape": list(shape),
                   "autotune_ms_per_step": None if tune is None else {",".join(map(str, k)): round(v, 4) for k, v in tune.items()}, "ms_per_step_direct_launch_with_events": round(1e3 * wall_phases / p_steps, 5),
                   "phase_ms_per_step": {k: round(v / p_steps, 5) for k, v in phase_ms.items()},
                   "phase_steps": p_steps, "clock_warmup_ms": args.clock_warmup_ms,
                   "reorder_every": args.single_reorder},
        "roofline": roofline,
    }
    if args.secondary_steps > 0 and args.workload == "single-65k":
        if "batched" in legs:
            out["batched"] = batched_run(args.secondary_steps)
        if "adjoint" in legs:
            out["adjoint"] = adjoint_run()
        if "rebound" in legs:
            out["rebound"] = rebound_run()
        if "plain" in legs:
            out["plain"] = plain_run()
        if "lf" in legs:
            out["lf"] = lf_run()
        if "mfmc" in legs:
            out["mfmc"] = mfmc_run()
        if "p3m" in legs:
            out["p3m"] = p3m_run(args.p3m_steps, p3m_names)
        if "large" in legs:
            out["large"] = large_run(args.large_steps)
    if cb is not None:
        out["cpu_baseline"] = {k: cb[k] for k in ("value", "unit", "cores", "kind", "sample")}
        out["cpu_baseline"]["value"] = round(cb["value"], 2)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
