"""Write the stored FP64-oracle reference states that the GPU parity tests compare against.

Every value written here comes from ``oracle/`` (the FP64 NumPy oracle) run on
the seeded inputs of ``synthetic/``; nothing is read from the HIP library.
The oracle's per-target force evaluation is spread over host processes
(``tests/oracle_pool.py``), which changes nothing in what it computes.

Usage (from the repository root)::

    python tests/golden/make_golden.py single65k   # 20 steps of the 65,536-particle workload
    python tests/golden/make_golden.py large4096   # 500 steps of 4,096 particles of the 2^20 recipe
    python tests/golden/make_golden.py p3m65k      # P3M sums of the 65,536-particle workload at seed
    python tests/golden/make_golden.py p3m1m       # P3M sums of 4,096 targets of the 2^20 workload at seed

Each file also stores a digest of the inputs it was made from, so a test can
tell when the generator of a workload has changed since.
"""

from __future__ import annotations

import hashlib
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def input_digest(w, field) -> str:
    """SHA-256 over the seeded inputs of a workload (positions, diameters, charges, parameters, field)."""
    h = hashlib.sha256()
    for a in (w.x, w.d, w.qbase, w.sample_params, w.offsets, field):
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def _trajectory(name, out, steps, **sizes):
    from synthetic import make_workload
    from tests.oracle_pool import PooledOracle
    w = make_workload(name, **sizes)
    f = w.field()
    t0 = time.perf_counter()
    ora = PooledOracle(w.params, f, w.x, w.d, w.qbase, w.offsets, w.sample_params)
    print(f"{name} {sizes}: seeded in {time.perf_counter() - t0:.1f} s", flush=True)
    for k in range(steps):
        ora.step(1)
        if (k + 1) % 10 == 0 or k + 1 == steps:
            print(f"  step {k + 1}/{steps}: {time.perf_counter() - t0:.1f} s, deposited {int((~ora.alive).sum())}",
                  flush=True)
    np.savez_compressed(os.path.join(HERE, out), x=ora.x, v=ora.v, dep_step=ora.dep_step.astype(np.int32),
                        steps=np.int64(steps), digest=np.array(input_digest(w, f)))
    print(f"wrote {out}", flush=True)


def single65k():
    """FP64 oracle state of the 65,536-particle workload (all forces, 128^3 field) after 20 steps."""
    _trajectory("single-65k", "single65k_fp64_step20.npz", 20)


def large4096():
    """FP64 oracle state after 500 steps of 4,096 particles drawn by the 2^20-particle recipe
    (d in {1, 5, 10, 20} um, Gaussian charges, 256^3 field at Re_tau = 300)."""
    _trajectory("large-1m", "large1m_n4096_fp64_step500.npz", 500, n=4096)


P3M_65K = dict(mesh_x=128, mesh_yz=64, alpha_h=0.5, rmax_alpha=3.5)


def p3m65k():
    """P3M sums S_i (lattice sum over x images by the P3M oracle, Appendix A.2.4) of every particle of the
    65,536-particle workload at its seeded positions, with the benchmark's mesh (128 x 128 x 128 padded,
    alpha h = 0.5, r_max = 3.5 / alpha), the normaliser sum_j |a_ij| of the direct sum and each particle's
    distance to its nearest neighbour."""
    from oracle import p3m as op3m
    from oracle.sim import OracleSim
    from synthetic import make_workload
    from tests.oracle_pool import pooled_coulomb_scale, pooled_nearest
    w = make_workload("single-65k")
    f = w.field()
    t0 = time.perf_counter()
    c = P3M_65K
    mesh = op3m.Mesh(w.params["R"], w.params["L"], c["mesh_x"], c["mesh_yz"], c["alpha_h"], c["rmax_alpha"])
    q = w.sample_params[0, 0] * w.qbase
    x = np.array(w.x)
    x[:, 0] = np.mod(x[:, 0], w.params["L"])
    ghat = op3m.green_hat(mesh)
    print(f"green's function: {time.perf_counter() - t0:.1f} s", flush=True)
    long = op3m.mesh_field(mesh, x, q, ghat)
    print(f"mesh field: {time.perf_counter() - t0:.1f} s", flush=True)
    short = op3m.short_range(mesh, x, q, w.d)
    print(f"short range: {time.perf_counter() - t0:.1f} s", flush=True)
    sim = OracleSim(w.params, f, w.x, w.d, w.qbase, w.offsets, w.sample_params, evaluate=False)
    scale = pooled_coulomb_scale(sim, np.arange(w.n_particles))
    r_min = pooled_nearest(sim, np.arange(w.n_particles))
    print(f"normaliser and nearest sources: {time.perf_counter() - t0:.1f} s", flush=True)
    np.savez_compressed(os.path.join(HERE, "p3m_single65k_seed.npz"), S=long + short, scale=scale, r_min=r_min,
                        config=np.array([c["mesh_x"], c["mesh_yz"], c["alpha_h"], c["rmax_alpha"]]),
                        digest=np.array(input_digest(w, f)))
    print("wrote p3m_single65k_seed.npz", flush=True)


P3M_1M = dict(mesh_x=256, mesh_yz=128, alpha_h=0.5, rmax_alpha=3.5)
P3M_1M_TARGETS = np.arange(0, 1 << 20, 256)


def p3m1m():
    """P3M sums S_i of the 4,096 targets i = 0 mod 256 of the 2^20-particle workload at its seeded
    positions (every particle a source), with the benchmark's mesh (256 x 256 x 256 padded, alpha h =
    0.5, r_max = 3.5 / alpha), the normaliser sum_j |a_ij| of the direct sum and each target's distance
    to its nearest neighbour."""
    from oracle import p3m as op3m
    from oracle.sim import OracleSim
    from synthetic import make_workload
    from tests.oracle_pool import pooled_coulomb_scale, pooled_nearest
    w = make_workload("large-1m")
    f = w.field()
    t0 = time.perf_counter()
    c = P3M_1M
    tg = P3M_1M_TARGETS
    mesh = op3m.Mesh(w.params["R"], w.params["L"], c["mesh_x"], c["mesh_yz"], c["alpha_h"], c["rmax_alpha"])
    q = w.sample_params[0, 0] * w.qbase
    x = np.array(w.x)
    x[:, 0] = np.mod(x[:, 0], w.params["L"])
    ghat = op3m.green_hat(mesh)
    print(f"green's function: {time.perf_counter() - t0:.1f} s", flush=True)
    rho_hat = np.fft.fftn(op3m.assign(mesh, x, q))
    E = [np.real(np.fft.ifftn(rho_hat * ghat[k])) for k in range(3)]
    del ghat, rho_hat
    long = op3m.interpolate(mesh, E, x[tg])
    del E
    print(f"mesh field: {time.perf_counter() - t0:.1f} s", flush=True)
    short = op3m.short_range(mesh, x, q, w.d, tg)
    print(f"short range: {time.perf_counter() - t0:.1f} s", flush=True)
    sim = OracleSim(w.params, f, w.x, w.d, w.qbase, w.offsets, w.sample_params, evaluate=False)
    scale = pooled_coulomb_scale(sim, tg)
    r_min = pooled_nearest(sim, tg)
    print(f"normaliser and nearest sources: {time.perf_counter() - t0:.1f} s", flush=True)
    np.savez_compressed(os.path.join(HERE, "p3m_large1m_seed_targets.npz"), S=long + short, scale=scale,
                        r_min=r_min, targets=tg,
                        config=np.array([c["mesh_x"], c["mesh_yz"], c["alpha_h"], c["rmax_alpha"]]),
                        digest=np.array(input_digest(w, f)))
    print("wrote p3m_large1m_seed_targets.npz", flush=True)


JOBS = {"single65k": single65k, "large4096": large4096, "p3m65k": p3m65k, "p3m1m": p3m1m}

if __name__ == "__main__":
    for job in sys.argv[1:] or list(JOBS):
        JOBS[job]()
