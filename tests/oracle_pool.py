"""Run the FP64 oracle's per-target force evaluation on a pool of host processes (test code only).

The oracle evaluates every target independently (its sum over sources belongs
to one target), so splitting the targets over forked worker processes changes
nothing in what is computed; it only spreads the O(N^2) work over the host
cores.  Used by the committed golden-file script and by the GPU tests that
check large workloads against the oracle.
"""

from __future__ import annotations

import multiprocessing as mp
import os

import numpy as np

from oracle.sim import OracleSim

_SIM = None
_CHUNK = 32


def host_processes(cap: int = 16) -> int:
    """Worker count: the cores this process may run on, at most ``cap``."""
    return max(1, min(cap, len(os.sched_getaffinity(0))))


def _accel_chunk(targets):
    return OracleSim.accelerations(_SIM, np.asarray(targets, dtype=np.int64), chunk=_CHUNK)


def _scale_chunk(targets):
    return coulomb_magnitude_sum(_SIM, np.asarray(targets, dtype=np.int64))


def _check_chunk(targets):
    t = np.asarray(targets, dtype=np.int64)
    a = OracleSim.accelerations(_SIM, t, chunk=_CHUNK)
    return np.concatenate([a, coulomb_magnitude_sum(_SIM, t)[:, None], nearest_distance(_SIM, t)[:, None]], axis=1)


def nearest_distance(sim: OracleSim, targets) -> np.ndarray:
    """Centre distance from each target to its nearest alive particle of the same sample (minimum image in x)."""
    out = np.full(len(targets), np.inf)
    for k, i in enumerate(targets):
        s = sim.sample[i]
        b, e = sim.offsets[s], sim.offsets[s + 1]
        src = np.arange(b, e)
        src = src[sim.alive[src] & (src != i)]
        if src.size:
            r = sim.x[i] - sim.x[src]
            r[:, 0] -= sim.L * np.round(r[:, 0] / sim.L)
            out[k] = np.sqrt(np.min(np.sum(r * r, axis=1)))
    return out


def coulomb_magnitude_sum(sim: OracleSim, targets) -> np.ndarray:
    """sum_j |a_ij| over the Coulomb pairs of each target (alive sources of its own sample, j != i)."""
    out = np.zeros(len(targets))
    q = sim.charge
    for k, i in enumerate(targets):
        s = sim.sample[i]
        b, e = sim.offsets[s], sim.offsets[s + 1]
        src = np.arange(b, e)
        src = src[sim.alive[src] & (src != i)]
        r = sim.x[i] - sim.x[src]
        r[:, 0] -= sim.L * np.round(r[:, 0] / sim.L)
        dist = np.sqrt(np.sum(r * r, axis=1))
        dij = 0.5 * (sim.d[i] + sim.d[src])
        out[k] = np.sum(np.abs(sim.k_e * q[i] * q[src]) / (sim.m[i] * np.maximum(dist, dij) ** 2))
    return out


def _map(fn, sim, targets, processes, pieces_per_process, chunk):
    global _SIM, _CHUNK
    targets = np.asarray(targets, dtype=np.int64)
    if targets.size == 0:
        return []
    procs = host_processes() if processes is None else processes
    parts = [p for p in np.array_split(targets, procs * pieces_per_process) if p.size]
    _SIM, _CHUNK = sim, chunk
    try:
        with mp.get_context("fork").Pool(procs) as pool:
            return pool.map(fn, parts)
    finally:
        _SIM = None


def pooled_accelerations(sim: OracleSim, targets=None, processes=None, chunk: int = 32) -> np.ndarray:
    """``sim.accelerations(targets)`` computed on a pool of forked processes."""
    n = sim.x.shape[0]
    tg = np.arange(n) if targets is None else np.asarray(targets, dtype=np.int64)
    res = _map(_accel_chunk, sim, tg, processes, 4, chunk)
    return np.concatenate(res, axis=0) if res else np.zeros((0, 3))


def pooled_coulomb_scale(sim: OracleSim, targets, processes=None) -> np.ndarray:
    """``coulomb_magnitude_sum`` on a pool of forked processes."""
    res = _map(_scale_chunk, sim, targets, processes, 4, 0)
    return np.concatenate(res) if res else np.zeros(0)


def _nearest_chunk(targets):
    return nearest_distance(_SIM, np.asarray(targets, dtype=np.int64))


def pooled_nearest(sim: OracleSim, targets, processes=None) -> np.ndarray:
    """``nearest_distance`` on a pool of forked processes."""
    res = _map(_nearest_chunk, sim, targets, processes, 4, 0)
    return np.concatenate(res) if res else np.zeros(0)


def pooled_force_check(sim: OracleSim, targets, processes=None, chunk: int = 8):
    """Per target: the oracle's acceleration (3 columns), sum_j |a_ij| of its Coulomb pairs and the distance to
    its nearest source, on a pool of forked processes."""
    res = _map(_check_chunk, sim, targets, processes, 4, chunk)
    return np.concatenate(res, axis=0) if res else np.zeros((0, 5))


class PooledOracle(OracleSim):
    """The oracle with its force evaluation spread over host processes; every other step unchanged."""

    processes = None

    def accelerations(self, targets=None, chunk: int = 32) -> np.ndarray:
        return pooled_accelerations(self, targets, self.processes, chunk)
