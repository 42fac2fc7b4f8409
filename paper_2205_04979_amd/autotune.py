"""Choose the Coulomb pair-kernel shape for a simulation by measurement.

Each compiled shape (targets per lane, wavefronts per workgroup, sources per
compensated block) is timed on the live simulation over whole steps as
``depo_step`` runs them (the captured step graph, in which the cell build and
short-range forces run beside the pair kernel), after a warm-up that brings
the clocks up, and the fastest is kept.  The particle state is saved before
and restored after, so tuning does not advance the simulation.  Results can be
cached in a JSON file keyed by precision, sample count, particle count and
device name.
"""

from __future__ import annotations

import json
import os
import time
from typing import Optional

FP32_SHAPES = [(1, 4, 32), (1, 8, 32), (1, 16, 32), (2, 4, 32), (2, 8, 32), (2, 16, 32), (4, 4, 32), (4, 8, 32),
               (1, 4, 64), (1, 8, 64), (1, 16, 64), (2, 8, 64), (2, 16, 64)]
# symmetric pair kernel (mode 2): (targets per lane, waves, 64-source rounds, 2); 64 IPL W targets per item
FP32_SYM_SHAPES = [(1, 4, 64, 2), (1, 8, 64, 2), (2, 2, 64, 2), (2, 4, 64, 2), (4, 1, 64, 2), (4, 2, 64, 2),
                   (4, 4, 64, 2), (8, 1, 64, 2)]
FP64_SHAPES = [(1, 4, 16), (1, 8, 16), (2, 4, 16), (1, 16, 16)]


def _key(sim) -> str:
    import torch
    name = torch.cuda.get_device_name(sim.device)
    return f"{name}|fp{8 * sim.real_bytes}|S={sim.s}|N={sim.n}"


def _ms_per_step(sim, steps: int) -> float:
    import torch
    torch.cuda.synchronize(sim.device)
    t0 = time.perf_counter()
    sim.step(steps)
    torch.cuda.synchronize(sim.device)
    return 1e3 * (time.perf_counter() - t0) / steps


def autotune(sim, steps: int = 3, cache_path: Optional[str] = None, verbose: bool = False, refine: int = 3,
             rounds: int = 3, shapes=None, warmup_s: float = 0.05):
    """Return (best_shape, {shape: ms per step}) and apply the best shape to ``sim``.

    Every shape (``shapes``, default: every compiled shape of the precision) is timed over ``steps``
    steps; the ``refine`` fastest are then timed again in ``rounds`` round-robin passes (so that
    clock drift affects them alike) and each keeps its fastest measurement."""
    key = _key(sim)
    custom = shapes is not None   # a caller's own candidate list is neither read from nor written to the cache
    cache = {}
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as fh:
            cache = json.load(fh)
        if key in cache and not custom:
            best = tuple(cache[key]["best"])
            sim.set_kernel_config(*best)
            return best, {tuple(json.loads(k)): v for k, v in cache[key]["ms"].items()}
    if shapes is None:
        shapes = FP32_SHAPES + FP32_SYM_SHAPES if sim.real_bytes == 4 else FP64_SHAPES
    blob = sim.state_download()
    # the state advances while shapes are timed (uploading it drops the captured graph, which would
    # put a capture into every measurement) and is restored once at the end
    first = _ms_per_step(sim, 1)
    n_warm = min(200, int(warmup_s / max(first * 1e-3, 1e-6)))   # about warmup_s: clocks ramp up under load
    if n_warm > 0:
        sim.step(n_warm)

    def measure(shp):
        sim.set_kernel_config(*shp)
        sim.step(1)                             # untimed: graph capture, first launch of the shape
        return _ms_per_step(sim, steps)

    times = {}
    for shp in shapes:
        try:
            ms = measure(shp)
        except Exception as exc:      # a symmetric shape the layout's partial arrays do not cover
            if verbose:
                print(f"[autotune] shape {shp} skipped: {exc}", flush=True)
            continue
        times[shp] = ms
        if verbose:
            print(f"[autotune] shape {shp}: {ms:.4f} ms per step", flush=True)
    finalists = sorted(times, key=times.get)[:max(1, refine)]
    for _ in range(rounds if len(finalists) > 1 else 0):
        for shp in finalists:
            times[shp] = min(times[shp], measure(shp))
    sim.state_upload(blob)
    best = min(finalists, key=times.get)
    sim.set_kernel_config(*best)
    if cache_path and not custom:
        cache[key] = {"best": list(best), "ms": {json.dumps(list(k)): v for k, v in times.items()}}
        with open(cache_path, "w") as fh:
            json.dump(cache, fh, indent=1)
    return best, times
