"""Multi-fidelity Monte Carlo on the GPU high-fidelity model (Section 3).

* ``allocate``: optimal control-variate coefficients alpha_i = rho_1i s_1 / s_i,
  evaluation ratios r_i = sqrt(w_1 (rho_1i^2 - rho_1,i+1^2) / (w_i (1 - rho_12^2)))
  (rho_1,k+1 = 0) and counts m_i = floor(m_1 r_i), m_1 = budget / (w . r)
  (Eqs. opt1-opt3), with the precondition of Eq. mf-precond;
* ``mf_mean`` / ``mf_variance``: control-variate combinations of per-model
  estimates on nested sample sets (Eq. MFMC_mean; Qian et al. for the variance
  and the Sobol' indices);
* ``main_effect`` / ``total_effect``: unbiased Owen estimator of V_j and the
  Jansen-type estimator of T_j on the hybrid points z^(j) (coordinate j from
  x, the rest from x');
* ``HighFidelityGPU``: evaluates V_dep+ for many input points (charge scale xi,
  Hamaker ratio zeta, temperature) as ONE batched launch of the particle step,
  one Monte Carlo sample per input point;
* ``LowFidelityGPU``: the one-dimensional Eulerian model (Appendix B) for the
  same inputs, one lane per input point;
* ``mfmc_sobol``: the full estimator pipeline (pilot statistics in, budget
  split p_eff = p / (d + 2), HF and LF runs on nested samples, MF mean,
  variance, main and total indices).
"""

from __future__ import annotations

from dataclasses import dataclass
from typing import Callable, Optional, Sequence

import numpy as np


# ------------------------------------------------------------------ allocation

def allocate(sigma: Sequence[float], rho: Sequence[float], w: Sequence[float], budget: float):
    s = np.asarray(sigma, dtype=np.float64)
    r1 = np.asarray(rho, dtype=np.float64)
    ww = np.asarray(w, dtype=np.float64)
    k = s.shape[0]
    if not (np.all(np.isfinite(s)) and np.all(s > 0) and np.all(np.isfinite(r1)) and np.all(np.abs(r1) <= 1)
            and abs(r1[1]) < 1 and np.all(ww > 0)):
        raise ValueError("allocation needs sigma > 0, |rho| <= 1 with |rho_12| < 1 and positive costs")
    alpha = np.ones(k)
    alpha[1:] = r1[1:] * s[0] / s[1:]
    nxt = np.zeros(k)
    nxt[:-1] = r1[1:]
    ratio = np.sqrt(ww[0] * (r1 * r1 - nxt * nxt) / (ww * (1.0 - r1[1] * r1[1])))
    m1 = budget / float(ww @ ratio)
    counts = np.floor(m1 * ratio).astype(np.int64)
    return alpha, ratio, counts


def precondition_holds(rho: Sequence[float], w: Sequence[float]) -> bool:
    r2 = np.concatenate([np.asarray(rho, dtype=np.float64) ** 2, [0.0]])
    ww = np.asarray(w, dtype=np.float64)
    return all(ww[i - 1] / ww[i] > (r2[i - 1] - r2[i]) / (r2[i] - r2[i + 1]) for i in range(1, ww.shape[0]))


def gamma(rho12: float, w1: float, w2: float) -> float:
    """Two-model MSE ratio MFMC / MC at equal cost."""
    return (np.sqrt(1.0 - rho12 * rho12) + rho12 * np.sqrt(w2 / w1)) ** 2


# ------------------------------------------------------------------ estimators

def mf_combine(per_model: Sequence[Sequence[float]], alpha: Sequence[float]) -> float:
    """Q = Q^(1)[m_1] + sum_i alpha_i (Q^(i)[m_i] - Q^(i)[m_{i-1}]); per_model[i] = (Q on m_i, Q on m_{i-1})."""
    q = float(per_model[0][0])
    for i in range(1, len(per_model)):
        q += float(alpha[i]) * (float(per_model[i][0]) - float(per_model[i][1]))
    return q


def mf_mean(outputs: Sequence[np.ndarray], alpha, counts) -> float:
    """MFMC mean from model outputs on the nested inputs x_1..x_{m_i} (outputs[i] has >= m_i entries)."""
    per = [(np.mean(outputs[0][: counts[0]]), None)]
    for i in range(1, len(outputs)):
        per.append((np.mean(outputs[i][: counts[i]]), np.mean(outputs[i][: counts[i - 1]])))
    return mf_combine(per, alpha)


def mf_variance(outputs: Sequence[np.ndarray], alpha, counts) -> float:
    per = [(np.var(outputs[0][: counts[0]], ddof=1), None)]
    for i in range(1, len(outputs)):
        per.append((np.var(outputs[i][: counts[i]], ddof=1), np.var(outputs[i][: counts[i - 1]], ddof=1)))
    return mf_combine(per, alpha)


def main_effect(fx: np.ndarray, fz: np.ndarray, fxp: np.ndarray) -> float:
    """Unbiased V_j = 2m/(2m-1) (mean(f(x) f(z)) - ((E+E')/2)^2 + (V+V')/(4m))."""
    m = fx.shape[0]
    e, ep = np.mean(fx), np.mean(fxp)
    v, vp = np.var(fx, ddof=1), np.var(fxp, ddof=1)
    return float(2.0 * m / (2.0 * m - 1.0) * (np.mean(fx * fz) - (0.5 * (e + ep)) ** 2 + (v + vp) / (4.0 * m)))


def total_effect(fxp: np.ndarray, fz: np.ndarray) -> float:
    """T_j = mean((f(x') - f(z))^2) / 2."""
    return float(0.5 * np.mean((fxp - fz) ** 2))


def hybrid(x: np.ndarray, xp: np.ndarray, j: int) -> np.ndarray:
    z = xp.copy()
    z[:, j] = x[:, j]
    return z


# ------------------------------------------------------------------ GPU high-fidelity model

@dataclass
class HighFidelityGPU:
    """V_dep+ of the particle step for a set of uncertain inputs, one batched GPU launch per call.

    Each input row (xi, zeta, T) becomes one Monte Carlo sample with charge scale xi on base charges
    q_max(d) (Eq. 1), Hamaker constant zeta * A0 (A0 = 1e-18 J) and temperature T; every sample
    starts from the same seeded particle set (common random numbers) and runs ``steps`` steps.
    Inputs: ``params`` (physical parameter dictionary), ``field`` (node-grid velocity), ``x``, ``d``
    (one sample's particles) and optionally ``v`` (initial velocities; default: the fluid's)."""

    params: dict
    field: np.ndarray
    x: np.ndarray
    d: np.ndarray
    steps: int
    real_bytes: int = 4
    a0: float = 1e-18
    v: Optional[np.ndarray] = None

    def __call__(self, inputs: np.ndarray) -> np.ndarray:
        from .depo import Simulation
        inputs = np.atleast_2d(np.asarray(inputs, dtype=np.float64))
        S, n = inputs.shape[0], self.x.shape[0]
        T = inputs[:, 2] if inputs.shape[1] > 2 else np.full(S, 300.0)
        sp = np.stack([inputs[:, 0], inputs[:, 1] * self.a0, T], axis=1)
        qb = 500.0 * 1.6e-19 * (self.d / 1e-6) ** 2
        offsets = np.arange(S + 1, dtype=np.int64) * n
        sim = Simulation(self.params, offsets, self.field.shape[:3], real_bytes=self.real_bytes)
        sim.init_field(self.field)
        v = None if self.v is None else np.tile(self.v, (S, 1))
        sim.seed(sp, np.tile(self.x, (S, 1)), np.tile(self.d, S), np.tile(qb, S), v=v)
        sim.step(self.steps)
        out = np.array([t["v_dep_plus"] for t in sim.tally()])
        sim.close()
        return out


@dataclass
class LowFidelityGPU:
    """V_dep+ of the one-dimensional Eulerian model (Appendix B) for one particle size, as the cheap model.

    Each input row (xi, zeta[, T]) gives the charge xi * q_max(d) (Eq. 1) and the Hamaker constant
    zeta * A0; the model is isothermal, so a temperature column is ignored.  All rows are solved by one
    launch, one lane per row."""

    params: dict
    d: float
    a0: float = 1e-18
    n_wall: int = 800
    n_core: int = 800

    def __call__(self, inputs: np.ndarray) -> np.ndarray:
        from .depo import lf_solve
        inputs = np.atleast_2d(np.asarray(inputs, dtype=np.float64))
        S = inputs.shape[0]
        d = np.full(S, float(self.d))
        q = inputs[:, 0] * 500.0 * 1.6e-19 * (d / 1e-6) ** 2
        return lf_solve(self.params, d, q, inputs[:, 1] * self.a0, self.n_wall, self.n_core)


# ------------------------------------------------------------------ pipeline

@dataclass
class MFResult:
    counts: np.ndarray
    alpha: np.ndarray
    mean: float
    variance: float
    main: np.ndarray
    total: np.ndarray


def mfmc_sobol(models: Sequence[Callable[[np.ndarray], np.ndarray]], sigma, rho, w, budget: float,
               sample_inputs: Callable[[np.random.Generator, int], np.ndarray], d: int,
               rng: Optional[np.random.Generator] = None) -> MFResult:
    """MF estimates of mean, variance and Sobol' main/total indices of model 1 (Section 3).

    ``models[i]`` maps an (m, d) array of inputs to m outputs; ``sample_inputs(rng, m)`` draws inputs.
    The budget is split as p_eff = p / (d + 2) (each Sobol' sample needs d + 2 runs)."""
    rng = np.random.default_rng() if rng is None else rng
    p_eff = budget / (d + 2.0)
    alpha, _, counts = allocate(sigma, rho, w, p_eff)
    if counts[0] < 2:
        raise ValueError("budget too small for two high-fidelity samples")
    mmax = int(counts[-1])
    x, xp = sample_inputs(rng, mmax), sample_inputs(rng, mmax)
    fx, fxp, fz = [], [], []
    for i, f in enumerate(models):
        mi = int(counts[i])
        pts = [x[:mi], xp[:mi]] + [hybrid(x[:mi], xp[:mi], j) for j in range(d)]
        y = f(np.concatenate(pts, axis=0))          # one batched evaluation per model
        fx.append(y[:mi])
        fxp.append(y[mi:2 * mi])
        fz.append([y[(2 + j) * mi:(3 + j) * mi] for j in range(d)])
    mean = mf_mean(fx, alpha, counts)
    var = mf_variance(fx, alpha, counts)
    main, tot = np.zeros(d), np.zeros(d)
    for j in range(d):
        pm = [(main_effect(fx[0], fz[0][j], fxp[0]), None)]
        pt = [(total_effect(fxp[0], fz[0][j]), None)]
        for i in range(1, len(models)):
            a, b = int(counts[i]), int(counts[i - 1])
            pm.append((main_effect(fx[i][:a], fz[i][j][:a], fxp[i][:a]),
                       main_effect(fx[i][:b], fz[i][j][:b], fxp[i][:b])))
            pt.append((total_effect(fxp[i][:a], fz[i][j][:a]), total_effect(fxp[i][:b], fz[i][j][:b])))
        main[j] = mf_combine(pm, alpha) / var
        tot[j] = mf_combine(pt, alpha) / var
    return MFResult(counts=counts, alpha=alpha, mean=mean, variance=var, main=main, total=tot)
