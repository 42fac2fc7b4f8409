"""Multi-fidelity Monte Carlo estimation and Sobol' indices (Section 3) — test infrastructure.

Plain NumPy statements of:

* the MC estimator of a mean and its mean-squared error (Eqs. 6-10);
* the MFMC control-variate estimator (Eq. MFMC_mean);
* the optimal coefficients, evaluation ratios and evaluation counts
  (Eqs. opt1-opt3) and the precondition on model costs (Eq. mf-precond);
* the two-model variance-reduction ratio gamma (Section 4.1);
* the main-effect and total-effect Sobol' indices with the unbiased Owen
  estimator of V_j and the Jansen-type estimator of T_j, and their MFMC
  combinations (Section 3.3); the effective budget p / (d + 2).

Readings: the paper writes rho_{1,k+1} = 1 in the precondition; with it the
optimal ratio r_k would be imaginary, so rho_{1,k+1} = 0 is used (this
reproduces Table 3).  Evaluation counts are rounded down (Table 3).  The
hybrid point z^(j) takes coordinate j from x and every other coordinate from
x' (as printed).

Pinned by Table 2 -> Table 3 and the printed gamma values, by closed-form
Sobol' indices of test functions, and by the closed-form variance of the
MFMC estimator (tests/test_oracle_mfmc.py).
"""

from __future__ import annotations

import numpy as np


def mc_mean(y) -> float:
    """ybar_m = (1/m) sum_j f(x_j)."""
    return float(np.mean(np.asarray(y, dtype=np.float64)))


def mfmc_coefficients(sigma, rho):
    """alpha_i = rho_{1,i} sigma_1 / sigma_i, i = 2..k (Eq. opt1); alpha_1 = 1 by convention."""
    sigma = np.asarray(sigma, dtype=np.float64)
    rho = np.asarray(rho, dtype=np.float64)
    a = rho * sigma[0] / sigma
    a[0] = 1.0
    return a


def mfmc_ratios(rho, w):
    """r_i = sqrt(w_1 (rho_{1,i}^2 - rho_{1,i+1}^2) / (w_i (1 - rho_{1,2}^2))) with rho_{1,k+1} = 0 (Eq. opt2)."""
    rho = np.asarray(rho, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    rho_next = np.append(rho[1:], 0.0)
    return np.sqrt(w[0] * (rho ** 2 - rho_next ** 2) / (w * (1.0 - rho[1] ** 2)))


def mfmc_allocation(sigma, rho, w, p):
    """Optimal (alpha, r, m) for budget p: m_1 = p / (w^T r), m_i = m_1 r_i (Eq. opt3), rounded down."""
    r = mfmc_ratios(rho, w)
    m1 = p / float(np.dot(np.asarray(w, dtype=np.float64), r))
    m = np.floor(m1 * r).astype(np.int64)
    return mfmc_coefficients(sigma, rho), r, m


def mfmc_precondition(rho, w) -> bool:
    """w_{i-1} / w_i > (rho_{1,i-1}^2 - rho_{1,i}^2) / (rho_{1,i}^2 - rho_{1,i+1}^2), i = 2..k (Eq. mf-precond)."""
    rho = np.asarray(rho, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    rr = np.append(rho, 0.0) ** 2
    for i in range(1, rho.shape[0]):
        if not w[i - 1] / w[i] > (rr[i - 1] - rr[i]) / (rr[i] - rr[i + 1]):
            return False
    return True


def mfmc_mean(y_models, alpha, m) -> float:
    """S_hat = ybar^(1)_{m_1} + sum_i alpha_i (ybar^(i)_{m_i} - ybar^(i)_{m_{i-1}}) (Eq. MFMC_mean).

    ``y_models[i]`` holds model i's outputs on the first m_i shared inputs x_1..x_{m_i}."""
    s = mc_mean(y_models[0][: m[0]])
    for i in range(1, len(y_models)):
        yi = np.asarray(y_models[i], dtype=np.float64)
        s += alpha[i] * (np.mean(yi[: m[i]]) - np.mean(yi[: m[i - 1]]))
    return float(s)


def mfmc_variance(sigma, rho, alpha, m) -> float:
    """Var[S_hat] = sigma_1^2/m_1 + sum_i (1/m_{i-1} - 1/m_i)(alpha_i^2 sigma_i^2 - 2 alpha_i rho_{1,i} sigma_1 sigma_i)."""
    v = sigma[0] ** 2 / m[0]
    for i in range(1, len(sigma)):
        v += (1.0 / m[i - 1] - 1.0 / m[i]) * (alpha[i] ** 2 * sigma[i] ** 2 - 2 * alpha[i] * rho[i] * sigma[0] * sigma[i])
    return float(v)


def variance_reduction_ratio(rho12, w1, w2) -> float:
    """gamma = MSE(MFMC) / MSE(MC) = (sqrt(1 - rho_12^2) + rho_12 sqrt(w_2 / w_1))^2 (two models, Section 4.1)."""
    return float((np.sqrt(1.0 - rho12 ** 2) + rho12 * np.sqrt(w2 / w1)) ** 2)


def effective_budget(p, d) -> float:
    """Sobol' estimation needs d + 2 model runs per sample: p_eff = p / (d + 2)."""
    return p / (d + 2.0)


def hybrid_points(x, xp, j):
    """z^(j): coordinate j from x, every other coordinate from x'."""
    z = np.array(xp, dtype=np.float64, copy=True)
    z[:, j] = np.asarray(x)[:, j]
    return z


def owen_main_effect(fx, fz, fxp) -> float:
    """V_hat_j = 2m/(2m-1) ( (1/m) sum f(x) f(z^(j)) - ((E + E')/2)^2 + (V + V')/(4m) ) (Owen, Section 3.3)."""
    fx, fz, fxp = (np.asarray(a, dtype=np.float64) for a in (fx, fz, fxp))
    m = fx.shape[0]
    E, Ep = fx.mean(), fxp.mean()
    V, Vp = fx.var(ddof=1), fxp.var(ddof=1)
    return float(2.0 * m / (2.0 * m - 1.0) * (np.mean(fx * fz) - ((E + Ep) / 2.0) ** 2 + (V + Vp) / (4.0 * m)))


def jansen_total_effect(fxp, fz) -> float:
    """T_hat_j = (1/(2m)) sum (f(x') - f(z^(j)))^2 (Section 3.3)."""
    fxp, fz = np.asarray(fxp, dtype=np.float64), np.asarray(fz, dtype=np.float64)
    return float(np.mean((fxp - fz) ** 2) / 2.0)


def mf_sobol(estimates, alpha):
    """MFMC combination of per-model index estimates: Q_mf = Q^(1)_{m_1} + sum_i alpha_i (Q^(i)_{m_i} - Q^(i)_{m_{i-1}}).

    ``estimates[i] = (Q^(i) on m_i samples, Q^(i) on m_{i-1} samples)``; for i = 0 only the first is used."""
    q = estimates[0][0]
    for i in range(1, len(estimates)):
        q += alpha[i] * (estimates[i][0] - estimates[i][1])
    return float(q)
