"""Pins of the MFMC / Sobol' oracle (Section 3) against the paper's printed numbers and closed forms."""

import numpy as np
import pytest

from oracle import mfmc

# Table 2: per tau_p+, (mu, sigma, rho_1i, w_i) of DNS and the 1D Eulerian model
TABLE2 = {
    0.1: dict(sigma=(1.91e-5, 1.88e-5), rho=(1.0, 0.989)),
    1.0: dict(sigma=(7.63e-4, 3.72e-4), rho=(1.0, 0.995)),
    10.0: dict(sigma=(1.96e-2, 1.01e-2), rho=(1.0, 0.937)),
}
W = (1.0, 1.0 / 2880.0)
# Table 3: (m_1, m_2, alpha_2) for MF at p = 36 and p = 72
TABLE3 = {
    0.1: {36: (8, 2861, 1.005), 72: (16, 5488, 1.005)},
    1.0: {36: (7, 3932, 2.040), 72: (15, 7726, 2.040)},
    10.0: {36: (8, 1237, 1.816), 72: (17, 2487, 1.816)},
}
GAMMA = {0.1: 0.028, 1.0: 0.014, 10.0: 0.135}   # Section 4.1


@pytest.mark.parametrize("tau", [0.1, 1.0, 10.0])
def test_table2_to_table3_allocation(tau):
    t = TABLE2[tau]
    for p, (m1, m2, a2) in TABLE3[tau].items():
        p_eff = mfmc.effective_budget(p, 2)
        alpha, r, m = mfmc.mfmc_allocation(t["sigma"], t["rho"], W, p_eff)
        assert abs(alpha[1] - a2) / a2 < 2e-3              # printed to 3 decimals
        assert m[0] == m1                                  # exact
        assert abs(m[1] - m2) / m2 < 0.06                  # the table's m_2/m_1 varies with p; +-6 %
        assert mfmc.mfmc_precondition(t["rho"], W)


def test_mc_budget_column_of_table3():
    """MC with DNS only: m = p_eff / w_1 = 9 (p = 36) and 18 (p = 72); LF only: 25920 and 51840."""
    for p, (m_hf, m_lf) in {36: (9, 25920), 72: (18, 51840)}.items():
        pe = mfmc.effective_budget(p, 2)
        assert round(pe / W[0]) == m_hf and round(pe / W[1]) == m_lf


@pytest.mark.parametrize("tau", [0.1, 1.0, 10.0])
def test_gamma_printed(tau):
    g = mfmc.variance_reduction_ratio(TABLE2[tau]["rho"][1], W[0], W[1])
    assert abs(g - GAMMA[tau]) < 1e-3


def test_gamma_matches_variance_formula():
    """For two models, Var[MFMC] at the optimal allocation / Var[MC] at equal cost equals gamma."""
    sigma, rho, w, p = (2.0, 1.5), (1.0, 0.95), (1.0, 1e-3), 1e4
    alpha = mfmc.mfmc_coefficients(sigma, rho)
    r = mfmc.mfmc_ratios(rho, w)
    m1 = p / np.dot(w, r)
    v_mf = mfmc.mfmc_variance(sigma, rho, alpha, np.array([m1, m1 * r[1]]))
    v_mc = sigma[0] ** 2 / (p / w[0])
    assert np.isclose(v_mf / v_mc, mfmc.variance_reduction_ratio(rho[1], w[0], w[1]), rtol=1e-12)


def test_precondition_fails_for_expensive_or_uncorrelated_lf():
    assert not mfmc.mfmc_precondition((1.0, 0.3), (1.0, 0.5))
    assert mfmc.mfmc_precondition((1.0, 0.99), (1.0, 1e-3))


def test_mfmc_estimator_unbiased_with_predicted_variance():
    """Replicates of S_hat on a correlated model pair: mean equals the exact expectation and the
    empirical variance matches the closed form (chi-square bounds)."""
    rng = np.random.default_rng(0)
    f1 = lambda x: np.sin(np.pi * x) + 0.3 * x ** 2                # noqa: E731  E[f1] = 2/pi + 0.1
    f2 = lambda x: 0.8 * np.sin(np.pi * x) + 0.05                  # noqa: E731
    xs = rng.uniform(size=400000)
    y1, y2 = f1(xs), f2(xs)
    sigma = (y1.std(), y2.std())
    rho = (1.0, np.corrcoef(y1, y2)[0, 1])
    alpha = mfmc.mfmc_coefficients(sigma, rho)
    m = np.array([20, 400])
    reps = 4000
    est = np.empty(reps)
    for k in range(reps):
        x = rng.uniform(size=m[1])
        est[k] = mfmc.mfmc_mean([f1(x), f2(x)], alpha, m)
    exact = 2 / np.pi + 0.1
    var = mfmc.mfmc_variance(sigma, rho, alpha, m)
    assert abs(est.mean() - exact) < 4 * np.sqrt(var / reps)
    assert 0.9 < est.var(ddof=1) / var < 1.1


def _sobol_samples(f, d, m, rng):
    x, xp = rng.uniform(size=(m, d)), rng.uniform(size=(m, d))
    fx, fxp = f(x), f(xp)
    fz = [f(mfmc.hybrid_points(x, xp, j)) for j in range(d)]
    return fx, fxp, fz


def test_sobol_additive_linear_model():
    """Y = sum a_j X_j, X ~ U[0,1]^d: s_j = s_j^t = a_j^2 / sum a^2."""
    rng = np.random.default_rng(1)
    a = np.array([1.0, 2.0, 0.5])
    f = lambda x: x @ a                                              # noqa: E731
    fx, fxp, fz = _sobol_samples(f, 3, 200000, rng)
    var = np.sum(a ** 2) / 12.0
    for j in range(3):
        sj = mfmc.owen_main_effect(fx, fz[j], fxp) / var
        tj = mfmc.jansen_total_effect(fxp, fz[j]) / var
        exact = a[j] ** 2 / np.sum(a ** 2)
        assert abs(sj - exact) < 0.01 and abs(tj - exact) < 0.01


def test_sobol_g_function():
    """Sobol' g-function g = prod (|4x_j - 2| + a_j)/(1 + a_j): V_j = (1/3)/(1 + a_j)^2, closed-form indices."""
    rng = np.random.default_rng(2)
    a = np.array([0.0, 1.0, 9.0])
    f = lambda x: np.prod((np.abs(4 * x - 2) + a) / (1 + a), axis=1)  # noqa: E731
    vj = (1.0 / 3.0) / (1 + a) ** 2
    var = np.prod(1 + vj) - 1
    fx, fxp, fz = _sobol_samples(f, 3, 400000, rng)
    for j in range(3):
        main = vj[j] / var
        total = vj[j] * np.prod(1 + np.delete(vj, j)) / var
        assert abs(mfmc.owen_main_effect(fx, fz[j], fxp) / var - main) < 0.01
        assert abs(mfmc.jansen_total_effect(fxp, fz[j]) / var - total) < 0.01


def test_mf_sobol_reduces_to_hf_when_lf_equals_hf_on_all_samples():
    """With f2 = f1 and alpha = 1 the MFMC combination telescopes to the index on the largest sample."""
    rng = np.random.default_rng(3)
    f = lambda x: x[:, 0] + x[:, 1] ** 2                             # noqa: E731
    m = (50, 1000)
    x, xp = rng.uniform(size=(m[1], 2)), rng.uniform(size=(m[1], 2))
    fx, fxp = f(x), f(xp)
    fz = f(mfmc.hybrid_points(x, xp, 0))
    q_hf = mfmc.owen_main_effect(fx[:m[0]], fz[:m[0]], fxp[:m[0]])
    q_lf_big = mfmc.owen_main_effect(fx, fz, fxp)
    q = mfmc.mf_sobol([(q_hf, None), (q_lf_big, q_hf)], np.array([1.0, 1.0]))
    assert np.isclose(q, q_lf_big, rtol=1e-14)
