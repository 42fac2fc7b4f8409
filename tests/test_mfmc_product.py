"""The product MFMC / Sobol' module against the oracle (CPU) and the GPU high-fidelity model (GPU)."""

import numpy as np
import pytest

from oracle import mfmc as omf
from paper_2205_04979_amd import mfmc as pmf


def test_allocation_matches_oracle():
    for sigma, rho in (((1.91e-5, 1.88e-5), (1.0, 0.989)), ((7.63e-4, 3.72e-4), (1.0, 0.995)),
                       ((1.96e-2, 1.01e-2), (1.0, 0.937)), ((1.0, 0.8, 0.5), (1.0, 0.95, 0.7))):
        w = (1.0, 1.0 / 2880.0) if len(sigma) == 2 else (1.0, 1e-2, 1e-4)
        a, r, m = pmf.allocate(sigma, rho, w, 9.0)
        a2, r2, m2 = omf.mfmc_allocation(sigma, rho, w, 9.0)
        assert np.allclose(a, a2, rtol=1e-14) and np.allclose(r, r2, rtol=1e-14) and np.array_equal(m, m2)
        assert pmf.precondition_holds(rho, w) == omf.mfmc_precondition(rho, w)
    assert np.isclose(pmf.gamma(0.995, 1.0, 1 / 2880), omf.variance_reduction_ratio(0.995, 1.0, 1 / 2880))


def test_estimators_match_oracle():
    rng = np.random.default_rng(0)
    f = lambda x: np.sin(3 * x[:, 0]) + x[:, 1] ** 2 + 0.3 * x[:, 0] * x[:, 1]   # noqa: E731
    x, xp = rng.uniform(size=(500, 2)), rng.uniform(size=(500, 2))
    for j in range(2):
        z = pmf.hybrid(x, xp, j)
        assert np.array_equal(z, omf.hybrid_points(x, xp, j))
        assert np.isclose(pmf.main_effect(f(x), f(z), f(xp)), omf.owen_main_effect(f(x), f(z), f(xp)), rtol=1e-13)
        assert np.isclose(pmf.total_effect(f(xp), f(z)), omf.jansen_total_effect(f(xp), f(z)), rtol=1e-13)
    y1, y2 = f(x), 0.9 * f(x) + 0.1
    alpha, _, m = pmf.allocate((y1.std(), y2.std()), (1.0, 0.99), (1.0, 0.01), 20.0)
    m = np.minimum(m, 500)
    assert np.isclose(pmf.mf_mean([y1, y2], alpha, m), omf.mfmc_mean([y1, y2], alpha, m), rtol=1e-13)


def test_pipeline_recovers_sobol_indices_of_a_test_function():
    """HF = Ishigami-like additive function, LF = a cheap correlated surrogate: the MF pipeline
    recovers the closed-form main and total indices of HF."""
    a = np.array([1.0, 2.0, 0.5])
    hf = lambda x: x @ a + 0.05 * np.sin(6 * x[:, 0])                  # noqa: E731
    lf = lambda x: 0.9 * (x @ a) + 0.2                                  # noqa: E731
    sample = lambda rng, m: rng.uniform(size=(m, 3))                    # noqa: E731
    xs = np.random.default_rng(5).uniform(size=(200000, 3))
    yh, yl = hf(xs), lf(xs)
    sigma, rho = (yh.std(), yl.std()), (1.0, np.corrcoef(yh, yl)[0, 1])
    res = pmf.mfmc_sobol([hf, lf], sigma, rho, (1.0, 1e-3), 5000.0, sample, 3, np.random.default_rng(1))
    exact = a ** 2 / np.sum(a ** 2)
    assert res.counts[0] >= 2 and res.counts[1] > res.counts[0]
    assert np.allclose(res.main, exact, atol=0.05) and np.allclose(res.total, exact, atol=0.05)
    assert abs(res.mean - (np.sum(a) / 2)) < 0.05


@pytest.mark.gpu
def test_gpu_hf_batch_equals_single_sample_runs_and_oracle():
    """Form 2 semantics: samples never interact, so V_dep+ of each input point is the same whether it
    runs alone or inside a batch, and equals the FP64 oracle's.  Rebound is on, so the Hamaker ratio
    decides between sticking and bouncing and the three points give different outputs."""
    from oracle.sim import OracleSim
    from synthetic import make_workload
    from synthetic.workloads import physical_params, q_max
    from tests.gpu_common import near_wall_particles
    rng = np.random.default_rng(2)
    n = 200
    p = physical_params(180.0, rebound_osu=True, dt=2e-7)
    d = rng.choice([5e-6, 10e-6], n)
    x, er = near_wall_particles(rng, n, p, d, band=100e-6)
    v0 = 1.5 * er + rng.normal(0, 0.1, (n, 3))
    f = make_workload("plain-1k", n=4, field_n=32).field()
    hf = pmf.HighFidelityGPU(p, f, x, d, steps=60, real_bytes=8, v=v0)
    pts = np.array([[0.02, 1e-4, 300.0], [0.1, 0.3, 320.0], [0.0, 1.0, 290.0]])
    print("case: HF batch of 3 vs single runs, fp64", flush=True)
    batch = hf(pts)
    single = np.array([hf(pts[k:k + 1])[0] for k in range(3)])
    assert np.allclose(batch, single, rtol=1e-13, atol=0)
    for k in range(3):
        sp = np.array([[pts[k, 0], pts[k, 1] * 1e-18, pts[k, 2]]])
        o = OracleSim(p, f, x, d, q_max(d), np.array([0, n]), sp, v0=v0)
        o.step(60)
        assert np.isclose(batch[k], o.tally()[0]["v_dep_plus"], rtol=1e-13, atol=0), k
    assert batch[0] != batch[2]


def _oracle_model(p, f, x, d, v0, steps):
    """The same evaluator as HighFidelityGPU, one FP64 oracle run per input point."""
    from oracle.sim import OracleSim
    from synthetic.workloads import q_max
    n = x.shape[0]

    def run(pts):
        out = np.empty(pts.shape[0])
        for k in range(pts.shape[0]):
            sp = np.array([[pts[k, 0], pts[k, 1] * 1e-18, pts[k, 2]]])
            o = OracleSim(p, f, x, d, q_max(d), np.array([0, n]), sp, v0=v0)
            o.step(steps)
            out[k] = o.tally()[0]["v_dep_plus"]
        return out
    return run


@pytest.mark.gpu
def test_gpu_mfmc_pipeline_matches_oracle_pipeline():
    """MFMC mean, variance and Sobol' indices with the GPU model (FP64) as HF and a cheaper GPU model
    (fewer particles, shorter run) as LF, against the same pipeline evaluated with the oracle as both
    models on the same seeded inputs."""
    from synthetic import make_workload
    from synthetic.workloads import physical_params
    from tests.gpu_common import near_wall_particles
    rng = np.random.default_rng(3)
    n = 200
    p = physical_params(180.0, rebound_osu=True, dt=2e-7)
    f = make_workload("plain-1k", n=4, field_n=32).field()
    d = rng.choice([5e-6, 10e-6], n)
    x, er = near_wall_particles(rng, n, p, d, band=100e-6)
    v0 = 1.5 * er + rng.normal(0, 0.1, (n, 3))
    hf = pmf.HighFidelityGPU(p, f, x, d, steps=60, real_bytes=8, v=v0)
    lf = pmf.HighFidelityGPU(p, f, x[:50], d[:50], steps=30, real_bytes=8, v=v0[:50])
    sample = lambda r, m: np.stack([r.uniform(0, 0.1, m), 10 ** r.uniform(-5, 0, m),   # noqa: E731
                                    r.uniform(280, 360, m)], 1)
    pilot = sample(np.random.default_rng(4), 16)
    print("case: MFMC pipeline, pilot", flush=True)
    yh, yl = hf(pilot), lf(pilot)
    assert yh.std() > 0 and yl.std() > 0
    sigma, rho = (yh.std(ddof=1), yl.std(ddof=1)), (1.0, float(np.corrcoef(yh, yl)[0, 1]))
    args = (sigma, rho, (1.0, 0.1), 40.0, sample, 3)
    print("case: MFMC pipeline, GPU models", sigma, rho, flush=True)
    res = pmf.mfmc_sobol([hf, lf], *args, rng=np.random.default_rng(5))
    assert res.counts[1] > res.counts[0] >= 2
    print("case: MFMC pipeline, oracle models", res.counts.tolist(), flush=True)
    ref = pmf.mfmc_sobol([_oracle_model(p, f, x, d, v0, 60), _oracle_model(p, f, x[:50], d[:50], v0[:50], 30)],
                         *args, rng=np.random.default_rng(5))
    assert np.array_equal(res.counts, ref.counts)
    for a, b in ((res.mean, ref.mean), (res.variance, ref.variance)):
        assert np.isclose(a, b, rtol=1e-11, atol=0), (a, b)
    assert np.allclose(res.main, ref.main, rtol=1e-9, atol=1e-12)
    assert np.allclose(res.total, ref.total, rtol=1e-9, atol=1e-12)


def test_allocation_rejects_degenerate_statistics():
    for sigma, rho in (((1.0, 0.0), (1.0, 0.5)), ((1.0, 1.0), (1.0, float("nan"))), ((1.0, 1.0), (1.0, 1.0))):
        with pytest.raises(ValueError):
            pmf.allocate(sigma, rho, (1.0, 0.1), 10.0)
