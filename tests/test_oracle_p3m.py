"""Pins of the P3M electrostatics oracle (Appendix A.2.4, Eq. coulomb_force) and of its exact reference,
the x-periodic lattice sum (brute force over images)."""

import math

import numpy as np
import pytest

from oracle import p3m

R, L = 0.01, 0.04


def particles(n, seed):
    rng = np.random.default_rng(seed)
    r = R * np.sqrt(rng.uniform(0, 0.95, n))
    phi = rng.uniform(0, 2 * np.pi, n)
    x = np.stack([rng.uniform(0, L, n), r * np.cos(phi), r * np.sin(phi)], 1)
    q = rng.normal(0.0, 1.0, n)
    d = np.full(n, 10e-6)
    return x, q, d


@pytest.fixture(scope="module")
def system():
    x, q, d = particles(60, 1)
    return x, q, d, p3m.lattice_sum(x, q, d, L, images=2000)


def test_lattice_sum_image_convergence_periodicity_and_third_law(system):
    x, q, d, S = system
    S1 = p3m.lattice_sum(x, q, d, L, images=1000)
    scale = np.sqrt(np.mean(S * S))
    assert np.max(np.abs(S1 - S)) < 1e-5 * scale                 # image tail ~ 1/n^2
    xs = x.copy()
    xs[:, 0] = np.mod(xs[:, 0] + 0.3 * L, L)
    assert np.allclose(p3m.lattice_sum(xs, q, d, L, images=2000), S, rtol=0, atol=1e-9 * scale)
    F = q[:, None] * S                                            # q_i E_i: pairwise equal and opposite
    assert np.all(np.abs(F.sum(0)) < 1e-9 * np.abs(F).sum(0))


def test_lattice_sum_single_image_limit():
    """With a period far longer than the particle cloud the lattice sum is the free-space direct sum."""
    x, q, d = particles(25, 2)
    big = 1e4
    S = p3m.lattice_sum(x, q, d, big, images=3)
    D = np.zeros_like(S)
    for i in range(x.shape[0]):
        r = x[i] - x
        rr = np.sqrt(np.sum(r * r, 1))
        m = np.arange(x.shape[0]) != i
        D[i] = ((q[m] / rr[m] ** 3)[:, None] * r[m]).sum(0)
    assert np.allclose(S, D, rtol=1e-9)


def test_split_reassembles_coulomb_and_tsc_moments():
    a = 700.0
    r = np.geomspace(1e-5, 0.02, 50)
    lng = np.linalg.norm(p3m.long_field(np.stack([r, 0 * r, 0 * r], 1), a), axis=1)
    assert np.allclose(lng + p3m.short_field_mag(r, a), 1.0 / r ** 2, rtol=1e-12)
    # truncation at r_max = 3.5 / alpha drops at most 2e-5 of the Coulomb field of a pair
    assert np.all(p3m.short_field_mag(np.array([3.5 / a]), a) * (3.5 / a) ** 2 < 2e-5)
    g = np.random.default_rng(0).uniform(2, 30, 1000)
    i, w = p3m.tsc_weights(g)
    assert np.allclose(w.sum(1), 1.0, rtol=0, atol=1e-15)
    assert np.allclose((w * (i[:, None] + np.array([-1, 0, 1]))).sum(1), g, rtol=0, atol=1e-12)
    assert np.all(np.abs(g - i) <= 0.5)


def _rel_rms(S, ref):
    return np.sqrt(np.mean(np.sum((S - ref) ** 2, 1)) / np.mean(np.sum(ref ** 2, 1)))


def test_p3m_converges_to_the_lattice_sum(system):
    """P3M against the exact lattice sum: the relative RMS field error is set by alpha h (mesh spacing in
    units of the splitting length) and falls as alpha h decreases (more of the field is summed directly,
    less is carried by the mesh, whose aliasing error grows with alpha h)."""
    x, q, d, S = system
    errs = []
    for ah in (0.8, 0.6, 0.4):
        mesh = p3m.Mesh(R, L, 32, 16, alpha_h=ah, rmax_alpha=3.5)
        errs.append(_rel_rms(p3m.p3m_sums(mesh, x, q, d), S))
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 2e-3


def test_short_range_rows_for_listed_targets(system):
    """The short range evaluated for listed targets gives exactly those rows of the full evaluation
    (same pairs, same order), and a particle with no source within r_max gets zero."""
    x, q, d, _ = system
    mesh = p3m.Mesh(R, L, 16, 16, 0.5, 3.5)
    full = p3m.short_range(mesh, x, q, d)
    tg = np.array([5, 0, 17, 5, x.shape[0] - 1])
    assert np.array_equal(p3m.short_range(mesh, x, q, d, tg), full[tg])
    assert 0.5 * L > mesh.rmax
    lone = p3m.short_range(mesh, np.array([[0.0, 0.0, 0.0], [0.5 * L, 0.0, 0.0]]), np.ones(2), np.full(2, 1e-5))
    assert np.all(lone == 0.0)
