"""The allocation-free adjoint (depo_adjoint_noalloc, static device workspace) against depo_adjoint with a
caller workspace, through the C ABI: two calls in a row, the second on a smaller input (the static array
still holds the first call's contents), in the FP64 form (bitwise reproducible: equal results) and the
FP32 form (symmetric pair adjoint combined with FP64 atomics: equal to 1e-9 relative); and a request
beyond the static array's 64 MiB is refused before anything runs."""

import sys

import numpy as np
import pytest

from tests.test_gpu_adjoint import gpu_sim, sensitive_case

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("real_bytes", [8, 4])
def test_adjoint_noalloc_matches_adjoint(real_bytes):
    for n_per, n, ce, seed in ((300, 24, 5, 12), (90, 9, 4, 13)):   # the second call is smaller
        p, f, x, d, q, off, sp, v0 = sensitive_case(n_per=n_per, seed=seed)
        say(f"case: noalloc adjoint, fp{8 * real_bytes}, {off[-1]} particles, {n} steps, ckpt {ce}")
        w = np.array([1.5, -0.25])
        sim = gpu_sim(p, f, off, real_bytes)
        sim.seed(sp, x, d, q, v=v0)
        g_ref = sim.adjoint(n, ce, weights=w)
        ref_state = sim.read()
        sim.seed(sp, x, d, q, v=v0)
        g = sim.adjoint_noalloc(n, ce, weights=w)
        state = sim.read()
        say("adjoint", g_ref[:, :2].tolist(), "noalloc", g[:, :2].tolist())
        assert np.all(g_ref[:, :2] != 0.0)
        if real_bytes == 8:
            assert np.array_equal(g, g_ref)
        else:
            assert np.allclose(g, g_ref, rtol=1e-9, atol=0.0)
        for k in ("x", "v", "a"):
            assert np.array_equal(state[k], ref_state[k]), k
        assert sim.tally() == sim.tally()
        sim.close()


def test_adjoint_noalloc_refuses_more_than_its_static_workspace():
    from paper_2205_04979_amd.depo import DepoError, E_CAPACITY
    from synthetic import make_workload
    w = make_workload("adjoint-64x16k", n_samples=4, n_per=16384)
    f = w.field()
    say("case: noalloc adjoint beyond 64 MiB")
    sim = gpu_sim(w.params, f, w.offsets, 4)
    sim.seed(w.sample_params, w.x, w.d, w.qbase)
    with pytest.raises(DepoError) as ei:
        sim.adjoint_noalloc(100, 10)
    assert ei.value.status == E_CAPACITY
    t = sim.tally()
    assert all(x["t"] == 0.0 for x in t)          # nothing ran
