"""C-ABI contract tests that need no GPU: the library loads, exports every
entry point declared in include/depo.h, and validates arguments on the host."""

import ctypes as C
import os
import re

import numpy as np
import pytest

from synthetic.workloads import physical_params

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def depo():
    from paper_2205_04979_amd import depo as d
    if not os.path.exists(d.library_path()):
        from paper_2205_04979_amd.build import build
        build()
    d.lib()
    return d


def declared_entry_points():
    src = open(os.path.join(ROOT, "include", "depo.h")).read()
    return sorted(set(re.findall(r"^\s*(?:depo_status|void|const char \*)\s*(depo_[a-z0-9_]+)\(", src, re.M)))


def test_every_declared_symbol_is_exported(depo):
    names = declared_entry_points()
    assert len(names) >= 18
    h = C.CDLL(depo.library_path())
    for n in names:
        assert hasattr(h, n), n
    assert sorted(depo.EXPORTED) == names


def test_struct_layouts_match_header(depo, tmp_path):
    """sizeof/offsetof of the C structs, as gcc lays them out from include/depo.h, equal the ctypes mirror."""
    import subprocess
    checks = []
    for cname, py in (("depo_params", depo.Params), ("depo_sample_params", depo.SampleParams),
                      ("depo_tally", depo.Tally)):
        checks.append(f'printf("{cname} %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            checks.append(f'printf("{cname}.{f} %zu\\n", offsetof({cname}, {f}));')
    src = tmp_path / "layout.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "depo.h"\nint main(void){' + "".join(checks)
                   + "return 0;}\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = dict(line.split() for line in subprocess.run([str(exe)], capture_output=True, text=True,
                                                      check=True).stdout.splitlines())
    for cname, py in (("depo_params", depo.Params), ("depo_sample_params", depo.SampleParams),
                      ("depo_tally", depo.Tally)):
        assert int(got[cname]) == C.sizeof(py), cname
        for f, _ in py._fields_:
            assert int(got[f"{cname}.{f}"]) == getattr(py, f).offset, (cname, f)


def test_status_strings(depo):
    L = depo.lib()
    for code, name in [(0, b"DEPO_OK"), (-1, b"DEPO_E_INVALID"), (-4, b"DEPO_E_NONFINITE"), (-6, b"DEPO_E_CORRUPT")]:
        assert L.depo_status_string(code) == name
    assert L.depo_status_string(99) == b"DEPO_E_UNKNOWN"


@pytest.mark.parametrize("key,value", [("R", 0.0), ("L", -1.0), ("nu", float("nan")), ("dt", 0.0),
                                       ("e_pp", 1.5), ("tau_col_steps", 0), ("eps0", float("inf")),
                                       ("u_bulk", -1.0), ("u_bulk", float("nan"))])
def test_create_rejects_bad_params(depo, key, value):
    p = physical_params()
    p[key] = value
    with pytest.raises(depo.DepoError) as ei:
        depo.Context(p)
    assert ei.value.status == depo.E_INVALID


def test_create_rejects_bad_precision_and_flags(depo):
    L = depo.lib()
    cp = depo.make_params(physical_params(), 4)
    h = C.c_void_p()
    cp.real_bytes = 2
    assert L.depo_create(C.byref(cp), C.byref(h)) == depo.E_INVALID and not h
    cp.real_bytes = 8
    cp.flags |= 1 << 20
    assert L.depo_create(C.byref(cp), C.byref(h)) == depo.E_INVALID
    cp.flags &= (1 << 10) - 1
    cp.reserved = 1
    assert L.depo_create(C.byref(cp), C.byref(h)) == depo.E_INVALID
    assert L.depo_create(None, C.byref(h)) == depo.E_INVALID


def test_layout_validation_and_workspace_size(depo):
    ctx = depo.Context(physical_params(), 4)
    with pytest.raises(depo.DepoError):
        ctx.set_layout([0, 10, 5], 16, 16, 16)           # decreasing offsets
    with pytest.raises(depo.DepoError):
        ctx.set_layout([1, 10], 16, 16, 16)               # offsets[0] != 0
    with pytest.raises(depo.DepoError):
        ctx.set_layout([0, 10], 3, 16, 16)                # grid too small
    with pytest.raises(depo.DepoError):
        ctx.set_layout([0, 1 << 27], 16, 16, 16)          # too many particles
    ctx.set_layout([0, 1000], 16, 16, 16)
    small = ctx.workspace_bytes()
    ctx.set_layout([0, 100000], 16, 16, 16)
    big = ctx.workspace_bytes()
    assert big > small > 16 ** 3 * 16
    # FP32 state is at least ~150 B per particle, FP64 more
    assert (big - small) / 99000 > 100
    ctx64 = depo.Context(physical_params(), 8)
    ctx64.set_layout([0, 100000], 16, 16, 16)
    assert ctx64.workspace_bytes() > big


def test_calls_out_of_order_are_state_errors(depo):
    L = depo.lib()
    ctx = depo.Context(physical_params(), 4)
    n = C.c_size_t()
    assert L.depo_workspace_bytes(ctx._h, C.byref(n)) == depo.E_STATE
    assert L.depo_step(ctx._h, 1, None) == depo.E_STATE
    assert L.depo_bind(ctx._h, C.c_void_p(256), 1 << 20) == depo.E_STATE
    ctx.set_layout([0, 100], 8, 8, 8)
    assert L.depo_bind(ctx._h, C.c_void_p(255), 1 << 30) == depo.E_INVALID     # misaligned
    assert L.depo_bind(ctx._h, C.c_void_p(256), 16) == depo.E_CAPACITY          # too small
    assert L.depo_seed(ctx._h, None, None, None, None, None, None) == depo.E_STATE
    assert L.depo_tally_read(ctx._h, None, None) == depo.E_STATE
    assert L.depo_state_upload(ctx._h, None, 0, None) == depo.E_STATE
    assert b"bind" in L.depo_last_error(ctx._h)


def test_kernel_config_validation(depo):
    ctx = depo.Context(physical_params(), 4)
    L = depo.lib()
    assert L.depo_set_kernel_config(ctx._h, 3, 8, 32, 1, 1) == depo.E_INVALID
    assert L.depo_set_kernel_config(ctx._h, 2, 8, 32, 1, 1) == depo.OK
    assert L.depo_set_kernel_config(ctx._h, 2, 8, 32, 0, 1) == depo.E_INVALID     # plain sums: one shape only
    assert L.depo_set_kernel_config(ctx._h, 1, 16, 32, 0, 1) == depo.OK
    assert L.depo_set_kernel_config(ctx._h, 1, 16, 64, 1, 0) == depo.OK
    # symmetric mode (2): FP32 only, items of at least 512 targets, compiled shapes only
    assert L.depo_set_kernel_config(ctx._h, 1, 8, 64, 2, 1) == depo.OK
    assert L.depo_set_kernel_config(ctx._h, 4, 2, 64, 2, 1) == depo.OK
    assert L.depo_set_kernel_config(ctx._h, 1, 2, 64, 2, 1) == depo.E_INVALID      # 128-target items
    assert L.depo_set_kernel_config(ctx._h, 1, 8, 32, 2, 1) == depo.E_INVALID      # rounds are 64 sources
    assert L.depo_set_kernel_config(ctx._h, 1, 8, 64, 3, 1) == depo.E_INVALID      # P3M not configured
    assert L.depo_set_kernel_config(ctx._h, 1, 8, 64, -1, 1) == depo.E_INVALID
    # symmetric mode with integer source records (4): the same shapes, FP32 only
    assert L.depo_set_kernel_config(ctx._h, 4, 2, 64, 4, 1) == depo.OK
    assert L.depo_set_kernel_config(ctx._h, 1, 8, 32, 4, 1) == depo.E_INVALID
    assert L.depo_set_kernel_config(ctx._h, 1, 8, 64, 5, 1) == depo.E_INVALID      # unknown mode
    ctx64 = depo.Context(physical_params(), 8)
    assert L.depo_set_kernel_config(ctx64._h, 2, 8, 32, 0, 1) == depo.E_INVALID
    assert L.depo_set_kernel_config(ctx64._h, 1, 4, 16, 0, 0) == depo.OK
    assert L.depo_set_kernel_config(ctx64._h, 1, 8, 64, 2, 1) == depo.E_INVALID
    assert L.depo_set_kernel_config(ctx64._h, 4, 2, 64, 4, 1) == depo.E_INVALID


def test_adjoint_host_validation(depo):
    L = depo.lib()
    soft = physical_params(soft_tally=True)
    ctx = depo.Context(soft, 4)
    n = C.c_size_t()
    assert L.depo_adjoint_workspace_bytes(ctx._h, 100, 10, C.byref(n)) == depo.E_STATE   # no layout yet
    ctx.set_layout([0, 1000, 3000], 16, 16, 16)
    assert L.depo_adjoint_workspace_bytes(ctx._h, 100, 101, C.byref(n)) == depo.E_INVALID
    assert L.depo_adjoint_workspace_bytes(ctx._h, 0, 1, C.byref(n)) == depo.E_INVALID
    sizes = []
    for ce in (100, 10, 1):
        assert L.depo_adjoint_workspace_bytes(ctx._h, 100, ce, C.byref(n)) == depo.OK
        sizes.append(n.value)
    # 1 checkpoint + 100 tape entries, 10 + 10, 100 + 1: per-entry cost is ~60 B per particle in FP32
    assert sizes[1] < sizes[0] and sizes[1] < sizes[2]
    w = (C.c_double * 2)(1.0, 1.0)
    g = (C.c_double * 6)()
    assert L.depo_adjoint(ctx._h, 10, 5, w, g, C.c_void_p(256), 1 << 30, None) == depo.E_STATE  # not seeded
    # the two halves: the forward needs a seeded state, the backward a pending forward run
    assert L.depo_adjoint_forward(ctx._h, 10, 5, C.c_void_p(256), 1 << 30, None) == depo.E_STATE
    assert L.depo_adjoint_backward(ctx._h, w, g, None) == depo.E_STATE
    assert b"pending" in L.depo_last_error(ctx._h)


def test_deposition_function_is_one_class(depo):
    """The autograd Function is built once and the same class is returned on every lookup."""
    pytest.importorskip("torch")
    assert depo.DepositionFn is depo.DepositionFn


def test_adjoint_workspace_holds_the_coulomb_tape(depo):
    """With Coulomb on, the adjoint workspace also holds the raw pair sums (3 FP32 values per particle)
    of the n_steps - ceil(n_steps / ckpt_every) steps the reverse sweep recomputes, so that it never
    reruns the pair kernel; with Coulomb off it holds none."""
    L = depo.lib()
    N = 3000
    on = depo.Context(physical_params(soft_tally=True), 4)
    off = depo.Context(physical_params(soft_tally=True, coulomb=False), 4)
    for c in (on, off):
        c.set_layout([0, 1000, N], 16, 16, 16)
    n = C.c_size_t()
    for steps, ce in ((100, 10), (100, 1), (37, 5), (1, 1)):
        K = -(-steps // ce)
        assert L.depo_adjoint_workspace_bytes(on._h, steps, ce, C.byref(n)) == depo.OK
        a = n.value
        assert L.depo_adjoint_workspace_bytes(off._h, steps, ce, C.byref(n)) == depo.OK
        b = n.value
        tape = (steps - K) * 3 * N * 4
        assert a - b == -(-tape // 256) * 256, (steps, ce)


def test_lf_solve_host_validation(depo):
    """The low-fidelity entry point checks its parameters and sizes before touching the device."""
    L = depo.lib()
    cp = depo.make_params(physical_params())
    nul = C.c_void_p(0)
    fake = C.c_void_p(256)
    assert L.depo_lf_solve(C.byref(cp), 0, nul, nul, nul, 800, 800, nul, None) == depo.OK      # empty batch
    assert L.depo_lf_solve(C.byref(cp), 4, nul, fake, fake, 800, 800, fake, None) == depo.E_INVALID
    assert L.depo_lf_solve(C.byref(cp), -1, fake, fake, fake, 800, 800, fake, None) == depo.E_INVALID
    assert L.depo_lf_solve(C.byref(cp), 4, fake, fake, fake, 1, 800, fake, None) == depo.E_INVALID
    assert L.depo_lf_solve(C.byref(cp), 4, fake, fake, fake, 800, 0, fake, None) == depo.E_INVALID
    assert L.depo_lf_solve(None, 4, fake, fake, fake, 800, 800, fake, None) == depo.E_INVALID
    for key, value in (("nu", 0.0), ("re_tau", float("nan")), ("eps0", -1.0)):
        bad = depo.make_params(dict(physical_params(), **{key: value}))
        assert L.depo_lf_solve(C.byref(bad), 4, fake, fake, fake, 800, 800, fake, None) == depo.E_INVALID


def test_p3m_configuration_validation(depo):
    """P3M is configured before the layout, with power-of-two meshes and bounded splitting; it needs a
    single-sample layout whose length holds three cutoff cells."""
    L = depo.lib()
    ctx = depo.Context(physical_params(), 4)
    assert L.depo_set_kernel_config(ctx._h, 1, 8, 64, 3, 1) == depo.E_INVALID           # not configured
    for args in ((48, 32, 0.5, 3.5), (64, 8, 0.5, 3.5), (64, 32, 0.0, 3.5), (64, 32, 0.5, 1.0), (2048, 32, 0.5, 3.5)):
        assert L.depo_set_p3m(ctx._h, *args) == depo.E_INVALID, args
    assert L.depo_set_p3m(ctx._h, 64, 32, 0.5, 3.5) == depo.OK
    with pytest.raises(depo.DepoError):
        ctx.set_layout([0, 100, 200], 16, 16, 16)                                           # two samples
    ctx.set_layout([0, 1000], 16, 16, 16)
    assert L.depo_set_p3m(ctx._h, 64, 32, 0.5, 3.5) == depo.E_STATE                      # after the layout
    assert L.depo_set_kernel_config(ctx._h, 1, 8, 64, 3, 1) == depo.OK
    small = depo.Context(physical_params(), 4)
    small.set_layout([0, 1000], 16, 16, 16)
    assert ctx.workspace_bytes() > small.workspace_bytes() + 64 * 64 * 64 * 8 * 5         # five FP32 complex meshes
    ctx64, small64 = depo.Context(physical_params(), 8), depo.Context(physical_params(), 8)
    assert L.depo_set_p3m(ctx64._h, 64, 32, 0.5, 3.5) == depo.OK
    ctx64.set_layout([0, 1000], 16, 16, 16)
    small64.set_layout([0, 1000], 16, 16, 16)
    mesh64 = ctx64.workspace_bytes() - small64.workspace_bytes()
    assert mesh64 > 64 * 64 * 64 * 16 * 5                                                   # five FP64 complex meshes
    assert ctx.workspace_bytes() - small.workspace_bytes() < mesh64 - 64 * 64 * 64 * 8 * 5 + 1
    coarse = depo.Context(physical_params(), 4)
    assert L.depo_set_p3m(coarse._h, 16, 16, 0.3, 6.0) == depo.OK                        # r_max > L / 3
    with pytest.raises(depo.DepoError):
        coarse.set_layout([0, 1000], 16, 16, 16)


def test_reorder_interval_validation(depo):
    """depo_set_reorder takes 0 (never) to 2^20 steps; anything else, and a null context, is rejected
    (with a message where there is a context)."""
    ctx = depo.Context(physical_params(), 4)
    L = depo.lib()
    assert L.depo_set_reorder(ctx._h, 16) == depo.OK
    assert L.depo_set_reorder(ctx._h, 0) == depo.OK
    assert L.depo_set_reorder(ctx._h, 1 << 20) == depo.OK
    for bad in (-1, (1 << 20) + 1):
        assert L.depo_set_reorder(ctx._h, bad) == depo.E_INVALID
        assert b"reorder" in L.depo_last_error(ctx._h)
    assert L.depo_set_reorder(None, 4) == depo.E_INVALID
