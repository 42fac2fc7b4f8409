"""ctypes binding of ``libdepo.so`` (declared in ``include/depo.h``).

Argument marshalling only: every step of the particle path runs in the HIP
kernels of the library.  PyTorch supplies the device workspace and the stream.
A missing library raises :class:`DepoError`; there is no fallback.
"""

from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libdepo.so")
_lib = None

OK, E_INVALID, E_STATE, E_HIP, E_NONFINITE, E_CAPACITY, E_CORRUPT = 0, -1, -2, -3, -4, -5, -6

FLAG_BITS = {
    "drag": 1 << 0, "coulomb": 1 << 1, "collide": 1 << 2, "vdw": 1 << 3, "vdw_gu": 1 << 4,
    "wall_image": 1 << 5, "wall_vdw": 1 << 6, "rebound_osu": 1 << 7, "soft_tally": 1 << 8,
    "body_force": 1 << 9,
}

PHASES = ("prepare", "cells", "coulomb", "short_range", "finish")


PAIR_PLAIN, PAIR_KAHAN, PAIR_SYMMETRIC, PAIR_P3M, PAIR_SYMMETRIC_INT = 0, 1, 2, 3, 4


class DepoError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{msg} (status {status})")
        self.status = status


class Params(C.Structure):
    _fields_ = [
        ("R", C.c_double), ("L", C.c_double), ("nu", C.c_double), ("rho_f", C.c_double),
        ("rho_p", C.c_double), ("dt", C.c_double), ("re_tau", C.c_double), ("e_pp", C.c_double),
        ("tau_col_steps", C.c_int32), ("real_bytes", C.c_int32),
        ("delta_min", C.c_double), ("kr_over_k", C.c_double), ("eps0", C.c_double),
        ("g_body", C.c_double * 3),
        ("E_young", C.c_double), ("delta_c", C.c_double), ("acont_coef", C.c_double),
        ("soft_eps", C.c_double), ("soft_tau", C.c_double),
        ("flags", C.c_uint32), ("reserved", C.c_uint32), ("u_bulk", C.c_double),
    ]


class SampleParams(C.Structure):
    _fields_ = [("charge_scale", C.c_double), ("hamaker", C.c_double), ("temperature", C.c_double)]


class Tally(C.Structure):
    _fields_ = [
        ("m_dep", C.c_double), ("n_dep", C.c_int64), ("m_alive_dt", C.c_double), ("t", C.c_double),
        ("v_dep", C.c_double), ("v_dep_plus", C.c_double), ("v_dep_se", C.c_double),
        ("j_soft", C.c_double), ("n_alive", C.c_int64), ("ce", C.c_double),
    ]


_P = C.c_void_p
_DP = C.POINTER(C.c_double)
_IP = C.POINTER(C.c_int32)

_SIGS = {
    "depo_status_string": (C.c_char_p, [C.c_int]),
    "depo_create": (C.c_int, [C.POINTER(Params), C.POINTER(_P)]),
    "depo_destroy": (None, [_P]),
    "depo_last_error": (C.c_char_p, [_P]),
    "depo_set_layout": (C.c_int, [_P, C.c_int32, C.POINTER(C.c_int64), C.c_int32, C.c_int32, C.c_int32]),
    "depo_workspace_bytes": (C.c_int, [_P, C.POINTER(C.c_size_t)]),
    "depo_bind": (C.c_int, [_P, _P, C.c_size_t]),
    "depo_init_field": (C.c_int, [_P, _DP, _P]),
    "depo_seed": (C.c_int, [_P, C.POINTER(SampleParams), _DP, _DP, _DP, _DP, _P]),
    "depo_set_sample_params": (C.c_int, [_P, C.POINTER(SampleParams), _P]),
    "depo_step": (C.c_int, [_P, C.c_int32, _P]),
    "depo_step_timed": (C.c_int, [_P, C.c_int32, _P, _DP]),
    "depo_set_kernel_config": (C.c_int, [_P, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32]),
    "depo_eval_accel": (C.c_int, [_P, _P]),
    "depo_read_particles": (C.c_int, [_P, _DP, _DP, _DP, _IP, _IP, _P]),
    "depo_tally_read": (C.c_int, [_P, C.POINTER(Tally), _P]),
    "depo_state_bytes": (C.c_int, [_P, C.POINTER(C.c_size_t)]),
    "depo_state_download": (C.c_int, [_P, _P, C.c_size_t, _P]),
    "depo_state_upload": (C.c_int, [_P, _P, C.c_size_t, _P]),
    "depo_adjoint_workspace_bytes": (C.c_int, [_P, C.c_int32, C.c_int32, C.POINTER(C.c_size_t)]),
    "depo_adjoint": (C.c_int, [_P, C.c_int32, C.c_int32, _DP, _DP, _P, C.c_size_t, _P]),
    "depo_adjoint_forward": (C.c_int, [_P, C.c_int32, C.c_int32, _P, C.c_size_t, _P]),
    "depo_adjoint_backward": (C.c_int, [_P, _DP, _DP, _P]),
    "depo_adjoint_noalloc": (C.c_int, [_P, C.c_int32, C.c_int32, _DP, _DP, _P]),
    "depo_set_p3m": (C.c_int, [_P, C.c_int32, C.c_int32, C.c_double, C.c_double]),
    "depo_set_reorder": (C.c_int, [_P, C.c_int32]),
    "depo_lf_solve": (C.c_int, [C.POINTER(Params), C.c_int64, _P, _P, _P, C.c_int32, C.c_int32, _P, _P]),
}

EXPORTED = tuple(_SIGS)


def lib():
    """Open ``libdepo.so`` (built in-tree by ``paper_2205_04979_amd.build``)."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise DepoError(E_STATE, f"{_LIB_PATH} is missing; run paper_2205_04979_amd.build.build() first")
        h = C.CDLL(_LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(h, name)
            f.restype = res
            f.argtypes = args
        _lib = h
    return _lib


def library_path() -> str:
    return _LIB_PATH


def make_params(p: dict, real_bytes: int = 4) -> Params:
    """Convert a parameter dictionary (keys as in ``synthetic.workloads.physical_params``) to the C struct."""
    out = Params()
    for k in ("R", "L", "nu", "rho_f", "rho_p", "dt", "re_tau", "e_pp", "delta_min", "kr_over_k", "eps0",
              "E_young", "delta_c", "acont_coef", "soft_eps", "soft_tau"):
        setattr(out, k, float(p[k]))
    out.tau_col_steps = int(p["tau_col_steps"])
    out.real_bytes = int(real_bytes)
    for i in range(3):
        out.g_body[i] = float(p["g_body"][i])
    flags = 0
    for name, bit in FLAG_BITS.items():
        if p.get(name, False):
            flags |= bit
    out.flags = flags
    out.reserved = 0
    out.u_bulk = float(p.get("u_bulk") or 0.0)
    return out


def _dptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(_DP)


def _f64(a, shape=None):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if shape is not None:
        a = a.reshape(shape)
    return a


def _stream_handle(stream) -> Optional[int]:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream or None
    if isinstance(stream, int):
        return stream or None
    return stream.cuda_stream or None


class Context:
    """Owns one ``depo_ctx`` (host side only; usable without a GPU up to binding)."""

    def __init__(self, params: dict, real_bytes: int = 4):
        self._L = lib()
        self._h = _P()
        self._cp = make_params(params, real_bytes)
        st = self._L.depo_create(C.byref(self._cp), C.byref(self._h))
        if st != OK:
            raise DepoError(st, "depo_create rejected the parameters")

    def check(self, st: int, what: str):
        if st != OK:
            msg = self._L.depo_last_error(self._h).decode()
            raise DepoError(st, f"{what}: {msg}")

    def set_layout(self, offsets, nx: int, ny: int, nz: int):
        off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
        self.check(self._L.depo_set_layout(self._h, int(off.shape[0] - 1), off.ctypes.data_as(C.POINTER(C.c_int64)),
                                           nx, ny, nz), "depo_set_layout")
        self.offsets = off

    def workspace_bytes(self) -> int:
        n = C.c_size_t()
        self.check(self._L.depo_workspace_bytes(self._h, C.byref(n)), "depo_workspace_bytes")
        return int(n.value)

    def state_bytes(self) -> int:
        n = C.c_size_t()
        self.check(self._L.depo_state_bytes(self._h, C.byref(n)), "depo_state_bytes")
        return int(n.value)

    def close(self):
        if self._h:
            self._L.depo_destroy(self._h)
            self._h = _P()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Simulation(Context):
    """One simulation (one or more Monte Carlo samples sharing a field) on a GPU."""

    def __init__(self, params: dict, offsets, field_shape, real_bytes: int = 4, device: str = "cuda:0",
                 p3m: Optional[dict] = None):
        """``p3m``: P3M electrostatics instead of the direct sums, dict(mesh_x, mesh_yz, alpha_h, rmax_alpha)."""
        import torch
        super().__init__(params, real_bytes)
        self.real_bytes = real_bytes
        if p3m is not None:
            self.check(self._L.depo_set_p3m(self._h, int(p3m["mesh_x"]), int(p3m["mesh_yz"]), float(p3m["alpha_h"]),
                                            float(p3m["rmax_alpha"])), "depo_set_p3m")
        self.device = torch.device(device)
        nx, ny, nz = (int(v) for v in field_shape)
        self.set_layout(offsets, nx, ny, nz)
        self.n = int(self.offsets[-1])
        self.s = int(self.offsets.shape[0] - 1)
        self.field_shape = (nx, ny, nz)
        nbytes = self.workspace_bytes()
        with torch.cuda.device(self.device):
            self._ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self._ws.data_ptr()
        aligned = (base + 255) // 256 * 256
        torch.cuda.synchronize(self.device)
        self.check(self._L.depo_bind(self._h, C.c_void_p(aligned), nbytes), "depo_bind")

    def _stream(self, stream=None):
        return C.c_void_p(_stream_handle(stream))

    def init_field(self, field: np.ndarray, stream=None):
        f = _f64(field)
        if f.shape != (*self.field_shape, 3):
            raise ValueError(f"field must have shape {(*self.field_shape, 3)}")
        self.check(self._L.depo_init_field(self._h, _dptr(f), self._stream(stream)), "depo_init_field")

    @staticmethod
    def _sp_array(sample_params):
        sp = np.asarray(sample_params, dtype=np.float64).reshape(-1, 3)
        arr = (SampleParams * sp.shape[0])()
        for k in range(sp.shape[0]):
            arr[k].charge_scale, arr[k].hamaker, arr[k].temperature = sp[k]
        return arr

    def seed(self, sample_params, x, d, qbase, v=None, stream=None):
        sp = self._sp_array(sample_params)
        if len(sp) != self.s:
            raise ValueError("need one parameter row per sample")
        x = _f64(x, (self.n, 3))
        d = _f64(d, (self.n,))
        q = _f64(qbase, (self.n,))
        vv = None if v is None else _f64(v, (self.n, 3))
        self.check(self._L.depo_seed(self._h, sp, _dptr(x), _dptr(vv), _dptr(d), _dptr(q), self._stream(stream)),
                   "depo_seed")

    def set_sample_params(self, sample_params, stream=None):
        self.check(self._L.depo_set_sample_params(self._h, self._sp_array(sample_params), self._stream(stream)),
                   "depo_set_sample_params")

    def set_kernel_config(self, targets_per_lane: int, waves: int, block: int, mode=None, use_graph: bool = True,
                          compensated: Optional[bool] = None):
        """Pair-kernel shape and mode: PAIR_PLAIN, PAIR_KAHAN, PAIR_SYMMETRIC or PAIR_SYMMETRIC_INT (FP32).  ``mode=None`` selects
        the one-sided Kahan mode in FP32 and plain in FP64 (before any call the library runs the symmetric
        mode, shape (4, 2, 64), in FP32).  ``compensated`` (bool) is accepted in place of ``mode`` for the
        one-sided modes.  The FP32 adjoint uses the symmetric pair adjoint when the mode is symmetric."""
        if mode is None:
            mode = (PAIR_KAHAN if compensated else PAIR_PLAIN) if compensated is not None else (
                PAIR_KAHAN if self.real_bytes == 4 else PAIR_PLAIN)
        self.check(self._L.depo_set_kernel_config(self._h, targets_per_lane, waves, block, int(mode),
                                                  int(use_graph)), "depo_set_kernel_config")

    def set_reorder(self, every: int):
        """Steps between storage reorders into cell order (0: never, the library default)."""
        self.check(self._L.depo_set_reorder(self._h, int(every)), "depo_set_reorder")

    def step(self, n: int = 1, stream=None):
        self.check(self._L.depo_step(self._h, int(n), self._stream(stream)), "depo_step")

    def step_timed(self, n: int, stream=None) -> dict:
        ms = np.zeros(5)
        self.check(self._L.depo_step_timed(self._h, int(n), self._stream(stream), _dptr(ms)), "depo_step_timed")
        return dict(zip(PHASES, ms.tolist()))

    def eval_accel(self, stream=None):
        self.check(self._L.depo_eval_accel(self._h, self._stream(stream)), "depo_eval_accel")

    def read(self, stream=None) -> dict:
        x = np.empty((self.n, 3)); v = np.empty((self.n, 3)); a = np.empty((self.n, 3))
        dep = np.empty(self.n, dtype=np.int32); nb = np.empty(self.n, dtype=np.int32)
        self.check(self._L.depo_read_particles(self._h, _dptr(x), _dptr(v), _dptr(a), dep.ctypes.data_as(_IP),
                                               nb.ctypes.data_as(_IP), self._stream(stream)), "depo_read_particles")
        return dict(x=x, v=v, a=a, dep_step=dep, neighbours=nb)

    def tally(self, stream=None) -> list:
        out = (Tally * self.s)()
        self.check(self._L.depo_tally_read(self._h, out, self._stream(stream)), "depo_tally_read")
        return [{k: getattr(t, k) for k, _ in Tally._fields_} for t in out]

    def state_download(self, stream=None) -> bytes:
        buf = C.create_string_buffer(self.state_bytes())
        self.check(self._L.depo_state_download(self._h, buf, len(buf), self._stream(stream)), "depo_state_download")
        return buf.raw

    def state_upload(self, blob: bytes, stream=None):
        buf = C.create_string_buffer(bytes(blob), len(blob))
        self.check(self._L.depo_state_upload(self._h, buf, len(blob), self._stream(stream)), "depo_state_upload")

    def _adjoint_workspace(self, n_steps: int, ckpt_every: int):
        import torch
        n = C.c_size_t()
        self.check(self._L.depo_adjoint_workspace_bytes(self._h, int(n_steps), int(ckpt_every), C.byref(n)),
                   "depo_adjoint_workspace_bytes")
        ws = torch.empty(n.value + 256, dtype=torch.uint8, device=self.device)
        return ws, (ws.data_ptr() + 255) // 256 * 256, n.value

    def adjoint(self, n_steps: int, ckpt_every: int, weights=None, stream=None) -> np.ndarray:
        """Run n_steps from the seeded state and return dJ/d(charge_scale, hamaker, temperature), shape (S, 3)."""
        ws, aligned, nbytes = self._adjoint_workspace(n_steps, ckpt_every)
        w = np.ones(self.s) if weights is None else _f64(weights, (self.s,))
        g = np.zeros((self.s, 3))
        self.check(self._L.depo_adjoint(self._h, int(n_steps), int(ckpt_every), _dptr(w), _dptr(g),
                                        C.c_void_p(aligned), nbytes, self._stream(stream)), "depo_adjoint")
        del ws
        return g

    def adjoint_noalloc(self, n_steps: int, ckpt_every: int, weights=None, stream=None) -> np.ndarray:
        """``adjoint`` with the library's static device workspace (no device allocation; at most 64 MiB)."""
        w = np.ones(self.s) if weights is None else _f64(weights, (self.s,))
        g = np.zeros((self.s, 3))
        self.check(self._L.depo_adjoint_noalloc(self._h, int(n_steps), int(ckpt_every), _dptr(w), _dptr(g),
                                                self._stream(stream)), "depo_adjoint_noalloc")
        return g

    def adjoint_forward(self, n_steps: int, ckpt_every: int, stream=None):
        """Forward half of the adjoint: run n_steps from the seeded state storing checkpoints.  Returns the
        device workspace, which must stay alive until ``adjoint_backward``."""
        ws, aligned, nbytes = self._adjoint_workspace(n_steps, ckpt_every)
        self.check(self._L.depo_adjoint_forward(self._h, int(n_steps), int(ckpt_every), C.c_void_p(aligned), nbytes,
                                                self._stream(stream)), "depo_adjoint_forward")
        return ws

    def adjoint_backward(self, weights, stream=None) -> np.ndarray:
        """Reverse half: dJ/d(charge_scale, hamaker, temperature) of J = sum_s w_s J_s, shape (S, 3)."""
        w = _f64(weights, (self.s,))
        g = np.zeros((self.s, 3))
        self.check(self._L.depo_adjoint_backward(self._h, _dptr(w), _dptr(g), self._stream(stream)),
                   "depo_adjoint_backward")
        return g


def lf_solve(params: dict, d, q, A, n_wall: int = 800, n_core: int = 800, device: str = "cuda:0") -> np.ndarray:
    """V_dep+ of the one-dimensional Eulerian low-fidelity model for each particle class (d[i], q[i], A[i]).

    Moves the three arrays to the device, runs ``depo_lf_solve`` on the current stream and copies the result back."""
    import torch
    d, q, A = (np.ascontiguousarray(np.broadcast_to(np.asarray(a, dtype=np.float64), np.shape(d))).ravel()
               for a in (d, q, A))
    n = d.shape[0]
    dev = [torch.from_numpy(a.copy()).to(device) for a in (d, q, A)]
    out = torch.empty(n, dtype=torch.float64, device=device)
    cp = make_params(params)
    st = lib().depo_lf_solve(C.byref(cp), n, *(C.c_void_p(t.data_ptr()) for t in dev), int(n_wall), int(n_core),
                             C.c_void_p(out.data_ptr()), C.c_void_p(_stream_handle(None)))
    if st != 0:
        raise DepoError(st, "depo_lf_solve: invalid arguments" if st == -1 else "depo_lf_solve failed")
    return out.cpu().numpy()


_DEPOSITION_FN = None


def _autograd_function():
    import torch

    class DepositionFn(torch.autograd.Function):
        """J_s = smoothed deposited mass of each sample after n_steps, differentiable in the per-sample
        charge scale, Hamaker constant and temperature (hand-written adjoint in the library).

        forward(charge_scale[S], hamaker[S], temperature[S], sim, seed, n_steps, ckpt_every) with
        ``seed = dict(x=..., d=..., qbase=..., v=None)`` reseeds ``sim`` with these parameters and runs the
        checkpointed forward only; backward runs the reverse sweep with the incoming gradient as the
        per-sample weights.  Between the two, ``sim`` must not be seeded, stepped or reconfigured."""

        @staticmethod
        def forward(ctx, charge_scale, hamaker, temperature, sim, seed, n_steps, ckpt_every):
            sp = torch.stack([charge_scale, hamaker, temperature], 1).detach().cpu().double().numpy()
            sim.seed(sp, seed["x"], seed["d"], seed["qbase"], v=seed.get("v"))
            ctx.sim = sim
            ctx.workspace = sim.adjoint_forward(n_steps, ckpt_every)
            J = torch.tensor([t["j_soft"] for t in sim.tally()], dtype=torch.float64)
            return J.to(charge_scale.device)

        @staticmethod
        def backward(ctx, gJ):
            g = torch.from_numpy(ctx.sim.adjoint_backward(gJ.detach().cpu().double().numpy()))
            ctx.workspace = None
            dev = gJ.device
            return g[:, 0].to(dev), g[:, 1].to(dev), g[:, 2].to(dev), None, None, None, None

    return DepositionFn


def __getattr__(name):
    global _DEPOSITION_FN
    if name == "DepositionFn":
        if _DEPOSITION_FN is None:
            _DEPOSITION_FN = _autograd_function()
        return _DEPOSITION_FN
    raise AttributeError(name)
