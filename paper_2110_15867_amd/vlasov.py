"""Thin ctypes binding of libvlasov (the HIP library built from ``csrc/``).

Each ``vlasov_*`` function has the name, argument order and meaning of the C
entry point declared in ``include/vlasov.h``; this layer only marshals torch
tensors (device memory) and the current HIP stream into pointers and turns a
non-zero return code into ``VlasovError``.  All arithmetic runs in the HIP
kernels.  The library must have been built (``python -m
paper_2110_15867_amd.build``); importing this module without it raises.

A few helpers (``new_state``, ``step``, ``moments``, ``advect``) allocate the
output tensors with torch and call the entry points.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
# VLASOV_LIB selects another build of the same sources (the sanitizer build of
# the host code, for the CPU test run)
LIB_PATH = os.environ.get("VLASOV_LIB", os.path.join(_HERE, "libvlasov.so"))

F32, F16, BF16 = 0, 1, 2
VBC_OUTFLOW, VBC_PERIODIC = 0, 1
TORCH_DTYPE = {F32: torch.float32, F16: torch.float16, BF16: torch.bfloat16}
PREC_NAME = {F32: "f32", F16: "f16", BF16: "bf16"}


class VlasovError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: {_lib.vlasov_strerror(code).decode()} (code {code})")
        self.code = code


class vlasov_grid(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32 * 3), ("nu", ctypes.c_int32 * 3),
                ("L", ctypes.c_double * 3), ("umax", ctypes.c_double * 3)]


class vlasov_cosmology(ctypes.Structure):
    _fields_ = [("omega_m", ctypes.c_double), ("H0", ctypes.c_double)]


def make_grid(n, nu, L=(1.0, 1.0, 1.0), umax=(1.0, 1.0, 1.0)) -> vlasov_grid:
    g = vlasov_grid()
    for a in range(3):
        g.n[a], g.nu[a] = int(n[a]), int(nu[a])
        g.L[a], g.umax[a] = float(L[a]), float(umax[a])
    return g


def grid_shape(g: vlasov_grid):
    return tuple(g.n) + tuple(g.nu)


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it with `python -m paper_2110_15867_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    P, D, I, S = ctypes.c_void_p, ctypes.c_double, ctypes.c_int, ctypes.c_size_t
    G = ctypes.POINTER(vlasov_grid)
    L.vlasov_abi_version.restype = I
    L.vlasov_abi_version.argtypes = []
    L.vlasov_strerror.restype = ctypes.c_char_p
    L.vlasov_strerror.argtypes = [I]
    L.vlasov_f_bytes.restype = S
    L.vlasov_f_bytes.argtypes = [G, I]
    L.vlasov_scale_bytes.restype = S
    L.vlasov_scale_bytes.argtypes = [G, I]
    for ax in "xyz":
        fn = getattr(L, f"vlasov_advect_{ax}")
        fn.restype = I
        fn.argtypes = [G, I, P, P, P, P, D, P]
        fn = getattr(L, f"vlasov_advect_u{ax}")
        fn.restype = I
        fn.argtypes = [G, I, I, P, P, P, P, P, D, P, P]
    L.vlasov_kick.restype = I
    L.vlasov_kick.argtypes = [G, I, I, P, P, P, P, P, D, P, S, P, P]
    L.vlasov_step_workspace_bytes.restype = S
    L.vlasov_step_workspace_bytes.argtypes = [G, I]
    L.vlasov_step.restype = I
    L.vlasov_step.argtypes = [G, I, I, P, P, P, P, P, P, D, D, P, S, P, P]
    L.vlasov_step_sc_workspace_bytes.restype = S
    L.vlasov_step_sc_workspace_bytes.argtypes = [G, I]
    L.vlasov_step_sc.restype = I
    L.vlasov_step_sc.argtypes = [G, I, I, P, P, P, P, P, P, P, D, D, D, P, S, P, P]
    L.vlasov_field_workspace_bytes.restype = S
    L.vlasov_field_workspace_bytes.argtypes = [G]
    L.vlasov_field.restype = I
    L.vlasov_field.argtypes = [G, P, D, P, P, S, P]
    L.vlasov_steps_workspace_bytes.restype = S
    L.vlasov_steps_workspace_bytes.argtypes = [G, I]
    L.vlasov_steps.restype = I
    L.vlasov_steps.argtypes = [G, I, I, P, P, P, P, P, I, D, P, P, S, P, P]
    L.vlasov_step_moments.restype = I
    L.vlasov_step_moments.argtypes = [G, I, I, P, P, P, P, P, P, D, D, P, S, P, P, P, P]
    L.vlasov_moments.restype = I
    L.vlasov_moments.argtypes = [G, I, P, P, P, P, P, P]
    C = ctypes.POINTER(vlasov_cosmology)
    DP = ctypes.POINTER(ctypes.c_double)
    L.vlasov_cosmo_a.restype = I
    L.vlasov_cosmo_a.argtypes = [C, D, DP]
    L.vlasov_cosmo_t.restype = I
    L.vlasov_cosmo_t.argtypes = [C, D, DP]
    L.vlasov_cosmo_steps.restype = I
    L.vlasov_cosmo_steps.argtypes = [C, D, D, I, DP, DP]
    L.vlasov_dispersion.restype = I
    L.vlasov_dispersion.argtypes = [G, I, P, P, P, P, P, P]
    L.vlasov_sum_f64.restype = I
    L.vlasov_sum_f64.argtypes = [P, ctypes.c_int64, P, P]
    L.vlasov_stream_copy.restype = I
    L.vlasov_stream_copy.argtypes = [P, P, S, P]
    L.vlasov_valu_probe.restype = I
    L.vlasov_valu_probe.argtypes = [P, ctypes.c_int64, ctypes.c_int, ctypes.POINTER(ctypes.c_double), P]
    L.vlasov_field_noalloc_max_bytes.restype = S
    L.vlasov_field_noalloc_max_bytes.argtypes = []
    L.vlasov_field_noalloc.restype = I
    L.vlasov_field_noalloc.argtypes = [G, P, D, P, P]
    L.vlasov_encode.restype = I
    L.vlasov_encode.argtypes = [G, I, P, P, P, P]
    L.vlasov_decode.restype = I
    L.vlasov_decode.argtypes = [G, I, P, P, P, P]
    _bind_adjoint(L)
    return L


def _bind_adjoint(L):
    P, D, I, S = ctypes.c_void_p, ctypes.c_double, ctypes.c_int, ctypes.c_size_t
    G = ctypes.POINTER(vlasov_grid)
    for ax in "xyz":
        for kind in ("tan", "adj"):
            fn = getattr(L, f"vlasov_advect_{ax}_{kind}")
            fn.restype = I
            fn.argtypes = [G, P, P, P, D, P]
        fn = getattr(L, f"vlasov_advect_u{ax}_tan")
        fn.restype = I
        fn.argtypes = [G, I, P, P, P, D, P, P, P]
        fn = getattr(L, f"vlasov_advect_u{ax}_adj")
        fn.restype = I
        fn.argtypes = [G, I, P, P, D, P, P, P, P]
    L.vlasov_step_adj_workspace_bytes.restype = S
    L.vlasov_step_adj_workspace_bytes.argtypes = [G]
    L.vlasov_step_adj.restype = I
    L.vlasov_step_adj.argtypes = [G, I, P, P, P, D, D, P, P, P, P, P, S, P]
    L.vlasov_moments_adj.restype = I
    L.vlasov_moments_adj.argtypes = [G, P, P, P, P, P, P]


_lib = _load()


def lib():
    return _lib


def _ptr(t):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError("expected a torch tensor")
    if not t.is_cuda:
        raise ValueError("libvlasov takes device tensors")
    if not t.is_contiguous():
        raise ValueError("libvlasov takes contiguous tensors")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _check(rc, what):
    if rc != 0:
        raise VlasovError(rc, what)


# --- C entry points, same names -------------------------------------------------------

def vlasov_abi_version() -> int:
    return _lib.vlasov_abi_version()


def vlasov_strerror(code: int) -> str:
    return _lib.vlasov_strerror(code).decode()


def vlasov_f_bytes(grid, prec) -> int:
    return _lib.vlasov_f_bytes(ctypes.byref(grid), prec)


def vlasov_scale_bytes(grid, prec) -> int:
    return _lib.vlasov_scale_bytes(ctypes.byref(grid), prec)


def _advect_pos(axis):
    name = f"vlasov_advect_{axis}"

    def fn(grid, prec, f_in, scale_in, f_out, scale_out, dt_over_a2, stream=None):
        _check(getattr(_lib, name)(ctypes.byref(grid), prec, _ptr(f_in), _ptr(scale_in),
                                   _ptr(f_out), _ptr(scale_out), float(dt_over_a2),
                                   _stream(stream)), name)
    fn.__name__ = name
    return fn


def _advect_vel(axis):
    name = f"vlasov_advect_u{axis}"

    def fn(grid, prec, vbc, f_in, scale_in, f_out, scale_out, g, dt, outflow=None, stream=None):
        _check(getattr(_lib, name)(ctypes.byref(grid), prec, vbc, _ptr(f_in), _ptr(scale_in),
                                   _ptr(f_out), _ptr(scale_out), _ptr(g), float(dt),
                                   _ptr(outflow), _stream(stream)), name)
    fn.__name__ = name
    return fn


vlasov_advect_x = _advect_pos("x")
vlasov_advect_y = _advect_pos("y")
vlasov_advect_z = _advect_pos("z")
vlasov_advect_ux = _advect_vel("x")
vlasov_advect_uy = _advect_vel("y")
vlasov_advect_uz = _advect_vel("z")


def vlasov_kick(grid, prec, vbc, f_in, scale_in, f_out, scale_out, g, dt, work=None,
                work_bytes=0, outflow=None, stream=None):
    _check(_lib.vlasov_kick(ctypes.byref(grid), prec, vbc, _ptr(f_in), _ptr(scale_in),
                            _ptr(f_out), _ptr(scale_out), _ptr(g), float(dt), _ptr(work),
                            int(work_bytes), _ptr(outflow), _stream(stream)), "vlasov_kick")


def vlasov_step_workspace_bytes(grid, prec) -> int:
    return _lib.vlasov_step_workspace_bytes(ctypes.byref(grid), prec)


def vlasov_step(grid, prec, vbc, f_in, scale_in, f_out, scale_out, g_n, g_np1, dt, a2inv,
                work, work_bytes, outflow=None, stream=None):
    _check(_lib.vlasov_step(ctypes.byref(grid), prec, vbc, _ptr(f_in), _ptr(scale_in),
                            _ptr(f_out), _ptr(scale_out), _ptr(g_n), _ptr(g_np1), float(dt),
                            float(a2inv), _ptr(work), int(work_bytes), _ptr(outflow),
                            _stream(stream)), "vlasov_step")


def vlasov_step_sc_workspace_bytes(grid, prec) -> int:
    return _lib.vlasov_step_sc_workspace_bytes(ctypes.byref(grid), prec)


def vlasov_step_sc(grid, prec, vbc, f_in, scale_in, f_out, scale_out, g_n, g_np1, rho_np1,
                   coupling, dt, a2inv, work, work_bytes, outflow=None, stream=None):
    _check(_lib.vlasov_step_sc(ctypes.byref(grid), prec, vbc, _ptr(f_in), _ptr(scale_in),
                               _ptr(f_out), _ptr(scale_out), _ptr(g_n), _ptr(g_np1),
                               _ptr(rho_np1), float(coupling), float(dt), float(a2inv),
                               _ptr(work), int(work_bytes), _ptr(outflow), _stream(stream)),
           "vlasov_step_sc")


def vlasov_field_workspace_bytes(grid) -> int:
    return _lib.vlasov_field_workspace_bytes(ctypes.byref(grid))


def vlasov_field(grid, rho, coupling, field, work, work_bytes, stream=None):
    _check(_lib.vlasov_field(ctypes.byref(grid), _ptr(rho), float(coupling), _ptr(field),
                             _ptr(work), int(work_bytes), _stream(stream)), "vlasov_field")


def field(grid, rho, coupling, stream=None):
    """Acceleration field [3][nx][ny][nz] (FP32) of an FP64 density."""
    n = tuple(grid.n)
    out = torch.empty((3,) + n, dtype=torch.float32, device=rho.device)
    nb = vlasov_field_workspace_bytes(grid)
    work = torch.empty(nb, dtype=torch.uint8, device=rho.device)
    vlasov_field(grid, rho, coupling, out, work, nb, stream)
    return out


def vlasov_steps_workspace_bytes(grid, prec) -> int:
    return _lib.vlasov_steps_workspace_bytes(ctypes.byref(grid), prec)


def vlasov_steps(grid, prec, vbc, f_in, scale_in, f_out, scale_out, fields, nsteps, dt, a2inv,
                 work, work_bytes, outflow=None, stream=None):
    """a2inv: None or a sequence of nsteps host values."""
    a2 = None
    if a2inv is not None:
        a2 = (ctypes.c_double * int(nsteps))(*[float(v) for v in a2inv])
    _check(_lib.vlasov_steps(ctypes.byref(grid), prec, vbc, _ptr(f_in), _ptr(scale_in),
                             _ptr(f_out), _ptr(scale_out), _ptr(fields), int(nsteps), float(dt),
                             ctypes.cast(a2, ctypes.c_void_p) if a2 is not None else None,
                             _ptr(work), int(work_bytes), _ptr(outflow), _stream(stream)),
           "vlasov_steps")


def vlasov_step_moments(grid, prec, vbc, f_in, scale_in, f_out, scale_out, g_n, g_np1, dt,
                        a2inv, work, work_bytes, outflow, rho, umean, stream=None):
    _check(_lib.vlasov_step_moments(ctypes.byref(grid), prec, vbc, _ptr(f_in), _ptr(scale_in),
                                    _ptr(f_out), _ptr(scale_out), _ptr(g_n), _ptr(g_np1),
                                    float(dt), float(a2inv), _ptr(work), int(work_bytes),
                                    _ptr(outflow), _ptr(rho), _ptr(umean), _stream(stream)),
           "vlasov_step_moments")


def vlasov_moments(grid, prec, f, scale, rho, umean, mass, stream=None):
    _check(_lib.vlasov_moments(ctypes.byref(grid), prec, _ptr(f), _ptr(scale), _ptr(rho),
                               _ptr(umean), _ptr(mass), _stream(stream)), "vlasov_moments")


def vlasov_cosmo_a(cosmo, t) -> float:
    a = ctypes.c_double()
    _check(_lib.vlasov_cosmo_a(ctypes.byref(cosmo), float(t), ctypes.byref(a)), "vlasov_cosmo_a")
    return a.value


def vlasov_cosmo_t(cosmo, a) -> float:
    t = ctypes.c_double()
    _check(_lib.vlasov_cosmo_t(ctypes.byref(cosmo), float(a), ctypes.byref(t)), "vlasov_cosmo_t")
    return t.value


def vlasov_cosmo_steps(cosmo, t0, dt, nsteps):
    """(a [nsteps + 1], a2inv [nsteps]) as lists of floats."""
    a = (ctypes.c_double * (nsteps + 1))()
    a2 = (ctypes.c_double * max(nsteps, 1))()
    _check(_lib.vlasov_cosmo_steps(ctypes.byref(cosmo), float(t0), float(dt), int(nsteps), a, a2),
           "vlasov_cosmo_steps")
    return list(a), list(a2)[:nsteps]


def vlasov_dispersion(grid, prec, f, scale, rho, umean, sigma, stream=None):
    _check(_lib.vlasov_dispersion(ctypes.byref(grid), prec, _ptr(f), _ptr(scale), _ptr(rho),
                                  _ptr(umean), _ptr(sigma), _stream(stream)), "vlasov_dispersion")


def vlasov_sum_f64(x, n, out, stream=None):
    _check(_lib.vlasov_sum_f64(_ptr(x), int(n), _ptr(out), _stream(stream)), "vlasov_sum_f64")


def vlasov_field_noalloc_max_bytes() -> int:
    return _lib.vlasov_field_noalloc_max_bytes()


def vlasov_field_noalloc(grid, rho, coupling, field, stream=None):
    _check(_lib.vlasov_field_noalloc(ctypes.byref(grid), _ptr(rho), float(coupling), _ptr(field),
                                     _stream(stream)), "vlasov_field_noalloc")


def vlasov_encode(grid, prec, f32, codes, scale, stream=None):
    _check(_lib.vlasov_encode(ctypes.byref(grid), int(prec), _ptr(f32), _ptr(codes), _ptr(scale),
                              _stream(stream)), "vlasov_encode")


def vlasov_decode(grid, prec, codes, scale, f32, stream=None):
    _check(_lib.vlasov_decode(ctypes.byref(grid), int(prec), _ptr(codes), _ptr(scale), _ptr(f32),
                              _stream(stream)), "vlasov_decode")


def vlasov_valu_probe(out, iters, stream=None) -> float:
    """Launch the VALU probe over out.numel() threads; returns the lane-operations."""
    ops = ctypes.c_double(0.0)
    _check(_lib.vlasov_valu_probe(_ptr(out), int(out.numel()), int(iters), ctypes.byref(ops),
                                  _stream(stream)), "vlasov_valu_probe")
    return ops.value


def vlasov_stream_copy(src, dst, nbytes, stream=None):
    _check(_lib.vlasov_stream_copy(_ptr(src), _ptr(dst), int(nbytes), _stream(stream)),
           "vlasov_stream_copy")


def _pos_deriv(axis, kind):
    name = f"vlasov_advect_{axis}_{kind}"

    def fn(grid, f_in, x_in, x_out, dt_over_a2, stream=None):
        _check(getattr(_lib, name)(ctypes.byref(grid), _ptr(f_in), _ptr(x_in), _ptr(x_out),
                                   float(dt_over_a2), _stream(stream)), name)
    fn.__name__ = name
    return fn


def _vel_tan(axis):
    name = f"vlasov_advect_u{axis}_tan"

    def fn(grid, vbc, f_in, g, g_dot, dt, v_in, v_out, stream=None):
        _check(getattr(_lib, name)(ctypes.byref(grid), vbc, _ptr(f_in), _ptr(g), _ptr(g_dot),
                                   float(dt), _ptr(v_in), _ptr(v_out), _stream(stream)), name)
    fn.__name__ = name
    return fn


def _vel_adj(axis):
    name = f"vlasov_advect_u{axis}_adj"

    def fn(grid, vbc, f_in, g, dt, lam_out, lam_in, lam_g=None, stream=None):
        _check(getattr(_lib, name)(ctypes.byref(grid), vbc, _ptr(f_in), _ptr(g), float(dt),
                                   _ptr(lam_out), _ptr(lam_in), _ptr(lam_g), _stream(stream)),
               name)
    fn.__name__ = name
    return fn


for _ax in "xyz":
    globals()[f"vlasov_advect_{_ax}_tan"] = _pos_deriv(_ax, "tan")
    globals()[f"vlasov_advect_{_ax}_adj"] = _pos_deriv(_ax, "adj")
    globals()[f"vlasov_advect_u{_ax}_tan"] = _vel_tan(_ax)
    globals()[f"vlasov_advect_u{_ax}_adj"] = _vel_adj(_ax)


def vlasov_step_adj_workspace_bytes(grid) -> int:
    return _lib.vlasov_step_adj_workspace_bytes(ctypes.byref(grid))


def vlasov_step_adj(grid, vbc, f_in, g_n, g_np1, dt, a2inv, lam_out, lam_in, lam_g_n, lam_g_np1,
                    work, work_bytes, stream=None):
    _check(_lib.vlasov_step_adj(ctypes.byref(grid), vbc, _ptr(f_in), _ptr(g_n), _ptr(g_np1),
                                float(dt), float(a2inv), _ptr(lam_out), _ptr(lam_in),
                                _ptr(lam_g_n), _ptr(lam_g_np1), _ptr(work), int(work_bytes),
                                _stream(stream)), "vlasov_step_adj")


def vlasov_moments_adj(grid, rho, umean, lam_rho, lam_umean, lam_f, stream=None):
    _check(_lib.vlasov_moments_adj(ctypes.byref(grid), _ptr(rho), _ptr(umean), _ptr(lam_rho),
                                   _ptr(lam_umean), _ptr(lam_f), _stream(stream)),
           "vlasov_moments_adj")


# --- convenience (allocation with torch, then the entry points) ----------------------------

class State:
    """f in one storage precision, with its scales for FP16/BF16."""

    def __init__(self, grid, prec, f, scale=None):
        self.grid, self.prec, self.f, self.scale = grid, prec, f, scale

    @property
    def shape(self):
        return grid_shape(self.grid)


def empty_state(grid, prec, device="cuda") -> State:
    shape = grid_shape(grid)
    f = torch.empty(shape, dtype=TORCH_DTYPE[prec], device=device)
    scale = None
    if prec != F32:
        scale = torch.empty(shape[:-1], dtype=torch.float32, device=device)
    return State(grid, prec, f, scale)


def encode(grid, prec, f32, stream=None) -> State:
    """Store an FP32 tensor in the given precision through vlasov_encode
    (per-uz-line max scale, RNE codes: what the sweeps store)."""
    f32 = f32.contiguous()
    if prec == F32:
        return State(grid, prec, f32)
    out = empty_state(grid, prec, f32.device)
    vlasov_encode(grid, prec, f32, out.f, out.scale, stream)
    return out


def decode(state: State, stream=None) -> torch.Tensor:
    """FP32 values of a state through vlasov_decode (code times scale)."""
    if state.prec == F32:
        return state.f
    out = torch.empty(state.f.shape, dtype=torch.float32, device=state.f.device)
    vlasov_decode(state.grid, state.prec, state.f, state.scale, out, stream)
    return out


def save(path, state: State, step: int = 0, t: float = 0.0, outflow=None):
    """Write a state to an .npz file (no pickled objects): the grid, the
    storage precision, f bit for bit (FP16/BF16 codes as their 16-bit
    patterns), the scales, the step index, the time and optionally the
    per-cell outflow tally."""
    g = state.grid
    f = state.f.detach()
    bits = f.view(torch.int16) if state.prec != F32 else f
    arrays = {
        "n": np.array(list(g.n), np.int64), "nu": np.array(list(g.nu), np.int64),
        "L": np.array(list(g.L), np.float64), "umax": np.array(list(g.umax), np.float64),
        "prec": np.array(int(state.prec), np.int64), "step": np.array(int(step), np.int64),
        "t": np.array(float(t), np.float64), "f": bits.cpu().numpy(),
    }
    if state.scale is not None:
        arrays["scale"] = state.scale.detach().cpu().numpy()
    if outflow is not None:
        arrays["outflow"] = outflow.detach().cpu().numpy()
    np.savez(path, **arrays)


def load(path, device="cuda"):
    """Read a state written by save: (State, step, t, outflow or None)."""
    with np.load(path, allow_pickle=False) as z:
        grid = make_grid(tuple(z["n"]), tuple(z["nu"]), tuple(z["L"]), tuple(z["umax"]))
        prec = int(z["prec"])
        f = torch.from_numpy(z["f"]).to(device)
        if prec != F32:
            f = f.view(TORCH_DTYPE[prec])
        scale = torch.from_numpy(z["scale"]).to(device) if "scale" in z else None
        outflow = torch.from_numpy(z["outflow"]).to(device) if "outflow" in z else None
        return State(grid, prec, f.contiguous(), scale), int(z["step"]), float(z["t"]), outflow


def advect(axis: str, state: State, dt, g=None, vbc=VBC_OUTFLOW, outflow=None, stream=None):
    out = empty_state(state.grid, state.prec, state.f.device)
    if axis in ("x", "y", "z"):
        globals()[f"vlasov_advect_{axis}"](state.grid, state.prec, state.f, state.scale, out.f,
                                          out.scale, dt, stream)
    else:
        globals()[f"vlasov_advect_{axis}"](state.grid, state.prec, vbc, state.f, state.scale,
                                          out.f, out.scale, g, dt, outflow, stream)
    return out


def kick(state: State, g, dt, vbc=VBC_OUTFLOW, outflow=None, stream=None) -> State:
    out = empty_state(state.grid, state.prec, state.f.device)
    nbytes = vlasov_step_workspace_bytes(state.grid, state.prec)
    work = torch.empty(nbytes, dtype=torch.uint8, device=state.f.device)
    vlasov_kick(state.grid, state.prec, vbc, state.f, state.scale, out.f, out.scale, g, dt, work,
                nbytes, outflow, stream)
    return out


def step(state: State, g_n, g_np1, dt, a2inv=1.0, vbc=VBC_OUTFLOW, outflow=None, work=None,
         out=None, stream=None) -> State:
    grid = state.grid
    nbytes = vlasov_step_workspace_bytes(grid, state.prec)
    if work is None:
        work = torch.empty(nbytes, dtype=torch.uint8, device=state.f.device)
    if out is None:
        out = empty_state(grid, state.prec, state.f.device)
    vlasov_step(grid, state.prec, vbc, state.f, state.scale, out.f, out.scale, g_n, g_np1, dt,
                a2inv, work, nbytes, outflow, stream)
    return out


def moments(state: State, with_mean=True, stream=None):
    n = tuple(state.grid.n)
    dev = state.f.device
    rho = torch.empty(n, dtype=torch.float64, device=dev)
    um = torch.empty((3,) + n, dtype=torch.float64, device=dev) if with_mean else None
    mass = torch.empty((), dtype=torch.float64, device=dev)
    vlasov_moments(state.grid, state.prec, state.f, state.scale, rho, um, mass, stream)
    return rho, um, mass


def dispersion(state: State, stream=None):
    """(rho, umean, sigma): sigma [6][nx][ny][nz] in the order xx, xy, xz, yy, yz, zz."""
    n = tuple(state.grid.n)
    dev = state.f.device
    rho = torch.empty(n, dtype=torch.float64, device=dev)
    um = torch.empty((3,) + n, dtype=torch.float64, device=dev)
    sig = torch.empty((6,) + n, dtype=torch.float64, device=dev)
    vlasov_dispersion(state.grid, state.prec, state.f, state.scale, rho, um, sig, stream)
    return rho, um, sig
