"""ctypes binding of libvpinn.so (include/vpinn.h).

Argument marshalling only: every step of the computation runs in the HIP
library.  torch supplies device memory and streams; device arguments are torch
CUDA tensors (float32, contiguous) and host arguments are numpy arrays.
Functions keep the C names.  A missing library raises immediately: there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libvpinn.so")

VPINN_OK = 0
VPINN_E_INVALID = -1
VPINN_E_MESH = -2
VPINN_E_NOMEM = -3
VPINN_E_NONFINITE = -4
VPINN_E_DEVICE = -5
VPINN_E_UNSUPPORTED = -6
VPINN_NOALLOC_MAX_POINTS = 2097152

VPINN_FORCING_CALLBACK = 0
VPINN_FORCING_SINSIN = 1
VPINN_PATH_FUSED = 0
VPINN_PATH_PLAIN = 1
VPINN_NORM_TEST = 0
VPINN_NORM_ELEM = 1
VPINN_TENSOR_GX, VPINN_TENSOR_GY, VPINN_TENSOR_F, VPINN_TENSOR_X, VPINN_TENSOR_M = 0, 1, 2, 3, 4
PROFILE_EVENTS = 5  # VPINN_PROFILE_EVENTS: forward | contraction | backward | reduction

SCALAR_FN = C.CFUNCTYPE(C.c_double, C.c_double, C.c_double, C.c_void_p)


class vpinn_mesh(C.Structure):
    _fields_ = [("n_nodes", C.c_int64), ("xy", C.POINTER(C.c_double)),
                ("n_elem", C.c_int64), ("quad", C.POINTER(C.c_int32))]


class vpinn_forcing(C.Structure):
    _fields_ = [("kind", C.c_int32), ("amp", C.c_double), ("kx", C.c_double), ("ky", C.c_double),
                ("fn", SCALAR_FN), ("user", C.c_void_p)]


class vpinn_problem_info(C.Structure):
    _fields_ = [("n_elem", C.c_int64), ("n_quad", C.c_int64), ("n_test", C.c_int64),
                ("n_points", C.c_int64), ("n_boundary", C.c_int64), ("n_sensors", C.c_int64),
                ("quad_order", C.c_int32), ("test_order", C.c_int32),
                ("diffusion", C.c_double), ("velocity_x", C.c_double), ("velocity_y", C.c_double),
                ("shared_premultiplier", C.c_int32), ("variable_diffusion", C.c_int32), ("matrix_free", C.c_int32),
                ("n_distinct_points", C.c_int64)]


class vpinn_loss_cfg(C.Structure):
    _fields_ = [("n_hidden", C.c_int32), ("width", C.c_int32), ("tau", C.c_float), ("gamma", C.c_float),
                ("loss_norm", C.c_int32), ("path", C.c_int32), ("n_outputs", C.c_int32)]


class vpinn_tuning(C.Structure):
    _fields_ = [("fwd_waves", C.c_int32), ("chunk_shift", C.c_int32), ("rows_per_pass", C.c_int32),
                ("store_activations", C.c_int32), ("one_pass", C.c_int32)]

    def as_tuple(self):
        return (self.fwd_waves, self.chunk_shift, self.rows_per_pass, self.store_activations, self.one_pass)


class VpinnError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"vpinn error {code}: {msg}")
        self.code = code


_lib = None

# every symbol of include/vpinn.h with its (restype, argtypes)
_SIGNATURES = {
    "vpinn_assemble_cd2d": (C.c_int32, [C.POINTER(vpinn_mesh), C.c_int32, C.c_int32, C.c_double, C.c_double,
                                        C.c_double, C.POINTER(vpinn_forcing), C.c_void_p, C.POINTER(C.c_void_p)]),
    "vpinn_assemble": (C.c_int32, [C.POINTER(vpinn_mesh), C.c_int32, C.c_int32, C.POINTER(vpinn_forcing),
                                   C.c_void_p, C.POINTER(C.c_void_p)]),
    "vpinn_set_boundary": (C.c_int32, [C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p]),
    "vpinn_set_sensors": (C.c_int32, [C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p]),
    "vpinn_set_shared_points": (C.c_int32, [C.c_void_p, C.POINTER(vpinn_mesh), C.c_int32]),
    "vpinn_get_info": (C.c_int32, [C.c_void_p, C.POINTER(vpinn_problem_info)]),
    "vpinn_read_tensor": (C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p, C.c_int64]),
    "vpinn_assemble_vardiff": (C.c_int32, [C.POINTER(vpinn_mesh), C.c_int32, C.c_int32, C.c_double, C.c_double,
                                           C.POINTER(vpinn_forcing), C.c_void_p, C.POINTER(C.c_void_p)]),
    "vpinn_assemble_matrix_free": (C.c_int32, [C.POINTER(vpinn_mesh), C.c_int32, C.c_int32, C.c_double,
                                               C.c_double, C.c_double, C.c_int32, C.POINTER(vpinn_forcing),
                                               C.c_void_p, C.POINTER(C.c_void_p)]),
    "vpinn_n_params": (C.c_int64, [C.c_int32, C.c_int32]),
    "vpinn_n_params_out": (C.c_int64, [C.c_int32, C.c_int32, C.c_int32]),
    "vpinn_loss_and_grad": (C.c_int32, [C.c_void_p, C.POINTER(vpinn_loss_cfg), C.c_void_p, C.c_void_p,
                                        C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "vpinn_residual": (C.c_int32, [C.c_void_p, C.POINTER(vpinn_loss_cfg), C.c_void_p, C.c_void_p,
                                   C.c_void_p, C.c_void_p]),
    "vpinn_eval_network": (C.c_int32, [C.c_int32, C.c_int32, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p,
                                       C.c_void_p, C.c_void_p, C.c_void_p]),
    "vpinn_eval_network_heads": (C.c_int32, [C.c_int32, C.c_int32, C.c_int32, C.c_void_p, C.c_int64, C.c_void_p,
                                             C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "vpinn_eval_error": (C.c_int32, [C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_void_p, C.c_int64, C.c_void_p,
                                     C.c_void_p, C.c_void_p, C.c_void_p]),
    "vpinn_eval_error_noalloc": (C.c_int32, [C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_void_p, C.c_int64,
                                             C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "vpinn_adam_step": (C.c_int32, [C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64,
                                    C.c_float, C.c_float, C.c_float, C.c_float, C.c_void_p]),
    "vpinn_batch_create": (C.c_int32, [C.c_int32, C.POINTER(C.c_void_p), C.POINTER(vpinn_loss_cfg),
                                       C.POINTER(C.c_void_p)]),
    "vpinn_batch_loss_and_grad": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                              C.c_void_p, C.c_void_p]),
    "vpinn_batch_step": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_float,
                                     C.c_float, C.c_float, C.c_float, C.c_void_p, C.c_void_p, C.c_void_p,
                                     C.c_void_p, C.c_void_p]),
    "vpinn_batch_capture": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_float,
                                        C.c_float, C.c_float, C.c_float, C.c_void_p, C.c_void_p, C.c_void_p,
                                        C.c_void_p, C.c_void_p]),
    "vpinn_batch_replay": (C.c_int32, [C.c_void_p, C.c_void_p]),
    "vpinn_batch_free": (None, [C.c_void_p]),
    "vpinn_batch_get_tuning": (C.c_int32, [C.c_void_p, C.POINTER(vpinn_tuning)]),
    "vpinn_batch_set_tuning": (C.c_int32, [C.c_void_p, C.POINTER(vpinn_tuning)]),
    "vpinn_batch_autotune": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_int32, C.POINTER(vpinn_tuning), C.c_void_p]),
    "vpinn_set_profile_events": (C.c_int32, [C.c_void_p, C.c_void_p]),
    "vpinn_batch_set_profile_events": (C.c_int32, [C.c_void_p, C.c_void_p]),
    "vpinn_problem_free": (None, [C.c_void_p]),
    "vpinn_last_error": (C.c_char_p, []),
}


def lib():
    """Load libvpinn.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                               "(there is no fallback implementation)")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(rc: int):
    if rc != VPINN_OK:
        raise VpinnError(rc, lib().vpinn_last_error().decode())


def _ptr(t) -> Optional[int]:
    """Device address of a torch tensor (float32, contiguous) or None."""
    if t is None:
        return None
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return t.data_ptr()


def _stream(stream) -> Optional[int]:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def vpinn_last_error() -> str:
    return lib().vpinn_last_error().decode()


def vpinn_n_params(width: int, n_hidden: int) -> int:
    return int(lib().vpinn_n_params(width, n_hidden))


def vpinn_n_params_out(width: int, n_hidden: int, n_outputs: int) -> int:
    return int(lib().vpinn_n_params_out(width, n_hidden, n_outputs))


class Problem:
    """Owner of a vpinn_problem handle (device G_x, G_y, F, points)."""

    def __init__(self, handle: int):
        self.handle = handle

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.vpinn_problem_free(self.handle)
            self.handle = None

    def info(self) -> vpinn_problem_info:
        return vpinn_get_info(self)


def vpinn_assemble(xy, quad, quad_order: int, test_order: int, amp: float = 0.0, kx: float = 0.0,
                   ky: float = 0.0, fn=None, stream=None, cd=None, vardiff=None, matrix_free: bool = False) -> Problem:
    """xy: host [n_nodes, 2] float64; quad: host [n_elem, 4] int32.  Forcing is amp*sin(kx x)sin(ky y),
    or the Python callable fn(x, y) evaluated on the host (kind VPINN_FORCING_CALLBACK).
    cd = (eps, bx, by): the convection-diffusion operator -eps Lap u + b . grad u (vpinn_assemble_cd2d);
    vardiff = (bx, by): -div(eps(x, y) grad u) + b . grad u with eps the network's second output
    (vpinn_assemble_vardiff).  matrix_free: store no G (vpinn_assemble_matrix_free), for any of the three."""
    xy = np.ascontiguousarray(xy, dtype=np.float64)
    quad = np.ascontiguousarray(quad, dtype=np.int32)
    mesh = vpinn_mesh(xy.shape[0], xy.ctypes.data_as(C.POINTER(C.c_double)), quad.shape[0],
                      quad.ctypes.data_as(C.POINTER(C.c_int32)))
    if fn is None:
        cb = SCALAR_FN(0)
        f = vpinn_forcing(VPINN_FORCING_SINSIN, amp, kx, ky, cb, None)
    else:
        cb = SCALAR_FN(lambda x, y, u: float(fn(x, y)))
        f = vpinn_forcing(VPINN_FORCING_CALLBACK, 0.0, 0.0, 0.0, cb, None)
    out = C.c_void_p()
    if matrix_free:
        eps, bx, by = (1.0, 0.0, 0.0) if cd is None else (float(v) for v in cd)
        if vardiff is not None:
            bx, by = (float(v) for v in vardiff)
        _check(lib().vpinn_assemble_matrix_free(C.byref(mesh), quad_order, test_order, eps, bx, by,
                                                1 if vardiff is not None else 0, C.byref(f), _stream(stream),
                                                C.byref(out)))
    elif vardiff is not None:
        bx, by = (float(v) for v in vardiff)
        _check(lib().vpinn_assemble_vardiff(C.byref(mesh), quad_order, test_order, bx, by, C.byref(f),
                                            _stream(stream), C.byref(out)))
    elif cd is None:
        _check(lib().vpinn_assemble(C.byref(mesh), quad_order, test_order, C.byref(f), _stream(stream),
                                    C.byref(out)))
    else:
        eps, bx, by = (float(v) for v in cd)
        _check(lib().vpinn_assemble_cd2d(C.byref(mesh), quad_order, test_order, eps, bx, by, C.byref(f),
                                         _stream(stream), C.byref(out)))
    return Problem(out.value)


def assemble_problem(prob, stream=None, matrix_free: bool = False, shared_points: bool = False) -> Problem:
    """Assemble a vpinn_inputs Problem (Poisson, convection-diffusion when it sets diff/conv, space-dependent
    diffusion when its network has two outputs) and upload its boundary and sensor sets."""
    diff, conv = getattr(prob, "diff", 1.0), tuple(getattr(prob, "conv", (0.0, 0.0)))
    two = getattr(prob, "heads", 1) == 2
    cd = None if two or (diff, conv) == (1.0, (0.0, 0.0)) else (diff, conv[0], conv[1])
    p = vpinn_assemble(prob.mesh.xy, prob.mesh.quad, prob.quad_order, prob.test_order, prob.f_amp, prob.f_kx,
                       prob.f_ky, fn=getattr(prob, "f_fn", None), stream=stream, cd=cd,
                       vardiff=conv if two else None, matrix_free=matrix_free)
    vpinn_set_boundary(p, prob.bnd_xy, prob.bnd_g)
    if len(prob.sens_xy):
        vpinn_set_sensors(p, prob.sens_xy, prob.sens_u)
    if shared_points:
        vpinn_set_shared_points(p, prob.mesh.xy, prob.mesh.quad)
    return p


def vpinn_set_shared_points(p: Problem, xy, quad, enable: bool = True):
    """Evaluate the network once per distinct interior point of the mesh (xy, quad) the problem came from."""
    xy = np.ascontiguousarray(xy, dtype=np.float64)
    quad = np.ascontiguousarray(quad, dtype=np.int32)
    mesh = vpinn_mesh(xy.shape[0], xy.ctypes.data_as(C.POINTER(C.c_double)), quad.shape[0],
                      quad.ctypes.data_as(C.POINTER(C.c_int32)))
    _check(lib().vpinn_set_shared_points(p.handle, C.byref(mesh), 1 if enable else 0))


def vpinn_set_boundary(p: Problem, xy, g):
    xy = np.ascontiguousarray(xy, dtype=np.float64).reshape(-1, 2)
    g = np.ascontiguousarray(g, dtype=np.float64)
    _check(lib().vpinn_set_boundary(p.handle, xy.shape[0], xy.ctypes.data, g.ctypes.data))


def vpinn_set_sensors(p: Problem, xy, d):
    xy = np.ascontiguousarray(xy, dtype=np.float64).reshape(-1, 2)
    d = np.ascontiguousarray(d, dtype=np.float64)
    _check(lib().vpinn_set_sensors(p.handle, xy.shape[0], xy.ctypes.data, d.ctypes.data))


def vpinn_get_info(p: Problem) -> vpinn_problem_info:
    info = vpinn_problem_info()
    _check(lib().vpinn_get_info(p.handle, C.byref(info)))
    return info


def vpinn_read_tensor(p: Problem, which: int) -> np.ndarray:
    info = vpinn_get_info(p)
    shapes = {VPINN_TENSOR_GX: (info.n_elem, info.n_test, info.n_quad),
              VPINN_TENSOR_GY: (info.n_elem, info.n_test, info.n_quad),
              VPINN_TENSOR_F: (info.n_elem, info.n_test),
              VPINN_TENSOR_X: (info.n_elem, info.n_quad, 2),
              VPINN_TENSOR_M: (info.n_elem, info.n_test, info.n_quad)}
    out = np.empty(shapes[which], dtype=np.float32)
    _check(lib().vpinn_read_tensor(p.handle, which, out.ctypes.data, out.size))
    return out


def loss_cfg(width: int = 30, n_hidden: int = 3, tau: float = 10.0, gamma: float = 0.0,
             loss_norm: int = VPINN_NORM_TEST, path: int = VPINN_PATH_FUSED, n_outputs: int = 1) -> vpinn_loss_cfg:
    return vpinn_loss_cfg(n_hidden, width, tau, gamma, loss_norm, path, n_outputs)


def vpinn_loss_and_grad(p: Problem, cfg: vpinn_loss_cfg, params, eps=None, loss=None, grad=None,
                        grad_eps=None, stream=None):
    _check(lib().vpinn_loss_and_grad(p.handle, C.byref(cfg), _ptr(params), _ptr(eps), _ptr(loss), _ptr(grad),
                                     _ptr(grad_eps), _stream(stream)))


def vpinn_residual(p: Problem, cfg: vpinn_loss_cfg, params, R, eps=None, stream=None):
    _check(lib().vpinn_residual(p.handle, C.byref(cfg), _ptr(params), _ptr(eps), _ptr(R), _stream(stream)))


def vpinn_eval_network(width: int, n_hidden: int, params, xy, u=None, ux=None, uy=None, stream=None):
    n = xy.shape[0]
    _check(lib().vpinn_eval_network(width, n_hidden, _ptr(params), n, _ptr(xy), _ptr(u), _ptr(ux), _ptr(uy),
                                    _stream(stream)))


def vpinn_eval_network_heads(width: int, n_hidden: int, n_outputs: int, params, xy, u=None, ux=None, uy=None,
                             e=None, stream=None):
    n = xy.shape[0]
    _check(lib().vpinn_eval_network_heads(width, n_hidden, n_outputs, _ptr(params), n, _ptr(xy), _ptr(u),
                                          _ptr(ux), _ptr(uy), _ptr(e), _stream(stream)))


def vpinn_eval_error(width: int, n_hidden: int, params, xy, ref, out, n_outputs: int = 1, output: int = 0,
                     stream=None):
    """out: device float64 tensor of 3: mean |p - ref|, max |p - ref|, relative L2 error."""
    _check(lib().vpinn_eval_error(width, n_hidden, n_outputs, output, _ptr(params), xy.shape[0], _ptr(xy), _ptr(ref),
                                  _ptr(out), _stream(stream)))


def vpinn_eval_error_noalloc(width: int, n_hidden: int, params, xy, ref, out, n_outputs: int = 1, output: int = 0,
                             stream=None, n=None):
    """As vpinn_eval_error, with the library's fixed workspace (n <= VPINN_NOALLOC_MAX_POINTS); n defaults to
    the number of points in xy."""
    _check(lib().vpinn_eval_error_noalloc(width, n_hidden, n_outputs, output, _ptr(params),
                                          xy.shape[0] if n is None else n, _ptr(xy), _ptr(ref), _ptr(out),
                                          _stream(stream)))


def vpinn_adam_step(params, grad, m, v, step: int, lr: float = 1e-3, beta1: float = 0.9, beta2: float = 0.999,
                    eps: float = 1e-8, stream=None):
    _check(lib().vpinn_adam_step(params.numel(), _ptr(params), _ptr(grad), _ptr(m), _ptr(v), step, lr, beta1,
                                 beta2, eps, _stream(stream)))


class Batch:
    """Owner of a vpinn_batch handle; keeps its problems alive."""

    def __init__(self, handle: int, problems):
        self.handle = handle
        self.problems = list(problems)

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.vpinn_batch_free(self.handle)
            self.handle = None


def vpinn_batch_create(problems, cfg: vpinn_loss_cfg) -> Batch:
    arr = (C.c_void_p * len(problems))(*[p.handle for p in problems])
    out = C.c_void_p()
    _check(lib().vpinn_batch_create(len(problems), arr, C.byref(cfg), C.byref(out)))
    return Batch(out.value, problems)


def vpinn_batch_loss_and_grad(b: Batch, params, eps=None, losses=None, grads=None, grad_eps=None, stream=None):
    _check(lib().vpinn_batch_loss_and_grad(b.handle, _ptr(params), _ptr(eps), _ptr(losses), _ptr(grads),
                                           _ptr(grad_eps), _stream(stream)))


def vpinn_batch_step(b: Batch, params, m, v, step, lr: float = 1e-3, beta1: float = 0.9, beta2: float = 0.999,
                     eps: float = 1e-8, losses=None, stream=None, diff=None, diff_m=None, diff_v=None):
    """step: device int64 tensor of one element (incremented by the call).  diff, diff_m, diff_v: device [n]
    float tensors (all or none): each problem's trainable diffusion coefficient and its Adam moments."""
    _check(lib().vpinn_batch_step(b.handle, _ptr(params), _ptr(m), _ptr(v), _ptr(step), lr, beta1, beta2, eps,
                                  _ptr(losses), _ptr(diff), _ptr(diff_m), _ptr(diff_v), _stream(stream)))


def vpinn_batch_capture(b: Batch, params, m, v, step, lr: float = 1e-3, beta1: float = 0.9, beta2: float = 0.999,
                        eps: float = 1e-8, losses=None, stream=None, diff=None, diff_m=None, diff_v=None):
    _check(lib().vpinn_batch_capture(b.handle, _ptr(params), _ptr(m), _ptr(v), _ptr(step), lr, beta1, beta2, eps,
                                     _ptr(losses), _ptr(diff), _ptr(diff_m), _ptr(diff_v), _stream(stream)))


def vpinn_batch_replay(b: Batch, stream=None):
    _check(lib().vpinn_batch_replay(b.handle, _stream(stream)))


def vpinn_batch_get_tuning(b: Batch):
    """(fwd_waves, chunk_shift, rows_per_pass, store_activations, one_pass) of the batch's plan."""
    t = vpinn_tuning()
    _check(lib().vpinn_batch_get_tuning(b.handle, C.byref(t)))
    return t.as_tuple()


def vpinn_batch_set_tuning(b: Batch, fwd_waves: int, chunk_shift: int, rows_per_pass: int,
                           store_activations: int = 0, one_pass: int = 0):
    t = vpinn_tuning(fwd_waves, chunk_shift, rows_per_pass, store_activations, one_pass)
    _check(lib().vpinn_batch_set_tuning(b.handle, C.byref(t)))


def vpinn_batch_autotune(b: Batch, params, reps: int = 5, stream=None):
    """Time the batch's candidate tile shapes at `params` and keep the fastest; returns it."""
    t = vpinn_tuning()
    _check(lib().vpinn_batch_autotune(b.handle, _ptr(params), reps, C.byref(t), _stream(stream)))
    return t.as_tuple()


def _event_array(events):
    if events is None:
        return None
    if len(events) != PROFILE_EVENTS:
        raise ValueError(f"expected {PROFILE_EVENTS} events, got {len(events)}")
    handles = []
    for e in events:
        if e is None:
            handles.append(None)
        else:
            h = e.cuda_event
            if not h:
                raise ValueError("torch events must be recorded once before their handles are passed")
            handles.append(h)
    return (C.c_void_p * PROFILE_EVENTS)(*handles)


def vpinn_set_profile_events(p: Problem, events=None):
    """events: PROFILE_EVENTS torch.cuda.Event(enable_timing=True) already recorded once (or None to disable)."""
    arr = _event_array(events)
    _check(lib().vpinn_set_profile_events(p.handle, arr))


def vpinn_batch_set_profile_events(b: Batch, events=None):
    arr = _event_array(events)
    _check(lib().vpinn_batch_set_profile_events(b.handle, arr))
