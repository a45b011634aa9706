"""Python access to the FP64 CPU oracle (``vpinn_oracle.c``).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the CPU-baseline
leg of the benchmark are the only callers.  The HIP library never imports,
links or executes anything here, and this module imports nothing from it.

The C source computes the FastVPINNs discrete loss of Section 4.4 (Algorithm 3)
element by element in double precision; see the header of the C file for the
passages each function follows.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "vpinn_oracle.c")
_LIB = os.path.join(_HERE, "libvpinn_oracle.so")

FN2 = C.CFUNCTYPE(C.c_double, C.c_double, C.c_double, C.c_void_p)
_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_ip = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, strict IEEE: no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-D_DEFAULT_SOURCE", "-ffp-contract=off",
                               "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = C.CDLL(_LIB)
        L.orc_legendre.restype = C.c_double
        L.orc_legendre.argtypes = [C.c_int, C.c_double]
        L.orc_legendre_deriv.restype = C.c_double
        L.orc_legendre_deriv.argtypes = [C.c_int, C.c_double]
        L.orc_gll.restype = C.c_int
        L.orc_gll.argtypes = [C.c_int, _dp, _dp]
        L.orc_test_fn.restype = None
        L.orc_test_fn.argtypes = [C.c_int, C.c_double, C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.orc_map_point.restype = None
        L.orc_map_point.argtypes = [_dp, C.c_double, C.c_double, C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.orc_jacobian.restype = None
        L.orc_jacobian.argtypes = [_dp, C.c_double, C.c_double, _dp, _dp, C.POINTER(C.c_double)]
        L.orc_assemble.restype = C.c_int
        L.orc_assemble.argtypes = [C.c_int64, _dp, C.c_int64, _ip, C.c_int, C.c_int, C.c_int, _dp,
                                   FN2, C.c_void_p, _dp, _dp, _dp, _dp, C.c_void_p, C.POINTER(C.c_int64)]
        L.orc_n_params.restype = C.c_int64
        L.orc_n_params.argtypes = [C.c_int, C.c_int]
        L.orc_n_params_heads.restype = C.c_int64
        L.orc_n_params_heads.argtypes = [C.c_int, C.c_int, C.c_int]
        L.orc_mlp_eval.restype = None
        L.orc_mlp_eval.argtypes = [C.c_int, C.c_int, C.c_int, _dp, C.c_int64, _dp, _dp, _dp, _dp, C.c_void_p]
        L.orc_mlp_vjp.restype = None
        L.orc_mlp_vjp.argtypes = [C.c_int, C.c_int, C.c_int, _dp, C.c_int64, _dp, _dp, _dp, _dp, C.c_void_p, _dp]
        L.orc_residual.restype = None
        L.orc_residual.argtypes = [C.c_int64, C.c_int, C.c_int, _dp, _dp, _dp, _dp, _dp, C.c_double, C.c_void_p,
                                   C.c_double, C.c_double, C.c_void_p, _dp]
        L.orc_loss_grad.restype = C.c_int
        L.orc_loss_grad.argtypes = [C.c_int64, C.c_int, C.c_int, _dp, _dp, _dp, _dp, C.c_void_p, C.c_double,
                                    C.c_double, C.c_int64, _dp, _dp, C.c_int64, _dp, _dp,
                                    C.c_int, C.c_int, C.c_int, _dp, C.c_double, C.c_double, C.c_double,
                                    C.c_double, _dp, C.c_void_p, C.c_void_p, C.c_void_p]
        L.orc_adam.restype = None
        L.orc_adam.argtypes = [C.c_int64, _dp, _dp, _dp, _dp, C.c_int64, C.c_double, C.c_double,
                               C.c_double, C.c_double]
        _lib = L
    return _lib


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


# --------------------------------------------------------------------------- 1D pieces

def legendre(m: int, t: float) -> float:
    return lib().orc_legendre(m, t)


def legendre_deriv(m: int, t: float) -> float:
    return lib().orc_legendre_deriv(m, t)


def gll(n: int):
    x = np.zeros(n)
    w = np.zeros(n)
    if lib().orc_gll(n, x, w) != 0:
        raise ValueError("bad GLL order")
    return x, w


def test_fn(r: int, t: float):
    p = C.c_double()
    d = C.c_double()
    lib().orc_test_fn(r, t, C.byref(p), C.byref(d))
    return p.value, d.value


def map_point(verts, xi, eta):
    x = C.c_double()
    y = C.c_double()
    lib().orc_map_point(_f64(verts).ravel(), xi, eta, C.byref(x), C.byref(y))
    return x.value, y.value


def jacobian(verts, xi, eta):
    J = np.zeros(4)
    Ji = np.zeros(4)
    D = C.c_double()
    lib().orc_jacobian(_f64(verts).ravel(), xi, eta, J, Ji, C.byref(D))
    return J.reshape(2, 2), Ji.reshape(2, 2), D.value


# --------------------------------------------------------------------------- assembly

@dataclass
class Assembled:
    Gx: np.ndarray   # [n_elem, n_test, n_quad]
    Gy: np.ndarray
    F: np.ndarray    # [n_elem, n_test]
    X: np.ndarray    # [n_elem, n_quad, 2]
    n: int
    nt: int
    M: Optional[np.ndarray] = None  # [n_elem, n_test, n_quad] w_q det J v_k (convection term), if asked for

    @property
    def n_elem(self):
        return self.F.shape[0]


class OracleError(RuntimeError):
    def __init__(self, code, elem):
        super().__init__(f"oracle assembly failed with code {code} at element {elem}")
        self.code = code
        self.elem = elem


def assemble(xy, quad, n: int, nt: int, f_amp: float = 0.0, f_kx: float = 0.0, f_ky: float = 0.0,
             f_callable=None, want_M: bool = False) -> Assembled:
    """G_x, G_y, F and physical quadrature points; f either amp*sin(kx x)sin(ky y) or a callable.
    want_M: also the convection-term weights M = w_q det J v_k (convection-diffusion, Section 2.1)."""
    xy = _f64(xy)
    quad = np.ascontiguousarray(np.asarray(quad, dtype=np.int32))
    ne = quad.shape[0]
    nq, ntest = n * n, nt * nt
    Gx = np.zeros((ne, ntest, nq))
    Gy = np.zeros((ne, ntest, nq))
    F = np.zeros((ne, ntest))
    X = np.zeros((ne, nq, 2))
    M = np.zeros((ne, ntest, nq)) if want_M else None
    bad = C.c_int64(-1)
    if f_callable is None:
        kind, par, cb = 1, np.array([f_amp, f_kx, f_ky], dtype=np.float64), FN2(lambda x, y, u: 0.0)
    else:
        kind, par, cb = 0, np.zeros(3), FN2(lambda x, y, u: float(f_callable(x, y)))
    rc = lib().orc_assemble(xy.shape[0], xy.ravel(), ne, quad.ravel(), n, nt, kind, par, cb, None,
                            Gx, Gy, F, X, M.ctypes.data_as(C.c_void_p) if want_M else None, C.byref(bad))
    if rc != 0:
        raise OracleError(rc, bad.value)
    return Assembled(Gx, Gy, F, X, n, nt, M)


def assemble_problem(prob) -> Assembled:
    conv = tuple(getattr(prob, "conv", (0.0, 0.0)))
    return assemble(prob.mesh.xy, prob.mesh.quad, prob.quad_order, prob.test_order,
                    prob.f_amp, prob.f_kx, prob.f_ky, f_callable=getattr(prob, "f_fn", None),
                    want_M=conv != (0.0, 0.0))


# --------------------------------------------------------------------------- network

def n_params(H: int, L: int, heads: int = 1) -> int:
    return int(lib().orc_n_params_heads(H, L, heads))


def mlp_eval(theta, H: int, L: int, xy, heads: int = 1):
    """u, u_x, u_y at the points; with heads = 2 also the second output e."""
    xy = _f64(xy).reshape(-1, 2)
    n = xy.shape[0]
    u, ux, uy, e = np.zeros(n), np.zeros(n), np.zeros(n), np.zeros(n)
    lib().orc_mlp_eval(H, L, heads, _f64(theta), n, xy.ravel(), u, ux, uy, e.ctypes.data_as(C.c_void_p))
    return (u, ux, uy) if heads == 1 else (u, ux, uy, e)


def mlp_vjp(theta, H: int, L: int, xy, ub, uxb, uyb, eb=None, heads: int = 1):
    xy = _f64(xy).reshape(-1, 2)
    g = np.zeros(n_params(H, L, heads))
    ebp = None if eb is None else _f64(eb)
    lib().orc_mlp_vjp(H, L, heads, _f64(theta), xy.shape[0], xy.ravel(), _f64(ub), _f64(uxb), _f64(uyb),
                      None if ebp is None else ebp.ctypes.data_as(C.c_void_p), g)
    return g


def prediction_error(theta, H: int, L: int, xy, ref, heads: int = 1, output: int = 0):
    """Accuracy of a network prediction against reference values at points (Sec. 4 reports the mean absolute
    error of u on a grid and point-wise absolute errors of u and of the predicted diffusion coefficient):
    mean |p - ref|, max |p - ref|, and the relative L2 error ||p - ref|| / ||ref||, where p is output 0 (u)
    or, for a two-output network, output 1 (e)."""
    outs = mlp_eval(theta, H, L, xy, heads)
    p = outs[0] if output == 0 else outs[3]
    d = p - _f64(ref).ravel()
    nr = float(np.sqrt(np.sum(_f64(ref) ** 2)))
    return float(np.mean(np.abs(d))), float(np.max(np.abs(d))), float(np.sqrt(np.sum(d * d))) / nr


def _conv_args(asm: Assembled, conv):
    if conv is None or tuple(conv) == (0.0, 0.0):
        return None, 0.0, 0.0
    if asm.M is None:
        raise ValueError("a convection term needs an assembly with want_M=True")
    return asm.M.ctypes.data_as(C.c_void_p), float(conv[0]), float(conv[1])


def residual(asm: Assembled, ux, uy, eps: float = 1.0, conv=None, epsq=None):
    """R = eps * A + sum_q (b . grad u) M - F; conv = (b_x, b_y) or None; epsq: a per-point diffusion
    coefficient (space-dependent, Sec. 4.7.2) replacing eps."""
    R = np.zeros_like(asm.F)
    Mp, bx, by = _conv_args(asm, conv)
    ep = None if epsq is None else _f64(epsq).ravel()
    lib().orc_residual(asm.n_elem, asm.n * asm.n, asm.nt * asm.nt, asm.Gx.ravel(), asm.Gy.ravel(),
                       asm.F.ravel(), _f64(ux).ravel(), _f64(uy).ravel(), eps, Mp, bx, by,
                       None if ep is None else ep.ctypes.data_as(C.c_void_p), R)
    return R


# --------------------------------------------------------------------------- loss

@dataclass
class LossGrad:
    loss: np.ndarray        # [L, L_v, L_b, L_s]
    grad: Optional[np.ndarray]
    grad_eps: float
    R: Optional[np.ndarray] = None


def c_v(asm: Assembled, loss_norm: int = 0) -> float:
    """loss_norm 0: 1/N_test (Algorithm 3); 1: 1/N_elem (variational-loss equation, Section 2.3)."""
    return 1.0 / (asm.nt * asm.nt) if loss_norm == 0 else 1.0 / asm.n_elem


def loss_grad(asm: Assembled, theta, H: int, L: int, bnd_xy=None, bnd_g=None, sens_xy=None, sens_u=None,
              eps: float = 1.0, tau: float = 10.0, gamma: float = 0.0, loss_norm: int = 0,
              want_grad: bool = True, want_R: bool = False, conv=None, heads: int = 1) -> LossGrad:
    """heads = 2: the network's second output is the space-dependent diffusion coefficient (eps unused)."""
    bxy = _f64(np.zeros((0, 2)) if bnd_xy is None else bnd_xy).reshape(-1, 2)
    bg = _f64(np.zeros(0) if bnd_g is None else bnd_g)
    sxy = _f64(np.zeros((0, 2)) if sens_xy is None else sens_xy).reshape(-1, 2)
    su = _f64(np.zeros(0) if sens_u is None else sens_u)
    loss = np.zeros(4)
    grad = np.zeros(n_params(H, L, heads)) if want_grad else None
    geps = C.c_double(0.0)
    R = np.zeros_like(asm.F) if want_R else None
    Mp, cbx, cby = _conv_args(asm, conv)
    rc = lib().orc_loss_grad(
        asm.n_elem, asm.n * asm.n, asm.nt * asm.nt, asm.Gx.ravel(), asm.Gy.ravel(), asm.F.ravel(),
        asm.X.ravel(), Mp, cbx, cby, bxy.shape[0], bxy.ravel(), bg, sxy.shape[0], sxy.ravel(), su,
        H, L, heads, _f64(theta), eps, tau, gamma, c_v(asm, loss_norm), loss,
        grad.ctypes.data_as(C.c_void_p) if want_grad else None,
        C.cast(C.pointer(geps), C.c_void_p) if want_grad else None,
        R.ctypes.data_as(C.c_void_p) if want_R else None)
    if rc != 0:
        raise RuntimeError(f"oracle loss failed: {rc}")
    return LossGrad(loss, grad, geps.value, R)


def problem_loss_grad(prob, asm: Assembled, theta, eps: Optional[float] = None, loss_norm: int = 0,
                      want_grad: bool = True) -> LossGrad:
    """eps: the trainable diffusion coefficient of the inverse problem; otherwise the problem's own
    diffusion coefficient (1 for Poisson); the problem's convection velocity enters through conv."""
    e = getattr(prob, "diff", 1.0) if eps is None else eps
    return loss_grad(asm, theta, prob.width, prob.n_hidden, prob.bnd_xy, prob.bnd_g,
                     prob.sens_xy, prob.sens_u, eps=e, tau=prob.tau, gamma=prob.gamma,
                     loss_norm=loss_norm, want_grad=want_grad, conv=getattr(prob, "conv", None),
                     heads=getattr(prob, "heads", 1))


def adam(theta, g, m, v, t: int, lr: float = 1e-3, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
    """In-place Adam step on float64 arrays."""
    lib().orc_adam(theta.size, theta, _f64(g), m, v, t, lr, b1, b2, eps)
