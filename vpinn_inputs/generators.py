"""Seeded synthetic inputs for the VPINN hot path.

This module produces *problem data only*: mesh vertex coordinates and quad
connectivity, boundary and sensor points with their prescribed values, network
initialisations and the batched-instance mix.  It contains none of the method's
arithmetic (no quadrature, no test functions, no geometry maps, no loss).  Both
the FP64 oracle and the HIP library consume what it returns, so neither side
can influence the other's inputs.

Random numbers come from SplitMix64 (Steele, Lea and Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014): a 64-bit counter incremented by
the golden-ratio constant, then finalised by two xor-shift-multiply rounds.
Every named substream is keyed by the user seed and an FNV-1a hash of its name,
so adding a new stream never shifts an existing one.

Workload shapes follow the paper's experiments (Poisson on the unit square with
a manufactured sin-sin solution, Section 4.6; a large skewed-quad mesh standing
in for the Gmsh spur gear, Section 4.6.4; the constant-epsilon inverse problem,
Section 4.7.1; the hyperparameter sweep over N_elem, N_quad and N_test,
Section 4.8).  The gear mesh itself is not available, so an annulus O-grid with
a sinusoidal toothed outer rim and jittered interior nodes stands in for it.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Callable, List, Optional, Tuple

import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def _fnv1a64(name: str) -> int:
    h = 0xCBF29CE484222325
    for byte in name.encode("utf-8"):
        h ^= byte
        h = (h * 0x100000001B3) & 0xFFFFFFFFFFFFFFFF
    return h


def _mix(z: np.ndarray) -> np.ndarray:
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


def splitmix64(seed: int, name: str, n: int) -> np.ndarray:
    """n consecutive outputs of the SplitMix64 stream keyed by (seed, name)."""
    key = np.array([(int(seed) ^ _fnv1a64(name)) & 0xFFFFFFFFFFFFFFFF], dtype=np.uint64)
    start = _mix(key)[0]
    with np.errstate(over="ignore"):
        counters = start + _GOLDEN * (np.arange(1, n + 1, dtype=np.uint64))
    return _mix(counters)


def uniform01(seed: int, name: str, n: int) -> np.ndarray:
    """Uniform doubles in [0, 1) from the top 53 bits of the stream."""
    bits = splitmix64(seed, name, n) >> np.uint64(11)
    return bits.astype(np.float64) * (1.0 / 9007199254740992.0)


def uniform(seed: int, name: str, n: int, lo: float, hi: float) -> np.ndarray:
    return lo + (hi - lo) * uniform01(seed, name, n)


def normal(seed: int, name: str, n: int) -> np.ndarray:
    """Standard normals by the Box-Muller transform of two uniform streams."""
    u1 = uniform01(seed, name + "/bm1", n)
    u2 = uniform01(seed, name + "/bm2", n)
    u1 = np.maximum(u1, 1e-300)
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * math.pi * u2)


# ----------------------------------------------------------------------------
# meshes: vertex coordinates (float64 [n_nodes, 2]) and quads (int32 [n_elem, 4])
# vertex order per quad is counter-clockwise, matching the reference corners
# (-1,-1), (1,-1), (1,1), (-1,1) of the bilinear map in Appendix A.1.
# ----------------------------------------------------------------------------

@dataclass
class Mesh:
    xy: np.ndarray      # float64 [n_nodes, 2]
    quad: np.ndarray    # int32 [n_elem, 4]
    name: str = ""

    @property
    def n_elem(self) -> int:
        return int(self.quad.shape[0])

    @property
    def n_nodes(self) -> int:
        return int(self.xy.shape[0])


def square_mesh(mx: int, my: int, perturb: float = 0.0, seed: int = 0,
                x0: float = 0.0, x1: float = 1.0, y0: float = 0.0, y1: float = 1.0) -> Mesh:
    """Structured mx-by-my quad mesh of [x0,x1]x[y0,y1].

    Interior nodes move independently in x and y by U(-perturb*hx, perturb*hx)
    and U(-perturb*hy, perturb*hy); boundary nodes stay fixed.  With perturb
    below 0.25 every corner cross product stays positive, so each bilinear
    element remains convex and counter-clockwise.
    """
    hx = (x1 - x0) / mx
    hy = (y1 - y0) / my
    ii, jj = np.meshgrid(np.arange(mx + 1), np.arange(my + 1), indexing="xy")
    x = x0 + ii.astype(np.float64) * hx
    y = y0 + jj.astype(np.float64) * hy
    if perturb > 0.0:
        interior = (ii > 0) & (ii < mx) & (jj > 0) & (jj < my)
        nn = (mx + 1) * (my + 1)
        dx = uniform(seed, "mesh/dx", nn, -perturb * hx, perturb * hx).reshape(my + 1, mx + 1)
        dy = uniform(seed, "mesh/dy", nn, -perturb * hy, perturb * hy).reshape(my + 1, mx + 1)
        x = np.where(interior, x + dx, x)
        y = np.where(interior, y + dy, y)
    xy = np.stack([x.ravel(), y.ravel()], axis=1)
    node = lambda i, j: j * (mx + 1) + i  # noqa: E731
    quads = []
    for j in range(my):
        for i in range(mx):
            quads.append((node(i, j), node(i + 1, j), node(i + 1, j + 1), node(i, j + 1)))
    return Mesh(xy=xy, quad=np.asarray(quads, dtype=np.int32), name=f"square{mx}x{my}p{perturb}")


def gear_outer_radius(theta, teeth: int = 24, amp: float = 0.05):
    return 1.0 + amp * np.sin(teeth * theta)


def annulus_gear_mesh(n_theta: int = 400, n_r: int = 35, r_in: float = 0.5, teeth: int = 24,
                      amp: float = 0.05, jitter: float = 0.15, seed: int = 0) -> Mesh:
    """O-grid between the circle r = r_in and the toothed rim 1 + amp*sin(teeth*theta).

    Node (i, j) sits at angle 2*pi*i/n_theta on ring j of n_r+1 rings spaced
    linearly between the two curves.  Interior rings are jittered radially by
    U(-jitter, jitter) of the local ring spacing and tangentially by
    U(-jitter, jitter) of the local arc spacing, which skews every element.
    """
    th = 2.0 * math.pi * np.arange(n_theta) / n_theta
    rout = gear_outer_radius(th, teeth, amp)
    xy = np.zeros((n_theta * (n_r + 1), 2))
    nn = n_theta * (n_r + 1)
    jr = uniform(seed, "mesh/jr", nn, -jitter, jitter).reshape(n_theta, n_r + 1)
    jt = uniform(seed, "mesh/jt", nn, -jitter, jitter).reshape(n_theta, n_r + 1)
    dth = 2.0 * math.pi / n_theta
    for i in range(n_theta):
        dr = (rout[i] - r_in) / n_r
        for j in range(n_r + 1):
            r = r_in + dr * j
            t = th[i]
            if 0 < j < n_r:
                r = r + jr[i, j] * dr
                t = t + jt[i, j] * dth
            xy[i * (n_r + 1) + j] = (r * math.cos(t), r * math.sin(t))
    node = lambda i, j: (i % n_theta) * (n_r + 1) + j  # noqa: E731
    quads = [(node(i, j), node(i, j + 1), node(i + 1, j + 1), node(i + 1, j))
             for i in range(n_theta) for j in range(n_r)]
    return Mesh(xy=xy, quad=np.asarray(quads, dtype=np.int32), name=f"gear{n_theta}x{n_r}")


# ----------------------------------------------------------------------------
# manufactured solution u*(x,y) = sin(kx x) sin(ky y) (problem data: boundary and
# sensor values; the forcing is handed to both sides as the triple (amp, kx, ky)
# of f = amp*sin(kx x)*sin(ky y) and each side evaluates it itself).
# ----------------------------------------------------------------------------

def sinsin(xy: np.ndarray, kx: float, ky: float) -> np.ndarray:
    return np.sin(kx * xy[:, 0]) * np.sin(ky * xy[:, 1])


def square_boundary_points(n_d: int, x0=0.0, x1=1.0, y0=0.0, y1=1.0) -> np.ndarray:
    """n_d points, n_d/4 per side at cell midpoints t=(i+1/2)/(n_d/4): no corner duplicates."""
    if n_d % 4:
        raise ValueError("n_d must be a multiple of 4")
    m = n_d // 4
    t = (np.arange(m) + 0.5) / m
    bottom = np.stack([x0 + (x1 - x0) * t, np.full(m, y0)], 1)
    right = np.stack([np.full(m, x1), y0 + (y1 - y0) * t], 1)
    top = np.stack([x1 - (x1 - x0) * t, np.full(m, y1)], 1)
    left = np.stack([np.full(m, x0), y1 - (y1 - y0) * t], 1)
    return np.concatenate([bottom, right, top, left], 0)


def annulus_boundary_points(n_d: int, r_in=0.5, teeth=24, amp=0.05) -> np.ndarray:
    """Split n_d between the inner circle and the toothed rim by arc length; equispaced in angle."""
    tt = np.linspace(0.0, 2.0 * math.pi, 20001)
    ro = gear_outer_radius(tt, teeth, amp)
    dro = amp * teeth * np.cos(teeth * tt)
    len_out = float(np.trapezoid(np.sqrt(ro ** 2 + dro ** 2), tt))
    len_in = 2.0 * math.pi * r_in
    n_out = int(round(n_d * len_out / (len_out + len_in)))
    n_in = n_d - n_out
    ti = 2.0 * math.pi * (np.arange(n_in) + 0.5) / n_in
    to = 2.0 * math.pi * (np.arange(n_out) + 0.5) / n_out
    inner = np.stack([r_in * np.cos(ti), r_in * np.sin(ti)], 1)
    r = gear_outer_radius(to, teeth, amp)
    outer = np.stack([r * np.cos(to), r * np.sin(to)], 1)
    return np.concatenate([inner, outer], 0)


def disk_mesh(m: int, cx: float = 0.5, cy: float = 0.5, radius: float = 0.5) -> Mesh:
    """m-by-m quads of a disk: the structured grid of [-1,1]^2 pushed onto the unit disk by the smooth map
    (u, v) -> (u sqrt(1 - v^2/2), v sqrt(1 - u^2/2)), then scaled and shifted.  The map preserves orientation
    and keeps every element convex and counter-clockwise for the sizes used here."""
    sq = square_mesh(m, m, 0.0, 0, -1.0, 1.0, -1.0, 1.0)
    u, v = sq.xy[:, 0], sq.xy[:, 1]
    x = u * np.sqrt(1.0 - 0.5 * v * v)
    y = v * np.sqrt(1.0 - 0.5 * u * u)
    xy = np.stack([cx + radius * x, cy + radius * y], 1)
    return Mesh(xy=xy, quad=sq.quad, name=f"disk{m}")


def circle_points(n: int, cx: float = 0.5, cy: float = 0.5, radius: float = 0.5) -> np.ndarray:
    t = 2.0 * math.pi * (np.arange(n) + 0.5) / n
    return np.stack([cx + radius * np.cos(t), cy + radius * np.sin(t)], 1)


def disk_sensor_points(n_s: int, seed: int, cx: float = 0.5, cy: float = 0.5, radius: float = 0.5) -> np.ndarray:
    """Uniform in the disk: radius sqrt(U) r, angle 2 pi U (two named substreams)."""
    r = radius * np.sqrt(uniform(seed, "dsensors/r", n_s, 0.0, 1.0))
    t = uniform(seed, "dsensors/t", n_s, 0.0, 2.0 * math.pi)
    return np.stack([cx + r * np.cos(t), cy + r * np.sin(t)], 1)


def sensor_points(n_s: int, seed: int, x0=0.0, x1=1.0, y0=0.0, y1=1.0) -> np.ndarray:
    return np.stack([uniform(seed, "sensors/x", n_s, x0, x1),
                     uniform(seed, "sensors/y", n_s, y0, y1)], 1)


# ----------------------------------------------------------------------------
# network parameters: flat layout W1[H][2], b1[H], (W_l[H][H], b_l[H]) for
# l = 2..L, W_out[H], b_out.  Values are rounded to float32 so that the FP64
# oracle and the FP32 kernels see bit-identical parameters.
# ----------------------------------------------------------------------------

def n_params(width: int, n_hidden: int, heads: int = 1) -> int:
    """heads = 2: the output layer is W_out[2][H], b_out[2] (the second output is a diffusion field)."""
    return width * 2 + width + (n_hidden - 1) * (width * width + width) + heads * (width + 1)


def glorot_params(width: int, n_hidden: int, seed: int, bias_scale: float = 0.0,
                  name: str = "params", heads: int = 1) -> np.ndarray:
    """Glorot-uniform weights U(+-sqrt(6/(fan_in+fan_out))); biases U(+-bias_scale) (zero by default)."""
    parts = []
    shapes = [(width, 2)] + [(width, width)] * (n_hidden - 1) + [(heads, width)]
    for li, (fo, fi) in enumerate(shapes):
        bound = math.sqrt(6.0 / (fi + fo))
        w = uniform(seed, f"{name}/W{li}", fo * fi, -bound, bound)
        parts.append(w)
        nb = fo
        if bias_scale > 0.0:
            parts.append(uniform(seed, f"{name}/b{li}", nb, -bias_scale, bias_scale))
        else:
            parts.append(np.zeros(nb))
    theta = np.concatenate(parts)
    assert theta.size == n_params(width, n_hidden, heads)
    return theta.astype(np.float32).astype(np.float64)


# ----------------------------------------------------------------------------
# problem presets (the five workloads) and the batched mix
# ----------------------------------------------------------------------------

@dataclass
class Problem:
    name: str
    mesh: Mesh
    quad_order: int            # GLL points per direction n (N_quad = n^2)
    test_order: int            # test functions per direction N_t (N_test = N_t^2)
    f_amp: float               # forcing f = f_amp * sin(f_kx x) * sin(f_ky y)
    f_kx: float
    f_ky: float
    bnd_xy: np.ndarray
    bnd_g: np.ndarray
    sens_xy: np.ndarray = field(default_factory=lambda: np.zeros((0, 2)))
    sens_u: np.ndarray = field(default_factory=lambda: np.zeros(0))
    tau: float = 10.0
    gamma: float = 0.0
    width: int = 30
    n_hidden: int = 3
    eps_init: Optional[float] = None   # trainable diffusion coefficient (inverse problem)
    eps_true: Optional[float] = None
    seed: int = 0
    # convection-diffusion -diff Lap u + conv . grad u = f (forward problem: constants, not trained)
    diff: float = 1.0
    conv: Tuple[float, float] = (0.0, 0.0)
    f_fn: Optional[Callable[[float, float], float]] = None  # forcing as a function of (x, y), else sin-sin
    # heads = 2: the network also outputs the diffusion coefficient eps(x, y) (space-dependent inverse problem)
    heads: int = 1

    @property
    def n_elem(self) -> int:
        return self.mesh.n_elem

    @property
    def n_points(self) -> int:
        return self.mesh.n_elem * self.quad_order ** 2

    def params(self, seed: Optional[int] = None, bias_scale: float = 0.0) -> np.ndarray:
        s = self.seed if seed is None else seed
        return glorot_params(self.width, self.n_hidden, s, bias_scale, name=f"params/{self.name}", heads=self.heads)


def poisson_sinsin_square(name: str, m: int, n: int, nt: int, k: int, n_d: int,
                          perturb: float, seed: int = 0, tau: float = 10.0) -> Problem:
    kp = k * math.pi
    mesh = square_mesh(m, m, perturb, seed)
    bxy = square_boundary_points(n_d)
    return Problem(name=name, mesh=mesh, quad_order=n, test_order=nt,
                   f_amp=2.0 * kp * kp, f_kx=kp, f_ky=kp,
                   bnd_xy=bxy, bnd_g=sinsin(bxy, kp, kp), tau=tau, seed=seed)


def config_c1(seed: int = 0) -> Problem:
    """2x2 uniform mesh, 5x5 GLL points, 5x5 test functions, k=2, 400 boundary points."""
    return poisson_sinsin_square("c1", 2, 5, 5, 2, 400, 0.0, seed)


def config_c2(seed: int = 0) -> Problem:
    """32x32 mesh with interior nodes jittered by +-20% h, 10x10 GLL, 5x5 tests, k=8, 1600 boundary points."""
    return poisson_sinsin_square("c2", 32, 10, 5, 8, 1600, 0.2, seed)


def config_c3(seed: int = 0) -> Problem:
    """Toothed-annulus O-grid, 400x35 = 14,000 skewed quads, 5x5 GLL, 5x5 tests, u*=sin4pix sin4piy."""
    kp = 4.0 * math.pi
    mesh = annulus_gear_mesh(seed=seed)
    bxy = annulus_boundary_points(4000)
    return Problem(name="c3", mesh=mesh, quad_order=5, test_order=5,
                   f_amp=2.0 * kp * kp, f_kx=kp, f_ky=kp,
                   bnd_xy=bxy, bnd_g=sinsin(bxy, kp, kp), seed=seed)


def config_c4(seed: int = 0) -> Problem:
    """Inverse problem -eps*Lap u = f, eps_true 0.3 (init 2.0), 64x64 jittered mesh, 10x10 GLL, 1000 sensors."""
    kp = 2.0 * math.pi
    eps_true = 0.3
    mesh = square_mesh(64, 64, 0.2, seed)
    bxy = square_boundary_points(1600)
    sxy = sensor_points(1000, seed)
    su = sinsin(sxy, kp, kp) + 0.01 * normal(seed, "sensors/noise", 1000)
    return Problem(name="c4", mesh=mesh, quad_order=10, test_order=5,
                   f_amp=eps_true * 2.0 * kp * kp, f_kx=kp, f_ky=kp,
                   bnd_xy=bxy, bnd_g=sinsin(bxy, kp, kp), sens_xy=sxy, sens_u=su,
                   tau=10.0, gamma=10.0, eps_init=2.0, eps_true=eps_true, seed=seed)


def gear_forcing(x: float, y: float) -> float:
    """Forcing of the convection-diffusion gear problem: 50 sin x + cos x."""
    return 50.0 * math.sin(x) + math.cos(x)


def config_gear_cd(seed: int = 0) -> Problem:
    """Convection-diffusion -Lap u + (0.1, 0) . grad u = 50 sin x + cos x with u = 0 on the boundary (the
    paper's gear experiment) on the toothed-annulus stand-in for its gear mesh (400x35 = 14,000 quads), 5x5 GLL,
    4x4 test functions, 6,096 boundary points."""
    mesh = annulus_gear_mesh(seed=seed)
    bxy = annulus_boundary_points(6096)
    return Problem(name="gear_cd", mesh=mesh, quad_order=5, test_order=4, f_amp=0.0, f_kx=0.0, f_ky=0.0,
                   bnd_xy=bxy, bnd_g=np.zeros(len(bxy)), seed=seed, diff=1.0, conv=(0.1, 0.0), f_fn=gear_forcing)


class VarDiffManufactured:
    """Manufactured data of -div(eps grad u) + b . grad u = f with eps(x, y) = 0.5 (sin x + cos y) (the
    coefficient field of the paper's space-dependent inverse problem), b = (1, 0) and
    u = sin(k x) sin(k y): f = -(eps Lap u + eps_x u_x + eps_y u_y) + b . grad u."""

    def __init__(self, k: float = 2.0 * math.pi, b=(1.0, 0.0)):
        self.k, self.b = k, b

    def u(self, x, y):
        return np.sin(self.k * x) * np.sin(self.k * y)

    def eps(self, x, y):
        return 0.5 * (np.sin(x) + np.cos(y))

    def f(self, x: float, y: float) -> float:
        k = self.k
        u = math.sin(k * x) * math.sin(k * y)
        ux, uy = k * math.cos(k * x) * math.sin(k * y), k * math.sin(k * x) * math.cos(k * y)
        e, ex, ey = 0.5 * (math.sin(x) + math.cos(y)), 0.5 * math.cos(x), -0.5 * math.sin(y)
        return -(e * (-2.0 * k * k * u) + ex * ux + ey * uy) + self.b[0] * ux + self.b[1] * uy


def config_disk_vareps(seed: int = 0, m: int = 32) -> Problem:
    """Space-dependent diffusion inverse problem on a disk (centre (0.5, 0.5), radius 0.5) of m x m = 1,024
    quads: the network outputs u and eps(x, y); 10x10 GLL, 5x5 tests, b = (1, 0), manufactured u and eps,
    1,600 boundary points and 1,000 sensors of u, tau = gamma = 10."""
    man = VarDiffManufactured()
    mesh = disk_mesh(m)
    bxy = circle_points(1600)
    sxy = disk_sensor_points(1000, seed)
    return Problem(name="disk_vareps", mesh=mesh, quad_order=10, test_order=5, f_amp=0.0, f_kx=0.0, f_ky=0.0,
                   bnd_xy=bxy, bnd_g=man.u(bxy[:, 0], bxy[:, 1]), sens_xy=sxy, sens_u=man.u(sxy[:, 0], sxy[:, 1]),
                   tau=10.0, gamma=10.0, seed=seed, conv=(1.0, 0.0), f_fn=man.f, heads=2)


def config_probe(seed: int = 0) -> Problem:
    """The C4 mesh with 20x20 test functions (the paper's largest p-refinement): G-stream dominated."""
    p = poisson_sinsin_square("probe", 64, 10, 20, 2, 1600, 0.2, seed)
    return p


def batched_instances(n_inst: int = 64, seed: int = 0, lo: int = 256, hi: int = 16384,
                      n_d: int = 400) -> List[Problem]:
    """Independent Poisson instances: element counts log-uniform in [lo, hi], n in {4,6,10},
    N_t in {3,5}, frequency k in 1..16, each with its own network seed."""
    u_n = uniform01(seed, "batch/nelem", n_inst)
    u_q = uniform01(seed, "batch/quad", n_inst)
    u_t = uniform01(seed, "batch/test", n_inst)
    u_k = uniform01(seed, "batch/freq", n_inst)
    out = []
    for i in range(n_inst):
        ne = math.exp(math.log(lo) + (math.log(hi) - math.log(lo)) * u_n[i])
        mx = max(1, int(round(math.sqrt(ne))))
        my = max(1, int(round(ne / mx)))
        n = (4, 6, 10)[min(2, int(u_q[i] * 3))]
        nt = (3, 5)[min(1, int(u_t[i] * 2))]
        k = 1 + min(15, int(u_k[i] * 16))
        kp = k * math.pi
        mesh = square_mesh(mx, my, 0.2, seed * 1000003 + i)
        bxy = square_boundary_points(n_d)
        out.append(Problem(name=f"b{i}", mesh=mesh, quad_order=n, test_order=nt,
                           f_amp=2.0 * kp * kp, f_kx=kp, f_ky=kp, bnd_xy=bxy,
                           bnd_g=sinsin(bxy, kp, kp), seed=seed * 1000003 + i))
    return out


class InverseConstManufactured:
    """Data of the constant-diffusion inverse problem of Sec. 4.7.1 on (-1, 1)^2: the solution
    u = 10 sin(x) tanh(x) exp(-eps x^2), a function of x alone, with eps = 0.3, and the forcing
    f = -eps u''(x) that makes it exact (u'' by the product rule over sin, tanh and the Gaussian)."""

    def __init__(self, eps: float = 0.3):
        self.eps = eps

    def u(self, x, y):
        return 10.0 * np.sin(x) * np.tanh(x) * np.exp(-self.eps * x * x)

    def f(self, x, y):
        a = self.eps
        s, c, t = np.sin(x), np.cos(x), np.tanh(x)
        dt = 1.0 - t * t
        ddt = -2.0 * t * dt
        r = np.exp(-a * x * x)
        dr = -2.0 * a * x * r
        ddr = (4.0 * a * a * x * x - 2.0 * a) * r
        upp = 10.0 * (-s * t * r + s * ddt * r + s * t * ddr + 2.0 * (c * dt * r + c * t * dr + s * dt * dr))
        return -a * upp


def config_inverse_const(seed: int = 0) -> Problem:
    """The inverse problem of Sec. 4.7.1 at the paper's sizes: -eps Lap u = f on (-1, 1)^2, 2x2 elements,
    40x40 GLL points an element, 5x5 test functions, 50 sensors of the exact u, eps trainable (init 2.0,
    true 0.3), 400 boundary points, 30x3 network."""
    man = InverseConstManufactured(0.3)
    mesh = square_mesh(2, 2, 0.0, seed, -1.0, 1.0, -1.0, 1.0)
    bxy = square_boundary_points(400, -1.0, 1.0, -1.0, 1.0)
    sxy = uniform(seed, "inverse_const/sensors", 100, -1.0, 1.0).reshape(50, 2)
    return Problem(name="inverse_const", mesh=mesh, quad_order=40, test_order=5, f_amp=0.0, f_kx=0.0, f_ky=0.0,
                   bnd_xy=bxy, bnd_g=man.u(bxy[:, 0], bxy[:, 1]), sens_xy=sxy, sens_u=man.u(sxy[:, 0], sxy[:, 1]),
                   tau=10.0, gamma=10.0, eps_init=2.0, eps_true=man.eps, seed=seed, f_fn=man.f)


def config_p_refine(seed: int = 0) -> Problem:
    """The p-refinement study of Sec. 4.1 at its largest test space: one element (the unit square), 80x80 GLL
    points, 20x20 test functions, u* = sin(4 pi x) sin(4 pi y), 400 boundary points."""
    return poisson_sinsin_square("p_refine", 1, 80, 20, 4, 400, 0.0, seed)


def config_h_refine(seed: int = 0) -> Problem:
    """The h-refinement study of Sec. 4.1 at its finest mesh: 8x8 uniform elements of the unit square, 80x80
    GLL points and 5x5 test functions each (409,600 points), u* = sin(4 pi x) sin(4 pi y), 1,600 boundary
    points."""
    return poisson_sinsin_square("h_refine", 8, 80, 5, 4, 1600, 0.0, seed)


CONFIGS = {"c1": config_c1, "c2": config_c2, "c3": config_c3, "c4": config_c4, "probe": config_probe,
           "gear_cd": config_gear_cd, "disk_vareps": config_disk_vareps, "inverse_const": config_inverse_const,
           "p_refine": config_p_refine, "h_refine": config_h_refine}
