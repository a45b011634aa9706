"""Pins of the FP64 oracle against facts that do not come from the oracle itself.

Each test checks one piece of the oracle against a closed form, a textbook or
library routine, an invariant of the weak form, or finite differences, chosen so
that a dropped term, a wrong sign, a swapped index or a transposed operand in
the oracle fails at least one of them.
"""
import ast
import math
import operator
import os

import numpy as np
import numpy.polynomial.legendre as npleg
import pytest

import vpinn_inputs as gen

HERE = os.path.dirname(os.path.abspath(__file__))


# ----------------------------------------------------------------------------- helpers

_OPS = {ast.Add: operator.add, ast.Sub: operator.sub, ast.Mult: operator.mul,
        ast.Div: operator.truediv, ast.USub: operator.neg}


def _eval_expr(s):
    """Evaluate a closed-form expression built from numbers, + - * / and sqrt."""
    def ev(node):
        if isinstance(node, ast.Expression):
            return ev(node.body)
        if isinstance(node, ast.Constant):
            return float(node.value)
        if isinstance(node, ast.BinOp):
            return _OPS[type(node.op)](ev(node.left), ev(node.right))
        if isinstance(node, ast.UnaryOp):
            return _OPS[type(node.op)](ev(node.operand))
        if isinstance(node, ast.Call) and node.func.id == "sqrt":
            return math.sqrt(ev(node.args[0]))
        raise ValueError(s)
    return ev(ast.parse(s, mode="eval"))


def _gll_golden():
    rows = {}
    with open(os.path.join(HERE, "golden", "gll_closed_forms.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            n, x, w = [c.strip() for c in line.split("|")]
            rows.setdefault(int(n), []).append((_eval_expr(x), _eval_expr(w)))
    return rows


def _numpy_gll(n):
    """GLL nodes from numpy's Legendre routines: -1, +1 and the roots of P'_{n-1}."""
    c = np.zeros(n)
    c[n - 1] = 1.0
    inner = np.sort(npleg.legroots(npleg.legder(c)).real)
    x = np.concatenate([[-1.0], inner, [1.0]])
    w = 2.0 / (n * (n - 1) * npleg.legval(x, c) ** 2)
    return x, w


def _np_phi(r, t):
    c = np.zeros(r + 2)
    c[r + 1] += 1.0
    c[r - 1] -= 1.0
    return npleg.legval(t, c), npleg.legval(t, npleg.legder(c))


def _skewed_mesh(m=3, seed=7, perturb=0.22):
    return gen.square_mesh(m, m, perturb, seed)


def _shoelace(verts):
    x, y = verts[:, 0], verts[:, 1]
    return 0.5 * np.sum(x * np.roll(y, -1) - np.roll(x, -1) * y)


# ----------------------------------------------------------------------------- quadrature

def test_gll_matches_closed_forms(oracle):
    for n, rows in _gll_golden().items():
        x, w = oracle.gll(n)
        xs, ws = zip(*rows)
        np.testing.assert_allclose(x, xs, rtol=0, atol=2e-15)
        np.testing.assert_allclose(w, ws, rtol=0, atol=2e-15)


@pytest.mark.parametrize("n", range(2, 21))
def test_gll_degree_of_exactness(oracle, n):
    """Exact for x^m, m <= 2n-3; at degree 2n-2 it fails by a known amount, which pins n."""
    x, w = oracle.gll(n)
    assert abs(w.sum() - 2.0) < 1e-13
    for m in range(0, 2 * n - 2):
        exact = 2.0 / (m + 1) if m % 2 == 0 else 0.0
        assert abs(np.dot(w, x ** m) - exact) < 2e-13, (n, m)
    # degree 2n-2: the discrete norm of P_{n-1} is 2/(n-1), not the exact 2/(2n-1)
    pn = npleg.legval(x, np.eye(n)[n - 1])
    assert abs(np.dot(w, pn * pn) - 2.0 / (n - 1)) < 1e-12
    assert abs(2.0 / (n - 1) - 2.0 / (2 * n - 1)) > 0.05


@pytest.mark.parametrize("n", [3, 7, 10, 16, 25, 40, 64, 65, 80, 100])
def test_gll_matches_numpy_legendre_roots(oracle, n):
    x, w = oracle.gll(n)
    xn, wn = _numpy_gll(n)
    np.testing.assert_allclose(x, xn, atol=1e-13)
    np.testing.assert_allclose(w, wn, rtol=1e-11)


def test_legendre_matches_numpy(oracle):
    ts = np.linspace(-1, 1, 17)
    for m in range(0, 26):
        c = np.zeros(m + 1)
        c[m] = 1.0
        dc = npleg.legder(c)
        for t in ts:
            assert abs(oracle.legendre(m, t) - npleg.legval(t, c)) < 1e-12
            assert abs(oracle.legendre_deriv(m, t) - npleg.legval(t, dc)) < 1e-9 * max(1, m * m)


# ----------------------------------------------------------------------------- test functions

@pytest.mark.parametrize("r", range(1, 21))
def test_test_functions(oracle, r):
    """phi_r = P_{r+1} - P_{r-1} vanishes at +-1; phi_r' = (2r+1) P_r; central FD agrees."""
    for t in (-1.0, 1.0):
        assert abs(oracle.test_fn(r, t)[0]) < 1e-13
    for t in np.linspace(-0.95, 0.95, 9):
        p, d = oracle.test_fn(r, t)
        pn, dn = _np_phi(r, t)
        assert abs(p - pn) < 1e-12
        assert abs(d - (2 * r + 1) * npleg.legval(t, np.eye(r + 1)[r])) < 1e-10 * r
        h = 1e-6
        fd = (oracle.test_fn(r, t + h)[0] - oracle.test_fn(r, t - h)[0]) / (2 * h)
        assert abs(d - fd) < 1e-6 * (r + 1) ** 2


# ----------------------------------------------------------------------------- geometry

def test_bilinear_map_hits_vertices_and_jacobian_is_derivative(oracle):
    verts = np.array([[0.1, 0.05], [0.42, 0.0], [0.5, 0.37], [0.03, 0.31]])
    ref = [(-1, -1), (1, -1), (1, 1), (-1, 1)]
    for (xi, eta), v in zip(ref, verts):
        np.testing.assert_allclose(oracle.map_point(verts, xi, eta), v, atol=1e-15)
    h = 1e-6
    for xi, eta in [(-0.3, 0.7), (0.9, -0.2), (0.0, 0.0)]:
        J, Ji, D = oracle.jacobian(verts, xi, eta)
        xp = np.array(oracle.map_point(verts, xi + h, eta))
        xm = np.array(oracle.map_point(verts, xi - h, eta))
        yp = np.array(oracle.map_point(verts, xi, eta + h))
        ym = np.array(oracle.map_point(verts, xi, eta - h))
        dxi = (xp - xm) / (2 * h)    # (dx/dxi, dy/dxi)
        deta = (yp - ym) / (2 * h)   # (dx/deta, dy/deta)
        np.testing.assert_allclose(J[0], dxi, atol=1e-9)
        np.testing.assert_allclose(J[1], deta, atol=1e-9)
        np.testing.assert_allclose(J @ Ji, np.eye(2), atol=1e-13)
        assert abs(D - np.linalg.det(J)) < 1e-15
        assert D > 0


def test_printed_inverse_would_be_wrong(oracle):
    """The inverse printed in Appendix A.1 swaps xi and eta in its second row; ours is the true inverse."""
    verts = np.array([[0.0, 0.0], [0.1, 0.01], [0.13, 0.12], [-0.02, 0.09]])
    xi, eta = 0.6, -0.8
    J, Ji, D = oracle.jacobian(verts, xi, eta)
    xc = np.array([verts[:, 0].sum(), -verts[0, 0] + verts[1, 0] + verts[2, 0] - verts[3, 0],
                   -verts[0, 0] - verts[1, 0] + verts[2, 0] + verts[3, 0],
                   verts[0, 0] - verts[1, 0] + verts[2, 0] - verts[3, 0]]) / 4
    printed_row2 = np.array([-(xc[2] + xc[3] * eta), xc[1] + xc[3] * xi]) / D
    assert np.max(np.abs(printed_row2 - Ji[1])) > 1e-3
    np.testing.assert_allclose(J @ Ji, np.eye(2), atol=1e-13)


@pytest.mark.parametrize("n", [2, 3, 5])
def test_quadrature_area_equals_shoelace(oracle, n):
    """sum_q w_q det J = element area exactly (det J is affine); the mesh sums to the domain area."""
    x, w = oracle.gll(n)
    for mesh, total in [(_skewed_mesh(4), 1.0), (gen.annulus_gear_mesh(40, 5, seed=3), None)]:
        s_all = 0.0
        for quad in mesh.quad:
            verts = mesh.xy[quad]
            s = sum(w[i] * w[j] * oracle.jacobian(verts, x[i], x[j])[2] for i in range(n) for j in range(n))
            assert abs(s - _shoelace(verts)) < 1e-14
            s_all += s
        if total is None:
            ring_out = mesh.xy[5::6]
            ring_in = mesh.xy[0::6]
            total = _shoelace(ring_out) - _shoelace(ring_in)
        assert abs(s_all - total) < 1e-12


def test_quadrature_points_are_mapped_gll_nodes(oracle):
    mesh = _skewed_mesh(2)
    asm = oracle.assemble(mesh.xy, mesh.quad, 4, 2, 1.0, 1.0, 1.0)
    x, _ = oracle.gll(4)
    for e, quad in enumerate(mesh.quad):
        for j in range(4):
            for i in range(4):
                np.testing.assert_allclose(asm.X[e, j * 4 + i], oracle.map_point(mesh.xy[quad], x[i], x[j]),
                                           atol=1e-15)


def test_rejects_clockwise_and_bad_index(oracle):
    mesh = gen.square_mesh(2, 2)
    cw = mesh.quad.copy()
    cw[3] = cw[3][::-1]
    with pytest.raises(oracle.OracleError) as ei:
        oracle.assemble(mesh.xy, cw, 3, 2, 1, 1, 1)
    assert ei.value.elem == 3
    bad = mesh.quad.copy()
    bad[1, 2] = 99
    with pytest.raises(oracle.OracleError) as ei:
        oracle.assemble(mesh.xy, bad, 3, 2, 1, 1, 1)
    assert ei.value.elem == 1


# ----------------------------------------------------------------------------- G and F

@pytest.mark.parametrize("n,nt", [(5, 5), (4, 3), (10, 5), (6, 2)])
def test_patch_test_sum_of_G_vanishes(oracle, n, nt):
    """int_K grad v_k = boundary integral of v_k n = 0 since v_k vanishes on the element boundary;
    GLL integrates it exactly when 2n-3 >= N_t+1."""
    mesh = _skewed_mesh(3)
    asm = oracle.assemble(mesh.xy, mesh.quad, n, nt, 1.0, 1.0, 1.0)
    assert 2 * n - 3 >= nt + 1
    scale = np.abs(asm.Gx).max()
    assert np.abs(asm.Gx.sum(axis=2)).max() < 1e-13 * scale * n * n
    assert np.abs(asm.Gy.sum(axis=2)).max() < 1e-13 * scale * n * n


def test_patch_test_fails_when_underintegrated(oracle):
    mesh = _skewed_mesh(3)
    asm = oracle.assemble(mesh.xy, mesh.quad, 4, 5, 1.0, 1.0, 1.0)
    assert np.abs(asm.Gx.sum(axis=2)).max() > 1e-6


@pytest.mark.parametrize("n,exact", [(6, True), (8, True), (10, True), (5, False)])
def test_manufactured_cubic_residual_vanishes(oracle, n, exact):
    """u = x^3 + x y^2 + 2y, f = -Lap u = -8x: the weak residual is exactly zero (v_k = 0 on the
    element boundary) and GLL integrates it exactly when 2n-3 >= N_t + 3 (N_t = 5)."""
    mesh = _skewed_mesh(3, seed=11)
    asm = oracle.assemble(mesh.xy, mesh.quad, n, 5, f_callable=lambda x, y: -8.0 * x)
    X = asm.X
    ux = 3 * X[..., 0] ** 2 + X[..., 1] ** 2
    uy = 2 * X[..., 0] * X[..., 1] + 2.0
    R = oracle.residual(asm, ux, uy)
    scale = np.abs(asm.F).max() + np.abs(asm.Gx).max()
    if exact:
        assert np.abs(R).max() < 1e-13 * scale
    else:
        assert np.abs(R).max() > 1e-8 * scale


def test_sinsin_residual_converges_spectrally(oracle):
    """Plugging the exact gradient of u* = sin(8 pi x) sin(8 pi y) into the contraction: R -> 0 fast in n."""
    kp = 8 * math.pi
    mesh = gen.square_mesh(10, 10, 0.2, seed=5)
    errs = []
    for n in (5, 10, 15):
        asm = oracle.assemble(mesh.xy, mesh.quad, n, 5, 2 * kp * kp, kp, kp)
        X = asm.X
        ux = kp * np.cos(kp * X[..., 0]) * np.sin(kp * X[..., 1])
        uy = kp * np.sin(kp * X[..., 0]) * np.cos(kp * X[..., 1])
        errs.append(np.abs(oracle.residual(asm, ux, uy)).max() / np.abs(asm.F).max())
    assert errs[0] > 10 * errs[1] > 100 * errs[2]
    assert errs[2] < 1e-9


@pytest.mark.parametrize("n,nt", [(5, 5), (10, 3)])
def test_uniform_mesh_reduces_to_reference_premultiplier(oracle, n, nt):
    """On an axis-aligned mesh of h x h squares the Jacobian is constant and every element's G equals
    w_q (h/2) phi'_r(xi) phi_s(eta) (the single reference premultiplier of Algorithm 2); with f = 1,
    F[e, k] = element area for k = (1,1) and 0 otherwise.  Built here from numpy's Legendre routines."""
    m = 4
    h = 1.0 / m
    mesh = gen.square_mesh(m, m)
    asm = oracle.assemble(mesh.xy, mesh.quad, n, nt, f_callable=lambda x, y: 1.0)
    xg, wg = _numpy_gll(n)
    Gx_ref = np.zeros((nt * nt, n * n))
    Gy_ref = np.zeros((nt * nt, n * n))
    for s in range(1, nt + 1):
        for r in range(1, nt + 1):
            k = (s - 1) * nt + (r - 1)
            for j in range(n):
                for i in range(n):
                    pr, dpr = _np_phi(r, xg[i])
                    ps, dps = _np_phi(s, xg[j])
                    Gx_ref[k, j * n + i] = wg[i] * wg[j] * (h / 2) * dpr * ps
                    Gy_ref[k, j * n + i] = wg[i] * wg[j] * (h / 2) * pr * dps
    for e in range(mesh.n_elem):
        np.testing.assert_allclose(asm.Gx[e], Gx_ref, atol=1e-14)
        np.testing.assert_allclose(asm.Gy[e], Gy_ref, atol=1e-14)
    F_ref = np.zeros(nt * nt)
    F_ref[0] = h * h
    np.testing.assert_allclose(asm.F, np.tile(F_ref, (mesh.n_elem, 1)), atol=1e-14)


def test_forcing_of_constant_on_skewed_mesh_is_element_area(oracle):
    """With f = 1, F[e, (1,1)] = int_K phi_1(xi) phi_1(eta) = 4 det J(0,0) = area of K (det J affine)."""
    mesh = _skewed_mesh(4, seed=3)
    asm = oracle.assemble(mesh.xy, mesh.quad, 4, 3, f_callable=lambda x, y: 1.0)
    for e, quad in enumerate(mesh.quad):
        assert abs(asm.F[e, 0] - _shoelace(mesh.xy[quad])) < 1e-14


# ----------------------------------------------------------------------------- network

def test_single_neuron_network_closed_form(oracle):
    theta = np.array([0.7, -1.3, 0.2, 1.9, -0.4])   # W1 = [0.7, -1.3], b1 = 0.2, Wo = 1.9, bo = -0.4
    xy = np.array([[0.3, 0.8], [-0.5, 0.1]])
    u, ux, uy = oracle.mlp_eval(theta, 1, 1, xy)
    for p in range(2):
        z = 0.7 * xy[p, 0] - 1.3 * xy[p, 1] + 0.2
        s = 1 - math.tanh(z) ** 2
        assert abs(u[p] - (1.9 * math.tanh(z) - 0.4)) < 1e-15
        assert abs(ux[p] - 1.9 * s * 0.7) < 1e-15
        assert abs(uy[p] + 1.9 * s * 1.3) < 1e-15


@pytest.mark.parametrize("H,L", [(3, 1), (4, 2), (30, 3), (5, 4)])
def test_network_tangents_match_finite_differences(oracle, H, L):
    theta = gen.glorot_params(H, L, seed=H * 10 + L, bias_scale=0.3)
    xy = gen.uniform(1, "fdpts", 16, -1, 1).reshape(8, 2)
    u, ux, uy = oracle.mlp_eval(theta, H, L, xy)
    h = 1e-5
    up, _, _ = oracle.mlp_eval(theta, H, L, xy + [h, 0])
    um, _, _ = oracle.mlp_eval(theta, H, L, xy - [h, 0])
    np.testing.assert_allclose(ux, (up - um) / (2 * h), atol=1e-8)
    up, _, _ = oracle.mlp_eval(theta, H, L, xy + [0, h])
    um, _, _ = oracle.mlp_eval(theta, H, L, xy - [0, h])
    np.testing.assert_allclose(uy, (up - um) / (2 * h), atol=1e-8)


@pytest.mark.parametrize("H,L", [(3, 1), (4, 3), (6, 2)])
def test_network_vjp_matches_finite_differences(oracle, H, L):
    theta = gen.glorot_params(H, L, seed=3, bias_scale=0.5)
    xy = gen.uniform(2, "vjp", 10, -1, 1).reshape(5, 2)
    ub, uxb, uyb = (gen.uniform(2, f"c{i}", 5, -1, 1) for i in range(3))
    g = oracle.mlp_vjp(theta, H, L, xy, ub, uxb, uyb)

    def J(th):
        u, ux, uy = oracle.mlp_eval(th, H, L, xy)
        return np.dot(ub, u) + np.dot(uxb, ux) + np.dot(uyb, uy)

    h = 1e-6
    fd = np.array([(J(theta + h * e) - J(theta - h * e)) / (2 * h) for e in np.eye(theta.size)])
    np.testing.assert_allclose(g, fd, rtol=1e-6, atol=1e-9)


# ----------------------------------------------------------------------------- loss and gradient

def _tiny_problem():
    mesh = gen.square_mesh(2, 1, 0.2, seed=4)
    asm = None
    return mesh, asm


def test_zero_network_gives_closed_form_loss(oracle):
    """All weights zero and b_out = c: u = c, grad u = 0, so R = -F exactly, L_v = c_v sum F^2,
    L_b = mean (c-g)^2, L_s = mean (c-d)^2 and dL/db_out = 2 tau mean(c-g) + 2 gamma mean(c-d)."""
    p = gen.config_c1()
    asm = oracle.assemble_problem(p)
    H, L = 30, 3
    theta = np.zeros(gen.n_params(H, L))
    c = 0.37
    theta[-1] = c
    sxy = gen.sensor_points(7, 1)
    su = gen.uniform(1, "su", 7, -1, 1)
    tau, gamma = 3.0, 2.0
    r = oracle.loss_grad(asm, theta, H, L, p.bnd_xy, p.bnd_g, sxy, su, tau=tau, gamma=gamma, want_R=True)
    np.testing.assert_array_equal(r.R, -asm.F)
    cv = 1.0 / 25
    assert abs(r.loss[1] - cv * np.sum(asm.F ** 2)) < 1e-12 * r.loss[1]
    assert abs(r.loss[2] - np.mean((c - p.bnd_g) ** 2)) < 1e-15
    assert abs(r.loss[3] - np.mean((c - su) ** 2)) < 1e-15
    assert abs(r.loss[0] - (r.loss[1] + tau * r.loss[2] + gamma * r.loss[3])) < 1e-12
    gb = 2 * tau * np.mean(c - p.bnd_g) + 2 * gamma * np.mean(c - su)
    assert abs(r.grad[-1] - gb) < 1e-13
    # with every weight zero, dL/dW_out = 0 (the last hidden layer outputs tanh(0) = 0)
    np.testing.assert_array_equal(r.grad[-31:-1], 0.0)


def test_loss_normalisations(oracle):
    """Algorithm 3 (mean over N_test, sum over elements) vs the Section 2.3 equation (1/N_elem)."""
    p = gen.config_c1()
    asm = oracle.assemble_problem(p)
    th = p.params()
    a = oracle.problem_loss_grad(p, asm, th, loss_norm=0)
    b = oracle.problem_loss_grad(p, asm, th, loss_norm=1)
    assert abs(a.loss[1] * 25 / 4 - b.loss[1]) < 1e-12 * b.loss[1]
    assert abs(a.loss[2] - b.loss[2]) < 1e-15


@pytest.mark.parametrize("H,L,eps", [(3, 2, 1.0), (4, 1, 1.7), (2, 3, 0.6)])
def test_loss_gradient_matches_finite_differences(oracle, H, L, eps):
    """dL/dtheta and dL/deps against central differences of the oracle's own loss (FP64)."""
    mesh = gen.square_mesh(2, 1, 0.2, seed=4)
    asm = oracle.assemble(mesh.xy, mesh.quad, 3, 2, 5.0, 2.0, 3.0)
    theta = gen.glorot_params(H, L, seed=9, bias_scale=0.4)
    bxy = gen.square_boundary_points(8)
    bg = gen.uniform(3, "bg", 8, -0.5, 0.5)
    sxy = gen.sensor_points(5, 2)
    su = gen.uniform(3, "su", 5, -0.5, 0.5)
    kw = dict(bnd_xy=bxy, bnd_g=bg, sens_xy=sxy, sens_u=su, tau=2.0, gamma=3.0)
    r = oracle.loss_grad(asm, theta, H, L, eps=eps, **kw)

    def f(th, ep):
        return oracle.loss_grad(asm, th, H, L, eps=ep, want_grad=False, **kw).loss[0]

    h = 1e-6
    fd = np.array([(f(theta + h * e, eps) - f(theta - h * e, eps)) / (2 * h) for e in np.eye(theta.size)])
    rel = np.linalg.norm(r.grad - fd) / np.linalg.norm(fd)
    assert rel < 1e-6, rel
    fde = (f(theta, eps + h) - f(theta, eps - h)) / (2 * h)
    assert abs(r.grad_eps - fde) < 1e-6 * abs(fde)


def test_c1_gradient_matches_finite_differences_sampled(oracle):
    """The full 2->30->30->30->1 network on the first workload: 40 sampled parameters by central FD."""
    p = gen.config_c1()
    asm = oracle.assemble_problem(p)
    th = p.params(bias_scale=0.1)
    r = oracle.problem_loss_grad(p, asm, th)
    idx = np.unique((gen.uniform01(0, "fdidx", 40) * th.size).astype(int))
    h = 1e-6
    for i in idx:
        e = np.zeros_like(th)
        e[i] = h
        fd = (oracle.problem_loss_grad(p, asm, th + e, want_grad=False).loss[0]
              - oracle.problem_loss_grad(p, asm, th - e, want_grad=False).loss[0]) / (2 * h)
        assert abs(r.grad[i] - fd) < 1e-6 * max(1.0, abs(fd)), (i, r.grad[i], fd)


# ----------------------------------------------------------------------------- Adam

def test_adam_first_step_is_signed_lr(oracle):
    """After one step m_hat = g and v_hat = g^2, so the update is -lr g / (|g| + eps)."""
    g = np.array([0.3, -2.0, 1e-9, 0.0, 5e4])
    th = np.array([1.0, 2.0, 3.0, 4.0, 5.0])
    m = np.zeros(5)
    v = np.zeros(5)
    t0 = th.copy()
    oracle.adam(th, g, m, v, 1, lr=1e-3, eps=1e-8)
    np.testing.assert_allclose(th - t0, -1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-10, atol=1e-20)


def test_adam_constant_gradient_keeps_step(oracle):
    """With a constant gradient the bias-corrected moments stay g and g^2: every step moves lr*sign(g)."""
    g = np.array([0.5, -0.25])
    th = np.zeros(2)
    m = np.zeros(2)
    v = np.zeros(2)
    for t in range(1, 51):
        before = th.copy()
        oracle.adam(th, g, m, v, t, lr=1e-2, eps=0.0)
        np.testing.assert_allclose(th - before, -1e-2 * np.sign(g), rtol=1e-12)


# ----------------------------------------------------------------------------- convection-diffusion

@pytest.mark.parametrize("n,exact", [(10, True), (12, True), (4, False)])
def test_cd_manufactured_cubic_residual_vanishes(oracle, n, exact):
    """-eps Lap u + b . grad u = f with u = x^3 + x y^2 + 2y (grad u = (3x^2 + y^2, 2xy + 2), Lap u = 8x):
    the weak residual eps int grad u . grad v + int (b . grad u) v - int f v is exactly zero, and GLL
    integrates every term exactly once 2n-3 covers the integrand's degree on a bilinear element."""
    eps, bx, by = 0.7, 0.9, -0.4
    f = lambda x, y: -eps * 8.0 * x + bx * (3 * x * x + y * y) + by * (2 * x * y + 2.0)  # noqa: E731
    mesh = _skewed_mesh(3, seed=12)
    asm = oracle.assemble(mesh.xy, mesh.quad, n, 4, f_callable=f, want_M=True)
    X = asm.X
    ux = 3 * X[..., 0] ** 2 + X[..., 1] ** 2
    uy = 2 * X[..., 0] * X[..., 1] + 2.0
    R = oracle.residual(asm, ux, uy, eps=eps, conv=(bx, by))
    scale = np.abs(asm.F).max() + np.abs(asm.Gx).max() + np.abs(asm.M).max()
    if exact:
        assert np.abs(R).max() < 1e-12 * scale
    else:
        assert np.abs(R).max() > 1e-8 * scale
    # the convection term is what closes the balance: without it the residual is far from zero
    R0 = oracle.residual(asm, ux, uy, eps=eps)
    assert np.abs(R0).max() > 1e-3 * scale


def test_cd_linear_field_closed_form(oracle):
    """u = a x + c y, f = 0 on axis-aligned rectangles: the diffusion part vanishes (patch test) and
    int_K (b . grad u) v_(r,s) = (b . (a, c)) * det J * (int phi_r)(int phi_s), with int phi_1 = -2 and
    int phi_r = 0 for r >= 2, so R[e, (1,1)] = (b . (a, c)) * area_e and every other R[e, k] = 0."""
    a, c, bx, by, eps = 1.7, -0.6, 0.3, 2.1, 1.3
    mesh = gen.square_mesh(3, 2, 0.0)
    asm = oracle.assemble(mesh.xy, mesh.quad, 6, 3, 0.0, 0.0, 0.0, want_M=True)
    X = asm.X
    R = oracle.residual(asm, np.full(X.shape[:2], a), np.full(X.shape[:2], c), eps=eps, conv=(bx, by))
    area = (1.0 / 3.0) * (1.0 / 2.0)
    expect = np.zeros_like(R)
    expect[:, 0] = (bx * a + by * c) * area
    np.testing.assert_allclose(R, expect, atol=1e-13)
    # M sums to the integral of the test function: area for (1,1), zero otherwise
    np.testing.assert_allclose(asm.M.sum(axis=2)[:, 0], area, rtol=1e-13)


def test_cd_gradient_matches_finite_differences(oracle):
    """With a convection term, dL/dtheta still equals central differences of the oracle's loss."""
    H, L = 4, 2
    mesh = gen.square_mesh(2, 2, 0.2, seed=6)
    asm = oracle.assemble(mesh.xy, mesh.quad, 4, 3, f_callable=gen.gear_forcing, want_M=True)
    theta = gen.glorot_params(H, L, seed=10, bias_scale=0.4)
    bxy = gen.square_boundary_points(8)
    kw = dict(bnd_xy=bxy, bnd_g=np.zeros(8), tau=2.0, eps=0.8, conv=(1.1, -0.5))
    r = oracle.loss_grad(asm, theta, H, L, **kw)

    def f(th):
        return oracle.loss_grad(asm, th, H, L, want_grad=False, **kw).loss[0]

    h = 1e-6
    fd = np.array([(f(theta + h * e) - f(theta - h * e)) / (2 * h) for e in np.eye(theta.size)])
    assert np.linalg.norm(r.grad - fd) / np.linalg.norm(fd) < 1e-6


def test_cd_zero_velocity_is_poisson(oracle):
    mesh = _skewed_mesh(2, seed=3)
    asm = oracle.assemble(mesh.xy, mesh.quad, 5, 3, 4.0, 2.0, 1.0, want_M=True)
    theta = gen.glorot_params(5, 2, seed=1, bias_scale=0.2)
    a = oracle.loss_grad(asm, theta, 5, 2, eps=0.9, conv=(0.0, 0.0))
    b = oracle.loss_grad(asm, theta, 5, 2, eps=0.9)
    np.testing.assert_array_equal(a.loss, b.loss)
    np.testing.assert_array_equal(a.grad, b.grad)


# ----------------------------------------------------------------------------- space-dependent diffusion

@pytest.mark.parametrize("n,exact", [(10, True), (4, False)])
def test_vardiff_manufactured_residual_vanishes(oracle, n, exact):
    """-div(eps grad u) + b . grad u = f with u = x^3 + x y^2 + 2y and eps = 1 + 0.3x - 0.2y:
    f = -(eps Lap u + eps_x u_x + eps_y u_y) + b . grad u; with the exact u, eps at the quadrature points
    the weak residual sum_q eps_q grad u . G + (b . grad u) M - F vanishes under exact quadrature."""
    bx, by = 0.6, 0.4
    ex_, ey_ = 0.3, -0.2

    def f(x, y):
        e = 1.0 + ex_ * x + ey_ * y
        ux, uy = 3 * x * x + y * y, 2 * x * y + 2.0
        return -(e * 8.0 * x + ex_ * ux + ey_ * uy) + bx * ux + by * uy

    mesh = _skewed_mesh(3, seed=13)
    asm = oracle.assemble(mesh.xy, mesh.quad, n, 4, f_callable=f, want_M=True)
    X = asm.X
    ux = 3 * X[..., 0] ** 2 + X[..., 1] ** 2
    uy = 2 * X[..., 0] * X[..., 1] + 2.0
    epsq = 1.0 + ex_ * X[..., 0] + ey_ * X[..., 1]
    R = oracle.residual(asm, ux, uy, conv=(bx, by), epsq=epsq)
    scale = np.abs(asm.F).max() + np.abs(asm.Gx).max()
    if exact:
        assert np.abs(R).max() < 1e-12 * scale
    else:
        assert np.abs(R).max() > 1e-8 * scale
    # a constant coefficient in place of the field leaves a clear residual
    assert np.abs(oracle.residual(asm, ux, uy, eps=1.0, conv=(bx, by))).max() > 1e-3 * scale


def test_second_head_equal_weights_reproduces_u(oracle):
    """With W_out[1] = W_out[0] and b_out[1] = b_out[0] the second output equals u."""
    H, L = 7, 2
    theta = gen.glorot_params(H, L, seed=4, bias_scale=0.3, heads=2)
    o = gen.n_params(H, L) - (H + 1)  # start of the output block
    theta[o + H:o + 2 * H] = theta[o:o + H]
    theta[o + 2 * H + 1] = theta[o + 2 * H]
    xy = gen.uniform(2, "pts", 40, -1, 1).reshape(-1, 2)
    u, ux, uy, e = oracle.mlp_eval(theta, H, L, xy, heads=2)
    np.testing.assert_array_equal(u, e)


def test_constant_second_head_is_constant_coefficient_cd(oracle):
    """A second head with zero weights and bias c gives eps(x) = c everywhere: the loss and the gradient of
    the first-head parameters equal the constant-coefficient convection-diffusion loss with eps = c."""
    H, L, c = 6, 2, 0.7
    mesh = _skewed_mesh(2, seed=14)
    asm = oracle.assemble(mesh.xy, mesh.quad, 5, 3, f_callable=gen.gear_forcing, want_M=True)
    t2 = gen.glorot_params(H, L, seed=6, bias_scale=0.3, heads=2)
    o = gen.n_params(H, L) - (H + 1)
    t2[o + H:o + 2 * H] = 0.0
    t2[o + 2 * H + 1] = c
    t1 = np.concatenate([t2[:o + H], t2[o + 2 * H:o + 2 * H + 1]])
    bxy = gen.square_boundary_points(8)
    kw = dict(bnd_xy=bxy, bnd_g=np.zeros(8), tau=2.0, conv=(0.9, -0.3))
    r2 = oracle.loss_grad(asm, t2, H, L, heads=2, **kw)
    r1 = oracle.loss_grad(asm, t1, H, L, eps=c, **kw)
    np.testing.assert_allclose(r2.loss, r1.loss, rtol=1e-12)
    np.testing.assert_allclose(r2.grad[:o + H], r1.grad[:o + H], rtol=1e-10, atol=1e-14)
    np.testing.assert_allclose(r2.grad[o + 2 * H], r1.grad[o + H], rtol=1e-10)


def test_vardiff_gradient_matches_finite_differences(oracle):
    H, L = 4, 2
    mesh = gen.disk_mesh(3)
    asm = oracle.assemble(mesh.xy, mesh.quad, 4, 3, f_callable=lambda x, y: 10.0, want_M=True)
    theta = gen.glorot_params(H, L, seed=12, bias_scale=0.4, heads=2)
    bxy = gen.circle_points(8)
    sxy = gen.disk_sensor_points(5, 1)
    kw = dict(bnd_xy=bxy, bnd_g=np.zeros(8), sens_xy=sxy, sens_u=gen.uniform(1, "s", 5, -1, 1), tau=2.0,
              gamma=3.0, conv=(1.0, 0.0), heads=2)
    r = oracle.loss_grad(asm, theta, H, L, **kw)

    def f(th):
        return oracle.loss_grad(asm, th, H, L, want_grad=False, **kw).loss[0]

    h = 1e-6
    fd = np.array([(f(theta + h * e) - f(theta - h * e)) / (2 * h) for e in np.eye(theta.size)])
    assert np.linalg.norm(r.grad - fd) / np.linalg.norm(fd) < 1e-6


def test_disk_mesh_is_valid_and_has_disk_area(oracle):
    """Every element of the disk mesh is convex and counter-clockwise (the oracle's assembly rejects det J <= 0),
    and the elements' areas add up to just under pi r^2 (the mesh is inscribed in the circle)."""
    mesh = gen.disk_mesh(32)
    oracle.assemble(mesh.xy, mesh.quad, 3, 1, 1.0, 1.0, 1.0)
    x, y = mesh.xy[mesh.quad][..., 0], mesh.xy[mesh.quad][..., 1]
    shoelace = 0.5 * np.sum(x * np.roll(y, -1, 1) - y * np.roll(x, -1, 1), axis=1)
    assert (shoelace > 0).all()
    assert 0.0 < math.pi * 0.25 - shoelace.sum() < 2e-3


def test_prediction_error_of_a_constant_network(oracle):
    """Zero weights: every output is its bias, so the three errors have closed forms."""
    H, L = 4, 2
    theta = np.zeros(gen.n_params(H, L, heads=2))
    theta[-2], theta[-1] = 0.75, -1.5          # b_out of u and of e
    xy = gen.uniform(3, "errpts", 40, 0, 1).reshape(20, 2)
    ref = np.full(20, 0.25)
    mae, mx, rel = oracle.prediction_error(theta, H, L, xy, ref, heads=2)
    assert abs(mae - 0.5) < 1e-15 and abs(mx - 0.5) < 1e-15 and abs(rel - 2.0) < 1e-14
    mae, mx, rel = oracle.prediction_error(theta, H, L, xy, ref, heads=2, output=1)
    assert abs(mae - 1.75) < 1e-15 and abs(mx - 1.75) < 1e-15 and abs(rel - 7.0) < 1e-14


def test_prediction_error_picks_the_worst_point(oracle):
    """A single tanh neuron against a reference equal to it except at one point: that point sets the max and
    the L2 error, and the mean is its error over n."""
    theta = np.array([0.7, -1.3, 0.2, 1.9, -0.4])
    xy = gen.uniform(4, "errpts1", 20, -1, 1).reshape(10, 2)
    u = 1.9 * np.tanh(0.7 * xy[:, 0] - 1.3 * xy[:, 1] + 0.2) - 0.4
    ref = u.copy()
    ref[6] += 0.3
    mae, mx, rel = oracle.prediction_error(theta, 1, 1, xy, ref)
    assert abs(mae - 0.03) < 1e-14 and abs(mx - 0.3) < 1e-14
    assert abs(rel - 0.3 / np.linalg.norm(ref)) < 1e-14


def test_assembly_refuses_an_order_the_rule_does_not_cover(oracle):
    """An order beyond the GLL routine's range is an error of the assembly, never garbage nodes."""
    m = gen.square_mesh(1, 1)
    with pytest.raises(Exception):
        oracle.assemble(m.xy, m.quad, 129, 2, 1.0, 1.0, 1.0)


def test_inverse_const_data_residual_vanishes_at_the_true_eps(oracle):
    """The constant-diffusion inverse problem of Sec. 4.7.1 at its sizes (2 x 2 elements of (-1, 1)^2, 40 x 40
    GLL points, 5 x 5 tests): with the exact gradient of u = 10 sin x tanh x exp(-0.3 x^2) at the quadrature
    points, eps A - F vanishes to quadrature error at the true eps = 0.3 and not at the initial 2.0.  The
    forcing's closed form is checked against a central second difference of u."""
    prob = gen.config_inverse_const()
    man = gen.InverseConstManufactured(0.3)
    x = np.linspace(-1.0, 1.0, 41)
    h = 1e-4
    fd = -0.3 * (man.u(x + h, 0.0) - 2.0 * man.u(x, 0.0) + man.u(x - h, 0.0)) / (h * h)
    assert np.abs(fd - man.f(x, 0.0)).max() < 1e-6 * np.abs(fd).max()
    asm = oracle.assemble_problem(prob)
    X = asm.X[..., 0]
    s, c, t, r = np.sin(X), np.cos(X), np.tanh(X), np.exp(-0.3 * X * X)
    ux = 10.0 * (c * t * r + s * (1.0 - t * t) * r + s * t * (-0.6 * X * r))
    uy = np.zeros_like(ux)
    scale = np.abs(asm.F).max()
    assert np.abs(oracle.residual(asm, ux, uy, eps=0.3)).max() < 1e-11 * scale
    assert np.abs(oracle.residual(asm, ux, uy, eps=2.0)).max() > 0.1 * scale
    assert np.allclose(prob.bnd_g, man.u(prob.bnd_xy[:, 0], prob.bnd_xy[:, 1]))


# ----------------------------------------------------------------------------- the loss tied to the residual

@pytest.mark.parametrize("eps,conv,heads", [(0.3, None, 1), (2.0, None, 1), (0.3, (1.1, -0.6), 1),
                                            (2.0, (0.4, 0.9), 1), (1.0, (1.0, 0.0), 2), (1.0, None, 2)])
def test_loss_residual_equals_pinned_residual_at_a_random_network(oracle, eps, conv, heads):
    """At a Glorot network with non-zero biases (so grad u != 0 and, with two outputs, e(x) varies), the
    residual the loss evaluates equals orc_residual fed with the network's own tangents at the quadrature
    points: R = eps A + sum_q (b . grad u) M - F (Sec. 2.3 cell residual, Sec. 4.7.1 eps scaling the
    diffusion term, the convection term of Sec. 4.6.4), or sum_q e_q (grad u . G) + ... - F with two outputs
    (Sec. 4.7.2).  orc_residual is pinned by the manufactured solutions above and the network tangents by
    finite differences, so a misplaced eps (eps (A - F), A - eps F), a swapped x/y or a dropped convection
    term in the loss fails here.  The loss terms are then the stated sums of that residual and of the
    boundary and sensor mismatches at the network's values."""
    H, L = 6, 2
    mesh = gen.square_mesh(3, 2, 0.2, seed=21)
    asm = oracle.assemble(mesh.xy, mesh.quad, 5, 3, 4.0, 3.0, 2.0, want_M=conv is not None)
    theta = gen.glorot_params(H, L, seed=22, bias_scale=0.5, heads=heads)
    bxy = gen.square_boundary_points(12)
    bg = gen.uniform(23, "bg", 12, -0.5, 0.5)
    sxy = gen.sensor_points(7, 24)
    su = gen.uniform(23, "su", 7, -0.5, 0.5)
    tau, gamma = 2.0, 3.0
    r = oracle.loss_grad(asm, theta, H, L, bxy, bg, sxy, su, eps=eps, tau=tau, gamma=gamma, want_R=True,
                         conv=conv, heads=heads)
    outs = oracle.mlp_eval(theta, H, L, asm.X.reshape(-1, 2), heads=heads)
    ux = outs[1].reshape(asm.n_elem, -1)
    uy = outs[2].reshape(asm.n_elem, -1)
    epsq = outs[3].reshape(asm.n_elem, -1) if heads == 2 else None
    assert np.abs(ux).max() > 0.02 and np.abs(uy).max() > 0.02
    if heads == 2:
        assert np.ptp(epsq) > 0.05
    R = oracle.residual(asm, ux, uy, eps=eps, conv=conv, epsq=epsq)
    scale = np.abs(R).max()
    np.testing.assert_allclose(r.R, R, rtol=0, atol=1e-13 * scale)
    # the diffusion term carries signal of its own, so the placement of eps is tested
    A = oracle.residual(asm, ux, uy, eps=1.0, epsq=epsq) + asm.F
    assert np.abs(A).max() > 0.01 * np.abs(asm.F).max()
    cv = 1.0 / 9
    assert abs(r.loss[1] - cv * np.sum(R ** 2)) <= 1e-13 * r.loss[1]
    ub = oracle.mlp_eval(theta, H, L, bxy, heads=heads)[0]
    us = oracle.mlp_eval(theta, H, L, sxy, heads=heads)[0]
    assert abs(r.loss[2] - np.mean((ub - bg) ** 2)) <= 1e-13 * r.loss[2]
    assert abs(r.loss[3] - np.mean((us - su) ** 2)) <= 1e-13 * r.loss[3]
    assert abs(r.loss[0] - (r.loss[1] + tau * r.loss[2] + gamma * r.loss[3])) <= 1e-13 * r.loss[0]
