"""Parity of the HIP library (through its C ABI) with the FP64 oracle on the same seeded inputs.

Bars: assembled tensors to FP32 rounding; loss within 1e-5 relative; gradient within 1e-4
relative L2 (and d/deps within 1e-4 relative); network values to FP32 rounding of the
activations; Adam to FP32 rounding.
"""
import functools

import numpy as np
import pytest

import vpinn_inputs as gen

pytestmark = pytest.mark.gpu

LOSS_RTOL = 1e-5
GRAD_RTOL = 1e-4


@pytest.fixture(scope="module")
def torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


@pytest.fixture(scope="module")
def V(torch):
    from paper_2404_12063_amd import vpinn as V
    V.lib()
    return V


@functools.lru_cache(maxsize=None)
def _oracle_asm(name):
    from oracle import oracle as O
    return O.assemble_problem(_problem(name))


@functools.lru_cache(maxsize=None)
def _problem(name):
    if name in gen.CONFIGS:
        return gen.CONFIGS[name]()
    if name == "ragged":      # 3x5 skewed mesh, odd sizes everywhere
        p = gen.poisson_sinsin_square("ragged", 1, 4, 3, 3, 12, 0.2, seed=5)
        p.mesh = gen.square_mesh(3, 5, 0.2, seed=5)
        p.width, p.n_hidden = 17, 2
        return p
    if name == "tiny_n2":     # smallest orders: 2x2 GLL (trapezoid), one test function
        p = gen.poisson_sinsin_square("tiny_n2", 2, 2, 1, 1, 8, 0.1, seed=2)
        p.width, p.n_hidden = 5, 1
        return p
    if name == "deep32":      # maximum width and depth
        p = gen.poisson_sinsin_square("deep32", 4, 6, 3, 2, 40, 0.2, seed=3)
        p.width, p.n_hidden = 32, 4
        return p
    if name == "nobnd":       # no boundary points, tau irrelevant
        p = gen.poisson_sinsin_square("nobnd", 5, 5, 5, 2, 4, 0.2, seed=4)
        p.bnd_xy = np.zeros((0, 2))
        p.bnd_g = np.zeros(0)
        return p
    if name == "p20":         # the p-refinement maximum (20x20 test functions) on a small mesh
        return gen.poisson_sinsin_square("p20", 4, 10, 20, 2, 80, 0.2, seed=6)
    if name == "q6t7":        # 49 test functions on 36 points: row-streaming contraction, one point per lane
        return gen.poisson_sinsin_square("q6t7", 3, 6, 7, 2, 40, 0.2, seed=8)
    if name == "q12t6":       # 144 points, 36 test functions: row streaming with four points a lane
        return gen.poisson_sinsin_square("q12t6", 2, 12, 6, 2, 40, 0.2, seed=9)
    if name == "uniform16":   # uniform 16x16 mesh: one shared premultiplier for every element (Algorithm 2)
        return gen.poisson_sinsin_square("uniform16", 16, 8, 5, 4, 200, 0.0, seed=1)
    if name == "q17":         # 289 points per element: the two-pass contraction for large elements
        return gen.poisson_sinsin_square("q17", 2, 17, 3, 2, 40, 0.2, seed=7)
    if name == "q80t20":      # the p-refinement study's element: 80 x 80 points, 20 x 20 test functions
        return gen.poisson_sinsin_square("q80t20", 1, 80, 20, 2, 80, 0.0, seed=10)
    if name == "q40t5":       # 2 x 2 skewed elements of 40 x 40 points, as in the constant-eps inverse problem
        return gen.poisson_sinsin_square("q40t5", 2, 40, 5, 2, 40, 0.2, seed=11)
    if name == "q100t3":      # the largest quadrature order (10,000 points an element)
        return gen.poisson_sinsin_square("q100t3", 1, 100, 3, 2, 40, 0.0, seed=12)
    if name == "q8t30":       # the largest test order (900 test functions) on 64-point elements
        return gen.poisson_sinsin_square("q8t30", 2, 8, 30, 2, 40, 0.2, seed=13)
    if name == "gear_small":  # a small toothed annulus: skewed elements, nonzero boundary data
        import math
        kp = 4 * math.pi
        mesh = gen.annulus_gear_mesh(48, 6, seed=2)
        bxy = gen.annulus_boundary_points(200)
        return gen.Problem("gear_small", mesh, 5, 5, 2 * kp * kp, kp, kp, bxy, gen.sinsin(bxy, kp, kp))
    raise KeyError(name)


def _gpu_problem(V, prob):
    p = V.vpinn_assemble(prob.mesh.xy, prob.mesh.quad, prob.quad_order, prob.test_order,
                         prob.f_amp, prob.f_kx, prob.f_ky)
    if len(prob.bnd_xy):
        V.vpinn_set_boundary(p, prob.bnd_xy, prob.bnd_g)
    if len(prob.sens_xy):
        V.vpinn_set_sensors(p, prob.sens_xy, prob.sens_u)
    return p


def _run(V, torch, p, prob, theta, path, eps=None, loss_norm=0):
    dev = torch.device("cuda:0")
    n = V.vpinn_n_params(prob.width, prob.n_hidden)
    th = torch.tensor(theta, dtype=torch.float32, device=dev)
    loss = torch.full((4,), float("nan"), dtype=torch.float32, device=dev)
    grad = torch.full((n,), float("nan"), dtype=torch.float32, device=dev)
    ep = None if eps is None else torch.tensor([eps], dtype=torch.float32, device=dev)
    gep = None if eps is None else torch.zeros(1, dtype=torch.float32, device=dev)
    cfg = V.loss_cfg(prob.width, prob.n_hidden, prob.tau, prob.gamma, loss_norm, path)
    V.vpinn_loss_and_grad(p, cfg, th, eps=ep, loss=loss, grad=grad, grad_eps=gep)
    torch.cuda.synchronize()
    return (loss.cpu().double().numpy(), grad.cpu().double().numpy(),
            None if gep is None else float(gep.cpu()))


def _params(prob):
    # Glorot weights plus nonzero biases, so every parameter group carries signal
    return prob.params(bias_scale=0.1)


def _oracle(prob, theta, eps=None, loss_norm=0):
    from oracle import oracle as O
    return O.problem_loss_grad(prob, _oracle_asm(prob.name), theta, eps=eps, loss_norm=loss_norm)


def _check(loss, grad, ref, geps=None, tag=""):
    rl = abs(loss[0] - ref.loss[0]) / abs(ref.loss[0])
    assert rl < LOSS_RTOL, f"{tag} loss {loss[0]} vs {ref.loss[0]} (rel {rl:.2e})"
    for i in (1, 2, 3):
        if ref.loss[i] != 0:
            assert abs(loss[i] - ref.loss[i]) / abs(ref.loss[i]) < LOSS_RTOL, (tag, i, loss[i], ref.loss[i])
        else:
            assert loss[i] == 0, (tag, i, loss[i])
    rg = np.linalg.norm(grad - ref.grad) / np.linalg.norm(ref.grad)
    assert rg < GRAD_RTOL, f"{tag} grad rel L2 {rg:.2e}"
    if geps is not None:
        assert abs(geps - ref.grad_eps) / abs(ref.grad_eps) < GRAD_RTOL, (tag, geps, ref.grad_eps)


PATHS = {"plain": 1, "fused": 0}


def _path_or_skip(V, name):
    return PATHS[name]


# ----------------------------------------------------------------------------- assembly

@pytest.mark.parametrize("name", ["c1", "c2", "gear_small", "ragged", "p20", "tiny_n2", "uniform16"])
def test_assembly_matches_oracle(V, name):
    prob = _problem(name)
    ref = _oracle_asm(name)
    p = _gpu_problem(V, prob)
    for which, r in [(V.VPINN_TENSOR_GX, ref.Gx), (V.VPINN_TENSOR_GY, ref.Gy), (V.VPINN_TENSOR_F, ref.F),
                     (V.VPINN_TENSOR_X, ref.X)]:
        g = V.vpinn_read_tensor(p, which).astype(np.float64)
        scale = np.abs(r).max()
        np.testing.assert_allclose(g, r, rtol=2e-6, atol=2e-7 * scale, err_msg=f"{name} tensor {which}")


def test_assembly_callback_forcing_matches_oracle(V):
    from oracle import oracle as O
    mesh = gen.square_mesh(4, 3, 0.2, seed=9)
    f = lambda x, y: x * x - 3.0 * y + 0.5  # noqa: E731
    p = V.vpinn_assemble(mesh.xy, mesh.quad, 6, 4, fn=f)
    ref = O.assemble(mesh.xy, mesh.quad, 6, 4, f_callable=f)
    g = V.vpinn_read_tensor(p, V.VPINN_TENSOR_F).astype(np.float64)
    np.testing.assert_allclose(g, ref.F, rtol=2e-6, atol=2e-7 * np.abs(ref.F).max())


def test_callback_nonfinite_is_reported(V):
    mesh = gen.square_mesh(2, 2)
    with pytest.raises(V.VpinnError) as ei:
        V.vpinn_assemble(mesh.xy, mesh.quad, 3, 2, fn=lambda x, y: float("nan") if x > 0.7 else 1.0)
    assert ei.value.code == V.VPINN_E_NONFINITE


# ----------------------------------------------------------------------------- network

@pytest.mark.parametrize("H,L", [(30, 3), (1, 1), (17, 2), (32, 4)])
def test_network_values_and_tangents(V, torch, H, L):
    from oracle import oracle as O
    theta = gen.glorot_params(H, L, seed=H + L, bias_scale=0.2)
    xy = gen.uniform(3, "netpts", 2 * 1000, -1.5, 1.5).reshape(-1, 2)
    dev = torch.device("cuda:0")
    th = torch.tensor(theta, dtype=torch.float32, device=dev)
    X = torch.tensor(xy, dtype=torch.float32, device=dev)
    u, ux, uy = (torch.empty(len(xy), dtype=torch.float32, device=dev) for _ in range(3))
    V.vpinn_eval_network(H, L, th, X, u, ux, uy)
    ru, rux, ruy = O.mlp_eval(theta, H, L, X.cpu().double().numpy())
    for a, b in [(u, ru), (ux, rux), (uy, ruy)]:
        a = a.cpu().double().numpy()
        np.testing.assert_allclose(a, b, rtol=1e-5, atol=2e-6 * np.abs(b).max())


# ----------------------------------------------------------------------------- loss and gradient

@pytest.mark.parametrize("path", ["plain", "fused"])
@pytest.mark.parametrize("name", ["c1", "c2", "gear_small", "ragged", "tiny_n2", "deep32", "nobnd", "p20", "q6t7",
                                  "q12t6", "q17", "uniform16", "q80t20", "q40t5", "q100t3", "q8t30"])
def test_loss_and_grad_match_oracle(V, torch, path, name):
    prob = _problem(name)
    theta = _params(prob)
    p = _gpu_problem(V, prob)
    loss, grad, _ = _run(V, torch, p, prob, theta, _path_or_skip(V, path))
    _check(loss, grad, _oracle(prob, theta), tag=f"{name}/{path}")


@pytest.mark.parametrize("orders", [(10, 5), (6, 7), (17, 3)])
@pytest.mark.parametrize("path", ["plain", "fused"])
def test_inverse_problem_eps_gradient(V, torch, path, orders):
    """C4-shaped inverse problem on a reduced mesh: trainable eps, sensors and boundary points (orders chosen
    so that each of the fused path's three contraction schemes is exercised)."""
    prob = gen.config_c4()
    nq, nt = orders
    small = gen.Problem("c4small", gen.square_mesh(12, 12, 0.2, seed=1), nq, nt, prob.f_amp, prob.f_kx, prob.f_ky,
                        prob.bnd_xy, prob.bnd_g, prob.sens_xy[:300], prob.sens_u[:300], tau=10.0, gamma=10.0)
    from oracle import oracle as O
    asm = O.assemble_problem(small)
    theta = _params(small)
    p = _gpu_problem(V, small)
    for eps in (2.0, 0.3):
        loss, grad, geps = _run(V, torch, p, small, theta, PATHS[path], eps=eps)
        ref = O.problem_loss_grad(small, asm, theta, eps=eps)
        _check(loss, grad, ref, geps=geps, tag=f"eps={eps}")


@pytest.mark.parametrize("path", ["plain", "fused"])
def test_inverse_const_at_the_papers_sizes(V, torch, path):
    """The constant-eps inverse problem of Sec. 4.7.1 exactly as the bench runs it (2 x 2 elements of
    (-1, 1)^2, 40 x 40 GLL points: the large-element contraction), loss, weight gradient and d loss / d eps
    at the initial, the true and a negative eps."""
    prob = gen.config_inverse_const()
    from oracle import oracle as O
    asm = O.assemble_problem(prob)
    theta = _params(prob)
    p = V.assemble_problem(prob)
    for eps in (2.0, 0.3, -0.5):
        loss, grad, geps = _run(V, torch, p, prob, theta, PATHS[path], eps=eps)
        _check(loss, grad, O.problem_loss_grad(prob, asm, theta, eps=eps), geps=geps, tag=f"eps={eps}")


@pytest.mark.parametrize("path", ["plain", "fused"])
def test_element_normalisation(V, torch, path):
    prob = _problem("c1")
    theta = _params(prob)
    p = _gpu_problem(V, prob)
    loss, grad, _ = _run(V, torch, p, prob, theta, PATHS[path], loss_norm=1)
    _check(loss, grad, _oracle(prob, theta, loss_norm=1))


@pytest.mark.slow
@pytest.mark.parametrize("path", ["plain", "fused"])
@pytest.mark.parametrize("name", ["c3", "c4"])
def test_full_size_configs(V, torch, path, name):
    prob = _problem(name)
    theta = _params(prob)
    p = _gpu_problem(V, prob)
    eps = prob.eps_init
    loss, grad, geps = _run(V, torch, p, prob, theta, PATHS[path], eps=eps)
    _check(loss, grad, _oracle(prob, theta, eps=eps), geps=geps, tag=f"{name}/{path}")


def test_residual_matches_oracle(V, torch):
    from oracle import oracle as O
    prob = _problem("c2")
    theta = _params(prob)
    p = _gpu_problem(V, prob)
    R = torch.empty((prob.n_elem, 25), dtype=torch.float32, device="cuda:0")
    th = torch.tensor(theta, dtype=torch.float32, device="cuda:0")
    V.vpinn_residual(p, V.loss_cfg(path=V.VPINN_PATH_PLAIN), th, R)
    ref = O.loss_grad(_oracle_asm("c2"), theta, 30, 3, want_grad=False, want_R=True).R
    np.testing.assert_allclose(R.cpu().double().numpy(), ref, rtol=1e-4, atol=1e-5 * np.abs(ref).max())


@pytest.mark.parametrize("path", ["plain", "fused"])
def test_deterministic_bitwise(V, torch, path):
    prob = _problem("c2")
    theta = _params(prob)
    p = _gpu_problem(V, prob)
    a = _run(V, torch, p, prob, theta, PATHS[path])
    b = _run(V, torch, p, prob, theta, PATHS[path])
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[1], b[1])


# ----------------------------------------------------------------------------- Adam

def test_adam_matches_oracle(V, torch):
    from oracle import oracle as O
    n = 1981
    th = gen.uniform(1, "a_th", n, -1, 1).astype(np.float32).astype(np.float64)
    g = gen.uniform(1, "a_g", n, -2, 2).astype(np.float32).astype(np.float64)
    dev = torch.device("cuda:0")
    T = torch.tensor(th, dtype=torch.float32, device=dev)
    G = torch.tensor(g, dtype=torch.float32, device=dev)
    M = torch.zeros(n, dtype=torch.float32, device=dev)
    Vv = torch.zeros(n, dtype=torch.float32, device=dev)
    rt, rm, rv = th.copy(), np.zeros(n), np.zeros(n)
    for t in range(1, 6):
        V.vpinn_adam_step(T, G, M, Vv, t, lr=1e-3)
        O.adam(rt, g, rm, rv, t, lr=1e-3)
    torch.cuda.synchronize()
    np.testing.assert_allclose(T.cpu().double().numpy(), rt, rtol=0, atol=2e-7)
    np.testing.assert_allclose(M.cpu().double().numpy(), rm, rtol=1e-6, atol=1e-9)


@pytest.mark.parametrize("path", ["plain", "fused"])
def test_c1_adam_trajectory(V, torch, path):
    """One loss + gradient, then 100 Adam steps at lr 1e-3 on the first workload, on both sides.
    The FP32 and FP64 trajectories are compared loosely (no closed form pins them); the oracle
    re-evaluated at the GPU's own parameters must match every sampled step to the parity bar."""
    from oracle import oracle as O
    prob = _problem("c1")
    asm = _oracle_asm("c1")
    theta = prob.params()
    p = _gpu_problem(V, prob)
    dev = torch.device("cuda:0")
    n = theta.size
    T = torch.tensor(theta, dtype=torch.float32, device=dev)
    M = torch.zeros(n, dtype=torch.float32, device=dev)
    Vv = torch.zeros(n, dtype=torch.float32, device=dev)
    G = torch.zeros(n, dtype=torch.float32, device=dev)
    loss = torch.zeros(4, dtype=torch.float32, device=dev)
    cfg = V.loss_cfg(30, 3, prob.tau, 0.0, 0, PATHS[path])
    rt, rm, rv = theta.copy(), np.zeros(n), np.zeros(n)
    for t in range(1, 101):
        V.vpinn_loss_and_grad(p, cfg, T, loss=loss, grad=G)
        if t in (1, 2, 10, 50, 100):
            torch.cuda.synchronize()
            th_gpu = T.cpu().double().numpy()
            ref = O.problem_loss_grad(prob, asm, th_gpu)
            _check(loss.cpu().double().numpy(), G.cpu().double().numpy(), ref, tag=f"step {t}")
        V.vpinn_adam_step(T, G, M, Vv, t, lr=1e-3)
        r = O.problem_loss_grad(prob, asm, rt)
        O.adam(rt, r.grad, rm, rv, t, lr=1e-3)
    torch.cuda.synchronize()
    l_gpu = O.problem_loss_grad(prob, asm, T.cpu().double().numpy(), want_grad=False).loss[0]
    l_cpu = O.problem_loss_grad(prob, asm, rt, want_grad=False).loss[0]
    assert abs(l_gpu - l_cpu) / l_cpu < 1e-3, (l_gpu, l_cpu)


@pytest.mark.parametrize("name,shared", [("c1", 1), ("uniform16", 1), ("c2", 0), ("tiny_n2", 0), ("gear_small", 0)])
def test_shared_premultiplier_detection(V, name, shared):
    """Uniform meshes store G once (Algorithm 2); jittered and curved ones per element."""
    p = _gpu_problem(V, _problem(name))
    assert V.vpinn_get_info(p).shared_premultiplier == shared


@pytest.mark.parametrize("path", ["plain", "fused"])
@pytest.mark.parametrize("tau,gamma", [(0.0, 0.0), (1.0, 0.0), (0.0, 1.0), (1.0, 1.0)])
def test_boundary_and_sensor_weights(V, torch, path, tau, gamma):
    """tau and gamma are arguments of the call: 0 removes a term from the gradient (its loss component is still
    reported), 1 weighs it as the plain mean."""
    import dataclasses
    from oracle import oracle as O
    base = _problem("ragged")
    sxy = gen.sensor_points(40, 9)
    prob = dataclasses.replace(base, name=f"w{tau}{gamma}", tau=tau, gamma=gamma, sens_xy=sxy,
                               sens_u=gen.uniform(9, "wsu", 40, -1, 1))
    theta = _params(prob)
    p = _gpu_problem(V, prob)
    loss, grad, _ = _run(V, torch, p, prob, theta, _path_or_skip(V, path))
    _check(loss, grad, O.problem_loss_grad(prob, _oracle_asm("ragged"), theta), tag=f"tau={tau}/gamma={gamma}/{path}")


@pytest.mark.parametrize("m,n,nt,kw,eps", [(23, 17, 3, 1, 2.0), (16, 23, 3, 2, 2.0), (16, 17, 3, 4, 2.0),
                                           (16, 17, 7, 4, None)])
def test_large_element_contraction_every_wavefront_grouping(V, torch, m, n, nt, kw, eps):
    """Many elements of more than 256 points: the adjoint blocks of the two-launch contraction then group
    kw = 1, 2 or 4 wavefronts per 64 points (the small shapes above use 16); loss and gradient against the
    oracle on a skewed mesh with sensors, and the eps gradient where it is resolvable in FP32: with 7 x 7
    test functions the stiffness sums A of this random network cancel to about 1e-6 of their terms, so
    d loss / d eps (proportional to A) is checked on the 3 x 3 cases only."""
    from oracle import oracle as O
    prob = gen.poisson_sinsin_square(f"split_{m}_{n}_{nt}", m, n, nt, 3, 400, 0.2, seed=m + n + nt)
    prob.sens_xy = gen.uniform(5, "split/sens", 2 * 60, 0.0, 1.0).reshape(60, 2)
    prob.sens_u = np.sin(3 * np.pi * prob.sens_xy[:, 0]) * np.sin(3 * np.pi * prob.sens_xy[:, 1])
    prob.gamma = 5.0
    # the grouping rule: at most 32 test functions a wavefront, more wavefronts below 512 blocks
    g = 1
    while g < 16 and (g * 32 < nt * nt or m * m * -(-n * n // (64 * (16 // g))) < 512):
        g *= 2
    assert g == kw
    asm = O.assemble_problem(prob)
    theta = _params(prob)
    p = _gpu_problem(V, prob)
    for path in ("fused", "plain"):
        loss, grad, geps = _run(V, torch, p, prob, theta, PATHS[path], eps=eps)
        _check(loss, grad, O.problem_loss_grad(prob, asm, theta, eps=eps), geps=geps, tag=f"{path}")


def test_batch_mixing_every_contraction_path(V, torch):
    """One batch holding a small-element instance, a row-streaming instance (N_test > 32), a one-element
    80 x 80 instance and a many-element large-element instance: each against the oracle."""
    from oracle import oracle as O
    probs = [gen.poisson_sinsin_square("mix_fast", 6, 6, 4, 2, 80, 0.2, seed=1),
             gen.poisson_sinsin_square("mix_rows", 3, 10, 8, 2, 80, 0.2, seed=2),
             gen.poisson_sinsin_square("mix_one", 1, 80, 12, 2, 80, 0.0, seed=3),
             gen.poisson_sinsin_square("mix_split", 16, 17, 3, 2, 80, 0.2, seed=4)]
    gp = [_gpu_problem(V, pr) for pr in probs]
    b = V.vpinn_batch_create(gp, V.loss_cfg(30, 3, 10.0, 0.0))
    th = np.stack([pr.params(seed=50 + i, bias_scale=0.1) for i, pr in enumerate(probs)])
    dev = torch.device("cuda:0")
    T = torch.tensor(th, dtype=torch.float32, device=dev)
    refs = [O.problem_loss_grad(pr, O.assemble_problem(pr), th[i]) for i, pr in enumerate(probs)]
    for tune in [(12, 0, 4, 0), (16, 2, 2, 1)]:
        V.vpinn_batch_set_tuning(b, *tune)
        losses = torch.zeros((len(probs), 4), device=dev)
        grads = torch.zeros((len(probs), th.shape[1]), device=dev)
        V.vpinn_batch_loss_and_grad(b, T, losses=losses, grads=grads)
        torch.cuda.synchronize()
        for i, pr in enumerate(probs):
            _check(losses[i].cpu().double().numpy(), grads[i].cpu().double().numpy(), refs[i], tag=f"{pr.name}/{tune}")


@pytest.mark.parametrize("m,n,nt", [(1, 40, 10), (16, 17, 3)])
def test_large_element_loss_without_gradient(V, torch, m, n, nt):
    """A loss-only call (no gradient buffer) on the two-launch contraction: the adjoint is skipped and the loss
    still matches the oracle, and a following call with a gradient gives the same loss bit for bit."""
    from oracle import oracle as O
    prob = gen.poisson_sinsin_square(f"lossonly_{m}_{n}_{nt}", m, n, nt, 2, 200, 0.2 if m > 1 else 0.0, seed=9)
    theta = _params(prob)
    p = _gpu_problem(V, prob)
    dev = torch.device("cuda:0")
    th = torch.tensor(theta, dtype=torch.float32, device=dev)
    cfg = V.loss_cfg(prob.width, prob.n_hidden, prob.tau, prob.gamma)
    l1 = torch.full((4,), float("nan"), device=dev)
    V.vpinn_loss_and_grad(p, cfg, th, loss=l1)
    l2 = torch.full((4,), float("nan"), device=dev)
    g = torch.zeros(V.vpinn_n_params(prob.width, prob.n_hidden), device=dev)
    V.vpinn_loss_and_grad(p, cfg, th, loss=l2, grad=g)
    torch.cuda.synchronize()
    ref = O.problem_loss_grad(prob, O.assemble_problem(prob), theta, want_grad=False)
    assert abs(float(l1[0]) - ref.loss[0]) <= LOSS_RTOL * abs(ref.loss[0])
    assert torch.equal(l1, l2)


def test_changed_weighting_on_another_stream_keeps_earlier_results(V, torch):
    """A problem's cached plan is rebuilt when tau changes; the rebuild rewrites device descriptors, so it must wait
    for earlier calls still running on other streams: a call with tau = 10 on one stream, followed at once by a call
    with tau = 1 on another, gives each its own loss (each against its own solitary evaluation)."""
    prob = gen.config_c4()
    p = V.assemble_problem(prob)
    dev = torch.device("cuda:0")
    th = torch.tensor(prob.params(bias_scale=0.1), dtype=torch.float32, device=dev)
    eps = torch.tensor([0.7], device=dev)
    n = th.numel()

    def solo(tau):
        l, g = torch.zeros(4, device=dev), torch.zeros(n, device=dev)
        V.vpinn_loss_and_grad(p, V.loss_cfg(30, 3, tau, 10.0), th, eps=eps, loss=l, grad=g)
        torch.cuda.synchronize()
        return l.cpu().numpy(), g.cpu().numpy()

    want10, want1 = solo(10.0), solo(1.0)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    for _ in range(3):
        l10, g10 = torch.zeros(4, device=dev), torch.zeros(n, device=dev)
        l1, g1 = torch.zeros(4, device=dev), torch.zeros(n, device=dev)
        torch.cuda.synchronize()
        with torch.cuda.stream(s1):
            V.vpinn_loss_and_grad(p, V.loss_cfg(30, 3, 10.0, 10.0), th, eps=eps, loss=l10, grad=g10, stream=s1)
        with torch.cuda.stream(s2):
            V.vpinn_loss_and_grad(p, V.loss_cfg(30, 3, 1.0, 10.0), th, eps=eps, loss=l1, grad=g1, stream=s2)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(l10.cpu().numpy(), want10[0])
        np.testing.assert_array_equal(g10.cpu().numpy(), want10[1])
        np.testing.assert_array_equal(l1.cpu().numpy(), want1[0])
        np.testing.assert_array_equal(g1.cpu().numpy(), want1[1])
