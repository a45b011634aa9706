"""Matrix-free problems: no premultiplied tensors are stored; the contraction regenerates G from the element's
bilinear map by sum factorisation every call.

Parity: loss and gradient against the FP64 oracle (which builds and stores G) for Poisson shapes from the
smallest element to N_quad = 256 and N_t = 30, the inverse problem's scalar eps and its gradient, constant
convection-diffusion, space-dependent diffusion with two network outputs, and batches that mix stored and
matrix-free instances; the same bars as the stored-G tests.
"""
import numpy as np
import pytest

import vpinn_inputs as gen

pytestmark = pytest.mark.gpu


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


def _square(name, m, n, nt, k=2, n_d=80, perturb=0.2, seed=0, ns=0, gamma=0.0):
    p = gen.poisson_sinsin_square(name, m, n, nt, k, n_d, perturb, seed=seed)
    if ns:
        p.sens_xy = gen.uniform(seed, "mf/sens", 2 * ns, 0.0, 1.0).reshape(ns, 2)
        p.sens_u = np.sin(k * np.pi * p.sens_xy[:, 0]) * np.sin(k * np.pi * p.sens_xy[:, 1])
        p.gamma = gamma
    return p


POISSON = {
    "uniform_n5_t5": lambda: _square("mf_u", 2, 5, 5, perturb=0.0),
    "skew_n6_t4_sens": lambda: _square("mf_s", 6, 6, 4, seed=1, ns=50, gamma=5.0),
    "skew_n10_t20": lambda: _square("mf_p", 4, 10, 20, k=3, seed=2),
    "skew_n16_t3": lambda: _square("mf_16", 3, 16, 3, seed=3),
    "skew_n2_t1": lambda: _square("mf_2", 5, 2, 1, seed=4),
    "skew_n7_t30": lambda: _square("mf_30", 2, 7, 30, seed=5),
    "skew_n9_t5_ragged": lambda: _square("mf_r", 7, 9, 5, seed=6),
}


def _check(loss, grad, ref, tag, geps=None):
    assert abs(loss[0] - ref.loss[0]) / abs(ref.loss[0]) < 1e-5, (tag, loss[0], ref.loss[0])
    for i in range(1, 4):
        assert abs(loss[i] - ref.loss[i]) <= 1e-5 * abs(ref.loss[0]) + 1e-6 * abs(ref.loss[i]), (tag, i)
    rel = np.linalg.norm(grad - ref.grad) / np.linalg.norm(ref.grad)
    assert rel < 1e-4, (tag, rel)
    if geps is not None:
        assert abs(geps - ref.grad_eps) / abs(ref.grad_eps) < 1e-4, (tag, geps, ref.grad_eps)


def _run(V, torch, p, prob, theta, eps=None, heads=1):
    dev = torch.device("cuda:0")
    th = torch.tensor(theta, dtype=torch.float32, device=dev)
    loss = torch.zeros(4, device=dev)
    grad = torch.zeros(theta.size, device=dev)
    ep = None if eps is None else torch.tensor([eps], dtype=torch.float32, device=dev)
    gep = None if eps is None else torch.zeros(1, device=dev)
    cfg = V.loss_cfg(prob.width, prob.n_hidden, prob.tau, prob.gamma, n_outputs=heads)
    V.vpinn_loss_and_grad(p, cfg, th, eps=ep, loss=loss, grad=grad, grad_eps=gep)
    torch.cuda.synchronize()
    return (loss.cpu().double().numpy(), grad.cpu().double().numpy(),
            None if gep is None else float(gep.item()))


@pytest.mark.parametrize("case", sorted(POISSON))
def test_matrix_free_poisson_matches_oracle(V, torch, case):
    from oracle import oracle as O
    prob = POISSON[case]()
    theta = prob.params(seed=3, bias_scale=0.1)
    p = V.assemble_problem(prob, matrix_free=True)
    info = V.vpinn_get_info(p)
    assert info.matrix_free == 1 and info.shared_premultiplier == 0
    loss, grad, _ = _run(V, torch, p, prob, theta)
    _check(loss, grad, O.problem_loss_grad(prob, O.assemble_problem(prob), theta), case)


@pytest.mark.parametrize("eps", [0.3, 2.0])
def test_matrix_free_inverse_eps_and_its_gradient(V, torch, eps):
    from oracle import oracle as O
    prob = _square("mf_inv", 5, 6, 5, seed=7, ns=60, gamma=10.0)
    theta = prob.params(seed=4, bias_scale=0.1)
    p = V.assemble_problem(prob, matrix_free=True)
    loss, grad, geps = _run(V, torch, p, prob, theta, eps=eps)
    _check(loss, grad, O.problem_loss_grad(prob, O.assemble_problem(prob), theta, eps=eps), f"eps={eps}", geps)


def test_matrix_free_agrees_with_stored_tensors(V, torch):
    """Same problem, stored G against regenerated G: equal up to FP32 rounding."""
    prob = _square("mf_vs", 8, 6, 5, seed=8)
    theta = prob.params(seed=5, bias_scale=0.1)
    l1, g1, _ = _run(V, torch, V.assemble_problem(prob), prob, theta)
    l2, g2, _ = _run(V, torch, V.assemble_problem(prob, matrix_free=True), prob, theta)
    assert abs(l1[0] - l2[0]) <= 2e-6 * abs(l1[0])
    assert np.linalg.norm(g1 - g2) <= 2e-5 * np.linalg.norm(g1)


def test_matrix_free_convection_diffusion(V, torch):
    from oracle import oracle as O
    prob = gen.poisson_sinsin_square("mf_cd", 6, 6, 4, 2, 80, 0.2, seed=21)
    prob.diff, prob.conv = 0.5, (1.0, -0.7)
    theta = prob.params(seed=6, bias_scale=0.1)
    p = V.assemble_problem(prob, matrix_free=True)
    info = V.vpinn_get_info(p)
    assert (info.diffusion, info.velocity_x, info.velocity_y) == (0.5, 1.0, -0.7)
    loss, grad, _ = _run(V, torch, p, prob, theta)
    _check(loss, grad, O.problem_loss_grad(prob, O.assemble_problem(prob), theta), "cd")


def test_matrix_free_space_dependent_diffusion(V, torch):
    from oracle import oracle as O
    man = gen.VarDiffManufactured(b=(1.0, 0.0))
    mesh = gen.disk_mesh(6)
    bxy = gen.circle_points(120)
    sxy = gen.disk_sensor_points(80, 1)
    prob = gen.Problem(name="mf_vd", mesh=mesh, quad_order=6, test_order=4, f_amp=0.0, f_kx=0.0, f_ky=0.0,
                       bnd_xy=bxy, bnd_g=man.u(bxy[:, 0], bxy[:, 1]), sens_xy=sxy, sens_u=man.u(sxy[:, 0], sxy[:, 1]),
                       tau=10.0, gamma=10.0, seed=1, conv=(1.0, 0.0), f_fn=man.f, heads=2)
    theta = prob.params(seed=7, bias_scale=0.1)
    p = V.assemble_problem(prob, matrix_free=True)
    info = V.vpinn_get_info(p)
    assert info.matrix_free == 1 and info.variable_diffusion == 1
    loss, grad, _ = _run(V, torch, p, prob, theta, heads=2)
    _check(loss, grad, O.problem_loss_grad(prob, O.assemble_problem(prob), theta), "vardiff")


def test_batch_mixing_stored_and_matrix_free(V, torch):
    from oracle import oracle as O
    probs = [_square("mf_b0", 5, 6, 5, seed=9), _square("mf_b1", 4, 10, 20, seed=10),
             _square("mf_b2", 6, 4, 3, seed=11), _square("mf_b3", 3, 12, 8, seed=12)]
    gp = [V.assemble_problem(pr, matrix_free=(i % 2 == 1)) for i, pr in enumerate(probs)]
    b = V.vpinn_batch_create(gp, V.loss_cfg(30, 3, 10.0, 0.0))
    th = np.stack([pr.params(seed=40 + i, bias_scale=0.1) for i, pr in enumerate(probs)])
    dev = torch.device("cuda:0")
    T = torch.tensor(th, dtype=torch.float32, device=dev)
    refs = [O.problem_loss_grad(pr, O.assemble_problem(pr), th[i]) for i, pr in enumerate(probs)]
    for tune in [(12, 0, 4), (16, 2, 2), (12, 0, 4, 1)]:
        V.vpinn_batch_set_tuning(b, *tune)
        losses = torch.zeros((len(probs), 4), device=dev)
        grads = torch.zeros((len(probs), th.shape[1]), device=dev)
        V.vpinn_batch_loss_and_grad(b, T, losses=losses, grads=grads)
        torch.cuda.synchronize()
        for i, pr in enumerate(probs):
            _check(losses[i].cpu().double().numpy(), grads[i].cpu().double().numpy(), refs[i], f"{pr.name}/{tune}")


def test_matrix_free_argument_checks(V, torch):
    prob = _square("mf_chk", 3, 5, 3, seed=13)
    p = V.assemble_problem(prob, matrix_free=True)
    dev = torch.device("cuda:0")
    th = torch.tensor(prob.params(seed=1), dtype=torch.float32, device=dev)
    loss = torch.zeros(4, device=dev)
    with pytest.raises(V.VpinnError) as ei:
        V.vpinn_loss_and_grad(p, V.loss_cfg(path=V.VPINN_PATH_PLAIN), th, loss=loss)
    assert ei.value.code == V.VPINN_E_UNSUPPORTED
    with pytest.raises(V.VpinnError) as ei:
        V.vpinn_residual(p, V.loss_cfg(), th, torch.zeros(prob.n_elem * 9, device=dev))
    assert ei.value.code == V.VPINN_E_UNSUPPORTED
    for which in (V.VPINN_TENSOR_GX, V.VPINN_TENSOR_GY, V.VPINN_TENSOR_M):
        with pytest.raises(V.VpinnError) as ei:
            V.vpinn_read_tensor(p, which)
        assert ei.value.code == V.VPINN_E_INVALID
    F = V.vpinn_read_tensor(p, V.VPINN_TENSOR_F)
    from oracle import oracle as O
    np.testing.assert_allclose(F.astype(np.float64), O.assemble_problem(prob).F, rtol=2e-6, atol=1e-9)


def test_probe_matrix_free_full_size(V, torch):
    """The probe shape (4,096 elements, 10 x 10 points, 20 x 20 test functions) without its 1.3 GB of G:
    at full size against the stored-G path (the oracle needs minutes here), and a 64-element slice of the
    same mesh against the oracle."""
    import dataclasses
    from oracle import oracle as O
    prob = gen.config_probe()
    theta = prob.params(seed=2, bias_scale=0.1)
    l1, g1, _ = _run(V, torch, V.assemble_problem(prob), prob, theta)
    l2, g2, _ = _run(V, torch, V.assemble_problem(prob, matrix_free=True), prob, theta)
    assert abs(l1[0] - l2[0]) <= 2e-6 * abs(l1[0])
    assert np.linalg.norm(g1 - g2) <= 2e-5 * np.linalg.norm(g1)
    part = dataclasses.replace(prob, name="probe_slice", mesh=gen.Mesh(prob.mesh.xy, prob.mesh.quad[:64].copy()))
    loss, grad, _ = _run(V, torch, V.assemble_problem(part, matrix_free=True), part, theta)
    _check(loss, grad, O.problem_loss_grad(part, O.assemble_problem(part), theta), "probe_slice")
