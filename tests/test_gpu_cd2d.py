"""Convection-diffusion -eps Lap u + b . grad u = f (the paper's gear problem): the GPU folds eps and b into
the premultiplied tensors at assembly; the FP64 oracle keeps the convection integral as its own term.

Parity: the folded tensors against eps * G + b * M from the oracle, and the loss and gradient of both paths
(single problem and batch) against the oracle, to the same tolerances as the Poisson problems.
"""
import math

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


def _cd_square():
    """Skewed 6x6 mesh, eps 0.5, b = (1.0, -0.7), sin-sin forcing and boundary data."""
    p = gen.poisson_sinsin_square("cd_square", 6, 6, 4, 2, 80, 0.2, seed=21)
    p.diff, p.conv = 0.5, (1.0, -0.7)
    return p


def _cd_gear_small():
    """The gear problem on a small toothed annulus: eps 1, b = (0.1, 0), f = 50 sin x + cos x, u = 0."""
    mesh = gen.annulus_gear_mesh(48, 6, seed=3)
    bxy = gen.annulus_boundary_points(300)
    return gen.Problem("cd_gear_small", mesh, 5, 4, 0.0, 0.0, 0.0, bxy, np.zeros(len(bxy)), diff=1.0,
                       conv=(0.1, 0.0), f_fn=gen.gear_forcing)


def _params(prob, seed=5):
    return prob.params(seed=seed, bias_scale=0.1)


def _check(loss, grad, ref, tag):
    assert abs(loss[0] - ref.loss[0]) / abs(ref.loss[0]) < 1e-5, (tag, loss[0], ref.loss[0])
    for i in range(1, 4):
        assert abs(loss[i] - ref.loss[i]) <= 1e-5 * abs(ref.loss[0]) + 1e-6 * abs(ref.loss[i]), (tag, i)
    rel = np.linalg.norm(grad - ref.grad) / np.linalg.norm(ref.grad)
    assert rel < 1e-4, (tag, rel)


@pytest.mark.parametrize("make", [_cd_square, _cd_gear_small])
def test_folded_tensors_match_oracle(V, make):
    from oracle import oracle as O
    prob = make()
    asm = O.assemble_problem(prob)
    p = V.assemble_problem(prob)
    info = V.vpinn_get_info(p)
    assert (info.diffusion, info.velocity_x, info.velocity_y) == (prob.diff, *prob.conv)
    bx, by = prob.conv
    for which, ref in [(V.VPINN_TENSOR_GX, prob.diff * asm.Gx + bx * asm.M),
                       (V.VPINN_TENSOR_GY, prob.diff * asm.Gy + by * asm.M), (V.VPINN_TENSOR_F, asm.F)]:
        g = V.vpinn_read_tensor(p, which).astype(np.float64).reshape(ref.shape)
        np.testing.assert_allclose(g, ref, rtol=2e-6, atol=2e-7 * np.abs(ref).max())


@pytest.mark.parametrize("path", ["plain", "fused"])
@pytest.mark.parametrize("make", [_cd_square, _cd_gear_small])
def test_cd_loss_and_grad_match_oracle(V, torch, make, path):
    from oracle import oracle as O
    prob = make()
    theta = _params(prob)
    p = V.assemble_problem(prob)
    dev = torch.device("cuda:0")
    n = V.vpinn_n_params(prob.width, prob.n_hidden)
    th = torch.tensor(theta, dtype=torch.float32, device=dev)
    loss = torch.zeros(4, device=dev)
    grad = torch.zeros(n, device=dev)
    cfg = V.loss_cfg(prob.width, prob.n_hidden, prob.tau, prob.gamma,
                     path=V.VPINN_PATH_PLAIN if path == "plain" else V.VPINN_PATH_FUSED)
    V.vpinn_loss_and_grad(p, cfg, th, loss=loss, grad=grad)
    torch.cuda.synchronize()
    ref = O.problem_loss_grad(prob, O.assemble_problem(prob), theta)
    _check(loss.cpu().double().numpy(), grad.cpu().double().numpy(), ref, f"{prob.name}/{path}")


def test_cd_rejects_trainable_eps(V, torch):
    prob = _cd_square()
    p = V.assemble_problem(prob)
    dev = torch.device("cuda:0")
    th = torch.tensor(_params(prob), dtype=torch.float32, device=dev)
    eps = torch.ones(1, device=dev)
    loss = torch.zeros(4, device=dev)
    with pytest.raises(V.VpinnError) as ei:
        V.vpinn_loss_and_grad(p, V.loss_cfg(), th, eps=eps, loss=loss)
    assert ei.value.code == V.VPINN_E_INVALID


def test_cd_and_poisson_in_one_batch(V, torch):
    """A batch mixing Poisson and convection-diffusion instances: each matches the oracle."""
    from oracle import oracle as O
    probs = [_cd_square(), gen.poisson_sinsin_square("poisson", 4, 5, 3, 1, 40, 0.2, seed=22), _cd_gear_small()]
    gp = [V.assemble_problem(pr) for pr in probs]
    b = V.vpinn_batch_create(gp, V.loss_cfg(30, 3, 10.0, 0.0))
    th = np.stack([_params(pr, seed=30 + i) for i, pr in enumerate(probs)])
    dev = torch.device("cuda:0")
    T = torch.tensor(th, dtype=torch.float32, device=dev)
    n = V.vpinn_n_params(30, 3)
    losses = torch.zeros((len(probs), 4), device=dev)
    grads = torch.zeros((len(probs), n), device=dev)
    V.vpinn_batch_loss_and_grad(b, T, losses=losses, grads=grads)
    torch.cuda.synchronize()
    for i, pr in enumerate(probs):
        ref = O.problem_loss_grad(pr, O.assemble_problem(pr), th[i])
        _check(losses[i].cpu().double().numpy(), grads[i].cpu().double().numpy(), ref, pr.name)
    with pytest.raises(V.VpinnError):
        V.vpinn_batch_loss_and_grad(b, T, eps=torch.ones(len(probs), device=dev), losses=losses)


@pytest.mark.slow
def test_gear_cd_full_size_sampled(V, torch):
    """The full gear workload (14,000 elements): loss and gradient against the oracle."""
    from oracle import oracle as O
    prob = gen.config_gear_cd()
    theta = _params(prob)
    p = V.assemble_problem(prob)
    dev = torch.device("cuda:0")
    th = torch.tensor(theta, dtype=torch.float32, device=dev)
    loss = torch.zeros(4, device=dev)
    grad = torch.zeros(V.vpinn_n_params(30, 3), device=dev)
    V.vpinn_loss_and_grad(p, V.loss_cfg(30, 3, prob.tau, 0.0), th, loss=loss, grad=grad)
    torch.cuda.synchronize()
    ref = O.problem_loss_grad(prob, O.assemble_problem(prob), theta)
    _check(loss.cpu().double().numpy(), grad.cpu().double().numpy(), ref, "gear_cd")
