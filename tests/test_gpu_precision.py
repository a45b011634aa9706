"""The network's products are FP32-accurate (split-bf16 MFMA products, checked through the C ABI).

The library evaluates every dense product of the network as six bf16 piece products of operands split
exactly into three pieces.  These tests bound the error against the FP64 oracle tightly enough that a
split keeping only two pieces (16 significant bits, error near 2^-16) fails them, while FP32-accurate
products pass with margin.  Measured on MI355X: network values, relative L2 of u, u_x, u_y at most
3.3e-7 with three pieces against 3.2e-6 or more with two; C1/C2 gradients 1.2e-7 against 3.0e-6 to
3.7e-6.  (The general parity bars, 1e-5 on the loss and 1e-4 on the gradient, would not tell them
apart.)
"""
import numpy as np
import pytest

import vpinn_inputs as gen

pytestmark = pytest.mark.gpu

NET_RTOL_L2 = 1e-6
GRAD_RTOL_L2 = 1e-6
LOSS_RTOL = 1e-6


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


@pytest.mark.parametrize("H,L", [(30, 3), (32, 4)])
def test_network_values_and_tangents_at_fp32_accuracy(V, torch, H, L):
    from oracle import oracle as O
    theta = gen.glorot_params(H, L, seed=H + L, bias_scale=0.2)
    xy = gen.uniform(3, "precpts", 2 * 4096, -1.5, 1.5).reshape(-1, 2)
    dev = torch.device("cuda:0")
    th = torch.tensor(theta, dtype=torch.float32, device=dev)
    X = torch.tensor(xy, dtype=torch.float32, device=dev)
    out = [torch.empty(len(xy), dtype=torch.float32, device=dev) for _ in range(3)]
    V.vpinn_eval_network(H, L, th, X, *out)
    ref = O.mlp_eval(theta, H, L, X.cpu().double().numpy())
    for name, a, b in zip(("u", "u_x", "u_y"), out, ref):
        a = a.cpu().double().numpy()
        e = np.linalg.norm(a - b) / np.linalg.norm(b)
        assert e < NET_RTOL_L2, f"{name}: relative L2 error {e:.2e} (H={H}, L={L})"


@pytest.mark.parametrize("name", ["c1", "c2"])
def test_fused_gradient_at_fp32_accuracy(V, torch, name):
    from oracle import oracle as O
    prob = gen.CONFIGS[name]()
    theta = prob.params(bias_scale=0.1)
    p = V.vpinn_assemble(prob.mesh.xy, prob.mesh.quad, prob.quad_order, prob.test_order,
                         prob.f_amp, prob.f_kx, prob.f_ky)
    V.vpinn_set_boundary(p, prob.bnd_xy, prob.bnd_g)
    dev = torch.device("cuda:0")
    th = torch.tensor(theta, dtype=torch.float32, device=dev)
    loss = torch.full((4,), float("nan"), dtype=torch.float32, device=dev)
    grad = torch.full((V.vpinn_n_params(prob.width, prob.n_hidden),), float("nan"), dtype=torch.float32, device=dev)
    cfg = V.loss_cfg(prob.width, prob.n_hidden, prob.tau, prob.gamma, 0, V.VPINN_PATH_FUSED)
    V.vpinn_loss_and_grad(p, cfg, th, loss=loss, grad=grad)
    torch.cuda.synchronize()
    ref = O.problem_loss_grad(prob, O.assemble_problem(prob), theta)
    l, g = loss.cpu().double().numpy(), grad.cpu().double().numpy()
    rl = abs(l[0] - ref.loss[0]) / abs(ref.loss[0])
    rg = np.linalg.norm(g - ref.grad) / np.linalg.norm(ref.grad)
    assert rl < LOSS_RTOL, f"{name}: loss relative error {rl:.2e}"
    assert rg < GRAD_RTOL_L2, f"{name}: gradient relative L2 error {rg:.2e}"
