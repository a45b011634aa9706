"""The torch.autograd wrapper: gradients equal the library's, an optimiser loop runs, and the
inverse problem's eps receives its gradient."""
import numpy as np
import pytest

import vpinn_inputs as gen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


def _problem(V, prob):
    p = V.vpinn_assemble(prob.mesh.xy, prob.mesh.quad, prob.quad_order, prob.test_order,
                         prob.f_amp, prob.f_kx, prob.f_ky)
    V.vpinn_set_boundary(p, prob.bnd_xy, prob.bnd_g)
    if len(prob.sens_xy):
        V.vpinn_set_sensors(p, prob.sens_xy, prob.sens_u)
    return p


def test_autograd_matches_library_and_oracle(torch):
    from oracle import oracle as O
    from paper_2404_12063_amd import vpinn as V
    from paper_2404_12063_amd.autograd import vpinn_loss
    prob = gen.config_c1()
    p = _problem(V, prob)
    th = prob.params(bias_scale=0.1)
    T = torch.tensor(th, dtype=torch.float32, device="cuda:0", requires_grad=True)
    L, comps = vpinn_loss(T, p, V.loss_cfg(30, 3, prob.tau))
    (3.0 * L).backward()
    ref = O.problem_loss_grad(prob, O.assemble_problem(prob), th)
    assert abs(float(L) - ref.loss[0]) / ref.loss[0] < 1e-5
    g = T.grad.cpu().double().numpy()
    assert np.linalg.norm(g - 3.0 * ref.grad) / np.linalg.norm(3.0 * ref.grad) < 1e-4
    np.testing.assert_allclose(comps.cpu().numpy()[1:3], ref.loss[1:3], rtol=1e-5)


def test_autograd_eps_gradient_and_adam_loop(torch):
    from oracle import oracle as O
    from paper_2404_12063_amd import vpinn as V
    from paper_2404_12063_amd.autograd import vpinn_loss
    c4 = gen.config_c4()
    prob = gen.Problem("c4ag", gen.square_mesh(8, 8, 0.2, seed=2), 6, 5, c4.f_amp, c4.f_kx, c4.f_ky,
                       c4.bnd_xy[::4], c4.bnd_g[::4], c4.sens_xy[:100], c4.sens_u[:100], tau=10.0, gamma=10.0)
    p = _problem(V, prob)
    th = prob.params(bias_scale=0.1)
    T = torch.tensor(th, dtype=torch.float32, device="cuda:0", requires_grad=True)
    E = torch.tensor([2.0], dtype=torch.float32, device="cuda:0", requires_grad=True)
    cfg = V.loss_cfg(30, 3, 10.0, 10.0)
    L, _ = vpinn_loss(T, p, cfg, E)
    L.backward()
    ref = O.problem_loss_grad(prob, O.assemble_problem(prob), th, eps=2.0)
    assert abs(float(E.grad) - ref.grad_eps) / abs(ref.grad_eps) < 1e-4
    opt = torch.optim.Adam([T, E], lr=1e-3)
    first = None
    for _ in range(20):
        opt.zero_grad()
        L, _ = vpinn_loss(T, p, cfg, E)
        L.backward()
        opt.step()
        first = float(L) if first is None else first
    assert float(L) < first
