"""The batched path: many independent problems in one fused launch.

Every instance of a batch must match its own single-problem evaluation and the
FP64 oracle; a batched training step must match loss_and_grad + Adam per
instance; a captured step replayed through a HIP graph must reproduce eager
steps bit for bit.
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


def _mixed_instances():
    """Small instances covering every (n, N_t) of the batched workload, uneven sizes, one with sensors."""
    out = []
    specs = [(3, 4, 4, 3, 1), (7, 5, 6, 5, 3), (2, 9, 10, 5, 2), (6, 6, 4, 5, 7), (11, 3, 6, 3, 16), (1, 1, 10, 3, 4)]
    for i, (mx, my, n, nt, k) in enumerate(specs):
        p = gen.poisson_sinsin_square(f"mix{i}", 1, n, nt, k, 40, 0.2, seed=100 + i)
        p.mesh = gen.square_mesh(mx, my, 0.2, seed=100 + i)
        out.append(p)
    out[3].sens_xy = gen.sensor_points(30, 3)
    out[3].sens_u = gen.uniform(3, "su", 30, -1, 1)
    for p in out:
        p.gamma = 5.0
    return out


def _gpu(V, prob):
    p = V.vpinn_assemble(prob.mesh.xy, prob.mesh.quad, prob.quad_order, prob.test_order,
                         prob.f_amp, prob.f_kx, prob.f_ky)
    V.vpinn_set_boundary(p, prob.bnd_xy, prob.bnd_g)
    if len(prob.sens_xy):
        V.vpinn_set_sensors(p, prob.sens_xy, prob.sens_u)
    return p


def _params(probs):
    return np.stack([p.params(seed=7 + i, bias_scale=0.1) for i, p in enumerate(probs)])


def test_batch_matches_single_and_oracle(V, torch):
    from oracle import oracle as O
    probs = _mixed_instances()
    gp = [_gpu(V, p) for p in probs]
    cfg = V.loss_cfg(30, 3, 10.0, 5.0)
    b = V.vpinn_batch_create(gp, cfg)
    n = V.vpinn_n_params(30, 3)
    th = _params(probs)
    dev = torch.device("cuda:0")
    T = torch.tensor(th, dtype=torch.float32, device=dev)
    losses = torch.zeros((len(probs), 4), device=dev)
    grads = torch.zeros((len(probs), n), device=dev)
    V.vpinn_batch_loss_and_grad(b, T, losses=losses, grads=grads)
    torch.cuda.synchronize()
    for i, (prob, p) in enumerate(zip(probs, gp)):
        l1 = torch.zeros(4, device=dev)
        g1 = torch.zeros(n, device=dev)
        V.vpinn_loss_and_grad(p, V.loss_cfg(30, 3, 10.0, 5.0, path=V.VPINN_PATH_FUSED), T[i].contiguous(),
                              loss=l1, grad=g1)
        torch.cuda.synchronize()
        lb, gb = losses[i].cpu().double().numpy(), grads[i].cpu().double().numpy()
        ls, gs = l1.cpu().double().numpy(), g1.cpu().double().numpy()
        np.testing.assert_allclose(lb, ls, rtol=1e-6, atol=0)
        assert np.linalg.norm(gb - gs) / np.linalg.norm(gs) < 1e-5
        ref = O.problem_loss_grad(prob, O.assemble_problem(prob), th[i])
        assert abs(lb[0] - ref.loss[0]) / ref.loss[0] < 1e-5, (i, lb[0], ref.loss[0])
        assert np.linalg.norm(gb - ref.grad) / np.linalg.norm(ref.grad) < 1e-4


def test_batch_step_matches_adam_per_instance(V, torch):
    probs = _mixed_instances()
    gp = [_gpu(V, p) for p in probs]
    cfg = V.loss_cfg(30, 3, 10.0, 5.0)
    b = V.vpinn_batch_create(gp, cfg)
    n = V.vpinn_n_params(30, 3)
    th = _params(probs)
    dev = torch.device("cuda:0")
    T = torch.tensor(th, dtype=torch.float32, device=dev)
    M = torch.zeros_like(T)
    Vv = torch.zeros_like(T)
    step = torch.zeros(1, dtype=torch.int64, device=dev)
    losses = torch.zeros((len(probs), 4), device=dev)
    Ts = [torch.tensor(th[i], dtype=torch.float32, device=dev) for i in range(len(probs))]
    Ms = [torch.zeros(n, device=dev) for _ in probs]
    Vs = [torch.zeros(n, device=dev) for _ in probs]
    g = torch.zeros(n, device=dev)
    l1 = torch.zeros(4, device=dev)
    for t in range(1, 4):
        V.vpinn_batch_step(b, T, M, Vv, step, lr=1e-3, losses=losses)
        torch.cuda.synchronize()
        assert int(step.item()) == t
        for i, p in enumerate(gp):
            V.vpinn_loss_and_grad(p, V.loss_cfg(30, 3, 10.0, 5.0), Ts[i], loss=l1, grad=g)
            V.vpinn_adam_step(Ts[i], g, Ms[i], Vs[i], t, lr=1e-3)
            torch.cuda.synchronize()
            np.testing.assert_allclose(losses[i].cpu().numpy(), l1.cpu().numpy(), rtol=2e-5)
    for i in range(len(probs)):
        np.testing.assert_allclose(T[i].cpu().numpy(), Ts[i].cpu().numpy(), atol=1e-4, rtol=0)


def test_batch_graph_replay_matches_eager(V, torch):
    probs = _mixed_instances()
    gp = [_gpu(V, p) for p in probs]
    b = V.vpinn_batch_create(gp, V.loss_cfg(30, 3, 10.0, 5.0))
    th = _params(probs)
    dev = torch.device("cuda:0")

    def fresh():
        T = torch.tensor(th, dtype=torch.float32, device=dev)
        return T, torch.zeros_like(T), torch.zeros_like(T), torch.zeros(1, dtype=torch.int64, device=dev), \
            torch.zeros((len(probs), 4), device=dev)

    Te, Me, Ve, Se, Le = fresh()
    for _ in range(5):
        V.vpinn_batch_step(b, Te, Me, Ve, Se, losses=Le)
    Tg, Mg, Vg, Sg, Lg = fresh()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        V.vpinn_batch_capture(b, Tg, Mg, Vg, Sg, losses=Lg, stream=s)
    torch.cuda.synchronize()
    assert int(Sg.item()) == 0  # capture records, it does not run
    seen = []
    for r in range(5):
        V.vpinn_batch_replay(b, stream=s)
        s.synchronize()
        seen.append(Lg.clone())
        _ = (Tg * 1.0).sum().item()  # unrelated eager work between replays
    torch.cuda.synchronize()
    assert int(Sg.item()) == 5
    np.testing.assert_array_equal(Tg.cpu().numpy(), Te.cpu().numpy())
    np.testing.assert_array_equal(Mg.cpu().numpy(), Me.cpu().numpy())
    np.testing.assert_array_equal(Lg.cpu().numpy(), Le.cpu().numpy())


def test_batch_of_one_equals_single(V, torch):
    prob = gen.config_c1()
    p = _gpu(V, prob)
    b = V.vpinn_batch_create([p], V.loss_cfg(30, 3, prob.tau))
    th = torch.tensor(prob.params(bias_scale=0.1), dtype=torch.float32, device="cuda:0")
    n = th.numel()
    lb, gb = torch.zeros((1, 4), device="cuda:0"), torch.zeros((1, n), device="cuda:0")
    ls, gs = torch.zeros(4, device="cuda:0"), torch.zeros(n, device="cuda:0")
    V.vpinn_batch_loss_and_grad(b, th, losses=lb, grads=gb)
    V.vpinn_loss_and_grad(p, V.loss_cfg(30, 3, prob.tau), th, loss=ls, grad=gs)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(lb[0].cpu().numpy(), ls.cpu().numpy())
    np.testing.assert_array_equal(gb[0].cpu().numpy(), gs.cpu().numpy())


def _oracle_all(probs, thetas, want_grad=True):
    """The FP64 oracle for every instance, one instance per task on a pool of host threads (its C calls
    release the interpreter lock and it holds no global state, so the threads run in parallel)."""
    import os
    from concurrent.futures import ThreadPoolExecutor
    from oracle import oracle as O
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    order = sorted(range(len(probs)), key=lambda i: -probs[i].n_points)

    def one(i):
        return O.problem_loss_grad(probs[i], O.assemble_problem(probs[i]), thetas[i], want_grad=want_grad)

    with ThreadPoolExecutor(max_workers=max(1, min(16, n))) as ex:
        res = dict(zip(order, ex.map(one, order)))
    return [res[i] for i in range(len(probs))]


@pytest.fixture(scope="module")
def c5_oracle():
    """The 64-instance batched workload, its parameters (Glorot weights, U(+-0.1) biases) and the oracle's
    loss and gradient of every instance at them."""
    probs = gen.batched_instances(64, seed=0)
    th = _params(probs)
    return probs, th, _oracle_all(probs, th)


@pytest.mark.slow
def test_c5_batched_workload_full(V, torch, c5_oracle):
    """The 64-instance batched workload at full size (12,962,384 quadrature points): every instance's loss
    (1e-5 relative) and gradient (1e-4 relative L2) against the FP64 oracle, and every instance's loss
    against its own single-problem run."""
    probs, th, refs = c5_oracle
    gp = [_gpu(V, p) for p in probs]
    b = V.vpinn_batch_create(gp, V.loss_cfg(30, 3, 10.0, 0.0))
    n = V.vpinn_n_params(30, 3)
    dev = torch.device("cuda:0")
    T = torch.tensor(th, dtype=torch.float32, device=dev)
    L, Gd = _batch_eval(V, torch, b, T, 64, n)
    l1 = torch.zeros(4, device=dev)
    for i, p in enumerate(gp):
        V.vpinn_loss_and_grad(p, V.loss_cfg(30, 3, 10.0, 0.0), T[i].contiguous(), loss=l1)
        torch.cuda.synchronize()
        assert abs(L[i, 0] - float(l1[0])) / abs(float(l1[0])) < 1e-5, i
    lerr = [abs(L[i, 0] - refs[i].loss[0]) / refs[i].loss[0] for i in range(64)]
    gerr = [np.linalg.norm(Gd[i] - refs[i].grad) / np.linalg.norm(refs[i].grad) for i in range(64)]
    print(f"c5: max loss rel err {max(lerr):.2e}, max grad rel L2 err {max(gerr):.2e}")
    assert max(lerr) < 1e-5, int(np.argmax(lerr))
    assert max(gerr) < 1e-4, int(np.argmax(gerr))


@pytest.mark.slow
def test_c5_in_the_bench_launch_configuration(V, torch, c5_oracle):
    """C5 as bench.py times it: autotuned, one batched Adam step captured in a HIP graph and replayed.  The
    losses the first replay reports are the oracle's at the starting parameters, and its update of every
    instance's weights is the oracle's Adam step from the oracle's gradient (Kingma-Ba, lr 1e-3)."""
    from oracle import oracle as O
    probs, th, refs = c5_oracle
    gp = [_gpu(V, p) for p in probs]
    b = V.vpinn_batch_create(gp, V.loss_cfg(30, 3, 10.0, 0.0))
    dev = torch.device("cuda:0")
    T = torch.tensor(th, dtype=torch.float32, device=dev)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        V.vpinn_batch_autotune(b, T, reps=1, stream=s)
    M, Vv = torch.zeros_like(T), torch.zeros_like(T)
    step = torch.zeros(1, dtype=torch.int64, device=dev)
    losses = torch.zeros((64, 4), device=dev)
    V.vpinn_batch_capture(b, T, M, Vv, step, lr=1e-3, losses=losses, stream=s)
    th32 = T.cpu().double().numpy()
    V.vpinn_batch_replay(b, stream=s)
    s.synchronize()
    assert int(step.item()) == 1
    L = losses.cpu().double().numpy()
    got, gm, gv = (x.cpu().double().numpy() for x in (T, M, Vv))
    for i in range(64):
        assert abs(L[i, 0] - refs[i].loss[0]) / refs[i].loss[0] < 1e-5, i
        g = refs[i].grad
        t_ref, m_ref, v_ref = th32[i].copy(), np.zeros_like(g), np.zeros_like(g)
        O.adam(t_ref, g, m_ref, v_ref, 1, lr=1e-3)
        # the moments carry the gradient itself: its tolerance
        assert np.linalg.norm(gm[i] - m_ref) / np.linalg.norm(m_ref) < 1e-4, i
        assert np.linalg.norm(gv[i] - v_ref) / np.linalg.norm(v_ref) < 2e-4, i
        # the first step is lr * g / (|g| + eps), about lr * sign(g): where |g| is not below the FP32
        # gradient's own error the step taken must be the oracle's
        big = np.abs(g) > 1e-4 * np.linalg.norm(g)
        assert big.mean() > 0.9, i
        np.testing.assert_allclose((got[i] - th32[i])[big], (t_ref - th32[i])[big], rtol=0,
                                   atol=2e-5 * 1e-3 + 1e-7, err_msg=f"instance {i}")


def _all_shapes():
    """Mixed instances plus one that streams contraction rows (N_t = 7), one with large elements (n = 17) and
    one uniform mesh with a single shared premultiplier."""
    out = _mixed_instances()
    for i, (m, n, nt, jitter) in enumerate([(3, 6, 7, 0.2), (2, 17, 3, 0.2), (5, 6, 4, 0.0)]):
        p = gen.poisson_sinsin_square(f"shape{i}", m, n, nt, 2, 40, jitter, seed=200 + i)
        p.gamma = 5.0
        out.append(p)
    return out


def _batch_eval(V, torch, b, T, n_inst, n):
    dev = torch.device("cuda:0")
    losses = torch.zeros((n_inst, 4), device=dev)
    grads = torch.zeros((n_inst, n), device=dev)
    V.vpinn_batch_loss_and_grad(b, T, losses=losses, grads=grads)
    torch.cuda.synchronize()
    return losses.cpu().double().numpy(), grads.cpu().double().numpy()


def test_tunings_agree_with_oracle(V, torch):
    """Every tile shape computes the same loss and gradient (to FP32 rounding) as the FP64 oracle."""
    from oracle import oracle as O
    probs = _all_shapes()
    gp = [_gpu(V, p) for p in probs]
    b = V.vpinn_batch_create(gp, V.loss_cfg(30, 3, 10.0, 5.0))
    assert V.vpinn_batch_get_tuning(b) == (12, 0, 4, 0, 0)
    n = V.vpinn_n_params(30, 3)
    th = _params(probs)
    T = torch.tensor(th, dtype=torch.float32, device="cuda:0")
    refs = [O.problem_loss_grad(p, O.assemble_problem(p), th[i]) for i, p in enumerate(probs)]
    for tune in [(8, 2, 2, 0, 0), (16, 1, 8, 1, 0), (12, 0, 4, 1, 0), (12, 0, 4, 0, 0)]:
        V.vpinn_batch_set_tuning(b, *tune)
        assert V.vpinn_batch_get_tuning(b) == tune
        L, G = _batch_eval(V, torch, b, T, len(probs), n)
        for i, ref in enumerate(refs):
            assert abs(L[i, 0] - ref.loss[0]) / ref.loss[0] < 1e-5, (tune, i)
            assert np.linalg.norm(G[i] - ref.grad) / np.linalg.norm(ref.grad) < 1e-4, (tune, i)
        # a fixed tuning is bitwise reproducible
        L2, G2 = _batch_eval(V, torch, b, T, len(probs), n)
        assert np.array_equal(L, L2) and np.array_equal(G, G2)


def test_autotune_picks_a_valid_tuning_and_keeps_parity(V, torch):
    probs = _all_shapes()
    gp = [_gpu(V, p) for p in probs]
    b = V.vpinn_batch_create(gp, V.loss_cfg(30, 3, 10.0, 5.0))
    n = V.vpinn_n_params(30, 3)
    T = torch.tensor(_params(probs), dtype=torch.float32, device="cuda:0")
    L0, G0 = _batch_eval(V, torch, b, T, len(probs), n)
    best = V.vpinn_batch_autotune(b, T, reps=2)
    assert best == V.vpinn_batch_get_tuning(b)
    assert best[0] in (8, 12, 16) and 0 <= best[1] <= 2 and best[2] in (2, 4, 8) and best[3] in (0, 1)
    assert best[4] == 0  # the batch has shapes the one-pass step does not take
    L1, G1 = _batch_eval(V, torch, b, T, len(probs), n)
    np.testing.assert_allclose(L1, L0, rtol=1e-5)
    for i in range(len(probs)):
        assert np.linalg.norm(G1[i] - G0[i]) / np.linalg.norm(G0[i]) < 1e-5
    # the parameters are not modified by tuning
    np.testing.assert_array_equal(T.cpu().numpy(), _params(probs).astype(np.float32))
    with pytest.raises(V.VpinnError):
        V.vpinn_batch_set_tuning(b, 10, 0, 4)
    with pytest.raises(V.VpinnError):
        V.vpinn_batch_set_tuning(b, 12, 0, 4, 2)
    with pytest.raises(V.VpinnError):
        V.vpinn_batch_autotune(b, T, reps=0)


def test_capture_after_tuning_replays(V, torch):
    """A new tuning drops the captured graph; capturing again gives a graph that matches eager steps."""
    probs = _all_shapes()[:3]
    gp = [_gpu(V, p) for p in probs]
    b = V.vpinn_batch_create(gp, V.loss_cfg(30, 3, 10.0, 5.0))
    dev = torch.device("cuda:0")
    th = _params(probs)
    T = torch.tensor(th, dtype=torch.float32, device=dev)
    M, Vv = torch.zeros_like(T), torch.zeros_like(T)
    step = torch.zeros(1, dtype=torch.int64, device=dev)
    s = torch.cuda.Stream()
    V.vpinn_batch_capture(b, T, M, Vv, step, stream=s)
    V.vpinn_batch_set_tuning(b, 8, 1, 2)
    with pytest.raises(V.VpinnError):
        V.vpinn_batch_replay(b, stream=s)
    V.vpinn_batch_capture(b, T, M, Vv, step, stream=s)
    for _ in range(3):
        V.vpinn_batch_replay(b, stream=s)
    s.synchronize()
    T2 = torch.tensor(th, dtype=torch.float32, device=dev)
    M2, V2 = torch.zeros_like(T2), torch.zeros_like(T2)
    step2 = torch.zeros(1, dtype=torch.int64, device=dev)
    for _ in range(3):
        V.vpinn_batch_step(b, T2, M2, V2, step2, stream=s)
    s.synchronize()
    assert int(step.item()) == 3 and int(step2.item()) == 3
    assert torch.equal(T, T2) and torch.equal(M, M2) and torch.equal(Vv, V2)


def test_changed_problem_makes_the_batch_refuse_until_replanned(V, torch):
    """The plan points into the problems' point buffers: after a boundary, sensor or shared-point change every
    batch call is refused (no stale pointers are used) until the plan is rebuilt, which then matches the oracle
    on the new data."""
    from oracle import oracle as O
    probs = _mixed_instances()[:3]
    gp = [_gpu(V, p) for p in probs]
    b = V.vpinn_batch_create(gp, V.loss_cfg(30, 3, 10.0, 5.0))
    n = V.vpinn_n_params(30, 3)
    th = _params(probs)
    T = torch.tensor(th, dtype=torch.float32, device="cuda:0")
    _batch_eval(V, torch, b, T, len(probs), n)
    dev = torch.device("cuda:0")
    M, Vv = torch.zeros_like(T), torch.zeros_like(T)
    S = torch.zeros(1, dtype=torch.int64, device=dev)
    s = torch.cuda.Stream()
    V.vpinn_batch_capture(b, T.clone(), M, Vv, S, stream=s)
    probs[1].bnd_xy = gen.square_boundary_points(48)
    probs[1].bnd_g = np.zeros(48)
    V.vpinn_set_boundary(gp[1], probs[1].bnd_xy, probs[1].bnd_g)
    for call in (lambda: _batch_eval(V, torch, b, T, len(probs), n),
                 lambda: V.vpinn_batch_replay(b, stream=s),
                 lambda: V.vpinn_batch_step(b, T.clone(), M, Vv, S),
                 lambda: V.vpinn_batch_capture(b, T.clone(), M, Vv, S, stream=s)):
        with pytest.raises(V.VpinnError) as ei:
            call()
        assert ei.value.code == V.VPINN_E_INVALID
    V.vpinn_batch_set_tuning(b, 12, 0, 4)
    L, G = _batch_eval(V, torch, b, T, len(probs), n)
    for i, p in enumerate(probs):
        ref = O.problem_loss_grad(p, O.assemble_problem(p), th[i])
        assert abs(L[i, 0] - ref.loss[0]) / ref.loss[0] < 1e-5, i
        assert np.linalg.norm(G[i] - ref.grad) / np.linalg.norm(ref.grad) < 1e-4, i
    with pytest.raises(V.VpinnError):  # the graph captured before the change is gone
        V.vpinn_batch_replay(b, stream=s)
    V.vpinn_set_shared_points(gp[0], probs[0].mesh.xy, probs[0].mesh.quad)
    with pytest.raises(V.VpinnError):
        _batch_eval(V, torch, b, T, len(probs), n)


def test_stored_activations_match_recompute(V, torch):
    """Reading the forward pass's activations instead of recomputing them gives the same loss and gradient
    (the same arithmetic, so equal up to FP32 summation order), for one and two network outputs."""
    probs = _all_shapes()
    gp = [_gpu(V, p) for p in probs]
    b = V.vpinn_batch_create(gp, V.loss_cfg(30, 3, 10.0, 5.0))
    n = V.vpinn_n_params(30, 3)
    T = torch.tensor(_params(probs), dtype=torch.float32, device="cuda:0")
    for fw in (8, 16):
        V.vpinn_batch_set_tuning(b, fw, 0, 4, 0)
        L0, G0 = _batch_eval(V, torch, b, T, len(probs), n)
        V.vpinn_batch_set_tuning(b, fw, 0, 4, 1)
        L1, G1 = _batch_eval(V, torch, b, T, len(probs), n)
        np.testing.assert_allclose(L1, L0, rtol=1e-6)
        for i in range(len(probs)):
            assert np.linalg.norm(G1[i] - G0[i]) <= 1e-6 * np.linalg.norm(G0[i]), (fw, i)


def test_c2_in_the_bench_launch_configuration(V, torch):
    """C2 exactly as bench.py times it: a batch of one, autotuned, one Adam step captured in a HIP graph and
    replayed.  The loss each replay reports is the oracle's at the parameters it started from, and the first
    replay's update is the oracle's Adam step (Kingma-Ba, lr 1e-3)."""
    from oracle import oracle as O
    prob = gen.config_c2()
    theta = prob.params()
    p = V.assemble_problem(prob)
    b = V.vpinn_batch_create([p], V.loss_cfg(prob.width, prob.n_hidden, prob.tau, prob.gamma))
    dev = torch.device("cuda:0")
    th = torch.tensor(theta, dtype=torch.float32, device=dev).reshape(1, -1).contiguous()
    V.vpinn_batch_autotune(b, th, reps=2)
    m, v = torch.zeros_like(th), torch.zeros_like(th)
    step = torch.zeros(1, dtype=torch.int64, device=dev)
    losses = torch.zeros((1, 4), device=dev)
    s = torch.cuda.Stream()
    V.vpinn_batch_capture(b, th, m, v, step, lr=1e-3, losses=losses, stream=s)
    asm = O.assemble_problem(prob)
    th32 = th.cpu().double().numpy()[0]
    V.vpinn_batch_replay(b, stream=s)
    s.synchronize()
    ref = O.problem_loss_grad(prob, asm, th32)
    assert abs(losses[0, 0].item() - ref.loss[0]) / ref.loss[0] < 1e-5
    t_ref, m_ref, v_ref = th32.copy(), np.zeros_like(th32), np.zeros_like(th32)
    O.adam(t_ref, ref.grad, m_ref, v_ref, 1, lr=1e-3)
    got = th.cpu().double().numpy()[0]
    # the update is lr * sign(g) on the first step, except where |g| is tiny: compare the step taken
    np.testing.assert_allclose(got - th32, t_ref - th32, rtol=0, atol=2e-5 * 1e-3 + 1e-7)
    # a second replay reports the loss at the updated parameters
    th_after = th.cpu().double().numpy()[0]
    V.vpinn_batch_replay(b, stream=s)
    s.synchronize()
    ref2 = O.problem_loss_grad(prob, asm, th_after, want_grad=False)
    assert abs(losses[0, 0].item() - ref2.loss[0]) / ref2.loss[0] < 1e-5
    assert int(step.item()) == 2


def test_batch_step_trains_eps_like_single_problem(V, torch):
    """The batched step with a trainable eps per instance (the inverse problem of Sec. 4.7.1): each step's
    losses, the weights and eps after it match the single-problem loss and gradient (with dL/deps) followed by
    Adam on the weights and on eps, instance by instance."""
    probs = _mixed_instances()[:4]
    gp = [_gpu(V, p) for p in probs]
    cfg = V.loss_cfg(30, 3, 10.0, 5.0)
    b = V.vpinn_batch_create(gp, cfg)
    n = V.vpinn_n_params(30, 3)
    th = _params(probs)
    eps0 = np.array([2.0, 0.7, 1.3, 0.4], dtype=np.float32)
    dev = torch.device("cuda:0")
    T = torch.tensor(th, dtype=torch.float32, device=dev)
    M, Vv = torch.zeros_like(T), torch.zeros_like(T)
    E = torch.tensor(eps0, device=dev)
    Em, Ev = torch.zeros_like(E), torch.zeros_like(E)
    step = torch.zeros(1, dtype=torch.int64, device=dev)
    losses = torch.zeros((len(probs), 4), device=dev)
    Ts = [torch.tensor(th[i], dtype=torch.float32, device=dev) for i in range(len(probs))]
    Ms = [torch.zeros(n, device=dev) for _ in probs]
    Vs = [torch.zeros(n, device=dev) for _ in probs]
    Es = [torch.tensor([eps0[i]], device=dev) for i in range(len(probs))]
    Ems = [torch.zeros(1, device=dev) for _ in probs]
    Evs = [torch.zeros(1, device=dev) for _ in probs]
    g, ge, l1 = torch.zeros(n, device=dev), torch.zeros(1, device=dev), torch.zeros(4, device=dev)
    for t in range(1, 4):
        V.vpinn_batch_step(b, T, M, Vv, step, lr=1e-3, losses=losses, diff=E, diff_m=Em, diff_v=Ev)
        torch.cuda.synchronize()
        for i, p in enumerate(gp):
            V.vpinn_loss_and_grad(p, cfg, Ts[i], eps=Es[i], loss=l1, grad=g, grad_eps=ge)
            V.vpinn_adam_step(Ts[i], g, Ms[i], Vs[i], t, lr=1e-3)
            V.vpinn_adam_step(Es[i], ge, Ems[i], Evs[i], t, lr=1e-3)
            torch.cuda.synchronize()
            np.testing.assert_allclose(losses[i].cpu().numpy(), l1.cpu().numpy(), rtol=2e-5)
    for i in range(len(probs)):
        np.testing.assert_allclose(T[i].cpu().numpy(), Ts[i].cpu().numpy(), atol=1e-4, rtol=0)
        assert abs(float(E[i]) - float(Es[i])) < 1e-6, i
        np.testing.assert_allclose(float(Em[i]), float(Ems[i][0]), rtol=1e-4)
    # eps moved: three Adam steps of lr 1e-3 each
    assert np.all(np.abs(E.cpu().numpy() - eps0) > 2e-3)


def test_batch_eps_arguments_are_checked(V, torch):
    """eps and its two moments go together, and problems with folded coefficients take no eps."""
    probs = _mixed_instances()[:2]
    gp = [_gpu(V, p) for p in probs]
    b = V.vpinn_batch_create(gp, V.loss_cfg(30, 3, 10.0, 5.0))
    dev = torch.device("cuda:0")
    T = torch.tensor(_params(probs), dtype=torch.float32, device=dev)
    M, Vv = torch.zeros_like(T), torch.zeros_like(T)
    S = torch.zeros(1, dtype=torch.int64, device=dev)
    E = torch.ones(2, device=dev)
    for kw in ({"diff": E}, {"diff": E, "diff_m": E.clone()}, {"diff_m": E, "diff_v": E.clone()}):
        with pytest.raises(V.VpinnError) as ei:
            V.vpinn_batch_step(b, T, M, Vv, S, **kw)
        assert ei.value.code == V.VPINN_E_INVALID
    pr = probs[0]
    pc = V.vpinn_assemble(pr.mesh.xy, pr.mesh.quad, pr.quad_order, pr.test_order, pr.f_amp, pr.f_kx, pr.f_ky,
                          cd=(1.0, 0.1, 0.0))
    V.vpinn_set_boundary(pc, pr.bnd_xy, pr.bnd_g)
    bc = V.vpinn_batch_create([pc], V.loss_cfg(30, 3, 10.0, 0.0))
    T1 = T[:1].contiguous()
    e1 = torch.ones(1, device=dev)
    with pytest.raises(V.VpinnError) as ei:
        V.vpinn_batch_step(bc, T1, torch.zeros_like(T1), torch.zeros_like(T1), S, diff=e1,
                           diff_m=torch.zeros(1, device=dev), diff_v=torch.zeros(1, device=dev))
    assert ei.value.code == V.VPINN_E_INVALID
    assert int(S.item()) == 0  # nothing ran


@pytest.mark.slow
def test_c4_in_the_bench_launch_configuration(V, torch):
    """C4 (the inverse problem: eps trained beside the weights, 4,096 elements, 1,000 noisy sensors) as
    bench.py times it: a batch of one, autotuned, one step captured in a HIP graph with eps, its moments
    and the weights all updated by it.  The first replay's loss is the oracle's at (theta, eps = 2), its
    update of the weights and of eps is the oracle's Adam step from the oracle's dL/dtheta and dL/deps, and
    the second replay's loss is the oracle's at the updated (theta, eps)."""
    from oracle import oracle as O
    prob = gen.config_c4()
    theta = prob.params()
    p = V.assemble_problem(prob)
    b = V.vpinn_batch_create([p], V.loss_cfg(prob.width, prob.n_hidden, prob.tau, prob.gamma))
    dev = torch.device("cuda:0")
    th = torch.tensor(theta, dtype=torch.float32, device=dev).reshape(1, -1).contiguous()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        V.vpinn_batch_autotune(b, th, reps=2, stream=s)
    m, v = torch.zeros_like(th), torch.zeros_like(th)
    E = torch.tensor([prob.eps_init], dtype=torch.float32, device=dev)
    Em, Ev = torch.zeros_like(E), torch.zeros_like(E)
    step = torch.zeros(1, dtype=torch.int64, device=dev)
    losses = torch.zeros((1, 4), device=dev)
    V.vpinn_batch_capture(b, th, m, v, step, lr=1e-3, losses=losses, stream=s, diff=E, diff_m=Em, diff_v=Ev)
    asm = O.assemble_problem(prob)
    th32 = th.cpu().double().numpy()[0]
    V.vpinn_batch_replay(b, stream=s)
    s.synchronize()
    ref = O.problem_loss_grad(prob, asm, th32, eps=prob.eps_init)
    assert abs(losses[0, 0].item() - ref.loss[0]) / ref.loss[0] < 1e-5
    g = ref.grad
    t_ref, m_ref, v_ref = th32.copy(), np.zeros_like(g), np.zeros_like(g)
    O.adam(t_ref, g, m_ref, v_ref, 1, lr=1e-3)
    got = th.cpu().double().numpy()[0]
    assert np.linalg.norm(m.cpu().double().numpy()[0] - m_ref) / np.linalg.norm(m_ref) < 1e-4
    big = np.abs(g) > 1e-4 * np.linalg.norm(g)
    assert big.mean() > 0.9
    np.testing.assert_allclose((got - th32)[big], (t_ref - th32)[big], rtol=0, atol=2e-5 * 1e-3 + 1e-7)
    # dL/deps = 2 c_v sum R A cancels heavily at a random network (here by about 1e3): its FP32 error is
    # bounded by the size of the terms, sum |2 c_v R A|, not by its own size
    rr = O.loss_grad(asm, th32, prob.width, prob.n_hidden, prob.bnd_xy, prob.bnd_g, prob.sens_xy, prob.sens_u,
                     eps=prob.eps_init, tau=prob.tau, gamma=prob.gamma, want_grad=False, want_R=True).R
    cv = 1.0 / prob.test_order ** 2
    terms = float(np.sum(np.abs(2 * cv * rr * (rr + asm.F) / prob.eps_init)))
    ge_gpu = float(Em[0]) / (1 - 0.9)  # the first moment after one step is (1 - beta1) g
    bound = 1e-4 * abs(ref.grad_eps) + 1e-5 * terms
    assert abs(ge_gpu - ref.grad_eps) <= bound, (ge_gpu, ref.grad_eps, terms)
    e_ref, em_ref, ev_ref = np.array([prob.eps_init]), np.zeros(1), np.zeros(1)
    O.adam(e_ref, np.array([ref.grad_eps]), em_ref, ev_ref, 1, lr=1e-3)
    assert abs(ref.grad_eps) > 10 * bound  # the sign of the step is decided
    np.testing.assert_allclose(float(E[0]), e_ref[0], rtol=0, atol=1e-6)
    assert (float(E[0]) - prob.eps_init) * ref.grad_eps < 0  # eps moved against its gradient
    th_after, e_after = got.copy(), float(E[0])
    V.vpinn_batch_replay(b, stream=s)
    s.synchronize()
    ref2 = O.problem_loss_grad(prob, asm, th_after, eps=e_after, want_grad=False)
    assert abs(losses[0, 0].item() - ref2.loss[0]) / ref2.loss[0] < 1e-5
    assert int(step.item()) == 2


def _one_pass_shapes():
    """Instances the one-pass step takes, chosen to exercise its grouping: N_quad from 4 (32 elements a group) to
    121 (one element of eight tiles, the last with nine points), element counts that do not fill the last group, no
    boundary points, boundary sets of one and of three groups, sensors, and a uniform mesh (one shared G)."""
    specs = [  # (mx, my, n, N_t, k, boundary points, jitter)
        (3, 4, 2, 1, 1, 40, 0.2), (5, 3, 3, 2, 2, 0, 0.2), (7, 5, 6, 5, 3, 300, 0.2), (1, 1, 11, 5, 2, 40, 0.2),
        (2, 3, 4, 3, 4, 128, 0.2), (9, 7, 5, 5, 5, 44, 0.2), (4, 4, 6, 4, 1, 40, 0.0)]
    out = []
    for i, (mx, my, n, nt, k, nd, jit) in enumerate(specs):
        p = gen.poisson_sinsin_square(f"op{i}", 1, n, nt, k, max(nd, 4), jit, seed=300 + i)
        p.mesh = gen.square_mesh(mx, my, jit, seed=300 + i)
        if nd == 0:
            p.bnd_xy, p.bnd_g = np.zeros((0, 2)), np.zeros(0)
        out.append(p)
    out[2].sens_xy = gen.sensor_points(70, 5)
    out[2].sens_u = gen.uniform(5, "su", 70, -1, 1)
    for p in out:
        p.gamma = 5.0
    return out


def test_one_pass_matches_oracle_and_four_kernels(V, torch):
    """The one-pass step (forward, contraction and reverse sweep in one kernel) computes each instance's loss and
    gradient to the oracle's tolerances, and agrees with the four-kernel step to FP32 summation order; a fixed
    tuning is bitwise reproducible, and a loss-only call gives the same losses."""
    from oracle import oracle as O
    probs = _one_pass_shapes()
    gp = [_gpu(V, p) for p in probs]
    b = V.vpinn_batch_create(gp, V.loss_cfg(30, 3, 10.0, 5.0))
    n = V.vpinn_n_params(30, 3)
    th = _params(probs)
    T = torch.tensor(th, dtype=torch.float32, device="cuda:0")
    L4, G4 = _batch_eval(V, torch, b, T, len(probs), n)
    V.vpinn_batch_set_tuning(b, 12, 0, 4, 0, 1)
    assert V.vpinn_batch_get_tuning(b) == (12, 0, 4, 0, 1)
    L1, G1 = _batch_eval(V, torch, b, T, len(probs), n)
    for i, p in enumerate(probs):
        print(f"one-pass instance {i}: n={p.quad_order} N_t={p.test_order} elements={p.n_elem}", flush=True)
        ref = O.problem_loss_grad(p, O.assemble_problem(p), th[i])
        for k in range(4):
            assert abs(L1[i, k] - ref.loss[k]) <= 1e-5 * abs(ref.loss[k]) + 1e-12, (i, k, L1[i, k], ref.loss[k])
        assert np.linalg.norm(G1[i] - ref.grad) / np.linalg.norm(ref.grad) < 1e-4, i
        np.testing.assert_allclose(L1[i], L4[i], rtol=2e-6, atol=1e-12)
        assert np.linalg.norm(G1[i] - G4[i]) <= 1e-5 * np.linalg.norm(G4[i]), i
    L2, G2 = _batch_eval(V, torch, b, T, len(probs), n)
    assert np.array_equal(L1, L2) and np.array_equal(G1, G2)
    lo = torch.zeros((len(probs), 4), device="cuda:0")
    V.vpinn_batch_loss_and_grad(b, T, losses=lo)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(lo.cpu().double().numpy(), L1)


def test_one_pass_step_with_eps_matches_eager_and_graph(V, torch):
    """The one-pass batched step training eps beside the weights: three eager steps against three replays of the
    captured step (bitwise); and one step against the four-kernel step: the same losses and the same first Adam
    moment (a tenth of the gradient) to FP32 summation order."""
    probs = _one_pass_shapes()[:5]
    gp = [_gpu(V, p) for p in probs]
    b = V.vpinn_batch_create(gp, V.loss_cfg(30, 3, 10.0, 5.0))
    th = _params(probs)
    dev = torch.device("cuda:0")
    eps0 = np.array([2.0, 0.5, 1.0, 1.5, 0.8], dtype=np.float32)

    def run(one_pass, graph, steps=3):
        V.vpinn_batch_set_tuning(b, 12, 0, 4, 0, one_pass)
        T = torch.tensor(th, dtype=torch.float32, device=dev)
        M, Vv = torch.zeros_like(T), torch.zeros_like(T)
        E = torch.tensor(eps0, device=dev)
        Em, Ev = torch.zeros_like(E), torch.zeros_like(E)
        S = torch.zeros(1, dtype=torch.int64, device=dev)
        Ls = torch.zeros((len(probs), 4), device=dev)
        s = torch.cuda.Stream()
        kw = dict(lr=1e-3, losses=Ls, stream=s, diff=E, diff_m=Em, diff_v=Ev)
        if graph:
            V.vpinn_batch_capture(b, T, M, Vv, S, **kw)
        seen = []
        for _ in range(steps):
            if graph:
                V.vpinn_batch_replay(b, stream=s)
            else:
                V.vpinn_batch_step(b, T, M, Vv, S, **kw)
            s.synchronize()
            seen.append(Ls.cpu().numpy().copy())
        assert int(S.item()) == steps
        return T.cpu().numpy(), E.cpu().numpy(), np.stack(seen), M.cpu().double().numpy()

    Te, Ee, Le, _ = run(1, False)
    Tg, Eg, Lg, _ = run(1, True)
    np.testing.assert_array_equal(Tg, Te)
    np.testing.assert_array_equal(Eg, Ee)
    np.testing.assert_array_equal(Lg, Le)
    # instance 0 has two GLL points per direction, the element corners, where every test function vanishes:
    # G = F = 0, so R = 0 and dL/deps = 0 and Adam leaves its eps; every other eps moves
    assert Ee[0] == eps0[0] and np.all(Ee[1:] != eps0[1:])
    _, _, L1, M1 = run(1, False, steps=1)
    _, _, L4, M4 = run(0, False, steps=1)
    np.testing.assert_allclose(L1, L4, rtol=2e-6)
    for i in range(len(probs)):
        assert np.linalg.norm(M1[i] - M4[i]) <= 1e-5 * np.linalg.norm(M4[i]), i


def test_one_pass_refuses_what_it_does_not_take(V, torch):
    """Elements above 128 points, more than 32 test functions and shared points make the one-pass tuning
    unsupported; the batch keeps its plan."""
    for n, nt in ((12, 3), (6, 7)):
        p = gen.poisson_sinsin_square("big", 2, n, nt, 2, 40, 0.2, seed=9)
        b = V.vpinn_batch_create([_gpu(V, p)], V.loss_cfg(30, 3, 10.0, 0.0))
        with pytest.raises(V.VpinnError) as ei:
            V.vpinn_batch_set_tuning(b, 12, 0, 4, 0, 1)
        assert ei.value.code == V.VPINN_E_UNSUPPORTED
        assert V.vpinn_batch_get_tuning(b) == (12, 0, 4, 0, 0)
    p = gen.poisson_sinsin_square("shared", 3, 5, 3, 2, 40, 0.2, seed=9)
    g = _gpu(V, p)
    V.vpinn_set_shared_points(g, p.mesh.xy, p.mesh.quad)
    b = V.vpinn_batch_create([g], V.loss_cfg(30, 3, 10.0, 0.0))
    with pytest.raises(V.VpinnError) as ei:
        V.vpinn_batch_set_tuning(b, 12, 0, 4, 0, 1)
    assert ei.value.code == V.VPINN_E_UNSUPPORTED
    with pytest.raises(V.VpinnError) as ei:
        V.vpinn_batch_set_tuning(b, 12, 0, 4, 1, 1)  # nothing to store in the one-pass step
    assert ei.value.code == V.VPINN_E_INVALID


@pytest.mark.slow
def test_c5_one_pass_full(V, torch, c5_oracle):
    """The 64-instance workload with the one-pass step: every instance's loss and gradient against the oracle."""
    probs, th, refs = c5_oracle
    gp = [_gpu(V, p) for p in probs]
    b = V.vpinn_batch_create(gp, V.loss_cfg(30, 3, 10.0, 0.0))
    V.vpinn_batch_set_tuning(b, 12, 0, 4, 0, 1)
    n = V.vpinn_n_params(30, 3)
    T = torch.tensor(th, dtype=torch.float32, device="cuda:0")
    L, Gd = _batch_eval(V, torch, b, T, 64, n)
    lerr = [abs(L[i, 0] - refs[i].loss[0]) / refs[i].loss[0] for i in range(64)]
    gerr = [np.linalg.norm(Gd[i] - refs[i].grad) / np.linalg.norm(refs[i].grad) for i in range(64)]
    print(f"c5 one-pass: max loss rel err {max(lerr):.2e}, max grad rel L2 err {max(gerr):.2e}")
    assert max(lerr) < 1e-5, int(np.argmax(lerr))
    assert max(gerr) < 1e-4, int(np.argmax(gerr))


@pytest.mark.parametrize("width,n_hidden", [(32, 3), (31, 2), (16, 4), (30, 1)])
def test_widths_without_and_with_a_padding_neuron(V, torch, width, n_hidden):
    """The hidden layers' bias gradients come out of the weight-gradient products through padding slot 31 when the
    width is below 32, and out of column sums at width 32: both against the oracle, on both step kernels."""
    from oracle import oracle as O
    probs = _mixed_instances()[:3]
    for p in probs:
        p.width, p.n_hidden = width, n_hidden
    gp = [_gpu(V, p) for p in probs]
    b = V.vpinn_batch_create(gp, V.loss_cfg(width, n_hidden, 10.0, 5.0))
    n = V.vpinn_n_params(width, n_hidden)
    th = np.stack([gen.glorot_params(width, n_hidden, 40 + i, 0.1, name=f"w{width}") for i in range(len(probs))])
    T = torch.tensor(th, dtype=torch.float32, device="cuda:0")
    refs = [O.problem_loss_grad(p, O.assemble_problem(p), th[i]) for i, p in enumerate(probs)]
    for one_pass in (0, 1):
        V.vpinn_batch_set_tuning(b, 12, 0, 4, 0, one_pass)
        L, G = _batch_eval(V, torch, b, T, len(probs), n)
        for i, ref in enumerate(refs):
            assert abs(L[i, 0] - ref.loss[0]) / ref.loss[0] < 1e-5, (one_pass, i)
            assert np.linalg.norm(G[i] - ref.grad) / np.linalg.norm(ref.grad) < 1e-4, (one_pass, i)
