"""The allocation-free prediction-error call (vpinn_eval_error_noalloc) through the C ABI: two calls in a row
on one device, the second with fewer points than the first, each against vpinn_eval_error on the same inputs
(the same kernels in the same order, so bit for bit), and its size limit."""
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


def _case(torch, n, seed, heads=1):
    dev = torch.device("cuda:0")
    xy = np.stack([gen.uniform(seed, "noalloc/x", n, 0.0, 1.0), gen.uniform(seed, "noalloc/y", n, 0.0, 1.0)], 1)
    ref = np.sin(2 * np.pi * xy[:, 0]) * np.sin(2 * np.pi * xy[:, 1])
    th = gen.glorot_params(30, 3, seed, 0.1, name="noalloc/params", heads=heads)
    return (torch.tensor(xy, dtype=torch.float32, device=dev).contiguous(),
            torch.tensor(ref, dtype=torch.float32, device=dev),
            torch.tensor(th, dtype=torch.float32, device=dev))


@pytest.mark.parametrize("heads,output", [(1, 0), (2, 1)])
def test_noalloc_matches_the_allocating_call_twice(V, torch, heads, output):
    dev = torch.device("cuda:0")
    for n, seed in ((300_001, 1), (1_000, 2)):   # the second call is smaller than the first
        xy, ref, th = _case(torch, n, seed, heads)
        print(f"noalloc heads={heads} output={output} n={n}", flush=True)
        a = torch.full((3,), -1.0, dtype=torch.float64, device=dev)
        b = torch.full((3,), -2.0, dtype=torch.float64, device=dev)
        V.vpinn_eval_error_noalloc(30, 3, th, xy, ref, a, n_outputs=heads, output=output)
        V.vpinn_eval_error(30, 3, th, xy, ref, b, n_outputs=heads, output=output)
        torch.cuda.synchronize()
        ga, gb = a.cpu().numpy(), b.cpu().numpy()
        assert np.array_equal(ga, gb), (n, ga, gb)
        assert np.all(np.isfinite(ga)) and ga[0] > 0 and ga[1] >= ga[0] and ga[2] > 0


def test_noalloc_against_the_oracle(V, torch):
    from oracle import oracle as O
    xy, ref, th = _case(torch, 5_000, 3)
    out = torch.zeros(3, dtype=torch.float64, device="cuda:0")
    V.vpinn_eval_error_noalloc(30, 3, th, xy, ref, out)
    torch.cuda.synchronize()
    want = O.prediction_error(th.cpu().double().numpy(), 30, 3, xy.cpu().double().numpy(), ref.cpu().double().numpy())
    np.testing.assert_allclose(out.cpu().numpy(), want, rtol=1e-5, atol=1e-6)


def test_noalloc_refuses_more_points_than_its_workspace(V, torch):
    xy, ref, th = _case(torch, 16, 4)
    out = torch.zeros(3, dtype=torch.float64, device="cuda:0")
    # the size is checked on the host before anything is launched
    with pytest.raises(V.VpinnError) as ei:
        V.vpinn_eval_error_noalloc(30, 3, th, xy, ref, out, n=V.VPINN_NOALLOC_MAX_POINTS + 1)
    assert ei.value.code == V.VPINN_E_INVALID
    assert "VPINN_NOALLOC_MAX_POINTS" in V.vpinn_last_error()
    with pytest.raises(V.VpinnError):
        V.vpinn_eval_error_noalloc(30, 3, th, xy, ref, out, n=0)
