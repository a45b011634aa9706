"""Prediction and its error on a grid (the accuracy evaluation of Sec. 4: mean absolute error on a 100 x 100
grid, point-wise errors of u and of the predicted diffusion coefficient) against the FP64 oracle."""
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


def _grid(m):
    t = (np.arange(m) + 0.3) / m
    X, Y = np.meshgrid(t, t, indexing="xy")
    return np.stack([X.ravel(), Y.ravel()], 1)


def _err(V, torch, H, L, theta, xy, ref, heads=1, output=0):
    dev = torch.device("cuda:0")
    out = torch.zeros(3, dtype=torch.float64, device=dev)
    V.vpinn_eval_error(H, L, torch.tensor(theta, dtype=torch.float32, device=dev),
                       torch.tensor(xy, dtype=torch.float32, device=dev),
                       torch.tensor(ref, dtype=torch.float32, device=dev), out, n_outputs=heads, output=output)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def _close(got, want, ref):
    """FP32 network values carry an absolute error of ~1e-7 of their terms: 1e-6 absolute on the mean and max
    errors, and that over ||ref|| / sqrt(n) on the relative L2 error."""
    n = ref.size
    assert abs(got[0] - want[0]) <= 1e-5 * want[0] + 1e-6, (got, want)
    assert abs(got[1] - want[1]) <= 1e-5 * want[1] + 1e-6, (got, want)
    assert abs(got[2] - want[2]) <= 1e-5 * want[2] + 1e-6 * np.sqrt(n) / np.linalg.norm(ref), (got, want)


def _expect(O, H, L, theta, xy, ref, heads=1, output=0):
    # the oracle at the FP32-rounded inputs the GPU sees
    xy32 = xy.astype(np.float32).astype(np.float64)
    ref32 = ref.astype(np.float32).astype(np.float64)
    return np.array(O.prediction_error(theta, H, L, xy32, ref32, heads=heads, output=output))


@pytest.mark.parametrize("m", [1, 37, 100, 1000])
def test_error_on_a_grid_matches_oracle(V, torch, m):
    from oracle import oracle as O
    prob = gen.config_c2()
    theta = prob.params(seed=4, bias_scale=0.1)
    xy = _grid(m)
    ref = np.sin(8 * np.pi * xy[:, 0]) * np.sin(8 * np.pi * xy[:, 1])
    got = _err(V, torch, 30, 3, theta, xy, ref)
    _close(got, _expect(O, 30, 3, theta, xy, ref), ref)
    assert np.array_equal(got, _err(V, torch, 30, 3, theta, xy, ref))  # fixed summation order


def test_second_output_error_matches_oracle(V, torch):
    from oracle import oracle as O
    man = gen.VarDiffManufactured()
    xy = gen.disk_sensor_points(5000, 3)
    theta = gen.glorot_params(30, 3, seed=6, bias_scale=0.1, heads=2)
    for output, ref in [(0, man.u(xy[:, 0], xy[:, 1])), (1, man.eps(xy[:, 0], xy[:, 1]))]:
        got = _err(V, torch, 30, 3, theta, xy, ref, heads=2, output=output)
        _close(got, _expect(O, 30, 3, theta, xy, ref, heads=2, output=output), ref)


# ----------------------------------------------------------------------------- the prediction kernel itself

def _eval(V, torch, H, L, theta, xy, heads=1, want=("u", "ux", "uy")):
    dev = torch.device("cuda:0")
    X = torch.tensor(xy, dtype=torch.float32, device=dev)
    outs = {k: (torch.full((len(xy),), float("nan"), device=dev) if k in want else None)
            for k in ("u", "ux", "uy", "e")}
    V.vpinn_eval_network_heads(H, L, heads, torch.tensor(theta, dtype=torch.float32, device=dev), X, **outs)
    torch.cuda.synchronize()
    return X.cpu().double().numpy(), {k: v.cpu().double().numpy() for k, v in outs.items() if v is not None}


@pytest.mark.parametrize("n", [29302, 1034772])
def test_prediction_at_the_papers_sizes(V, torch, n):
    """The smallest and largest point counts of the paper's prediction-time table (Appendix, FastVPINNs vs FEM),
    both with a ragged last tile (n mod 16 = 6 and 4): values alone (the timed prediction) and with tangents,
    every output finite, 4,096 sampled points and the last 40 against the oracle."""
    from oracle import oracle as O
    theta = gen.config_c2().params(seed=8, bias_scale=0.1)
    xy = gen.uniform(11, "predict", 2 * n, 0.0, 1.0).reshape(n, 2)
    X, vals = _eval(V, torch, 30, 3, theta, xy, want=("u",))
    _, full = _eval(V, torch, 30, 3, theta, xy)
    assert np.isfinite(vals["u"]).all() and all(np.isfinite(a).all() for a in full.values())
    assert np.array_equal(vals["u"], full["u"])  # the value chain is the same with or without tangents
    rng = np.random.default_rng(n)
    idx = np.concatenate([rng.choice(n - 40, 4096, replace=False), np.arange(n - 40, n)])
    ref = O.mlp_eval(theta, 30, 3, X[idx])
    for k, want in zip(("u", "ux", "uy"), ref):
        np.testing.assert_allclose(full[k][idx], want, rtol=1e-5, atol=2e-6 * np.abs(want).max(), err_msg=k)


def test_prediction_output_combinations(V, torch):
    """Each subset of outputs of a two-output network writes exactly those outputs, with the same values."""
    from oracle import oracle as O
    theta = gen.glorot_params(30, 3, seed=12, bias_scale=0.1, heads=2)
    xy = gen.uniform(12, "predict2", 2 * 1001, 0.0, 1.0).reshape(-1, 2)
    X, all4 = _eval(V, torch, 30, 3, theta, xy, heads=2, want=("u", "ux", "uy", "e"))
    ref = dict(zip(("u", "ux", "uy", "e"), O.mlp_eval(theta, 30, 3, X, heads=2)))
    for k in all4:
        np.testing.assert_allclose(all4[k], ref[k], rtol=1e-5, atol=2e-6 * np.abs(ref[k]).max(), err_msg=k)
    for want in [("e",), ("u",), ("u", "e"), ("ux",), ("uy", "e")]:
        _, got = _eval(V, torch, 30, 3, theta, xy, heads=2, want=want)
        assert set(got) == set(want)
        for k in want:
            assert np.array_equal(got[k], all4[k]), (want, k)


def test_prediction_of_no_points(V, torch):
    dev = torch.device("cuda:0")
    theta = torch.tensor(gen.config_c2().params(seed=1), dtype=torch.float32, device=dev)
    u = torch.full((4,), 7.0, device=dev)
    V.vpinn_eval_network(30, 3, theta, torch.zeros((0, 2), device=dev), u)
    torch.cuda.synchronize()
    assert (u == 7.0).all()


@pytest.mark.parametrize("H,L,heads", [(1, 1, 1), (17, 2, 2), (30, 3, 2), (32, 4, 1), (8, 4, 2)])
def test_prediction_values_only_every_shape(V, torch, H, L, heads):
    """The values-only kernel (no tangent products) for each depth and both output counts, on a ragged point
    count: against the oracle, and equal to the values the tangent kernel writes."""
    from oracle import oracle as O
    theta = gen.glorot_params(H, L, seed=20 + H + L, bias_scale=0.2, heads=heads)
    xy = gen.uniform(13, f"predict/{H}/{L}", 2 * 777, -1.0, 1.0).reshape(-1, 2)
    want = ("u", "e") if heads == 2 else ("u",)
    X, vals = _eval(V, torch, H, L, theta, xy, heads=heads, want=want)
    _, full = _eval(V, torch, H, L, theta, xy, heads=heads, want=want + ("ux", "uy"))
    ref = O.mlp_eval(theta, H, L, X, heads=heads)
    for k, r in zip(("u", "e"), (ref[0], ref[3] if heads == 2 else None)):
        if k not in want:
            continue
        np.testing.assert_allclose(vals[k], r, rtol=1e-5, atol=2e-6 * np.abs(r).max(), err_msg=k)
        assert np.array_equal(vals[k], full[k]), k
