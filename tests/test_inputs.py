"""The seeded synthetic inputs: deterministic, well-formed, and shaped like the paper's workloads."""
import numpy as np

import vpinn_inputs as gen


def _signed_areas(mesh):
    v = mesh.xy[mesh.quad]
    x, y = v[..., 0], v[..., 1]
    return 0.5 * np.sum(x * np.roll(y, -1, 1) - np.roll(x, -1, 1) * y, 1)


def test_splitmix64_reference_values():
    # SplitMix64 finaliser of the counter sequence is deterministic and uniform-looking
    a = gen.splitmix64(0, "x", 5)
    b = gen.splitmix64(0, "x", 5)
    np.testing.assert_array_equal(a, b)
    assert len(set(a.tolist())) == 5
    u = gen.uniform01(42, "u", 100000)
    assert 0.0 <= u.min() and u.max() < 1.0
    assert abs(u.mean() - 0.5) < 0.005
    z = gen.normal(42, "z", 100000)
    assert abs(z.mean()) < 0.02 and abs(z.std() - 1.0) < 0.02


def test_meshes_counter_clockwise_and_sized():
    for mesh, ne, area in [(gen.config_c2().mesh, 1024, 1.0), (gen.config_c4().mesh, 4096, 1.0)]:
        a = _signed_areas(mesh)
        assert mesh.n_elem == ne and a.min() > 0 and abs(a.sum() - area) < 1e-12
    g = gen.config_c3().mesh
    assert g.n_elem == 14000 and _signed_areas(g).min() > 0


def test_perturbation_bounds():
    m = gen.square_mesh(8, 8, 0.2, seed=3)
    base = gen.square_mesh(8, 8)
    d = np.abs(m.xy - base.xy)
    assert d.max() <= 0.2 / 8 + 1e-15 and d.max() > 0.15 / 8
    on_bnd = (base.xy[:, 0] % 1 == 0) | (base.xy[:, 1] % 1 == 0)
    assert np.all(d[on_bnd] == 0)


def test_boundary_points_on_boundary():
    b = gen.square_boundary_points(400)
    assert b.shape == (400, 2)
    on = np.isclose(b[:, 0], 0) | np.isclose(b[:, 0], 1) | np.isclose(b[:, 1], 0) | np.isclose(b[:, 1], 1)
    assert on.all()
    assert len({tuple(p) for p in b.round(12)}) == 400


def test_params_glorot_and_fp32_representable():
    th = gen.glorot_params(30, 3, seed=0)
    assert th.size == gen.n_params(30, 3) == 1981
    np.testing.assert_array_equal(th, th.astype(np.float32).astype(np.float64))
    w2 = th[90:990]
    assert np.abs(w2).max() <= np.sqrt(6 / 60) and np.abs(w2).max() > 0.9 * np.sqrt(6 / 60)


def test_batched_mix():
    inst = gen.batched_instances(64, seed=0)
    ne = np.array([p.n_elem for p in inst])
    assert len(inst) == 64 and ne.min() >= 200 and ne.max() <= 17000
    assert {p.quad_order for p in inst} <= {4, 6, 10} and {p.test_order for p in inst} <= {3, 5}
