"""Host-side checks of bench.py: the single-GPU refusal, the algorithmic work it divides by (hand-derived for the
C2 shape), and the rules by which it attaches counter-measured traffic to a roofline line."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402
import vpinn_inputs as gen  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_c2_algorithmic_counts():
    """C2: H = 30, L = 3, N_test = 25, 102,400 interior and 1,600 boundary points.  Multiply-adds per interior
    point: forward 60 + 5,400 + 60 = 5,520, reverse 60 + 10,800 + 120 = 10,980, contraction and adjoint 100, so
    33,200 FLOPs; per boundary point 90 + 1,800 forward and 90 + 3,600 reverse, 11,160 FLOPs."""
    prob = gen.config_c2()
    assert (prob.width, prob.n_hidden, prob.test_order ** 2, prob.n_points, len(prob.bnd_xy)) == (30, 3, 25, 102400, 1600)
    assert bench.flops_per_epoch(prob) == 33200 * 102400 + 11160 * 1600 == 3417536000
    work = bench.kernel_work(prob)
    four = ("k_fwd", "k_contract", "k_bwd")
    assert sum(work[k]["flop"] for k in four) == bench.flops_per_epoch(prob)
    # the one-pass kernel does the three kernels' work and reads G, F and the points once
    assert work["k_step"]["flop"] == bench.flops_per_epoch(prob)
    assert work["k_step"]["bytes"] == 8 * 25 * 102400 + 4 * 25 * 1024 + 8 * 102400 + 12 * 1600
    assert work["k_fwd"]["flop"] == 2 * (5520 * 102400 + 1890 * 1600)
    assert work["k_bwd"]["flop"] == 2 * (10980 * 102400 + 3690 * 1600)
    # G_x and G_y once, F, the point buffer in and out
    assert work["k_contract"]["bytes"] == 8 * 25 * 102400 + 4 * 25 * 1024 + 16 * 102400
    # matrix-free: 6 N_t n^2 + 4 N_t^2 n multiply-adds an element (n = 10, N_t = 5) and 32 B of geometry
    mf = bench.kernel_work(prob, matrix_free=True)["k_contract"]
    assert mf["flop"] == 2 * 1024 * (6 * 5 * 100 + 4 * 25 * 10)
    assert mf["bytes"] == 4 * 25 * 1024 + 32 * 1024 + 16 * 102400


def test_prediction_flops_per_point():
    # input layer 2 x 2 x 30, two hidden products 2 x 900 each, output 2 x 30
    assert bench.predict_flop_per_point(30, 3) == 120 + 3600 + 60
    assert bench.predict_flop_per_point(1, 1) == 6


def _fake_tree(tmp_path, src_text, entry):
    csrc = tmp_path / "paper_2404_12063_amd" / "csrc"
    csrc.mkdir(parents=True)
    (csrc / "k.hip").write_text(src_text)
    (tmp_path / "profiles").mkdir()
    (tmp_path / "profiles" / "traffic.json").write_text(json.dumps({"c2": entry}))


def test_traffic_needs_the_measured_sources_and_tuning(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    _fake_tree(tmp_path, "kernel v1", {})
    digest = bench.source_digest()
    entry = {k: {"source_digest": digest, "tuning": [16, 2, 4, 1], "hbm_bytes_per_launch": b}
             for k, b in [("k_fwd", 1.0), ("k_bwd", 2.0), ("k_contract", 3.0)]}
    (tmp_path / "profiles" / "traffic.json").write_text(json.dumps({"c2": entry}))
    assert bench.traffic_from_profile("c2", "k_bwd", (16, 2, 4, 1)) == 2.0
    # only the fields that change a kernel's own traffic must agree
    assert bench.traffic_from_profile("c2", "k_bwd", (8, 0, 2, 1)) == 2.0
    assert bench.traffic_from_profile("c2", "k_bwd", (16, 2, 4, 0)) is None
    assert bench.traffic_from_profile("c2", "k_fwd", (16, 0, 8, 1)) == 1.0
    assert bench.traffic_from_profile("c2", "k_fwd", (12, 2, 4, 1)) is None
    assert bench.traffic_from_profile("c2", "k_contract", (12, 2, 4, 0)) == 3.0
    assert bench.traffic_from_profile("c2", "k_contract", (16, 1, 4, 1)) is None
    assert bench.traffic_from_profile("probe", "k_bwd", None) is None
    # a source edit makes every stored figure stale
    (tmp_path / "paper_2404_12063_amd" / "csrc" / "k.hip").write_text("kernel v2")
    assert bench.traffic_from_profile("c2", "k_bwd", (16, 2, 4, 1)) is None


@pytest.mark.parametrize("args", [["--tuning", "1,2"], ["--tuning", "1,2,3,4,5,6"], ["--workload", "nope"],
                                  ["--steps", "0"], ["--warmup", "-1"]])
def test_argument_errors_exit_before_any_device_work(args):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py")] + args, capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2 and r.stdout == "" and "error" in r.stderr


def test_oracle_pool_equals_the_oracle_called_in_turn():
    """The CPU baseline of the batched workload runs the unchanged oracle one instance per task on host threads:
    each instance's loss and gradient must be exactly those of a plain call (threads change nothing in FP64), the
    epoch's wall time positive and the one-thread time the sum of the instances' times."""
    from oracle import oracle as O
    import numpy as np
    probs = gen.batched_instances(3, seed=4, lo=16, hi=48)
    th = np.stack([p.params(seed=11 + i, bias_scale=0.1) for i, p in enumerate(probs)])
    ref, wall, osum = bench.oracle_batched(probs, th, threads=2)
    assert wall > 0 and osum > 0
    for i, p in enumerate(probs):
        r = O.problem_loss_grad(p, O.assemble_problem(p), th[i])
        assert np.array_equal(ref[i].loss, r.loss) and np.array_equal(ref[i].grad, r.grad), i


def test_pool_threads_stay_within_one_gpu_share():
    assert 1 <= bench.pool_threads() <= 16
