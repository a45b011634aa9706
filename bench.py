"""Training-step throughput of the FastVPINNs hot path on one MI355X.

A step is one full epoch of Algorithm 3 for every problem of the workload: forward
values and tangents at every quadrature point, contraction with G_x/G_y and F, loss,
adjoint through the contraction and the network, and an Adam update.  The default
workload is a batch of 64 independent Poisson problems of uneven size and order
(256 to 16,384 skewed quads each, 4x4, 6x6 or 10x10 GLL points, 3x3 or 5x5 test
functions, 12,962,384 quadrature points in all, one 2-30-30-30-1 tanh network each),
trained together by one graph-replayed batched step.  Inputs (premultiplied tensors,
points, parameters) are resident in device memory before the timed region.

Prints one JSON line (rank 0).  --gpus above 1 is rejected: the library runs on one GPU.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "epochs/s and Mquadpts/s fwd+adjoint, fused batched vs plain HIP, loss err\u22641e-5"
# the paper's own timings (NVIDIA RTX A6000, TensorFlow, FP32): context beside a workload, not a target
PAPER_CONTEXT = {
    "gear_cd": {"value": 1000.0 / 13.0, "unit": "epochs/s", "mquadpts_per_s": 27.3,
                "hardware": "NVIDIA RTX A6000, TensorFlow, FP32",
                "workload": "CD2D on a 14,192-quad Gmsh gear, 25 quadrature points an element, 4x4 test functions, "
                            "MLP 3x50 tanh, 6,096 boundary points: about 13 ms a training iteration (Sec. 4.6.4)"},
    "inverse_const": {"value": 500.0, "unit": "epochs/s", "mquadpts_per_s": 3.2,
                      "hardware": "NVIDIA RTX A6000, TensorFlow, FP32",
                      "workload": "constant-eps inverse problem on (-1,1)^2, 2x2 elements with 40x40 quadrature points, "
                                  "30x3 network, 50 sensors: 2 ms mean time per epoch, 8,909 epochs in about 18 s "
                                  "(Sec. 4.7.1)"},
    "disk_vareps": {"value": 500.0, "unit": "epochs/s", "bound": "at least",
                    "hardware": "NVIDIA RTX A6000, TensorFlow, FP32",
                    "workload": "space-dependent eps on a 1,024-quad disk: under 200 s for 100,000 epochs "
                                "(Sec. 4.7.2 and the conclusions; quadrature and test orders not stated)"},
}
PEAK_FP32_TFLOPS = 157.3    # MI355X published FP32 (vector and matrix) peak
# how the network kernels compute: every line carries it
ARITHMETIC = {
    "products": ("FP32: each operand split exactly into three bf16 pieces, the six piece products of an FP32 "
                 "product accumulated in FP32 on the bf16 matrix cores (16x16x32 and 16x16x16 MFMAs); error "
                 "below that of the FP32 MFMA"),
    "elementwise": "FP32 vector ALU (tanh, derivatives, the splitting itself)",
    "reductions": "losses summed in FP64, gradient partials in FP32, both in a fixed order",
}
# roofline note of the network kernels: what `achieved` counts and what bounds them
ROOF_NOTE = ("achieved counts the algorithmic FP32 multiply-adds (the network's own width, no padding, no "
             "recomputation) against the FP32 matrix peak; the matrix cores execute six bf16 products per FP32 "
             "product, and what bounds the kernel is vector-ALU issue (the splitting and the elementwise work)")
PEAK_HBM_GBS = 8000.0       # MI355X HBM3E
# VALU FP32 without packed instructions (they are switched off at build time):
# 256 CUs x 64 lanes x 2 FLOP per FMA x 2.4 GHz
PEAK_FP32_VALU_TFLOPS = 78.6


def n_outputs(prob) -> int:
    return getattr(prob, "heads", 1)


def kernel_work(prob, matrix_free: bool = False, n_interior=None):
    """Algorithmic work of each fused-path kernel for one epoch (dense products as 2 x multiply-adds).

    k_fwd: values and tangents, interior 2H + 3(L-1)H^2 + 2H MACs a point, boundary/sensor 3H + (L-1)H^2;
    k_contract: 4 N_test MACs a point (contraction and its adjoint); bytes: G_x, G_y once (8 N_test a point),
    F (4 N_test an element), (u_x, u_y) in and (dL/du_x, dL/du_y) out (16 a point);
    k_bwd: reverse sweep, interior 2H + 6(L-1)H^2 + 4H MACs a point, boundary/sensor 3H + 2(L-1)H^2.
    A second network output (space-dependent diffusion e): k_fwd + H MACs an interior point; k_contract
    7 N_test MACs a point (terms e (u_x G_x + u_y G_y) + (b . grad u) M, adjoint sums of G_x, G_y, M) and
    M read once (12 N_test bytes a point) plus e in and dL/de out (8 a point); k_bwd + 2H MACs.
    Matrix-free problems (no G stored): the sum-factorised contraction takes 6 N_t n^2 + 4 N_t^2 n MACs an
    element (forward 3 N_t n^2 + 2 N_t^2 n, adjoint the same) and reads F, 32 B of geometry, the point buffer.
    n_interior: the network's interior points when shared points are on (distinct points, not slots).
    """
    H, L = prob.width, prob.n_hidden
    nt = prob.test_order ** 2
    n_extra = len(prob.bnd_xy) + len(prob.sens_xy)
    two = n_outputs(prob) == 2
    ni = prob.n_points if n_interior is None else n_interior
    if matrix_free:
        n, t = prob.quad_order, prob.test_order
        contract = {"flop": 2.0 * prob.n_elem * (6 * t * n * n + 4 * t * t * n),
                    "bytes": 4.0 * nt * prob.n_elem + 32.0 * prob.n_elem + (24.0 if two else 16.0) * prob.n_points}
    else:
        contract = {"flop": 2.0 * prob.n_points * (7 if two else 4) * nt,
                    "bytes": (12.0 if two else 8.0) * nt * prob.n_points + 4.0 * nt * prob.n_elem
                    + (24.0 if two else 16.0) * prob.n_points}
    out = {
        "k_fwd": {"flop": 2.0 * (ni * (2 * H + 3 * (L - 1) * H * H + 2 * H + (H if two else 0))
                                 + n_extra * (3 * H + (L - 1) * H * H))},
        "k_contract": contract,
        "k_bwd": {"flop": 2.0 * (ni * (2 * H + 6 * (L - 1) * H * H + 4 * H + (2 * H if two else 0))
                                 + n_extra * (3 * H + 2 * (L - 1) * H * H))},
    }
    # the one-pass kernel does all three; it reads G, F and the points once and keeps the rest on chip
    out["k_step"] = {"flop": out["k_fwd"]["flop"] + contract["flop"] + out["k_bwd"]["flop"],
                     "bytes": 8.0 * nt * prob.n_points + 4.0 * nt * prob.n_elem + 8.0 * prob.n_points
                     + 12.0 * n_extra}
    return out


def flops_per_epoch(prob) -> float:
    """Algorithmic FLOPs of one forward+adjoint epoch: 2 x the multiply-adds of the dense products.

    interior point: forward 2H + 3(L-1)H^2 + 2H, backward 2H + 6(L-1)H^2 + 4H, contraction 4 N_test;
    boundary/sensor point (value stream only): forward 3H + (L-1)H^2, backward 3H + 2(L-1)H^2.
    """
    H, L = prob.width, prob.n_hidden
    nt = prob.test_order ** 2
    mac_int = (2 * H + 3 * (L - 1) * H * H + 2 * H) + (2 * H + 6 * (L - 1) * H * H + 4 * H) + 4 * nt
    if n_outputs(prob) == 2:
        mac_int += 3 * H + 3 * nt  # the second output, its adjoint, and the larger contraction
    mac_bnd = (3 * H + (L - 1) * H * H) + (3 * H + 2 * (L - 1) * H * H)
    n_extra = len(prob.bnd_xy) + len(prob.sens_xy)
    return 2.0 * (prob.n_points * mac_int + n_extra * mac_bnd)


def bytes_per_epoch(prob, matrix_free: bool = False) -> float:
    """Algorithmic HBM bytes: G_x and G_y once (matrix-free: 32 B of geometry an element instead), F,
    quadrature and boundary points, parameters."""
    nt = prob.test_order ** 2
    n_extra = len(prob.bnd_xy) + len(prob.sens_xy)
    g = 12.0 if n_outputs(prob) == 2 else 8.0  # G_x, G_y (and M)
    tensors = 32.0 * prob.n_elem if matrix_free else g * nt * prob.n_points
    return (tensors + 4.0 * nt * prob.n_elem + 8.0 * prob.n_points + 12.0 * n_extra)


def whole_step_rates(flops: float, nbytes: float, ms: float) -> dict:
    """The three rates of a step: FLOP/s and (effective: cache-resident data counts) GB/s against their peaks,
    and the governing-roofline fraction max(bytes / BW, flops / F) / t."""
    t = ms * 1e-3
    tf, gbs = flops / t / 1e12, nbytes / t / 1e9
    return {"algorithmic_flop": flops, "algorithmic_bytes": nbytes,
            "achieved_tflops": round(tf, 3), "frac_of_fp32_peak": round(tf / PEAK_FP32_TFLOPS, 4),
            "effective_gbs": round(gbs, 1), "frac_of_hbm_peak": round(gbs / PEAK_HBM_GBS, 4),
            "governing_roofline_frac": round(max(nbytes / (PEAK_HBM_GBS * 1e9), flops / (PEAK_FP32_TFLOPS * 1e12)) / t, 4)}


def host_info() -> dict:
    """Cores this process may use and the CPU model, for the CPU baseline."""
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 0
    return {"host_cores": n, "cpu_model": model}


def measure_copy_gbs(torch, nbytes: int = 1 << 30, reps: int = 10) -> float:
    """Read+write rate of a device-to-device copy of `nbytes` (torch's own kernel): what a plain streaming
    kernel reaches on this part, beside the published 8 TB/s."""
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    return 2.0 * nbytes / (ms * 1e-3) / 1e9


def source_digest() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2404_12063_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(name.encode())
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_from_profile(workload: str, kernel: str, tuning=None):
    """HBM bytes per launch of `kernel` on `workload` from the committed counter summary, if it was taken on
    the current sources and, when the summary names one, with the same tuning (else None)."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    entry = rec.get(workload, {}).get(kernel)
    if not entry or entry.get("source_digest") != source_digest():
        return None
    # only the tuning fields that change the kernel's own memory traffic must agree: forward wavefronts and
    # stored activations for k_fwd, stored activations for k_bwd, chunking and rows per pass for the contraction
    fields = {"k_fwd": (0, 3), "k_bwd": (3,), "k_contract": (1, 2), "k_step": ()}.get(kernel, (0, 1, 2, 3))
    tr = entry.get("tuning")
    if tuning is not None and tr is not None and any(list(tr)[i] != list(tuning)[i] for i in fields):
        return None
    return entry.get("hbm_bytes_per_launch")


COPY_PROBE_BYTES = 256 << 20


def _pmc_rows(path):
    import csv
    with open(path) as f:
        return list(csv.DictReader(f))


def write_traffic(workload: str, fetch_csv: str, write_csv: str, tuning=None):
    """Scale the per-dispatch FETCH_SIZE / WRITE_SIZE (KiB) of each fused-path kernel by what the same
    counters read for the 256 MiB copy (known: 256 MiB read, 256 MiB written); store under `workload`."""
    def per_kernel(path, counter):
        vals = {}
        for r in _pmc_rows(path):
            if r.get("Counter_Name") != counter:
                continue
            vals.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
        return vals
    fetch = per_kernel(fetch_csv, "FETCH_SIZE")
    write = per_kernel(write_csv, "WRITE_SIZE")
    def copy_kib(vals):
        # the probe's copy dispatches: the runtime's copy kernel reading more than a quarter of the probe's bytes
        # (the other copies are small uploads); their median
        cand = sorted(v for k, vs in vals.items() if "copyBuffer" in k for v in vs
                      if v > 0.25 * (COPY_PROBE_BYTES >> 10))
        return cand[len(cand) // 2]
    f_scale = (COPY_PROBE_BYTES / 1024.0) / copy_kib(fetch)
    w_scale = (COPY_PROBE_BYTES / 1024.0) / copy_kib(write)
    out = {}
    # kernel families (template arguments vary with the tuning); a --profile-run bench runs one plan only
    for name, key in [("k_bwd", "k_bwd<"), ("k_fwd", "k_fwd<"), ("k_contract", "k_contract_"), ("k_eval", "k_eval<"),
                      ("k_step", "k_step<")]:
        fk = sorted(v for k, vs in fetch.items() if key in k for v in vs)
        wk = sorted(v for k, vs in write.items() if key in k for v in vs)
        if not fk or not wk:
            continue
        fb = fk[len(fk) // 2] * 1024.0 * f_scale
        wb = wk[len(wk) // 2] * 1024.0 * w_scale
        out[name] = {"source_digest": source_digest(), "tuning": None if tuning is None else list(tuning),
                     "fetch_bytes_per_launch": fb, "write_bytes_per_launch": wb,
                     "hbm_bytes_per_launch": fb + wb, "fetch_scale": f_scale, "write_scale": w_scale,
                     "dispatches": len(fk)}
    path = os.path.join(ROOT, "profiles", "traffic.json")
    rec = {}
    if os.path.exists(path):
        with open(path) as f:
            rec = json.load(f)
        if not all(isinstance(v, dict) and all(isinstance(x, dict) for x in v.values()) for v in rec.values()):
            rec = {}
    rec[workload] = out
    with open(path, "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps(out))


def time_path(V, torch, p, prob, theta, path: int, steps: int, warmup: int, eps0=None):
    """Eager steps: vpinn_loss_and_grad then vpinn_adam_step.  On the fused path the library records
    events between its kernels, which gives the per-kernel durations of every timed step.  eps0: the
    inverse problem's trainable diffusion coefficient (its gradient comes from the same call and Adam
    updates it too)."""
    dev = torch.device("cuda:0")
    n = V.vpinn_n_params_out(prob.width, prob.n_hidden, n_outputs(prob))
    th = torch.tensor(theta, dtype=torch.float32, device=dev)
    m = torch.zeros(n, dtype=torch.float32, device=dev)
    v = torch.zeros(n, dtype=torch.float32, device=dev)
    g = torch.zeros(n, dtype=torch.float32, device=dev)
    loss = torch.zeros(4, dtype=torch.float32, device=dev)
    cfg = V.loss_cfg(prob.width, prob.n_hidden, prob.tau, prob.gamma, V.VPINN_NORM_TEST, path,
                     n_outputs=n_outputs(prob))
    stream = torch.cuda.current_stream()
    fused = path == V.VPINN_PATH_FUSED
    if eps0 is not None:
        ep = torch.tensor([eps0], dtype=torch.float32, device=dev)
        gep, mep, vep = (torch.zeros(1, dtype=torch.float32, device=dev) for _ in range(3))

    def step(t):
        if eps0 is None:
            V.vpinn_loss_and_grad(p, cfg, th, loss=loss, grad=g, stream=stream)
        else:
            V.vpinn_loss_and_grad(p, cfg, th, eps=ep, loss=loss, grad=g, grad_eps=gep, stream=stream)

    def update(t):
        V.vpinn_adam_step(th, g, m, v, t, lr=1e-3, stream=stream)
        if eps0 is not None:
            V.vpinn_adam_step(ep, gep, mep, vep, t, lr=1e-3, stream=stream)

    t = 0
    for _ in range(warmup):
        t += 1
        step(t)
        update(t)
    NE = V.PROFILE_EVENTS
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(NE + 1)] for _ in range(steps)]
    for e in ev:
        for x in e:
            x.record(stream)  # creates the underlying events before their handles are handed over
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    for i in range(steps):
        t += 1
        if fused:
            V.vpinn_set_profile_events(p, ev[i][:NE])
        else:
            ev[i][0].record(stream)
        step(t)
        if not fused:
            ev[i][NE - 1].record(stream)
        update(t)
        ev[i][NE].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    if fused:
        V.vpinn_set_profile_events(p, None)
    mean = lambda xs: sum(xs) / len(xs)  # noqa: E731
    out = {"wall_s": wall, "lg_ms_mean": mean([e[0].elapsed_time(e[NE - 1]) for e in ev]),
           "step_ms_mean": mean([e[0].elapsed_time(e[NE]) for e in ev])}
    if eps0 is not None:
        out["eps_final"] = float(ep.item())
    if fused:
        for k, name in enumerate(["k_fwd_ms", "k_contract_ms", "k_bwd_ms", "k_final_ms"]):
            out[name] = mean([e[k].elapsed_time(e[k + 1]) for e in ev])
    return out


def profile_batch_kernels(V, torch, b, s, T, M, Vv, step, losses, n_steps: int, diff=None):
    """Mean duration of each fused-path kernel over eager batched steps of plan `b` (its profiling events).

    An event pair around a kernel also times the event markers themselves; that overhead, measured as the
    mean interval of back-to-back event pairs with nothing between them on the same stream, is subtracted
    (reported as event_overhead_ms)."""
    NE = V.PROFILE_EVENTS
    pev = [[torch.cuda.Event(enable_timing=True) for _ in range(NE)] for _ in range(n_steps)]
    for e in pev:
        for x in e:
            x.record(s)
    kw = {} if diff is None else {"diff": diff[0], "diff_m": diff[1], "diff_v": diff[2]}
    for i in range(n_steps):
        V.vpinn_batch_set_profile_events(b, pev[i])
        V.vpinn_batch_step(b, T, M, Vv, step, lr=1e-3, losses=losses, stream=s, **kw)
    V.vpinn_batch_set_profile_events(b, None)
    empty = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n_steps)]
    for e0, e1 in empty:
        e0.record(s)
        e1.record(s)
    torch.cuda.synchronize()
    over = sum(e0.elapsed_time(e1) for e0, e1 in empty) / n_steps
    ms = [max(0.0, sum(e[k].elapsed_time(e[k + 1]) for e in pev) / n_steps - over) for k in range(NE - 1)]
    if V.vpinn_batch_get_tuning(b)[4]:
        # the one-pass step: its kernel between the first two events, the reduction between the last two
        out = {"k_step": ms[0], "k_fused_final": ms[3]}
    else:
        out = dict(zip(["k_fwd", "k_contract", "k_bwd", "k_fused_final"], ms))
    out["steps"] = n_steps
    out["event_overhead_ms"] = over
    return out


def kernel_table(work, kms, extra=""):
    """Per-kernel rates of the step's kernels (those kms times) and the dominant one."""
    names = [k for k in ("k_step", "k_fwd", "k_contract", "k_bwd") if k in kms]
    kernels = {}
    for name in names:
        ent = {"ms": round(kms[name], 5), "tflops": round(work[name]["flop"] / (kms[name] * 1e-3) / 1e12, 3)}
        ent["frac_fp32_peak"] = round(ent["tflops"] / PEAK_FP32_TFLOPS, 4)
        if "bytes" in work[name]:
            ent["gbs"] = round(work[name]["bytes"] / (kms[name] * 1e-3) / 1e9, 1)
            ent["frac_hbm_peak"] = round(ent["gbs"] / PEAK_HBM_GBS, 4)
        kernels[name] = ent
    kernels["k_fused_final"] = {"ms": round(kms["k_fused_final"], 5), "note": "reduction + Adam" + extra}
    return kernels, max(names, key=lambda k: kms[k])


def tune_batch(V, b, params, stream, fixed, reps):
    """Autotune the batch's tile shapes, or apply a fixed tuning (profiling runs want one plan only).
    The kernels are the same for any eps, so an inverse problem is tuned at eps = 1."""
    if fixed is not None:
        V.vpinn_batch_set_tuning(b, *fixed)
        tuning = V.vpinn_batch_get_tuning(b)
        print(f"[bench] fixed tile shapes (fwd_waves, chunk_shift, rows_per_pass) = {tuning}", file=sys.stderr, flush=True)
    else:
        tuning = V.vpinn_batch_autotune(b, params, reps=reps, stream=stream)
        print(f"[bench] autotuned tile shapes (fwd_waves, chunk_shift, rows_per_pass) = {tuning}", file=sys.stderr,
              flush=True)
    return tuning


def time_graph(V, torch, p, prob, theta, steps: int, warmup: int, fixed_tuning=None, eps0=None):
    """The step of one problem as a batch of one: forward + adjoint + Adam (Adam inside the reduction
    kernel, step counter in device memory) captured once in a HIP graph and replayed.  eps0: the inverse
    problem's trainable diffusion coefficient, updated by the same captured step.
    Throughput: `steps` replays back to back, bracketed by synchronisations (host wall clock) and by one
    pair of events; the per-step distribution comes from a separate run with an event pair per step."""
    dev = torch.device("cuda:0")
    b = V.vpinn_batch_create([p], V.loss_cfg(prob.width, prob.n_hidden, prob.tau, prob.gamma,
                                             n_outputs=n_outputs(prob)))
    th = torch.tensor(theta, dtype=torch.float32, device=dev).reshape(1, -1).contiguous()
    m = torch.zeros_like(th)
    v = torch.zeros_like(th)
    step = torch.zeros(1, dtype=torch.int64, device=dev)
    losses = torch.zeros((1, 4), dtype=torch.float32, device=dev)
    diff = None if eps0 is None else (torch.tensor([eps0], dtype=torch.float32, device=dev),
                                      torch.zeros(1, dtype=torch.float32, device=dev),
                                      torch.zeros(1, dtype=torch.float32, device=dev))
    s = torch.cuda.Stream()
    n_dist = min(steps, 200)
    with torch.cuda.stream(s):
        tuning = tune_batch(V, b, th, s, fixed_tuning, reps=5)
        kms = profile_batch_kernels(V, torch, b, s, th, m, v, step, losses, n_steps=min(steps, 100), diff=diff)
        V.vpinn_batch_capture(b, th, m, v, step, lr=1e-3, losses=losses, stream=s,
                              **({} if diff is None else {"diff": diff[0], "diff_m": diff[1], "diff_v": diff[2]}))
        for _ in range(warmup):
            V.vpinn_batch_replay(b, stream=s)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        e0.record(s)
        for _ in range(steps):
            V.vpinn_batch_replay(b, stream=s)
        e1.record(s)
        torch.cuda.synchronize()
        wall = time.perf_counter() - w0
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n_dist)]
        for i in range(n_dist):
            ev[i][0].record(s)
            V.vpinn_batch_replay(b, stream=s)
            ev[i][1].record(s)
        torch.cuda.synchronize()
    st = sorted(a.elapsed_time(c) for a, c in ev)
    q = lambda xs, f: xs[min(len(xs) - 1, int(f * len(xs)))]  # noqa: E731
    out = {"wall_s": wall, "event_ms_total": e0.elapsed_time(e1), "tuning": list(tuning), "kernel_ms": kms,
           "step_ms_p10": q(st, 0.1),
           "step_ms_p50": q(st, 0.5), "step_ms_p90": q(st, 0.9), "steps_done": int(step.item()) - n_dist - kms["steps"],
           "final_loss": float(losses[0, 0].item())}
    if diff is not None:
        out["eps_final"] = float(diff[0].item())
        out["eps_steps"] = int(step.item())
    return out


def cpu_baseline(prob, theta, seconds: float):
    """The FP64 oracle (single-threaded C) on full epochs of the same workload, as many as fit in ~seconds
    (the inverse problem at its initial eps, which is then held: the work of an epoch does not depend on it)."""
    from oracle import oracle as O
    import numpy as np
    asm = O.assemble_problem(prob)
    th = theta.copy()
    m = np.zeros_like(th)
    v = np.zeros_like(th)
    n_ep = 0
    first = None
    t0 = time.perf_counter()
    while True:
        r = O.problem_loss_grad(prob, asm, th, eps=prob.eps_init)
        if first is None:
            first = r.loss[0]
        O.adam(th, r.grad, m, v, n_ep + 1, lr=1e-3)
        n_ep += 1
        el = time.perf_counter() - t0
        if n_ep >= 2 and el >= seconds:
            break
    return {"value": n_ep / el, "unit": "epochs/s", "cores": 1, "kind": "oracle",
            "sample": f"{n_ep} full epochs (loss+grad+Adam, FP64, single-threaded C) of the same workload in "
                      f"{el:.1f} s; assembly not timed", **host_info()}, first


def pool_threads() -> int:
    """Host threads for the oracle pool: the cores this process may use, at most 16 (one GPU's share of
    the host)."""
    return max(1, min(16, host_info()["host_cores"] or 1))


def oracle_batched(probs, thetas, threads: int):
    """The FP64 oracle (the single-threaded C code, unchanged) over every instance of a batch, one instance
    per task on a pool of host threads (the oracle holds no global state and its C calls release the
    interpreter lock, so the threads run on separate cores).  Assembly first (not timed), then one full
    epoch: loss, gradient and Adam of every instance.  Returns the per-instance results, the epoch's wall
    time on `threads` threads and the sum of the per-instance times (what one thread would take)."""
    from concurrent.futures import ThreadPoolExecutor
    from oracle import oracle as O
    import numpy as np
    order = sorted(range(len(probs)), key=lambda i: -probs[i].n_points)  # largest first: shortest makespan
    with ThreadPoolExecutor(max_workers=threads) as ex:
        asm = dict(zip(order, ex.map(lambda i: O.assemble_problem(probs[i]), order)))

        def epoch(i):
            t0 = time.perf_counter()
            r = O.problem_loss_grad(probs[i], asm[i], thetas[i])
            th = np.array(thetas[i], dtype=np.float64)
            m, v = np.zeros_like(th), np.zeros_like(th)
            O.adam(th, r.grad, m, v, 1, lr=1e-3)
            return r, time.perf_counter() - t0

        w0 = time.perf_counter()
        res = dict(zip(order, ex.map(epoch, order)))
        wall = time.perf_counter() - w0
    return [res[i][0] for i in range(len(probs))], wall, sum(res[i][1] for i in range(len(probs)))


def time_eager_batch(V, torch, b, s, T, M, Vv, step, losses, n_steps: int) -> float:
    """ms per eager (not graph-replayed) batched step: the fused kernels launched by vpinn_batch_step."""
    with torch.cuda.stream(s):
        V.vpinn_batch_step(b, T, M, Vv, step, lr=1e-3, losses=losses, stream=s)
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        for _ in range(n_steps):
            V.vpinn_batch_step(b, T, M, Vv, step, lr=1e-3, losses=losses, stream=s)
        torch.cuda.synchronize()
    return (time.perf_counter() - w0) / n_steps * 1e3


C5_TEXT = ("c5: 64 independent Poisson instances on +-20% jittered square meshes, element counts log-uniform in "
           "[256,16384], GLL n in {4,6,10}, test N_t in {3,5}, k in 1..16, each with its own 2-30-30-30-1 tanh MLP; "
           "one batched forward+adjoint+Adam step per epoch replayed from a HIP graph")


def bench_batched(args, V, torch, gen):
    """The headline: 64 independent Poisson instances (log-uniform sizes, mixed orders), one batched step
    per epoch replayed from a captured HIP graph.  Beside it: the same step launched eagerly, the unfused
    path looping over the instances (the comparator), and the FP64 oracle over all 64 instances on a pool
    of host threads (the CPU baseline and the loss and gradient check of every instance)."""
    import numpy as np
    probs = gen.batched_instances(64, seed=0)
    gp = []
    for pr in probs:
        p = V.vpinn_assemble(pr.mesh.xy, pr.mesh.quad, pr.quad_order, pr.test_order, pr.f_amp, pr.f_kx, pr.f_ky)
        V.vpinn_set_boundary(p, pr.bnd_xy, pr.bnd_g)
        if args.shared_points:
            V.vpinn_set_shared_points(p, pr.mesh.xy, pr.mesh.quad)
        gp.append(p)
    n_int = [V.vpinn_get_info(p).n_distinct_points or pr.n_points for p, pr in zip(gp, probs)]
    P = sum(pr.n_points for pr in probs)
    print(f"[bench] workload c5: 64 instances, {sum(pr.n_elem for pr in probs)} elements, {P} quadrature points",
          file=sys.stderr, flush=True)
    cfg = V.loss_cfg(30, 3, 10.0, 0.0)
    b = V.vpinn_batch_create(gp, cfg)
    dev = torch.device("cuda:0")
    th = np.stack([pr.params() for pr in probs])
    T = torch.tensor(th, dtype=torch.float32, device=dev)
    M = torch.zeros_like(T)
    Vv = torch.zeros_like(T)
    step = torch.zeros(1, dtype=torch.int64, device=dev)
    losses = torch.zeros((64, 4), device=dev)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        tuning = tune_batch(V, b, T, s, args.tuning, reps=3)
        # loss and gradient of every instance at the initial parameters, for the oracle check
        L0 = torch.zeros((64, 4), device=dev)
        G0 = torch.zeros_like(T)
        if not args.profile_run:
            V.vpinn_batch_loss_and_grad(b, T, losses=L0, grads=G0, stream=s)
        V.vpinn_batch_capture(b, T, M, Vv, step, lr=1e-3, losses=losses, stream=s)
        for _ in range(args.warmup):
            V.vpinn_batch_replay(b, stream=s)
        s.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        for i in range(args.steps):
            ev[i][0].record(s)
            V.vpinn_batch_replay(b, stream=s)
            ev[i][1].record(s)
        torch.cuda.synchronize()
        wall = time.perf_counter() - w0
    print(f"[bench] fused graph: {wall / args.steps * 1e3:.4f} ms/step", file=sys.stderr, flush=True)
    st = sorted(a.elapsed_time(c) for a, c in ev)
    ms = wall / args.steps * 1e3
    # per-kernel durations: eager batched steps of the same plan with the library's profiling events
    with torch.cuda.stream(s):
        kms = profile_batch_kernels(V, torch, b, s, T, M, Vv, step, losses, n_steps=10)
    work = {}
    for pr, ni in zip(probs, n_int):
        for name, w in kernel_work(pr, n_interior=ni).items():
            for key, val in w.items():
                work.setdefault(name, {}).setdefault(key, 0.0)
                work[name][key] += val
    kernels, dom = kernel_table(work, kms, " for 64 instances")
    dom_tf = work[dom]["flop"] / (kms[dom] * 1e-3) / 1e12
    eps_s = 1e3 / ms
    flops = sum(flops_per_epoch(pr) for pr in probs)
    out = {
        "metric": METRIC,
        "value": round(eps_s, 3), "unit": "epochs/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms, 5), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": C5_TEXT, "instances": 64, "quad_points": P, "parallelism": "single GPU",
                   "tuning": list(tuning), "shared_points": bool(args.shared_points),
                   "network_interior_points": sum(n_int)},
        "mquadpts_per_s": round(P * eps_s / 1e6, 2),
        "step_ms_p10_p50_p90": [round(st[len(st) // 10], 4), round(st[len(st) // 2], 4),
                                round(st[(9 * len(st)) // 10], 4)],
        "roofline": {"bound": "mfma", "kernel": dom + " (all 64 instances in one launch)",
                     "achieved": round(dom_tf, 3), "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(dom_tf / PEAK_FP32_TFLOPS, 4),
                     "traffic": traffic_from_profile("c5", dom, tuning),
                     "algorithmic_flop_per_launch": work[dom]["flop"], "launch_ms_mean": round(kms[dom], 4),
                     "note": ROOF_NOTE},
        "arithmetic": ARITHMETIC,
        "whole_step": whole_step_rates(flops, sum(bytes_per_epoch(pr) for pr in probs), ms),
        "kernels": kernels,
        "kernels_note": ("mean durations over eager batched steps of the same tuned plan as the timed graph, "
                         "from the library's profiling events, less the event-pair overhead"),
        "event_overhead_ms": round(kms["event_overhead_ms"], 5),
    }
    if args.profile_run:
        print(json.dumps(out), flush=True)
        return
    n_eager = max(3, min(20, args.steps // 10))
    ems = time_eager_batch(V, torch, b, s, T, M, Vv, step, losses, n_eager)
    out["fused_eager_ms_per_step"] = round(ems, 5)
    print(f"[bench] fused eager: {ems:.4f} ms/step", file=sys.stderr, flush=True)
    if not args.no_plain:
        # unfused comparator: each instance's plain loss/grad and Adam, in a loop
        pcfg = V.loss_cfg(30, 3, 10.0, 0.0, path=V.VPINN_PATH_PLAIN)
        Ts = [torch.tensor(th[i], dtype=torch.float32, device=dev) for i in range(64)]
        Ms = [torch.zeros_like(t) for t in Ts]
        Vs = [torch.zeros_like(t) for t in Ts]
        g = torch.zeros(T.shape[1], device=dev)
        l1 = torch.zeros(4, device=dev)
        n_plain = max(3, min(20, args.steps // 10))
        for t in range(1, 3):
            for i in range(64):
                V.vpinn_loss_and_grad(gp[i], pcfg, Ts[i], loss=l1, grad=g)
                V.vpinn_adam_step(Ts[i], g, Ms[i], Vs[i], t)
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        for t in range(3, 3 + n_plain):
            for i in range(64):
                V.vpinn_loss_and_grad(gp[i], pcfg, Ts[i], loss=l1, grad=g)
                V.vpinn_adam_step(Ts[i], g, Ms[i], Vs[i], t)
        torch.cuda.synchronize()
        pms = (time.perf_counter() - w0) / n_plain * 1e3
        print(f"[bench] plain eager: {pms:.4f} ms/step", file=sys.stderr, flush=True)
        out["plain_hip"] = {"ms_per_step": round(pms, 4), "epochs_per_s": round(1e3 / pms, 3),
                            "note": "eager: 64 x (unfused loss/grad + Adam) per step"}
        out["speedup_vs_plain"] = round(pms / ems, 3)
        out["speedup_vs_plain_note"] = "fused eager batched step vs the plain path looped eagerly"
        out["speedup_graph_vs_plain_eager"] = round(pms / ms, 3)
    out["hbm_copy_gbs_measured"] = round(measure_copy_gbs(torch), 1)
    if not args.no_cpu_baseline:
        nthr = pool_threads()
        print(f"[bench] oracle: 64 instances on {nthr} host threads", file=sys.stderr, flush=True)
        ref, owall, osum = oracle_batched(probs, th, nthr)
        l0 = L0.cpu().numpy().astype(np.float64)
        g0 = G0.cpu().numpy().astype(np.float64)
        lerr = [abs(l0[i, 0] - ref[i].loss[0]) / abs(ref[i].loss[0]) for i in range(64)]
        gerr = [float(np.linalg.norm(g0[i] - ref[i].grad) / np.linalg.norm(ref[i].grad)) for i in range(64)]
        out["cpu_baseline"] = {
            "value": round(1.0 / owall, 5), "unit": "epochs/s", "cores": nthr, "kind": "oracle",
            "sample": (f"one full epoch of all 64 instances ({P} quadrature points: loss, gradient and Adam in "
                       f"FP64, the unchanged single-threaded C oracle, one instance per task on {nthr} host "
                       f"threads) in {owall:.1f} s wall; assembly not timed"),
            "one_thread_epoch_s": round(osum, 2),
            "one_thread_note": "sum of the per-instance times measured in the pool (what one core would take)",
            **host_info()}
        out["loss_rel_err_vs_oracle"] = max(lerr)
        out["grad_rel_l2_err_vs_oracle"] = max(gerr)
        out["oracle_check"] = ("every instance's loss and gradient at the initial parameters (batched fused "
                               "path) against the FP64 oracle: the maxima over the 64 instances")
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--path", choices=["fused", "plain"], default="fused")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true", help="skip timing the unfused comparator")
    ap.add_argument("--workload", choices=["c5", "c2", "c3", "c4", "probe", "gear_cd", "disk_vareps", "c2_mf",
                                           "probe_mf", "predict", "inverse_const", "p_refine", "h_refine"],
                    default="c5",
                    help="c5 (default, the headline): 64 independent instances of mixed sizes and orders in one "
                         "batched step; c2: one 1,024-element problem; c3: Poisson on the 14,000-element toothed "
                         "annulus; c4: the inverse problem (eps trained) on 4,096 elements; probe: "
                         "20x20 test functions on 4,096 elements (G-stream bound); gear_cd: the convection-diffusion "
                         "gear problem on 14,000 elements; disk_vareps: space-dependent diffusion inverse problem, "
                         "a two-output network on a 1,024-element disk; c2_mf, probe_mf: the same as c2, probe with "
                         "G regenerated per step from the element geometry (matrix-free); predict: network values "
                         "of a trained-size MLP at the six point counts of the paper's prediction-time table; "
                         "inverse_const: the constant-eps inverse problem at the paper's sizes (2x2 elements, 40x40 "
                         "points), eps trained beside the weights; p_refine, h_refine: the paper's p- and "
                         "h-refinement shapes (one element, or 8x8 elements, of 80x80 points)")
    ap.add_argument("--shared-points", action="store_true",
                    help="evaluate the network once per distinct interior GLL point (vpinn_set_shared_points); the "
                         "result equals per-slot evaluation up to rounding")
    ap.add_argument("--copy-probe", action="store_true",
                    help="first copy a 256 MiB device buffer 3 times: a kernel of known traffic that calibrates "
                         "the FETCH_SIZE / WRITE_SIZE counters")
    ap.add_argument("--traffic-from", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="no GPU work: turn two rocprofv3 --pmc counter_collection.csv files (FETCH_SIZE, then "
                         "WRITE_SIZE, taken with --copy-probe on --workload W and --tuning T) into "
                         "profiles/traffic.json[W] (give the same --tuning T)")
    ap.add_argument("--profile-run", action="store_true",
                    help="counter runs: time only the tuned batch-of-one plan (no single-problem-API steps, no "
                         "loss check), so every fused kernel in the trace belongs to that plan; implies no CPU baseline")
    ap.add_argument("--tuning", type=lambda t: tuple(int(x) for x in t.split(",")), default=None,
                    metavar="FWD_WAVES,CHUNK_SHIFT,ROWS_PER_PASS[,STORE_ACTIVATIONS[,ONE_PASS]]",
                    help="use this tile-shape tuning instead of autotuning (profiling runs)")
    args = ap.parse_args()
    if args.tuning is not None and len(args.tuning) not in (3, 4, 5):
        ap.error("--tuning takes 3 to 5 comma-separated integers")
    if args.steps < 1 or args.warmup < 0:
        ap.error("--steps must be at least 1 and --warmup at least 0")
    if args.traffic_from:
        write_traffic(args.workload, *args.traffic_from, tuning=args.tuning)
        return
    if args.profile_run:
        args.no_cpu_baseline = True
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); no multi-GPU path is implemented",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2404_12063_amd import vpinn as V
    import vpinn_inputs as gen

    assert torch.cuda.is_available(), "needs a HIP device"
    if args.copy_probe:
        src = torch.ones(COPY_PROBE_BYTES // 4, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.workload == "c5":
        bench_batched(args, V, torch, gen)
        return
    if args.workload == "predict":
        bench_predict(args, V, torch, gen)
        return
    bench_single(args, V, torch, gen)


# point counts of the paper's prediction-time table (Appendix, FastVPINNs vs FEM) and its network times there
# (NVIDIA RTX A6000, TensorFlow): context, not a target
PREDICT_SIZES = [29302, 115868, 259698, 460792, 719150, 1034772]
PREDICT_PAPER_S = [7.807e-4, 7.978e-4, 1.777e-3, 3.139e-3, 4.890e-3, 7.023e-3]


def predict_flop_per_point(H: int, L: int) -> int:
    """Algorithmic FLOPs of one network value: input layer (2 products and a bias, per neuron), L - 1 hidden
    products, the output layer; the H L tanh are not counted."""
    return 2 * 2 * H + (L - 1) * 2 * H * H + 2 * H


def bench_predict(args, V, torch, gen):
    """Network values at N points (the prediction step timed in the paper's Appendix table), for each of its six
    point counts: seeded uniform points in the unit square stand in for the FEM mesh's degrees of freedom, with
    the C2 network (2-30-30-30-1 tanh).  Points and weights are resident in device memory; each call is timed
    between HIP events on the stream it is launched on."""
    import numpy as np
    prob = gen.config_c2()
    H, L = prob.width, prob.n_hidden
    theta = prob.params(seed=8, bias_scale=0.1)
    dev = torch.device("cuda:0")
    th = torch.tensor(theta, dtype=torch.float32, device=dev)
    stream = torch.cuda.current_stream()
    reps = args.steps
    rows = []
    # a counter run times the largest size only, so every k_eval dispatch in it has the same size
    sizes = list(zip(PREDICT_SIZES, PREDICT_PAPER_S))[-1:] if args.profile_run else zip(PREDICT_SIZES, PREDICT_PAPER_S)
    for n, paper_s in sizes:
        X = torch.tensor(gen.uniform(11, "predict", 2 * n, 0.0, 1.0).reshape(n, 2), dtype=torch.float32,
                         device=dev)
        u = torch.empty(n, dtype=torch.float32, device=dev)
        for _ in range(args.warmup):
            V.vpinn_eval_network(H, L, th, X, u, stream=stream)
        torch.cuda.synchronize()
        # per-call events, so the mean is over launches; the event-pair cost is taken off
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
        t0 = time.perf_counter()
        for a, b in ev:
            a.record(stream)
            V.vpinn_eval_network(H, L, th, X, u, stream=stream)
            b.record(stream)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / reps
        e0 = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
        for a, b in e0:
            a.record(stream)
            b.record(stream)
        torch.cuda.synchronize()
        over = float(np.mean([a.elapsed_time(b) for a, b in e0]))
        ms = float(np.mean([a.elapsed_time(b) for a, b in ev])) - over
        assert torch.isfinite(u).all()
        rows.append({"n_points": n, "kernel_ms": round(ms, 5), "wall_ms_per_call": round(wall * 1e3, 5),
                     "mpoints_per_s": round(n / (ms * 1e-3) / 1e6, 1), "paper_s": paper_s,
                     "ratio_vs_paper": round(paper_s / (ms * 1e-3), 1)})
        print(f"[bench] predict n={n}: {ms * 1e3:.2f} us/call ({rows[-1]['mpoints_per_s']} Mpoints/s), "
              f"wall {wall * 1e6:.1f} us/call", file=sys.stderr, flush=True)
        del X, u
    big = rows[-1]
    fpp = predict_flop_per_point(H, L)
    achieved = fpp * big["n_points"] / (big["kernel_ms"] * 1e-3) / 1e12
    out = {
        "metric": "prediction Mpoints/s (network values at N points, paper's FEM-vs-network timing table)",
        "value": big["mpoints_per_s"], "unit": "Mpoints/s", "n_gpus": 1, "steps": reps, "warmup": args.warmup,
        "ms_per_step": big["kernel_ms"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "predict: MLP 2-30-30-30-1 tanh (the C2 network) evaluated at N seeded uniform "
                               "points of the unit square, N = 29,302 .. 1,034,772 (the paper's prediction-time "
                               "table; value at the largest)", "parallelism": "single GPU"},
        "sizes": rows,
        "roofline": {"bound": "mfma", "kernel": "k_eval<3,1,false>", "achieved": round(achieved, 3),
                     "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_TFLOPS, 4),
                     "traffic": traffic_from_profile("predict", "k_eval"),
                     "algorithmic_bytes_per_point": 12, "algorithmic_flop_per_point": fpp,
                     "algorithmic_flop_per_launch": fpp * big["n_points"], "launch_ms_mean": big["kernel_ms"],
                     "note": ROOF_NOTE},
        "arithmetic": ARITHMETIC,
        "paper_context": {"hardware": "NVIDIA RTX A6000, TensorFlow", "seconds_at_largest": PREDICT_PAPER_S[-1],
                          "note": "the paper does not state the network used for the timing"},
    }
    if not args.no_cpu_baseline:
        from oracle import oracle as O
        n_s = 20000
        xs = gen.uniform(11, "predict", 2 * n_s, 0.0, 1.0).reshape(n_s, 2)
        calls, t0 = 0, time.perf_counter()
        while True:
            O.mlp_eval(theta, H, L, xs)
            calls += 1
            el = time.perf_counter() - t0
            if el >= args.cpu_seconds:
                break
        out["cpu_baseline"] = {"value": round(calls * n_s / el / 1e6, 4), "unit": "Mpoints/s", "cores": 1,
                               "kind": "oracle",
                               "sample": f"{calls} oracle evaluations (FP64, single-threaded C, values and tangents) "
                                         f"of {n_s} of the same points in {el:.1f} s", **host_info()}
    print(json.dumps(out), flush=True)


WORKLOAD_TEXT = {
    "c3": "c3: Poisson -Lap u = f on a toothed-annulus O-grid (r from 0.5 to the rim 1 + 0.05 sin 24 theta, "
          "400x35 = 14,000 jittered quads, standing in for the paper's gear mesh), 5x5 GLL points, 5x5 test "
          "functions, u*=sin(4pi x)sin(4pi y), 4000 boundary points, MLP 2-30-30-30-1 tanh, Adam lr 1e-3",
    "c4": "c4: inverse problem -eps Lap u = f on [0,1]^2, 64x64 quad mesh with interior nodes jittered +-20% h, "
          "10x10 GLL points, 5x5 test functions, u*=sin(2pi x)sin(2pi y), eps trained beside the weights (init 2.0, "
          "true 0.3), 1000 sensors with N(0, 0.01^2) noise, 1600 boundary points, tau = gamma = 10, MLP "
          "2-30-30-30-1 tanh, Adam lr 1e-3 on the weights and on eps",
    "c2": "c2: Poisson -Lap u = f on [0,1]^2, 32x32 quad mesh with interior nodes jittered +-20% h, 10x10 GLL "
          "points, 5x5 test functions, u*=sin(8pi x)sin(8pi y), 1600 boundary points, MLP 2-30-30-30-1 tanh, "
          "Adam lr 1e-3",
    "gear_cd": "gear_cd: convection-diffusion -Lap u + (0.1, 0) . grad u = 50 sin x + cos x, u = 0 on the boundary "
               "(the paper's gear experiment) on a toothed-annulus O-grid of 400x35 = 14,000 skewed quads (24 teeth, "
               "amplitude 0.05), 5x5 GLL points, 4x4 test functions, 6096 boundary points, MLP 2-30-30-30-1 tanh; "
               "eps and b folded into G at assembly",
    "disk_vareps": "disk_vareps: inverse problem -div(eps(x,y) grad u) + (1, 0) . grad u = f on the disk of centre "
                   "(0.5, 0.5) and radius 0.5 (32x32 quads of a squircle-mapped grid), eps = 0.5 (sin x + cos y) and "
                   "u = sin(2pi x) sin(2pi y) manufactured, 10x10 GLL points, 5x5 test functions, 1600 boundary "
                   "points, 1000 sensors of u, tau = gamma = 10, MLP 2-30-30-30-2 tanh whose second output is eps",
    "inverse_const": "inverse_const: -eps Lap u = f on (-1,1)^2 (the paper's constant-eps inverse problem), 2x2 "
                     "elements, 40x40 GLL points, 5x5 test functions, u = 10 sin(x) tanh(x) exp(-0.3 x^2), 50 "
                     "sensors of u, 400 boundary points, tau = gamma = 10, eps trainable (init 2.0, true 0.3), MLP "
                     "2-30-30-30-1 tanh, Adam lr 1e-3 on the weights and on eps",
    "p_refine": "p_refine: Poisson on the unit square as one element (the paper's p-refinement study), 80x80 GLL "
                "points, 20x20 test functions, u* = sin(4pi x) sin(4pi y), 400 boundary points, MLP 2-30-30-30-1 tanh",
    "h_refine": "h_refine: Poisson on the unit square, 8x8 uniform elements (the paper's finest h-refinement), 80x80 "
                "GLL points and 5x5 test functions each (409,600 points), u* = sin(4pi x) sin(4pi y), 1600 boundary "
                "points, MLP 2-30-30-30-1 tanh",
    "c2_mf": "c2_mf: c2 with no stored G: the contraction regenerates G every step from the 8 geometry floats of "
             "each element by sum factorisation (matrix-free)",
    "probe_mf": "probe_mf: probe with no stored G (matrix-free): 1.3 GB of G a step replaced by 32 B of geometry per "
                "element and a sum-factorised contraction",
    "probe": "probe: the c4 mesh (64x64 jittered, 4096 elements) with 10x10 GLL points and 20x20 test functions "
             "(the paper's largest p-refinement), u*=sin(2pi x)sin(2pi y), 1600 boundary points, MLP "
             "2-30-30-30-1 tanh: the only shape whose G stream (1.3 GB) outweighs the network arithmetic",
}


def bench_single(args, V, torch, gen):
    mf = args.workload.endswith("_mf")
    prob = gen.CONFIGS[args.workload[:-3] if mf else args.workload]()
    theta = prob.params()
    p = V.assemble_problem(prob, matrix_free=mf, shared_points=args.shared_points)
    n_int = V.vpinn_get_info(p).n_distinct_points or prob.n_points
    print(f"[bench] workload {args.workload}: {prob.n_elem} elements, {prob.n_points} quadrature points, "
          f"{len(prob.bnd_xy)} boundary points", file=sys.stderr, flush=True)

    main_path = V.VPINN_PATH_FUSED if args.path == "fused" else V.VPINN_PATH_PLAIN
    fused = main_path == V.VPINN_PATH_FUSED
    # an inverse problem trains a scalar eps beside the weights, in the same captured step
    inverse = prob.eps_init is not None
    graph = fused
    eager_steps = min(args.steps, 300)
    if args.profile_run and graph:
        eager = None
    else:
        eager = time_path(V, torch, p, prob, theta, main_path, eager_steps, args.warmup, eps0=prob.eps_init)
        print(f"[bench] {args.path} eager: {eager['wall_s'] / eager_steps * 1e3:.4f} ms/step", file=sys.stderr,
              flush=True)
    if graph:
        res = time_graph(V, torch, p, prob, theta, args.steps, args.warmup, args.tuning, eps0=prob.eps_init)
        assert res["steps_done"] == args.warmup + args.steps
        print(f"[bench] fused graph: {res['wall_s'] / args.steps * 1e3:.4f} ms/step", file=sys.stderr, flush=True)
    else:  # the plain path: eager steps only
        res = {"wall_s": eager["wall_s"] * args.steps / eager_steps}
    plain = None
    if not args.no_plain and fused and n_outputs(prob) == 1 and not mf:
        plain = time_path(V, torch, p, prob, theta, V.VPINN_PATH_PLAIN, min(args.steps, 300), 20,
                          eps0=prob.eps_init)
        print(f"[bench] plain eager: {plain['wall_s'] / min(args.steps, 300) * 1e3:.4f} ms/step", file=sys.stderr,
              flush=True)

    # loss parity at the initial parameters (one extra evaluation outside the timed region)
    dev = torch.device("cuda:0")
    loss0 = torch.zeros(4, dtype=torch.float32, device=dev)
    if not args.profile_run:
        ep0 = None if not inverse else torch.tensor([prob.eps_init], dtype=torch.float32, device=dev)
        V.vpinn_loss_and_grad(p, V.loss_cfg(prob.width, prob.n_hidden, prob.tau, prob.gamma, 0, main_path,
                                            n_outputs=n_outputs(prob)),
                              torch.tensor(theta, dtype=torch.float32, device=dev), eps=ep0, loss=loss0)
        torch.cuda.synchronize()
    gpu_loss0 = float(loss0[0].item())

    ms = res["wall_s"] / args.steps * 1e3
    eps_s = 1e3 / ms
    flops = flops_per_epoch(prob)
    work = kernel_work(prob, mf, n_int)
    kernels = {}
    if fused:
        km = res["kernel_ms"]
        kernels, dom = kernel_table(work, km)
        k_ms = km[dom]
        if dom == "k_contract" and mf:
            achieved = work[dom]["flop"] / (k_ms * 1e-3) / 1e12
            roof = {"bound": "alu", "kernel": dom + " (matrix-free)", "achieved": round(achieved, 3),
                    "peak": PEAK_FP32_VALU_TFLOPS, "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_VALU_TFLOPS, 4),
                    "algorithmic_flop_per_launch": work[dom]["flop"]}
        elif dom == "k_contract" and work[dom]["flop"] / work[dom]["bytes"] < 1.0:
            achieved = work[dom]["bytes"] / (k_ms * 1e-3) / 1e9
            roof = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS,
                    "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4),
                    "algorithmic_bytes_per_launch": work[dom]["bytes"]}
        else:
            achieved = work[dom]["flop"] / (k_ms * 1e-3) / 1e12
            roof = {"bound": "mfma", "kernel": dom, "achieved": round(achieved, 3), "peak": PEAK_FP32_TFLOPS,
                    "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_TFLOPS, 4),
                    "algorithmic_flop_per_launch": work[dom]["flop"], "note": ROOF_NOTE}
        roof["traffic"] = traffic_from_profile(args.workload, dom, res.get("tuning"))
        roof["launch_ms_mean"] = round(k_ms, 5)
    else:
        k_ms = eager["lg_ms_mean"]
        achieved = flops / (k_ms * 1e-3) / 1e12
        roof = {"bound": "alu", "kernel": "plain loss_and_grad sequence", "achieved": round(achieved, 3),
                "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_TFLOPS, 4),
                "traffic": None, "algorithmic_flop_per_launch": flops, "launch_ms_mean": round(k_ms, 5)}
    out = {
        "metric": METRIC,
        "value": round(eps_s, 3),
        "unit": "epochs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": WORKLOAD_TEXT[args.workload],
                   "path": args.path + ((" (HIP graph replay of the batch-of-one step" +
                                         (", Adam on the weights and on eps)" if inverse else ")")) if graph else
                                        " (eager; Adam on the weights and on eps)" if inverse else " (eager)"),
                   "tuning": res.get("tuning"),
                   "n_elem": prob.n_elem, "quad_points": prob.n_points,
                   "shared_points": bool(args.shared_points), "network_interior_points": n_int,
                   "boundary_points": len(prob.bnd_xy), "parallelism": "single GPU"},
        "mquadpts_per_s": round(prob.n_points * eps_s / 1e6, 2),
        "roofline": roof,
        "arithmetic": ARITHMETIC,
        "whole_step": whole_step_rates(flops, bytes_per_epoch(prob, mf), ms),
    }
    if graph:
        if inverse:
            out["eps_after_steps"] = {"initial": prob.eps_init, "after": round(res["eps_final"], 6),
                                      "true": prob.eps_true, "steps": res["eps_steps"]}
        if eager is not None:
            out["single_problem_api_eager_ms_per_step"] = round(eager["wall_s"] / eager_steps * 1e3, 5)
        out["step_ms_p10_p50_p90"] = [round(res["step_ms_p10"], 5), round(res["step_ms_p50"], 5),
                                      round(res["step_ms_p90"], 5)]
        out["gpu_event_ms_per_step"] = round(res["event_ms_total"] / args.steps, 5)
        out["kernels"] = kernels
        out["kernels_note"] = ("mean durations over eager batched steps of the same tuned plan as the timed graph, "
                               "from the library's profiling events, less the event-pair overhead")
        out["event_overhead_ms"] = round(res["kernel_ms"]["event_overhead_ms"], 5)
    if plain is not None:
        pms = plain["wall_s"] / min(args.steps, 300) * 1e3
        out["plain_hip"] = {"ms_per_step": round(pms, 5), "epochs_per_s": round(1e3 / pms, 3),
                            "loss_and_grad_ms_mean": round(plain["lg_ms_mean"], 5),
                            "note": "eager: unfused loss_and_grad then Adam through the single-problem API"}
        # fusion alone (both eager, the same API) and fusion plus the graph replay, reported apart
        if eager is not None:
            out["speedup_vs_plain"] = round(pms / (eager["wall_s"] / eager_steps * 1e3), 3)
            out["speedup_vs_plain_note"] = "fused eager vs plain eager, both through vpinn_loss_and_grad + Adam"
        out["speedup_graph_vs_plain_eager"] = round(pms / ms, 3)
    if args.workload in PAPER_CONTEXT:
        out["paper_context"] = PAPER_CONTEXT[args.workload]
    if not args.profile_run:
        out["hbm_copy_gbs_measured"] = round(measure_copy_gbs(torch), 1)
    if not args.no_cpu_baseline:
        cb, oracle_loss0 = cpu_baseline(prob, theta, args.cpu_seconds)
        out["cpu_baseline"] = cb
        out["loss_rel_err_vs_oracle"] = abs(gpu_loss0 - oracle_loss0) / abs(oracle_loss0)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
