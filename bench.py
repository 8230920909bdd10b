"""Benchmark of the CNN-VMC hot path on one MI355X.

Workload: 36x36 periodic J1-J2 lattice (J1 = 1, J2 = 0.5), CNN of 8 layers of
3x3 circular convolutions with 32 channels (P = 65,056), weights N(0, 0.02^2),
1024 synthetic Sz = 0 configurations.  One step is the whole hot path:

  bond enumeration + Marshall ratios + queue (integer), base pass, exchanged-
  configuration pass (matrix cores, incremental receptive cone), FP64 ratio
  sums -> E_loc; energy mean / variance; per-sample log-derivatives O (FP32
  out, FP64 backward); SR solve by conjugate gradient (at most 100
  iterations; the iterations run are reported).

value = samples per second of that whole step (inputs resident in HBM) in the
split-BF16 form (every operand hi + lo BF16, three products per multiply-add,
FP32 accumulation), the step captured once in a HIP graph and replayed
(--no-graph: eager calls).  The form is gated on the metric's bar where it is
not vacuous: at stress weights, whose exchanged configurations differ at O(1)
in log amplitude, its mean energy over 16 samples must lie within 1e-5
(relative) of the plain FP64 GPU form.  (At the workload's own weights the
log ratios are below FP64 resolution, so any form passes there; that check is
reported too.)  The plain BF16 form is timed beside it as a non-gating row
with its own stress error; the plain FP64 GPU form is timed on all 1024
samples, in full and by its receptive cone (FP64 matrix cores; every
neuron bit-identical to the full pass).  Further non-gating rows: the mixed-lattice workload (12x12, 16x16,
20x20) through one multi-lattice call, SR at 24x24 (P = 46,560, B = 4096, 100
iterations), SR with O recomputed, Metropolis steps, a graph-replayed VMC
iteration, the t-J local energy (12x12, hole doping 1/8), the CNN1
network (10x10, FP64; 36x36 by full recomputation and by the receptive cone),
CNN2 (t-J 12x12), the split-form cone at K = 6 and 7 (two workgroups per
CU), and at K = 8 at the stress weights.  The FP64 CPU oracle is timed on the host cores on a
bounded sample.  Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_BF16_TFLOPS = 2500.0      # MI355X dense BF16 MFMA
PEAK_HBM_GBS = 8000.0
# stress gain of the 36x36, K = 8 network: std of the log ratios ~0.3
STRESS_GAIN_K8 = 1.26


def form_peak(form: str) -> float:
    """Peak in algorithmic FLOP/s of a form's convolutions: the split form
    issues three BF16 products per multiply-add."""
    return PEAK_BF16_TFLOPS / 3.0 if form == "bf16x3" else PEAK_BF16_TFLOPS


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cone_sites(L: int, k: int, diagonal: bool) -> int:
    """Sites within Chebyshev distance k of an exchanged pair (exact cone, no
    clamping needed when 2k + 2 <= L)."""
    if diagonal:
        n = 4 * k * k + 8 * k + 2
        side = 2 * k + 2
    else:
        n = (2 * k + 2) * (2 * k + 1)
        side = 2 * k + 2
    return min(n, L * L) if side <= L else L * L


def item_flops(L: int, K: int, C: int, diagonal: bool) -> float:
    """Algorithmic FLOPs of one exchanged configuration in incremental mode:
    every layer recomputed on the cone of sites it can change."""
    f = 0.0
    for k in range(1, K + 1):
        cin = 1 if k == 1 else C
        f += cone_sites(L, k, diagonal) * C * 9 * cin * 2
    return f


def source_hash() -> str:
    """Hash of the dominant kernel's sources (counter summaries are tied to it)."""
    h = hashlib.sha256()
    for f in ("k_net_cone.hip", "mfma_common.h"):
        h.update(open(os.path.join(ROOT, "paper_2204_07816_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def traffic_from_profile(form: str):
    """HBM bytes per launch of the dominant kernel from the committed rocprofv3
    counter summary, if it was taken on the current kernel source."""
    p = os.path.join(ROOT, "profiles", f"k_net_cone_{form}_36x36_counters.json")
    if not os.path.exists(p):
        return None
    try:
        d = json.load(open(p))
    except (OSError, ValueError):
        return None
    if d.get("source_sha256_16") != source_hash():
        return None
    return d.get("hbm_bytes_per_launch")


def cpu_baseline(L, J2, K, C, w, sp, mean_conn, budget_s=12.0):
    """Oracle (plain FP64 C, OpenMP over configurations) on a bounded sample:
    the log-amplitude of exchanged configurations of the workload.  The oracle's
    local energy of one sample is exactly (n_conn + 1) such evaluations plus
    O(n_conn N) bookkeeping, so samples/s = 1 / ((mean_conn + 1) t_forward)."""
    import numpy as np

    import oracle
    cores = len(os.sched_getaffinity(0))
    counts, bonds, _, _ = oracle.connected(L, 1.0, J2, sp[:1])
    flat = sp[0].reshape(-1)
    cfgs = []
    for b in bonds[0]:
        i, j, _ = oracle.bond_sites(L, int(b))
        s2 = flat.copy()
        s2[i], s2[j] = flat[j], flat[i]
        cfgs.append(s2)
    cfgs = np.array(cfgs, np.int8).reshape(-1, L, L)
    m = min(len(cfgs), cores)
    t0 = time.perf_counter()
    oracle.log_psi(L, K, C, w, cfgs[:m], nthreads=cores)
    t1 = time.perf_counter()
    per = (t1 - t0) / m
    m2 = int(min(len(cfgs), max(m, budget_s / max(per, 1e-9))))
    m2 = max(cores, (m2 // cores) * cores)
    t0 = time.perf_counter()
    oracle.log_psi(L, K, C, w, cfgs[:m2], nthreads=cores)
    t1 = time.perf_counter()
    per = (t1 - t0) / m2
    sps = 1.0 / ((mean_conn + 1.0) * per)
    return {
        "value": sps, "unit": "E_loc samples/s", "cores": cores, "kind": "oracle",
        "sample": (f"oracle log|psi| of {m2} exchanged configurations of sample 0 "
                   f"({L}x{L}, K={K}, C={C}), {t1 - t0:.1f} s on {cores} threads; "
                   f"scaled by (mean connected count {mean_conn:.1f} + 1) forwards per sample"),
    }


def stress_row(L, J2, K, C, sp, dev, form, gain=STRESS_GAIN_K8, n_samples=16):
    """Precision at weights where the log ratios are O(1): layer 1 N(0, 0.5^2),
    later layers gain / sqrt(9 C_in), zero biases (gain 1.26 puts the standard
    deviation of f(S') - f(s) near 0.3 at 36x36, K = 8).  E_loc of the form
    (incremental) against the plain FP64 GPU form (full recompute) on
    n_samples samples."""
    import numpy as np
    import torch

    from paper_2204_07816_amd import inputs, nqs
    sub = torch.as_tensor(sp[:n_samples]).to(dev)
    w = inputs.stress_weights(K, C, gain, 77)
    cf = nqs.Context(L, 1.0, J2, K, C, w, dtype="fp64")
    ef = cf.local_energy(sub, mode="full").cpu().numpy()
    n = int(cf.connected(sub[:2])[0].sum().item())
    d = cf.log_ratios(sub[:2].contiguous(), mode="full")[:n].cpu().numpy()
    cf.close()
    cb = nqs.Context(L, 1.0, J2, K, C, w, dtype=form)
    eb = cb.local_energy(sub, mode="incremental").cpu().numpy()
    cb.close()
    rel = float(abs(eb.mean() - ef.mean()) / abs(ef.mean()))
    return {"form": form, "gain": gain, "std_log_ratio": float(np.std(d)), "samples": n_samples,
            "mean_rel_err_vs_fp64": rel,
            "max_rel_err_vs_fp64": float(np.max(np.abs(eb - ef)) / np.max(np.abs(ef))),
            "bar_1e-5_met": bool(rel <= 1e-5)}


def sr24_row(dev, n_iter=100):
    """Non-gating row, the differentiation + SR workload: 24x24 J1-J2, K = 6,
    C = 32 (P = 46,560), 4096 configurations.  O (FP32) of all samples, then
    the SR solve (lambda = 1e-4) timed over n_iter iterations at stress
    weights (gain 1.1: S is not small next to lambda there, so every
    iteration runs); per iteration the two streaming passes read O twice."""
    import torch

    from paper_2204_07816_amd import inputs, nqs
    L, J2, K, C, _, sp = inputs.config_inputs("sr24")
    w = inputs.stress_weights(K, C, 1.1, 77)
    B = sp.shape[0]
    ctx = nqs.Context(L, 1.0, J2, K, C, w, dtype="bf16x3")
    spd = torch.as_tensor(sp).to(dev)
    O = torch.empty(B, ctx.P, dtype=torch.float32, device=dev)
    e = torch.empty(B, dtype=torch.float64, device=dev)
    ctx.local_energy(spd, mode="incremental", out=e)
    ctx.log_deriv(spd, dtype="fp32", out=O)
    x = torch.empty(ctx.P, dtype=torch.float64, device=dev)
    st = torch.empty(4, dtype=torch.float64, device=dev)
    ctx.sr_solve(O, e, 1e-4, 2, out=x, stats=st)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    ctx.log_deriv(spd, dtype="fp32", out=O)
    b.record()
    torch.cuda.synchronize()
    t_o = a.elapsed_time(b)
    a.record()
    ctx.sr_solve(O, e, 1e-4, n_iter, out=x, stats=st)
    b.record()
    torch.cuda.synchronize()
    t_sr = a.elapsed_time(b)
    it = int(st[3].item())
    o_bytes = B * ctx.P * 4
    out = {"workload": f"{L}x{L} J1-J2, CNN {K}x3x3x{C} (P={ctx.P}), {B} configurations, "
                       "stress weights (gain 1.1)",
           "log_deriv_ms": t_o, "sr_ms": t_sr, "iterations_run": it,
           "rel_residual": float(st[2].item()), "ms_per_iteration": t_sr / max(it, 1),
           "o_bytes": o_bytes,
           "streaming_gbs": 2 * o_bytes * it / (t_sr * 1e-3) / 1e9,
           "frac_hbm_peak": 2 * o_bytes * it / (t_sr * 1e-3) / 1e9 / PEAK_HBM_GBS}
    assert ctx.get_error() == 0
    ctx.close()
    return out


def mixed_row(dev, reps=3):
    """Non-gating row: the mixed-lattice workload (12x12 J2=0, 16x16 J2=0.5,
    20x20 J2=0.55; K=6, C=32, weights N(0, 0.02^2), 4096 configurations each)
    through one nqs_local_energy_multi call per step, every context autotuned
    first on 64 of its samples."""
    import torch

    from paper_2204_07816_amd import inputs, nqs
    jobs, modes, items = [], [], 0
    for lat in range(3):
        L, J2, K, C, w, sp = inputs.config_inputs("mixed", lattice=lat)
        ctx = nqs.Context(L, 1.0, J2, K, C, w, dtype="bf16")
        spd = torch.as_tensor(sp).to(dev)
        modes.append(ctx.autotune(spd[:64].contiguous()))
        ctx.reserve(sp.shape[0], modes[-1])
        e = torch.empty(sp.shape[0], dtype=torch.float64, device=dev)
        jobs.append((ctx, spd, e))
        items += int(ctx.connected(spd)[0].sum().item())
    nqs.local_energy_multi(jobs, mode="auto")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        nqs.local_energy_multi(jobs, mode="auto")
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1000.0 / reps
    samples = sum(j[1].shape[0] for j in jobs)
    out = {"samples_per_s": samples / (ms * 1e-3), "ms": ms, "samples": samples,
           "exchanged_configurations": items,
           "lattices": {f"{j[0].L}x{j[0].L}": m for j, m in zip(jobs, modes)}}
    for ctx, _, _ in jobs:
        assert ctx.get_error() == 0
        ctx.close()
    return out


def tj_row(dev, reps=3, fp64_samples=256):
    """Non-gating row: the t-J workload (12x12, t = 1, J = 0.4, hole doping
    1/8, K=6, C=32, weights N(0, 0.02^2), 4096 configurations): E_loc per
    pass in BF16 (autotuned on 64 samples), the exchanged-configuration
    kernel's average launch and algorithmic rate, and the BF16 mean against
    the FP64 GPU form on a subset."""
    import torch

    from paper_2204_07816_amd import inputs, nqs
    L, t, J, K, C, w, sp = inputs.tj_config_inputs("tj12")
    B = sp.shape[0]
    ctx = nqs.Context.tj(L, t, J, K, C, w, dtype="bf16")
    spd = torch.as_tensor(sp).to(dev)
    mode = ctx.autotune(spd[:64].contiguous())
    ctx.reserve(B, mode)
    e = torch.empty(B, dtype=torch.float64, device=dev)
    ctx.local_energy(spd, mode=mode, out=e)
    torch.cuda.synchronize()
    ctx.enable_timing(True)
    ctx.kernel_time()
    t0 = time.perf_counter()
    for _ in range(reps):
        ctx.local_energy(spd, mode=mode, out=e)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1000.0 / reps
    k_ms, k_n = ctx.kernel_time()
    ctx.enable_timing(False)
    items = int(ctx.connected(spd)[0].sum().item())
    if mode == "incremental":
        per_item = item_flops(L, K, C, False)
    else:
        per_item = L * L * C * 9 * 2 + (K - 1) * L * L * C * 9 * C * 2
    avg = k_ms / max(k_n, 1)
    achieved = items * per_item / (avg * 1e-3) / 1e12
    c64 = nqs.Context.tj(L, t, J, K, C, w, dtype="fp64")
    e64 = c64.local_energy(spd[:fp64_samples].contiguous(), mode="full").cpu().numpy()
    eb = e.cpu().numpy()[:fp64_samples]
    rel = abs(eb.mean() - e64.mean()) / abs(e64.mean())
    assert ctx.get_error() == 0 and c64.get_error() == 0
    out = {"workload": f"{L}x{L} t-J (t={t}, J={J}, {inputs.TJ_CONFIGS['tj12']['n_holes']} "
                       f"holes), CNN {K}x3x3x{C}, {B} configurations",
           "samples_per_s": B / (ms * 1e-3), "ms": ms, "mode": mode,
           "exchanged_configurations": items, "mean_energy": float(e.mean().item()),
           "kernel_avg_launch_ms": avg, "kernel_tflops": achieved,
           "kernel_frac_bf16_peak": achieved / PEAK_BF16_TFLOPS,
           "kernel_frac_bf16_sustained": achieved / SUSTAINED["bf16_tflops"],
           "bf16_mean_rel_err_vs_fp64": float(rel), "fp64_samples": fp64_samples,
           "bar_1e-5_met": bool(rel <= 1e-5)}
    ctx.close()
    c64.close()
    return out


PEAK_FP64_TFLOPS = 78.6        # MI355X FP64 (vector and dense matrix cores alike)
SUSTAINED = {}                 # register-only MFMA loop rates, filled by main()


def cnn1_row(dev, reps=2):
    """Non-gating row: the CNN1 network (6 blocks of convolution, channel-pair
    max-pool and transposed convolution, 16 channels, P = 37,440; product of
    the output neurons) on 10x10 J1-J2 (J2 = 0.5), 1024 configurations, FP64:
    E_loc by full recomputation (blocks 2.. on the FP64 matrix cores), the
    exchanged-configuration pass's rate against the FP64 peak, and O_k."""
    import torch

    from paper_2204_07816_amd import inputs, nqs
    L, J2, Kb, C, w, sp = inputs.cnn1_config_inputs()
    B = sp.shape[0]
    ctx = nqs.Context.cnn1(L, 1.0, J2, Kb, C, w)
    ctx.reserve(B, "full")
    spd = torch.as_tensor(sp).to(dev)
    e = torch.empty(B, dtype=torch.float64, device=dev)
    ctx.local_energy(spd[:8].contiguous(), mode="full")
    torch.cuda.synchronize()
    ctx.enable_timing(True)
    ctx.kernel_time()
    t0 = time.perf_counter()
    for _ in range(reps):
        ctx.local_energy(spd, mode="full", out=e)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1000.0 / reps
    k_ms, k_n = ctx.kernel_time()
    ctx.enable_timing(False)
    O = torch.empty(B, ctx.P, dtype=torch.float32, device=dev)
    ctx.log_deriv(spd, dtype="fp32", out=O)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.log_deriv(spd, dtype="fp32", out=O)
    torch.cuda.synchronize()
    ms_o = (time.perf_counter() - t0) * 1000.0
    items = int(ctx.connected(spd)[0].sum().item())
    N = L * L
    per_item = sum(2 * N * (2 * C * (1 if k == 0 else C) * 9 + C * C * 9) for k in range(Kb))
    avg = k_ms / max(k_n, 1)
    achieved = items * per_item / (avg * 1e-3) / 1e12
    assert ctx.get_error() == 0
    ctx.close()
    return {"workload": f"{L}x{L} J1-J2 (J2={J2}), CNN1 {Kb} blocks x {C} channels "
                        f"(P={inputs.cnn1_num_params(Kb, C)}), {B} configurations, FP64",
            "samples_per_s": B / (ms * 1e-3), "ms": ms, "exchanged_configurations": items,
            "conn_pass_ms": avg, "conn_pass_tflops": achieved,
            "bound": "mfma" if C == 16 else "alu",
            "frac_fp64_peak": achieved / PEAK_FP64_TFLOPS,
            "frac_fp64_sustained": achieved / SUSTAINED["fp64_tflops"],
            "log_deriv_ms": ms_o}


def cnn1_cone_flops(L, Kb, C, bonds):
    """Algorithmic FLOPs of the CNN1 receptive-cone pass over the given bond
    ids: layer l (block b's convolution is layer 2b - 1, its transposed
    convolution layer 2b) forms the box of the exchanged pair widened by l
    sites, |R_l| = (w0 + 2l)(h0 + 2l), at 2 * 9 * c_in * c_out per site."""
    import numpy as np
    tau = np.asarray(bonds) & 3
    total = 0
    for t, (w0, h0) in enumerate(((2, 1), (1, 2), (2, 2), (2, 2))):
        n = int((tau == t).sum())
        per = 0
        for l in range(1, 2 * Kb + 1):
            if l == 1:
                f = 2 * 9 * 1 * 2 * C
            elif l % 2:
                f = 2 * 9 * C * 2 * C
            else:
                f = 2 * 9 * C * C
            per += (w0 + 2 * l) * (h0 + 2 * l) * f
        total += n * per
    return total


def cnn1_36_row(dev, reps=2):
    """Non-gating row: CNN1 (6 blocks x 16 channels) on 36x36 J1-J2 (J2 =
    0.5), the paper's largest lattice for this network, 128 configurations,
    FP64: E_loc by full recomputation and by the receptive cone, the cone
    kernel's rate against the FP64 peak, and the largest relative difference
    of the two forms' E_loc."""
    import numpy as np
    import torch

    from paper_2204_07816_amd import inputs, nqs
    L, J2, Kb, C, w, sp = inputs.cnn1_36_config_inputs()
    B = sp.shape[0]
    ctx = nqs.Context.cnn1(L, 1.0, J2, Kb, C, w)
    spd = torch.as_tensor(sp).to(dev)
    out = {"workload": f"{L}x{L} J1-J2 (J2={J2}), CNN1 {Kb} blocks x {C} channels "
                       f"(P={inputs.cnn1_num_params(Kb, C)}), {B} configurations, FP64"}
    es = {}
    for mode in ("full", "incremental"):
        ctx.reserve(B, mode)
        e = torch.empty(B, dtype=torch.float64, device=dev)
        ctx.local_energy(spd, mode=mode, out=e)
        torch.cuda.synchronize()
        ctx.enable_timing(True)
        ctx.kernel_time()
        t0 = time.perf_counter()
        for _ in range(reps):
            ctx.local_energy(spd, mode=mode, out=e)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1000.0 / reps
        k_ms, k_n = ctx.kernel_time()
        ctx.enable_timing(False)
        es[mode] = e.cpu().numpy()
        out[mode] = {"samples_per_s": B / (ms * 1e-3), "ms": ms,
                     "conn_pass_ms": k_ms / max(k_n, 1)}
    _, offs, bonds, _, _ = ctx.connected(spd)
    n = int(offs[-1].item())
    bonds = bonds[:n].cpu().numpy()
    flops = cnn1_cone_flops(L, Kb, C, bonds)
    tf = flops / (out["incremental"]["conn_pass_ms"] * 1e-3) / 1e12
    out["exchanged_configurations"] = n
    out["cone_flops_per_item"] = flops / max(n, 1)
    out["speedup_incremental_vs_full"] = out["full"]["ms"] / out["incremental"]["ms"]
    out["cone_kernel"] = {"name": "k_c1_cone", "bound": "mfma", "tflops": tf,
                          "frac_fp64_peak": tf / PEAK_FP64_TFLOPS,
                          "frac_fp64_sustained": tf / SUSTAINED["fp64_tflops"]}
    ref = es["full"]
    out["eloc_max_rel_diff_incremental_vs_full"] = float(
        np.max(np.abs(es["incremental"] - ref)) / np.max(np.abs(ref)))
    assert ctx.get_error() == 0
    ctx.close()
    return out


def split_depths_row(dev, depths=(6, 7), reps=2, gain=None):
    """Non-gating row: the split-BF16 cone kernel on the 36x36 workload's 1024
    configurations (weights N(0, 0.02^2), or the stress weights of the
    precision gate when `gain` is given) at the given depths.  Up to K = 7 the
    windows of two workgroups fit a CU's LDS and the kernel runs two of four
    waves per CU (two configurations in flight); at K = 8 it runs the frame
    form, also two workgroups of four waves per CU."""
    import numpy as np
    import torch

    from paper_2204_07816_amd import inputs, nqs
    L, J2, _, C, _, sp = inputs.config_inputs("full36")
    B = sp.shape[0]
    spd = torch.as_tensor(sp).to(dev)
    out = {}
    for K in depths:
        w = inputs.weights(K, C, 0.02, 1004) if gain is None else \
            inputs.stress_weights(K, C, gain, 77)
        ctx = nqs.Context(L, 1.0, J2, K, C, w, dtype="bf16x3")
        ctx.reserve(B, "incremental")
        e = torch.empty(B, dtype=torch.float64, device=dev)
        ctx.local_energy(spd, mode="incremental", out=e)
        torch.cuda.synchronize()
        ctx.kernel_time()
        ctx.enable_timing(True)
        for _ in range(reps):
            ctx.local_energy(spd, mode="incremental", out=e)
        torch.cuda.synchronize()
        ctx.enable_timing(False)
        k_ms, k_n = ctx.kernel_time()
        _, offs, bonds, _, _ = ctx.connected(spd)
        b = bonds[:int(offs[-1].item())].cpu().numpy()
        nd = int(np.sum(b % 4 >= 2))
        fl = (b.shape[0] - nd) * item_flops(L, K, C, False) + nd * item_flops(L, K, C, True)
        ms = k_ms / max(k_n, 1)
        tf = fl / (ms * 1e-3) / 1e12
        out[f"K{K}"] = {"cone_ms": ms, "items": int(b.shape[0]), "tflops": tf,
                        "frac": tf / form_peak("bf16x3"),
                        "shape": "2 workgroups x 4 waves per CU" + ("" if K <= 7 else
                                                                     ", frame form")}
        if gain is not None:
            out[f"K{K}"]["weights"] = f"stress (gain {gain}, seed 77)"
        assert ctx.get_error() == 0
        ctx.close()
    return out


def cmp10_row(dev, reps=3):
    """Non-gating row: the precision comparison workload (10x10 J1-J2, J2 =
    0.5, CNN 4x3x3x16, weights N(0, 0.02^2), 8192 configurations): E_loc per
    pass in the FP64, FP32 and BF16 GPU forms (BF16 autotuned on 256 samples),
    each form's mean and largest per-sample error against the FP64 GPU form."""
    import numpy as np
    import torch

    from paper_2204_07816_amd import inputs, nqs
    L, J2, K, C, w, sp = inputs.config_inputs("cmp10")
    B = sp.shape[0]
    spd = torch.as_tensor(sp).to(dev)
    out = {"workload": f"{L}x{L} J1-J2 (J2={J2}), CNN {K}x3x3x{C}, {B} configurations, weights "
                       "N(0, 0.02^2)", "forms": {}}
    ref = None
    for form in ("fp64", "fp32", "bf16"):
        ctx = nqs.Context(L, 1.0, J2, K, C, w, dtype=form)
        mode = ctx.autotune(spd[:256].contiguous()) if form == "bf16" else "full"
        ctx.reserve(B, mode)
        e = torch.empty(B, dtype=torch.float64, device=dev)
        ctx.local_energy(spd, mode=mode, out=e)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            ctx.local_energy(spd, mode=mode, out=e)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1000.0 / reps
        ev = e.cpu().numpy()
        assert ctx.get_error() == 0
        ctx.close()
        row = {"mode": mode, "ms": ms, "samples_per_s": B / (ms * 1e-3)}
        if ref is None:
            ref = ev
        else:
            row["mean_rel_err_vs_fp64"] = float(abs(ev.mean() - ref.mean()) / abs(ref.mean()))
            row["max_sample_rel_err_vs_fp64"] = float(np.max(np.abs(ev - ref)) /
                                                      np.max(np.abs(ref)))
        out["forms"][form] = row
    return out


def cnn2_row(dev, reps=2):
    """Non-gating row: CNN2 (an embedding of hole/up/down, 6 blocks of a
    convolution, stride-one channel max and transposed convolution, 32
    channels, a final convolution to one channel; P = 111,361) on the 12x12
    t-J model (t = 1, J = 0.4, 18 holes), 1024 configurations, FP64: E_loc by
    full recomputation (every block convolution on the FP64 matrix cores), the
    exchanged-configuration pass's rate against the FP64 peak, and O_k."""
    import torch

    from paper_2204_07816_amd import inputs, nqs
    L, t, J, Kb, C, w, sp = inputs.cnn2_tj_config_inputs()
    B = sp.shape[0]
    ctx = nqs.Context.cnn2_tj(L, t, J, Kb, C, w)
    ctx.reserve(B, "full")
    spd = torch.as_tensor(sp).to(dev)
    e = torch.empty(B, dtype=torch.float64, device=dev)
    ctx.local_energy(spd[:8].contiguous(), mode="full")
    torch.cuda.synchronize()
    ctx.enable_timing(True)
    ctx.kernel_time()
    t0 = time.perf_counter()
    for _ in range(reps):
        ctx.local_energy(spd, mode="full", out=e)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1000.0 / reps
    k_ms, k_n = ctx.kernel_time()
    ctx.enable_timing(False)
    O = torch.empty(B, ctx.P, dtype=torch.float32, device=dev)
    ctx.log_deriv(spd, dtype="fp32", out=O)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.log_deriv(spd, dtype="fp32", out=O)
    torch.cuda.synchronize()
    ms_o = (time.perf_counter() - t0) * 1000.0
    del O
    items = int(ctx.connected(spd)[0].sum().item())
    N = L * L
    # per exchanged configuration: two 3x3 convolutions C -> C per block and
    # the final 3x3 convolution C -> 1 (multiply-adds counted as 2 flops)
    per_item = Kb * 2 * (2 * N * 9 * C * C) + 2 * N * 9 * C
    avg = k_ms / max(k_n, 1)
    achieved = items * per_item / (avg * 1e-3) / 1e12
    assert ctx.get_error() == 0
    ctx.close()
    return {"workload": f"{L}x{L} t-J (t={t}, J={J}, {inputs.CNN2_TJ_CONFIG['n_holes']} holes), "
                        f"CNN2 {Kb} blocks x {C} channels (P={inputs.cnn2_num_params(Kb, C)}), "
                        f"{B} configurations, FP64",
            "samples_per_s": B / (ms * 1e-3), "ms": ms, "exchanged_configurations": items,
            "conn_pass_ms": avg, "conn_pass_tflops": achieved, "bound": "mfma",
            "frac_fp64_peak": achieved / PEAK_FP64_TFLOPS,
            "frac_fp64_sustained": achieved / SUSTAINED["fp64_tflops"], "flops_per_item": per_item,
            "log_deriv_fp32_ms": ms_o}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--fp64-samples", type=int, default=1024)
    ap.add_argument("--no-stress", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-recompute", action="store_true")
    ap.add_argument("--no-mcmc", action="store_true")
    ap.add_argument("--no-vmc", action="store_true")
    ap.add_argument("--no-tj", action="store_true")
    ap.add_argument("--no-cnn1", action="store_true")
    ap.add_argument("--no-cnn1-36", action="store_true")
    ap.add_argument("--no-cnn2", action="store_true")
    ap.add_argument("--no-cmp10", action="store_true")
    ap.add_argument("--no-depths", action="store_true")
    ap.add_argument("--no-graph", action="store_true",
                    help="time eager calls instead of replays of the captured step")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--mode", default="incremental", choices=["incremental", "full"])
    ap.add_argument("--form", default="bf16x3", choices=["bf16x3", "bf16"],
                    help="arithmetic of the timed step's convolutions")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain BF16 row")
    ap.add_argument("--no-sr24", action="store_true")
    ap.add_argument("--only", default=None, choices=["eloc", "oderiv", "eloc64", "tj", "cnn1", "cnn1_36",
                                                     "cnn2", "sr24", "cmp10", "depths",
                                                     "stress_cone"],
                    help="profiling aid: eloc runs only the local-energy call --steps times, "
                         "then a 1 GiB device copy (reference for the HBM byte counters); "
                         "oderiv likewise the FP32 log-derivative call; eloc64 likewise the "
                         "FP64 local-energy call in --mode; tj runs only the t-J "
                         "row and prints it; cnn1, cnn2, sr24, cmp10 and depths likewise their rows")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(samples would be split across GPUs, with one all-reduce of P values "
              "per CG iteration); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2204_07816_amd import inputs, nqs

    dev = torch.device("cuda:0")
    # the matrix cores' sustained rate in a register-only MFMA loop: the
    # published dense peaks are what the fractions are quoted against; this
    # is what full-load MFMA work reaches on this device (context)
    sustained = {"bf16_tflops": nqs.mfma_rate("bf16", 4096, 8000)[1],
                 "fp64_tflops": nqs.mfma_rate("fp64", 4096, 2000)[1]}
    log(f"sustained MFMA rate: {sustained['bf16_tflops']:.0f} TFLOP/s BF16, "
        f"{sustained['fp64_tflops']:.1f} TFLOP/s FP64 (register-only loop)")
    SUSTAINED.update(sustained)
    if args.only == "tj":
        print(json.dumps(tj_row(dev)), flush=True)
        return
    if args.only == "cnn1":
        print(json.dumps(cnn1_row(dev)), flush=True)
        return
    if args.only == "cnn1_36":
        print(json.dumps(cnn1_36_row(dev)), flush=True)
        return
    if args.only == "cnn2":
        print(json.dumps(cnn2_row(dev)), flush=True)
        return
    if args.only == "sr24":
        print(json.dumps(sr24_row(dev)), flush=True)
        return
    if args.only == "cmp10":
        print(json.dumps(cmp10_row(dev)), flush=True)
        return
    if args.only == "depths":
        print(json.dumps(split_depths_row(dev)), flush=True)
        return
    if args.only == "stress_cone":
        print(json.dumps(split_depths_row(dev, depths=(8,), gain=STRESS_GAIN_K8)), flush=True)
        return
    L, J2, K, C, w, sp = inputs.config_inputs("full36")
    B = sp.shape[0]
    if args.only == "eloc64":
        c64 = nqs.Context(L, 1.0, J2, K, C, w, dtype="fp64")
        c64.reserve(B, args.mode)
        spd = torch.as_tensor(sp).to(dev)
        e = torch.empty(B, dtype=torch.float64, device=dev)
        for i in range(args.steps):
            c64.local_energy(spd, mode=args.mode, out=e)
            torch.cuda.synchronize()
            log(f"eloc64 ({args.mode}) {i + 1}/{args.steps} done")
        assert c64.get_error() == 0
        return
    log(f"workload 36x36 K={K} C={C} B={B}, form {args.form}")
    spd = torch.as_tensor(sp).to(dev)
    ctx = nqs.Context(L, 1.0, J2, K, C, w, dtype=args.form)
    ctx.reserve(B, args.mode)
    P = ctx.P
    e = torch.empty(B, dtype=torch.float64, device=dev)
    st2 = torch.empty(2, dtype=torch.float64, device=dev)
    O = torch.empty(B, P, dtype=torch.float32, device=dev)
    x = torch.empty(P, dtype=torch.float64, device=dev)
    st4 = torch.empty(4, dtype=torch.float64, device=dev)

    def step():
        ctx.local_energy(spd, mode=args.mode, out=e)
        ctx.energy_stats(e, out=st2)
        ctx.log_deriv(spd, dtype="fp32", out=O)
        ctx.sr_solve(O, e, 1e-4, 100, out=x, stats=st4)

    if args.only in ("eloc", "oderiv"):
        for i in range(args.steps):
            if args.only == "eloc":
                ctx.local_energy(spd, mode=args.mode, out=e)
            else:
                ctx.log_deriv(spd, dtype="fp32", out=O)
            torch.cuda.synchronize()
            log(f"{args.only} {i + 1}/{args.steps} done")
        src = torch.empty(1 << 27, dtype=torch.float64, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log("reference copy of 1 GiB done")
        return

    for i in range(args.warmup):
        step()
        torch.cuda.synchronize()
        log(f"warmup {i + 1}/{args.warmup} done")
    graph = None
    # the step captured once in a HIP graph and replayed (every workspace was
    # grown by the warm-up calls, so the captured calls allocate nothing)
    run = step
    if not args.no_graph:
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            step()
        torch.cuda.synchronize()
        run = graph.replay
        log("step captured in a HIP graph")
    # dominant-kernel time from HIP events around its launches, in an eager
    # pass (events are not recorded inside the graph)
    ctx.kernel_time()                      # reset
    ctx.enable_timing(True)
    for _ in range(2):
        ctx.local_energy(spd, mode=args.mode, out=e)
    torch.cuda.synchronize()
    ctx.enable_timing(False)
    k_ms, k_n = ctx.kernel_time()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        run()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1000.0 / args.steps
    log(f"timed {args.steps} steps: {ms_step:.2f} ms/step")
    assert ctx.get_error() == 0

    # breakdown of one step (events on the current stream)
    def timed(fn, reps=2):
        fn()
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    t_eloc = timed(lambda: ctx.local_energy(spd, mode=args.mode, out=e))
    t_od = timed(lambda: ctx.log_deriv(spd, dtype="fp32", out=O))
    t_sr = timed(lambda: ctx.sr_solve(O, e, 1e-4, 100, out=x, stats=st4))
    # CG stops early once the residual is below 1e-30 ||F|| (converged beyond
    # FP64 resolution): report how far it went on this workload
    sr_info = {"iterations_run": int(st4[3].item()), "rel_residual": float(st4[2].item()),
               "iteration_cap": 100}
    e_b = e.cpu().numpy()
    log(f"breakdown ms: eloc {t_eloc:.2f} log_deriv {t_od:.2f} sr {t_sr:.2f}")

    # algorithmic work of the dominant kernel: the integer stage's queue,
    # listed by the library outside the timed region (bond id = 4 site + type,
    # types 2 and 3 the diagonal J2 bonds)
    cnt_d, offs_d, bonds_d, _, _ = ctx.connected(spd)
    counts = cnt_d.cpu().numpy()
    allb = bonds_d[:int(offs_d[B].item())].cpu().numpy()
    n_diag = int(np.sum(allb % 4 >= 2))
    n_j1 = int(allb.shape[0] - n_diag)
    flops_launch = n_j1 * item_flops(L, K, C, False) + n_diag * item_flops(L, K, C, True)
    if args.mode == "full":
        per_item = L * L * C * 9 * 2 + (K - 1) * L * L * C * 9 * C * 2
        flops_launch = float(allb.shape[0]) * per_item

    # the split form's shape at C = 32: two workgroups' compact windows fit a
    # CU's LDS up to K = 7; deeper cones take the frame form (one frame per
    # configuration, updated in place)
    split_label = ("k_net_cone<2, false, %d> (split BF16: hi*hi + hi*lo + lo*hi per "
                   "multiply-add, so the peak is the 2.5 PFLOP/s BF16 MFMA rate / 3), "
                   "exchanged configurations, incremental cone, %s"
                   % ((5, "frame form") if K >= 8 else (4, "compact windows")))

    def roofline_of(form, kms, kn):
        avg = kms / max(kn, 1)
        ach = flops_launch / (avg * 1e-3) / 1e12
        peak = form_peak(form)
        return {"bound": "mfma", "achieved": ach, "peak": peak, "unit": "TFLOP/s",
                "frac": ach / peak, "traffic": traffic_from_profile(form),
                "kernel": split_label if form == "bf16x3" else
                          "k_net_cone<2, false, 1> (plain BF16), exchanged configurations, "
                          "incremental cone, compact windows",
                "avg_launch_ms": avg, "launches": kn, "flops_per_launch": flops_launch,
                "items_per_launch": int(allb.shape[0]),
                "mfma_instruction_tflops": ach * (3 if form == "bf16x3" else 1),
                "sustained_peak": SUSTAINED["bf16_tflops"] / (3 if form == "bf16x3" else 1),
                "frac_of_sustained": ach * (3 if form == "bf16x3" else 1) / SUSTAINED["bf16_tflops"],
                "sustained_note": "sustained_peak: the BF16 MFMA rate a register-only loop of "
                                  "independent MFMAs reaches on this device (nqs_mfma_rate), per "
                                  "algorithmic flop of this form"}

    roofline = roofline_of(args.form, k_ms, k_n)

    # the other form's whole step, non-gating (same timing as the headline)
    plain = None
    other = "bf16" if args.form == "bf16x3" else "bf16x3"
    if not args.no_plain:
        co = nqs.Context(L, 1.0, J2, K, C, w, dtype=other)
        co.reserve(B, args.mode)
        eo = torch.empty_like(e)

        def step_o():
            co.local_energy(spd, mode=args.mode, out=eo)
            co.energy_stats(eo, out=st2)
            co.log_deriv(spd, dtype="fp32", out=O)
            co.sr_solve(O, eo, 1e-4, 100, out=x, stats=st4)

        step_o()
        torch.cuda.synchronize()
        co.kernel_time()
        co.enable_timing(True)
        for _ in range(2):
            co.local_energy(spd, mode=args.mode, out=eo)
        torch.cuda.synchronize()
        co.enable_timing(False)
        ko_ms, ko_n = co.kernel_time()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            step_o()
        torch.cuda.synchronize()
        ms_o = (time.perf_counter() - t0) * 1000.0 / args.steps
        plain = {"form": other, "samples_per_s": B / (ms_o * 1e-3), "ms_per_step": ms_o,
                 "hip_graph": False, "roofline": roofline_of(other, ko_ms, ko_n),
                 "mean_rel_err_vs_headline_form": float(
                     abs(eo.mean().item() - e.mean().item()) / abs(e.mean().item()))}
        assert co.get_error() == 0
        co.close()
        log(f"{other} step (eager): {ms_o:.2f} ms, kernel frac {plain['roofline']['frac']:.3f}")

    # plain FP64 GPU form, and the bar at the workload's own weights (vacuous:
    # the log ratios there are below FP64 resolution)
    fp64 = None
    if not args.no_fp64:
        nsub = args.fp64_samples
        c64 = nqs.Context(L, 1.0, J2, K, C, w, dtype="fp64")
        sub = spd[:nsub].contiguous()
        e64 = torch.empty(nsub, dtype=torch.float64, device=dev)
        c64.reserve(nsub, "full")
        # one warm call on a few samples, then the timed call on all of them
        c64.local_energy(sub[:4], mode="full", out=e64[:4])
        torch.cuda.synchronize()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record()
        c64.local_energy(sub, mode="full", out=e64)
        ev1.record()
        torch.cuda.synchronize()
        t64 = ev0.elapsed_time(ev1)
        e64n = e64.cpu().numpy()
        rel = abs(e_b[:nsub].mean() - e64n.mean()) / abs(e64n.mean())
        fp64 = {"samples_per_s": nsub / (t64 * 1e-3), "samples": nsub, "ms": t64,
                "headline_form_mean_rel_err": rel, "headline_form_max_rel_err": float(
                    np.max(np.abs(e_b[:nsub] - e64n)) / np.max(np.abs(e64n))),
                "note": "at the workload's weights the log ratios are below FP64 resolution, "
                        "so this comparison cannot fail; the gate is precision_gate"}
        log(f"fp64 plain: {fp64['samples_per_s']:.2f} samples/s, {args.form} mean rel err {rel:.3e}")
        # the FP64 receptive cone on the same samples: whole call, and the cone
        # kernel's algorithmic FP64 rate (item_flops over the queue)
        c64.reserve(nsub, "incremental")
        e64i = torch.empty_like(e64)
        c64.local_energy(sub[:4], mode="incremental", out=e64i[:4])
        torch.cuda.synchronize()
        c64.kernel_time()
        c64.enable_timing(True)
        ev0.record()
        c64.local_energy(sub, mode="incremental", out=e64i)
        ev1.record()
        torch.cuda.synchronize()
        c64.enable_timing(False)
        t64i = ev0.elapsed_time(ev1)
        ki_ms, ki_n = c64.kernel_time()
        _, offs64, bonds64, _, _ = c64.connected(sub)
        b64 = bonds64[:int(offs64[-1].item())].cpu().numpy()
        nd64 = int(np.sum(b64 % 4 >= 2))
        fl64 = (b64.shape[0] - nd64) * item_flops(L, K, C, False) + nd64 * item_flops(L, K, C, True)
        tf64 = fl64 / (ki_ms / max(ki_n, 1) * 1e-3) / 1e12
        e64in = e64i.cpu().numpy()
        fp64["incremental"] = {
            "samples_per_s": nsub / (t64i * 1e-3), "ms": t64i,
            "speedup_vs_full": t64 / t64i,
            "eloc_max_rel_diff_vs_full": float(np.max(np.abs(e64in - e64n)) / np.max(np.abs(e64n))),
            "cone_kernel": {"name": "k_net_cone64<32>", "bound": "mfma", "ms": ki_ms / max(ki_n, 1),
                            "items": int(b64.shape[0]), "flops": fl64, "tflops": tf64,
                            "frac_fp64_peak": tf64 / PEAK_FP64_TFLOPS,
                            "frac_fp64_sustained": tf64 / SUSTAINED["fp64_tflops"]}}
        log(f"fp64 cone: {fp64['incremental']['samples_per_s']:.1f} samples/s "
            f"({fp64['incremental']['speedup_vs_full']:.2f}x full), kernel {tf64:.1f} TFLOP/s "
            f"({tf64 / PEAK_FP64_TFLOPS:.3f} of peak)")
        c64.close()

    gate, stress_other = None, None
    if not args.no_stress:
        gate = stress_row(L, J2, K, C, sp, dev, args.form)
        gate["gating"] = True
        log(f"precision gate ({args.form}): std log ratio {gate['std_log_ratio']:.3f}, "
            f"mean rel err {gate['mean_rel_err_vs_fp64']:.3e}, met {gate['bar_1e-5_met']}")
        stress_other = stress_row(L, J2, K, C, sp, dev, other)
        stress_other["gating"] = False
        log(f"stress row ({other}): mean rel err {stress_other['mean_rel_err_vs_fp64']:.3e}")

    sr24 = None
    if not args.no_sr24:
        sr24 = sr24_row(dev)
        log(f"sr 24x24: {sr24['iterations_run']} iterations, {sr24['ms_per_iteration']:.3f} ms "
            f"each, {sr24['streaming_gbs']:.0f} GB/s")

    mixed = None
    if not args.no_mixed:
        mixed = mixed_row(dev)
        log(f"mixed lattices: {mixed['samples_per_s']:.1f} samples/s ({mixed['lattices']})")

    recompute = None
    if not args.no_recompute:
        # SR with O recomputed from the spins in chunks of 256 samples (for
        # batches whose O does not fit): per-iteration cost, and equality with
        # the stored-O solve over the same iterations
        n_it, rows = 5, 256
        xr = torch.empty_like(x)
        sr4 = torch.empty_like(st4)
        ctx.sr_solve_recompute(spd, e, 1e-4, 1, dtype="fp32", chunk_rows=rows, out=xr, stats=sr4)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.sr_solve_recompute(spd, e, 1e-4, n_it, dtype="fp32", chunk_rows=rows, out=xr,
                               stats=sr4)
        torch.cuda.synchronize()
        t_rc = (time.perf_counter() - t0) * 1000.0
        t0 = time.perf_counter()
        ctx.sr_solve(O, e, 1e-4, n_it, out=x, stats=st4)
        torch.cuda.synchronize()
        t_st = (time.perf_counter() - t0) * 1000.0
        recompute = {"chunk_rows": rows, "iterations": n_it, "ms_total": t_rc,
                     "stored_O_ms_total": t_st,
                     "equal_to_stored_O": bool(torch.equal(xr, x))}
        log(f"sr recompute: {t_rc:.1f} ms for {n_it} iterations, equal {recompute['equal_to_stored_O']}")

    mcmc = None
    if not args.no_mcmc:
        # Metropolis steps of the 1024 chains (one pair-exchange proposal per
        # chain per step), seeded random numbers on the device
        n_st = 20
        gen = torch.Generator(device=dev)
        gen.manual_seed(2024)
        rb = torch.randint(0, 2 ** 31 - 1, (n_st, B), device=dev, dtype=torch.int64,
                           generator=gen).to(torch.int32)
        ru = torch.rand(n_st, B, device=dev, dtype=torch.float64, generator=gen)
        chains = spd.clone()
        ctx.mcmc(chains, rb[:1], ru[:1], mode=args.mode)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        acc = ctx.mcmc(chains, rb, ru, mode=args.mode)
        torch.cuda.synchronize()
        t_mc = (time.perf_counter() - t0) * 1000.0
        mcmc = {"chains": B, "steps": n_st, "ms_per_step": t_mc / n_st,
                "proposals_per_s": B * n_st / (t_mc * 1e-3),
                "acceptance": float(acc.sum().item()) / (B * n_st)}
        log(f"mcmc: {mcmc['ms_per_step']:.3f} ms per step of {B} chains, "
            f"acceptance {mcmc['acceptance']:.3f}")

    vmc = None
    if not args.no_vmc:
        # whole VMC iterations captured in one HIP graph: 10 Metropolis steps
        # of the chains, E_loc, statistics, O (FP32), SR and the weight update
        # on the device; each iteration's random numbers are staged first
        from paper_2204_07816_amd.vmc import VMC
        cv = nqs.Context(L, 1.0, J2, K, C, w, dtype=args.form)
        run = VMC(cv, spd.clone(), steps=10, lr=0.01, diag_shift=1e-3, cg_iters=100,
                  seed=3, o_dtype="fp32", mode=args.mode)
        run.step()                                  # sizes every workspace
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            run.stage()
            run.enqueue()
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        gv = torch.cuda.CUDAGraph()
        with torch.cuda.graph(gv):
            run.enqueue()
        n_v, t_v, energies = 3, 0.0, []
        for i in range(n_v):
            run.stage(10 + i)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            gv.replay()
            torch.cuda.synchronize()
            t_v += (time.perf_counter() - t0) * 1000.0
            energies.append(run.stats()["energy"])
        t_v /= n_v
        vmc = {"ms_per_iteration": t_v, "chains": B, "mcmc_steps_per_iteration": 10,
               "samples_per_s": B / (t_v * 1e-3), "hip_graph": True, "energies": energies}
        log(f"vmc: {t_v:.1f} ms per graph-replayed iteration")
        del gv
        cv.close()

    tj = None
    if not args.no_tj:
        tj = tj_row(dev)
        log(f"t-J 12x12: {tj['samples_per_s']:.1f} samples/s ({tj['mode']}), kernel "
            f"{tj['kernel_tflops']:.0f} TFLOP/s, bf16 mean rel err {tj['bf16_mean_rel_err_vs_fp64']:.2e}")

    cnn1 = None
    if not args.no_cnn1:
        cnn1 = cnn1_row(dev)
        log(f"CNN1 10x10: {cnn1['samples_per_s']:.1f} samples/s, exchanged-configuration pass "
            f"{cnn1['conn_pass_tflops']:.2f} TFLOP/s FP64")
    cnn1_36 = None
    if not args.no_cnn1_36:
        cnn1_36 = cnn1_36_row(dev)
        log(f"CNN1 36x36: full {cnn1_36['full']['samples_per_s']:.1f}, cone "
            f"{cnn1_36['incremental']['samples_per_s']:.1f} samples/s, cone kernel "
            f"{cnn1_36['cone_kernel']['tflops']:.2f} TFLOP/s FP64")

    depths = None
    if not args.no_depths:
        depths = split_depths_row(dev)
        log("split cone by depth: " + ", ".join(f"{k} {v['cone_ms']:.1f} ms ({v['frac']:.3f})"
                                                 for k, v in depths.items()))
        # the headline depth at the precision gate's stress weights, where most
        # pre-activations take ln cosh's exponential branch
        depths["K8_stress"] = split_depths_row(dev, depths=(8,), gain=STRESS_GAIN_K8)["K8"]
        log(f"split cone at stress weights, K = 8: {depths['K8_stress']['cone_ms']:.1f} ms")

    cnn2 = None
    if not args.no_cnn2:
        cnn2 = cnn2_row(dev)
        log(f"CNN2 t-J 12x12: {cnn2['samples_per_s']:.1f} samples/s, exchanged-configuration pass "
            f"{cnn2['conn_pass_tflops']:.2f} TFLOP/s FP64")

    cmp10 = None
    if not args.no_cmp10:
        cmp10 = cmp10_row(dev)
        f = cmp10["forms"]
        log(f"10x10 precision comparison: fp64 {f['fp64']['samples_per_s']:.0f}, fp32 "
            f"{f['fp32']['samples_per_s']:.0f}, bf16 {f['bf16']['samples_per_s']:.0f} samples/s "
            f"(bf16 mean rel err {f['bf16']['mean_rel_err_vs_fp64']:.1e})")

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(L, J2, K, C, w, sp, float(counts.mean()))
        log(f"cpu oracle: {cpu['value']:.4f} samples/s on {cpu['cores']} cores")

    value = B / (ms_step * 1e-3)
    out = {
        "metric": "E_loc samples/s, 36x36 J1-J2, BF16 vs FP64 GPU at mean-energy rel err <=1e-5",
        "value": value, "unit": "samples/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": args.form, "data": "synthetic",
        "config": {"workload": "36x36 J1-J2 (J2=0.5), CNN 8x3x3x32 (P=65056), 1024 Sz=0 "
                               f"configurations; step = E_loc + stats + O_k + SR (CG, "
                               f"{sr_info['iterations_run']} of at most 100 iterations run)",
                   "L": L, "K": K, "C": C, "B": B, "mode": args.mode, "form": args.form,
                   "hip_graph": not args.no_graph,
                   "mean_connected": float(counts.mean())},
        "breakdown_ms": {"e_loc": t_eloc, "log_deriv": t_od, "sr_solve": t_sr},
        "sr_cg": sr_info,
        "eloc_only_samples_per_s": B / (t_eloc * 1e-3),
        "precision_gate": gate,
        "other_form_nongating": plain,
        "other_form_stress_nongating": stress_other,
        "fp64_gpu": fp64,
        "sr24_nongating": sr24,
        "mixed_lattices_nongating": mixed,
        "sr_recompute_nongating": recompute,
        "mcmc_nongating": mcmc,
        "vmc_iteration_nongating": vmc,
        "tj_nongating": tj,
        "cnn1_nongating": cnn1,
        "cnn1_36x36_nongating": cnn1_36,
        "split_cone_depths_nongating": depths,
        "cnn2_tj_nongating": cnn2,
        "cmp10_nongating": cmp10,
        "roofline": roofline,
        "mfma_sustained_tflops": SUSTAINED,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
