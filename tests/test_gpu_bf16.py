"""GPU BF16-MFMA path (FP32 accumulate, FP64 ratios and sums).

* Incremental receptive-cone mode vs full recompute: both run the same tile
  arithmetic, so their log ratios agree to FP64 summation order
  (|diff| <= 1e-12 (1 + |d|)); this pins the cone / window / cache logic.
* Mean energy within 1e-5 relative of the FP64 oracle and of the FP64 GPU
  form (the BF16 bar); per-item errors at large weights are reported.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2204_07816_amd import inputs
from gpu_helpers import make_ctx, oracle_item_dlog, rel_inf, say, to_dev

pytestmark = pytest.mark.gpu


CONE_CASES = [
    ("36x36 K8 C32 stress", 36, 0.5, 8, 32, 3, "stress"),
    ("12x12 K6 C32 J2=0 (cones wrap)", 12, 0.0, 6, 32, 6, "stress"),
    ("20x20 K6 C32 J2=0.55", 20, 0.55, 6, 32, 3, "stress"),
    ("10x10 K4 C16", 10, 0.5, 4, 16, 16, "stress"),
    ("16x16 K6 C32 bj", 16, 0.5, 6, 32, 4, "bj"),
    ("8x8 K2 C16", 8, 0.5, 2, 16, 8, "stress"),
    # unwrapped-window kernel at its smallest lattice, and with rings larger
    # than its prefetch registers
    ("8x8 K2 C32 unwrapped", 8, 0.5, 2, 32, 6, "stress"),
    ("28x28 K12 C32 ring tail", 28, 0.5, 12, 32, 2, "stress"),
]


@pytest.mark.parametrize("name,L,J2,K,C,B,wk", CONE_CASES, ids=[c[0] for c in CONE_CASES])
def test_incremental_equals_full(name, L, J2, K, C, B, wk):
    say("case", name)
    w = inputs.stress_weights(K, C, 1.0, 21) if wk == "stress" else inputs.weights(K, C, 0.02, 21)
    sp = inputs.spins_sz0(L, B, 22)
    ctx = make_ctx(L, J2, K, C, w, dtype="bf16")
    dfull = ctx.log_ratios(to_dev(sp), mode="full").cpu().numpy()
    dinc = ctx.log_ratios(to_dev(sp), mode="incremental").cpu().numpy()
    n = ctx.capacity(B)
    counts, _, _, _ = oracle.connected(L, 1.0, J2, sp)
    q = int(counts.sum())
    diff = np.abs(dfull[:q] - dinc[:q])
    say("  items", q, "max |full-incr|", diff.max(), "max |d|", np.abs(dfull[:q]).max())
    assert np.all(diff <= 1e-12 * (1 + np.abs(dfull[:q])))
    assert ctx.get_error() == 0
    del n


def test_bf16_vs_oracle_items_stress():
    """Per-item BF16 log ratios against the oracle at weights where they are O(1)."""
    L, J2, K, C = 10, 0.5, 4, 16
    w = inputs.stress_weights(K, C, 1.0, 31)
    sp = inputs.spins_sz0(L, 4, 32)
    ctx = make_ctx(L, J2, K, C, w, dtype="bf16")
    d = ctx.log_ratios(to_dev(sp), mode="auto").cpu().numpy()
    counts, bonds, _, _ = oracle.connected(L, 1.0, J2, sp)
    offs = np.concatenate([[0], np.cumsum(counts)])
    errs, mags = [], []
    for s in range(4):
        for q in range(0, counts[s], 7):
            ref = oracle_item_dlog(L, K, C, w, sp, s, bonds[s][q])
            errs.append(abs(d[offs[s] + q] - ref))
            mags.append(abs(ref))
    errs, mags = np.array(errs), np.array(mags)
    say("bf16 stress: max err", errs.max(), "median err", np.median(errs), "median |d|",
        np.median(mags))
    assert np.median(errs) <= 0.02 * max(np.median(mags), 1e-3)


def test_cmp10_mean_energy_bf16_vs_oracle_and_fp64():
    """10x10, K=4, C=16, sigma=0.02: BF16 mean energy within 1e-5 of FP64."""
    L, J2, K, C, w, sp = inputs.config_inputs("cmp10")
    sub = sp[:48]
    cb = make_ctx(L, J2, K, C, w, dtype="bf16")
    cf = make_ctx(L, J2, K, C, w, dtype="fp64")
    eb = cb.local_energy(to_dev(sp)).cpu().numpy()
    ef = cf.local_energy(to_dev(sp), mode="full").cpu().numpy()
    rel_mean = abs(eb.mean() - ef.mean()) / abs(ef.mean())
    say("cmp10 B=8192: mean bf16", eb.mean(), "fp64", ef.mean(), "rel", rel_mean,
        "max per-sample rel", rel_inf(eb, ef))
    assert rel_mean <= 1e-5
    ref = oracle.local_energy(L, 1.0, J2, K, C, w, sub)
    assert abs(eb[:48].mean() - ref.mean()) <= 1e-5 * abs(ref.mean())
    assert rel_inf(ef[:48], ref) <= 1e-10
    f32 = make_ctx(L, J2, K, C, w, dtype="fp32")
    e32 = f32.local_energy(to_dev(sp[:512]), mode="full").cpu().numpy()
    say("cmp10 fp32 mean rel", abs(e32.mean() - ef[:512].mean()) / abs(ef[:512].mean()))
    assert abs(e32.mean() - ef[:512].mean()) <= 1e-6 * abs(ef[:512].mean())


def test_full36_bf16_incremental_vs_fp64():
    """36x36 J1-J2, K=8, C=32: BF16 incremental E_loc for 1024 samples; FP64 on a subset."""
    L, J2, K, C, w, sp = inputs.config_inputs("full36")
    cb = make_ctx(L, J2, K, C, w, dtype="bf16")
    assert cb.auto_mode() == "incremental"
    eb = cb.local_energy(to_dev(sp), mode="incremental").cpu().numpy()
    cf = make_ctx(L, J2, K, C, w, dtype="fp64")
    ef = cf.local_energy(to_dev(sp[:8]), mode="full").cpu().numpy()
    rel = abs(eb[:8].mean() - ef.mean()) / abs(ef.mean())
    say("full36: mean bf16(8)", eb[:8].mean(), "fp64(8)", ef.mean(), "rel", rel,
        "max per-sample rel", rel_inf(eb[:8], ef))
    assert rel <= 1e-5
    assert np.all(np.isfinite(eb))
    la_b = cb.log_psi(to_dev(sp[:4]))[0].cpu().numpy()
    la_o, _ = oracle.log_psi(L, K, C, w, sp[:4])
    say("full36 log_psi bf16 rel err", rel_inf(la_b, la_o))
    assert rel_inf(la_b, la_o) <= 1e-2
    assert cb.get_error() == 0


def test_log_psi_bf16_matches_oracle_small():
    L, K, C = 8, 3, 16
    w = inputs.weights(K, C, 0.3, 3)
    sp = inputs.spins_any(L, 16, 4)
    ctx = make_ctx(L, 0.5, K, C, w, dtype="bf16")
    la, sg = ctx.log_psi(to_dev(sp))
    ol, os_ = oracle.log_psi(L, K, C, w, sp)
    say("bf16 log_psi rel", rel_inf(la.cpu().numpy(), ol))
    assert rel_inf(la.cpu().numpy(), ol) <= 2e-2
    assert np.array_equal(sg.cpu().numpy(), os_)
