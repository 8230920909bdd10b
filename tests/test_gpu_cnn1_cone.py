"""The CNN1 receptive-cone pass [Sec. 5.2 network, Sec. 5.4.1 local energy]
on the GPU: INCREMENTAL mode of a CNN1 context with 16 channels, K <= 6 and
L >= 4K + 4, against the oracle's CNN1.

Exchanging a pair changes layer l (block b's convolution is layer 2b - 1, its
transposed convolution layer 2b) only on the box widened by l sites, so the
kernel forms log|psi(S')| - log|psi(S)| as a sum over that region of the last
layer.  Every neuron it forms has the full pass's operand order, so the two
differ only in the order of the final sum; the oracle's f(S') - f(S), a
difference of two sums of N C logarithms, carries the larger rounding.  The
per-item bound used below is that sum's random-walk rounding scale with a
factor 64, 64 eps sqrt(N C) (|f(S)| + |f(S')|), plus 1e-10.

* every item's log ratio, from oracle forwards of S and S' (network only),
  on 12x12 (the smallest lattice the cone serves at K = 2, J1 bonds 2x1 and
  1x2 and J2 bonds 2x2), 14x14 (J1 only) and 16x16 at K = 3;
* E_loc (network sign ratios and the Marshall sign included) within 1e-10
  relative of the oracle;
* 36x36 with 6 blocks (the paper's largest lattice and CNN1 depth): every item
  against the full recomputation on the GPU (itself pinned to the oracle),
  sampled items against the oracle, E_loc against the full pass;
* the smallest lattice the cone serves at K = 4 and 5 (L = 4K + 4);
* edge cases: a Neel state (every J1 bond exchanged), a ferromagnet (no
  items), the AUTO choice, refusals below 4K + 4;
* the t-J model with the CNN1 amplitude (hops and spin exchanges, 12x12 at
  hole doping 1/8) against the oracle;
* Metropolis chains in INCREMENTAL mode equal the oracle's; the autotuner
  times both forms; a VMC iteration captured in a HIP graph (the cone pass
  and the cache copies inside) equals the eager iterations.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2204_07816_amd import inputs, nqs
from gpu_helpers import DEV, graph_replays_equal_eager, rel_inf, say, to_dev

pytestmark = pytest.mark.gpu

EPS = np.finfo(np.float64).eps
C16 = 16


def c1_ctx(L, Kb, w, J2=0.5, marshall=True):
    return nqs.Context.cnn1(L, 1.0, J2, Kb, C16, w, marshall_sign=marshall)


def items_of(ctx, d):
    """(sample, bond) of every queue item, in the order of the log ratios."""
    counts, offs, bonds, _, _ = ctx.connected(d)
    offs = offs.cpu().numpy()
    bonds = bonds.cpu().numpy()
    n = int(offs[-1])
    sample = np.repeat(np.arange(len(offs) - 1), np.diff(offs))
    return sample[:n], bonds[:n]


def oracle_items(L, Kb, w, sp, sample, bond):
    """f(S) and f(S') of the given items from the oracle (network only)."""
    base = np.ascontiguousarray(sp[sample]).reshape(len(sample), -1).copy()
    ex = base.copy()
    for r, b in enumerate(bond):
        i, j, _ = oracle.bond_sites(L, int(b))
        ex[r, i], ex[r, j] = base[r, j], base[r, i]
    f0, _ = oracle.cnn1_log_psi(L, Kb, C16, w, base.reshape(-1, L, L), marshall=False)
    f1, _ = oracle.cnn1_log_psi(L, Kb, C16, w, ex.reshape(-1, L, L), marshall=False)
    return f0, f1


def item_tol(L, f0, f1):
    return 1e-10 + 64 * EPS * np.sqrt(L * L * C16) * (np.abs(f0) + np.abs(f1))


ITEM_CASES = [(12, 0.5, 2, 0.2, 1.0, 3), (14, 0.0, 2, 0.3, 0.0, 3), (16, 0.55, 3, 0.15, 1.0, 2),
              (12, 0.5, 1, 0.4, 0.0, 4)]


@pytest.mark.parametrize("L,J2,Kb,sigma,ob,B", ITEM_CASES)
def test_cone_items_match_oracle(L, J2, Kb, sigma, ob, B):
    say("cnn1 cone items", L, J2, Kb, B)
    w = inputs.cnn1_weights(Kb, C16, sigma, 201, out_bias=ob)
    sp = inputs.spins_sz0(L, B, 202)
    ctx = c1_ctx(L, Kb, w, J2=J2)
    d = to_dev(sp)
    inc = ctx.log_ratios(d, mode="incremental").cpu().numpy()
    full = ctx.log_ratios(d, mode="full").cpu().numpy()
    sample, bond = items_of(ctx, d)
    n = len(sample)
    assert n > 0
    f0, f1 = oracle_items(L, Kb, w, sp, sample, bond)
    ref = f1 - f0
    tol = item_tol(L, f0, f1)
    err = np.abs(inc[:n] - ref)
    say("  items", n, "max |inc - oracle|", err.max(), "max |inc - full|",
        np.abs(inc[:n] - full[:n]).max(), "std dlog", ref.std())
    assert np.all(err <= tol)
    assert np.all(np.abs(inc[:n] - full[:n]) <= tol)
    assert ctx.get_error() == 0


ELOC_CASES = [(12, 0.5, 2, 0.2, 1.0, 4, True), (14, 0.0, 2, 0.3, 0.0, 3, True),
              (16, 0.55, 3, 0.15, 1.0, 2, False), (12, 0.5, 1, 0.4, 0.0, 6, True)]


@pytest.mark.parametrize("L,J2,Kb,sigma,ob,B,marshall", ELOC_CASES)
def test_cone_local_energy_matches_oracle(L, J2, Kb, sigma, ob, B, marshall):
    say("cnn1 cone eloc", L, J2, Kb, B, marshall)
    w = inputs.cnn1_weights(Kb, C16, sigma, 211, out_bias=ob)
    sp = inputs.spins_sz0(L, B, 212)
    ctx = c1_ctx(L, Kb, w, J2=J2, marshall=marshall)
    e = ctx.local_energy(to_dev(sp), mode="incremental").cpu().numpy()
    ref = oracle.cnn1_local_energy(L, 1.0, J2, Kb, C16, w, sp, marshall=marshall)
    say("  max rel", rel_inf(e, ref))
    assert rel_inf(e, ref) <= 1e-10
    assert ctx.get_error() == 0


def test_cone_36x36_six_blocks():
    L, J2, Kb, B = 36, 0.5, 6, 2
    w = inputs.cnn1_weights(Kb, C16, 0.05, 221, out_bias=1.0)
    sp = inputs.spins_sz0(L, B, 222)
    ctx = c1_ctx(L, Kb, w, J2=J2)
    d = to_dev(sp)
    inc = ctx.log_ratios(d, mode="incremental").cpu().numpy()
    full = ctx.log_ratios(d, mode="full").cpu().numpy()
    sample, bond = items_of(ctx, d)
    n = len(sample)
    # every item against the full pass (scale of the full pass's own sums)
    fb, _ = ctx.log_psi(d)
    fb = fb.cpu().numpy()
    tol_all = item_tol(L, fb[sample], fb[sample] + full[:n])
    say("36x36 items", n, "max |inc - full|", np.abs(inc[:n] - full[:n]).max(),
        "std dlog", full[:n].std())
    assert np.all(np.abs(inc[:n] - full[:n]) <= tol_all)
    # sampled items against the oracle, the first and the last included
    rng = np.random.default_rng(223)
    pick = np.unique(np.concatenate([rng.choice(n, 10, replace=False), [0, n - 1]]))
    f0, f1 = oracle_items(L, Kb, w, sp, sample[pick], bond[pick])
    err = np.abs(inc[pick] - (f1 - f0))
    say("  sampled vs oracle", err.max())
    assert np.all(err <= item_tol(L, f0, f1))
    e_inc = ctx.local_energy(d, mode="incremental")
    e_full = ctx.local_energy(d, mode="full")
    say("  eloc rel", rel_inf(e_inc.cpu().numpy(), e_full.cpu().numpy()))
    assert rel_inf(e_inc.cpu().numpy(), e_full.cpu().numpy()) <= 1e-10
    assert ctx.get_error() == 0


@pytest.mark.parametrize("L,Kb,J2", [(20, 4, 0.5), (24, 5, 0.0)])
def test_cone_minimal_lattice_per_depth(L, Kb, J2):
    # L = 4K + 4, the smallest lattice the cone serves at this depth: the frame
    # spans the whole width, and K = 4, 5 give other staging and ring sizes
    B = 2
    w = inputs.cnn1_weights(Kb, C16, 0.1, 281 + Kb, out_bias=1.0)
    sp = inputs.spins_sz0(L, B, 282 + Kb)
    ctx = c1_ctx(L, Kb, w, J2=J2)
    d = to_dev(sp)
    inc = ctx.log_ratios(d, mode="incremental").cpu().numpy()
    full = ctx.log_ratios(d, mode="full").cpu().numpy()
    sample, bond = items_of(ctx, d)
    n = len(sample)
    fb = ctx.log_psi(d)[0].cpu().numpy()
    assert np.all(np.abs(inc[:n] - full[:n]) <= item_tol(L, fb[sample], fb[sample] + full[:n]))
    rng = np.random.default_rng(283)
    pick = np.unique(np.concatenate([rng.choice(n, 8, replace=False), [0, n - 1]]))
    f0, f1 = oracle_items(L, Kb, w, sp, sample[pick], bond[pick])
    err = np.abs(inc[pick] - (f1 - f0))
    say("L", L, "K", Kb, "items", n, "sampled vs oracle", err.max())
    assert np.all(err <= item_tol(L, f0, f1))
    e_inc = ctx.local_energy(d, mode="incremental").cpu().numpy()
    e_full = ctx.local_energy(d, mode="full").cpu().numpy()
    assert rel_inf(e_inc, e_full) <= 1e-10
    assert ctx.get_error() == 0


def test_cone_edge_cases():
    L, Kb = 12, 2
    w = inputs.cnn1_weights(Kb, C16, 0.3, 231, out_bias=1.0)
    neel = np.fromfunction(lambda y, x: np.where((x + y) % 2 == 0, 1, -1), (L, L)).astype(np.int8)
    ferro = np.ones((L, L), np.int8)
    sp = np.stack([neel, ferro, -neel])
    ctx = c1_ctx(L, Kb, w, J2=0.0)
    d = to_dev(sp)
    counts, _, _, _, _ = ctx.connected(d)
    assert counts.cpu().tolist() == [2 * L * L, 0, 2 * L * L]
    e = ctx.local_energy(d, mode="incremental").cpu().numpy()
    ref = oracle.cnn1_local_energy(L, 1.0, 0.0, Kb, C16, w, sp)
    assert rel_inf(e, ref) <= 1e-10
    # AUTO picks the cone here (its positions are 38% of the full pass's)
    assert ctx.auto_mode() == "incremental"
    assert torch.equal(ctx.local_energy(d), ctx.local_energy(d, mode="incremental"))
    # below 4K + 4 (the frame would overlap itself), other widths: refused
    small = c1_ctx(10, Kb, w, J2=0.0)
    with pytest.raises(nqs.NqsError) as info:
        small.local_energy(to_dev(inputs.spins_sz0(10, 2, 232)), mode="incremental")
    assert info.value.code == 10
    assert small.auto_mode() == "full"
    w8 = inputs.cnn1_weights(Kb, 8, 0.3, 233)
    c8 = nqs.Context.cnn1(L, 1.0, 0.5, Kb, 8, w8)
    with pytest.raises(nqs.NqsError) as info:
        c8.local_energy(to_dev(inputs.spins_sz0(L, 2, 234)), mode="incremental")
    assert info.value.code == 10
    assert ctx.get_error() == 0


@pytest.mark.parametrize("marshall", [True, False])
def test_cone_tj_local_energy_matches_oracle(marshall):
    # t-J with the CNN1 amplitude on 12x12 (hole doping 1/8): hops and spin
    # exchanges both swap the values of two neighbouring sites, so the same
    # cone serves them; the network's sign ratio meets the Jordan-Wigner sign
    L, Kb, B, t, J = 12, 2, 3, 1.0, 0.4
    w = inputs.cnn1_weights(Kb, C16, 0.3, 271, out_bias=1.0)
    sp = inputs.spins_tj(L, B, 18, 272)
    ctx = nqs.Context.cnn1_tj(L, t, J, Kb, C16, w, marshall_sign=marshall)
    d = to_dev(sp)
    e = ctx.local_energy(d, mode="incremental").cpu().numpy()
    ref = oracle.tj_cnn1_local_energy(L, t, J, Kb, C16, w, sp, marshall=marshall)
    say("t-J cnn1 cone: max rel", rel_inf(e, ref))
    assert rel_inf(e, ref) <= 1e-10
    assert torch.equal(ctx.local_energy(d), ctx.local_energy(d, mode="incremental"))
    assert ctx.get_error() == 0


def test_cone_mcmc_equals_oracle():
    L, Kb, B, T = 12, 2, 16, 6
    w = inputs.cnn1_weights(Kb, C16, 0.3, 241, out_bias=1.0)
    sp = inputs.spins_sz0(L, B, 242)
    rb, ru = inputs.mcmc_randoms(243, 0, T, B)
    ctx = c1_ctx(L, Kb, w)
    d = to_dev(sp)
    acc = ctx.mcmc(d, torch.tensor(rb, device=DEV), torch.tensor(ru, device=DEV),
                   mode="incremental")
    ref, racc = oracle.cnn1_mcmc(L, 1.0, 0.5, Kb, C16, w, sp, rb, ru)
    say("accepted", int(acc.sum()), "of", B * T)
    assert np.array_equal(d.cpu().numpy(), ref)
    assert np.array_equal(acc.cpu().numpy(), racc)
    assert ctx.get_error() == 0


def test_cone_autotune_times_both_forms():
    L, Kb, B = 16, 3, 8
    w = inputs.cnn1_weights(Kb, C16, 0.15, 251, out_bias=1.0)
    d = to_dev(inputs.spins_sz0(L, B, 252))
    ctx = c1_ctx(L, Kb, w)
    got = ctx.autotune(d)
    say("autotune picks", got)
    assert got in ("full", "incremental") and ctx.auto_mode() == got
    e = ctx.local_energy(d)
    assert torch.equal(e, ctx.local_energy(d, mode=got))
    assert ctx.get_error() == 0


def test_cone_vmc_iteration_captured_in_graph():
    L, Kb, B = 12, 2, 16
    w = inputs.cnn1_weights(Kb, C16, 0.05, 261, out_bias=1.0)
    ctx = c1_ctx(L, Kb, w)
    assert ctx.auto_mode() == "incremental"
    graph_replays_equal_eager(ctx, w, to_dev(inputs.spins_sz0(L, B, 262)), steps=3, lr=0.01,
                              diag_shift=1e-2, cg_iters=10, seed=263)
    assert ctx.get_error() == 0
