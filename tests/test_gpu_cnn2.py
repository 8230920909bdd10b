"""The CNN2 network family [Sec. 5.2] with the t-J model [Sec. 6.1] on the
GPU (nqs_create_cnn2_tj, FP64, 16 or 32 channels on the FP64 matrix cores)
against the oracle.  The architecture is a reading of a missing figure (see
oracle/nqs_oracle.h); these tests pin the GPU to the oracle's CNN2.

* log|psi| within 1e-12 relative and signs (network times Marshall) equal,
  4x4 to 12x12, 1 to 6 blocks, with and without the Marshall sign;
* E_loc within 1e-10 relative of the oracle, the network's sign ratios
  entering every term with the Jordan-Wigner and Marshall signs;
* the Rayleigh quotient over the 4x4 sector of two up and two down electrons
  from GPU amplitudes and local energies equals the exact-diagonalisation
  value (1e-10);
* O rows (FP64) within 1e-10 of the oracle at each row's scale, FP32 rows
  within 1e-6;
* Metropolis chains equal the oracle's bit for bit; SR on recomputed O equals
  SR on stored O; the device weight update equals setting the weights; a VMC
  iteration captured in a HIP graph equals the eager iterations;
* incremental mode, other channel counts, wrong parameter counts and a
  multi-lattice call mixing network families are refused; the autotuner
  answers FULL and the multi-lattice call equals the single calls.
"""
import numpy as np
import pytest
import torch

import oracle
from oracle import ed
from paper_2204_07816_amd import inputs, nqs
from gpu_helpers import DEV, graph_replays_equal_eager, rel_inf, say, to_dev

pytestmark = pytest.mark.gpu

T_HOP, J_EX = 1.0, 0.4


def c2_ctx(L, Kb, C, w, marshall=True):
    return nqs.Context.cnn2_tj(L, T_HOP, J_EX, Kb, C, w, marshall_sign=marshall)


PSI_CASES = [(4, 2, 16, 2, 64), (8, 3, 16, 8, 24), (6, 1, 32, 4, 20), (12, 6, 32, 18, 4),
             (10, 2, 16, 0, 8)]


@pytest.mark.parametrize("L,Kb,C,nh,B", PSI_CASES)
def test_cnn2_log_psi(L, Kb, C, nh, B):
    say("log_psi cnn2", L, Kb, C, nh, B)
    w = inputs.cnn2_weights(Kb, C, 1.2, 201, out_bias=1.0)
    sp = inputs.spins_tj(L, B, nh, 202)
    for marshall in (True, False):
        ctx = c2_ctx(L, Kb, C, w, marshall=marshall)
        la, sg = ctx.log_psi(to_dev(sp))
        ol, os_ = oracle.cnn2_log_psi(L, Kb, C, w, sp, marshall=marshall)
        np.testing.assert_allclose(la.cpu().numpy(), ol, rtol=1e-12, atol=1e-12)
        assert np.array_equal(sg.cpu().numpy(), os_)
        assert ctx.get_error() == 0


ELOC_CASES = [(8, 8, 3, 16, 1.2, 1.0, 12), (6, 4, 2, 32, 1.5, 0.5, 8),
              (12, 18, 2, 16, 1.0, 1.0, 4), (4, 2, 6, 16, 1.2, 1.0, 16)]


@pytest.mark.parametrize("L,nh,Kb,C,gain,ob,B", ELOC_CASES)
def test_cnn2_tj_local_energy(L, nh, Kb, C, gain, ob, B):
    say("t-J cnn2 eloc", L, nh, Kb, C, B)
    w = inputs.cnn2_weights(Kb, C, gain, 211, out_bias=ob)
    sp = inputs.spins_tj(L, B, nh, 212)
    for marshall in (True, False):
        ctx = c2_ctx(L, Kb, C, w, marshall=marshall)
        e = ctx.local_energy(to_dev(sp)).cpu().numpy()
        ref = oracle.tj_cnn2_local_energy(L, T_HOP, J_EX, Kb, C, w, sp, marshall=marshall)
        say("  marshall", marshall, "max rel", rel_inf(e, ref))
        assert rel_inf(e, ref) <= 1e-10
        assert ctx.get_error() == 0


def test_cnn2_tj_rayleigh_quotient_against_ed():
    L, Kb, C = 4, 2, 16
    H, basis = ed.tj_hamiltonian(L, T_HOP, J_EX, 2, 2)
    w = inputs.cnn2_weights(Kb, C, 1.5, 221, out_bias=0.5)
    spins = ed.tj_modes_to_spins(basis, 16).reshape(-1, 4, 4)
    ctx = c2_ctx(L, Kb, C, w)
    la, sg = ctx.log_psi(to_dev(spins))
    la, sg = la.cpu().numpy(), sg.cpu().numpy()
    assert 0 < (sg < 0).sum() < sg.shape[0]
    e = ctx.local_energy(to_dev(spins)).cpu().numpy()
    psi = sg * np.exp(la - la.max())
    lhs = np.sum(psi ** 2 * e) / np.sum(psi ** 2)
    rhs = psi @ (H @ psi) / (psi @ psi)
    say("t-J sector (2,2) with CNN2: <H> gpu", lhs, "ed", rhs)
    assert lhs == pytest.approx(rhs, rel=1e-10)
    assert ctx.get_error() == 0


@pytest.mark.parametrize("L,nh,Kb,C,B", [(4, 2, 2, 16, 8), (8, 8, 3, 16, 4), (6, 4, 2, 32, 3),
                                         (12, 18, 6, 32, 2)])
def test_cnn2_log_deriv(L, nh, Kb, C, B):
    say("log_deriv cnn2", L, Kb, C, B)
    w = inputs.cnn2_weights(Kb, C, 1.2, 231, out_bias=1.0)
    sp = inputs.spins_tj(L, B, nh, 232)
    ctx = c2_ctx(L, Kb, C, w)
    O = ctx.log_deriv(to_dev(sp), dtype="fp64").cpu().numpy()
    O32 = ctx.log_deriv(to_dev(sp), dtype="fp32").cpu().numpy()
    ref = oracle.cnn2_log_deriv(L, Kb, C, w, sp)
    for s in range(B):
        scale = np.abs(ref[s]).max()
        say("  sample", s, "fp64", np.abs(O[s] - ref[s]).max() / scale,
            "fp32", np.abs(O32[s] - ref[s]).max() / scale)
        assert np.abs(O[s] - ref[s]).max() <= 1e-10 * scale
        assert np.abs(O32[s] - ref[s]).max() <= 1e-6 * scale
    assert ctx.get_error() == 0


def test_cnn2_tj_mcmc_equals_oracle():
    L, Kb, C, B, T = 6, 2, 16, 32, 20
    w = inputs.cnn2_weights(Kb, C, 1.0, 241, out_bias=1.0)
    sp = inputs.spins_tj(L, B, 4, 242)
    rb, ru = inputs.mcmc_randoms(243, 0, T, B)
    ctx = c2_ctx(L, Kb, C, w)
    d = to_dev(sp)
    acc = ctx.mcmc(d, torch.tensor(rb, device=DEV), torch.tensor(ru, device=DEV))
    ref, racc = oracle.tj_cnn2_mcmc(L, T_HOP, J_EX, Kb, C, w, sp, rb, ru)
    say("accepted", int(acc.sum()), "of", B * T)
    assert np.array_equal(d.cpu().numpy(), ref)
    assert np.array_equal(acc.cpu().numpy(), racc)
    assert 0 < racc.sum() < B * T
    assert ctx.get_error() == 0


def test_cnn2_sr_recompute_and_device_update():
    L, Kb, C, B = 6, 3, 16, 96
    w = inputs.cnn2_weights(Kb, C, 0.8, 251, out_bias=2.0)
    sp = to_dev(inputs.spins_tj(L, B, 4, 252))
    ctx = c2_ctx(L, Kb, C, w)
    e = ctx.local_energy(sp)
    O = ctx.log_deriv(sp, dtype="fp64")
    x1, st1 = ctx.sr_solve(O, e, 1e-3, 30)
    x2, st2 = ctx.sr_solve_recompute(sp, e, 1e-3, 30, dtype="fp64", chunk_rows=32)
    assert torch.equal(x1, x2) and torch.equal(st1, st2)
    other = c2_ctx(L, Kb, C, w + (-0.01) * x1.cpu().numpy())
    ctx.update_weights(x1, -0.01)
    assert np.array_equal(ctx.get_weights(), w + (-0.01) * x1.cpu().numpy())
    assert torch.equal(ctx.local_energy(sp), other.local_energy(sp))
    assert ctx.get_error() == 0


def test_cnn2_refusals():
    L, Kb, C = 6, 2, 16
    w = inputs.cnn2_weights(Kb, C, 1.0, 261, out_bias=1.0)
    sp = to_dev(inputs.spins_tj(L, 4, 4, 262))
    ctx = c2_ctx(L, Kb, C, w)
    e = torch.empty(4, dtype=torch.float64, device=DEV)
    with pytest.raises(nqs.NqsError) as info:
        ctx.local_energy(sp, mode="incremental")
    assert info.value.code == 10                # NQS_E_UNSUPPORTED
    assert ctx.autotune(sp) == "full" and ctx.auto_mode() == "full"
    other = c2_ctx(8, Kb, C, w)
    sp8 = to_dev(inputs.spins_tj(8, 3, 8, 264))
    e8 = torch.empty(3, dtype=torch.float64, device=DEV)
    nqs.local_energy_multi([(ctx, sp, e), (other, sp8, e8)], mode="full")
    assert torch.equal(e, ctx.local_energy(sp)) and torch.equal(e8, other.local_energy(sp8))
    # jobs of different network families are refused
    lc = nqs.Context.tj(L, T_HOP, J_EX, Kb, C, inputs.weights(Kb, C, 0.1, 265))
    with pytest.raises(nqs.NqsError) as info:
        nqs.local_energy_multi([(ctx, sp, e), (lc, sp, torch.empty_like(e))], mode="full")
    assert info.value.code == 3                 # NQS_E_SPEC
    with pytest.raises(nqs.NqsError) as info:
        c2_ctx(L, Kb, 8, inputs.cnn2_weights(Kb, 8, 1.0, 263))
    assert info.value.code == 3                 # NQS_E_SPEC
    with pytest.raises(nqs.NqsError) as info:
        c2_ctx(L, Kb, C, w[:-1])
    assert info.value.code == 4                 # NQS_E_NPARAMS
    assert ctx.get_error() == 0


def test_cnn2_vmc_iteration_captured_in_graph():
    L, Kb, C, B = 8, 3, 16, 32
    w = inputs.cnn2_weights(Kb, C, 0.8, 271, out_bias=2.0)
    ctx = c2_ctx(L, Kb, C, w)
    graph_replays_equal_eager(ctx, w, to_dev(inputs.spins_tj(L, B, 8, 272)), steps=4, lr=0.01,
                              diag_shift=1e-2, cg_iters=20, seed=273)
    assert ctx.get_error() == 0


def test_cnn2_empty_batch():
    L, Kb, C = 6, 2, 32
    ctx = c2_ctx(L, Kb, C, inputs.cnn2_weights(Kb, C, 1.0, 281, out_bias=1.0))
    empty = to_dev(np.zeros((0, L, L), np.int8))
    assert ctx.local_energy(empty).numel() == 0
    la, sg = ctx.log_psi(empty)
    assert la.numel() == 0 and sg.numel() == 0
    assert ctx.log_deriv(empty, dtype="fp64").shape == (0, ctx.P)
    assert ctx.get_error() == 0


def test_cnn2_largest_lattice_and_degenerate_sectors():
    """64x64 (the largest lattice) log|psi| and a 20x20 local energy against
    the oracle; a lattice of holes only (no term at all: E_loc = 0) and a
    single electron (hops only, no exchange) on 8x8."""
    Kb, C = 2, 16
    w = inputs.cnn2_weights(Kb, C, 1.0, 291, out_bias=2.0)
    sp = inputs.spins_tj(64, 2, 512, 292)
    ctx = c2_ctx(64, Kb, C, w)
    la, sg = ctx.log_psi(to_dev(sp))
    ol, os_ = oracle.cnn2_log_psi(64, Kb, C, w, sp)
    np.testing.assert_allclose(la.cpu().numpy(), ol, rtol=1e-12)
    assert np.array_equal(sg.cpu().numpy(), os_)
    sp32 = inputs.spins_tj(20, 2, 50, 293)
    c32 = c2_ctx(20, Kb, C, w)
    e = c32.local_energy(to_dev(sp32)).cpu().numpy()
    ref = oracle.tj_cnn2_local_energy(20, T_HOP, J_EX, Kb, C, w, sp32)
    say("20x20 cnn2 E_loc max rel", rel_inf(e, ref))
    assert rel_inf(e, ref) <= 1e-10
    c8 = c2_ctx(8, Kb, C, w)
    holes = np.zeros((3, 8, 8), np.int8)
    one = np.zeros((3, 8, 8), np.int8)
    one[0, 0, 0], one[1, 3, 5], one[2, 7, 7] = 1, -1, 1
    e0 = c8.local_energy(to_dev(holes)).cpu().numpy()
    assert np.array_equal(e0, np.zeros(3))
    e1 = c8.local_energy(to_dev(one)).cpu().numpy()
    r1 = oracle.tj_cnn2_local_energy(8, T_HOP, J_EX, Kb, C, w, one)
    say("single electron E_loc", e1, "oracle", r1)
    assert rel_inf(e1, r1) <= 1e-10
    for c in (ctx, c32, c8):
        assert c.get_error() == 0
