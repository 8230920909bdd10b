"""GPU per-sample log-derivatives O_k (hand-written backward, FP64) and the
matrix-free SR conjugate-gradient solve, vs the oracle, central finite
differences and autograd."""
import numpy as np
import pytest
import torch

import oracle
from paper_2204_07816_amd import inputs, nqs
from gpu_helpers import DEV, make_ctx, say, to_dev

pytestmark = pytest.mark.gpu


def rownorm_rel(a, b):
    return max(np.max(np.abs(a[s] - b[s])) / max(np.max(np.abs(b[s])), 1e-300)
               for s in range(b.shape[0]))


@pytest.mark.parametrize("L,K,C,B,sigma", [(4, 1, 4, 16, 0.4), (4, 2, 4, 64, 0.05), (10, 4, 16, 8, 0.3),
                                           (6, 3, 5, 6, 0.5), (8, 2, 32, 4, 0.2)])
def test_log_deriv_vs_oracle(L, K, C, B, sigma):
    say("log_deriv", L, K, C, B)
    w = inputs.weights(K, C, sigma, 8)
    sp = inputs.spins_sz0(L, B, 9)
    ctx = make_ctx(L, 0.5, K, C, w)
    O64 = ctx.log_deriv(to_dev(sp), dtype="fp64").cpu().numpy()
    O32 = ctx.log_deriv(to_dev(sp), dtype="fp32").cpu().numpy()
    ref = oracle.log_deriv(L, K, C, w, sp)
    say("  fp64 rel", rownorm_rel(O64, ref), "fp32 rel", rownorm_rel(O32, ref))
    assert rownorm_rel(O64, ref) <= 1e-10
    assert rownorm_rel(O32, ref) <= 1e-5


def test_log_deriv_bf16_context_is_fp64_backward():
    L, K, C = 10, 4, 16
    w = inputs.weights(K, C, 0.2, 1)
    sp = inputs.spins_sz0(L, 4, 2)
    ctx = make_ctx(L, 0.5, K, C, w, dtype="bf16")
    O = ctx.log_deriv(to_dev(sp), dtype="fp64").cpu().numpy()
    assert rownorm_rel(O, oracle.log_deriv(L, K, C, w, sp)) <= 1e-10


def test_log_deriv_finite_differences_24x24():
    """24x24, K=6, C=32: 32 sampled parameters by central differences (h=1e-6, FP64)
    of the GPU log-amplitude."""
    L, J2, K, C, w, sp = inputs.config_inputs("sr24", B=4)
    w = inputs.weights(K, C, 0.05, 1003)
    ctx = make_ctx(L, J2, K, C, w)
    dsp = to_dev(sp)
    O = ctx.log_deriv(dsp, dtype="fp64").cpu().numpy()
    rng = np.random.default_rng(5)
    idx = rng.choice(w.shape[0], size=32, replace=False)
    h = 1e-6
    for p in idx:
        wp, wm = w.copy(), w.copy()
        wp[p] += h
        wm[p] -= h
        ctx.set_weights(wp)
        fp = ctx.log_psi(dsp)[0].cpu().numpy()
        ctx.set_weights(wm)
        fm = ctx.log_psi(dsp)[0].cpu().numpy()
        fd = (fp - fm) / (2 * h)
        assert np.all(np.abs(fd - O[:, p]) <= 1e-7 * (1 + np.abs(O[:, p]))), (p, fd, O[:, p])
    ctx.set_weights(w)


def test_autograd_function():
    """Two forwards at different weights on one context, then both backwards:
    each sees its own weights (set on the device, no host round trip)."""
    L, K, C = 6, 2, 4
    w = inputs.weights(K, C, 0.4, 3)
    w2 = inputs.weights(K, C, 0.3, 7)
    sp = inputs.spins_sz0(L, 5, 4)
    ctx = make_ctx(L, 0.5, K, C, w)
    theta = torch.tensor(w, requires_grad=True)
    theta2 = torch.tensor(w2, device=DEV, requires_grad=True)
    la = nqs.LogPsiFn.apply(theta, to_dev(sp), ctx)
    la2 = nqs.LogPsiFn.apply(theta2, to_dev(sp), ctx)
    np.testing.assert_allclose(la.detach().cpu().numpy(), oracle.log_psi(L, K, C, w, sp)[0], rtol=1e-12)
    np.testing.assert_allclose(la2.detach().cpu().numpy(), oracle.log_psi(L, K, C, w2, sp)[0], rtol=1e-12)
    g = torch.linspace(-1, 1, 5, dtype=torch.float64, device=DEV)
    (la * g).sum().backward()
    (la2 * g * g).sum().backward()
    ref = g.cpu().numpy() @ oracle.log_deriv(L, K, C, w, sp)
    ref2 = (g * g).cpu().numpy() @ oracle.log_deriv(L, K, C, w2, sp)
    np.testing.assert_allclose(theta.grad.numpy(), ref, rtol=1e-10, atol=1e-13)
    assert theta2.grad.device.type == "cuda"
    np.testing.assert_allclose(theta2.grad.cpu().numpy(), ref2, rtol=1e-10, atol=1e-13)


def test_set_weights_device_equals_host_set():
    """nqs_set_weights_device gives the kernels exactly what nqs_set_weights
    gives them: log|psi|, E_loc and O bit for bit, in FP64 and BF16."""
    L, K, C = 12, 3, 16
    w = inputs.stress_weights(K, C, 1.0, 9)
    w2 = inputs.stress_weights(K, C, 0.9, 10)
    spd = to_dev(inputs.spins_sz0(L, 16, 11))
    for dt in ("fp64", "bf16"):
        a = make_ctx(L, 0.5, K, C, w, dtype=dt)
        b = make_ctx(L, 0.5, K, C, w, dtype=dt)
        a.set_weights(w2)
        b.set_weights_device(torch.tensor(w2, device=DEV))
        assert torch.equal(a.log_psi(spd)[0], b.log_psi(spd)[0])
        assert torch.equal(a.local_energy(spd), b.local_energy(spd))
        assert torch.equal(a.log_deriv(spd, dtype="fp64"), b.log_deriv(spd, dtype="fp64"))
        assert np.array_equal(b.get_weights(), w2)


# (S + 1e-4 I) condition numbers: ~4.7e3, ~60, ~110 (converged within 100 CG steps)
# and ~3.6e5 (not converged after 100 steps: both sides stop at the same
# iterate only up to rounding, so that case carries a looser bound).
@pytest.mark.parametrize("L,K,C,B,sigma,odt,tol", [(4, 2, 4, 256, 0.1, "fp64", 1e-6),
                                                   (4, 2, 4, 256, 0.05, "fp32", 1e-6),
                                                   (10, 4, 16, 300, 0.1, "fp64", 1e-6),
                                                   (10, 4, 16, 300, 0.15, "fp64", 1e-4)])
def test_sr_cg_vs_oracle(L, K, C, B, sigma, odt, tol):
    say("sr", L, K, C, B, sigma, odt)
    w = inputs.weights(K, C, sigma, 13)
    sp = inputs.spins_sz0(L, B, 14)
    O = oracle.log_deriv(L, K, C, w, sp)
    e = oracle.local_energy(L, 1.0, 0.5, K, C, w, sp)
    if odt == "fp32":
        O = O.astype(np.float32).astype(np.float64)    # both sides see the same FP32 values
    ctx = make_ctx(L, 0.5, K, C, w)
    Od = torch.tensor(O, dtype=torch.float32 if odt == "fp32" else torch.float64, device=DEV)
    x, st = ctx.sr_solve(Od, torch.tensor(e, device=DEV), 1e-4, 100)
    x, st = x.cpu().numpy(), st.cpu().numpy()
    ref, rel, it = oracle.sr_cg(O, e, 1e-4, 100)
    say("  |dx|/|x|", np.linalg.norm(x - ref) / np.linalg.norm(ref), "res gpu", st[2], "oracle", rel,
        "it", st[3], it)
    assert np.linalg.norm(x - ref) <= tol * np.linalg.norm(ref)
    if it == 100:
        assert int(st[3]) == it
    else:
        # both converged past the early-exit threshold (||r|| < 1e-30 ||F||),
        # which rounding can cross a step or two apart
        assert abs(int(st[3]) - it) <= 5 and st[2] < 1e-29
    m, v = oracle.energy_stats(e)
    assert st[0] == pytest.approx(m, rel=1e-13) and st[1] == pytest.approx(v, rel=1e-11)


def test_sr_converged_matches_dense_solve():
    L, K, C, B = 4, 2, 4, 200
    w = inputs.weights(K, C, 0.1, 15)
    sp = inputs.spins_sz0(L, B, 16)
    O = oracle.log_deriv(L, K, C, w, sp)
    e = oracle.local_energy(L, 1.0, 0.5, K, C, w, sp)
    ctx = make_ctx(L, 0.5, K, C, w)
    x, st = ctx.sr_solve(torch.tensor(O, device=DEV), torch.tensor(e, device=DEV), 1e-2, 1000)
    ref = oracle.sr_dense(O, e, 1e-2)
    assert np.linalg.norm(x.cpu().numpy() - ref) <= 1e-8 * np.linalg.norm(ref)


def test_sr_zero_iterations_and_zero_force():
    L, K, C, B = 4, 2, 4, 16
    ctx = make_ctx(L, 0.5, K, C, inputs.weights(K, C, 0.1, 1))
    O = torch.randn(B, ctx.P, dtype=torch.float64, device=DEV)
    x, st = ctx.sr_solve(O, torch.ones(B, dtype=torch.float64, device=DEV), 1e-4, 100)
    assert torch.all(x == 0) and st[3].item() == 0       # E constant: F = 0
    x, st = ctx.sr_solve(O, torch.randn(B, dtype=torch.float64, device=DEV), 1e-4, 0)
    assert torch.all(x == 0)
