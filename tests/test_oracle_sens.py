"""Pins of the oracle's rounding-error sensitivities (oracle_sens_layers,
oracle_dlog_sens), the quantities a reduced-precision evaluation of the
network is bounded by.

* z, h, g = df/dh_k and d = df/dz_k against torch-CPU FP64 autograd through
  the network built from torch's conv2d with circular padding; a against
  torch's conv2d of |h| with |W| plus |b|.
* The per-item sums against the same sums formed from the per-layer arrays of
  both configurations (values equal outside the changed region share one
  rounding).
* The bound itself: an FP64 forward whose activations of layers 1..K-1 are
  rounded to BF16 (round to nearest even), written here with numpy, changes
  every f(S') - f(S) by no more than the first-order worst-case bound
  u S1_act (u = 2^-8), and by no more than the probabilistic bound
  6 u S2_act; the typical error is of the probabilistic bound's order.
"""
import numpy as np
import pytest
import torch
import torch.nn.functional as F

import oracle
from paper_2204_07816_amd import inputs


def _layers(w, K, C):
    """(W [C, cin, 3, 3], b [C]) per layer from the canonical vector."""
    out, off = [], 0
    for k in range(K):
        cin = 1 if k == 0 else C
        W = w[off:off + C * cin * 9].reshape(C, cin, 3, 3)
        off += C * cin * 9
        out.append((W, w[off:off + C]))
        off += C
    return out


def test_sens_layers_match_torch_autograd():
    L, K, C = 6, 3, 4
    w = inputs.stress_weights(K, C, 1.0, 5)
    w[np.arange(w.size) % 7 == 0] += 0.05          # non-zero biases too
    sp = inputs.spins_sz0(L, 1, 6)
    o = oracle.sens_layers(L, K, C, w, sp)
    h = torch.tensor(sp.reshape(1, 1, L, L), dtype=torch.float64, requires_grad=True)
    zs, hs, a_ref = [], [], []
    for W, b in _layers(w, K, C):
        Wt, bt = torch.tensor(W), torch.tensor(b)
        hp = F.pad(h, (1, 1, 1, 1), mode="circular")
        a_ref.append((F.conv2d(hp.abs(), Wt.abs()) + bt.abs()[None, :, None, None])[0].detach())
        z = F.conv2d(hp, Wt, bt)
        z.retain_grad()
        h = torch.log(torch.cosh(z))
        h.retain_grad()
        zs.append(z)
        hs.append(h)
    hs[-1].sum().backward()
    for k in range(K):
        np.testing.assert_allclose(o["z"][k], zs[k][0].detach().numpy(), rtol=1e-13, atol=1e-15)
        np.testing.assert_allclose(o["h"][k], hs[k][0].detach().numpy(), rtol=1e-12, atol=1e-15)
        np.testing.assert_allclose(o["a"][k], a_ref[k].numpy(), rtol=1e-13)
        np.testing.assert_allclose(o["g"][k], hs[k].grad[0].numpy(), rtol=1e-10, atol=1e-14)
        np.testing.assert_allclose(o["d"][k], zs[k].grad[0].numpy(), rtol=1e-10, atol=1e-14)


def test_dlog_sens_sums_from_layer_arrays():
    L, K, C = 6, 3, 4
    w = inputs.stress_weights(K, C, 1.1, 7)
    sp = inputs.spins_sz0(L, 2, 8)
    _, bonds, _, _ = oracle.connected(L, 1.0, 0.5, sp)
    items = [(0, b) for b in bonds[0][:5]] + [(1, b) for b in bonds[1][-3:]] + [(1, -1)]
    out = oracle.dlog_sens(L, K, C, w, sp, [s for s, _ in items], [b for _, b in items])
    for m, (s, b) in enumerate(items):
        A = oracle.sens_layers(L, K, C, w, sp[s])
        if b < 0:
            th = np.abs(A["g"] * A["h"])
            tz = np.abs(A["d"]) * A["a"]
            exp = [oracle.log_psi(L, K, C, w, sp[s:s + 1])[0][0], th[:-1].sum(),
                   np.sqrt((th[:-1] ** 2).sum()), tz.sum(), th.sum(), np.sqrt((tz ** 2).sum())]
        else:
            i, j, _ = oracle.bond_sites(L, int(b))
            s2 = sp[s].reshape(-1).copy()
            s2[i], s2[j] = s2[j], s2[i]
            Bp = oracle.sens_layers(L, K, C, w, s2.reshape(L, L))
            f = oracle.log_psi(L, K, C, w, np.stack([sp[s].reshape(-1), s2]).reshape(2, L, L))[0]

            def sums(vp, v, cp, c):
                same = vp == v
                t_in1, t_in2 = np.abs(cp * vp)[~same], np.abs(c * v)[~same]
                t_out = np.abs((cp - c) * v)[same]
                return (t_in1.sum() + t_in2.sum() + t_out.sum(),
                        np.sqrt((t_in1 ** 2).sum() + (t_in2 ** 2).sum() + (t_out ** 2).sum()))
            a1, a2 = sums(Bp["h"][:-1], A["h"][:-1], Bp["g"][:-1], A["g"][:-1])
            l1, _ = sums(Bp["h"], A["h"], Bp["g"], A["g"])
            same = Bp["z"] == A["z"]
            tz = np.concatenate([(np.abs(Bp["d"]) * Bp["a"])[~same], (np.abs(A["d"]) * A["a"])[~same],
                                 (np.abs(Bp["d"] - A["d"]) * A["a"])[same]])
            exp = [f[1] - f[0], a1, a2, tz.sum(), l1, np.sqrt((tz ** 2).sum())]
        np.testing.assert_allclose(out[m], exp, rtol=1e-11, atol=1e-15)


def _bf16(x):
    """Round to BF16 (nearest even) from the FP32 value, as the device does."""
    u = np.ascontiguousarray(x, np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def _f_rounded(sp, layers, L, round_act):
    """FP64 forward with explicit per-tap accumulation (every output site runs
    the same operations, so sites with equal inputs give equal values);
    activations of layers 1..K-1 optionally rounded to BF16."""
    h = sp.reshape(1, L, L).astype(np.float64)
    K = len(layers)
    for k, (W, b) in enumerate(layers):
        z = np.repeat(b[:, None, None], L, axis=1).repeat(L, axis=2).astype(np.float64)
        for ci in range(W.shape[1]):
            for ky in range(3):
                for kx in range(3):
                    sh = np.roll(h[ci], (1 - ky, 1 - kx), axis=(0, 1))
                    z = z + W[:, ci, ky, kx][:, None, None] * sh[None]
        a = np.abs(z)
        h = a + np.log1p(np.exp(-2 * a)) - np.log(2.0)
        if round_act and k < K - 1:
            h = _bf16(h)
    return h.sum()


@pytest.mark.parametrize("gain", [1.0, 1.3])
def test_bound_covers_bf16_rounded_activations(gain):
    L, K, C, J2 = 6, 4, 8, 0.5
    u = 2.0 ** -8
    w = inputs.stress_weights(K, C, gain, 11)
    sp = inputs.spins_sz0(L, 2, 12)
    layers = _layers(w, K, C)
    _, bonds, _, _ = oracle.connected(L, 1.0, J2, sp)
    sm = np.concatenate([[s] * len(bonds[s]) for s in range(2)])
    bd = np.concatenate(bonds)
    out = oracle.dlog_sens(L, K, C, w, sp, sm, bd)
    ratios, mags = [], []
    for m, (s, b) in enumerate(zip(sm, bd)):
        i, j, _ = oracle.bond_sites(L, int(b))
        s2 = sp[s].reshape(-1).copy()
        s2[i], s2[j] = s2[j], s2[i]
        s2 = s2.reshape(L, L)
        d_rnd = _f_rounded(s2, layers, L, True) - _f_rounded(sp[s], layers, L, True)
        d_ex = _f_rounded(s2, layers, L, False) - _f_rounded(sp[s], layers, L, False)
        err = abs(d_rnd - d_ex)
        assert abs(d_ex - out[m, 0]) <= 1e-12 * (1 + abs(d_ex))
        assert err <= 1.05 * u * out[m, 1] + 1e-15, (m, err, u * out[m, 1])
        assert err <= 6.0 * u * out[m, 2] + 1e-15, (m, err, u * out[m, 2])
        ratios.append(err / max(u * out[m, 2], 1e-300))
        mags.append(abs(d_ex))
    med = float(np.median(ratios))
    print("gain", gain, "items", len(ratios), "median |d|", np.median(mags),
          "median err / (u S2)", med, "max", max(ratios))
    assert 0.05 <= med <= 2.0
