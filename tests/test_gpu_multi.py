"""Several lattices in one launch (nqs_local_energy_multi): the exchanged
configurations of every lattice of one mode go through a single persistent
kernel launch over their concatenated queues.  Each lattice's E_loc must equal
what the single-lattice call gives: bit for bit where both use the same kernel,
to FP64 summation order (1e-12 relative) where the single call takes the
unwrapped-window kernel and the mixed launch the general one; and against the
FP64 oracle on a few samples.  The mixed workload is 12x12 (J2 = 0), 16x16
(J2 = 0.5) and 20x20 (J2 = 0.55), K = 6, C = 32."""
import numpy as np
import pytest
import torch

import oracle
from paper_2204_07816_amd import inputs, nqs
from gpu_helpers import make_ctx, rel_inf, say, to_dev

pytestmark = pytest.mark.gpu

K, C = 6, 32
LATTICES = [(12, 0.0, 40), (16, 0.5, 24), (20, 0.55, 16)]   # (L, J2, B)


def _setup(weights_seed=61, stress=True):
    jobs = []
    for idx, (L, J2, B) in enumerate(LATTICES):
        w = (inputs.stress_weights(K, C, 1.0, weights_seed + idx) if stress
             else inputs.weights(K, C, 0.02, weights_seed + idx))
        sp = inputs.spins_sz0(L, B, 70 + idx)
        ctx = make_ctx(L, J2, K, C, w, dtype="bf16")
        jobs.append((L, J2, B, w, sp, ctx))
    return jobs


def _single(jobs, mode):
    out = []
    for L, J2, B, w, sp, ctx in jobs:
        out.append(ctx.local_energy(to_dev(sp), mode=mode).cpu().numpy())
    return out


def _multi(jobs, mode):
    es = [torch.empty(B, dtype=torch.float64, device="cuda:0") for (_, _, B, _, _, _) in jobs]
    nqs.local_energy_multi([(ctx, to_dev(sp), e) for (_, _, _, _, sp, ctx), e in zip(jobs, es)],
                           mode=mode)
    return [e.cpu().numpy() for e in es]


def test_multi_full_mode_bit_exact():
    jobs = _setup()
    ref = _single(jobs, "full")
    got = _multi(jobs, "full")
    for (L, _, _, _, _, ctx), a, b in zip(jobs, got, ref):
        say("full", L, "max |diff|", float(np.max(np.abs(a - b))))
        assert np.array_equal(a, b)
        assert ctx.get_error() == 0


def test_multi_incremental_mixed_wrapped_and_unwrapped():
    """12x12 needs the general (wrapped-window) kernel; 16x16 and 20x20 share one
    launch of the unwrapped-window kernel.  Each lattice runs the kernel of its
    single-lattice call, so the energies are equal bit for bit."""
    jobs = _setup()
    ref = _single(jobs, "incremental")
    got = _multi(jobs, "incremental")
    for (L, _, _, _, _, ctx), a, b in zip(jobs, got, ref):
        say("incremental", L, "max |diff|", float(np.max(np.abs(a - b))))
        assert np.array_equal(a, b)
        assert ctx.get_error() == 0


def test_multi_incremental_unwrapped_only_bit_exact():
    """16x16 and 20x20 alone: the one launch is the unwrapped-window kernel,
    exactly as in the single-lattice calls."""
    jobs = _setup()[1:]
    ref = _single(jobs, "incremental")
    got = _multi(jobs, "incremental")
    for (L, _, _, _, _, ctx), a, b in zip(jobs, got, ref):
        assert np.array_equal(a, b), L


def test_multi_auto_groups_modes_and_matches_oracle():
    jobs = _setup(stress=False)
    ref = _single(jobs, "auto")
    got = _multi(jobs, "auto")
    for (L, J2, B, w, sp, ctx), a, b in zip(jobs, got, ref):
        say("auto", L, ctx.auto_mode(), "rel vs single", rel_inf(a, b))
        assert rel_inf(a, b) <= 1e-12
        o = oracle.local_energy(L, 1.0, J2, K, C, w, sp[:3])
        say("  vs oracle (3 samples) mean rel", abs(a[:3].mean() - o.mean()) / abs(o.mean()))
        assert abs(a[:3].mean() - o.mean()) <= 1e-5 * abs(o.mean())


def test_multi_more_jobs_than_one_launch_and_empty_job():
    """Nine lattices (more than one launch holds) including an empty batch."""
    base = _setup()
    jobs, es = [], []
    for r in range(3):
        for idx, (L, J2, B, w, sp, _) in enumerate(base):
            b = 0 if (r == 1 and idx == 0) else max(1, B // (r + 1))
            ctx = make_ctx(L, J2, K, C, w, dtype="bf16")
            jobs.append((L, J2, b, w, sp[:b], ctx))
    ref = _single(jobs, "full")
    got = _multi(jobs, "full")
    for (L, _, b, _, _, _), a, r in zip(jobs, got, ref):
        assert a.shape == (b,)
        assert np.array_equal(a, r)
