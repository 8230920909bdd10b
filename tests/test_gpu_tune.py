"""Autotuner on the device: it picks one of the available forms of the
exchanged-configuration pass, AUTO follows the pick, the pick is written to
the tune cache and read back by a new context of the same configuration, and
results under the tuned choice agree with the explicit modes."""
import numpy as np
import pytest

from paper_2204_07816_amd import inputs, nqs
from gpu_helpers import make_ctx, rel_inf, say, to_dev

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("L,J2,K,C,dt", [(16, 0.5, 6, 32, "bf16"), (10, 0.5, 4, 16, "bf16"),
                                         (16, 0.5, 6, 32, "bf16x3")])
def test_autotune_round_trip(tmp_path, monkeypatch, L, J2, K, C, dt):
    cache = tmp_path / "tune.json"
    monkeypatch.setenv("NQS_TUNE_CACHE", str(cache))
    w = inputs.stress_weights(K, C, 1.0, 81)
    sp = to_dev(inputs.spins_sz0(L, 12, 82))
    ctx = make_ctx(L, J2, K, C, w, dtype=dt)
    m = ctx.autotune(sp)
    say(f"{L}x{L} K={K} C={C} {dt}: tuned mode {m}", cache.read_text().strip())
    assert m in ("full", "incremental")
    assert ctx.auto_mode() == m
    entry = nqs.tune_lookup(str(cache), nqs.tune_key(L, K, C, dt, J2))
    assert entry is not None and entry["mode"] == m
    if L >= 2 * K + 4 and C == 32:
        # the cone kernel's shape is tuned too: a lockstep shape or the
        # one-configuration kernel (items 1, waves 0)
        assert entry["cone_items"] >= 1 and entry["cone_waves"] in (0, 4, 8)
    ctx2 = make_ctx(L, J2, K, C, w, dtype=dt)          # reads the cache at creation
    assert ctx2.auto_mode() == m
    e_auto = ctx2.local_energy(sp, mode="auto").cpu().numpy()
    e_m = ctx2.local_energy(sp, mode=m).cpu().numpy()
    assert np.array_equal(e_auto, e_m)
    # the tuned cone shape against the default shape (same arithmetic; the
    # per-configuration sums may be taken in another order)
    e_inc_tuned = ctx2.local_energy(sp, mode="incremental").cpu().numpy() \
        if ctx2.auto_mode() == "incremental" else None
    # the full pass with the tuned tile variant against a context without a cache
    monkeypatch.setenv("NQS_TUNE_CACHE", str(tmp_path / "empty.json"))
    ctx3 = make_ctx(L, J2, K, C, w, dtype=dt)
    e_full_tuned = ctx2.local_energy(sp, mode="full").cpu().numpy()
    e_full_default = ctx3.local_energy(sp, mode="full").cpu().numpy()
    assert rel_inf(e_full_tuned, e_full_default) <= 1e-12
    if e_inc_tuned is not None:
        e_inc_default = ctx3.local_energy(sp, mode="incremental").cpu().numpy()
        assert rel_inf(e_inc_tuned, e_inc_default) <= 1e-12
    assert ctx.get_error() == 0 and ctx2.get_error() == 0


def test_autotune_fp64_has_only_full(tmp_path, monkeypatch):
    monkeypatch.setenv("NQS_TUNE_CACHE", str(tmp_path / "tune.json"))
    w = inputs.weights(3, 8, 0.1, 83)
    ctx = make_ctx(6, 0.5, 3, 8, w, dtype="fp64")
    assert ctx.autotune(to_dev(inputs.spins_sz0(6, 4, 84))) == "full"
    assert ctx.auto_mode() == "full"
