"""The C-ABI library loads, exports every entry point include/nqs.h declares,
and rejects bad arguments on the host (no GPU needed for any of this)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nqs.h")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(nqs_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    import torch  # noqa: F401 - the binding loads torch's HIP runtime first
    from paper_2204_07816_amd import nqs
    if not os.path.exists(nqs.LIB_PATH):
        # hipcc cross-compiles for gfx950 without a GPU
        from paper_2204_07816_amd import build
        build.build()
    return nqs.load()


def test_every_declared_symbol_is_exported(lib):
    syms = declared_symbols()
    assert len(syms) >= 18
    for s in syms:
        assert hasattr(lib, s), f"{s} declared in nqs.h but not exported"


def test_status_strings(lib):
    for code in range(11):
        assert lib.nqs_status_str(code)
    assert b"lattice" in lib.nqs_status_str(2)


def _create(lib, L, K, C, n, dtype=0, marshall=1, w=None, spec=True):
    from paper_2204_07816_amd import nqs
    sp = nqs.CnnSpec(K, C, marshall, dtype)
    buf = (ctypes.c_double * max(n, 1))()
    h = ctypes.c_void_p()
    return lib.nqs_create(L, 1.0, 0.5, ctypes.byref(sp) if spec else None,
                          buf if w is None else w, n, ctypes.byref(h))


@pytest.mark.parametrize("L", [3, 5, 2, 66, 0, -4])
def test_create_rejects_bad_lattice(lib, L):
    assert _create(lib, L, 2, 4, 188) == 2          # NQS_E_LATTICE


def test_create_rejects_bad_spec_and_counts(lib):
    from paper_2204_07816_amd import nqs
    assert _create(lib, 4, 0, 4, 10) == 3           # K < 1
    assert _create(lib, 4, 2, 33, 10) == 3          # C > 32
    assert _create(lib, 4, 2, 4, 188, dtype=7) == 3
    assert _create(lib, 4, 2, 4, 188, marshall=2) == 3
    assert _create(lib, 4, 2, 4, 187) == 4          # NQS_E_NPARAMS
    assert _create(lib, 4, 2, 4, nqs.num_params(2, 4), dtype=2) == 3   # BF16 needs C in {16, 32}
    assert _create(lib, 38, 2, 32, nqs.num_params(2, 32), dtype=2) == 3  # BF16 needs L <= 36
    assert _create(lib, 4, 2, 4, 188, spec=False) == 1                 # null spec


def test_calls_reject_null_context(lib):
    vp = ctypes.c_void_p
    assert lib.nqs_local_energy(None, None, 0, None, 0, None) == 1
    assert lib.nqs_log_psi(None, None, 0, None, None, None) == 1
    assert lib.nqs_log_deriv(None, None, 0, None, 0, None) == 1
    assert lib.nqs_sr_solve(None, None, 0, None, 0, 1e-4, 100, None, None, None) == 1
    assert lib.nqs_destroy(None) == 1
    assert lib.nqs_local_energy_multi(None, 0, 0, None) == 1
    assert lib.nqs_sr_solve_recompute(None, None, 0, None, 0, 1e-4, 100, 0, None, None,
                                      None) == 1
    assert lib.nqs_mcmc(None, None, 0, 0, None, None, None, 0, None) == 1
    assert lib.nqs_update_weights(None, None, 1.0, None) == 1
    assert lib.nqs_get_weights(None, None, 0) == 1
    p = ctypes.c_int64()
    assert lib.nqs_num_params(None, ctypes.byref(p)) == 1
    del vp


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    from paper_2204_07816_amd import nqs
    monkeypatch.setattr(nqs, "_lib", None)
    monkeypatch.setattr(nqs, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError, match="no fallback"):
        nqs.load()


def test_create_tj_rejects_bad_arguments(lib):
    from paper_2204_07816_amd import nqs
    sp = nqs.CnnSpec(2, 4, 1, 0)
    buf = (ctypes.c_double * 188)()
    h = ctypes.c_void_p()
    assert lib.nqs_create_tj(5, 1.0, 0.4, ctypes.byref(sp), buf, 188, ctypes.byref(h)) == 2
    assert lib.nqs_create_tj(4, float("nan"), 0.4, ctypes.byref(sp), buf, 188,
                             ctypes.byref(h)) == 1
    assert lib.nqs_create_tj(4, 1.0, float("inf"), ctypes.byref(sp), buf, 188,
                             ctypes.byref(h)) == 1
    assert lib.nqs_create_tj(4, 1.0, 0.4, None, buf, 188, ctypes.byref(h)) == 1
    assert lib.nqs_create_tj(4, 1.0, 0.4, ctypes.byref(sp), buf, 187, ctypes.byref(h)) == 4
    assert not h.value


def test_create_cnn1_rejects_bad_arguments(lib):
    buf = (ctypes.c_double * 2000)()
    h = ctypes.c_void_p()
    # CNN1 with 2 blocks of 4 channels: 2*4*1*9 + 8 + 144 + 4 + 2*4*4*9 + 8 + 144 + 4 = 672
    assert lib.nqs_create_cnn1(5, 1.0, 0.5, 2, 4, 1, buf, 672, ctypes.byref(h)) == 2
    assert lib.nqs_create_cnn1(4, 1.0, 0.5, 0, 4, 1, buf, 672, ctypes.byref(h)) == 3
    assert lib.nqs_create_cnn1(4, 1.0, 0.5, 2, 33, 1, buf, 672, ctypes.byref(h)) == 3
    assert lib.nqs_create_cnn1(4, 1.0, 0.5, 2, 4, 2, buf, 672, ctypes.byref(h)) == 3
    assert lib.nqs_create_cnn1(4, 1.0, 0.5, 2, 4, 1, buf, 671, ctypes.byref(h)) == 4
    assert lib.nqs_create_cnn1(4, float("nan"), 0.5, 2, 4, 1, buf, 672, ctypes.byref(h)) == 1
    assert lib.nqs_create_cnn1(4, 1.0, 0.5, 2, 4, 1, None, 672, ctypes.byref(h)) == 1
    assert not h.value


def test_binding_rejects_cnn1_outside_fp64(lib):
    from paper_2204_07816_amd import inputs, nqs
    w = inputs.cnn1_weights(2, 4, 0.1, 1)
    with pytest.raises(ValueError):
        nqs.Context(4, 1.0, 0.5, 2, 4, w, dtype="bf16", net="cnn1")
    with pytest.raises(ValueError):
        nqs.Context(4, 0.4, 0.5, 2, 4, w, net="cnn1", tj_hop=1.0)     # t-J has no J2


def test_create_cnn1_tj_rejects_bad_arguments(lib):
    buf = (ctypes.c_double * 2000)()
    h = ctypes.c_void_p()
    assert lib.nqs_create_cnn1_tj(5, 1.0, 0.4, 2, 4, 1, buf, 672, ctypes.byref(h)) == 2
    assert lib.nqs_create_cnn1_tj(4, 1.0, 0.4, 2, 4, 1, buf, 671, ctypes.byref(h)) == 4
    assert lib.nqs_create_cnn1_tj(4, float("inf"), 0.4, 2, 4, 1, buf, 672, ctypes.byref(h)) == 1
    assert not h.value


def test_mfma_rate_rejects_bad_arguments(lib):
    """nqs_mfma_rate checks its arguments before touching the device."""
    ms, tf = ctypes.c_double(), ctypes.c_double()
    for kind, wg, it in ((2, 16, 10), (0, 0, 10), (1, 16, 0), (0, 1 << 21, 10)):
        assert lib.nqs_mfma_rate(kind, ctypes.c_int64(wg), it, ctypes.byref(ms),
                                 ctypes.byref(tf), None) == 1          # NQS_E_ARG
    assert lib.nqs_mfma_rate(0, ctypes.c_int64(16), 10, None, ctypes.byref(tf), None) == 1
