"""The autotuner's cache file, through the host-only entry points (no GPU):
keys, lookups of well-formed entries, and that a missing, malformed or
truncated file or a missing key yields no entry (the library then falls back
to its defaults) without touching the outputs."""
import json
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def nqs():
    import torch  # noqa: F401 - the binding loads torch's HIP runtime first
    from paper_2204_07816_amd import nqs as m
    if not os.path.exists(m.LIB_PATH):
        pytest.fail("libnqs.so is not built: run __graft_entry__.build()")
    m.load()
    return m


def test_keys_distinguish_configurations(nqs):
    a = nqs.tune_key(36, 8, 32, "bf16", 0.5)
    assert a == "gfx950 L=36 K=8 C=32 bf16 J2"
    assert nqs.tune_key(36, 8, 32, "bf16", 0.0) != a
    assert nqs.tune_key(24, 8, 32, "bf16", 0.5) != a
    assert nqs.tune_key(36, 8, 32, "fp64", 0.5) != a


def test_lookup_of_well_formed_cache(nqs, tmp_path):
    k1 = nqs.tune_key(36, 8, 32, "bf16", 0.5)
    k2 = nqs.tune_key(10, 4, 16, "bf16", 0.5)
    p = tmp_path / "tune.json"
    p.write_text(json.dumps({
        k1: {"mode": "incremental", "full_nw": 8, "full_maxt": 11, "cone_items": 6,
             "cone_waves": 4, "ms_full": 900.5, "ms_incremental": 83.0},
        k2: {"mode": "full", "full_nw": 4, "full_maxt": 2, "ms_full": 3.5, "ms_incremental": 4.1},
    }, indent=1))
    assert nqs.tune_lookup(str(p), k1) == {"mode": "incremental", "full_nw": 8, "full_maxt": 11,
                                           "cone_items": 6, "cone_waves": 4}
    # an entry without the cone kernel's shape keeps the default one
    assert nqs.tune_lookup(str(p), k2) == {"mode": "full", "full_nw": 4, "full_maxt": 2,
                                           "cone_items": -1, "cone_waves": -1}
    assert nqs.tune_lookup(str(p), nqs.tune_key(12, 6, 32, "bf16", 0.0)) is None
    assert nqs.tune_lookup(str(p), "") is None


@pytest.mark.parametrize("text", [
    "",                                            # empty
    "{",                                           # truncated
    "not json",
    '{"k": {"mode": "sideways"}}',                 # unknown mode
    '{"k": {"mode": "full", "full_nw": }}',        # missing value
    '{"k": {"mode": "full"}} trailing',            # trailing garbage
    '[1, 2, 3]',                                   # wrong shape
    '{"k": {"mode": "full", "full_nw": 4}',        # unbalanced
])
def test_malformed_cache_gives_no_entry(nqs, tmp_path, text):
    p = tmp_path / "tune.json"
    p.write_text(text)
    assert nqs.tune_lookup(str(p), "k") is None


def test_missing_file_gives_no_entry(nqs, tmp_path):
    assert nqs.tune_lookup(str(tmp_path / "absent.json"), "k") is None
