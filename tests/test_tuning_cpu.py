"""Zero plan options resolve through the autotuner's database (host only:
ntt_plan_resolve_opts answers without creating a plan, so no GPU is needed)."""
import json
import os

import pytest

from paper_2509_22684_amd import _lib

DEV = "gfx950:sramecc+:xnack-"


@pytest.fixture(autouse=True)
def clean_registry():
    _lib.ntt_tuning_clear()
    _lib._tuning_loaded.clear()
    yield
    _lib.ntt_tuning_clear()
    _lib._tuning_loaded.clear()


def test_builtin_defaults_without_registration():
    assert _lib.ntt_plan_resolve_opts("bls12_381_fr", 24) == dict(
        twiddle_mode=1, log2_radix=2, log2_tile=10, flags=0, log2_pass_radix=8)
    assert _lib.ntt_plan_resolve_opts("bls12_381_fr", 16) == dict(
        twiddle_mode=1, log2_radix=1, log2_tile=8, flags=0, log2_pass_radix=9)
    assert _lib.ntt_plan_resolve_opts("bls12_381_fr", 9)["log2_tile"] == 10
    assert _lib.ntt_plan_resolve_opts("bls12_381_fr", 17)["log2_tile"] == 10
    assert _lib.ntt_plan_resolve_opts("bls12_381_fr", 12, log2_radix=3)["log2_tile"] == 10


def test_default_plan_picks_up_the_database_schedule(tmp_path):
    db = {"devices": {DEV: {
        "bn254_fr:20:single": {"opts": {"log2_pass_radix": 7, "log2_radix": 3, "log2_tile": 11, "twiddle_mode": 2},
                               "ms": 1.0, "candidates": []},
        "bn254_fr:20:batch": {"opts": {"log2_pass_radix": 6, "log2_radix": 2, "twiddle_mode": 1},
                              "ms": 1.0, "candidates": []},
        "bls12_381_fr:12:single": {"opts": {"log2_radix": 3}, "ms": 1.0, "candidates": []}},
        "gfx942:sramecc+:xnack-": {
        "bn254_fr:21:single": {"opts": {"log2_radix": 3}, "ms": 1.0, "candidates": []}}}}
    path = tmp_path / "db.json"
    path.write_text(json.dumps(db))
    assert _lib.register_tuning_db(DEV, str(path)) == 2
    # every zero field comes from the database's stand-alone schedule
    assert _lib.ntt_plan_resolve_opts("bn254_fr", 20) == dict(
        twiddle_mode=2, log2_radix=3, log2_tile=11, flags=0, log2_pass_radix=7)
    # fields the database leaves open keep the built-in defaults
    assert _lib.ntt_plan_resolve_opts("bls12_381_fr", 12) == dict(
        twiddle_mode=1, log2_radix=3, log2_tile=10, flags=0, log2_pass_radix=9)  # radix 8 keeps 2^10 tiles
    # explicit options win over the database
    assert _lib.ntt_plan_resolve_opts("bn254_fr", 20, log2_radix=1, flags=1)["log2_radix"] == 1
    assert _lib.ntt_plan_resolve_opts("bn254_fr", 20, log2_radix=1, flags=1)["flags"] == 1
    # another device's entries and other sizes are untouched
    assert _lib.ntt_plan_resolve_opts("bn254_fr", 21)["log2_radix"] == 2
    # registering the same database again is a no-op
    assert _lib.register_tuning_db(DEV, str(path)) == 0


def test_committed_database_matches_the_headline_schedule():
    """The committed database's 2^24 BLS12-381 entry is the schedule the
    measurement step runs with zero options."""
    from paper_2509_22684_amd.autotune import DEFAULT_DB

    with open(DEFAULT_DB) as f:
        devs = json.load(f)["devices"]
    dev = next(iter(devs))
    _lib.register_tuning_db(dev, DEFAULT_DB)
    got = _lib.ntt_plan_resolve_opts("bls12_381_fr", 24)
    want = devs[dev]["bls12_381_fr:24:single"]["opts"]
    for k, v in want.items():
        assert got[k] == v


def test_bad_registrations_and_arguments_are_refused():
    with pytest.raises(_lib.ZkError):
        _lib.ntt_tuning_register("bls12_381_fr", 40, log2_radix=2)  # beyond the 2-adicity
    with pytest.raises(_lib.ZkError):
        _lib.ntt_tuning_register("bls12_381_fr", 20, log2_tile=12)
    with pytest.raises(_lib.ZkError):
        _lib.ntt_plan_resolve_opts("bls12_381_fr", 20, log2_pass_radix=3)
    with pytest.raises(_lib.ZkError):
        _lib.ntt_plan_resolve_opts(9, 20)
    L = _lib.lib()
    assert L.ntt_plan_resolve_opts(1, 20, None, None) == -1
    out = _lib._Opts()
    assert L.ntt_plan_resolve_opts(1, 20, None, out) == 0
    assert L.ntt_plan_get_opts(None, out) == -1
    assert os.path.exists(_lib.LIB_PATH)


def test_plan_table_bytes_on_the_host():
    """Table bytes of the 2^24 plan: w_256 (256 entries), the second pass's
    [r][j mod 256] table (2^16), the third pass's (2^24) and three coset
    tables (3 x 2^24), 32 bytes each; unsupported sizes give 0."""
    n = 1 << 24
    assert _lib.ntt_plan_table_bytes("bls12_381_fr", 24) == 32 * (256 + (1 << 16) + n + 3 * n)
    assert _lib.ntt_plan_table_bytes("bls12_381_fr", 33) == 0
    assert _lib.ntt_plan_table_bytes("bn254_fr", 10, log2_tile=10) == 32 * ((1 << 10) + 3 * (1 << 10))
    two = _lib.ntt_plan_table_bytes("bls12_381_fr", 20, twiddle_mode=2)
    one = _lib.ntt_plan_table_bytes("bls12_381_fr", 20, twiddle_mode=1)
    assert 0 < two < one
