"""The tuning cache keys on the exact plan precision: an entry stored for
one precision is never applied to a plan of another (host only)."""
import pytest

from paper_1801_09263_amd import lace, tuning

PRECS = [lace.LACE_FP64, lace.LACE_FP32, lace.LACE_FP64_GAMMA,
         lace.LACE_FP32_GAMMA]


def test_keys_differ_by_precision():
    keys = {tuning.tune_key(120, 256, p) for p in PRECS}
    assert len(keys) == 4
    with pytest.raises(ValueError):
        tuning.tune_key(120, 256, 7)


def test_fp32_gamma_entry_not_applied_to_fp64_gamma(tmp_path):
    path = str(tmp_path / "tuning.json")
    tuning.store({tuning.tune_key(120, 256, lace.LACE_FP32_GAMMA):
                  dict(pairs_per_batch=64, use_plane=1)}, path)
    # no entry for the FP64 real-orbital plan: nothing is applied (and the
    # plan, None here, is never touched)
    assert not tuning.apply_cached(None, 0, 120, 256, lace.LACE_FP64_GAMMA, path)
    assert tuning.load(path).get(tuning.tune_key(120, 256, lace.LACE_FP32_GAMMA))
