"""Host logic of the autotuner: which kernel variants and overlap shapes it
considers, and its cache records (no GPU needed)."""

from paper_1907_01005_amd import api
from paper_1907_01005_amd.autotune import TM_STEPS, TuneChoice, candidates


def test_candidates_by_degree_form_and_geometry():
    c2 = candidates(256, False, 2, api.FP64)
    assert (8, 0) in c2 and (9, 0) in c2          # register waves and the line kernel at p = 2
    c4 = candidates(256, False, 4, api.FP64)
    assert (9, 0) in c4 and (8, 0) not in c4      # no register waves past p = 2
    assert (9, 0) in candidates(256, False, 3, api.FP32)
    for prec in (api.FP64_MFMA, api.FP32_MFMA):   # the line kernel has no matrix-core form
        assert (9, 0) not in candidates(256, False, 4, prec)
    curved = candidates(256, True, 4, api.FP64)
    assert all(k in (0, 2, 7) for k, _ in curved)  # curved cells: the fused kernels only
    assert candidates(256, False, 5, api.FP64) == [(0, 0)]
    assert candidates(256, False, 1, api.FP64).count((9, 0)) == 0  # p = 1: not offered


def test_tune_choice_records():
    old = TuneChoice(**{"prec": 0, "kernel": 0, "grid": 4, "us": 58.7})  # a record without shapes
    assert (old.tm_unit_steps, old.tm_long_steps, old.tm_us) == (0, 0, 0.0)
    assert "overlap" not in old.describe()
    new = TuneChoice(0, 9, 0, 52.6, 8, 4, 19.2)
    assert "line-per-cell" in new.describe() and "overlap 8/4" in new.describe()
    assert set(TM_STEPS) == {4, 8, 16}
