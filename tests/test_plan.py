"""Host-side planning of the gradient (no GPU needed): filter groups and the
compact BF16 residual, as reported by hicu_filter_group."""
import numpy as np

import paper_2004_08962_amd as hicu

VOL = ((256, 320, 320, 8), (5, 5, 5))


def _s(shape, kd):
    return int(np.prod([d - k + 1 for d, k in zip(shape[:3], kd)]))


def test_volume_groups_and_compact_residual():
    hicu.set_filter_group_budget(0)
    # 900 filters x 25 163 712 outputs: complex64 Y needs 181 GB > 16 GiB
    assert hicu.filter_group(*VOL, 900, "fp32") == (64, False)
    assert hicu.filter_group(*VOL, 900, "bf16x3") == (64, False)
    assert hicu.filter_group(*VOL, 900, "fp16") == (64, False)
    # BF16 stores Y as BF16 pairs: half the bytes, twice the filters per group
    assert hicu.filter_group(*VOL, 900, "bf16") == (128, True)


def test_small_problems_keep_complex64_residual():
    hicu.set_filter_group_budget(0)
    assert hicu.filter_group((1, 256, 232, 16), (1, 5, 5), 280, "bf16") == (280, False)
    assert hicu.filter_group((16, 28, 28, 8), (5, 5, 5), 900, "bf16") == (900, False)


def test_budget_sets_group_size():
    shape, kd = (9, 14, 12, 4), (3, 3, 3)
    s = _s(shape, kd)
    try:
        hicu.set_filter_group_budget(s * 4 * 64)
        assert hicu.filter_group(shape, kd, 100, "bf16") == (64, True)
        assert hicu.filter_group(shape, kd, 100, "fp32") == (64, False)
        hicu.set_filter_group_budget(s * 8 * 128)
        assert hicu.filter_group(shape, kd, 300, "fp32") == (128, False)
        assert hicu.filter_group(shape, kd, 300, "bf16") == (256, True)
        # never below 64 filters, never above p
        hicu.set_filter_group_budget(1)
        assert hicu.filter_group(shape, kd, 100, "fp32") == (64, False)
        assert hicu.filter_group(shape, kd, 50, "fp32") == (50, False)
    finally:
        hicu.set_filter_group_budget(0)
    # 2-D problems (one plane per tile) never use the compact residual
    try:
        hicu.set_filter_group_budget(1)
        assert hicu.filter_group((1, 40, 36, 6), (1, 5, 5), 97, "bf16") == (64, False)
    finally:
        hicu.set_filter_group_budget(0)
