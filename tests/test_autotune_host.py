"""Host logic of the autotuner (CPU only): size classes of a batch."""
import numpy as np

from paper_2505_08174_amd import autotune as AT


def test_size_classes_group_by_power_of_two_and_kind():
    off = np.array([0, 5000, 12000, 200000, 205000, 205001])
    g = AT.size_classes(off, ["s", "f", "s", "s", "f"])
    assert g == {(12, "s"): [0, 3], (12, "f"): [1], (17, "s"): [2], (0, "f"): [4]}
    g2 = AT.size_classes(off)
    assert sorted(sum(g2.values(), [])) == [0, 1, 2, 3, 4]
    assert g2[(12, None)] == [0, 1, 3]
