"""The tile autotuner's host side: every candidate is a setting the library
accepts (sizes multiples of 256, item caps >= 1, 256- or 512-thread blocks,
CG form 0, 1 or 2, as sip_batch_set_tiles documents), candidates are distinct,
and the workload key separates the classes it is meant to separate."""
import pytest

from paper_1902_09699_amd import autotune


def test_candidates_are_valid_and_distinct():
    seen = set()
    for c in autotune.CANDIDATES:
        pt_points, pt_max_items, thr_points, thr_max_items, pt_threads, cg_form = c
        assert pt_points % 256 == 0 and thr_points % 256 == 0 and pt_points >= 256 and thr_points >= 256
        assert pt_max_items >= 1 and thr_max_items >= 1
        assert pt_threads in (256, 512)
        assert cg_form in (0, 1, 2)
        assert c not in seen
        seen.add(c)
    # every CG arrangement and both block sizes are on the list
    assert {c[5] for c in autotune.CANDIDATES} == {0, 1, 2}
    assert {c[4] for c in autotune.CANDIDATES} == {256, 512}


@pytest.mark.parametrize("a,b", [
    (("f32", [(341, 1361)]), ("f64", [(341, 1361)])),
    (("f32", [(341, 1361)]), ("f32", [(200, 200, 100)])),
    (("f32", [(64, 64)]), ("f32", [(341, 1361)])),
    (("f32", [(64, 64)]), ("f32", [(64, 64)] * 256)),
])
def test_workload_key_separates_classes(a, b):
    assert autotune.workload_key(*a) != autotune.workload_key(*b)


def test_workload_key_groups_nearby_sizes():
    assert autotune.workload_key("f32", [(341, 1361)]) == autotune.workload_key("f32", [(340, 1360)])
