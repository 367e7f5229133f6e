"""Host-side checks of the batched-launch planner (no device work)."""
import numpy as np

import paper_1910_09020_amd as ss


def test_plan_validation_without_device():
    L = ss.lib()
    assert L.ss_plan_create(None, None, None, 0, 8, None) == ss.SS_EINVAL
    bad = ss.SS_EINVAL
    assert L.ss_plan_info(None, None, None, None, None) == bad
    assert L.ss_plan_launch(None, None) == bad
    assert L.ss_plan_destroy(None) == bad
