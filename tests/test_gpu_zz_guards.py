"""Runs last among the GPU tests: with TR_ALS_CANARY=1 every context created
by the earlier tests carried guard bands behind its workspace buffers, checked
when it was destroyed; none may have been written."""
import pytest

pytestmark = pytest.mark.gpu


def test_no_workspace_overrun_detected():
    import os
    from paper_2210_11362_amd import _lib as C
    assert os.environ.get("TR_ALS_CANARY") == "1", "guard bands are off: this check would be empty"
    assert C.lib().tr_als_debug_overruns() == 0
