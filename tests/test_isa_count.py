"""The per-event unit of bench.py's ALU roofline is frozen at the VALU count of
the step kernel's event loop at a named commit, so that the roofline fraction
follows throughput.  The loop as it is built now must not have grown past
that unit (a leaner loop is fine: the same events then cost less)."""
import os
import shutil

import pytest

import bench
from paper_1711_05095_amd import isa_count


@pytest.mark.skipif(not (shutil.which("hipcc") or os.path.exists("/opt/rocm/bin/hipcc")),
                    reason="hipcc not available")
def test_event_loop_within_the_frozen_unit():
    assert isa_count.count() <= bench.VALU_PER_EVENT_W2
    assert isa_count.count("_ZN2pd6k_stepILi7E") <= bench.VALU_PER_EVENT_W7
    # the default compacting kernel runs the same event with the next event's
    # random numbers formed ahead: two moves more per event
    assert isa_count.count("_ZN2pd8k_step_cILi2E") <= bench.VALU_PER_EVENT_W2 + 2


@pytest.mark.skipif(not (shutil.which("hipcc") or os.path.exists("/opt/rocm/bin/hipcc")),
                    reason="hipcc not available")
def test_guided_paths_within_the_frozen_unit():
    per_draw, per_hop = isa_count.guided_paths()
    assert per_draw <= bench.VALU_PER_DRAW_G2 and per_hop <= bench.VALU_PER_HOP_G2
