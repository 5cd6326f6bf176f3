"""The per-event VALU count used by bench.py's roofline equals the count in the
gfx950 assembly of the step kernel as it is built now."""
import os
import shutil

import pytest

import bench
from paper_1711_05095_amd import isa_count


@pytest.mark.skipif(not (shutil.which("hipcc") or os.path.exists("/opt/rocm/bin/hipcc")),
                    reason="hipcc not available")
def test_bench_valu_count_matches_assembly():
    assert isa_count.count() == bench.VALU_PER_EVENT_W2
    assert isa_count.count("_ZN2pd6k_stepILi7E") == bench.VALU_PER_EVENT_W7
