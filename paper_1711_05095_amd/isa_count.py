"""VALU instructions in the event loop of a step kernel, counted from the
gfx950 assembly of this repository's own kernels.

The count is the per-event work figure of the ALU roofline in bench.py: one
event (a Philox4x32-10 block, the waiting time, the choice and execution of a
hop) executes the loop body once.  The loop is the smallest backward-branch
region of the kernel that contains the Philox multiplies (v_mad_u64_u32).

    python -m paper_1711_05095_amd.isa_count [kernel-symbol-prefix]
"""
import os
import re
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "csrc", "pd_kernels.hip")


def assembly():
    from .build import HIPCC_FLAGS
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    d = tempfile.mkdtemp()
    subprocess.check_call([hipcc] + HIPCC_FLAGS + ["-x", "hip", "-c", SRC, "-o",
                                                   os.path.join(d, "k.o"), "--save-temps"],
                          cwd=d, stderr=subprocess.DEVNULL)
    name = [f for f in os.listdir(d) if f.endswith("gfx950.s")][0]
    return open(os.path.join(d, name)).read().splitlines()


def kernel_lines(lines, prefix):
    for i, l in enumerate(lines):
        if l.startswith(prefix) and l.split(":")[0].startswith(prefix) and ":" in l:
            out = []
            for m in lines[i + 1:]:
                out.append(m)
                if "s_endpgm" in m:
                    return out
    raise KeyError(prefix)


def event_loop_valu(body):
    labels = {}
    for i, l in enumerate(body):
        m = re.match(r"^(\.LBB\w+):", l)
        if m:
            labels[m.group(1)] = i
    best = None
    for i, l in enumerate(body):
        m = re.search(r"s_c?branch\w*\s+(\.LBB\w+)", l)
        if not m or m.group(1) not in labels:
            continue
        start = labels[m.group(1)]
        if start >= i:
            continue  # not a backward branch
        region = body[start:i + 1]
        if sum("v_mad_u64_u32" in r for r in region) < 10:
            continue
        if best is None or len(region) < len(best):
            best = region
    if best is None:
        raise RuntimeError("no event loop found")
    return sum(1 for r in best if re.match(r"^\s*v_", r))


def count(prefix="_ZN2pd6k_stepILi2E"):
    return event_loop_valu(kernel_lines(assembly(), prefix))


if __name__ == "__main__":
    print(count(*sys.argv[1:]))
