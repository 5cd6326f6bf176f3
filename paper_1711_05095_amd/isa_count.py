"""VALU instructions in the event loop of a step kernel, counted from the
gfx950 assembly of this repository's own kernels.

The count is the per-event work figure of the ALU roofline in bench.py: one
event (a Philox4x32-10 block, the waiting time, the choice and execution of a
hop) executes the loop body once.  The loop is the smallest backward-branch
region of the kernel that contains the Philox multiplies (v_mad_u64_u32).

The guided step's loop is split the same way into the path every random draw
runs and the path a taken proposal adds (guided_paths).

    python -m paper_1711_05095_amd.isa_count [kernel-symbol-prefix | guided]
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


# The guided step's loop (pd_guided.hip) runs one random draw per pass: a
# proposal, or the interval's closing draw.  A taken proposal then runs the hop
# path (the jump term, the 14 + 14 table reads that keep S, the hop).  The two
# paths are told apart by assembler comments placed in a copy of the source at
# the start and the end of the hop path; the copy is also fixed to the branch a
# trained table and L >= 26 take (tables below 2^32 / 14, the 26-site window),
# which are uniform over a launch.
GUIDED_SRC = os.path.join(HERE, "csrc", "pd_guided.hip")
_TAKEN = "(uint32_t)egmax) >= e) continue;\n"
_HOP_END = "        r = popcount_words<W>(m);\n        ++kb;\n    }\n"


def guided_paths(W=2):
    """(VALU instructions per draw, extra VALU instructions per taken proposal)
    in the loop of k_step_g<W, false>."""
    from .build import HIPCC_FLAGS
    src = open(GUIDED_SRC).read()
    for piece, n in ((_TAKEN, 1), (_HOP_END, 1), ("if (narrow) {", 1), ("if (L >= 26) {", 2)):
        if src.count(piece) != n:
            raise RuntimeError("guided loop source changed: %r" % piece)
    src = src.replace(_TAKEN, _TAKEN + '        asm volatile("; hop path begins");\n')
    src = src.replace(_HOP_END, _HOP_END[:-6] + '\n        asm volatile("; hop path ends");\n    }\n')
    src = src.replace("if (narrow) {", "if (true) {").replace("if (L >= 26) {", "if (true) {")
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    d = tempfile.mkdtemp()
    open(os.path.join(d, "g.hip"), "w").write(src)
    subprocess.check_call([hipcc] + HIPCC_FLAGS + ["-I", os.path.dirname(GUIDED_SRC), "-x", "hip",
                                                   "-c", "g.hip", "-o", "g.o", "--save-temps"],
                          cwd=d, stderr=subprocess.DEVNULL)
    name = [f for f in os.listdir(d) if f.endswith("gfx950.s")][0]
    lines = open(os.path.join(d, name)).read().splitlines()
    body = kernel_lines(lines, "_ZN2pd8k_step_gILi%dELb0E" % W)
    loop = event_loop_valu(body)
    b = [i for i, l in enumerate(body) if "hop path begins" in l]
    e = [i for i, l in enumerate(body) if "hop path ends" in l]
    if len(b) != 1 or len(e) != 1 or e[0] <= b[0]:
        raise RuntimeError("hop path markers not found once each")
    hop = sum(1 for r in body[b[0]:e[0] + 1] if re.match(r"^\s*v_", r))
    return loop - hop, hop


if __name__ == "__main__":
    print(guided_paths() if sys.argv[1:] == ["guided"] else count(*sys.argv[1:]))
