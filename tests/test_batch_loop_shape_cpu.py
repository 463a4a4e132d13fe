"""Shape of the persistent batch kernel's task loop in the compiled gfx950 code (no GPU needed).

Every wave of a workgroup must fetch the task index, pass the two queue
barriers and test for the end of the queue in one loop.  If the compiler
nests the barriers in a loop inside the one that holds the queue atomic,
the inner loop's exit is per lane: lanes re-read a stale index and the
kernel never ends.  This compiles spin_batch_kernels.hip to assembly and
checks, for every instantiation of k_batch, that the two barriers after the
atomic sit in the outermost loop, not in a nested one.
"""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1006_3865_amd", "csrc")


def loop_of_blocks(lines, start, end):
    """Block label -> (enclosing header label or None, nested?) from the compiler's loop comments."""
    info = {}
    for l in lines[start:end]:
        m = re.match(r"^(\.LBB\d+_\d+):(.*)$", l)
        if not m:
            continue
        c = m.group(2)
        if "Parent Loop" in c:
            info[m.group(1)] = ("nested", re.search(r"Parent Loop (BB\d+_\d+)", c).group(1))
        elif "This Loop Header" in c:
            info[m.group(1)] = ("header", m.group(1)[1:])
        else:
            h = re.search(r"Header=(BB\d+_\d+) Depth=(\d+)", c)
            info[m.group(1)] = ("in", h.group(1)) if h and h.group(2) == "1" else ("other", None)
    return info


def test_queue_barriers_in_outermost_loop(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    asm = str(tmp_path / "batch.s")
    subprocess.check_call([hipcc, "--offload-arch=gfx950", "-O3", "-std=c++17", "-Xclang", "-target-feature",
                           "-Xclang", "-packed-fp32-ops", "-I", os.path.join(ROOT, "include"), "-I", CSRC,
                           "-x", "hip", "--cuda-device-only", "-S", os.path.join(CSRC, "spin_batch_kernels.hip"),
                           "-o", asm], stderr=subprocess.DEVNULL)
    lines = open(asm).read().split("\n")
    names = [l.split(":")[0] for l in lines if re.match(r"^_ZN4spin7k_batch\w+:", l)]
    assert len(names) == 16
    for name in names:
        start = next(i for i, l in enumerate(lines) if l.startswith(name + ":"))
        end = next(i for i in range(start, len(lines)) if lines[i].strip().startswith(".Lfunc_end"))
        info = loop_of_blocks(lines, start, end)
        blk, seen, bars = None, False, []
        for l in lines[start:end]:
            m = re.match(r"^(\.LBB\d+_\d+):", l)
            if m:
                blk = m.group(1)
            t = l.strip()
            if t.startswith("global_atomic"):
                seen = True
            elif seen and t.startswith("s_barrier") and len(bars) < 2:
                bars.append(blk)
        assert seen and len(bars) == 2, name
        for b in bars:
            kind, _ = info[b]
            assert kind in ("in", "header"), "%s: a queue barrier sits in a nested loop (%s)" % (name, b)
