"""Control-flow check of the persistent dataflow kernel's gfx950 assembly.

The kernel's item loop holds workgroup barriers.  If any loop whose exit
depends on the exec mask (a lane-divergent loop, as the compiler builds for
a branch on the thread id) contains a barrier, part of a wave can return to
the barrier while another part of it is parked outside the loop, and the
workgroup never makes progress.  The kernel keeps its loop control uniform
per wave; this test compiles persist_kernels.hip to assembly and checks, for
every instantiation, that no divergent loop (one whose latch clears exec
lanes with s_andn2_b64) has an s_barrier in its body, nested loops included.
"""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "paper_2208_05740_amd", "csrc", "persist_kernels.hip")


def _blocks(lines):
    """(name, first line, end line) of every basic block; the entry block is 'entry'."""
    out, cur = [], ("entry", 0)
    for i, line in enumerate(lines):
        m = re.match(r"^\.L(BB\d+_\d+):", line) or re.match(r"^; %(bb\.\d+):", line)
        if m:
            out.append((cur[0], cur[1], i))
            cur = (m.group(1), i)
    out.append((cur[0], cur[1], len(lines)))
    return out


def divergent_loops_with_barriers(asm: str):
    lines = asm.split("\n")
    chain, inner = {}, {}
    for name, s, _ in _blocks(lines):
        head = lines[s]
        comments = [head] + [x for x in lines[s + 1:s + 64] if x.strip().startswith(";")]
        text = "\n".join(comments)
        if re.search(r"This (Inner )?Loop Header", text):
            chain[name] = re.findall(r"Parent Loop (BB\d+_\d+) Depth", text) + [name]
            inner[name] = name
        else:
            m = re.search(r"in Loop: Header=(BB\d+_\d+) Depth", head)
            inner[name] = m.group(1) if m else None
    has_barrier, divergent = {}, set()
    for name, s, e in _blocks(lines):
        body = lines[s:e]
        bar = any("s_barrier" in x for x in body)
        for loop in chain.get(inner.get(name), []):
            has_barrier[loop] = has_barrier.get(loop, False) or bar
        if inner.get(name) and any("s_andn2_b64 exec, exec," in x for x in body):
            divergent.add(inner[name])
    return sorted(loop for loop in divergent if has_barrier.get(loop))


def _kernels(asm: str):
    out = {}
    for m in re.finditer(r"^(_Z\w*persist_kernel\w*):", asm, re.M):
        end = asm.index("s_endpgm", m.end())
        out[m.group(1)] = asm[m.end():end]
    return out


@pytest.mark.skipif(shutil.which("hipcc") is None and not os.path.exists("/opt/rocm/bin/hipcc"),
                    reason="hipcc not available")
def test_no_barrier_inside_a_lane_divergent_loop(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    out = tmp_path / "persist.s"
    cmd = [hipcc, "-O3", "-std=c++17", "--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang",
           "-packed-fp32-ops", "--cuda-device-only", "-S", SRC, "-o", str(out)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    kernels = _kernels(out.read_text())
    assert len(kernels) == 8, sorted(kernels)   # {fp32, bf16} x {agent, xcd} x {4, 5 waves}
    for name, body in kernels.items():
        assert divergent_loops_with_barriers(body) == [], name


def test_scanner_flags_a_divergent_loop_around_a_barrier():
    """The scanner itself: a hand-written loop whose latch is exec-based and
    whose body has a barrier is reported; the same loop with a scalar latch
    is not."""
    bad = "\n".join([
        ".LBB0_1:                                ; =>This Loop Header: Depth=1",
        "\ts_barrier",
        "\tv_cmp_eq_u32_e32 vcc, 0, v0",
        "; %bb.2:                                ;   in Loop: Header=BB0_1 Depth=1",
        "\ts_andn2_b64 exec, exec, s[4:5]",
        "\ts_cbranch_execnz .LBB0_1",
        ".LBB0_3:",
        "\ts_endpgm",
    ])
    assert divergent_loops_with_barriers(bad) == ["BB0_1"]
    good = bad.replace("s_andn2_b64 exec, exec, s[4:5]", "s_and_b64 vcc, exec, s[4:5]")
    assert divergent_loops_with_barriers(good) == []
