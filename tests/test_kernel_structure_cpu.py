"""CPU check of the compiled tile kernels' control flow (gfx950 assembly, compiled here with hipcc).

A workgroup barrier (s_barrier) counts waves, not lanes. If a loop that contains a barrier exits through an
exec mask (some lanes of a wave leave the loop while others go round again), the lanes still in the loop
reach the barrier again without the lanes that left, and the wave can run forever. The persistent tile
kernels once compiled to exactly that: the work-queue claim at the top of the loop and the completion
count at its bottom, each under its own `threadIdx.x == 0` test, were joined by the compiler across the
back edge, so wave 0's other lanes re-read the old item at the top barrier while lane 0 waited outside
the inner loop to claim the next one. This test compiles the kernels to assembly and checks, from the
compiler's own loop annotations, that no loop holding a barrier has a divergent exit.
"""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2406_03466_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def _loops(lines):
    """Blocks of one function: (label, innermost loop header, instructions) and the loop tree."""
    blocks, parent, cur = [], {}, None
    for ln in lines:
        m = re.match(r"^(\.LBB\d+_\d+|; %bb\.\d+):\s*(;.*)?$", ln)
        if m or cur is None:
            lab = m.group(1) if m else "entry"
            comment = (m.group(2) or "") if m else ""
            hdr = None
            mh = re.search(r"Header=BB(\d+_\d+)", comment)
            if mh:
                hdr = "BB" + mh.group(1)
            if "This Loop Header" in comment or "This Inner Loop Header" in comment:
                hdr = "BB" + lab.split("BB")[-1]
            cur = [lab, hdr, []]
            blocks.append(cur)
            continue
        mp = re.search(r"Parent Loop BB(\d+_\d+)", ln)
        if mp and cur[1] and cur[0].startswith(".LBB") and cur[1] == "BB" + cur[0].split("BB")[-1]:
            parent[cur[1]] = "BB" + mp.group(1)  # the last one listed is the innermost parent
        cur[2].append(ln)
    return blocks, parent


def barrier_loops_with_divergent_exit(lines):
    blocks, parent = _loops(lines)

    def ancestors(h):
        out = []
        while h:
            out.append(h)
            h = parent.get(h)
        return out

    with_barrier, divergent = set(), set()
    for _, hdr, ins in blocks:
        if any("s_barrier" in x for x in ins):
            with_barrier.update(ancestors(hdr))
        if hdr and any(re.search(r"s_andn2_b64 exec, exec, s\[", x) for x in ins):
            divergent.add(hdr)
    return sorted(divergent & with_barrier), sorted(with_barrier)


@pytest.fixture(scope="module")
def asm(tmp_path_factory):
    out = tmp_path_factory.mktemp("asm") / "kernels.s"
    cmd = [HIPCC, "-O3", "-std=c++17", "--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang",
           "-packed-fp32-ops", "-I", os.path.join(ROOT, "include"), "-I", CSRC, "--cuda-device-only", "-S",
           "-o", str(out), os.path.join(CSRC, "kernels.hip")]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    return out.read_text().split("\n")


def _functions(lines, pattern):
    starts = [i for i, ln in enumerate(lines) if re.match(r"^_Z\S*:", ln) and re.search(pattern, ln)]
    for st in starts:
        end = next(i for i in range(st, len(lines)) if lines[i].startswith(".Lfunc_end"))
        yield lines[st].split(":")[0], lines[st:end]


def test_checker_flags_a_barrier_loop_with_divergent_exit():
    """The checker itself, on a hand-made function shaped like the old persistent claim loop: a loop with a
    barrier whose latch drops lanes through an exec mask."""
    fn = """_Zfake:
.LBB0_2:                               ; =>This Loop Header: Depth=1
	s_barrier
	ds_read_b64 v[2:3], v83
.LBB0_9:                               ;   in Loop: Header=BB0_2 Depth=1
	s_andn2_b64 exec, exec, s[82:83]
	s_cbranch_execnz .LBB0_2
	s_endpgm
.Lfunc_end0:""".split("\n")
    bad, withb = barrier_loops_with_divergent_exit(fn)
    assert bad == ["BB0_2"] and withb == ["BB0_2"]
    ok = [ln for ln in fn if "s_andn2_b64" not in ln]
    assert barrier_loops_with_divergent_exit(ok)[0] == []


@pytest.mark.parametrize("pattern", [r"k_rtile_(fwd|adj)_persist", r"k_rtile_(fwd|adj)I"])
def test_tile_kernels_keep_barrier_loops_uniform(asm, pattern):
    found = 0
    for name, body in _functions(asm, pattern):
        found += 1
        bad, withb = barrier_loops_with_divergent_exit(body)
        assert withb, f"{name}: no loop with a barrier found (the parser no longer matches the assembly)"
        assert not bad, f"{name}: loops {bad} hold a barrier and exit through an exec mask"
    assert found == 4
