"""CPU checks of the tile passes the library generates at run time (option "specialize"): for circuits
covering every op code (rotations, fixed gates, diagonal ops on register and thread qubits, CNOTs between
register bits and with thread controls, CZ, fused blocks), every register-tiled pass's generated source
compiles with hipRTC for gfx950 in both directions and both precisions, its code holds no packed FP32
instruction, and no loop holding a barrier exits through an exec mask (the property the precompiled tile
kernels are held to in test_kernel_structure_cpu.py). No GPU is used.
"""
import os
import re
import subprocess

import numpy as np
import pytest

from paper_2406_03466_amd import build as B
from paper_2406_03466_amd import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))
OBJDUMP = "/opt/rocm/llvm/bin/llvm-objdump"


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    B._embed_headers()
    exe = str(tmp_path_factory.mktemp("gen") / "gen_driver")
    cmd = [B.HIPCC, "-O1", "-std=c++17", "-I", B.INCLUDE, "-I", B.CSRC, "-I", B.OBJDIR, "-o", exe,
           os.path.join(HERE, "gen_driver.cpp"), os.path.join(B.CSRC, "planner.cpp"), os.path.join(B.CSRC, "jit.cpp"),
           "-lhiprtc"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    return exe


def _circuit_text(n, gates, tile, lowc, rb, fuse, prec, inner_f64):
    lines = [f"{n} {tile} {lowc} {rb} {fuse} {prec} {inner_f64}"]
    for g in gates:
        lines.append(f"{int(g['kind'])} {int(g['q0'])} {int(g['q1'])} {1 if g['param'] >= 0 else 0}")
    return "\n".join(lines) + "\n"


def _mixed_circuit(n, seed):
    """Every gate kind on random qubits, with trainable and fixed rotations."""
    rng = np.random.default_rng(seed)
    gates, p = [], 0
    for i in range(90):
        kind = int(rng.integers(0, 11))
        if kind in (W.CNOT, W.CZ):
            a, b = rng.choice(n, 2, replace=False)
            gates.append(W.gate(kind, int(a), int(b)))
        elif kind in (W.RX, W.RY, W.RZ):
            gates.append(W.gate(kind, int(rng.integers(n)), -1, p if i % 3 else -1, 0.3))
            p += i % 3 != 0
        else:
            gates.append(W.gate(kind, int(rng.integers(n))))
    return np.array(gates, W.GATE_DTYPE)


CASES = [
    ("hea12_L2_c64_fused", 12, lambda: W.hea_layers(12, 2)[0], 10, 4, 4, 3, 0, 0),
    ("hea12_L2_c64_inner_f64", 12, lambda: W.hea_layers(12, 2)[0], 10, 4, 4, 0, 0, 1),
    ("hea12_L2_c128", 12, lambda: W.hea_layers(12, 2)[0], 10, 3, 3, 0, 1, 0),
    ("mixed14_c64", 14, lambda: _mixed_circuit(14, 5), 11, 4, 4, 2, 0, 0),
    ("mixed14_c128", 14, lambda: _mixed_circuit(14, 6), 10, 3, 3, 0, 1, 0),
]


@pytest.mark.parametrize("name,n,make,tile,lowc,rb,fuse,prec,inner", CASES, ids=[c[0] for c in CASES])
def test_generated_passes_compile(driver, tmp_path, name, n, make, tile, lowc, rb, fuse, prec, inner):
    gates = np.array(make(), W.GATE_DTYPE)
    r = subprocess.run([driver, str(tmp_path)], input=_circuit_text(n, gates, tile, lowc, rb, fuse, prec, inner),
                       capture_output=True, text=True, timeout=900)
    assert r.returncode == 0, r.stdout[-4000:] + r.stderr[-2000:]
    objs = sorted(tmp_path.glob("*.co"))
    assert objs and len(objs) % 2 == 0
    for co in objs:
        asm = subprocess.run([OBJDUMP, "-d", str(co)], capture_output=True, text=True).stdout
        assert not re.search(r"v_pk_(fma|mul|add)_f32", asm), f"{co.name}: packed FP32 instruction"
        # the disassembly has no loop annotations: rebuild them from backward branches
        lines = asm.split("\n")
        bad, withb = barrier_loops_from_branches(lines)
        assert withb, f"{co.name}: no loop with a barrier found (the parser no longer matches the disassembly)"
        assert not bad, f"{co.name}: a loop holding a barrier exits through an exec mask"


def barrier_loops_from_branches(lines):
    """Loops of a disassembled kernel from its backward branches: the span [target, branch] is a loop; it
    holds a barrier if any instruction in it is s_barrier, and exits divergently if it holds an
    s_andn2_b64 exec write followed by a conditional branch on exec back to its head."""
    addr_of, ins = {}, []
    for ln in lines:
        m = re.match(r"^\s+([sv]_\w+)(.*?)//\s*([0-9A-Fa-f]+):", ln)
        if m:
            ins.append((int(m.group(3), 16), m.group(1), m.group(2)))
    bad, withb = [], []
    for i, (addr, op, rest) in enumerate(ins):
        if not op.startswith("s_cbranch") and op != "s_branch":
            continue
        imm = re.match(r"\s*(\d+)", rest)
        if not imm:
            continue
        simm = int(imm.group(1))
        simm = simm - 65536 if simm >= 32768 else simm   # 16-bit signed offset in dwords
        t = addr + 4 + 4 * simm
        if t >= addr:
            continue
        body = [x for x in ins if t <= x[0] <= addr]
        if any(x[1] == "s_barrier" for x in body):
            withb.append((t, addr))
            if op == "s_cbranch_execnz" and any(x[1] == "s_andn2_b64" and x[2].strip().startswith("exec")
                                                for x in body):
                bad.append((t, addr))
    return bad, withb
