"""Builds libqvpu.so (HIP, gfx950) in-tree with hipcc.

    python -m paper_2406_03466_amd.build
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libqvpu.so")
OBJDIR = os.path.join(HERE, "_build")

SOURCES = ["kernels.hip", "qvpu_api.cpp", "planner.cpp", "jit.cpp"]
# headers compiled again at run time with a generated op program (jit.cpp): embedded as text
GEN_HEADERS = [("tile_device.h", CSRC), ("engine.h", CSRC), ("qvpu.h", INCLUDE)]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

# Packed FP32 instructions are kept out of the generated code on purpose.
COMMON = ["-O3", "-fPIC", "-std=c++17", f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang",
          "-packed-fp32-ops", "-Wall", "-Wno-unused-function", "-I", INCLUDE, "-I", CSRC, "-I", OBJDIR]


def _embed_headers() -> None:
    """Writes _build/jit_headers.inc: the texts of the headers a generated tile pass includes."""
    names, texts = [], []
    for i, (name, d) in enumerate(GEN_HEADERS):
        text = open(os.path.join(d, name)).read()
        delim = f"QVGEN{i}"
        if f"){delim}\"" in text:
            raise RuntimeError(f"{name} holds the raw-string delimiter {delim}")
        names.append(f'"{name}"')
        texts.append(f'R"{delim}({text}){delim}"')
    out = (f"static const int kGenHeaderCount = {len(names)};\n"
           f"static const char *kGenHeaderNames[] = {{{', '.join(names)}}};\n"
           f"static const char *kGenHeaderText[] = {{\n" + ",\n".join(texts) + "};\n")
    path = os.path.join(OBJDIR, "jit_headers.inc")
    tmp = f"{path}.tmp{os.getpid()}"   # parallel test workers each write their own before the rename
    with open(tmp, "w") as f:
        f.write(out)
    os.replace(tmp, path)


def _compile(src: str) -> str:
    obj = os.path.join(OBJDIR, os.path.splitext(src)[0] + ".o")
    defines = []
    if os.environ.get("QV_ADJ_INNER_F64") == "1":   # the precompiled adjoint's inner products in FP64
        defines.append("-DQV_ADJ_INNER_F64=1")
    cmd = [HIPCC, *COMMON, *defines, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(OBJDIR, exist_ok=True)
    _embed_headers()
    with ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs, "-lhiprtc"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
