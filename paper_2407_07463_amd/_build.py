"""Build steps for the native parts of the package (all in-tree).

- `libvofmt.so`: the HIP kernels and their C ABI, compiled by hipcc for gfx950.
  No FMA contraction (-ffp-contract=off): every floating-point expression of
  the method is evaluated exactly as written, like the CPU reference it is
  checked against. Packed-FP32 instruction selection is disabled.
- `synth/libsynth.so`: the seeded input generator (plain C, OpenMP).
"""
from __future__ import annotations

import glob
import os
import subprocess

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIBVOFMT = os.path.join(PKG, "libvofmt.so")
LIBSYNTH = os.path.join(PKG, "synth", "libsynth.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

HIP_FLAGS = [
    f"--offload-arch={ARCH}",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
    "-Wno-unused-function",
    "-Werror=shadow",  # a local that hides a parameter or outer local is an error
    f"-I{INCLUDE}",
    f"-I{CSRC}",
]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def build_synth(verbose: bool = False) -> str:
    src = os.path.join(PKG, "synth", "synth.c")
    _run(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", LIBSYNTH + ".tmp", src, "-lm"], verbose)
    os.replace(LIBSYNTH + ".tmp", LIBSYNTH)
    return LIBSYNTH


def build_hip(verbose: bool = False, jobs: int = 8) -> str:
    """Compile every csrc/*.hip and csrc/*.cpp to objects, link libvofmt.so."""
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip"))) + sorted(glob.glob(os.path.join(CSRC, "*.cpp")))
    objdir = os.path.join(PKG, "_build")
    os.makedirs(objdir, exist_ok=True)
    objs = []
    procs = []
    for s in srcs:
        o = os.path.join(objdir, os.path.basename(s) + ".o")
        objs.append(o)
        lang = ["-x", "hip"] if s.endswith(".hip") else []
        cmd = [HIPCC] + HIP_FLAGS + lang + ["-c", s, "-o", o]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((s, subprocess.Popen(cmd)))
        if len(procs) >= jobs:
            s0, p0 = procs.pop(0)
            if p0.wait() != 0:
                raise RuntimeError(f"hipcc failed on {s0}")
    for s0, p0 in procs:
        if p0.wait() != 0:
            raise RuntimeError(f"hipcc failed on {s0}")
    _run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", LIBVOFMT + ".tmp"] + objs, verbose)
    os.replace(LIBVOFMT + ".tmp", LIBVOFMT)
    return LIBVOFMT


def build_all(verbose: bool = False) -> None:
    build_synth(verbose)
    build_hip(verbose)
