"""Build libaoresp.so (HIP, gfx950) in-tree with hipcc.

Every source is compiled with contraction off, fp32 denormals kept, correctly
rounded fp32 division and without packed-fp32 instructions, then linked into
paper_2502_06337_amd/libaoresp.so next to this file.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libaoresp.so")
BUILD = os.path.join(HERE, "_build")
SOURCES = ["kernels.hip", "api.cpp", "batch.cpp", "server.cpp", "tuner.cpp", "noalloc.cpp"]
ARCH = os.environ.get("AORESP_ARCH", "gfx950")

FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    "-ffp-contract=off", "-fno-fast-math",
    "-fno-gpu-flush-denormals-to-zero", "-fhip-fp32-correctly-rounded-divide-sqrt",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-result",
]


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, src.replace(".", "_") + ".o")
    cmd = ["hipcc", *FLAGS, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    err = "\n".join(l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{err}")
    if err.strip():
        sys.stderr.write(err + "\n")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = ["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


# Device probes the benchmark runs to measure its roofs (a separate small library).
PROBE_SRC = os.path.join(CSRC, "probe.hip")
PROBE_LIB = os.path.join(HERE, "libaoresp_probe.so")


def build_probe(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    tmp = PROBE_LIB + ".tmp%d" % os.getpid()
    cmd = ["hipcc", *FLAGS, "-shared", "-x", "hip", PROBE_SRC, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        err = "\n".join(l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l)
        raise RuntimeError(f"probe build failed: {' '.join(cmd)}\n{err}")
    os.replace(tmp, PROBE_LIB)
    if verbose:
        print("built", PROBE_LIB)
    return PROBE_LIB


# Device check programs that the GPU tests run (test code, not part of the library).
CHECKS = {"recip_check": os.path.join(os.path.dirname(HERE), "tests", "recip_check.hip")}


def build_checks(verbose: bool = False) -> list:
    out = []
    for name, src in CHECKS.items():
        exe = os.path.join(os.path.dirname(src), name)
        cmd = ["hipcc", *[f for f in FLAGS if f not in ("-fPIC",)], "-x", "hip", src, "-o", exe]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            err = "\n".join(l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l)
            raise RuntimeError(f"check build failed: {' '.join(cmd)}\n{err}")
        if verbose:
            print("built", exe)
        out.append(exe)
    return out


if __name__ == "__main__":
    build(verbose=True)
    build_probe(verbose=True)
    build_checks(verbose=True)
