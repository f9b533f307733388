"""Builds the host-side harnesses of the device arithmetic (tests/native/*.hip)
into paper_2605_23088_amd/_build/ with hipcc; rebuilt when a source is newer."""
import ctypes
import glob
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
BUILD = os.path.join(ROOT, "paper_2605_23088_amd", "_build")


def load(name):
    src = os.path.join(ROOT, "tests", "native", name + ".hip")
    out = os.path.join(BUILD, "lib" + name + ".so")
    deps = [src] + glob.glob(os.path.join(ROOT, "paper_2605_23088_amd", "csrc", "*.h"))
    os.makedirs(BUILD, exist_ok=True)
    if not os.path.exists(out) or os.path.getmtime(out) < max(os.path.getmtime(p) for p in deps):
        cmd = ["/opt/rocm/bin/hipcc", "--offload-arch=gfx950", "-O2", "-std=c++17", "-fPIC", "-shared",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", src, "-o", out + ".tmp"]
        subprocess.run(cmd, check=True, capture_output=True)
        os.replace(out + ".tmp", out)
    return ctypes.CDLL(out)
