"""Build libraysh.so (HIP, gfx950) in-tree with hipcc.

Every HIP source is compiled with packed-FP32 instructions disabled.
"""
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libraysh.so")
SOURCES = ["raysh_api.hip", "raysh_batch.hip", "raysh_tune.hip", "shoot_fp64.hip",
           "shoot_fp32.hip", "shoot_expansion.hip", "histogram.hip", "light_curves.hip", "mlp.hip",
           "fma_probe.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
         "-Wall", "-Wno-unused-function",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", INCLUDE, "-I", CSRC]


def sources():
    return [os.path.join(CSRC, s) for s in SOURCES]


def build(out=LIB, extra=(), verbose=False):
    tmp = out + ".tmp"
    cmd = [HIPCC, *FLAGS, *extra, *sources(), "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    msgs = "\n".join(l for l in (r.stdout + r.stderr).splitlines()
                     if "packed-fp32-ops" not in l and "is not a recognized feature" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed ({r.returncode}):\n{msgs}")
    if verbose and msgs.strip():
        print(msgs)
    os.replace(tmp, out)
    return out


def assemble(source, out, extra=()):
    """Device assembly of one source (for reading the generated ISA)."""
    cmd = [HIPCC, *[f for f in FLAGS if f not in ("-shared", "-fPIC")], *extra,
           "--cuda-device-only", "-S", os.path.join(CSRC, source), "-o", out]
    subprocess.run(cmd, check=True, capture_output=True)
    return out


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
