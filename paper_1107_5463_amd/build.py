"""Build libsmc.so (HIP, gfx950) in-tree.

    python -m paper_1107_5463_amd.build

hipcc cross-compiles for gfx950 without a GPU.  Packed-FP32 instructions are
disabled for all device code (-packed-fp32-ops).
"""
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libsmc.so")
SOURCES = ["ising.hip", "fused.hip", "packed.hip", "tiles.hip", "batch.hip", "chains.hip", "continuous.hip", "init.hip", "measure.hip",
           "probe.hip", "runtime.cpp"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def flags():
    return ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Wall",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I", os.path.join(ROOT, "include"), "-I", CSRC]


def build(verbose: bool = False) -> str:
    objs = []
    objdir = os.path.join(PKG, "_build")
    os.makedirs(objdir, exist_ok=True)
    procs = []
    for src in SOURCES:
        obj = os.path.join(objdir, os.path.splitext(src)[0] + ".o")
        lang = ["-x", "hip"]
        cmd = [HIPCC] + flags() + lang + ["-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((subprocess.Popen(cmd, stderr=subprocess.PIPE, text=True), src))
        objs.append(obj)
    failed = []
    for p, src in procs:
        _, err = p.communicate()
        msgs = [line for line in err.splitlines()
                if "packed-fp32-ops" not in line and line.strip()]
        if p.returncode != 0:
            failed.append(src)
            sys.stderr.write("\n".join(msgs) + "\n")
        elif verbose and msgs:
            sys.stderr.write("\n".join(msgs) + "\n")
    if failed:
        raise RuntimeError(f"hipcc failed for {failed}")
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", LIB + ".tmp"] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
