"""Compile the HIP library ``libp2m.so`` for gfx950, in-tree.

Host preprocessing sources (``csrc/host/*.cpp``) are built with g++; the
kernels and the C ABI (``csrc/*.hip``) with hipcc for gfx950.  Packed FP32
instructions are disabled for all device code.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT_DIR = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libp2m.so")
INCLUDE = os.path.join(ROOT, "include")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = os.environ.get("P2M_OFFLOAD_ARCH", "gfx950")

HOST_FLAGS = ["-O3", "-std=c++17", "-fPIC", "-pthread", "-Wall", "-Wno-sign-compare",
              "-I", INCLUDE, "-I", CSRC]
HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-I", INCLUDE, "-I", CSRC, "-Wno-unused-result"]


def sources():
    host = sorted(os.path.join(CSRC, "host", f) for f in os.listdir(os.path.join(CSRC, "host"))
                  if f.endswith(".cpp"))
    hip = sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))
    return host, hip


def build(verbose=False):
    os.makedirs(OUT_DIR, exist_ok=True)
    host, hip = sources()
    jobs = []
    objs = []
    for src in host:
        obj = os.path.join(OUT_DIR, os.path.basename(src) + ".o")
        jobs.append(["g++", *HOST_FLAGS, "-c", src, "-o", obj])
        objs.append(obj)
    for src in hip:
        obj = os.path.join(OUT_DIR, os.path.basename(src) + ".o")
        # the preprocessing kernels reproduce the host's FP64 arithmetic exactly
        extra = ["-ffp-contract=off"] if os.path.basename(src) in ("lists.hip", "voronoi.hip") else []
        jobs.append([HIPCC, *HIP_FLAGS, *extra, "-c", src, "-o", obj])
        objs.append(obj)
    procs = []
    for cmd in jobs:
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
    failed = []
    for cmd, p in procs:
        out, _ = p.communicate()
        text = out.decode(errors="replace")
        # hipcc's host pass does not know the packed-fp32 feature; that warning is harmless
        text = "\n".join(l for l in text.splitlines() if "packed-fp32-ops" not in l)
        if p.returncode != 0:
            failed.append((cmd, text))
        elif verbose and text.strip():
            print(text)
    if failed:
        for cmd, text in failed:
            sys.stderr.write(" ".join(cmd) + "\n" + text + "\n")
        raise RuntimeError("libp2m build failed")
    tmp = LIB + ".tmp"
    subprocess.check_call([HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp, *objs,
                           "-pthread"])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
