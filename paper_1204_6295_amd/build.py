"""Builds libdisc.so for gfx950 in-tree (paper_1204_6295_amd/libdisc.so).

Each HIP translation unit is compiled separately (in parallel) and then
linked into one shared library. Packed FP32 instructions are disabled for
all device code.
"""
import concurrent.futures
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
OUT = os.path.join(HERE, "libdisc.so")
BENCH_EXE = os.path.join(HERE, "disc_bench")
OBJDIR = os.path.join(HERE, "_build")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
FLAGS = [
    "--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-Wall",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + INCLUDE, "-I" + CSRC,
]


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))


def _link_driver():
    """Native driver of the C ABI (disc_bench), linked against libdisc.so."""
    src = os.path.join(CSRC, "disc_bench_main.cpp")
    tmp = BENCH_EXE + ".tmp"
    cmd = [HIPCC, "-O2", "-std=c++17", "-I" + INCLUDE, src, "-o", tmp, "-L" + HERE, "-ldisc",
           "-Wl,-rpath,$ORIGIN"]
    p = subprocess.run(cmd, capture_output=True, text=True)
    if p.returncode != 0:
        raise RuntimeError("driver build failed:\n" + p.stdout + p.stderr)
    os.replace(tmp, BENCH_EXE)


def _compile(src):
    obj = os.path.join(OBJDIR, os.path.basename(src)[:-4] + ".o")
    cmd = [HIPCC] + FLAGS + ["-c", src, "-o", obj]
    p = subprocess.run(cmd, capture_output=True, text=True)
    # hipcc's host pass does not know the device-only feature name; that note is harmless
    msgs = [l for l in (p.stdout + p.stderr).splitlines() if "packed-fp32-ops" not in l]
    if p.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s" % (src, "\n".join(msgs)))
    return obj, [m for m in msgs if "warning" in m]


def build(verbose=False):
    """Compile every HIP source for gfx950 and link libdisc.so. Returns its path."""
    os.makedirs(OBJDIR, exist_ok=True)
    srcs = sources()
    with concurrent.futures.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        results = list(ex.map(_compile, srcs))
    objs = [o for o, _ in results]
    for _, warns in results:
        for w in warns:
            if verbose:
                print(w)
    tmp = OUT + ".tmp"
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs
    p = subprocess.run(cmd, capture_output=True, text=True)
    if p.returncode != 0:
        raise RuntimeError("link failed:\n" + p.stdout + p.stderr)
    os.replace(tmp, OUT)
    _link_driver()
    return OUT


if __name__ == "__main__":
    print(build(verbose=True))
