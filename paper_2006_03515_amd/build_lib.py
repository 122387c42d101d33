"""Build libkifmm.so for gfx950 with hipcc (in-tree).

    python -m paper_2006_03515_amd.build_lib [-j N]

Each .hip source is compiled to an object in _build/ (parallel), then linked
into paper_2006_03515_amd/libkifmm.so.  Packed FP32 instructions are disabled
for the device code.
"""
import concurrent.futures
import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libkifmm.so")
BUILD = os.path.join(ROOT, "_build")
ARCH = os.environ.get("KIFMM_ARCH", "gfx950")

FLAGS = ["-O3", "-fPIC", "-std=c++17", "--offload-arch=" + ARCH,
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function", "-I", os.path.join(ROOT, "include")]


def _compile(src):
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = ["hipcc", "-c", src, "-o", obj] + FLAGS
    r = subprocess.run(cmd, capture_output=True, text=True)
    msg = "\n".join(l for l in (r.stdout + r.stderr).splitlines()
                    if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed on %s:\n%s" % (src, msg))
    return obj, msg


def build(jobs=8, verbose=False):
    os.makedirs(BUILD, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    with concurrent.futures.ThreadPoolExecutor(max_workers=jobs) as ex:
        res = list(ex.map(_compile, srcs))
    for obj, msg in res:
        if verbose and msg.strip():
            print(msg)
    objs = [o for o, _ in res]
    tmp = OUT + ".tmp"
    subprocess.check_call(["hipcc", "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp] + objs)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    j = 8
    if "-j" in sys.argv:
        j = int(sys.argv[sys.argv.index("-j") + 1])
    print(build(jobs=j, verbose=True))
