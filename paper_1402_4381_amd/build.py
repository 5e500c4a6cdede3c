"""Build the gfx950 shared library ``liblalm.so`` in-tree with hipcc.

Every HIP source is compiled for ``--offload-arch=gfx950`` with packed-FP32
instruction selection disabled, then linked into one shared library next to
this file.  Run ``python -m paper_1402_4381_amd.build``.
"""
import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
OUT = os.path.join(HERE, "liblalm.so")
BUILD_DIR = os.path.join(HERE, "_build")
SOURCES = ["plan.hip", "project.hip", "backproject.hip", "reduce.hip", "api.hip", "unet.hip", "fbp.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-fPIC", "-std=c++17",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", INCLUDE, "-I", CSRC,
    "-Wall", "-Wno-unused-function", "-fvisibility=hidden",
]


def _compile(src):
    obj = os.path.join(BUILD_DIR, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC] + FLAGS + ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    # the host pass does not know the packed-fp32 feature: harmless warning
    lines = [l for l in r.stdout.splitlines() if "packed-fp32-ops" not in l]
    return src, r.returncode, "\n".join(lines), obj


def build(verbose=False):
    os.makedirs(BUILD_DIR, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        results = list(ex.map(_compile, SOURCES))
    objs = []
    for src, rc, out, obj in results:
        if out.strip() and (verbose or rc != 0):
            print("[%s]\n%s" % (src, out), file=sys.stderr)
        if rc != 0:
            raise RuntimeError("hipcc failed on %s" % src)
        objs.append(obj)
    tmp = OUT + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        print(r.stdout, file=sys.stderr)
        raise RuntimeError("link failed")
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
