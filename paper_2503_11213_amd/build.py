"""Build libsdirt.so (HIP for gfx950) in-tree with hipcc.

    python -m paper_2503_11213_amd.build

Every HIP source is compiled for gfx950 only, with packed-FP32 instruction
selection disabled (-target-feature -packed-fp32-ops); the host C++ parts
go through the same driver.  The shared library lands next to this file.
"""

import os
import shutil
import subprocess
import sys
import concurrent.futures as cf

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libsdirt.so")

HIP_SOURCES = ["trace.hip", "trace_bwd.hip", "render.hip", "mlp.hip", "mlp_fused.hip", "calib.hip"]
CPP_SOURCES = ["host_optics.cpp", "pack.cpp", "api.cpp"]

COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
          "-I" + os.path.join(HERE, "..", "include")]
HIP_FLAGS = ["-x", "hip", "--offload-arch=gfx950", "-munsafe-fp-atomics",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _compile(args):
    src, obj, is_hip = args
    cmd = [hipcc()] + COMMON + (HIP_FLAGS if is_hip else []) + ["-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    return src, r.returncode, r.stdout + r.stderr


def build(verbose=False):
    os.makedirs(OBJ, exist_ok=True)
    jobs = []
    for s in HIP_SOURCES:
        if os.path.exists(os.path.join(CSRC, s)):
            jobs.append((os.path.join(CSRC, s), os.path.join(OBJ, s + ".o"), True))
    for s in CPP_SOURCES:
        jobs.append((os.path.join(CSRC, s), os.path.join(OBJ, s + ".o"), False))
    with cf.ThreadPoolExecutor(max_workers=min(8, len(jobs))) as ex:
        results = list(ex.map(_compile, jobs))
    failed = False
    for src, rc, log in results:
        if rc != 0:
            failed = True
            sys.stderr.write("compile failed: %s\n%s\n" % (src, log))
        elif verbose and log.strip():
            sys.stderr.write(log)
    if failed:
        raise RuntimeError("HIP build failed")
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp] + \
        [j[1] for j in jobs] + ["-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx",
                                "-Wl,-rpath,/opt/rocm/lib"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stdout + r.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
