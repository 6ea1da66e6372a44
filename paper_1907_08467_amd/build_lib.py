"""Build libvcs355.so (the HIP library) for gfx950 with hipcc."""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "csrc")
OUT_DIR = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libvcs355.so")
SOURCES = ["interp.hip", "render.hip", "envops.hip", "stack.hip", "policy.hip", "api.hip"]
# Control flow that the compiler can prove wave-uniform (the interpreter's
# scalar loop) is left as plain scalar branches instead of being rewritten into
# the structured form divergent code needs, which would add a copy of every
# live value at each merge point.
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Wall",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-mllvm", "-structurizecfg-skip-uniform-regions=true",
         "-I", os.path.join(ROOT, "include")]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    msgs = "\n".join(l for l in (r.stdout + r.stderr).splitlines()
                     if "packed-fp32-ops" not in l and "not a recognized feature" not in l)
    return r.returncode, msgs


def build(verbose=False):
    os.makedirs(OUT_DIR, exist_ok=True)
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    objs = [os.path.join(OUT_DIR, s.replace(".hip", ".o")) for s in SOURCES]
    jobs = [[hipcc] + FLAGS + ["-c", os.path.join(SRC, s), "-o", o] for s, o in zip(SOURCES, objs)]
    with ThreadPoolExecutor(max_workers=len(jobs)) as ex:
        results = list(ex.map(_run, jobs))
    for (rc, msg), src in zip(results, SOURCES):
        if rc != 0:
            sys.stderr.write(msg + "\n")
            raise RuntimeError(f"hipcc failed on {src}")
        if verbose and msg.strip():
            sys.stderr.write(msg + "\n")
    tmp = LIB + ".tmp"
    rc, msg = _run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs)
    if rc != 0:
        sys.stderr.write(msg + "\n")
        raise RuntimeError("link of libvcs355.so failed")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
