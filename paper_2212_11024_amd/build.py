"""Build the HIP library libflame.so in-tree for gfx950 with hipcc.

Usage: python -m paper_2212_11024_amd.build   (or call build()).
"""

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libflame.so")
SOURCES = ["flame_step.hip", "flame_api.hip", "flame_adjoint.hip", "flame_lattice.hip"]
ARCH = os.environ.get("FLAME_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False, out: str = LIB, defines=()) -> str:
    """Compile libflame.so (to ``out``); ``defines`` are extra -D tuning macros."""
    objs = []
    common = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
              # packed FP32 instructions stay off: hipcc must not emit v_pk_* FP32 forms
              "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
              "-munsafe-fp-atomics", "-Wno-unused-command-line-argument", *[f"-D{d}" for d in defines]]
    procs = []
    for src in SOURCES:          # the translation units compile in parallel
        obj = os.path.join(CSRC, os.path.splitext(src)[0] + f".{os.getpid()}.o")
        cmd = [hipcc(), *common, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((subprocess.Popen(cmd), cmd))
        objs.append(obj)
    failed = [cmd for proc, cmd in procs if proc.wait() != 0]
    if failed:
        for o in objs:
            if os.path.exists(o):
                os.remove(o)
        raise subprocess.CalledProcessError(1, failed[0])
    tmp = out + ".tmp"
    cmd = [hipcc(), "-shared", f"--offload-arch={ARCH}", "-fPIC", *objs, "-o", tmp,
           "-L/opt/rocm/lib", "-lhipfft", "-Wl,-rpath,/opt/rocm/lib"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    for o in objs:
        os.remove(o)
    return out


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
