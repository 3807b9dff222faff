"""Build libdg.so (HIP, gfx950) in place with hipcc.

    python paper_1710_03887_amd/build.py

Every HIP source is compiled with packed-FP32 instruction generation
disabled; the library is written next to this file.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
SOURCES = ["setup.cpp", "abi.cpp", "batch_abi.cpp", "autotune.cpp", "mlp_abi.cpp", "kernels.hip", "curved.hip",
           "spec_stage.hip", "batch.hip", "mlp.hip", "probes.hip", "quad.hip"]
LIB = os.path.join(HERE, "libdg.so")
ARCH = os.environ.get("DG_OFFLOAD_ARCH", "gfx950")


def hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if cand and (os.path.sep not in cand or os.path.exists(cand)):
            return cand
    raise RuntimeError("hipcc not found")


FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         # FP32 division and square root from the hardware reciprocal and
         # square-root instructions (1 ulp) instead of correctly rounded
         # multi-instruction expansions
         "-fno-hip-fp32-correctly-rounded-divide-sqrt",
         "-Wall", "-Wno-unused-function"]


def build(verbose=False):
    objs = []
    flags = FLAGS
    os.makedirs(os.path.join(HERE, "_build"), exist_ok=True)
    for src in SOURCES:
        obj = os.path.join(HERE, "_build", src + ".o")
        cmd = [hipcc(), *flags, "-c", os.path.join(CSRC, src), "-o", obj]
        if src.endswith(".cpp"):
            cmd.insert(1, "-x")
            cmd.insert(2, "hip")
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            sys.stderr.write(r.stdout + r.stderr)
            raise RuntimeError(f"compiling {src} failed")
        if verbose:
            sys.stderr.write("".join(l + "\n" for l in r.stderr.splitlines()
                                     if "packed-fp32-ops" not in l and "warnings generated" not in l))
        objs.append(obj)
    tmp = LIB + ".tmp"
    r = subprocess.run([hipcc(), "-shared", f"--offload-arch={ARCH}", *objs, "-o", tmp],
                       capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("linking libdg.so failed")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
