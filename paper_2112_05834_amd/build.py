"""Build libchem.so (all HIP sources, gfx950) in-tree with hipcc."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libchem.so")
SOURCES = ["mech.cpp", "capi.cpp", "integrator.hip", "integrator_wide.hip", "model.hip", "zonal.hip",
           "rocsolver_cmp.cpp"]
ARCH = os.environ.get("CHEM_OFFLOAD_ARCH", "gfx950")

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
    "--offload-arch=" + ARCH,
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable", "-Wno-unused-value", "-Wno-unused-result",
]


def _obj(src):
    return os.path.join(CSRC, "_build", os.path.splitext(src)[0] + ".o")


def build(verbose=False, jobs=4):
    """Compile every source (always) and link libchem.so."""
    os.makedirs(os.path.join(CSRC, "_build"), exist_ok=True)
    procs = []
    for src in SOURCES:
        lang = ["-x", "hip"]
        cmd = ["hipcc"] + FLAGS + lang + ["-c", os.path.join(CSRC, src), "-o", _obj(src)]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd)))
        if len(procs) >= jobs:
            src0, p0 = procs.pop(0)
            if p0.wait() != 0:
                raise RuntimeError("hipcc failed on " + src0)
    for src0, p0 in procs:
        if p0.wait() != 0:
            raise RuntimeError("hipcc failed on " + src0)
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = ["hipcc", "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + [_obj(s) for s in SOURCES] + ["-ldl"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
