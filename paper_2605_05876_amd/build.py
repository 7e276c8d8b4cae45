"""Build libsurfsplat.so (HIP for gfx950) in the package directory."""
import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libsurfsplat.so")
SOURCES = ["api.hip", "preprocess.hip", "binning.hip", "raster.hip", "envmap.hip"]
ARCH = os.environ.get("SURFSPLAT_ARCH", "gfx950")


def _hipcc():
    for c in ("/opt/rocm/bin/hipcc", "hipcc"):
        if os.path.sep not in c or os.path.exists(c):
            return c
    return "hipcc"


FLAGS = ["-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC",
         # packed FP32 instructions stay off: some of their forms have given wrong
         # results on these machines
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", os.path.join(ROOT, "include"), "-I", SRC]


def build(verbose: bool = False, jobs: int = 5) -> str:
    os.makedirs(os.path.join(HERE, "_build"), exist_ok=True)
    objs = []
    cmds = []
    for s in SOURCES:
        o = os.path.join(HERE, "_build", s.replace(".hip", ".o"))
        objs.append(o)
        cmds.append([_hipcc(), *FLAGS, "-c", os.path.join(SRC, s), "-o", o])

    def run(cmd):
        if verbose:
            print(" ".join(cmd), file=sys.stderr)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
        return r.stderr
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        for err in ex.map(run, cmds):
            if verbose and err.strip():
                print(err, file=sys.stderr)
    run([_hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", LIB + ".tmp"])
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
