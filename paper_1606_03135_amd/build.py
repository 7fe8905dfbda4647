"""Build liborbf.so (HIP, gfx950) in-tree from paper_1606_03135_amd/csrc."""
import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "liborbf.so")
SOURCES = ["api.hip", "scan.hip", "knn.hip", "cover.hip", "weights.hip",
           "weights_reg.hip", "weights_reg_3_6.hip", "weights_reg_7_8.hip",
           "weights_reg_9.hip", "weights_ir.hip", "weights_wg.hip",
           "weights_mfma.hip",
           "lebesgue.hip", "csr.hip", "gershgorin.hip", "krylov.hip", "ilu.hip",
           "batch.hip", "peak.hip"]
ARCH = os.environ.get("ORBF_OFFLOAD_ARCH", "gfx950")
FLAGS = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=" + ARCH,
         "-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
         # no packed FP32 instructions anywhere in this library
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function", "-Wno-unused-result",
         "-Wno-unused-value"]


def _compile(src):
    obj = os.path.join(OBJ, os.path.splitext(src)[0] + ".o")
    cmd = ["hipcc", "-c"] + FLAGS + [os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s%s" % (src, r.stdout,
                                                          r.stderr))
    return obj, r.stderr


def build(verbose=False, jobs=8):
    os.makedirs(OBJ, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        results = list(ex.map(_compile, SOURCES))
    objs = [o for o, _ in results]
    if verbose:
        for o, err in results:
            warn = [l for l in err.splitlines()
                    if "packed-fp32-ops" not in l and l.strip()]
            if warn:
                print("\n".join(warn))
    tmp = LIB + ".tmp"
    cmd = ["hipcc", "-shared", "--offload-arch=" + ARCH, "-o", tmp] + objs
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
    sys.exit(0)
