"""Build the HIP library ``libfmm_hip.so`` in-tree for gfx950.

Every ``csrc/*.hip`` and ``csrc/*.cpp`` is compiled by hipcc into
``_build/`` and linked into ``paper_1311_1006_amd/libfmm_hip.so``.  HIP code
is compiled with packed FP32 instructions disabled.
"""
import concurrent.futures as cf
import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libfmm_hip.so")
ARCH = os.environ.get("FMM_OFFLOAD_ARCH", "gfx950")

COMMON = ["-O3", "-fPIC", "-std=c++17", "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
          "-Wno-unknown-pragmas", "-Wno-pass-failed"]
HIPFLAGS = ["--offload-arch=" + ARCH, "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            ]


# geometry, split axes and the theta-criterion: every operation rounded alone
EXACT_FILES = {"tree_build.hip", "lists.hip"}
# MFMA accumulators in ordinary vector registers (no copies out of the
# accumulation registers after every product)
MFMA_VGPR_FILES = {"m2l.hip"}


def _compile(src):
    obj = os.path.join(OUT, os.path.basename(src) + ".o")
    cmd = ["hipcc", "-c", src, "-o", obj] + COMMON
    if src.endswith(".hip"):
        cmd += HIPFLAGS
    if os.path.basename(src) in EXACT_FILES:
        cmd += ["-ffp-contract=off"]
    if os.path.basename(src) in MFMA_VGPR_FILES:
        cmd += ["-mllvm", "-amdgpu-mfma-vgpr-form=1"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    # hipcc's host pass does not know the packed-fp32 target feature: harmless
    err = "\n".join(l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s" % (" ".join(cmd), err))
    return obj, err


def build(verbose=False):
    os.makedirs(OUT, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.cpp")))
    with cf.ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 4)) as ex:
        res = list(ex.map(_compile, srcs))
    for obj, err in res:
        if verbose and err.strip():
            print(err)
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = ["hipcc", "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp] + [o for o, _ in res]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed: %s\n%s" % (" ".join(cmd), r.stderr))
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
