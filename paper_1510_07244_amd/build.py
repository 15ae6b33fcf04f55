"""Build ``libbem.so`` (the C-ABI library) in-tree with hipcc for gfx950.

Every HIP translation unit is compiled with packed FP32 instructions turned
off (``-Xclang -target-feature -Xclang -packed-fp32-ops``); hipcc's host pass
warns that it does not know that feature, which is harmless.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libbem.so")
ARCH = os.environ.get("BEM_OFFLOAD_ARCH", "gfx950")

SOURCES = ["bem_blocks.hip", "bem_kernels.hip", "bem_bases.hip", "bem_mlp.hip", "bem_peak.hip",
           "bem_h2mv.hip", "bem_p1.hip",
           "bem_quadrature.cpp", "bem_capi.cpp", "bem_plan.cpp", "bem_learned.cpp",
           "bem_h2_tree.cpp", "bem_h2_host.cpp"]
OPENMP = {"bem_h2_host.cpp"}
OMP_LIB = "/opt/rocm/llvm/lib"
COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    p = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    lines = [l for l in p.stdout.splitlines() if "packed-fp32-ops" not in l]
    if lines and (verbose or p.returncode):
        print("\n".join(lines), flush=True)
    if p.returncode:
        raise RuntimeError("command failed: " + " ".join(cmd))


def build(verbose: bool = False) -> str:
    from concurrent.futures import ThreadPoolExecutor
    os.makedirs(BUILD, exist_ok=True)
    objs, cmds = [], []
    for src in SOURCES:
        obj = os.path.join(BUILD, src.rsplit(".", 1)[0] + ".o")
        cmd = ["hipcc", *COMMON, "-c", os.path.join(CSRC, src), "-o", obj]
        if src.endswith(".hip"):
            cmd[1:1] = ["-x", "hip", f"--offload-arch={ARCH}"]
        else:
            cmd[1:1] = ["-ffp-contract=off"] + (["-fopenmp"] if src in OPENMP else [])
        cmds.append(cmd)
        objs.append(obj)
    with ThreadPoolExecutor(max_workers=min(8, len(cmds))) as pool:
        list(pool.map(lambda c: _run(c, verbose), cmds))
    _run(["hipcc", "-shared", "-fPIC", f"--offload-arch={ARCH}", "-fopenmp",
          f"-Wl,-rpath,{OMP_LIB}", "-o", LIB + ".tmp", *objs], verbose)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
