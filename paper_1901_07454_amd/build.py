"""Build the HIP library libarbmi.so in-tree (hipcc, gfx950)."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libarbmi.so")
SOURCES = ["kernels.hip", "reg_kernels.hip", "reg_adjoint_kernels.hip", "adjoint_kernels.hip", "arbmi.cpp", "lower.cpp",
           "plan.cpp", "adjoint.cpp", "autotune.cpp", "noalloc.hip", "var_kernels.hip"]
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
         # packed FP32 instructions are kept out of every kernel
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
# The register-resident kernel holds its branches' coefficients in VGPRs for
# a whole launch; hoisting the FP64 exp/expm1 polynomial constants out of the
# step loop (machine LICM) would pin another ~40 VGPRs and cost occupancy.
EXTRA = {"reg_kernels.hip": ["-mllvm", "-disable-machine-licm"],
         "reg_adjoint_kernels.hip": ["-mllvm", "-disable-machine-licm"],
         "var_kernels.hip": ["-mllvm", "-disable-machine-licm"]}


def build(verbose: bool = False) -> str:
    from concurrent.futures import ThreadPoolExecutor
    sys.path.insert(0, HERE)
    import mechgen
    mechgen.generate()  # csrc/gen/*.hpp from mechanisms/*.mech
    os.makedirs(os.path.join(HERE, "_build"), exist_ok=True)
    jobs = []
    for src in SOURCES:
        path = os.path.join(CSRC, src)
        if not os.path.exists(path):
            continue
        obj = os.path.join(HERE, "_build", src.replace(".", "_") + ".o")
        jobs.append((src, ["hipcc", *FLAGS, *EXTRA.get(src, []), "-c", path, "-o", obj], obj))

    def run(job):
        src, cmd, _ = job
        return src, cmd, subprocess.run(cmd, capture_output=True, text=True)

    with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        results = list(ex.map(run, jobs))
    for src, cmd, r in results:
        if r.returncode != 0:
            sys.stderr.write(r.stderr)
            raise RuntimeError(f"hipcc failed on {src}")
        if verbose:
            sys.stderr.write(" ".join(cmd) + "\n")
    objs = [obj for _, _, obj in jobs]
    tmp = LIB + ".tmp"
    r = subprocess.run(["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs],
                       capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stderr)
        raise RuntimeError("link failed")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
