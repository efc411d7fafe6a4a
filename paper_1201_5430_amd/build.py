"""Build liblhfmm.so (HIP, gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "liblhfmm.so")
SOURCES = ["lhf_plan.hip", "lhf_eval.hip", "lhf_m2l.hip", "lhf_m2l_half.hip", "lhf_m2l_quarter.hip",
           "lhf_m2l_mfma.hip", "lhf_batch.hip", "lhf_filament.hip"]
ARCH = os.environ.get("LHF_OFFLOAD_ARCH", "gfx950")

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared", f"--offload-arch={ARCH}",
    # no packed-FP32 instructions in any device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


# per-source additions: the half-vector M2L's fully unrolled FP32 p = 16 body exceeds the
# default size limit of '#pragma unroll' (a partly rolled loop would move its vectors to scratch)
EXTRA = {"lhf_m2l_half.hip": ["-mllvm", "-pragma-unroll-threshold=200000"],
         "lhf_m2l_quarter.hip": ["-mllvm", "-pragma-unroll-threshold=200000"]}


def _stale(obj: str, src: str) -> bool:
    """True if obj is missing or older than its source or any header of csrc/ or include/."""
    if not os.path.exists(obj):
        return True
    t = os.path.getmtime(obj)
    inc = os.path.join(os.path.dirname(HERE), "include")
    deps = [src] + [os.path.join(CSRC, h) for h in os.listdir(CSRC) if h.endswith((".h", ".inc"))]
    deps += [os.path.join(inc, h) for h in os.listdir(inc) if h.endswith(".h")]
    return any(os.path.getmtime(d) > t for d in deps)


def build(verbose: bool = False, jobs: int = 0, incremental: bool = False) -> str:
    """Compile every source (in parallel, at most ``jobs`` at once) and link liblhfmm.so.

    incremental=True recompiles only the sources whose object is older than the source or a header.
    """
    from concurrent.futures import ThreadPoolExecutor
    objs, cmds = [], []
    for src in SOURCES:
        obj = os.path.join(CSRC, src.replace(".hip", ".o"))
        objs.append(obj)
        if incremental and not _stale(obj, os.path.join(CSRC, src)):
            continue
        cmds.append(["hipcc", "-c", *[f for f in FLAGS if f != "-shared"], *EXTRA.get(src, []), "-o", obj,
                     os.path.join(CSRC, src)])

    def run(cmd):
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)

    jobs = jobs or max(1, min(len(cmds), 8, os.cpu_count() or 1))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        for f in [ex.submit(run, c) for c in cmds]:
            f.result()
    tmp = LIB + ".tmp"
    cmd = ["hipcc", "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, incremental="-i" in sys.argv))
