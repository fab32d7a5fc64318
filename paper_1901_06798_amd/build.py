"""Build step of the HIP library (hipcc, gfx950) -- run on the host, before use."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
# (source, contracted multiply-adds): the FP32 surface-deviation kernels
# are instantiated in units of their own and built with -ffp-contract=fast
# (that path is held to its surface bar in metres against FP64, so a fused
# multiply-add is as good as a product and a sum; its step issues about 7 %
# fewer VALU instructions); everything else rounds every product and sum as
# written (-ffp-contract=off), so that the FP64 step performs the reference
# solver's operations and a cell's result does not depend on the tile or
# launch that computed it.
SOURCES = [("swe_step.hip", False), ("swe_step_f32.hip", True), ("swe_batched.hip", False),
           ("swe_batched_f32.hip", True), ("swe_amr.hip", False)]
OUT = os.path.join(HERE, "libswe.so")

# -packed-fp32-ops: keep the compiler from emitting packed FP32 instructions.
# -structurizecfg-skip-uniform-regions: branches whose condition is the same
# for the whole wave (the row loop's quiet-edge skips, the task bounds) stay
# scalar branches instead of exec-masked regions; the FP64 step launch is 3 %
# faster (0.368 against 0.379-0.381 ms on the 4096^2 shelf), the arithmetic
# is unchanged.
HIPFLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-mllvm", "-structurizecfg-skip-uniform-regions=1",
            "-Wall", "-Wno-unused-function"]
CONTRACT_FLAG = "-ffp-contract=fast"


def flags_for(contract: bool) -> list[str]:
    return [CONTRACT_FLAG if (contract and f == "-ffp-contract=off") else f for f in HIPFLAGS]


def build(verbose: bool = False) -> str:
    import tempfile
    hipcc = "/opt/rocm/bin/hipcc"
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    noise = "packed-fp32-ops"
    with tempfile.TemporaryDirectory(prefix="swe_build_") as tmp:
        procs, objs = [], []
        for name, contract in SOURCES:
            obj = os.path.join(tmp, name + ".o")
            cmd = [hipcc] + flags_for(contract) + inc + ["-c", os.path.join(CSRC, name), "-o", obj]
            if verbose:
                print(" ".join(cmd), flush=True)
            procs.append((name, subprocess.Popen(cmd, stdout=subprocess.PIPE,
                                                 stderr=subprocess.PIPE, text=True)))
            objs.append(obj)
        failed = []
        for name, pr in procs:
            _, stderr = pr.communicate()
            err = "\n".join(l for l in stderr.splitlines() if noise not in l)
            if pr.returncode != 0:
                failed.append(f"{name} ({pr.returncode}):\n{err}")
            elif verbose and err.strip():
                print(err, file=sys.stderr)
        if failed:
            raise RuntimeError("hipcc failed: " + "\n".join(failed))
        cmd = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC"] + objs + ["-o", OUT + ".tmp"]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc link failed ({r.returncode}):\n{r.stderr}")
    os.replace(OUT + ".tmp", OUT)
    return OUT

if __name__ == "__main__":
    print(build(verbose=True))
