"""Build the C oracle and the rocRAND Philox reference.  TEST INFRASTRUCTURE ONLY."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ORACLE_SO = os.path.join(HERE, "libee_oracle.so")
ROCRAND_REF_SO = os.path.join(HERE, "libphilox_rocrand_ref.so")


def build_oracle(verbose: bool = False) -> str:
    # -ffp-contract=off and no fast-math: the thresholds are FP64 libm exp,
    # evaluated exactly as written.
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math",
           "-Wall", "-Wextra", os.path.join(HERE, "ee_oracle.c"), "-o", ORACLE_SO + ".tmp", "-lm"]
    subprocess.run(cmd, check=True, capture_output=not verbose)
    os.replace(ORACLE_SO + ".tmp", ORACLE_SO)
    return ORACLE_SO


def build_rocrand_ref(verbose: bool = False) -> str | None:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    if not os.path.exists(hipcc):
        return None
    cmd = [hipcc, "-O2", "-fPIC", "-shared", "-x", "hip", "--offload-arch=gfx950",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           os.path.join(HERE, "philox_rocrand_ref.hip"), "-o", ROCRAND_REF_SO + ".tmp"]
    subprocess.run(cmd, check=True, capture_output=not verbose)
    os.replace(ROCRAND_REF_SO + ".tmp", ROCRAND_REF_SO)
    return ROCRAND_REF_SO


def build_all(verbose: bool = False) -> None:
    build_oracle(verbose)
    build_rocrand_ref(verbose)


if __name__ == "__main__":
    build_all(verbose="-v" in sys.argv)
    print("built", ORACLE_SO, ROCRAND_REF_SO)
