"""Build the FP64 oracle's shared library with gcc (test infrastructure).

Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg may use
anything under oracle/.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ppf_oracle.c")
LIB = os.path.join(HERE, "_liboracle.so")


def build(verbose: bool = False, sanitize: bool = False) -> str:
    """Compile ppf_oracle.c into oracle/_liboracle.so (always recompiles);
    sanitize=True builds it with AddressSanitizer and UBSan."""
    tmp = LIB + ".tmp"
    # -ffp-contract=off: no fused multiply-add, so every operation rounds as written.
    # -fopenmp: the per-particle loops may use several host threads (same results).
    cmd = ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-ffp-contract=off", "-fopenmp", "-fPIC",
           "-shared", "-Wall", "-Wextra"]
    if sanitize:
        # address and undefined-behaviour checks of the host code; a Python
        # process loads this build only with libasan and libubsan preloaded
        # (LD_PRELOAD) and ASAN_OPTIONS=detect_leaks=0
        cmd += ["-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                "-fno-sanitize-recover=undefined"]
    cmd += ["-o", tmp, SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, sanitize="--sanitize" in sys.argv))
