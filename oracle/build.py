"""Build the CPU oracle shared libraries (test infrastructure only).

liboracle.so       -- the oracle, OpenMP over independent outputs only.
liboracle_count.so -- the same source with every floating-point operation
                      counted by kind (used to check Tables 1 and 2).

Flags: -ffp-contract=off keeps a*b+c unfused (the only fused operation is the
explicit fma() of TwoProd); -fno-fast-math keeps IEEE semantics; x86-64 SSE2
arithmetic rounds to nearest even.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "mpx_oracle.c")
FLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared", "-std=c11",
         "-D_GNU_SOURCE", "-Wall", "-Wno-unused-function", "-Wno-unknown-pragmas"]


def build(verbose: bool = False) -> None:
    outs = [
        (os.path.join(HERE, "liboracle.so"), ["-fopenmp"]),
        (os.path.join(HERE, "liboracle_count.so"), ["-DMPXO_COUNT"]),
    ]
    for out, extra in outs:
        cmd = ["gcc", *FLAGS, *extra, SRC, "-o", out + ".tmp", "-lm"]
        if verbose:
            print(" ".join(cmd))
        subprocess.check_call(cmd)
        os.replace(out + ".tmp", out)


def build_asan(out: str) -> str:
    """The oracle with AddressSanitizer and UndefinedBehaviorSanitizer (for
    the CPU tests; load it with libasan preloaded)."""
    cmd = ["gcc", *FLAGS, "-fopenmp", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
           "-g", SRC, "-o", out, "-lm"]
    subprocess.check_call(cmd)
    return out


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
