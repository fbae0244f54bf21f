"""Loader of the values the paper prints (text fixtures under tests/golden/,
each citing its source in its header)."""
import os

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _rows(name):
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.split("#", 1)[0].strip()
            if line:
                yield line.split()


def bf_operation_counts():
    """{(K, op): (add, sub, mul, fma)} of the branch-free operations."""
    return {(int(k), op): tuple(int(v) for v in rest) for k, op, *rest in _rows("bf_operation_counts.txt")}


def gemm_digits(kind):
    """{K: digits} for kind "real" or "complex"."""
    return {int(k): float(d) for kd, k, d in _rows("gemm_digits.txt") if kd == kind}
