"""The product path has no CPU fallback: without libmpx.so every call raises,
and no module of the package imports the CPU oracle."""
import os
import re
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2603_14926_amd")


def test_missing_library_raises_on_every_entry():
    code = r"""
import sys
sys.path.insert(0, %r)
from paper_2603_14926_amd import mpx
mpx.LIB_PATH = "/nonexistent/libmpx.so"
import torch
x = torch.zeros((4, 8), dtype=torch.float64)
for call in (lambda: mpx.lib(), lambda: mpx.add("qd", x, x), lambda: mpx.dot("qd", x, x),
             lambda: mpx.gemm("qd", x.view(4, 2, 4), x.view(4, 4, 2))):
    try:
        call()
    except mpx.MpxError:
        continue
    except Exception as e:       # a CPU tensor must not be accepted either
        if "GPU" in str(e):
            continue
        raise
    raise SystemExit("a call returned without the library")
print("ok")
""" % ROOT
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), r.stdout + r.stderr


def test_package_does_not_import_the_oracle():
    for name in os.listdir(PKG):
        if name.endswith(".py"):
            src = open(os.path.join(PKG, name)).read()
            assert not re.search(r"^\s*(from|import)\s+oracle\b", src, re.M), name
            assert "liboracle" not in src, name
