"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

* The oracle's pins (every tests/test_oracle_*.py) against an ASan/UBSan
  build of the oracle (gcc), with gcc's ASan runtime preloaded.
* The library's host code -- argument checks, workspace sizes, the tune
  cache, the plan constructors' schedule builders -- through the ABI tests
  (tests/test_abi.py, tests/test_tune_cache.py) against the host-sanitised
  build of libmpx that the library build makes beside the product, with the
  compiler's ASan runtime preloaded.  Without a GPU every device call fails
  cleanly, so only host paths run.

Each set runs in a child process; a failing test or any sanitizer report
fails this test."""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(env_extra, tests):
    env = dict(os.environ)
    env.update(env_extra)
    env["ASAN_OPTIONS"] = "detect_leaks=0:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    env.pop("MPX_TUNE_CACHE", None)
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        "-m", "not gpu", *tests], cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=1200)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-6000:]
    assert "ERROR: AddressSanitizer" not in out and "runtime error:" not in out, out[-6000:]
    return out


def test_oracle_pins_under_asan(tmp_path):
    from oracle import build as ob
    lib = ob.build_asan(str(tmp_path / "liboracle_asan.so"))
    rt = subprocess.check_output(["gcc", "-print-file-name=libasan.so"], text=True).strip()
    assert os.path.isabs(rt), rt
    tests = sorted(glob.glob(os.path.join(ROOT, "tests", "test_oracle_*.py")))
    assert len(tests) >= 7
    out = _run({"LD_PRELOAD": rt, "MPX_ORACLE_LIBRARY": lib}, tests)
    assert " passed" in out


def _asan_lib_fresh(lib):
    from paper_2603_14926_amd import build as b
    if not os.path.exists(lib):
        return False
    srcs = b.sources() + glob.glob(os.path.join(b.CSRC, "*.hpp")) + \
        glob.glob(os.path.join(ROOT, "include", "*.h"))
    return os.path.getmtime(lib) >= max(os.path.getmtime(s) for s in srcs)


def test_host_code_under_asan():
    from paper_2603_14926_amd import build as b
    if not _asan_lib_fresh(b.ASAN_LIB):
        b.build()   # the product library and its host-sanitised variant
    rt = "/opt/rocm/llvm/lib/clang"
    cand = sorted(glob.glob(os.path.join(rt, "*", "lib", "linux", "libclang_rt.asan-x86_64.so")))
    if not cand:
        pytest.skip("no clang ASan runtime in this image")
    out = _run({"LD_PRELOAD": cand[-1], "MPX_LIBRARY": b.ASAN_LIB},
               [os.path.join(ROOT, "tests", "test_abi.py"), os.path.join(ROOT, "tests", "test_tune_cache.py")])
    assert " passed" in out
