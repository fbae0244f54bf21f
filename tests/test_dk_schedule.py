"""CPU checks of the host-side lane-packed Durand-Kerner schedule builder
(the library's own C++ header, compiled with g++): the schedule covers every
root exactly once inside the job that owns its polynomial, never puts a root
in an item shorter than its polynomial, orders jobs heaviest first, and keeps
the share of padded lane-steps small on the benchmark's degree mix; static
schedules put every job in exactly one workgroup's range and balance the
workgroups' totals."""
import ctypes as C
import os
import subprocess

import numpy as np
import pytest

from paper_2603_14926_amd import synth

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "native", "dk_sched_check.cpp")


@pytest.fixture(scope="module")
def lib(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("dks") / "libdks.so")
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-Wall", SRC, "-o", out])
    L = C.CDLL(out)
    L.dk_sched_check.restype = C.c_int
    L.dk_sched_check.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_double, C.c_longlong, C.c_int,
                                 C.c_void_p]
    return L


def _check(L, deg, W, lscale, slots, static=False):
    deg = np.ascontiguousarray(deg, np.int32)
    st = (C.c_double * 4)()
    r = L.dk_sched_check(deg.ctypes.data_as(C.c_void_p), deg.size, W, lscale, slots, int(static), st)
    assert r == 0, r
    return st[0], st[1], st[2], st[3]


@pytest.mark.parametrize("static", [False, True])
@pytest.mark.parametrize("W,lscale,slots", [(4, 1.5, 512), (8, 1.5, 256), (8, 2.0, 256), (12, 2.0, 256),
                                            (16, 1.0, 256), (4, 1.0, 1), (16, 1.0, 7)])
def test_schedule_invariants(lib, W, lscale, slots, static):
    rng = np.random.default_rng(W)
    for deg in ([1], [64], [65, 1, 1, 1], [512] * 3, list(range(1, 200)),
                rng.integers(1, 700, 300).tolist(), [3, 130, 7, 64, 64, 63, 129, 2]):
        _check(lib, deg, W, lscale, slots, static)


def test_schedule_padding_on_benchmark_mix(lib):
    """4096 polynomials of degrees 16..512: at least 94 % of the issued
    lane-steps are roots' own steps (a 64-root chunk per wave leaves 8 % idle)."""
    deg, *_ = synth.dk_batch(1, 4096, 16, 512, seed=synth.seed_for(2, 0), n_known=16)
    for W, ls, slots in ((4, 1.5, 512), (8, 1.5, 256), (8, 2.0, 256), (12, 2.0, 256), (16, 1.0, 256)):
        jobs, eff, bal, span = _check(lib, deg, W, ls, slots)
        assert eff >= 0.94, (W, ls, eff)


def test_static_schedule_balance_on_benchmark_mix(lib):
    """16-wave jobs on 256 workgroups over the benchmark's degree mix: the
    jobs' waves are within 1 % of even, and the static assignment brings the
    most-loaded workgroup within 2 % of an even share of all the work (the
    dynamic order, heaviest job first to the first free workgroup, leaves
    it 5 % above)."""
    deg, *_ = synth.dk_batch(1, 4096, 16, 512, seed=synth.seed_for(2, 0), n_known=16)
    _, _, bal, span_static = _check(lib, deg, 16, 1.0, 256, static=True)
    _, _, _, span_dynamic = _check(lib, deg, 16, 1.0, 256, static=False)
    assert bal >= 0.99, bal
    assert span_static <= 1.02, span_static
    assert span_dynamic > span_static, (span_dynamic, span_static)
