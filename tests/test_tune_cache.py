"""The persistent autotune cache and its environment overrides (host logic:
which GEMM tiling and which root-solver variant a call would use).  These run
without a GPU: the device architecture then reads "unknown", so the cache
files carry lines for both that name and gfx950."""
import os

import pytest

from paper_2603_14926_amd import mpx

QD = 4
SHAPE = (2048, 2048, 2048)


def _key_line(arch, name):
    return f"{arch} gemm {QD} 0 0 11 11 11 {name}\n"


@pytest.fixture
def env(tmp_path, monkeypatch):
    for v in ("MPX_TUNE_CACHE", "MPX_TUNE", "MPX_GEMM_VARIANT", "MPX_DK_VARIANT"):
        monkeypatch.delenv(v, raising=False)
    L = mpx.lib()
    yield L, tmp_path, monkeypatch
    for v in ("MPX_TUNE_CACHE", "MPX_TUNE", "MPX_GEMM_VARIANT", "MPX_DK_VARIANT"):
        os.environ.pop(v, None)
    L.mpx_tune_reload()


def _names(L):
    return [L.mpx_gemm_variant_name(QD, v).decode() for v in range(L.mpx_gemm_variant_count(QD))]


def test_cache_file_forced_and_disabled(env):
    L, tmp, mp = env
    names = _names(L)
    default = L.mpx_gemm_selected_variant(QD, 0, 0, *SHAPE)
    assert 0 <= default < len(names)
    other = (default + 1) % len(names)
    path = tmp / "tune.txt"
    path.write_text("# a comment line is not an entry\n" + _key_line("unknown", names[other]) +
                    _key_line("gfx950", names[other]) + "gfx1100 gemm 4 0 0 11 11 11 whatever\n")
    mp.setenv("MPX_TUNE_CACHE", str(path))
    assert L.mpx_tune_reload() == 0
    assert L.mpx_gemm_selected_variant(QD, 0, 0, *SHAPE) == other          # from the file
    assert L.mpx_gemm_selected_variant(QD, 1, 0, *SHAPE) == default        # other bucket
    forced = (other + 1) % len(names)
    mp.setenv("MPX_GEMM_VARIANT", f"no_such_tiling,{names[forced]}")
    assert L.mpx_gemm_selected_variant(QD, 0, 0, *SHAPE) == forced         # forced wins
    mp.setenv("MPX_GEMM_VARIANT", "dd_4x4_k8")                             # another precision's
    assert L.mpx_gemm_selected_variant(QD, 0, 0, *SHAPE) == other
    mp.delenv("MPX_GEMM_VARIANT")
    mp.setenv("MPX_TUNE", "off")
    assert L.mpx_gemm_selected_variant(QD, 0, 0, *SHAPE) == default        # tuning ignored
    mp.delenv("MPX_TUNE")
    L.mpx_gemm_autotune_reset()                                            # forget this process's
    assert L.mpx_gemm_selected_variant(QD, 0, 0, *SHAPE) == default
    assert L.mpx_tune_reload() == 0                                        # the file again
    assert L.mpx_gemm_selected_variant(QD, 0, 0, *SHAPE) == other


def test_unknown_names_and_bad_arguments(env):
    L, tmp, mp = env
    path = tmp / "tune.txt"
    default = L.mpx_gemm_selected_variant(QD, 0, 0, *SHAPE)
    path.write_text(_key_line("unknown", "no_such_tiling") + _key_line("gfx950", "no_such_tiling"))
    mp.setenv("MPX_TUNE_CACHE", str(path))
    L.mpx_tune_reload()
    assert L.mpx_gemm_selected_variant(QD, 0, 0, *SHAPE) == default        # ignored
    assert L.mpx_gemm_selected_variant(7, 0, 0, *SHAPE) == -2
    assert L.mpx_gemm_selected_variant(QD, 2, 0, *SHAPE) == -1
    assert L.mpx_gemm_selected_variant(QD, 0, 0, 0, 5, 5) == -1
    mp.setenv("MPX_TUNE_CACHE", str(tmp / "missing.txt"))                  # no file: empty cache
    assert L.mpx_tune_reload() == 0
    assert L.mpx_gemm_selected_variant(QD, 0, 0, *SHAPE) == default
