"""The autotuners write their choice to the tune-cache file (keeping other
GPUs' lines), and a new root-solver plan starts on the cached variant, or on
the one MPX_DK_VARIANT forces."""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2603_14926_amd import mpx, synth
from tests.gpu_util import to_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture
def cache(tmp_path, monkeypatch):
    for v in ("MPX_TUNE", "MPX_GEMM_VARIANT", "MPX_DK_VARIANT"):
        monkeypatch.delenv(v, raising=False)
    path = tmp_path / "tune.txt"
    path.write_text("gfx1100 gemm 4 0 0 6 6 6 kept_as_is\n")
    monkeypatch.setenv("MPX_TUNE_CACHE", str(path))
    L = mpx.lib()
    L.mpx_tune_reload()
    yield L, path, monkeypatch
    for v in ("MPX_TUNE_CACHE", "MPX_DK_VARIANT"):
        os.environ.pop(v, None)
    L.mpx_tune_reload()
    L.mpx_gemm_autotune_reset()


def test_gemm_autotune_writes_the_cache(cache):
    L, path, _ = cache
    A = to_gpu(synth.mp_array(4, (100, 90), 1, "U"))
    B = to_gpu(synth.mp_array(4, (90, 80), 2, "U"))
    Cm = torch.empty((4, 100, 80), dtype=torch.float64, device="cuda")
    v, _ = mpx.gemm_autotune("qd", A, B, Cm, reps=1)
    name = L.mpx_gemm_variant_name(4, v).decode()
    lines = path.read_text().splitlines()
    assert "gfx1100 gemm 4 0 0 6 6 6 kept_as_is" in lines
    mine = [l for l in lines if l.split()[1:8] == ["gemm", "4", "0", "0", "6", "6", "6"] and
            not l.startswith("gfx1100")]
    assert len(mine) == 1 and mine[0].split()[-1] == name
    L.mpx_gemm_autotune_reset()
    L.mpx_tune_reload()                                    # a later process reads it back
    assert L.mpx_gemm_selected_variant(4, 0, 0, 100, 80, 90) == v


def test_dk_plan_uses_cached_and_forced_variant(cache):
    L, path, mp = cache
    deg = np.array([17, 64, 5, 130, 40] * 4, np.int32)
    K = 4
    total = int((deg + 1).sum())
    cre, cim = to_gpu(synth.mp_array(K, total, 3, "N")), to_gpu(synth.mp_array(K, total, 4, "N"))
    zr = torch.zeros((K, int(deg.sum())), dtype=torch.float64, device="cuda")
    zi = torch.zeros_like(zr)
    mpx.RootsPlan("qd", deg, iters=0, init=True, graph=False).run(cre, cim, zr, zi)
    plan = mpx.RootsPlan("qd", deg, iters=2, init=False, graph=False)
    kept, _ = plan.autotune(cre, cim, zr, zi, iters_probe=1)
    assert plan.variant() == kept
    assert any(l.split()[1] == "dk" and l.split()[-1] == str(kept) for l in path.read_text().splitlines())
    # the cache line names a variant; rewrite it to another one and reload
    other = (kept + 1) % mpx.polyroots_variant_count()
    path.write_text("".join((" ".join(l.split()[:-1] + [str(other)]) if l.split()[1] == "dk" else l) + "\n"
                            for l in path.read_text().splitlines()))
    L.mpx_tune_reload()
    assert mpx.RootsPlan("qd", deg, iters=2, init=False, graph=False).variant() == other
    mp.setenv("MPX_DK_VARIANT", "1")
    assert mpx.RootsPlan("qd", deg, iters=2, init=False, graph=False).variant() == 1


def test_gemm_autotune_keeps_row_wave_tilings_to_small_products(cache):
    """A product with 64 x 64 tiles of 32 x 32 (4096, the limit) is not given
    to a row-wave tiling ("_rw"), which re-reads B for every few rows; the
    picked tiling still gives the same bits as the row-wave ones."""
    L, _, _ = cache
    m = n = 2048
    A = to_gpu(synth.mp_array(2, (m, 16), 5, "U"))
    B = to_gpu(synth.mp_array(2, (16, n), 6, "U"))
    Cm = torch.empty((2, m, n), dtype=torch.float64, device="cuda")
    v, _ = mpx.gemm_autotune("dd", A, B, Cm, reps=1)
    assert "_rw" not in mpx.gemm_variants("dd")[v]
    want = mpx.gemm("dd", A, B, variant=v).cpu().numpy()
    for i, name in enumerate(mpx.gemm_variants("dd")):
        if "_rw" in name:
            got = mpx.gemm("dd", A, B, variant=i).cpu().numpy()
            assert np.array_equal(got.view(np.int64), want.view(np.int64)), name
