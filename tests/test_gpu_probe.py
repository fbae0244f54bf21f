"""The VALU issue-rate probe runs and reports plausible rates (it backs the
FP64 / FP32 peaks of the rooflines; it computes nothing of the method)."""
import pytest

torch = pytest.importorskip("torch")

from paper_2603_14926_amd import mpx

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("kind", sorted(mpx.PROBES))
def test_probe_rates_are_plausible(kind):
    r = mpx.probe_valu(kind, iters=1 << 8, reps=1)
    assert 1e12 < r < 2e14, r
