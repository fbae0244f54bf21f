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


def test_chain_probe_more_chains_issue_faster():
    """At one wave per SIMD, sixteen independent chains issue faster than one
    (a lone dependent chain waits for each result)."""
    one = mpx.probe_chains(1, 1, iters=1 << 10, reps=3, warmup=1)
    many = mpx.probe_chains(16, 1, iters=1 << 8, reps=3, warmup=1)
    assert 1e12 < one < many < 2e14, (one, many)
