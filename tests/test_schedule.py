"""The library's host-side combine schedule (Algorithm 6, appendix A) equals the
oracle's padded power-of-two tree for every K up to 600 and a few large K
(CPU only: dsmc_schedule does no device work)."""
import pytest

from oracle import dsmc as D


@pytest.mark.parametrize("Ks", [range(1, 601), [1023, 1024, 1025, 4095, 4096, 4097, 8191, 16384]])
def test_schedule_equals_oracle(Ks):
    from paper_2202_02264_amd import dsmc as G
    for K in Ks:
        assert G.dsmc_schedule(K) == [lv for lv in D.schedule(K)], K


def test_schedule_structure():
    """Every time point is a boundary exactly once, blocks are contiguous and
    ragged K has ceil(log2 K) levels."""
    from paper_2202_02264_amd import dsmc as G
    for K in (2, 3, 5, 37, 300, 4097):
        levels = G.dsmc_schedule(K)
        cs = sorted(c for lv in levels for (_, c, _) in lv)
        assert cs == list(range(1, K))
        assert len(levels) == (K - 1).bit_length()
        for lv in levels:
            for a, c, b in lv:
                assert 0 <= a < c < b <= K


def test_schedule_rejects_bad_arguments():
    import ctypes as C
    from paper_2202_02264_amd import dsmc as G
    assert G._lib.dsmc_schedule(0, 0, None, None, None, None) == G.DSMC_EINVAL
    assert G._lib.dsmc_schedule(10, 3, None, None, None, None) == G.DSMC_EINVAL
    assert G._lib.dsmc_schedule(1, 0, None, None, None, None) == 0
