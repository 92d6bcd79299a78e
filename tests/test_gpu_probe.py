"""The gather-rate probe (louvain_probe_gather), the measured ceiling that bench.py sets the
move and merge kernels against: it runs through the C-ABI, returns a plausible rate for every
slicing, and rejects bad arguments. (Rates are hardware measurements, so only their range is
checked here.)"""

import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lv(gpu_device):
    from paper_2301_12390_amd import Louvain, build as B
    if not __import__("os").path.exists(B.LIB):
        B.build()
    ctx = Louvain(0)
    yield ctx
    ctx.close()


@pytest.mark.parametrize("slices", [1, 8, 64])
def test_probe_rates(lv, slices):
    # 4.2M threads x 64 gathers: anything below 10^9/s or above 10^13/s would be a broken timer
    for mib in (1, 64):
        rate = lv.probe_gather(mib << 20, slices)
        assert 1e9 < rate < 1e13, (mib, slices, rate)
    # a table smaller than its slice count in ints is rejected, one exactly that size works
    assert lv.probe_gather(4 * slices, slices) > 0


def test_probe_errors(lv):
    from paper_2301_12390_amd import LouvainError
    for table, slices in ((1 << 20, 0), (1 << 20, 65), (0, 1), (12, 4)):
        with pytest.raises(LouvainError, match="EINVAL"):
            lv.probe_gather(table, slices)
