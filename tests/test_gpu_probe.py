"""The random-read probe used for roofline reports runs and times itself."""
import pytest

from gpu_util import scc

pytestmark = pytest.mark.gpu


def test_probe_times_random_reads():
    import torch
    S = scc()
    buf = torch.zeros(1 << 23, dtype=torch.int64, device="cuda")   # 64 MiB
    for rb in (8, 64, 256):
        ms = S.probe_random_reads(buf, rb, 1 << 16, salt=rb)
        assert ms > 0
    assert S.probe_random_reads(buf, 64, 0) == 0.0
    with pytest.raises(S.SccError):
        S.probe_random_reads(buf, 48 + 4, 16)
