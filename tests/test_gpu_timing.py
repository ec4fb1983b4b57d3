"""Timing of the fused particle kernel (pic_timing, pic_kernel_time): HIP
events around every k-th launch on the context's stream; timing changes no
result."""
from __future__ import annotations

import pytest

from pic_inputs import build_tables
from tests.test_gpu_parity import _gpu, _same_state, _state, ragged_small

pytestmark = pytest.mark.gpu


def test_timing_stride_counts_launches_and_changes_no_result():
    from paper_0705_0495_amd import PicError
    wl = ragged_small()
    tabs = build_tables()
    a = _gpu()(wl, *tabs, precision="fp32")
    b = _gpu()(wl, *tabs, precision="fp32")
    a.timing(True, every=3)
    a.step(10)                      # launches 0, 3, 6 and 9 are timed
    ms, n = a.kernel_time()
    assert n == 4 and ms > 0
    a.timing(True)                  # every launch, counts restart
    a.step(5)
    ms, n = a.kernel_time()
    assert n == 5 and ms > 0
    a.timing(False)
    with pytest.raises(PicError):
        a.timing(True, every=-2)
    b.step(15)
    a.sync()
    b.sync()
    _same_state(_state(a), _state(b), "timed against untimed")
    a.close()
    b.close()
