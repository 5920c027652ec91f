"""GPU: the atomicMin measurement entry point runs, reports a rate, lowers the slots it touches and
rejects bad arguments."""
import ctypes

import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    from paper_1903_12085_amd import binding
    binding.load()
    return binding


def test_atomic_min_measurement(B):
    import torch
    for slots, blocks, iters in ((1 << 20, 256, 16), (32, 8, 8), (1, 2, 4)):
        rate = B.measure_atomic_min(slots, blocks, iters)
        assert rate > 1e6, (slots, rate)
    buf = torch.full((64,), -1, dtype=torch.int64, device="cuda")
    ms = ctypes.c_float(0)
    B._check(B.load().sssp_measure_atomic_min(ctypes.c_void_p(buf.data_ptr()), 64, 4, 8, None, ctypes.byref(ms)))
    torch.cuda.synchronize()
    assert (buf != -1).sum().item() > 0 and ms.value > 0   # some slots lowered below all-ones
    for slots, blocks, iters in ((48, 4, 4), (64, 0, 4), (64, 4, 0)):
        with pytest.raises(B.SsspError):
            B._check(B.load().sssp_measure_atomic_min(ctypes.c_void_p(buf.data_ptr()), slots, blocks, iters, None,
                                                      ctypes.byref(ms)))
