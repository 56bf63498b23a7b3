"""Host-link calibration on the GPU (the toy zero-copy copy study, Sec. 3.3)."""
import pytest

pytestmark = pytest.mark.gpu


def test_calibration_profile(gpu_device):
    import paper_2006_06890_amd as E
    p = E.emogi.calibrate_link(256 << 20)
    print(p, flush=True)
    assert p["memcpy_GBps"] > 1.0
    assert all(v > 0.5 for v in p["seq_read_GBps"].values())
    R = p["request_unit"]
    assert R >= 32 and R <= 4096 and (R & (R - 1)) == 0
    assert 0.05 < p["latency_us"] < 100
    # merged + aligned beats a 32-byte shift at the request unit (Fig. 4 (b) vs (c))
    assert p["rand_aligned_GBps"][R] >= p["rand_shift32_GBps"][R] * 0.95


def test_calibration_rejects_small_buffer(gpu_device):
    import paper_2006_06890_amd as E
    with pytest.raises(E.EmogiError) as ei:
        E.emogi.calibrate_link(1 << 20)
    assert ei.value.code == -1
