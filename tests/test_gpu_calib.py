"""Host-link calibration on the GPU (the toy zero-copy copy study, Sec. 3.3)."""
import pytest

from oracle import linkmodel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def profile(gpu_device):
    import paper_2006_06890_amd as E
    p = E.emogi.calibrate_link(256 << 20)
    print(p, flush=True)
    return p


def test_calibration_profile(profile):
    p = profile
    assert p["memcpy_GBps"] > 1.0
    assert all(v > 0.5 for v in p["seq_read_GBps"].values())
    R = p["request_unit"]
    assert R >= 32 and R <= 4096 and (R & (R - 1)) == 0
    assert 0.05 < p["latency_us"] < 100
    # merged + aligned beats a 32-byte shift at the request unit (Fig. 4 (b) vs (c))
    assert p["rand_aligned_GBps"][R] >= p["rand_shift32_GBps"][R] * 0.95


def test_waves_in_flight_knee_follows_littles_law(profile):
    """Sec. 3.3: the link runs at rate B only with B * RTT / R requests in
    flight.  Each wave of the sweep keeps one R-byte block outstanding, so
    the rate climbs with the waves until about that many are in flight."""
    p = profile
    R = p["request_unit"]
    rates = p["waves_GBps"]
    waves = sorted(rates)
    assert all(rates[w] > 0 for w in waves)
    assert rates[waves[-1]] > 4 * rates[waves[0]]  # more requests in flight, more bandwidth
    best = max(rates.values())
    model = linkmodel.outstanding_needed(best * 1e9, R, p["latency_us"] * 1e-6)
    knee = p["knee_waves"]
    assert knee in rates and rates[knee] >= 0.9 * best
    assert model / 2 <= knee <= 2 * model, (knee, model, rates)


def test_offsets_and_pinning(profile):
    p = profile
    off = p["offset_GBps"]
    R = p["request_unit"]
    assert min(off) == 0 and max(off) == R
    # a block that starts on a request boundary (0 or R) is not slower than
    # one that straddles two (Fig. 4 (b) vs (c))
    mid = [v for o, v in off.items() if 0 < o < R]
    assert max(off[0], off[R]) >= 0.95 * max(mid)
    nc = p["noncoherent"]
    if nc["memcpy_GBps"] > 0:  # measured when the buffer could be pinned
        assert nc["seq_read_GBps"] > 0.5 and nc["rand_GBps"] > 0.5 and nc["coherent_rand_GBps"] > 0.5
    # GPU memory is far faster than the host link
    assert p["hbm_read_GBps"] > 10 * p["memcpy_GBps"]
    assert p["hbm_copy_GBps"] > 10 * p["memcpy_GBps"]


def test_calibration_rejects_small_buffer(gpu_device):
    import paper_2006_06890_amd as E
    with pytest.raises(E.EmogiError) as ei:
        E.emogi.calibrate_link(1 << 20)
    assert ei.value.code == -1
