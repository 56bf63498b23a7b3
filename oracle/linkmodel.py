"""Closed-form host-link arithmetic of EMOGI Sec. 3.3 (test infrastructure).

The paper reasons about zero-copy bandwidth with four simple models; each is
written out here so the bench can predict, and the tests can pin, what a
request size implies.  Sizes are bytes, times are seconds, bandwidths are
bytes per second; the paper's "GB" are 2**30 bytes.
"""
import math

GIB = float(1 << 30)


def littles_law_bandwidth(outstanding, request_bytes, round_trip_s):
    """Sec. 3.3 (strided access): with at most ``outstanding`` requests in
    flight, each carrying ``request_bytes``, and a round trip of
    ``round_trip_s``, the link moves outstanding * size / RTT bytes/s."""
    return outstanding * request_bytes / round_trip_s


def tlp_overhead(payload_bytes, header_bytes=18):
    """Sec. 3.3: share of the wire taken by the packet header when each
    request returns ``payload_bytes`` (header / (header + payload))."""
    return header_bytes / (header_bytes + payload_bytes)


def outstanding_needed(bandwidth, request_bytes, round_trip_s):
    """Sec. 3.3 (merged and aligned access): requests that must be in flight
    to sustain ``bandwidth`` (Little's law solved for the queue length)."""
    return math.ceil(bandwidth * round_trip_s / request_bytes)


def dram_effective_bandwidth(peak, request_bytes, dram_burst_bytes=64):
    """Sec. 3.3: a request smaller than the DRAM burst still costs a burst."""
    bursts = math.ceil(request_bytes / dram_burst_bytes)
    return peak * request_bytes / (bursts * dram_burst_bytes)


def aligned_start_probability(elem_bytes, request_bytes):
    """Sec. 5.3.1: chance that a list starting at a uniformly random element
    index begins on a request boundary."""
    return elem_bytes / request_bytes
