"""The block -> element-chunk renumbering of the tensor kernels (block_chunk in
csrc/pcpf_device.h) is a permutation of the grid for both of its regimes: planes up to
XCD_MAP_MAX_PLANE_BYTES (one contiguous range of chunks per XCD) and larger planes (runs of
XCD_RUN consecutive chunks per XCD, a last partial round in plain order). Every element
chunk must be processed exactly once; a gap would leave elements un-updated that a sampled
full-size comparison might miss. The constants are read from the header; the formula is
restated here (CPU only)."""
import os
import re

import numpy as np
import pytest

HDR = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                   "paper_2006_10967_amd", "csrc", "pcpf_device.h")


def constants():
    s = open(HDR).read()
    run = int(re.search(r"constexpr uint32_t XCD_RUN = (\d+);", s).group(1))
    mib = int(re.search(r"XCD_MAP_MAX_PLANE_BYTES = int64_t\((\d+)\) << 20;", s).group(1))
    return run, mib << 20


def chunk(b, g, large, run, X=8):
    if large:
        rnd = b // (X * run)
        plain = (rnd + 1) * X * run > g
        return np.where(plain, b, rnd * X * run + (b % X) * run + (b // X) % run)
    x, q, r = b % X, g // X, g % X
    return x * q + np.minimum(x, r) + b // X


@pytest.mark.parametrize("g", [1, 7, 8, 255, 256, 257, 1000, 8 * 32 * 5 + 3, 110592, 442368,
                               (884736 + 7) // 8])
@pytest.mark.parametrize("large", [False, True])
def test_block_chunk_is_a_permutation(g, large):
    run, _ = constants()
    b = np.arange(g, dtype=np.int64)
    c = chunk(b, g, large, run)
    assert c.min() == 0 and c.max() == g - 1
    assert np.unique(c).size == g


def test_block_chunk_runs():
    """Large planes: the 8 run-long groups of each full round go to the 8 XCDs (block b runs
    on XCD b mod 8), each group consecutive chunks."""
    run, limit = constants()
    assert run >= 1 and limit == 24 << 20
    g = 8 * run * 3
    b = np.arange(g)
    c = chunk(b, g, True, run)
    for x in range(8):
        mine = np.sort(c[b % 8 == x])
        for r in range(3):
            part = mine[r * run:(r + 1) * run]
            assert np.array_equal(part, np.arange(part[0], part[0] + run))
