"""Host check of the bitmap layouts the kernels rely on: the library's own
helpers (snn_device.h), compiled for the host, must map the slots of a row
one-to-one onto bits, in the documented orders."""
import os
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.fixture(scope="module")
def table(tmp_path_factory):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    exe = str(tmp_path_factory.mktemp("layout") / "layout_dump")
    src = os.path.join(ROOT, "tests", "host", "layout_dump.cpp")
    subprocess.check_call([HIPCC, "-x", "hip", "--offload-arch=gfx950", "-O1", "-I",
                           os.path.join(ROOT, "paper_2301_10622_amd", "csrc"), src, "-o", exe])
    out = subprocess.check_output([exe]).decode().split()
    return np.array(out, dtype=np.int64).reshape(-1, 5)


def test_posting_bits_are_lane_major_per_block(table):
    s, w, b = table[:, 0], table[:, 1], table[:, 2]
    pos = w * 64 + b  # bit position within the row
    assert len(np.unique(pos)) == len(s) and pos.min() == 0 and pos.max() == len(s) - 1
    # slot 256 g + 4 l + i of block B is bit 4 g + i of the 16-bit chunk l of that block
    blk, g, lane, i = s >> 10, (s >> 8) & 3, (s >> 2) & 63, s & 3
    assert np.array_equal(pos, blk * 1024 + lane * 16 + g * 4 + i)
    # so a lane's 16 slots of a block are one contiguous 16-bit chunk
    for B in range(4):
        for l in (0, 1, 31, 63):
            sl = [B * 1024 + 256 * gg + 4 * l + ii for gg in range(4) for ii in range(4)]
            p = np.sort(pos[sl])
            assert p[0] == B * 1024 + 16 * l and np.array_equal(np.diff(p), np.ones(15))


def test_live_bits_are_lane_masks_per_group(table):
    s, w, b = table[:, 0], table[:, 3], table[:, 4]
    pos = w * 64 + b
    assert len(np.unique(pos)) == len(s)
    # word 4 g + i of group g has bit l set for slot 256 g + 4 l + i: a wavefront lane mask
    g, lane, i = s >> 8, (s >> 2) & 63, s & 3
    assert np.array_equal(w, 4 * g + i) and np.array_equal(b, lane)


def test_id_map_against_unordered_map(tmp_path):
    """The library's open-addressing id -> slot map (snn_host.h), compiled for
    the host, agrees with std::unordered_map over 400,000 random puts,
    overwrites and erases with colliding ids."""
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    exe = str(tmp_path / "idmap_check")
    src = os.path.join(ROOT, "tests", "host", "idmap_check.cpp")
    subprocess.check_call([HIPCC, "-x", "hip", "--offload-arch=gfx950", "-O1", "-I",
                           os.path.join(ROOT, "paper_2301_10622_amd", "csrc"), "-I", os.path.join(ROOT, "include"),
                           src, "-o", exe])
    assert subprocess.check_output([exe]).decode().strip() == "ok"


def test_slot_pool_order(tmp_path):
    """The library's free-slot pool (snn_host.h), compiled for the host, against
    a plain model over 300,000 random inserts, deletes and compactions, with
    and without array containers: no slot handed out twice, and every choice in
    the pool's order (stale blocks' free slots, then fresh slots when array
    containers exist, then the clean block with the most free slots)."""
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    exe = str(tmp_path / "slotpool_check")
    src = os.path.join(ROOT, "tests", "host", "slotpool_check.cpp")
    subprocess.check_call([HIPCC, "-x", "hip", "--offload-arch=gfx950", "-O1", "-I",
                           os.path.join(ROOT, "paper_2301_10622_amd", "csrc"), "-I", os.path.join(ROOT, "include"),
                           src, "-o", exe])
    assert subprocess.check_output([exe]).decode().strip() == "ok"
