"""Host checks of the static tile of the one-launch batch (batch.hip, tile13),
emulated with the kernel's index arithmetic for every row length it is
instantiated for (WDIG 0, 4..12; 2^13-element tiles, 512 threads x 16):

  * the load mapping (e = tid + 512 k) and the store mapping
    (e = lane + 64 k + 1024 w) reach every tile element once, at the global
    offset (e mod W) + (e / W) sd0 that the kernel's offset formulas give;
  * the three stage sets (register index of the load mapping, the LDS register
    groups for e bits [WDIG, 6), register index of the read-back mapping)
    transform exactly the row bits [WDIG, 13) of e, each once, and never a
    column bit.
"""
import numpy as np
import pytest

TH, EPT, E = 512, 16, 8192


def off1(tid, k, wdig, sd0):
    """batch.hip tile13, load mapping."""
    W = 1 << wdig
    if wdig <= 9:
        return (tid & (W - 1)) + ((tid >> wdig) + k * (TH >> wdig)) * sd0
    return tid + TH * (k & ((W // TH) - 1)) + (k >> (wdig - 9)) * sd0


def off2(lane, wv, k, wdig, sd0):
    """batch.hip tile13, store mapping."""
    W = 1 << wdig
    if wdig <= 6:
        return (lane & (W - 1)) + ((lane >> wdig) + wv * (1024 >> wdig) + k * (64 >> wdig)) * sd0
    return lane + 64 * (k & ((W >> 6) - 1)) + ((k >> (wdig - 6)) + wv * (1024 >> wdig)) * sd0


def natural(e, wdig, sd0):
    return (e & ((1 << wdig) - 1)) + (e >> wdig) * sd0


WDIGS = [0, 4, 5, 6, 7, 8, 9, 10, 11, 12]


@pytest.mark.parametrize("wdig", WDIGS)
def test_load_and_store_mappings(wdig):
    sd0 = (1 << 13) + 7  # any row stride
    tid = np.arange(TH)
    seen = np.zeros(E, np.int64)
    for k in range(EPT):
        e = tid + TH * k
        assert np.array_equal(off1(tid, k, wdig, sd0), natural(e, wdig, sd0))
        np.add.at(seen, e, 1)
    assert np.all(seen == 1)
    if wdig >= 9:
        return  # stored from the load mapping
    lane, wv = np.meshgrid(np.arange(64), np.arange(8), indexing="ij")
    seen[:] = 0
    for k in range(EPT):
        e = lane + 64 * k + 1024 * wv
        assert np.array_equal(off2(lane, wv, k, wdig, sd0), natural(e, wdig, sd0))
        np.add.at(seen, e.ravel(), 1)
    assert np.all(seen == 1)


@pytest.mark.parametrize("wdig", WDIGS)
def test_stage_sets_cover_the_row_bits_once(wdig):
    # register index of the load mapping: k bit b is e bit 9 + b (e = tid + 512 k)
    step1 = [9 + b for b in range(max(0, wdig - 9), 4)]
    # LDS groups (P2Groups<13, WDIG, 0, ..., 6 - WDIG>): row digits 0..5-WDIG = e bits WDIG..5
    step2 = list(range(wdig, 6)) if wdig < 6 else []
    # read-back mapping e = lane + 64 k + 1024 w: k bit b is e bit 6 + b; bits [max(0, WDIG-6), 3)
    step3 = [6 + b for b in range(max(0, wdig - 6), 3)] if wdig < 9 else []
    bits = step1 + step2 + step3
    assert sorted(bits) == list(range(wdig, 13)), (wdig, bits)
    assert min(bits) >= wdig  # no column bit is transformed
    # the read-back mapping's register index really is e bits 6..9
    lane, wv = 5, 3
    for k in range(EPT):
        e = lane + 64 * k + 1024 * wv
        assert (e >> 6) & 15 == k
