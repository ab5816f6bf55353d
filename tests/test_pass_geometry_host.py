"""Host checks of the static p = 2 pass kernel's index arithmetic (fwt.hip,
fwt_p2 and P2Groups), emulated in Python for every instantiated shape: the
padded LDS index cpad(e) = e + e/32 folds over every sum the kernel splits
(cpad(a + b) = cpad(a) + cpad(b)), each register group and thread mapping
visits every tile element exactly once, and the stage digits of the three
groups (the loaded registers, the LDS groups, the stored registers) tile the
pass's digits [WDIG, LOGE) without overlap."""
import pytest


def cpad(e):
    return e + (e >> 5)


def shape(loge, wdig):
    E = 1 << loge
    th = max(64, min(1024, E // 16))
    ept = E // th
    return E, 1 << wdig, th, ept, min(4, ept.bit_length() - 1)


def groups(loge, wdig, kgm, rdl):
    """(Q, KG, list of element-index lists) of P2Groups<LOGE, WDIG, 0, T, KGM, RDL>."""
    E, W, th, ept, kgmax = shape(loge, wdig)
    q, out = 0, []
    while q < rdl:
        kg = min(kgmax, kgm, rdl - q)
        R, stq = 1 << kg, W << q
        gpt = (E >> kg) // th
        sets = []
        for t in range(gpt):
            for tid in range(th):
                g = tid + t * th
                c, rem = g & (W - 1), g >> wdig
                il, ih = rem & ((1 << q) - 1), rem >> q
                e0 = c + W * (il + (ih << (q + kg)))
                for j in range(R):
                    assert cpad(e0) + cpad(j * stq) == cpad(e0 + j * stq), (loge, wdig, q, e0, j)
                sets.append([e0 + j * stq for j in range(R)])
        out.append((q, kg, sets))
        q += kg
    return out


SHAPES = [(loge, wdig) for loge in range(7, 15) for wdig in (0, 4, 5)]


@pytest.mark.parametrize("loge,wdig", SHAPES)
@pytest.mark.parametrize("kgm", [4, 2])
def test_stage_groups_fold_and_cover(loge, wdig, kgm):
    E, W, th, ept, _ = shape(loge, wdig)
    assert th % W == 0 and ept >= 2
    # first mapping: element tid + k TH at LDS cpad(tid) + cpad(k TH)
    seen = set()
    for tid in range(th):
        for k in range(ept):
            e = tid + k * th
            assert cpad(tid) + cpad(k * th) == cpad(e)
            seen.add(e)
    assert seen == set(range(E))
    rdl = (6 - wdig) if loge >= 10 else loge - wdig
    for q, kg, sets in groups(loge, wdig, kgm, rdl):
        flat = [e for s in sets for e in s]
        assert sorted(flat) == list(range(E)), (loge, wdig, q)
        # the group's elements differ exactly in row digits [q, q + kg)
        for s in sets:
            diffs = {e ^ s[0] for e in s}
            mask = ((1 << kg) - 1) << (wdig + q)
            assert all(d & ~mask == 0 for d in diffs) and len(diffs) == 1 << kg


@pytest.mark.parametrize("loge,wdig", [s for s in SHAPES if s[0] >= 10])
def test_three_group_digits_tile_the_pass(loge, wdig):
    """LOGE >= 10: loaded registers hold bits LOGE-4..LOGE-1 of e, the LDS
    groups bits [WDIG, 6), the stored mapping e = lane + 64 k + 1024 w bits
    6..6+NS-1 (NS = min(LOGE - 10, 4)); together exactly [WDIG, LOGE)."""
    E, W, th, ept, _ = shape(loge, wdig)
    ns = min(loge - 10, 4)
    bits = list(range(loge - 4, loge)) + list(range(wdig, 6)) + list(range(6, 6 + ns))
    assert sorted(bits) == list(range(wdig, loge))
    seen = set()
    for wv in range(th // 64):
        for lane in range(64):
            for k in range(16):
                e = lane + 64 * k + 1024 * wv
                assert cpad(lane + 1024 * wv) + 66 * k == cpad(e)
                seen.add(e)
    assert seen == set(range(E))


@pytest.mark.parametrize("m,F", [(15, 12), (16, 13), (17, 14), (19, 14)])
def test_blocked_intermediate_layout(m, F):
    """Two-pass float64 plans with the blocked intermediate (PassDesc::oblk):
    the first pass (tiles of 2^F, thread mapping e = lane + 64 k + 1024 w)
    stores element e of tile t at (e >> 4) * 16 NH + 16 t + (e & 15), NH =
    2^(m - F); the strided pass (rows of 16, NH rows) reads its tile b as the
    contiguous block b * 16 NH + 16 i + w; the weights kernel maps a blocked
    position back to the coefficient index h = t 2^F + 16 (e >> 4) + (e & 15).
    All three agree, and each is a bijection onto [0, 2^m)."""
    N, E, NH = 1 << m, 1 << F, 1 << (m - F)
    th = E // 16
    rs = 16 * NH
    store = {}
    for t in range(NH):
        for wv in range(th // 64):
            for lane in range(64):
                for k in range(16):
                    e = lane + 64 * k + 1024 * wv
                    off = ((lane >> 4) + 64 * wv) * rs + t * 16 + (lane & 15) + k * 4 * rs
                    assert off == (e >> 4) * rs + 16 * t + (e & 15)
                    store[(t, e)] = off
    assert sorted(store.values()) == list(range(N))
    inv = {off: te for te, off in store.items()}
    for b in range(N // rs):                     # strided tiles: one per 16-element column block
        for i in range(NH):
            for w in range(16):
                off = b * rs + 16 * i + w        # base tile*shi (shi = E_strided = rs), row stride 16
                t, e = inv[off]
                assert (t, e >> 4, e & 15) == (i, b, w)
    for off in range(N):
        w, hi, mid = off & 15, (off >> 4) & (NH - 1), off >> (4 + m - F)
        h = (hi << F) + mid * 16 + w
        t, e = inv[off]
        assert h == (t << F) + e
