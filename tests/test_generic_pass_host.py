"""Host checks of the generic radix-p pass (fwt.hip, fwt_pass; pass_core.h,
run_group and divmod_small), emulated in Python:

  * divmod_small's float-reciprocal division (IEEE float32 operations,
    emulated bit for bit with numpy) equals integer division for every
    dividend and divisor the passes use;
  * for every pass of every plan (p = 3, 5, 7; complex float and complex
    double; all m up to 2^26 points), the thread mapping loads and stores each
    tile element exactly once (the running row/column counters equal
    e mod w and e / w) and every register-group step partitions the tile
    into groups of p^kk elements that differ in exactly the step's digits.
"""
import numpy as np
import pytest

LDS_WIDE = 160 * 1024


def divmod_small(a, dv):
    """The device arithmetic: q = (int)((float)a * (1.0f / dv)), one
    correction step."""
    a = np.asarray(a, dtype=np.int64)
    inv = np.float32(1.0) / np.float32(dv)
    q = (a.astype(np.float32) * inv).astype(np.int64)  # truncation, as (int) in C
    r = a - q * dv
    lo, hi = r < 0, r >= dv
    q = np.where(lo, q - 1, np.where(hi, q + 1, q))
    r = np.where(lo, r + dv, np.where(hi, r - dv, r))
    return q, r


@pytest.mark.parametrize("p", [2, 3, 5, 7])
def test_divmod_small_is_exact_for_every_power_divisor(p):
    a = np.arange(0, 1 << 20, dtype=np.int64)
    k = 0
    while p ** k < (1 << 20):
        q, r = divmod_small(a, p ** k)
        assert np.array_equal(q, a // p ** k) and np.array_equal(r, a % p ** k), (p, k)
        k += 1


def test_divmod_small_near_its_range_limit():
    g = np.random.default_rng(1)
    a = np.concatenate([g.integers(0, 1 << 22, 200000), (1 << 22) - 1 - np.arange(1000)])
    for dv in [3 ** 13, 5 ** 9, 7 ** 7, 3, 25, 1023, 1024, 6561, 19683]:
        q, r = divmod_small(a, dv)
        assert np.array_equal(q, a // dv) and np.array_equal(r, a % dv), dv


# ------------------------------------------------------------------ planner
def loads_per_thread(p):
    return {2: 16, 3: 9, 5: 16, 7: 7}[p]


def kreg(p):
    return {2: 4, 3: 2}.get(p, 1)


def plan(p, m, nbytes):
    """The generic planner (fwt.hip, plan): first pass of emax digits, then
    strided passes over the rest with rows of >= 64 bytes, split evenly."""
    budget = LDS_WIDE if nbytes >= 8 else 80 * 1024
    per_block = 1024 * loads_per_thread(p)
    emax = 0
    for e in range(1, 31):
        E = p ** e
        if (E + E // 32 + 1) * nbytes > budget or E > per_block:
            break
        emax = e
    wpref = 0
    while p ** wpref * nbytes < 64:
        wpref += 1
    out = [(0, min(m, emax), 0)]
    r1 = min(m, emax)
    rest = m - r1
    if rest > 0:
        cap = emax - min(wpref, r1)
        nstr = (rest + cap - 1) // cap
        d = r1
        for i in range(nstr):
            r = (rest - (d - r1) + (nstr - i) - 1) // (nstr - i)
            out.append((d, r, min(wpref, d)))
            d += r
    return out


def check_pass(p, d0, r, wdig):
    w = p ** wdig
    E = p ** r * w
    lpt = loads_per_thread(p)
    th = max(64, min(1024, (E + lpt - 1) // lpt))
    th = (th + 63) // 64 * 64
    assert th * lpt >= E and E < (1 << 22)
    sd0 = p ** d0
    # element sweep: running counters from divmod_small(tid), divmod_small(TH)
    tid = np.arange(th)
    i0, c0 = divmod_small(tid, w)
    ti, tc = divmod_small(th, w)
    c, i = c0.copy(), i0.copy()
    seen = np.zeros(E, dtype=np.int64)
    for k in range(lpt):
        e = tid + k * th
        ok = e < E
        assert np.array_equal(c[ok], e[ok] % w) and np.array_equal(i[ok], e[ok] // w)
        off = c + i * sd0
        assert np.array_equal(off[ok], (e % w + (e // w) * sd0)[ok])
        np.add.at(seen, e[ok], 1)
        c, i = c + tc, i + ti
        wrap = c >= w
        c, i = np.where(wrap, c - w, c), np.where(wrap, i + 1, i)
    assert np.all(seen == 1)
    # register-group steps over the r digits
    q = 0
    while q < r:
        kk = min(kreg(p), r - q)
        R, pq = p ** kk, p ** q
        ng = E // R
        g = np.arange(ng)
        rem, cc = divmod_small(g, w)
        ih, il = divmod_small(rem, pq)
        e0 = cc + w * (il + pq * R * ih)
        elems = e0[:, None] + np.arange(R)[None, :] * (w * pq)
        cover = np.zeros(E, dtype=np.int64)
        np.add.at(cover, elems.ravel(), 1)
        assert np.all(cover == 1), (p, d0, r, wdig, q)
        # members of a group differ only in row digits q..q+kk-1
        rows = elems // w
        assert np.all((rows // (pq * R)) == (rows[:, :1] // (pq * R)))
        assert np.all((rows % pq) == (rows[:, :1] % pq))
        q += kk


@pytest.mark.parametrize("p,nbytes", [(3, 8), (3, 16), (5, 8), (5, 16), (7, 8), (7, 16)])
def test_every_plan_covers_each_tile_element_once(p, nbytes):
    m = 1
    while p ** m <= 2 ** 26:
        done = 0
        for (d0, r, wdig) in plan(p, m, nbytes):
            check_pass(p, d0, r, wdig)
            assert d0 == done
            done += r
        assert done == m
        m += 1
